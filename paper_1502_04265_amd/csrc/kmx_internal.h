// Internal declarations shared by the kmx translation units.  Not installed;
// the public contract is include/kmx.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <string>
#include <utility>
#include <vector>

#include "../../include/kmx.h"

namespace kmx {

// Per-row statistics written once per dataset by the prep kernel.
//   xn2 : ||x||^2 (FP64 sum, rounded to nearest float)
//   nx  : ||x||, rounded up
//   nxq : ||x~|| of the quantized row (== nx for FP32), rounded up
//   rx  : ||x - x~|| (0 for FP32), rounded up
struct RowStats {
  float xn2, nx, nxq, rx;
};

// Per-iteration center statistics (maxima over centers), set by prep_centers
// through atomicMax on the bit patterns of non-negative floats.
//   cq_max : max_j ||c~_j||    (rounded up)
//   rc_max : max_j ||c_j - c~_j|| (rounded up)
//   cn_max : max_j ||c_j||     (rounded up)
//   O      : score offset of the BF16 / FP8 GEMM (see k_assign.hip)
//   c_amax : max_j max_i |c_ji| (FP8 only)
//   c_exp  : E8M0 exponent byte of the FP8 center scale (FP8 only)
struct CenterStats {
  unsigned int cq_max, rc_max, cn_max;
  float O;
  unsigned int c_amax;
  int c_exp;
};

// Device-side Lloyd state, one instance per context.
struct LoopState {
  int done;          // set once the stopping rule fired
  int iter;          // completed update steps
  int max_iter;
  int track_changes; // count label changes against the previous labels
  double tol;        // < 0: fixed iteration count
  unsigned long long changed;
  unsigned long long flagged;      // entries of the re-check list (last assign)
  unsigned long long full_count;   // rows sent to the FP32 GEMM pass (BF16 only)
  unsigned long long flagged_full; // rows re-checked against every center
  unsigned long long undecided;    // rows the first GEMM pass could not decide
  double cost_at_centroids;
  double cost_last;
  unsigned long long full_count2;      // rows the BF16 pass of an FP8 cascade sent to FP32
  unsigned long long routed_fallback;  // rows the certificate sent to the GEMM (last assign)
  unsigned long long routed_listed;    // certified rows that needed the short re-check
  unsigned long long bound_fail;       // rows the carried bounds could not keep (last assign)
  unsigned long long bound_pair;       // rows they sent to the re-check with their runner-up
  unsigned long long dcount;           // changed rows listed for the delta update (this update)
  unsigned long long need_rows;        // rows whose proposals are computed in this assignment
  unsigned long long listed_total;     // re-check list entries of the earlier assignments of the run
  unsigned long long full_total;       // every-center rows of the earlier assignments of the run
  int acc_valid;                       // the carried clustering features hold the last labels
  int pad_;
};

// Entry of the short re-check list: row index and the other candidates (the
// leader is the row's current label; cand3 = -1 when there are only two).
struct FlagEntry {
  int row;
  int cand2;
  int cand3;
  int pad;
};

// Batched assignment (many independent instances, one launch).  Instances of
// equal d form a bucket whose rows, centers and labels are concatenated;
// labels and list entries use bucket-global center indices and global rows.
struct BatchInst {
  int64_t row0;        // first row of the instance in its bucket
  int64_t grow0;       // first row in the global numbering (all buckets)
  int n, d, dp, k;
  int kpad;            // padded center count (multiple of the variant's tile)
  int koff;            // first center of the instance in its bucket
  int kg0;             // first center in the global numbering (all buckets)
  int cpad0;           // first padded center row in the bucket's quantized centers
  int variant;         // tile shape, index into the batched kernel's variant list
  int ib;              // index bits of the packed keys
  int bucket;
  int pad_;
  const uint16_t* xq;  // bucket BF16 rows (dp per row)
  const RowStats* rs;  // bucket row statistics
  uint16_t* cq;        // bucket quantized centers (dp per padded center)
  double* hd;          // per padded center (global numbering of padded centers)
  CenterStats* cs;     // this instance's statistics
  const float* X;      // bucket FP32 rows (d per row)
  const float* C;      // bucket FP32 centers (d per center)
  const unsigned* xq_max;  // bucket max ||x~||
  int hd0;             // first padded center in the global numbering of padded centers
  int pad2_;
  float* ch;           // per padded center (global numbering): O - h_j, the GEMM start value
};

// Center drift of one Lloyd step (the bound-carrying assignment): the two
// largest drifts and the center of the largest.
struct DriftStat {
  float max1, max2, max3;
  int arg1, arg2;
  int pad[3];
};

// Bounds carried across Lloyd iterations, one entry per row (all nullable
// together).  For label a: ub >= ||x - c_a||; sec = a runner-up center b (or
// -1), l2 <= ||x - c_b||; lb <= ||x - c|| for every other center c (not a,
// not b).  Distances, not squares; rounded outward.
struct BoundsOut {
  float* ub = nullptr;
  float* lb = nullptr;
  float* l2 = nullptr;
  int* sec = nullptr;
};

struct BatchItem {
  int inst;
  int blk;             // block of points within the instance
};

struct BatchBucket {
  int64_t grow0;       // first global row
  int64_t n;
  int d, K;            // width, centers of all its instances
  const float* X;      // FP32 rows (d per row)
  const float* C;      // FP32 centers (d per center)
};

enum TimingClass {
  T_PREP = 0, T_ASSIGN = 1, T_RECHECK = 2, T_SORT = 3, T_REDUCE = 4,
  T_FINAL = 5, T_SEED = 6, T_OTHER = 7, T_ROUTER = 8, T_CERT = 9, T_TRAIN = 10,
  T_PROJECT = 11, T_BOUND = 12, T_SHORT = 13, T_NCLASS = 14
};

// Grow-only device buffer.
struct Buf {
  void* p = nullptr;
  size_t bytes = 0;
};

// Sizes of the row blocks used by the sort and the seeding rounds.
constexpr int kSortRows = 2048;     // rows per histogram / scatter block
constexpr int kReduceRows = 512;    // rows per segmented-reduction chunk
constexpr int kSeedRows = 2048;     // rows per seeding block
constexpr int kScanSegs = 64;       // column-scan segments
constexpr int kMaxK = 16384;        // largest k (LDS histograms)
constexpr int kGemmMaxD = 1024;     // widest row the GEMM passes take (wider: every-center re-check)
// FP32-pass lists of at most kShortList rows go to the every-center re-check
// instead when k d >= kShortListMinKD: the pass then costs one workgroup's
// walk over many long centers however few rows it has, while for small k d
// the pass is short and the every-center re-check (a workgroup per row) is
// the slower one
constexpr int kShortList = 4096;
constexpr int64_t kShortListMinKD = 65536;

// Candidate router (k_router.hip, k_train.hip).
constexpr int kRouterH = 256;       // hidden units
constexpr int kRouterHU = kRouterH / 32;  // layer-2 K units of 32
constexpr int kRouterBN1 = 16;      // hidden units per layer-1 LDS tile
constexpr int kRouterBN2 = 64;      // centers per layer-2 LDS tile
constexpr int kRouterM = 16;        // proposals per point
constexpr int kRouterMaxK = 4096;   // largest k the router supports
constexpr int kNbrL = 32;           // sorted neighbours kept per center
constexpr int kRouterMaxBatch = 65536;  // largest training batch

}  // namespace kmx

struct kmx_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  int num_cus = 256;
  bool validate = false;   // KMX_VALIDATE=1: scan X and C for non-finite values
  void* na_scratch = nullptr;   // device address of this device's static scratch array
  std::string err;
  // the problems whose rows, weights, row statistics and feature grids the
  // batched path's grouped buffers hold (empty: none; kmx_invalidate clears)
  std::vector<int64_t> batch_key;

  // cached per-dataset data
  const float* cache_X = nullptr;
  int64_t cache_n = 0, cache_ldx = 0;
  int cache_d = 0, cache_prec = -1;
  bool cache_valid = false;

  kmx::Buf xq, rowstats, xstats;
  // FP8 copy of X (rows of dp bytes), E8M0 row scales and its row statistics
  const float* cache8_X = nullptr;
  int64_t cache8_n = 0, cache8_ldx = 0;
  int cache8_d = 0;
  bool cache8_valid = false;
  int last_prec = -1;   // precision of the most recent assignment
  kmx::Buf xq8, sx8, rowstats8, xstats8, cq8, ch8, hd8, cstats8, full_rows2;
  kmx::Buf cq, ch, hd, cstats, cq32, ch32, cstats32, full_rows, brute;
  kmx::Buf lab_a, lab_prev, d1, d2;
  kmx::Buf flags, counters;
  kmx::Buf counts, segsum, base, chunk_base, perm;
  kmx::Buf partS, partWQ;
  // exactly summed clustering features: per-dataset column maxima and row
  // norms (cached like the quantized copies), the call's grids, the features
  // carried across Lloyd iterations and the delta update's lists
  const float* cf_X = nullptr;
  int64_t cf_n = 0, cf_ldx = 0;
  int cf_d = 0;
  bool cf_valid = false;
  kmx::Buf cf_colmax, cf_q, cf_qmax, cf_wmax, cfs, cf_acc;
  kmx::Buf ecount, ebase, ecursor, dchunk, clist, cold, dent, cfflag;
  kmx::Buf W, termC, termMu;
  kmx::Buf state;
  kmx::Buf vcheck;   // argument-check counters
  kmx::Buf D2, chosen, seed_part, seed_ctr, seed_a, seed_cc, seed_nread;
  kmx::Buf bs_D2, bs_sa, bs_cc, bs_chosen, bs_part, bs_ctr, bs_insts;   // batched seeding
  kmx::Buf scratch_c, hist;
  kmx::Buf fb_rows, keys, cdist, nbr, nbd, fbh;   // routed assignment
  kmx::Buf prop_have, prop_rows;   // bounded routed: rows with proposals, rows needing them
  kmx::Buf hub, hlb, hl2, hsec, bl_rows, cprev, drift, dstat, bkh;   // carried bounds
  // batched Lloyd: concatenated instances and their descriptors
  kmx::Buf vt;                          // transposed projection basis
  kmx::Buf sv_om, sv_y, sv_y2, sv_z, sv_g, sv_part, sv_r, sv_v;   // range finder
  kmx::Buf bX, bXq, brs, bw, bC, bCq, bhd, bch, bcs, blab, bitems, binsts, bbuckets, bcinst, bxstats;
  kmx::Buf btermC, btermMu, bW, bcost;
  kmx::Buf bstate, blab_prev, bacc;   // batched delta update: per-bucket states, labels, features
  kmx::Buf bcf_colmax, bcf_q, bcf_qmax, bcf_wmax, bcfs;   // per-bucket feature grids
  hipStream_t cap_stream = nullptr;                // stream graphs are captured on (batched, graphed Lloyd)
  uint64_t ws_gen = 0;                             // bumped whenever a workspace buffer moves
  // the last captured Lloyd iteration of kmx_lloyd_graph and what it was captured for
  hipGraph_t lg_graph = nullptr;
  hipGraphExec_t lg_exec = nullptr;
  hipEvent_t lg_event = nullptr;                   // orders the capture stream after the context stream
  uint64_t lg_key[12] = {0};
  std::map<std::pair<int, int>, int> tune;         // (d, k class) -> tile-shape variant

  // timing
  bool timing = false;
  struct Rec { int cls; hipEvent_t a, b; };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  double ms_acc[kmx::T_NCLASS] = {0};
  int64_t cnt_acc[kmx::T_NCLASS] = {0};
};

namespace kmx {

// Device address of the calling device's static scratch array of
// kmx_assign_noalloc (looked up once per device; the device must be current).
hipError_t noalloc_init(int device, void** ptr);

// ---- launchers (each returns hipSuccess or the launch error) --------------
// prep
hipError_t launch_prep_rows(hipStream_t s, const float* X, int64_t n, int d, int64_t ldx,
                            int dp, uint16_t* Xq, RowStats* st, unsigned* xq_max, int num_cus);
hipError_t launch_prep_centers(hipStream_t s, const float* C, int k, int d, int kpad, int dp,
                               int prec, void* Cq, float* ch, double* hd, CenterStats* cs,
                               const unsigned* xq_max);
hipError_t launch_prep_rows_f8(hipStream_t s, const float* X, int64_t n, int d, int64_t ldx,
                               int dp, uint8_t* Xq8, uint8_t* sx8, RowStats* st,
                               unsigned* xq_max, int num_cus);
// argument checks: out[0] += rows with w > 0, out[1] += bad entries (not
// finite, or negative weights); out must be cleared first
hipError_t launch_check_weights(hipStream_t s, const float* w, int64_t n, unsigned long long* out,
                                int num_cus);
hipError_t launch_scan_finite(hipStream_t s, const float* A, int64_t rows, int cols, int64_t ld,
                              unsigned long long* out, int num_cus);
hipError_t launch_fill_i32(hipStream_t s, int32_t* p, int64_t n, int32_t v);
hipError_t launch_fill_u8(hipStream_t s, uint8_t* p, int64_t n, uint8_t v);
hipError_t launch_reset_small(hipStream_t s, CenterStats* cs, CenterStats* cs2, CenterStats* cs3,
                              LoopState* st, int reset_iter);

// Batched seeding: one instance's arguments and workspace (k_seed.hip).
struct SeedInst {
  const float* X;
  const float* w;      // nullable
  float* C;            // k x d out
  int64_t* idx;        // k out, nullable
  double* D2;          // n
  int32_t* sa;         // n: index of the row's closest chosen center
  double* cc2;         // k: squared gaps of the newest center to the earlier ones
  uint8_t* chosen;     // n
  double* part;        // nb block masses
  unsigned int* ctr;   // the instance's ticket
  int64_t n, ldx, blk0;
  uint64_t seed;
  int d, k, nb;
};
hipError_t launch_seed_batched_round(hipStream_t s, const SeedInst* insts, int m, int r,
                                     int64_t blocks);
// the gaps of round r (r >= 2) of the first m instances
hipError_t launch_seed_batched_gaps(hipStream_t s, const SeedInst* insts, int m, int r);

// assign
// Operand code of the last GEMM pass of the BF16 and FP8 cascades (besides
// KMX_FP32, KMX_BF16, KMX_FP8E4M3): FP32 rows and centers each split into two
// BF16 parts, x = x_hi + x_lo, and three BF16 products per coordinate (see
// k_assign.hip).  Center rows hold dp high parts, then dp low parts.
constexpr int kSplitBf16 = 3;
int assign_tile_n(int prec, int d, int k);   // centers per tile (kpad granularity)
int assign_dpad(int prec, int d);     // padded row length of the GEMM operands
hipError_t launch_assign(hipStream_t s, int prec, const float* X, int64_t ldx,
                         const void* Xq, const uint8_t* sx8, int64_t n, const int* rows,
                         const unsigned long long* row_count, int d, int dp,
                         const RowStats* rs, const void* Cq, const float* ch,
                         int k, int kpad, const CenterStats* cs, int32_t* label,
                         float* d1, float* d2, FlagEntry* flags, int* full_rows,
                         unsigned long long* full_ctr, int cascade_all, int* brute,
                         LoopState* st, const int* gate, int num_cus, BoundsOut bo = {});
// count instances of one matrix instruction of the assignment (FP8 16x16x128
// scaled, BF16 16x16x32 or FP32 16x16x4) from C (nullable: zero)
hipError_t launch_mfma_probe(hipStream_t s, int prec, const uint8_t* A, const uint8_t* B,
                             const uint8_t* sa, const uint8_t* sb, const float* C, float* D,
                             int count);
hipError_t launch_recheck(hipStream_t s, const float* X, int64_t n, int d, int64_t ldx,
                          const float* C, int k, int32_t* label, float* d1,
                          const FlagEntry* flags, const int* brute, const LoopState* st,
                          int num_cus, const int* gate, BoundsOut bo = {}, float* d2 = nullptr);
// brute[0 .. m) = rows[0 .. m) (m = *row_count) or 0 .. n - 1, and
// st->flagged_full = st->undecided = m: every listed row to the every-center
// re-check (the assignment of rows wider than the GEMM takes)
hipError_t launch_list_all(hipStream_t s, int* brute, int64_t n, const int* rows,
                           const unsigned long long* row_count, LoopState* st, const int* gate);
// Moves a list meant for the FP32 GEMM pass onto the every-center re-check
// list when it holds at most kShortList rows and k d >= kShortListMinKD (one
// workgroup; gate as above).
hipError_t launch_route_small(hipStream_t s, unsigned long long* ctr, const int* list, int* brute,
                              LoopState* st, int k, int d, const int* gate);

// update
// Stable counting sort of rows by label.  counts holds nb x k entries
// (nb = ceil(n / kSortRows)); with track, 4 nb more after them, and the number
// of labels that differ from lab_prev is added to st->changed.
hipError_t launch_sort(hipStream_t s, const int32_t* label, int32_t* lab_prev, int64_t n,
                       int k, int32_t* counts, int32_t* segsum, int32_t* base,
                       int32_t* chunk_base, int32_t* perm, LoopState* st, int track,
                       const int* gate);
// Exactly summed clustering features (k_update.hip).  cf_prep: column maxima
// of |x| (d entries) and FP64 row norms (n entries) with their maximum, once
// per dataset.  cf_scales: the call's grids (cfs: 2 d + 4 doubles) from them
// and the largest weight (w == nullptr: unit weights; wmax is scratch).
hipError_t launch_cf_prep(hipStream_t s, const float* X, int64_t n, int d, int64_t ldx,
                          unsigned* colmax, double* qrow, unsigned long long* qmax, int num_cus);
hipError_t launch_cf_scales(hipStream_t s, const unsigned* colmax, int d,
                            const unsigned long long* qmax, const float* w, int64_t n,
                            unsigned* wmax, double* cfs, int num_cus);
// Chunk reduction into limb sums: partS holds 2 d doubles per chunk, partWQ 4.
// delta = 0: ent is the sorted permutation (base / chunk_base from the sort);
// delta = 1: signed entries (ebase / dchunk from the delta plan).
hipError_t launch_reduce(hipStream_t s, const float* X, int64_t n, int d, int64_t ldx,
                         const float* w, const double* qrow, const int32_t* ent,
                         const int32_t* base, const int32_t* chunk_base, int k,
                         const double* cfs, double* partS, double* partWQ, int delta,
                         int num_cus, const int* gate);
// New centers and cost terms from the chunk sums.  acc (nullable, k d 2 + 4 k
// int64) carries the features across iterations; *mode_p = 1 stores the full
// reduction's sums in it, 0 adds the delta reduction's; mode_p == nullptr
// means 1.  Sets st->acc_valid when acc is written.
hipError_t launch_finalize(hipStream_t s, const double* partS, const double* partWQ,
                           const int32_t* chunk_base, const int32_t* dchunk, const int* mode_p,
                           long long* acc, int k, int d, const double* cfs, const float* C_prev,
                           float* C_out, double* W_out, double* termC, double* termMu,
                           int write_c, LoopState* st, const int* gate);
// Delta update set-up: mark the changed rows (updating lab_prev, st->changed,
// st->dcount; st->dcount must be zero before), plan (flags[0] / flags[1]:
// skip the full / delta path, flags[2]: finalize mode) and scatter the signed
// entries into dent.  ecount (k) must be zero before the first call; the plan
// clears it again.  gate: a set value skips both paths.
hipError_t launch_delta_prepare(hipStream_t s, const int32_t* label, int32_t* lab_prev, int64_t n,
                                int k, int32_t* ecount, int32_t* clist, int32_t* cold,
                                int32_t* ebase, int32_t* cursor, int32_t* dchunk, int32_t* ent,
                                int* flags, LoopState* st, int num_cus, const int* gate);
hipError_t launch_cost_sum(hipStream_t s, const double* termC, const double* termMu, int k,
                           LoopState* st, double* cost_hist, int mode, const int* gate);

// seeding: one round r (r >= 2 first fills cc2 with the squared distances of
// c_{r-1} to the earlier centers).  sa: n ints, the index of each row's
// closest chosen center; cc2: k doubles; nread: one int per 2048-row block;
// rows_read: adds the rows whose distance was computed.
hipError_t launch_seed_round(hipStream_t s, const float* X, int64_t n, int d, int64_t ldx,
                             const float* w, int r, uint64_t seed, double* D2,
                             uint8_t* chosen, double* part, unsigned int* ctr,
                             float* C_out, int64_t* idx_out, int32_t* sa, double* cc2,
                             int* nread, unsigned long long* rows_read);

// batched (k_assign.hip, k_batch.hip)
int batched_variants(int d);                  // number of tile shapes for width d
int batched_variant_tile(int d, int v);       // centers per tile of variant v
int batched_variant_ppb(int d, int v);        // points per block of variant v
int batched_variant_id(int d, int v);         // variant index over all groups
int batched_dpad(int d);                      // BF16 row length of a bucket of width d
int batched_group(int d);                     // width group (one kernel per group)
hipError_t launch_assign_batched(hipStream_t s, int group, const BatchItem* items, int begin,
                                 int end, const BatchInst* insts, FlagEntry* flags, int* brute,
                                 LoopState* st, int32_t* label, int grid);
hipError_t launch_recheck_batched(hipStream_t s, const BatchBucket* buckets, int nbuckets,
                                  const BatchInst* insts, int ninst, int32_t* label,
                                  const FlagEntry* flags, const int* brute, const LoopState* st,
                                  int64_t nrows, int num_cus);
// per-bucket delta-update states (dcount, changed; init: acc_valid too)
hipError_t launch_bucket_states(hipStream_t s, LoopState* bst, int nb, int init);
hipError_t launch_batch_reset(hipStream_t s, const BatchInst* insts, int ninst, LoopState* st,
                              unsigned* work_ctr);
hipError_t launch_batch_prep_centers(hipStream_t s, const BatchInst* insts, const int* cinst,
                                     int npad);
hipError_t launch_batch_cost(hipStream_t s, const BatchInst* insts, int ninst,
                             const double* termC, double* cost, int stride, LoopState* st,
                             int advance);
hipError_t launch_batch_labels(hipStream_t s, const int32_t* glabel, int64_t grow0, int n,
                               int koff, int32_t* out);

// carried bounds (k_bounds.hip)
hipError_t launch_drift(hipStream_t s, const float* Cold, const float* Cnew, int k, int d,
                        float* drift, DriftStat* ds, const int* gate);
// rows whose bounds keep their label are left alone; rows where only the
// runner-up can win go to the short re-check list (flags, st->flagged) as a
// pair; the others to fail_rows (st->bound_fail)
hipError_t launch_bounds_test(hipStream_t s, int64_t n, const int32_t* label, BoundsOut bo,
                              const float* drift, const DriftStat* ds, int k, int* fail_rows,
                              FlagEntry* flags, LoopState* st, const int* gate, int num_cus);
hipError_t launch_copy_f32(hipStream_t s, const float* src, float* dst, int64_t count,
                           const int* gate);
hipError_t launch_record_kept(hipStream_t s, const LoopState* st, int64_t* kept, int slot,
                              int64_t n, const int* gate);

// projection (k_project.hip)
hipError_t launch_project(hipStream_t s, const float* X, int64_t rows, int d_in, int64_t ldx,
                          const float* V, int d_out, float* Y, int64_t ldy, float* Vt,
                          int num_cus);
int project_dpad(int d_in);
// Y = Z V^T (Z rows x m, V d x m row-major, m <= 128, rows < 65535 * 64).
hipError_t launch_lift(hipStream_t s, const float* Z, int64_t rows, int m, int64_t ldz,
                       const float* V, int d, float* Y, int64_t ldy);            // row length of the transposed basis workspace

// range finder (k_svd.hip)
hipError_t launch_gauss_fill(hipStream_t s, float* out, int64_t count, uint64_t seed);
hipError_t launch_scale_rows(hipStream_t s, float* Y, int64_t n, int q, int64_t ldy,
                             const float* w);   // Y_i *= sqrt(w_i)
int atb_slices(int64_t n, int p, int num_cus);
// out (p x q, FP64) = A^T diag(sqrt w) B, A n x p, B n x q (q <= 128), w nullable;
// part: slices x p x q doubles
hipError_t launch_atb(hipStream_t s, const float* A, int64_t n, int p, int64_t lda, const float* B,
                      int q, int64_t ldb, const float* w, double* part, int slices, double* out);
hipError_t launch_f64_to_f32(hipStream_t s, const double* in, float* out, int64_t count);

// router: inference (k_router.hip)
int router_units(int d, int dp);
hipError_t launch_router_layout(hipStream_t s, const float* W1, const float* W2, const float* b2,
                                int d, int k, int kpad, int r1, uint16_t* W1a, uint16_t* W2a,
                                float* b2p);
// Forward pass of the router for rows 0 .. n-1, or with a row list for rows
// rows[0 .. *row_count) (keys written at each row's position).
hipError_t launch_router_fwd(hipStream_t s, const uint16_t* Xq, int64_t dp, int64_t n, int d,
                             const uint16_t* W1a, const float* b1, const uint16_t* W2a,
                             const float* b2p, int kpad, uint32_t* keys, const int* gate,
                             int num_cus, const int* rows = nullptr,
                             const unsigned long long* row_count = nullptr);
// Rows of rows[0 .. *count) without proposals yet (have[row] == 0) are
// marked and listed in out (*out_count, which must be zero before).
hipError_t launch_need_proposals(hipStream_t s, const int* rows, const unsigned long long* count,
                                 int64_t max_rows, uint8_t* have, int* out,
                                 unsigned long long* out_count, const int* gate, int num_cus);
hipError_t launch_router_decode(hipStream_t s, const uint32_t* keys, int64_t count, int k,
                                int kpad, int32_t* cand);
hipError_t launch_center_table(hipStream_t s, const float* C, int k, int d, float* D, int32_t* nbr,
                               float* nbd, const int* gate);
hipError_t launch_router_cert(hipStream_t s, const uint16_t* Xq, int64_t dp, int64_t n, int d,
                              const float* C, int k, const RowStats* rs, const uint32_t* keys,
                              int kpad, const int32_t* nbr, const float* nbd, int32_t* label,
                              FlagEntry* flags, int* fb_rows, LoopState* st, const int* gate,
                              int num_cus, const int* rows = nullptr,
                              const unsigned long long* row_count = nullptr, BoundsOut bo = {});
hipError_t launch_record_fallback(hipStream_t s, const LoopState* st, int64_t* fbh, int slot,
                                  int all_rows, int64_t all, const int* gate);

// router: training (k_train.hip)
hipError_t launch_gather_batch(hipStream_t s, const float* X, int64_t n, int d, int64_t ldx,
                               const int32_t* labels, uint64_t total, int64_t first, int bsz,
                               int d8, int shuffle, uint64_t key, int k, uint16_t* Xb,
                               int32_t* yb);
int gemm_splits(int M, int N, int K, int num_cus, int* kchunk);
hipError_t launch_gemm_bf16(hipStream_t s, int M, int N, int K, const uint16_t* A, int64_t lda,
                            bool ak, const uint16_t* B, int64_t ldb, bool bk, float* Cp, int splits,
                            int kchunk);
hipError_t launch_ep_hidden(hipStream_t s, const float* P, int S, int M, int N, const float* bias,
                            const uint16_t* Hb, uint16_t* out, int mode);
hipError_t launch_softmax_ce(hipStream_t s, const float* P, int bsz, int k, int k8,
                             const float* b2, const int32_t* yb, uint16_t* dZ, float* lossrow);
hipError_t launch_sum_partials(hipStream_t s, const float* P, int S, int64_t zstride, int rows,
                               int cols, int ldp, float* out);
int colsum_segments(int rows);
hipError_t launch_colsum(hipStream_t s, const uint16_t* Mx, int rows, int cols, int ld,
                         float* part, float* out);
hipError_t launch_loss_mean(hipStream_t s, const float* lossrow, int bsz, double* out);
hipError_t launch_adam(hipStream_t s, float* p, const float* g, float* m, float* v, int rows,
                       int cols, float lr, float beta1, float beta2, float eps, float bc1, float bc2,
                       uint16_t* bf, int ldb);
hipError_t launch_to_bf16_pad(hipStream_t s, const float* src, int rows, int cols, int prow,
                              int ldb, uint16_t* dst);

}  // namespace kmx
