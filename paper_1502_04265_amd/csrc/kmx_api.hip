// Host side of the kmx C ABI: argument checks, the grow-only workspace, the
// per-dataset cache and the launch sequences of seed / assign / update / cost
// / lloyd.  All device work is enqueued on the context's stream.
#include <algorithm>
#include <climits>
#include <cstdlib>
#include <cstdint>
#include <cstring>
#include <string>

#include "host_util.h"

using namespace kmx;
using namespace kmx::host;

namespace kmx {
namespace host {

thread_local std::string g_create_err;

kmx_status check_problem(kmx_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx,
                         int32_t k) {
  if (!X) return fail(ctx, KMX_EINVAL, "X is NULL");
  if (n < 1 || n > (int64_t)INT32_MAX - 1)
    return fail(ctx, KMX_EINVAL, "n must lie in [1, 2^31 - 2], got " + std::to_string(n));
  if (d < 1) return fail(ctx, KMX_EINVAL, "d must be >= 1, got " + std::to_string(d));
  if (ldx < d) return fail(ctx, KMX_EINVAL, "ldx must be >= d");
  if (k < 1) return fail(ctx, KMX_EINVAL, "k must be >= 1, got " + std::to_string(k));
  if ((int64_t)k > n) return fail(ctx, KMX_EINVAL, "k must be <= n");
  if (k > kMaxK)
    return fail(ctx, KMX_EUNSUPPORTED, "k above " + std::to_string(kMaxK) + " is not supported");
  return KMX_OK;
}

kmx_status check_prec(kmx_ctx* ctx, int prec, int d, bool allow_wide) {
  if (prec != KMX_FP32 && prec != KMX_BF16 && prec != KMX_FP8E4M3)
    return fail(ctx, KMX_EINVAL, "unknown precision");
  if (d > kGemmMaxD && !allow_wide)
    return fail(ctx, KMX_EUNSUPPORTED,
                "this call supports d <= " + std::to_string(kGemmMaxD) + ", got " +
                    std::to_string(d));
  return KMX_OK;
}

// Checks that need the data, before any work of the call is enqueued: the
// weights (when given) must be finite and >= 0, and at least min_pos of them
// positive; with KMX_VALIDATE=1 set when the context was created, X (n x d)
// and C (k x d, when given) must be finite too.  Synchronizes the context's
// stream when it launches anything; does nothing when w == NULL and the scan
// is off.
kmx_status check_data(kmx_ctx* ctx, const float* X, int64_t n, int d, int64_t ldx, const float* w,
                      int64_t min_pos, const float* C, int k) {
  const bool scan = ctx->validate;
  if (!w && !scan) return KMX_OK;
  KMX_TRY(grow(ctx, ctx->vcheck, 6 * sizeof(unsigned long long)));
  unsigned long long* v = P<unsigned long long>(ctx->vcheck);
  KMX_HIP(ctx, launch_fill_i32(ctx->stream, P<int32_t>(ctx->vcheck), 12, 0));
  if (w) KMX_HIP(ctx, launch_check_weights(ctx->stream, w, n, v, ctx->num_cus));
  if (scan) {
    KMX_HIP(ctx, launch_scan_finite(ctx->stream, X, n, d, ldx, v + 2, ctx->num_cus));
    if (C) KMX_HIP(ctx, launch_scan_finite(ctx->stream, C, k, d, d, v + 4, ctx->num_cus));
  }
  unsigned long long h[6];
  KMX_HIP(ctx, hipMemcpyAsync(h, v, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
  KMX_HIP(ctx, hipStreamSynchronize(ctx->stream));
  if (w && h[1] != 0)
    return fail(ctx, KMX_EINVAL, "w holds " + std::to_string(h[1]) +
                                     " entries that are negative or not finite");
  if (w && (int64_t)h[0] < min_pos)
    return fail(ctx, KMX_EINVAL, "k = " + std::to_string(min_pos) + " exceeds the number of rows "
                                 "with positive weight (" + std::to_string(h[0]) + ")");
  if (scan && h[3] != 0)
    return fail(ctx, KMX_EINVAL,
                "X holds " + std::to_string(h[3]) + " entries that are not finite (KMX_VALIDATE)");
  if (scan && C && h[5] != 0)
    return fail(ctx, KMX_EINVAL, "the centers hold " + std::to_string(h[5]) +
                                     " entries that are not finite (KMX_VALIDATE)");
  return KMX_OK;
}

// Row statistics and (BF16) the quantized copy of X, cached per dataset.  The
// BF16 preparation also serves the FP32 path (which only reads ||x||).
kmx_status ensure_prep(kmx_ctx* ctx, const float* X, int64_t n, int d, int64_t ldx, int prec) {
  if (d > kGemmMaxD) return KMX_OK;   // wide rows: no GEMM operands (see run_assign_gemm)
  if (prec == KMX_FP8E4M3) {
    KMX_TRY(ensure_prep(ctx, X, n, d, ldx, KMX_BF16));   // the cascade's BF16 pass
    if (ctx->cache8_valid && ctx->cache8_X == X && ctx->cache8_n == n && ctx->cache8_d == d &&
        ctx->cache8_ldx == ldx)
      return KMX_OK;
    ctx->cache8_valid = false;
    const int dp8 = assign_dpad(KMX_FP8E4M3, d);
    KMX_TRY(grow(ctx, ctx->rowstats8, (size_t)n * sizeof(RowStats)));
    KMX_TRY(grow(ctx, ctx->xstats8, 16));
    KMX_TRY(grow(ctx, ctx->xq8, (size_t)n * dp8));
    KMX_TRY(grow(ctx, ctx->sx8, (size_t)n));
    {
      Timed tm(ctx, T_PREP);
      KMX_HIP(ctx, launch_fill_i32(ctx->stream, P<int32_t>(ctx->xstats8), 4, 0));
      KMX_HIP(ctx, launch_prep_rows_f8(ctx->stream, X, n, d, ldx, dp8, P<uint8_t>(ctx->xq8),
                                       P<uint8_t>(ctx->sx8), P<RowStats>(ctx->rowstats8),
                                       P<unsigned>(ctx->xstats8), ctx->num_cus));
    }
    ctx->cache8_X = X;
    ctx->cache8_n = n;
    ctx->cache8_d = d;
    ctx->cache8_ldx = ldx;
    ctx->cache8_valid = true;
    return KMX_OK;
  }
  if (ctx->cache_valid && ctx->cache_X == X && ctx->cache_n == n && ctx->cache_d == d &&
      ctx->cache_ldx == ldx && (ctx->cache_prec == prec || ctx->cache_prec == KMX_BF16))
    return KMX_OK;
  ctx->cache_valid = false;
  KMX_TRY(grow(ctx, ctx->rowstats, (size_t)n * sizeof(RowStats)));
  KMX_TRY(grow(ctx, ctx->xstats, 16));
  uint16_t* xq = nullptr;
  const int dp = assign_dpad(prec, d);
  if (prec == KMX_BF16) {
    KMX_TRY(grow(ctx, ctx->xq, (size_t)n * dp * sizeof(uint16_t)));
    xq = P<uint16_t>(ctx->xq);
  }
  {
    Timed tm(ctx, T_PREP);
    KMX_HIP(ctx, launch_fill_i32(ctx->stream, P<int32_t>(ctx->xstats), 4, 0));
    KMX_HIP(ctx, launch_prep_rows(ctx->stream, X, n, d, ldx, dp, xq, P<RowStats>(ctx->rowstats),
                                  P<unsigned>(ctx->xstats), ctx->num_cus));
  }
  ctx->cache_X = X;
  ctx->cache_n = n;
  ctx->cache_d = d;
  ctx->cache_ldx = ldx;
  ctx->cache_prec = prec;
  ctx->cache_valid = true;
  return KMX_OK;
}

// Buffers of the assignment step alone (n rows, k centers).
kmx_status ensure_assign(kmx_ctx* ctx, int64_t n, int k) {
  (void)k;
  KMX_TRY(grow(ctx, ctx->state, sizeof(LoopState)));
  KMX_TRY(grow(ctx, ctx->lab_a, (size_t)n * sizeof(int32_t)));
  KMX_TRY(grow(ctx, ctx->flags, (size_t)n * sizeof(FlagEntry)));
  KMX_TRY(grow(ctx, ctx->cstats, sizeof(CenterStats)));
  KMX_TRY(grow(ctx, ctx->cstats32, sizeof(CenterStats)));
  KMX_TRY(grow(ctx, ctx->full_rows, (size_t)n * sizeof(int)));
  KMX_TRY(grow(ctx, ctx->full_rows2, (size_t)n * sizeof(int)));
  KMX_TRY(grow(ctx, ctx->cstats8, sizeof(CenterStats)));
  KMX_TRY(grow(ctx, ctx->brute, (size_t)n * sizeof(int)));
  return KMX_OK;
}

// Assignment plus update buffers.
kmx_status ensure_common(kmx_ctx* ctx, int64_t n, int d, int k) {
  const int64_t nb = (n + kSortRows - 1) / kSortRows;
  const int64_t maxchunks = (n + kReduceRows - 1) / kReduceRows + k;
  KMX_TRY(ensure_assign(ctx, n, k));
  // nb x k block counts, then the changed labels of each of the 4 nb hist waves
  KMX_TRY(grow(ctx, ctx->counts, ((size_t)nb * k + 4 * nb) * sizeof(int32_t)));
  KMX_TRY(grow(ctx, ctx->segsum, (size_t)kScanSegs * k * sizeof(int32_t)));
  KMX_TRY(grow(ctx, ctx->base, (size_t)(k + 1) * sizeof(int32_t)));
  KMX_TRY(grow(ctx, ctx->chunk_base, (size_t)(k + 1) * sizeof(int32_t)));
  KMX_TRY(grow(ctx, ctx->perm, (size_t)n * sizeof(int32_t)));
  KMX_TRY(grow(ctx, ctx->partS, (size_t)maxchunks * d * 2 * sizeof(double)));
  KMX_TRY(grow(ctx, ctx->partWQ, (size_t)maxchunks * 4 * sizeof(double)));
  KMX_TRY(grow(ctx, ctx->cfs, (size_t)(2 * d + 4) * sizeof(double)));
  KMX_TRY(grow(ctx, ctx->cf_wmax, 16));
  KMX_TRY(grow(ctx, ctx->cf_acc, ((size_t)k * d * 2 + (size_t)k * 4) * sizeof(long long)));
  KMX_TRY(grow(ctx, ctx->ecount, (size_t)(k + 1) * sizeof(int32_t)));
  KMX_TRY(grow(ctx, ctx->ebase, (size_t)(k + 1) * sizeof(int32_t)));
  KMX_TRY(grow(ctx, ctx->ecursor, (size_t)(k + 1) * sizeof(int32_t)));
  KMX_TRY(grow(ctx, ctx->dchunk, (size_t)(k + 1) * sizeof(int32_t)));
  KMX_TRY(grow(ctx, ctx->clist, (size_t)n * sizeof(int32_t)));
  KMX_TRY(grow(ctx, ctx->cold, (size_t)n * sizeof(int32_t)));
  KMX_TRY(grow(ctx, ctx->dent, (size_t)n * sizeof(int32_t)));
  KMX_TRY(grow(ctx, ctx->cfflag, 16));
  KMX_TRY(grow(ctx, ctx->W, (size_t)k * sizeof(double)));
  KMX_TRY(grow(ctx, ctx->termC, (size_t)k * sizeof(double)));
  KMX_TRY(grow(ctx, ctx->termMu, (size_t)k * sizeof(double)));
  return KMX_OK;
}

// Grids of the exactly summed clustering features: the dataset's column
// maxima and row norms (cached per dataset like the quantized copies), then
// the call's scales, which also depend on the largest weight.
kmx_status ensure_cf(kmx_ctx* ctx, const float* X, int64_t n, int d, int64_t ldx,
                     const float* w) {
  if (!(ctx->cf_valid && ctx->cf_X == X && ctx->cf_n == n && ctx->cf_d == d &&
        ctx->cf_ldx == ldx)) {
    ctx->cf_valid = false;
    KMX_TRY(grow(ctx, ctx->cf_colmax, (size_t)d * sizeof(unsigned)));
    KMX_TRY(grow(ctx, ctx->cf_q, (size_t)n * sizeof(double)));
    KMX_TRY(grow(ctx, ctx->cf_qmax, 16));
    Timed tm(ctx, T_PREP);
    KMX_HIP(ctx, launch_cf_prep(ctx->stream, X, n, d, ldx, P<unsigned>(ctx->cf_colmax),
                                P<double>(ctx->cf_q), P<unsigned long long>(ctx->cf_qmax),
                                ctx->num_cus));
    ctx->cf_X = X;
    ctx->cf_n = n;
    ctx->cf_d = d;
    ctx->cf_ldx = ldx;
    ctx->cf_valid = true;
  }
  KMX_HIP(ctx, launch_cf_scales(ctx->stream, P<unsigned>(ctx->cf_colmax), d,
                                P<unsigned long long>(ctx->cf_qmax), w, n,
                                P<unsigned>(ctx->cf_wmax), P<double>(ctx->cfs), ctx->num_cus));
  return KMX_OK;
}

// Start of a Lloyd run: no carried features, entry counts clear, previous
// labels unknown.
kmx_status begin_lloyd(kmx_ctx* ctx, int32_t* prev, int64_t n) {
  KMX_HIP(ctx, launch_fill_i32(ctx->stream, prev, n, -1));
  KMX_HIP(ctx, launch_fill_i32(ctx->stream, P<int32_t>(ctx->ecount), (int64_t)ctx->ecount.bytes / 4, 0));
  KMX_HIP(ctx, launch_fill_i32(ctx->stream, P<int32_t>(ctx->cfflag), 4, 1));
  return KMX_OK;
}

kmx_status write_state(kmx_ctx* ctx, int max_iter, double tol) {
  LoopState h;
  std::memset(&h, 0, sizeof(h));
  h.max_iter = max_iter;
  h.tol = tol;
  KMX_HIP(ctx, hipMemcpyAsync(ctx->state.p, &h, sizeof(h), hipMemcpyHostToDevice, ctx->stream));
  KMX_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return KMX_OK;
}

kmx_status run_prep_centers(kmx_ctx* ctx, const float* C, int k, int d, int prec) {
  LoopState* st = ST(ctx);
  CenterStats* cs = P<CenterStats>(ctx->cstats);
  CenterStats* cs32 = P<CenterStats>(ctx->cstats32);
  CenterStats* cs8 = P<CenterStats>(ctx->cstats8);
  if (d > kGemmMaxD) {   // wide rows: only the per-assignment counters
    KMX_HIP(ctx, launch_reset_small(ctx->stream, cs, cs32, cs8, st, 0));
    return KMX_OK;
  }
  // the FP32 path's operands, or those of the split-BF16 pass that ends the
  // BF16 and FP8 cascades (2 dp BF16 values per row: the same bytes)
  const int p32 = (prec == KMX_FP32) ? KMX_FP32 : kSplitBf16;
  const int dp32 = assign_dpad(p32, d);
  const int bn32 = assign_tile_n(p32, d, k);
  const int kpad32 = (k + bn32 - 1) / bn32 * bn32;
  KMX_TRY(grow(ctx, ctx->cq32, (size_t)kpad32 * dp32 * sizeof(float)));
  KMX_TRY(grow(ctx, ctx->ch32, (size_t)kpad32 * sizeof(float)));
  Timed tm(ctx, T_PREP);
  KMX_HIP(ctx, launch_reset_small(ctx->stream, cs, cs32, cs8, st, 0));
  KMX_HIP(ctx, launch_prep_centers(ctx->stream, C, k, d, kpad32, dp32, p32, ctx->cq32.p,
                                   P<float>(ctx->ch32), nullptr, cs32, nullptr));
  if (prec == KMX_BF16 || prec == KMX_FP8E4M3) {   // FP8 cascades into BF16
    const int dp = assign_dpad(KMX_BF16, d);
    const int bn = assign_tile_n(KMX_BF16, d, k);
    const int kpad = (k + bn - 1) / bn * bn;
    KMX_TRY(grow(ctx, ctx->cq, (size_t)kpad * dp * sizeof(uint16_t)));
    KMX_TRY(grow(ctx, ctx->ch, (size_t)kpad * sizeof(float)));
    KMX_TRY(grow(ctx, ctx->hd, (size_t)kpad * sizeof(double)));
    KMX_HIP(ctx, launch_prep_centers(ctx->stream, C, k, d, kpad, dp, KMX_BF16, ctx->cq.p,
                                     P<float>(ctx->ch), P<double>(ctx->hd), cs,
                                     P<unsigned>(ctx->xstats)));
  }
  if (prec == KMX_FP8E4M3) {
    const int dp = assign_dpad(KMX_FP8E4M3, d);
    const int bn = assign_tile_n(KMX_FP8E4M3, d, k);
    const int kpad = (k + bn - 1) / bn * bn;
    KMX_TRY(grow(ctx, ctx->cq8, (size_t)kpad * dp));
    KMX_TRY(grow(ctx, ctx->ch8, (size_t)kpad * sizeof(float)));
    KMX_TRY(grow(ctx, ctx->hd8, (size_t)kpad * sizeof(double)));
    KMX_HIP(ctx, launch_prep_centers(ctx->stream, C, k, d, kpad, dp, KMX_FP8E4M3, ctx->cq8.p,
                                     P<float>(ctx->ch8), P<double>(ctx->hd8), cs8,
                                     P<unsigned>(ctx->xstats8)));
  }
  return KMX_OK;
}

// GEMM passes: FP8 (rows with more than three centers inside its bound to
// the BF16 pass), BF16 (likewise to the split-BF16 pass; a short list with
// long centers, see kShortList, goes to the every-center re-check instead),
// split BF16 (rows still open to the every-center re-check); rows with two or
// three candidates inside a pass's bound go to the short re-check.  With
// KMX_FP32 one FP32 pass.  gate: skip when *gate != 0.
kmx_status run_assign_gemm(kmx_ctx* ctx, const float* X, int64_t n, int d, int64_t ldx,
                           const float* C, int k, int prec, int32_t* label, float* d1,
                           float* d2, const int* rows, const unsigned long long* row_count,
                           const int* gate, BoundsOut bo) {
  LoopState* st = ST(ctx);
  if (d > kGemmMaxD) {
    // Rows wider than the GEMM's register-resident point fragments: every row
    // (or every listed row) goes to the every-center re-check, which computes
    // the plain FP32 distances to all centers and decides the candidates
    // within their error bound by double-float sums (exact labels).
    ctx->last_prec = prec;
    Timed tm(ctx, T_RECHECK);
    KMX_HIP(ctx, launch_list_all(ctx->stream, P<int>(ctx->brute), n, rows, row_count, st, gate));
    KMX_HIP(ctx, launch_recheck(ctx->stream, X, n, d, ldx, C, k, label, d1, P<FlagEntry>(ctx->flags),
                                P<int>(ctx->brute), st, ctx->num_cus, gate, bo, d2));
    return KMX_OK;
  }
  CenterStats* cs = P<CenterStats>(ctx->cstats);
  CenterStats* cs32 = P<CenterStats>(ctx->cstats32);
  CenterStats* cs8 = P<CenterStats>(ctx->cstats8);
  // operands of the FP32 path, or of the split-BF16 pass of the cascades
  // (prepared by run_prep_centers for the same precision)
  const int p32 = (prec == KMX_FP32) ? KMX_FP32 : kSplitBf16;
  const int dp32 = assign_dpad(p32, d);
  const int bn32 = assign_tile_n(p32, d, k);
  const int kpad32 = (k + bn32 - 1) / bn32 * bn32;
  const RowStats* rs = P<RowStats>(ctx->rowstats);
  FlagEntry* flags = P<FlagEntry>(ctx->flags);
  int* brute = P<int>(ctx->brute);
  ctx->last_prec = prec;
  if (prec == KMX_FP32) {
    Timed tm(ctx, T_ASSIGN);
    KMX_HIP(ctx, launch_assign(ctx->stream, KMX_FP32, X, ldx, nullptr, nullptr, n, rows,
                               row_count, d, dp32, rs, ctx->cq32.p, P<float>(ctx->ch32), k,
                               kpad32, cs32, label, d1, d2, flags, nullptr, nullptr, 0, brute,
                               st, gate, ctx->num_cus, bo));
  } else {
    const int dp = assign_dpad(KMX_BF16, d);
    const int bn = assign_tile_n(KMX_BF16, d, k);
    const int kpad = (k + bn - 1) / bn * bn;
    // rows the BF16 pass covers, and where it sends rows for the FP32 pass
    const int* rows16 = rows;
    const unsigned long long* cnt16 = row_count;
    int* next16 = P<int>(ctx->full_rows);
    unsigned long long* ctr16 = &st->full_count;
    if (prec == KMX_FP8E4M3) {
      const int dp8 = assign_dpad(KMX_FP8E4M3, d);
      const int bn8 = assign_tile_n(KMX_FP8E4M3, d, k);
      const int kpad8 = (k + bn8 - 1) / bn8 * bn8;
      Timed tm(ctx, T_ASSIGN);
      KMX_HIP(ctx, launch_assign(ctx->stream, KMX_FP8E4M3, X, ldx, ctx->xq8.p,
                                 P<uint8_t>(ctx->sx8), n, rows, row_count, d, dp8,
                                 P<RowStats>(ctx->rowstats8), ctx->cq8.p, P<float>(ctx->ch8), k,
                                 kpad8, cs8, label, d1, d2, flags, P<int>(ctx->full_rows),
                                 &st->full_count, 0, brute, st, gate, ctx->num_cus, bo));
      rows16 = P<int>(ctx->full_rows);
      cnt16 = &st->full_count;
      next16 = P<int>(ctx->full_rows2);
      ctr16 = &st->full_count2;
    }
    {
      Timed tm(ctx, prec == KMX_FP8E4M3 ? T_RECHECK : T_ASSIGN);
      KMX_HIP(ctx, launch_assign(ctx->stream, KMX_BF16, X, ldx, ctx->xq.p, nullptr, n, rows16,
                                 cnt16, d, dp, rs, ctx->cq.p, P<float>(ctx->ch), k, kpad, cs,
                                 label, d1, d2,
                                 flags, next16, ctr16, 0, brute, st, gate, ctx->num_cus, bo));
    }
    {
      Timed tm(ctx, T_RECHECK);
      KMX_HIP(ctx, launch_route_small(ctx->stream, ctr16, next16, brute, st, k, d, gate));
      KMX_HIP(ctx, launch_assign(ctx->stream, kSplitBf16, X, ldx, nullptr, nullptr, n, next16,
                                 ctr16, d, dp32, rs, ctx->cq32.p, P<float>(ctx->ch32), k, kpad32,
                                 cs32, label, d1, d2, flags, nullptr, nullptr, 0, brute, st, gate,
                                 ctx->num_cus, bo));
    }
  }
  {
    Timed tm(ctx, T_SHORT);
    KMX_HIP(ctx, launch_recheck(ctx->stream, X, n, d, ldx, C, k, label, d1, flags, brute, st,
                                ctx->num_cus, gate, bo));
  }
  return KMX_OK;
}

kmx_status run_assign(kmx_ctx* ctx, const float* X, int64_t n, int d, int64_t ldx, const float* C,
                      int k, int prec, int32_t* label, float* d1, float* d2, const int* gate) {
  KMX_TRY(run_prep_centers(ctx, C, k, d, prec));
  return run_assign_gemm(ctx, X, n, d, ldx, C, k, prec, label, d1, d2, nullptr, nullptr, gate);
}

// Update step: finalize + cost sums after a full reduction (sort by label,
// then every row) or, with lab_prev, after whichever of the full and the
// delta reduction the device-side plan picks (the rows whose label differs
// from lab_prev, added to the features carried from the previous update).
kmx_status run_update(kmx_ctx* ctx, const float* X, int64_t n, int d, int64_t ldx, const float* w,
                      const int32_t* label, int k, const float* C_prev, float* C_out,
                      double* W_out, int write_c, int32_t* lab_prev, double* hist, int mode,
                      const int* gate) {
  LoopState* st = ST(ctx);
  int* flags = P<int>(ctx->cfflag);
  const int* gate_full = lab_prev ? flags : gate;
  {
    Timed tm(ctx, T_SORT);
    if (lab_prev)
      KMX_HIP(ctx, launch_delta_prepare(ctx->stream, label, lab_prev, n, k,
                                        P<int32_t>(ctx->ecount), P<int32_t>(ctx->clist),
                                        P<int32_t>(ctx->cold), P<int32_t>(ctx->ebase),
                                        P<int32_t>(ctx->ecursor), P<int32_t>(ctx->dchunk),
                                        P<int32_t>(ctx->dent), flags, st, ctx->num_cus, gate));
    KMX_HIP(ctx, launch_sort(ctx->stream, label, nullptr, n, k, P<int32_t>(ctx->counts),
                             P<int32_t>(ctx->segsum), P<int32_t>(ctx->base),
                             P<int32_t>(ctx->chunk_base), P<int32_t>(ctx->perm), st, 0,
                             gate_full));
  }
  {
    Timed tm(ctx, T_REDUCE);
    KMX_HIP(ctx, launch_reduce(ctx->stream, X, n, d, ldx, w, P<double>(ctx->cf_q),
                               P<int32_t>(ctx->perm), P<int32_t>(ctx->base),
                               P<int32_t>(ctx->chunk_base), k, P<double>(ctx->cfs),
                               P<double>(ctx->partS), P<double>(ctx->partWQ), 0, ctx->num_cus,
                               gate_full));
    if (lab_prev)
      KMX_HIP(ctx, launch_reduce(ctx->stream, X, n, d, ldx, w, P<double>(ctx->cf_q),
                                 P<int32_t>(ctx->dent), P<int32_t>(ctx->ebase),
                                 P<int32_t>(ctx->dchunk), k, P<double>(ctx->cfs),
                                 P<double>(ctx->partS), P<double>(ctx->partWQ), 1, ctx->num_cus,
                                 flags + 1));
  }
  {
    Timed tm(ctx, T_FINAL);
    KMX_HIP(ctx, launch_finalize(ctx->stream, P<double>(ctx->partS), P<double>(ctx->partWQ),
                                 P<int32_t>(ctx->chunk_base), P<int32_t>(ctx->dchunk),
                                 lab_prev ? flags + 2 : nullptr,
                                 lab_prev ? P<long long>(ctx->cf_acc) : nullptr, k, d,
                                 P<double>(ctx->cfs), C_prev, C_out,
                                 W_out ? W_out : P<double>(ctx->W), P<double>(ctx->termC),
                                 P<double>(ctx->termMu), write_c, st, gate));
    KMX_HIP(ctx, launch_cost_sum(ctx->stream, P<double>(ctx->termC), P<double>(ctx->termMu), k,
                                 st, hist, mode, gate));
  }
  return KMX_OK;
}

}  // namespace host
}  // namespace kmx

extern "C" {

kmx_status kmx_create(kmx_ctx** out, int device, void* hip_stream) {
  if (!out) return fail(nullptr, KMX_EINVAL, "out is NULL");
  *out = nullptr;
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev < 1) {
    (void)hipGetLastError();
    return fail(nullptr, KMX_EDEVICE, "no HIP device available");
  }
  if (device < 0 || device >= ndev) return fail(nullptr, KMX_EINVAL, "device index out of range");
  e = hipSetDevice(device);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(nullptr, KMX_EDEVICE, std::string("hipSetDevice: ") + hipGetErrorString(e));
  }
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, device);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(nullptr, KMX_EDEVICE, "hipGetDeviceProperties failed");
  }
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(nullptr, KMX_EUNSUPPORTED,
                std::string("the library is compiled for gfx950, device is ") + prop.gcnArchName);
  void* na = nullptr;
  e = noalloc_init(device, &na);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(nullptr, KMX_EDEVICE,
                std::string("address of the static scratch array: ") + hipGetErrorString(e));
  }
  kmx_ctx* c = new (std::nothrow) kmx_ctx();
  if (!c) return fail(nullptr, KMX_ENOMEM, "out of host memory");
  c->na_scratch = na;
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  c->num_cus = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  const char* val = std::getenv("KMX_VALIDATE");
  c->validate = val && val[0] && std::strcmp(val, "0") != 0;
  *out = c;
  return KMX_OK;
}

kmx_status kmx_destroy(kmx_ctx* ctx) {
  if (!ctx) return KMX_EINVAL;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  kmx::Buf* bufs[] = {
      &ctx->xq,        &ctx->xstats,   &ctx->hd,         &ctx->cq32,       &ctx->ch32,
      &ctx->cstats32,  &ctx->full_rows, &ctx->brute,     &ctx->rowstats,   &ctx->cq,
      &ctx->ch,        &ctx->cstats,   &ctx->lab_a,      &ctx->lab_prev,   &ctx->d1,
      &ctx->d2,        &ctx->flags,    &ctx->counters,   &ctx->counts,     &ctx->segsum,
      &ctx->base,      &ctx->chunk_base, &ctx->perm,     &ctx->partS,      &ctx->partWQ,
      &ctx->cf_colmax, &ctx->cf_q,     &ctx->cf_qmax,    &ctx->cf_wmax,    &ctx->cfs,
      &ctx->cf_acc,    &ctx->ecount,   &ctx->ebase,      &ctx->ecursor,    &ctx->dchunk,
      &ctx->clist,     &ctx->cold,     &ctx->dent,       &ctx->cfflag,
      &ctx->W,        &ctx->termC,      &ctx->termMu,     &ctx->state,     &ctx->vcheck,    &ctx->hub,
      &ctx->hlb,       &ctx->hl2,      &ctx->hsec,       &ctx->bl_rows,  &ctx->cprev,      &ctx->drift,      &ctx->dstat,
      &ctx->bkh,
      &ctx->D2,        &ctx->chosen,   &ctx->seed_part,  &ctx->seed_ctr,   &ctx->scratch_c,
      &ctx->seed_a,    &ctx->seed_cc,  &ctx->seed_nread,
      &ctx->bs_D2,     &ctx->bs_sa,    &ctx->bs_cc,      &ctx->bs_chosen,  &ctx->bs_part,
      &ctx->bs_ctr,    &ctx->bs_insts,
      &ctx->hist,      &ctx->fb_rows,  &ctx->keys,       &ctx->cdist,      &ctx->nbr,
      &ctx->nbd,       &ctx->fbh,      &ctx->prop_have,  &ctx->prop_rows,      &ctx->xq8,        &ctx->sx8,        &ctx->rowstats8,
      &ctx->xstats8,   &ctx->cq8,      &ctx->ch8,        &ctx->hd8,        &ctx->cstats8,
      &ctx->full_rows2, &ctx->bX,       &ctx->bXq,        &ctx->brs,        &ctx->bw,
      &ctx->bC,        &ctx->bCq,      &ctx->bhd,        &ctx->bch,        &ctx->vt,        &ctx->bcs,        &ctx->blab,
      &ctx->sv_om,     &ctx->sv_y,     &ctx->sv_y2,      &ctx->sv_z,       &ctx->sv_g,      &ctx->sv_part,
      &ctx->sv_r,      &ctx->sv_v,
      &ctx->bitems,    &ctx->binsts,   &ctx->bbuckets,   &ctx->bcinst,     &ctx->bxstats,
      &ctx->btermC,    &ctx->btermMu,  &ctx->bW,         &ctx->bcost,      &ctx->bcf_colmax,
      &ctx->bcf_q,     &ctx->bcf_qmax, &ctx->bcf_wmax,   &ctx->bcfs};
  for (kmx::Buf* b : bufs)
    if (b->p) (void)hipFree(b->p);
  if (ctx->lg_exec) (void)hipGraphExecDestroy(ctx->lg_exec);
  if (ctx->lg_graph) (void)hipGraphDestroy(ctx->lg_graph);
  if (ctx->lg_event) (void)hipEventDestroy(ctx->lg_event);
  if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
  for (auto& r : ctx->recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (hipEvent_t e : ctx->pool) (void)hipEventDestroy(e);
  delete ctx;
  return KMX_OK;
}

kmx_status kmx_set_stream(kmx_ctx* ctx, void* hip_stream) {
  if (!ctx) return KMX_EINVAL;
  ctx->stream = (hipStream_t)hip_stream;
  return KMX_OK;
}

kmx_status kmx_invalidate(kmx_ctx* ctx, const float* X) {
  if (!ctx) return KMX_EINVAL;
  if (X == nullptr || ctx->cache_X == X) ctx->cache_valid = false;
  if (X == nullptr || ctx->cache8_X == X) ctx->cache8_valid = false;
  if (X == nullptr || ctx->cf_X == X) ctx->cf_valid = false;
  ctx->batch_key.clear();   // the batched path's grouped copies of any problem
  return KMX_OK;
}

const char* kmx_last_error(const kmx_ctx* ctx) {
  return ctx ? ctx->err.c_str() : g_create_err.c_str();
}

kmx_status kmx_seed(kmx_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx,
                    const float* w, int32_t k, uint64_t rng_seed, float* C_out,
                    int64_t* idx_out) {
  if (!ctx) return KMX_EINVAL;
  ctx->err.clear();
  KMX_TRY(check_problem(ctx, X, n, d, ldx, k));
  if (!C_out) return fail(ctx, KMX_EINVAL, "C_out is NULL");
  KMX_TRY(set_device(ctx));
  KMX_TRY(check_data(ctx, X, n, d, ldx, w, k, nullptr, 0));
  const int64_t nb = (n + kSeedRows - 1) / kSeedRows;
  KMX_TRY(grow(ctx, ctx->D2, (size_t)n * sizeof(double)));
  KMX_TRY(grow(ctx, ctx->chosen, (size_t)n));
  KMX_TRY(grow(ctx, ctx->seed_part, (size_t)nb * sizeof(double)));
  KMX_TRY(grow(ctx, ctx->seed_ctr, 16));   // ticket (4 bytes), rows read (8 bytes at 8)
  KMX_TRY(grow(ctx, ctx->seed_a, (size_t)n * sizeof(int32_t)));
  KMX_TRY(grow(ctx, ctx->seed_cc, (size_t)k * sizeof(double)));
  KMX_TRY(grow(ctx, ctx->seed_nread, (size_t)nb * sizeof(int)));
  Timed tm(ctx, T_SEED);
  KMX_HIP(ctx, launch_fill_u8(ctx->stream, P<uint8_t>(ctx->chosen), n, 0));
  KMX_HIP(ctx, launch_fill_i32(ctx->stream, P<int32_t>(ctx->seed_ctr), 4, 0));
  for (int r = 0; r < k; ++r) {
    KMX_HIP(ctx, launch_seed_round(ctx->stream, X, n, d, ldx, w, r, rng_seed, P<double>(ctx->D2),
                                   P<uint8_t>(ctx->chosen), P<double>(ctx->seed_part),
                                   P<unsigned int>(ctx->seed_ctr), C_out, idx_out,
                                   P<int32_t>(ctx->seed_a), P<double>(ctx->seed_cc),
                                   P<int>(ctx->seed_nread),
                                   (unsigned long long*)(P<unsigned char>(ctx->seed_ctr) + 8)));
  }
  return KMX_OK;
}

kmx_status kmx_seed_batched(kmx_ctx* ctx, const kmx_problem* probs, int32_t count,
                            const uint64_t* rng_seeds, int64_t* idx_out) {
  if (!ctx) return KMX_EINVAL;
  ctx->err.clear();
  if (count < 1 || !probs || !rng_seeds)
    return fail(ctx, KMX_EINVAL, "count must be >= 1 with probs and rng_seeds given");
  for (int i = 0; i < count; ++i) {
    const kmx_problem& q = probs[i];
    const kmx_status st = check_problem(ctx, q.X, q.n, q.d, q.ldx, q.k);
    if (st != KMX_OK) return fail(ctx, st, "problem " + std::to_string(i) + ": " + ctx->err);
    if (!q.C) return fail(ctx, KMX_EINVAL, "problem " + std::to_string(i) + ": C is NULL");
  }
  KMX_TRY(set_device(ctx));
  for (int i = 0; i < count; ++i) {
    const kmx_problem& q = probs[i];
    const kmx_status st = check_data(ctx, q.X, q.n, q.d, q.ldx, q.w, q.k, nullptr, 0);
    if (st != KMX_OK) return fail(ctx, st, "problem " + std::to_string(i) + ": " + ctx->err);
  }
  // instances by decreasing k (ties: problem order), so round r's active
  // instances and their blocks are prefixes
  std::vector<int> ord(count);
  for (int i = 0; i < count; ++i) ord[i] = i;
  std::stable_sort(ord.begin(), ord.end(),
                   [&](int a, int b) { return probs[a].k > probs[b].k; });
  std::vector<int64_t> koff(count + 1, 0);
  for (int i = 0; i < count; ++i) koff[i + 1] = koff[i] + probs[i].k;
  int64_t sn = 0, snb = 0;
  for (int i = 0; i < count; ++i) {
    sn += probs[i].n;
    snb += (probs[i].n + kSeedRows - 1) / kSeedRows;
  }
  KMX_TRY(grow(ctx, ctx->bs_D2, (size_t)sn * sizeof(double)));
  KMX_TRY(grow(ctx, ctx->bs_sa, (size_t)sn * sizeof(int32_t)));
  KMX_TRY(grow(ctx, ctx->bs_cc, (size_t)koff[count] * sizeof(double)));
  KMX_TRY(grow(ctx, ctx->bs_chosen, (size_t)sn));
  KMX_TRY(grow(ctx, ctx->bs_part, (size_t)snb * sizeof(double)));
  KMX_TRY(grow(ctx, ctx->bs_ctr, (size_t)count * sizeof(unsigned int)));
  KMX_TRY(grow(ctx, ctx->bs_insts, (size_t)count * sizeof(SeedInst)));
  std::vector<SeedInst> h(count);
  int64_t off = 0, boff = 0;
  for (int t = 0; t < count; ++t) {
    const int i = ord[t];
    const kmx_problem& q = probs[i];
    SeedInst& I = h[t];
    I.X = q.X;
    I.w = q.w;
    I.C = q.C;
    I.idx = idx_out ? idx_out + koff[i] : nullptr;
    I.D2 = P<double>(ctx->bs_D2) + off;
    I.sa = P<int32_t>(ctx->bs_sa) + off;
    I.cc2 = P<double>(ctx->bs_cc) + koff[i];
    I.chosen = P<uint8_t>(ctx->bs_chosen) + off;
    I.nb = (int)((q.n + kSeedRows - 1) / kSeedRows);
    I.part = P<double>(ctx->bs_part) + boff;
    I.ctr = P<unsigned int>(ctx->bs_ctr) + t;
    I.n = q.n;
    I.ldx = q.ldx;
    I.blk0 = boff;
    I.seed = rng_seeds[i];
    I.d = q.d;
    I.k = q.k;
    off += q.n;
    boff += I.nb;
  }
  Timed tm(ctx, T_SEED);
  KMX_HIP(ctx, hipMemcpyAsync(ctx->bs_insts.p, h.data(), (size_t)count * sizeof(SeedInst),
                              hipMemcpyHostToDevice, ctx->stream));
  KMX_HIP(ctx, launch_fill_u8(ctx->stream, P<uint8_t>(ctx->bs_chosen), sn, 0));
  KMX_HIP(ctx, launch_fill_i32(ctx->stream, P<int32_t>(ctx->bs_ctr), count, 0));
  const int kmax = h[0].k;
  int m = count;
  for (int r = 0; r < kmax; ++r) {
    while (m > 0 && h[m - 1].k <= r) --m;   // instances with k > r
    const int64_t blocks = h[m - 1].blk0 + h[m - 1].nb;
    KMX_HIP(ctx, launch_seed_batched_gaps(ctx->stream, P<SeedInst>(ctx->bs_insts), m, r));
    KMX_HIP(ctx, launch_seed_batched_round(ctx->stream, P<SeedInst>(ctx->bs_insts), m, r, blocks));
  }
  // the host descriptors must outlive their copy
  KMX_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return KMX_OK;
}

kmx_status kmx_seed_stats(kmx_ctx* ctx, int64_t* rows_read) {
  if (!ctx) return KMX_EINVAL;
  ctx->err.clear();
  if (!rows_read) return fail(ctx, KMX_EINVAL, "rows_read is NULL");
  *rows_read = 0;
  if (!ctx->seed_ctr.p) return KMX_OK;
  KMX_TRY(set_device(ctx));
  unsigned long long h = 0;
  KMX_HIP(ctx, hipMemcpyAsync(&h, P<unsigned char>(ctx->seed_ctr) + 8, sizeof(h),
                              hipMemcpyDeviceToHost, ctx->stream));
  KMX_HIP(ctx, hipStreamSynchronize(ctx->stream));
  *rows_read = (int64_t)h;
  return KMX_OK;
}

kmx_status kmx_assign(kmx_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx,
                      const float* C, int32_t k, kmx_prec prec, int32_t* label_out, float* d1_out,
                      float* d2_out, int64_t* n_flagged) {
  if (!ctx) return KMX_EINVAL;
  ctx->err.clear();
  KMX_TRY(check_problem(ctx, X, n, d, ldx, k));
  KMX_TRY(check_prec(ctx, prec, d, true));
  if (!C) return fail(ctx, KMX_EINVAL, "C is NULL");
  if (!label_out) return fail(ctx, KMX_EINVAL, "label_out is NULL");
  KMX_TRY(set_device(ctx));
  KMX_TRY(check_data(ctx, X, n, d, ldx, nullptr, 0, C, k));
  KMX_TRY(ensure_assign(ctx, n, k));
  KMX_TRY(ensure_prep(ctx, X, n, d, ldx, prec));
  KMX_TRY(run_assign(ctx, X, n, d, ldx, C, k, prec, label_out, d1_out, d2_out, nullptr));
  if (n_flagged) {
    LoopState h;
    KMX_HIP(ctx, hipMemcpyAsync(&h, ctx->state.p, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
    KMX_HIP(ctx, hipStreamSynchronize(ctx->stream));
    *n_flagged = (int64_t)h.undecided;
  }
  return KMX_OK;
}

kmx_status kmx_update(kmx_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx,
                      const float* w, const int32_t* label, int32_t k, const float* C_prev,
                      float* C_out, double* W_out, double* cost_at_centroids) {
  if (!ctx) return KMX_EINVAL;
  ctx->err.clear();
  if (!X) return fail(ctx, KMX_EINVAL, "X is NULL");
  if (n < 1 || n > (int64_t)INT32_MAX - 1) return fail(ctx, KMX_EINVAL, "n out of range");
  if (d < 1 || ldx < d) return fail(ctx, KMX_EINVAL, "bad d or ldx");
  if (k < 1) return fail(ctx, KMX_EINVAL, "k must be >= 1");
  if (k > kMaxK) return fail(ctx, KMX_EUNSUPPORTED, "k too large");
  if (!label || !C_prev || !C_out) return fail(ctx, KMX_EINVAL, "NULL label or centers");
  KMX_TRY(set_device(ctx));
  if (ctx->validate) KMX_TRY(check_data(ctx, X, n, d, ldx, w, 0, C_prev, k));
  KMX_TRY(ensure_common(ctx, n, d, k));
  KMX_TRY(ensure_cf(ctx, X, n, d, ldx, w));
  KMX_TRY(run_update(ctx, X, n, d, ldx, w, label, k, C_prev, C_out, W_out, 1, nullptr, nullptr, 2,
                     nullptr));
  if (cost_at_centroids) {
    LoopState h;
    KMX_HIP(ctx, hipMemcpyAsync(&h, ctx->state.p, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
    KMX_HIP(ctx, hipStreamSynchronize(ctx->stream));
    *cost_at_centroids = h.cost_at_centroids;
  }
  return KMX_OK;
}

kmx_status kmx_cost(kmx_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx,
                    const float* w, const float* C, int32_t k, kmx_prec prec, double* cost_out) {
  if (!ctx) return KMX_EINVAL;
  ctx->err.clear();
  KMX_TRY(check_problem(ctx, X, n, d, ldx, k));
  KMX_TRY(check_prec(ctx, prec, d, true));
  if (!C || !cost_out) return fail(ctx, KMX_EINVAL, "NULL C or cost_out");
  KMX_TRY(set_device(ctx));
  KMX_TRY(check_data(ctx, X, n, d, ldx, w, 0, C, k));
  KMX_TRY(ensure_common(ctx, n, d, k));
  KMX_TRY(ensure_prep(ctx, X, n, d, ldx, prec));
  KMX_TRY(ensure_cf(ctx, X, n, d, ldx, w));
  int32_t* lab = P<int32_t>(ctx->lab_a);
  KMX_TRY(run_assign(ctx, X, n, d, ldx, C, k, prec, lab, nullptr, nullptr, nullptr));
  KMX_TRY(run_update(ctx, X, n, d, ldx, w, lab, k, C, nullptr, nullptr, 0, nullptr, nullptr, 2,
                     nullptr));
  LoopState h;
  KMX_HIP(ctx, hipMemcpyAsync(&h, ctx->state.p, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
  KMX_HIP(ctx, hipStreamSynchronize(ctx->stream));
  *cost_out = h.cost_last;
  return KMX_OK;
}

// The Lloyd loop; with graph != 0 one iteration is captured as a HIP graph on
// the context's capture stream and replayed max_iter times (the iterations
// are gated on the device by the stop flag, so the host never waits inside
// the loop either way).
static kmx_status lloyd_impl(kmx_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx,
                             const float* w, float* C_inout, int32_t k, int32_t max_iter,
                             double tol, kmx_prec prec, int32_t* label_out, double* cost_hist,
                             int32_t* iters_done, int graph) {
  if (!ctx) return KMX_EINVAL;
  ctx->err.clear();
  KMX_TRY(check_problem(ctx, X, n, d, ldx, k));
  KMX_TRY(check_prec(ctx, prec, d, true));
  if (!C_inout || !cost_hist || !iters_done)
    return fail(ctx, KMX_EINVAL, "NULL C_inout, cost_hist or iters_done");
  if (max_iter < 0) return fail(ctx, KMX_EINVAL, "max_iter must be >= 0");
  KMX_TRY(set_device(ctx));
  KMX_TRY(check_data(ctx, X, n, d, ldx, w, 0, C_inout, k));
  KMX_TRY(ensure_common(ctx, n, d, k));
  KMX_TRY(ensure_prep(ctx, X, n, d, ldx, prec));
  KMX_TRY(grow(ctx, ctx->lab_prev, (size_t)n * sizeof(int32_t)));
  KMX_TRY(grow(ctx, ctx->hist, (size_t)(max_iter + 1) * sizeof(double)));
  KMX_TRY(ensure_cf(ctx, X, n, d, ldx, w));
  KMX_TRY(write_state(ctx, max_iter, tol));
  int32_t* lab = label_out ? label_out : P<int32_t>(ctx->lab_a);
  int32_t* prev = P<int32_t>(ctx->lab_prev);
  double* hist = P<double>(ctx->hist);
  LoopState* st = ST(ctx);
  KMX_TRY(begin_lloyd(ctx, prev, n));
  if (graph && max_iter > 0) {
    // every buffer an iteration touches exists before the capture starts
    KMX_TRY(run_prep_centers(ctx, C_inout, k, d, prec));
    if (!ctx->cap_stream)
      KMX_HIP(ctx, hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
    hipStream_t cs = ctx->cap_stream;
    // the captured iteration depends on these pointers and sizes only (the
    // loop state is read by its kernels), so it is kept for the next call
    const uint64_t key[12] = {(uint64_t)(uintptr_t)X, (uint64_t)n, (uint64_t)d, (uint64_t)ldx,
                              (uint64_t)(uintptr_t)w, (uint64_t)(uintptr_t)C_inout, (uint64_t)k,
                              (uint64_t)prec, (uint64_t)(uintptr_t)lab, ctx->ws_gen,
                              (uint64_t)(uintptr_t)cs, 1};
    if (!ctx->lg_event)
      KMX_HIP(ctx, hipEventCreateWithFlags(&ctx->lg_event, hipEventDisableTiming));
    KMX_HIP(ctx, hipEventRecord(ctx->lg_event, ctx->stream));
    KMX_HIP(ctx, hipStreamWaitEvent(cs, ctx->lg_event, 0));
    const bool cached = ctx->lg_exec && std::memcmp(key, ctx->lg_key, sizeof(key)) == 0;
    if (!cached) {
      if (ctx->lg_exec) (void)hipGraphExecDestroy(ctx->lg_exec);
      if (ctx->lg_graph) (void)hipGraphDestroy(ctx->lg_graph);
      ctx->lg_exec = nullptr;
      ctx->lg_graph = nullptr;
      // the iteration's launches go to the capture stream; no event timing inside
      const hipStream_t saved = ctx->stream;
      const int saved_timing = ctx->timing;
      ctx->stream = cs;
      ctx->timing = 0;
      hipGraph_t g = nullptr;
      kmx_status ks = KMX_OK;
      hipError_t he = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
      if (he == hipSuccess) {
        ks = run_assign(ctx, X, n, d, ldx, C_inout, k, prec, lab, nullptr, nullptr, &st->done);
        if (ks == KMX_OK)
          ks = run_update(ctx, X, n, d, ldx, w, lab, k, C_inout, C_inout, nullptr, 1, prev, hist,
                          0, &st->done);
        const hipError_t he2 = hipStreamEndCapture(cs, &g);
        if (he == hipSuccess) he = he2;
      }
      ctx->stream = saved;
      ctx->timing = saved_timing;
      hipGraphExec_t ge = nullptr;
      if (he == hipSuccess && ks == KMX_OK) he = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
      if (ks != KMX_OK || he != hipSuccess) {
        if (ge) (void)hipGraphExecDestroy(ge);
        if (g) (void)hipGraphDestroy(g);
        if (ks != KMX_OK) return ks;
        (void)hipGetLastError();
        return fail(ctx, KMX_EDEVICE,
                    std::string("graph of the Lloyd iteration: ") + hipGetErrorString(he));
      }
      ctx->lg_graph = g;
      ctx->lg_exec = ge;
      std::memcpy(ctx->lg_key, key, sizeof(key));
    }
    for (int t = 0; t < max_iter; ++t) KMX_HIP(ctx, hipGraphLaunch(ctx->lg_exec, cs));
    KMX_HIP(ctx, hipEventRecord(ctx->lg_event, cs));
    KMX_HIP(ctx, hipStreamWaitEvent(ctx->stream, ctx->lg_event, 0));
  } else {
    for (int t = 0; t < max_iter; ++t) {
      KMX_TRY(run_assign(ctx, X, n, d, ldx, C_inout, k, prec, lab, nullptr, nullptr, &st->done));
      KMX_TRY(run_update(ctx, X, n, d, ldx, w, lab, k, C_inout, C_inout, nullptr, 1, prev, hist,
                         0, &st->done));
    }
  }
  // final assignment: labels and cost of the returned centers (the features
  // of its labels come from the last update's by the rows that changed)
  KMX_TRY(run_assign(ctx, X, n, d, ldx, C_inout, k, prec, lab, nullptr, nullptr, nullptr));
  KMX_TRY(run_update(ctx, X, n, d, ldx, w, lab, k, C_inout, nullptr, nullptr, 0, prev, hist, 1,
                     nullptr));
  LoopState h;
  KMX_HIP(ctx, hipMemcpyAsync(&h, ctx->state.p, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
  KMX_HIP(ctx, hipStreamSynchronize(ctx->stream));
  const int it = h.iter;
  KMX_HIP(ctx, hipMemcpy(cost_hist, hist, (size_t)(it + 1) * sizeof(double),
                         hipMemcpyDeviceToHost));
  *iters_done = it;
  return KMX_OK;
}

kmx_status kmx_lloyd(kmx_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx,
                     const float* w, float* C_inout, int32_t k, int32_t max_iter, double tol,
                     kmx_prec prec, int32_t* label_out, double* cost_hist, int32_t* iters_done) {
  return lloyd_impl(ctx, X, n, d, ldx, w, C_inout, k, max_iter, tol, prec, label_out, cost_hist,
                    iters_done, 0);
}

kmx_status kmx_lloyd_graph(kmx_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx,
                           const float* w, float* C_inout, int32_t k, int32_t max_iter,
                           double tol, kmx_prec prec, int32_t* label_out, double* cost_hist,
                           int32_t* iters_done) {
  return lloyd_impl(ctx, X, n, d, ldx, w, C_inout, k, max_iter, tol, prec, label_out, cost_hist,
                    iters_done, 1);
}

kmx_status kmx_project(kmx_ctx* ctx, const float* X, int64_t rows, int32_t d_in, int64_t ldx,
                       const float* V, int32_t d_out, float* Y, int64_t ldy) {
  if (!ctx) return KMX_EINVAL;
  ctx->err.clear();
  if (!X || !V || !Y) return fail(ctx, KMX_EINVAL, "NULL X, V or Y");
  if (rows < 1 || d_in < 1 || ldx < d_in) return fail(ctx, KMX_EINVAL, "bad rows, d_in or ldx");
  if (d_out < 16 || d_out > 128 || d_out % 16 != 0)
    return fail(ctx, KMX_EUNSUPPORTED, "d_out must be a multiple of 16 in [16, 128]");
  if (ldy < d_out || ldy % 4 != 0 || (((uintptr_t)Y) & 15))
    return fail(ctx, KMX_EINVAL, "Y needs 16-byte alignment and ldy >= d_out, ldy % 4 == 0");
  KMX_TRY(set_device(ctx));
  KMX_TRY(grow(ctx, ctx->vt, (size_t)d_out * project_dpad(d_in) * sizeof(float)));
  Timed tm(ctx, T_PROJECT);
  KMX_HIP(ctx, launch_project(ctx->stream, X, rows, d_in, ldx, V, d_out, Y, ldy, P<float>(ctx->vt),
                              ctx->num_cus));
  return KMX_OK;
}

kmx_status kmx_lift(kmx_ctx* ctx, const float* Z, int64_t rows, int32_t m, int64_t ldz,
                    const float* V, int32_t d, float* Y, int64_t ldy) {
  if (!ctx) return KMX_EINVAL;
  ctx->err.clear();
  if (!Z || !V || !Y) return fail(ctx, KMX_EINVAL, "NULL Z, V or Y");
  if (rows < 1 || d < 1 || ldy < d) return fail(ctx, KMX_EINVAL, "bad rows, d or ldy");
  if (m < 1 || m > 128 || ldz < m)
    return fail(ctx, KMX_EUNSUPPORTED, "m must lie in [1, 128] with ldz >= m");
  if (rows > (int64_t)65535 * 64) return fail(ctx, KMX_EUNSUPPORTED, "rows above 4,194,240");
  KMX_TRY(set_device(ctx));
  Timed tm(ctx, T_PROJECT);
  KMX_HIP(ctx, launch_lift(ctx->stream, Z, rows, m, ldz, V, d, Y, ldy));
  return KMX_OK;
}

kmx_status kmx_assign_stats(kmx_ctx* ctx, int64_t* listed, int64_t* fp32, int64_t* full) {
  if (!ctx) return KMX_EINVAL;
  ctx->err.clear();
  if (!ctx->state.p) {
    if (listed) *listed = 0;
    if (fp32) *fp32 = 0;
    if (full) *full = 0;
    return KMX_OK;
  }
  KMX_TRY(set_device(ctx));
  LoopState h;
  KMX_HIP(ctx, hipMemcpyAsync(&h, ctx->state.p, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
  KMX_HIP(ctx, hipStreamSynchronize(ctx->stream));
  if (listed) *listed = (int64_t)h.flagged;
  if (fp32) *fp32 = (int64_t)(ctx->last_prec == KMX_FP8E4M3 ? h.full_count2 : h.full_count);
  if (full) *full = (int64_t)h.flagged_full;
  return KMX_OK;
}

kmx_status kmx_run_stats(kmx_ctx* ctx, int64_t* listed_total, int64_t* full_total) {
  if (!ctx) return KMX_EINVAL;
  ctx->err.clear();
  if (listed_total) *listed_total = 0;
  if (full_total) *full_total = 0;
  if (!ctx->state.p) return KMX_OK;
  KMX_TRY(set_device(ctx));
  LoopState h;
  KMX_HIP(ctx, hipMemcpyAsync(&h, ctx->state.p, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
  KMX_HIP(ctx, hipStreamSynchronize(ctx->stream));
  if (listed_total) *listed_total = (int64_t)(h.listed_total + h.flagged);
  if (full_total) *full_total = (int64_t)(h.full_total + h.flagged_full);
  return KMX_OK;
}

kmx_status kmx_update_stats(kmx_ctx* ctx, int64_t* changed, int32_t* delta) {
  if (!ctx) return KMX_EINVAL;
  ctx->err.clear();
  if (changed) *changed = 0;
  if (delta) *delta = 0;
  if (!ctx->state.p || !ctx->cfflag.p) return KMX_OK;
  KMX_TRY(set_device(ctx));
  LoopState h;
  int f[4];
  KMX_HIP(ctx, hipMemcpyAsync(&h, ctx->state.p, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
  KMX_HIP(ctx, hipMemcpyAsync(f, ctx->cfflag.p, sizeof(f), hipMemcpyDeviceToHost, ctx->stream));
  KMX_HIP(ctx, hipStreamSynchronize(ctx->stream));
  if (changed) *changed = (int64_t)h.dcount;
  if (delta) *delta = f[2] == 0 ? 1 : 0;
  return KMX_OK;
}

kmx_status kmx_mfma_probe(kmx_ctx* ctx, kmx_prec prec, const void* A, const void* B,
                          const uint8_t* scale_a, const uint8_t* scale_b, const float* C, float* D,
                          int32_t count) {
  if (!ctx) return KMX_EINVAL;
  ctx->err.clear();
  if (prec != KMX_FP32 && prec != KMX_BF16 && prec != KMX_FP8E4M3)
    return fail(ctx, KMX_EINVAL, "unknown precision");
  if (!A || !B || !D) return fail(ctx, KMX_EINVAL, "NULL A, B or D");
  if (prec == KMX_FP8E4M3 && (!scale_a || !scale_b))
    return fail(ctx, KMX_EINVAL, "the FP8 instruction needs scale_a and scale_b");
  if (count < 1 || count > (1 << 24)) return fail(ctx, KMX_EINVAL, "count out of range");
  KMX_TRY(set_device(ctx));
  KMX_HIP(ctx, launch_mfma_probe(ctx->stream, prec, (const uint8_t*)A, (const uint8_t*)B, scale_a,
                                 scale_b, C, D, count));
  return KMX_OK;
}

kmx_status kmx_timing(kmx_ctx* ctx, int enable, int reset) {
  if (!ctx) return KMX_EINVAL;
  if (reset) {
    (void)hipStreamSynchronize(ctx->stream);
    for (auto& r : ctx->recs) {
      ctx->pool.push_back(r.a);
      ctx->pool.push_back(r.b);
    }
    ctx->recs.clear();
    for (int i = 0; i < T_NCLASS; ++i) {
      ctx->ms_acc[i] = 0.0;
      ctx->cnt_acc[i] = 0;
    }
  }
  ctx->timing = enable != 0;
  return KMX_OK;
}

kmx_status kmx_timing_read(kmx_ctx* ctx, int n_classes, double* ms_out, int64_t* count_out) {
  if (!ctx) return KMX_EINVAL;
  if (n_classes < 0 || n_classes > T_NCLASS) return fail(ctx, KMX_EINVAL, "n_classes out of range");
  KMX_HIP(ctx, hipStreamSynchronize(ctx->stream));
  for (auto& r : ctx->recs) {
    float ms = 0.f;
    KMX_HIP(ctx, hipEventElapsedTime(&ms, r.a, r.b));
    ctx->ms_acc[r.cls] += ms;
    ctx->cnt_acc[r.cls] += 1;
    ctx->pool.push_back(r.a);
    ctx->pool.push_back(r.b);
  }
  ctx->recs.clear();
  for (int i = 0; i < n_classes; ++i) {
    if (ms_out) ms_out[i] = ctx->ms_acc[i];
    if (count_out) count_out[i] = ctx->cnt_acc[i];
  }
  return KMX_OK;
}

}  // extern "C"
