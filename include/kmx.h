/*
 * kmx -- weighted k-means++ seeding and Lloyd iterations on one AMD Instinct
 * MI355X (gfx950).  Plain C ABI: every array argument is a raw pointer, every
 * size a plain integer; no C++ or framework types cross this boundary.
 *
 * The problem (Sec. 1, definition of k-means; Sec. 1, coreset cost): given n
 * points x_i in R^d with weights w_i >= 0 and k centers c_j, the cost is
 *     cost(C) = sum_i w_i * min_j ||x_i - c_j||^2 .
 * Lloyd's algorithm (Sec. 1) alternates assignment to the closest center and
 * replacement of each center by the weighted centroid of its points (Sec. 2,
 * centroid; Sec. 2.1, clustering feature (W, S, Q) = (sum w, sum w x,
 * sum w x^T x)).  k-means++ (Sec. 1) draws the first center by weight and each
 * further center with probability proportional to w_i * D2_i, D2_i being the
 * squared distance to the closest center chosen so far; Sec. 2.2 runs it on
 * the weighted summary.
 *
 * Conventions shared by all calls
 *   - X is row-major n x d float32 with leading dimension ldx >= d (elements);
 *     C arrays are row-major k x d float32 with leading dimension d.
 *   - Array arguments are DEVICE pointers on the context's device, owned by
 *     the caller, unless marked "host".  Host scalar outputs are written after
 *     the call synchronizes the context's stream; every other call is
 *     stream-ordered and asynchronous (results valid once the stream reaches
 *     that point).
 *   - w may be NULL (all weights 1).  Weights must be finite and >= 0: the
 *     calls that synchronize anyway (kmx_seed, kmx_cost, kmx_lloyd,
 *     kmx_lloyd_graph, kmx_lloyd_routed, kmx_lloyd_batched) read w once
 *     before any other work and return KMX_EINVAL otherwise; kmx_update, which
 *     does not wait, checks w only under KMX_VALIDATE.
 *   - KMX_VALIDATE=1 (read when the context is created): calls that take X
 *     and centers also scan them for values that are not finite first (one
 *     extra read of X; the call synchronizes), KMX_EINVAL if one is found.
 *   - Ties in the argmin go to the lowest center index.  An empty cluster
 *     keeps its previous center.
 *   - Return codes only; nothing throws or aborts across the ABI.  On failure
 *     kmx_last_error() describes the cause.  Argument checks run before any
 *     work is enqueued, so a KMX_EINVAL call leaves outputs untouched.
 *   - Calls on one context are not thread-safe; use one context per thread.
 */
#ifndef KMX_H
#define KMX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct kmx_ctx kmx_ctx;

typedef enum {
  KMX_OK = 0,
  KMX_EINVAL = 1,       /* bad argument (null pointer, size, range)          */
  KMX_ENOMEM = 2,       /* device workspace allocation failed                */
  KMX_EDEVICE = 3,      /* a HIP runtime call or kernel launch failed        */
  KMX_EUNSUPPORTED = 4  /* valid request outside what the library implements */
} kmx_status;

/* Arithmetic of the distance GEMM inside assignment.  Labels are exact for
 * every precision: rows whose top-2 margin lies inside the rigorous error
 * bound of the chosen precision are re-checked with compensated FP32
 * direct differences.  Centroid and cost accumulation is always FP64.
 * Rows wider than 1024 (kmx_assign, kmx_cost, kmx_lloyd, kmx_lloyd_graph;
 * any precision) take the exact every-center path instead: plain FP32
 * direct-difference distances to every center, double-float sums for the
 * centers inside their error bound; no matrix cores. */
typedef enum {
  KMX_FP32 = 0,     /* FP32 MFMA, FP32 accumulate                            */
  KMX_BF16 = 1,     /* BF16 inputs (round to nearest even), FP32 accumulate  */
  KMX_FP8E4M3 = 2   /* FP8 E4M3 inputs with a power-of-two scale per row of X
                       and one for all centers, FP32 accumulate; rows the
                       FP8 bound cannot decide go through the BF16 GEMM;
                       d <= 1024 */
} kmx_prec;

/* Context: binds a device and a HIP stream (hip_stream == NULL: the null
 * stream).  Owns a grow-only device workspace freed by kmx_destroy.  A
 * quantized copy of X is cached per (pointer, n, d, ldx, precision) until
 * kmx_invalidate is called for that pointer or a different X is used. */
kmx_status kmx_create(kmx_ctx** out, int device, void* hip_stream);
kmx_status kmx_destroy(kmx_ctx* ctx);
kmx_status kmx_set_stream(kmx_ctx* ctx, void* hip_stream);
/* Drop cached derived data of X (call after X's contents change; X == NULL:
 * of every X).  Every call also drops the grouped copies of the batched
 * path (call it after changing any batched problem's X or w). */
kmx_status kmx_invalidate(kmx_ctx* ctx, const float* X);
/* Message of the last failed call on ctx ("" if none).  Valid until the next
 * call on ctx.  kmx_last_error(NULL) reports failures of kmx_create. */
const char* kmx_last_error(const kmx_ctx* ctx);

/* Weighted k-means++ seeding (Sec. 1 k-means++; Sec. 2.2 on the weighted
 * summary).  Round 0 draws i_0 with probability w_i / sum w; round r >= 1
 * draws i_r with probability w_i D2_i / sum_j w_j D2_j, where D2 is the FP64
 * squared distance to the closest chosen center.  If that mass is zero, round
 * r draws by weight among rows not chosen yet.  The draws are inverse-CDF
 * picks (first index whose inclusive prefix strictly exceeds u_r * total)
 * with u_r = (z_r >> 11) * 2^-53, z_r the r-th SplitMix64 output for state
 * rng_seed.
 *   C_out   device, k x d float32: exact copies of the chosen rows.
 *   idx_out device, k int64, nullable: the chosen row indices.
 * Requires 1 <= k <= #{i : w_i > 0} (= n when w is NULL; a weight-w point
 * stands for w copies, Sec. 2.3.1, so a zero-weight row stands for none and
 * is never chosen): KMX_EINVAL otherwise.  A round skips the rows whose D2
 * provably cannot drop (the new center is at least twice as far from the
 * row's closest chosen center as the row is), so D2 is the same as with every
 * row read. */
kmx_status kmx_seed(kmx_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx,
                    const float* w, int32_t k, uint64_t rng_seed,
                    float* C_out, int64_t* idx_out);

/* Rows whose distance to the new center the most recent kmx_seed on ctx
 * computed, summed over its rounds 1 .. k-1 (the other rows kept their D2 by
 * the triangle-inequality test).  rows_read: host output.  Synchronizes. */
kmx_status kmx_seed_stats(kmx_ctx* ctx, int64_t* rows_read);

/* Assignment step (Sec. 1): label_i = argmin_j ||x_i - c_j||^2, lowest j on
 * ties.  The distance GEMM runs in `prec`; flagged rows are re-checked.
 *   label_out device, n int32.
 *   d1_out    device, n float32, nullable: distance to the assigned center.
 *   d2_out    device, n float32, nullable: second smallest distance as
 *             evaluated by the GEMM (within the GEMM's error bound; +inf if
 *             k == 1); for rows wider than 1024, the second smallest plain
 *             FP32 distance.
 *   n_flagged host, nullable: rows the first GEMM pass could not decide, i.e.
 *             rows that went to the exact re-check or to a later GEMM pass
 *             (BF16 and FP8: the cascade's split-BF16 pass; synchronizes).
 */
kmx_status kmx_assign(kmx_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx,
                      const float* C, int32_t k, kmx_prec prec,
                      int32_t* label_out, float* d1_out, float* d2_out,
                      int64_t* n_flagged);

/* Update step (Sec. 1; Sec. 2 centroid; Sec. 2.1 clustering features).  For
 * each j: W_j = sum w_i, S_j = sum w_i x_i over label_i == j, in FP64;
 * C_out[j] = float32(S_j / W_j) if W_j > 0 else C_prev[j].  C_out may equal
 * C_prev.  Labels must lie in [0, k).
 *   W_out             device, k float64, nullable.
 *   cost_at_centroids host, nullable: sum_j (Q_j - ||S_j||^2 / W_j), the cost
 *                     of this partition against its own centroids
 *                     (synchronizes). */
kmx_status kmx_update(kmx_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx,
                      const float* w, const int32_t* label, int32_t k,
                      const float* C_prev, float* C_out, double* W_out,
                      double* cost_at_centroids);

/* Weighted cost sum_i w_i min_j ||x_i - c_j||^2 in FP64 (Sec. 1), evaluated
 * through the clustering-feature identity of Sec. 2.1 over the exact
 * assignment:  sum_j Q_j - 2 c_j . S_j + W_j ||c_j||^2.  Synchronizes. */
kmx_status kmx_cost(kmx_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx,
                    const float* w, const float* C, int32_t k, kmx_prec prec,
                    double* cost_out);

/* Lloyd's algorithm (Sec. 1 and its footnote on stopping).  Iteration t
 * assigns against C_t, records cost_hist[t] = cost(C_t) and replaces the
 * centers by the weighted centroids.  tol < 0: exactly max_iter iterations.
 * tol >= 0: stop after iteration t >= 1 when no label changed or when
 * cost_hist[t-1] - cost_hist[t] <= tol * cost_hist[t-1].  One final
 * assignment gives cost_hist[iters] = cost(C_iters) and the labels.
 *   C_inout   device, k x d float32: C_0 in, C_iters out.
 *   label_out device, n int32, nullable: labels against C_iters.
 *   cost_hist host, max_iter + 1 doubles (entries past iters untouched).
 *   iters_done host: number of update steps performed.
 * Synchronizes once at the end. */
kmx_status kmx_lloyd(kmx_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx,
                     const float* w, float* C_inout, int32_t k, int32_t max_iter,
                     double tol, kmx_prec prec, int32_t* label_out,
                     double* cost_hist, int32_t* iters_done);

/* kmx_lloyd with the iteration launched as a graph (Sec. 1, as kmx_lloyd):
 * one iteration's launches are captured once on the context's capture
 * stream, which waits for the context stream first, and replayed max_iter
 * times; the stop rule is evaluated on the device, so iterations after the
 * stop do nothing, as in kmx_lloyd.  Same arguments, results (bitwise) and
 * errors as kmx_lloyd, plus KMX_EDEVICE when capture or replay fails.  For
 * small problems, where launch overhead dominates.  Synchronizes once at
 * the end. */
kmx_status kmx_lloyd_graph(kmx_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx,
                           const float* w, float* C_inout, int32_t k, int32_t max_iter,
                           double tol, kmx_prec prec, int32_t* label_out,
                           double* cost_hist, int32_t* iters_done);

/* Projection onto a subspace (Sec. 2.2, "Using SVD to project to the best
 * fit subspace": dimension reduction of each piece, a
 * row's coordinates in the span of the top right singular vectors, which
 * keeps squared distances within that span):
 *     Y[r][j] = sum_i X[r][i] V[i][j],  r < rows, j < d_out,
 * FP32 MFMA with FP32 accumulation.  X rows x d_in (leading dimension ldx),
 * V d_in x d_out row-major, Y rows x d_out (leading dimension ldy), all
 * device.  d_out a multiple of 16 in [16, 128]; Y 16-byte aligned with
 * ldy % 4 == 0.  Stream-ordered; call once per chunk of rows. */
kmx_status kmx_project(kmx_ctx* ctx, const float* X, int64_t rows, int32_t d_in, int64_t ldx,
                       const float* V, int32_t d_out, float* Y, int64_t ldy);

/* The rows of A_m = A V V^T (Sec. 2.2, "Using SVD to project to the best fit
 * subspace": a projected point keeps its d coordinates, its intrinsic
 * dimension drops to m) from their coordinates Z = A V:
 *     Y[r][c] = sum_j Z[r][j] V[c][j],  r < rows, c < d,
 * FP32 FMAs in j order.  Z rows x m (leading dimension ldz >= m), V d x m
 * row-major (the basis kmx_project takes), Y rows x d (ldy >= d), all device;
 * 1 <= m <= 128, rows <= 4,194,240 per call.  Stream-ordered. */
kmx_status kmx_lift(kmx_ctx* ctx, const float* Z, int64_t rows, int32_t m, int64_t ldz,
                    const float* V, int32_t d, float* Y, int64_t ldy);

/* kmx_assign with KMX_FP32 that allocates nothing, for callers that cannot
 * allocate device memory (code under graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same labels, d1 and d2 bit for bit as
 * kmx_assign(..., KMX_FP32, ...); n_flagged and kmx_assign_stats are not
 * reported.  Its working memory is one static device array per GPU of 32 MiB,
 * held until the process ends: rows are taken in chunks of 262,144, and the
 * padded FP32 centers must fit the rest of the array, about 22 MB (k * d up to
 * roughly 5.5 million floats after padding); larger k * d returns KMX_EINVAL
 * with the sizes in the message.  Every call on one GPU shares that GPU's
 * array, whichever context it comes through: calls that overlap on one GPU
 * (other streams, other threads) race and must be serialized by the caller.
 * The call clears what it needs at its start.  No KMX_VALIDATE scan.
 * Stream-ordered and asynchronous; d <= 1024. */
kmx_status kmx_assign_noalloc(kmx_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx,
                              const float* C, int32_t k, int32_t* label_out, float* d1_out,
                              float* d2_out);

/* Top-r right singular vectors of A' = diag(sqrt(w)) A by a randomized
 * range finder (Sec. 2.2, "Computation of the SVD": multiply A by a random
 * matrix to reduce its columns, then a small SVD, after Halko, Martinsson and
 * Tropp 2011, subspace iteration with power_iters passes; Sec. 2.3.2: a point
 * of weight w enters as its row scaled by sqrt(w), which gives the best-fit
 * subspace of the point set with w copies of every point).  Projecting the
 * rows onto V (kmx_project) reduces them to that subspace (Sec. 2.2, "Using
 * SVD to project to the best fit subspace").
 *   A        device, n x d float32, leading dimension lda >= d.
 *   w        device, n float32, nullable (all 1); finite and >= 0.
 *   r        rank; r + oversample rounded up to a multiple of 16 (the sample
 *            width l) must be <= 128 and <= min(n, d).
 *   seed     the Gaussian test matrix: element i is a Box-Muller normal of
 *            SplitMix64 outputs 2 i and 2 i + 1 from state seed.
 *   V_out    device, d x r float32 (row-major, leading dimension r):
 *            orthonormal columns, in decreasing order of singular value.
 *   sigma_out host, r doubles, nullable: the singular values of the sample.
 * Products with A run on the device (FP32 projection; A^T X with FP64 sums);
 * the l x l factorizations (CholeskyQR2, Jacobi eigenproblem) in FP64 on the
 * host.  Synchronizes. */
kmx_status kmx_range_basis(kmx_ctx* ctx, const float* A, int64_t n, int32_t d, int64_t lda,
                           const float* w, int32_t r, int32_t oversample, int32_t power_iters,
                           uint64_t seed, float* V_out, double* sigma_out);

/* Re-check counts of the most recent assignment on ctx (kmx_assign, kmx_cost,
 * or the final assignment of kmx_lloyd); host outputs, each nullable:
 *   listed   rows on the exact re-check list (pairs and full rows),
 *   fp32     rows the BF16 GEMM passed to the cascade's last GEMM pass
 *            (FP32 values split into two BF16 parts each, three BF16 products
 *            per coordinate) because more than three centers lay within its
 *            error bound (with KMX_FP8E4M3 the
 *            FP8 pass first hands the rows with more than three centers
 *            inside its bound to the BF16 pass); 0 when there were at most
 *            4096 such rows and k d >= 65536, which then go to the
 *            every-center re-check,
 *   full     rows re-checked against every center.
 * Synchronizes. */
kmx_status kmx_assign_stats(kmx_ctx* ctx, int64_t* listed, int64_t* fp32, int64_t* full);

/* Exact re-check work of the most recent Lloyd run on ctx (or, outside a run,
 * since the context was created); host outputs, each nullable: entries of the
 * short re-check lists (pairs and triples) and rows re-checked against every
 * center, summed over every assignment.  Synchronizes. */
kmx_status kmx_run_stats(kmx_ctx* ctx, int64_t* listed_total, int64_t* full_total);

/* The most recent update of a Lloyd run on ctx (the final assignment's, after
 * kmx_lloyd and its variants); host outputs, each nullable:
 *   changed  rows whose label differed from the previous update's,
 *   delta    1 when the features were formed from the previous update's by
 *            removing and adding only those rows (Sec. 2.1: clustering
 *            features add and subtract), 0 when every row was summed (the
 *            first update of a run, or more than half of the rows changed).
 * Both give the same bits.  Synchronizes. */
kmx_status kmx_update_stats(kmx_ctx* ctx, int64_t* changed, int32_t* delta);

/* Measurement of the arithmetic the assignment's error bounds rely on:
 * instance q < count runs one matrix instruction of the distance GEMM of
 * `prec`, exactly as the assignment issues it, on A_q and B_q (device,
 * instance after instance, 16 rows each, row-major) starting from C (device,
 * count x 16 x 16 float32, nullable: zero), and stores
 *     D[q][i][j] = C[q][i][j] + sum_t A_q[i][t] B_q[j][t]
 * as the matrix core rounds it (device, count x 16 x 16 float32):
 *   KMX_FP8E4M3: 16 x 128 E4M3 bytes per row; every row of A_q is scaled by
 *     2^(scale_a[q] - 127) and row j of B_q by 2^(scale_b[16 q + j] - 127)
 *     (E8M0 bytes, device);
 *   KMX_BF16: 16 x 32 BF16 values (bit patterns) per row; scales unused;
 *   KMX_FP32: 16 x 4 floats per row; scales unused.
 * The FP8 bound takes an instruction's error to be at most
 * 2^-10 sum |a_t b_t| + 2^-19 (|C| + sum |a_t b_t|) plus the FP32 rounding of
 * the result; the BF16 and FP32 bounds take K faithful FP32 steps (K = 32 or
 * 4 products).  This call lets a test check that on the device at hand.
 * Stream-ordered. */
kmx_status kmx_mfma_probe(kmx_ctx* ctx, kmx_prec prec, const void* A, const void* B,
                          const uint8_t* scale_a, const uint8_t* scale_b, const float* C, float* D,
                          int32_t count);

/* Kernel timing for measurement: while enabled, HIP events bracket every
 * kernel class on the context's stream.  kmx_timing_read returns the summed
 * milliseconds and launch counts per class since the last reset:
 *   class 0 prep (row statistics, quantization), 1 assign GEMM (first pass),
 *   2 the further GEMM passes of the cascade, 3 label sort / delta lists, 4
 *   segmented reduction, 5 finalize, 6 seeding, 7 other, 8 router forward
 *   pass, 9 center table + certificate, 10 router training, 11 projection,
 *   range finder and lift, 12 carried bounds (bound test, center drift), 13
 *   the exact short and every-center re-check.
 * ms_out and count_out are host arrays of length n_classes (<= 14).
 * Reading synchronizes.  enable = 0 stops recording; reset clears sums. */
kmx_status kmx_timing(kmx_ctx* ctx, int enable, int reset);
kmx_status kmx_timing_read(kmx_ctx* ctx, int n_classes, double* ms_out, int64_t* count_out);

/* ---------------------------------------------------------------------------
 * Batched Lloyd: many independent weighted problems at once (Sec. 2.2 runs
 * k-means++ and Lloyd on weighted summaries; pieces and restarts give many
 * such problems).  Every iteration assigns all problems with one persistent
 * launch per width group (d rounded to the BF16 tile width: up to six
 * groups; BF16 distance GEMM, exact labels as for kmx_assign), updates each
 * problem's centroids in FP64 and records its cost; the iteration is
 * captured once as a HIP graph and replayed.  The tile shape used for each
 * (d, k class) is the autotuner's choice when kmx_batched_autotune ran on
 * the context, otherwise a default.
 * ------------------------------------------------------------------------- */
typedef struct {
  const float* X;   /* device, n x d, leading dimension ldx                  */
  int64_t n;
  int32_t d;        /* 1 <= d <= 512                                        */
  int64_t ldx;
  const float* w;   /* device, n weights, nullable (all 1)                   */
  float* C;         /* device, k x d: C_0 in, C_iters out                    */
  int32_t k;        /* 1 <= k <= n                                           */
  int32_t* label;   /* device, n, nullable: labels against C_iters           */
} kmx_problem;

/* iters Lloyd iterations of every problem (no early stop), then one
 * assignment for the final cost and labels.
 *   prec      KMX_BF16.
 *   cost_hist host, count x (iters + 1) doubles, row i = problem i:
 *             cost_hist[i][t] = cost of problem i at C_t.
 * Synchronizes.  X and w are copied into a grouped layout (with their row
 * statistics and feature grids) when the problems differ from those of the
 * previous batched call on ctx (X and w pointers, sizes, order); otherwise
 * those copies are reused, so call kmx_invalidate after changing the contents
 * of any X or w.  C is read on every call. */
kmx_status kmx_lloyd_batched(kmx_ctx* ctx, const kmx_problem* probs, int32_t count,
                             int32_t iters, kmx_prec prec, double* cost_hist);

/* Weighted k-means++ seeding (as kmx_seed) of every problem at once: round r
 * of all problems with k > r runs in one launch, each problem drawing from
 * its own SplitMix64 stream, so problem i gets the same centers and indices
 * as kmx_seed(X_i, n_i, d_i, ldx_i, w_i, k_i, rng_seeds[i]) (rows whose D2
 * provably cannot drop are skipped as there).
 *   probs      X, n, d (any d >= 1), ldx, w, k as for kmx_seed; C receives
 *              the k x d centers; label unused.
 *   rng_seeds  host, count seeds.
 *   idx_out    device, sum_i k_i int64, nullable: the chosen row indices of
 *              problem i at offset k_0 + ... + k_{i-1}.
 * Requirements per problem as kmx_seed (KMX_EINVAL names the problem).
 * Synchronizes. */
kmx_status kmx_seed_batched(kmx_ctx* ctx, const kmx_problem* probs, int32_t count,
                            const uint64_t* rng_seeds, int64_t* idx_out);

/* Autotuner: for each (d, k class) present in probs (k classes: k <= 24,
 * k <= 96, larger), times the batched assignment of those problems under
 * each tile shape and keeps the fastest on ctx.  cache_path (nullable): a
 * file of JSON lines; entries for this device are loaded instead of tuning
 * when present (*loaded = 1), new results are appended otherwise. */
kmx_status kmx_batched_autotune(kmx_ctx* ctx, const kmx_problem* probs, int32_t count,
                                kmx_prec prec, const char* cache_path, int32_t* loaded);

/* Tile shape the batched assignment uses for (d, k) on ctx: centers per LDS
 * tile and points per workgroup (host outputs, nullable). */
kmx_status kmx_batched_tiles(kmx_ctx* ctx, int32_t d, int32_t k, int32_t* tile,
                             int32_t* points_per_block);

/* ---------------------------------------------------------------------------
 * Candidate router with a certificate.
 *
 * Not part of the paper's method: an accelerator of its assignment step
 * (Sec. 1) that leaves every label unchanged.  A two-layer perceptron
 *     z(x) = W2 relu(W1 x + b1) + b2,   W1: 256 x d, W2: k x 256,
 * evaluated in BF16 with FP32 accumulation, proposes 16 candidate centers
 * per point: the four highest logits within each quarter of the centers
 * (quarter of center j: (j mod 16) div 4), which always contain the four
 * highest logits overall.  An assignment using the proposals takes the best
 * proposal b and an upper bound D of ||x - c_b||; a table of lower bounds of
 * the center distances gives the centers within 2 D of c_b (Elkan's
 * triangle-inequality lemma: no other center can be closer than c_b).  With
 * none, c_b is the label; with one or two, all among the candidates, the
 * exact comparison decides; otherwise the point goes through the GEMM
 * assignment.  Requirements: 1 <= d <= 1024, 1 <= k <= 4096.
 * ------------------------------------------------------------------------- */
typedef struct kmx_router kmx_router;

/* New router for inputs of width d and k centers, on ctx's device.
 * Initial weights: W1 ~ N(0, 2/d), W2 ~ N(0, 1/256) from a SplitMix64 /
 * Box-Muller stream seeded by init_seed; zero biases; Adam state cleared. */
kmx_status kmx_router_create(kmx_ctx* ctx, int32_t d, int32_t k, uint64_t init_seed,
                             kmx_router** out);
kmx_status kmx_router_destroy(kmx_ctx* ctx, kmx_router* r);

/* FP32 parameters, device arrays: W1 256 x d, b1 256, W2 k x 256, b2 k (row
 * major).  set_params also clears the Adam state; get_params outputs are
 * nullable. */
kmx_status kmx_router_set_params(kmx_ctx* ctx, kmx_router* r, const float* W1, const float* b1,
                                 const float* W2, const float* b2);
kmx_status kmx_router_get_params(kmx_ctx* ctx, kmx_router* r, float* W1, float* b1, float* W2,
                                 float* b2);

/* Mean softmax cross-entropy of labels (device, n int32 in [0, k)) over the
 * n rows of X (n <= 65536, one batch) and its gradients (device FP32 arrays
 * shaped like the parameters, each nullable).  The network runs as in
 * training: BF16 inputs, weights and activations, FP32 accumulation.
 *   loss host, nullable (synchronizes). */
kmx_status kmx_router_loss_grad(kmx_ctx* ctx, kmx_router* r, const float* X, int64_t n, int32_t d,
                                int64_t ldx, const int32_t* labels, double* loss, float* dW1,
                                float* db1, float* dW2, float* db2);

/* Adam training (beta1 0.9, beta2 0.999, eps 1e-8, learning rate lr) on the
 * n * n_sets pairs (x_i, labels[s * n + i]), s < n_sets (device int32): each
 * epoch visits every pair once in batches of `batch` (<= 65536; the last one
 * may be smaller), in a pseudo-random order drawn from shuffle_seed (0: the
 * order s-major, i-minor).
 *   loss_hist  host, nullable: mean loss of every step (epochs * steps per
 *              epoch entries);
 *   steps_done host, nullable.
 * Synchronizes. */
kmx_status kmx_router_train(kmx_ctx* ctx, kmx_router* r, const float* X, int64_t n, int32_t d,
                            int64_t ldx, const int32_t* labels, int32_t n_sets, int32_t epochs,
                            int32_t batch, float lr, uint64_t shuffle_seed, double* loss_hist,
                            int64_t* steps_done);

/* Proposals for the rows of X: cand_out device n x 16 int32; entries
 * 4q .. 4q+3 are quarter q's four highest logits in decreasing order (-1
 * where the quarter has fewer than four centers). */
kmx_status kmx_router_propose(kmx_ctx* ctx, kmx_router* r, const float* X, int64_t n, int32_t d,
                              int64_t ldx, int32_t* cand_out);

/* Lloyd's algorithm as kmx_lloyd (same arguments, results and stopping
 * rule) with the assignment step accelerated by certified proposals.  r
 * gives the proposals (one forward pass per call: they depend on X only);
 * r == NULL uses each point's previous label as its only candidate, the
 * first assignment then running the full GEMM.  prec is the GEMM's
 * precision for the remaining rows.
 *   gemm_rows host, nullable, max_iter + 1 entries: rows of each
 *             assignment (entries 0 .. iters) that went through the GEMM. */
kmx_status kmx_lloyd_routed(kmx_ctx* ctx, kmx_router* r, const float* X, int64_t n, int32_t d,
                            int64_t ldx, const float* w, float* C_inout, int32_t k,
                            int32_t max_iter, double tol, kmx_prec prec, int32_t* label_out,
                            double* cost_hist, int32_t* iters_done, int64_t* gemm_rows);

/* Lower bounds of the distances between centers, the table the certificate
 * of kmx_lloyd_routed and kmx_lloyd_bounded uses (Elkan's test: a center c
 * cannot be closer to x than c_b when ||c_b - c|| >= 2 ||x - c_b||).
 *   C      device, k x d float32, rows contiguous.
 *   D_out  device, k x k float32: D_out[b k + c] <= ||c_b - c_c|| (+inf for
 *          b == c), from the Gram form ||c_b||^2 + ||c_c||^2 - 2 c_b.c_c with
 *          the dot products on the FP32 matrix cores and their error bound
 *          subtracted (loose only where the distance is tiny against the
 *          norms).
 * 1 <= k <= 4096, d >= 1; stream-ordered, asynchronous. */
kmx_status kmx_center_bounds(kmx_ctx* ctx, const float* C, int32_t k, int32_t d, float* D_out);

/* Lloyd's algorithm as kmx_lloyd (same arguments, results and stopping rule)
 * with bounds carried across iterations (Hamerly's form of Elkan's
 * triangle-inequality filtering; not in the paper, an exact accelerator of the
 * Sec. 1 assignment step).  Every row keeps an upper bound of the distance to
 * its center and a lower bound of the distance to every other center, set by
 * the assignment that decided it (rounded outward from that pass's rigorous
 * error bound or from the exact re-check).  After each update the centers'
 * drifts (FP64 norms of the moves, rounded up) loosen the bounds by the
 * triangle inequality; a row whose upper bound stays strictly below its lower
 * bound keeps its label without its data being read.  The other rows go
 * through the certificate of kmx_lloyd_routed (the router's proposals when r
 * is given, else the previous label) and then the GEMM cascade of `prec`.
 * The proposals of a row are computed the first time the bounds cannot keep
 * it and kept for the rest of the call (they depend on the row only).
 * The first assignment runs the GEMM on every row.
 *   gemm_rows host, nullable, max_iter + 1 entries: rows of each assignment
 *             that went through the GEMM.
 *   kept_rows host, nullable, max_iter + 1 entries: rows of each assignment
 *             the bounds kept (0 for the first).
 * Requirements as kmx_lloyd_routed (k <= 4096, d <= 1024). */
kmx_status kmx_lloyd_bounded(kmx_ctx* ctx, kmx_router* r, const float* X, int64_t n, int32_t d,
                             int64_t ldx, const float* w, float* C_inout, int32_t k,
                             int32_t max_iter, double tol, kmx_prec prec, int32_t* label_out,
                             double* cost_hist, int32_t* iters_done, int64_t* gemm_rows,
                             int64_t* kept_rows);

/* ---- BICO summary (Sec. 2.1; weighted insertion Sec. 2.3.1) --------------
 * A tree of clustering features (W, S, Q) -- weight, weighted sum of the
 * points, weighted sum of their squared lengths -- kept on the host; the
 * search for the closest reference point among the children of a node, which
 * the paper names as dominating insertion time, runs on ctx's device in
 * blocks of points (the assignment step's distance GEMM with fused argmin).
 * The device searches cover the root's children and the 15 largest child
 * lists of at least 32 features (the rest are searched on the host).
 * Insertion: a point (w copies) goes down the tree to the closest reference
 * among the children of the current node (ties: the oldest); it opens a
 * feature (w, w x, w ||x||^2) when no reference lies within the level's
 * radius R_i = sqrt(T / 2^(3 + i)) (level 1: children of the root); otherwise
 * w' = min(w, floor((sT - sc) / (s D - T + c))) copies join that feature (all
 * of them when s D - T + c <= 0; s = W, c = Q - ||S||^2 / W its cost,
 * D = ||x - S / W||^2) and the rest descend.  More than m features: T doubles
 * and every feature is re-inserted (breadth-first order of the old tree) into
 * an empty tree, merging into the closest feature within the radius when the
 * merged cost stays within T.  All decisions use FP64 sums in coordinate
 * order.  The summary is the centroids S / W with weights W, breadth-first.
 * A kmx_bico belongs to the ctx it was created with; not thread-safe. */
typedef struct kmx_bico kmx_bico;

/* Empty summary of at most m >= 1 features in R^d, starting threshold
 * T0 > 0 (finite).  Host memory grows with the features: m x d doubles for the
 * sums and m x d floats for the references. */
kmx_status kmx_bico_create(kmx_ctx* ctx, int32_t d, int64_t m, double T0, kmx_bico** out);
kmx_status kmx_bico_destroy(kmx_ctx* ctx, kmx_bico* b);

/* Inserts rows 0 .. n-1 of X (device, n x d, leading dimension ldx >= d) in
 * order, row i with weight w[i] (device, nullable: 1; entries must be finite
 * and >= 0, a zero weight inserts nothing).  Copies blocks of rows to the host
 * and synchronizes.  KMX_EINVAL on a bad weight (rows before it are in). */
kmx_status kmx_bico_insert(kmx_ctx* ctx, kmx_bico* b, const float* X, int64_t n, int64_t ldx,
                           const float* w);

/* Host outputs, each nullable: number of features, current threshold, rebuilds
 * so far, rows (points and re-inserted features) whose searches ran on the
 * device, searches whose two closest references were too near for the
 * device's FP32 distances (so that the host compared them in FP64), and the
 * (row, reference) distances the device searches computed. */
kmx_status kmx_bico_stats(kmx_ctx* ctx, const kmx_bico* b, int64_t* count, double* T,
                          int64_t* rebuilds, int64_t* gpu_rows, int64_t* host_scans,
                          int64_t* pairs);

/* The features in breadth-first order (count from kmx_bico_stats), host
 * arrays, each nullable: W (count), S (count x d), Q (count), reference
 * points (count x d), tree level (count; 1 = child of the root). */
kmx_status kmx_bico_features(kmx_ctx* ctx, const kmx_bico* b, double* W, double* S, double* Q,
                             float* ref, int32_t* level);

/* The summary on the device: P_out (count x d, float32(S / W)) and w_out
 * (count, float32(W)), breadth-first.  Synchronizes. */
kmx_status kmx_bico_coreset(kmx_ctx* ctx, const kmx_bico* b, float* P_out, float* w_out);

#ifdef __cplusplus
}
#endif
#endif /* KMX_H */
