// Update step of Lloyd's algorithm (Sec. 1: replace each center by the
// centroid of its subset) as a deterministic, HBM-bound segmented reduction.
//
// For every cluster j the kernels form the weighted clustering feature of
// Sec. 2.1 / Sec. 2.3.1: W_j = sum w_i, S_j = sum w_i x_i, Q_j = sum w_i ||x_i||^2,
// each summed exactly on a fixed-point grid (section 6 below), so that the
// features of a Lloyd iteration can also be formed from the previous
// iteration's by removing and adding only the rows whose label changed.  The
// cost of the partition against any center c follows from the identity of
// Sec. 2.1:
//     sum_{i in P_j} w_i ||x_i - c||^2 = Q_j - 2 c.S_j + W_j ||c||^2 .
//
// Full update: a stable counting sort of row ids by label (block histograms,
// column scans, in-block ranks from one ballot per label bit), then one
// workgroup per chunk of at most kReduceRows rows of one cluster gathers whole
// rows (coalesced) and accumulates the limb sums, and one workgroup per
// cluster sums its chunks.  Delta update (Lloyd iterations after the first):
// the changed rows are listed, grouped by cluster as signed entries (removal
// from the old cluster, addition to the new) and reduced the same way; the
// finalize adds the chunk sums to the features carried from the previous
// iteration.  Both give the same bits, since every sum is exact.
#include "kmx_device.h"
#include "kmx_internal.h"

namespace kmx {

// ---- 1. block histograms; optional label-change count against lab_prev ----
__global__ __launch_bounds__(256) void hist_kernel(const int32_t* __restrict__ label,
                                                   int32_t* __restrict__ lab_prev, int64_t n,
                                                   int k, int32_t* __restrict__ counts,
                                                   int32_t* __restrict__ chg, int track,
                                                   const int* __restrict__ gate) {
  if (gate && *gate) return;
  extern __shared__ int hsm[];
  constexpr int PER = kSortRows / 256;
  const int b = blockIdx.x;
  const int64_t r0 = (int64_t)b * kSortRows;
  const int64_t r1 = min(n, r0 + kSortRows);
  // the block's labels (and previous labels) are in flight together
  int lab[PER], prev[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int64_t i = r0 + threadIdx.x + 256 * q;
    lab[q] = (i < r1) ? label[i] : -1;
    prev[q] = (track && i < r1) ? lab_prev[i] : -1;
  }
  for (int j = threadIdx.x; j < k; j += blockDim.x) hsm[j] = 0;
  __syncthreads();
  int ch = 0;
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int64_t i = r0 + threadIdx.x + 256 * q;
    if (lab[q] >= 0 && lab[q] < k) atomicAdd(&hsm[lab[q]], 1);
    if (track && i < r1) {
      ch += (prev[q] != lab[q]);
      lab_prev[i] = lab[q];
    }
  }
  __syncthreads();
  int32_t* out = counts + (int64_t)b * k;
  for (int j = threadIdx.x; j < k; j += blockDim.x) out[j] = hsm[j];
  if (track) {
    // changed labels per wave, summed by scan_top_kernel (no global atomics)
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) ch += __shfl_xor(ch, m, 64);
    if ((threadIdx.x & 63) == 0) chg[4 * b + (threadIdx.x >> 6)] = ch;
  }
}

// ---- 2. per-segment column sums of the count matrix ----
__global__ __launch_bounds__(256) void scan_seg_kernel(const int32_t* __restrict__ counts,
                                                       int nb, int k,
                                                       int32_t* __restrict__ segsum,
                                                       const int* __restrict__ gate) {
  if (gate && *gate) return;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int s = blockIdx.y;
  if (j >= k) return;
  const int per = (nb + kScanSegs - 1) / kScanSegs;
  const int b0 = s * per, b1 = min(nb, b0 + per);
  int acc = 0;
  for (int b = b0; b < b1; ++b) acc += counts[(int64_t)b * k + j];
  segsum[(int64_t)s * k + j] = acc;
}

// Block-wide exclusive scan of one int per thread (1024 threads).
__device__ int block_excl_scan_1024(int v, int* sh, int& total) {
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  int x = v;
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) {
    int y = __shfl_up(x, m, 64);
    if (lane >= m) x += y;
  }
  if (lane == 63) sh[w] = x;
  __syncthreads();
  if (tid < 64) {
    int s = (tid < 16) ? sh[tid] : 0;
#pragma unroll
    for (int m = 1; m < 16; m <<= 1) {
      int y = __shfl_up(s, m, 64);
      if (lane >= m) s += y;
    }
    if (tid < 16) sh[16 + tid] = s;
  }
  __syncthreads();
  const int wexcl = (w == 0) ? 0 : sh[16 + w - 1];
  total = sh[16 + 15];
  const int r = wexcl + x - v;
  __syncthreads();
  return r;
}

// ---- 3. exclusive scans: segment offsets per column, cluster bases, chunk bases ----
// 3a. One thread per column: exclusive scan of the column over the segments
// (in place); base[j] and chunk_base[j] temporarily hold the column's rows
// and reduction chunks.
__global__ __launch_bounds__(256) void scan_col_kernel(int32_t* __restrict__ segsum, int k,
                                                       int32_t* __restrict__ base,
                                                       int32_t* __restrict__ chunk_base,
                                                       const int* __restrict__ gate) {
  if (gate && *gate) return;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= k) return;
  int run = 0;
  for (int s = 0; s < kScanSegs; ++s) {
    const int v = segsum[(int64_t)s * k + j];
    segsum[(int64_t)s * k + j] = run;
    run += v;
  }
  base[j] = run;
  chunk_base[j] = (run + kReduceRows - 1) / kReduceRows;
}

// 3b. One workgroup of 1024 threads: exclusive scans of the column totals.
// base[j] = first sorted position of cluster j (base[k] = number of valid
// rows); chunk_base likewise for reduction chunks.
__global__ __launch_bounds__(1024) void scan_top_kernel(int k, int32_t* __restrict__ base,
                                                        int32_t* __restrict__ chunk_base,
                                                        const int32_t* __restrict__ chg, int nb,
                                                        LoopState* __restrict__ st,
                                                        const int* __restrict__ gate) {
  if (gate && *gate) return;
  __shared__ int sh[64];
  if (chg) {
    // labels changed in this sort: the hist blocks' counts
    int c = 0;
    for (int b = threadIdx.x; b < 4 * nb; b += 1024) c += chg[b];
    int total_changed;
    block_excl_scan_1024(c, sh, total_changed);
    if (threadIdx.x == 0) st->changed += (unsigned long long)total_changed;
  }
  const int per = (k + 1023) / 1024;  // columns per thread, contiguous
  const int j0 = threadIdx.x * per;
  int tot_local = 0, ch_local = 0;
  for (int q = 0; q < per; ++q) {
    const int j = j0 + q;
    if (j < k) {
      tot_local += base[j];
      ch_local += chunk_base[j];
    }
  }
  int total_rows, total_chunks;
  int off = block_excl_scan_1024(tot_local, sh, total_rows);
  int coff = block_excl_scan_1024(ch_local, sh, total_chunks);
  for (int q = 0; q < per; ++q) {
    const int j = j0 + q;
    if (j < k) {
      const int t = base[j], c = chunk_base[j];
      base[j] = off;
      chunk_base[j] = coff;
      off += t;
      coff += c;
    }
  }
  if (threadIdx.x == 0) {
    base[k] = total_rows;
    chunk_base[k] = total_chunks;
  }
}

// ---- 4. per-block offsets: counts[b][j] <- base[j] + rows of j in earlier blocks ----
__global__ __launch_bounds__(256) void scan_fill_kernel(int32_t* __restrict__ counts, int nb,
                                                        int k, const int32_t* __restrict__ segsum,
                                                        const int32_t* __restrict__ base,
                                                        const int* __restrict__ gate) {
  if (gate && *gate) return;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int s = blockIdx.y;
  if (j >= k) return;
  const int per = (nb + kScanSegs - 1) / kScanSegs;
  const int b0 = s * per, b1 = min(nb, b0 + per);
  int run = base[j] + segsum[(int64_t)s * k + j];
  for (int b = b0; b < b1; ++b) {
    const int64_t o = (int64_t)b * k + j;
    const int c = counts[o];
    counts[o] = run;
    run += c;
  }
}

// ---- 5. stable scatter: one wave per block, 64 rows at a time; a row's
// rank among the step's rows of its cluster comes from the lanes below it
// whose label matches bit for bit ----
__global__ __launch_bounds__(64) void scatter_kernel(const int32_t* __restrict__ label, int64_t n,
                                                     int k, const int32_t* __restrict__ offs,
                                                     int32_t* __restrict__ perm,
                                                     const int* __restrict__ gate) {
  if (gate && *gate) return;
  extern __shared__ int cnt[];
  const int b = blockIdx.x;
  const int lane = threadIdx.x;
  const int32_t* ob = offs + (int64_t)b * k;
  for (int j = lane; j < k; j += 64) cnt[j] = ob[j];
  __syncthreads();
  const int64_t r0 = (int64_t)b * kSortRows;
  const int nbits = 32 - __clz(k);
  const unsigned long long below = (1ull << lane) - 1ull;
  constexpr int STEPS = kSortRows / 64, GRP = 8;
  for (int g = 0; g < STEPS; g += GRP) {
    if (r0 + 64 * g >= n) break;
    int labs[GRP];                     // eight steps' labels in flight together
#pragma unroll
    for (int c = 0; c < GRP; ++c) {
      const int64_t i = r0 + 64 * (g + c) + lane;
      labs[c] = (i < n) ? label[i] : -1;
    }
#pragma unroll
    for (int c = 0; c < GRP; ++c) {
      const int64_t i = r0 + 64 * (g + c) + lane;
      if (r0 + 64 * (g + c) >= n) break;
      int lab = labs[c];
      if (lab < 0 || lab >= k) lab = -1;
      // lanes holding the same label: one ballot per label bit (labels and
      // -1 differ in their low nbits bits, since k < 2^nbits)
      unsigned long long same = ~0ull;
      for (int bit = 0; bit < nbits; ++bit) {
        const bool on = (lab >> bit) & 1;
        const unsigned long long bal = __ballot(on);
        same &= on ? bal : ~bal;
      }
      const int rank = __popcll(same & below), tot = __popcll(same);
      int pos = 0;
      if (lab >= 0) pos = cnt[lab] + rank;
      __syncthreads();
      if (lab >= 0) {
        perm[pos] = (int32_t)i;
        if (rank == tot - 1) cnt[lab] = pos + 1;
      }
      __syncthreads();
    }
  }
}

hipError_t launch_sort(hipStream_t s, const int32_t* label, int32_t* lab_prev, int64_t n, int k,
                       int32_t* counts, int32_t* segsum, int32_t* base, int32_t* chunk_base,
                       int32_t* perm, LoopState* st, int track, const int* gate) {
  const int nb = (int)((n + kSortRows - 1) / kSortRows);
  const size_t lds = (size_t)k * sizeof(int);
  // with track, counts has 4 nb more entries after the nb x k matrix: the
  // numbers of changed labels per hist wave
  int32_t* chg = track ? counts + (int64_t)nb * k : nullptr;
  hipLaunchKernelGGL(hist_kernel, dim3(nb), dim3(256), lds, s, label, lab_prev, n, k, counts, chg,
                     track, gate);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  dim3 g2((k + 255) / 256, kScanSegs);
  hipLaunchKernelGGL(scan_seg_kernel, g2, dim3(256), 0, s, counts, nb, k, segsum, gate);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(scan_col_kernel, dim3((unsigned)((k + 255) / 256)), dim3(256), 0, s, segsum,
                     k, base, chunk_base, gate);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(scan_top_kernel, dim3(1), dim3(1024), 0, s, k, base, chunk_base, chg, nb, st,
                     gate);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(scan_fill_kernel, g2, dim3(256), 0, s, counts, nb, k, segsum, base, gate);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(scatter_kernel, dim3(nb), dim3(64), lds, s, label, n, k, counts, perm, gate);
  return hipGetLastError();
}

// ---- 6. exactly summed clustering features ----
// The sums are formed on a fixed-point grid per column: with 2^E_c an upper
// bound on |w_i x_ic| over all rows, the product w_i x_ic (exact in FP64) is
// scaled by 2^(62 - E_c) and cut toward zero into two 31-bit limbs,
//     v = w x 2^(62 - E_c) = h 2^31 + m + f,   |h|, |m| < 2^31,  |f| < 1,
// and only the integers h and m are summed (the fraction f, at most 2^-62 of
// the column's bound, is dropped).  Integer sums do not depend on their
// order, and cutting toward zero is odd, so removing a row later subtracts
// exactly what adding it added: the features of a cluster after rows moved
// in and out (Sec. 2.1: features add under union and subtract under removal)
// are the bits a fresh sum over its members gives.  W uses the grid of the
// largest weight and Q the grid of the largest w_i ||x_i||^2, with ||x_i||^2
// summed in FP64 in a fixed order per row.
//
// cfs layout (doubles): [0, d) column scales 2^(62 - E_c), [d, 2d) their
// inverses, then sW, 1/sW, sQ, 1/sQ.

// 6a. Column maxima of |x| (bit patterns of non-negative floats, atomicMax).
__global__ __launch_bounds__(256) void cf_colmax_kernel(const float* __restrict__ X, int64_t n,
                                                        int d, int64_t ldx,
                                                        int64_t rows_per_slice,
                                                        unsigned* __restrict__ colmax) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= d) return;
  const int64_t r0 = (int64_t)blockIdx.y * rows_per_slice;
  const int64_t r1 = min(n, r0 + rows_per_slice);
  float m = 0.0f;
#pragma unroll 8
  for (int64_t i = r0; i < r1; ++i) m = fmaxf(m, fabsf(X[i * ldx + c]));
  atomicMax(colmax + c, __float_as_uint(m));
}

// 6b. ||x_i||^2 in FP64, one wave per row: lane l sums columns l, l + 64, ...
// in order, then a butterfly (a fixed order).  The maximum goes to qmax as
// the bit pattern of a non-negative double.
__global__ __launch_bounds__(256) void cf_rowq_kernel(const float* __restrict__ X, int64_t n,
                                                      int d, int64_t ldx, double* __restrict__ q,
                                                      unsigned long long* __restrict__ qmax) {
  const int lane = threadIdx.x & 63;
  const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  double mx = 0.0;
  for (int64_t i = wid; i < n; i += nw) {
    const float* xr = X + i * ldx;
    double s = 0.0;
    for (int c = lane; c < d; c += 64) {
      const double x = (double)xr[c];
      s = fma(x, x, s);
    }
    s = wave_sum_f64(s);
    if (lane == 0) q[i] = s;
    mx = fmax(mx, s);
  }
  if (lane == 0) atomicMax(qmax, (unsigned long long)__double_as_longlong(mx));
}

// 6c. Largest weight (bit pattern of a non-negative float).
__global__ __launch_bounds__(256) void cf_wmax_kernel(const float* __restrict__ w, int64_t n,
                                                      unsigned* __restrict__ wmax) {
  float m = 0.0f;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    m = fmaxf(m, w[i]);
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) atomicMax(wmax, __float_as_uint(m));
}

// 2^(62 - E) with bound < 2^E (1 for a zero bound: every product is zero).
__device__ __forceinline__ double cf_scale(double bound) {
  if (!(bound > 0.0)) return 1.0;
  int e;
  (void)frexp(bound, &e);   // bound = f 2^e, f in [0.5, 1): bound < 2^e
  return ldexp(1.0, 62 - e);
}

// 6d. The grids of one call (one workgroup).  wmax == nullptr: unit weights.
__global__ __launch_bounds__(256) void cf_scales_kernel(const unsigned* __restrict__ colmax, int d,
                                                        const unsigned long long* __restrict__ qmax,
                                                        const unsigned* __restrict__ wmax,
                                                        double* __restrict__ cfs) {
  const double wm = wmax ? (double)__uint_as_float(*wmax) : 1.0;
  for (int c = threadIdx.x; c < d; c += 256) {
    const double s = cf_scale(wm * (double)__uint_as_float(colmax[c]));
    cfs[c] = s;
    cfs[d + c] = 1.0 / s;
  }
  if (threadIdx.x == 0) {
    const double sW = cf_scale(wm);
    // w_i ||x_i||^2 is rounded once in FP64: a factor 2 of margin
    const double sQ = cf_scale(2.0 * wm * __longlong_as_double((long long)*qmax));
    cfs[2 * d] = sW;
    cfs[2 * d + 1] = 1.0 / sW;
    cfs[2 * d + 2] = sQ;
    cfs[2 * d + 3] = 1.0 / sQ;
  }
}

// The two limbs of v (|v| < 2^62), cut toward zero.
__device__ __forceinline__ void cf_split(double v, double& h, double& m) {
  h = trunc(v * 0x1p-31);
  m = trunc(fma(-h, 0x1p31, v));
}

// 6e. Chunk reduction.  A chunk is at most kReduceRows entries of one
// cluster: rows of the sorted permutation (DELTA = false), or signed entries
// (DELTA = true: e >= 0 adds row e, e < 0 removes row -e - 1).  The chunk's
// row ids, signed weights and the W and Q limbs are staged first; then four
// waves walk the rows in an interleaved order (wave v: rows v, v + 4, ...),
// each wave split into SUB = 64 / LPR sub-waves of LPR lanes, a lane owning
// VEC consecutive columns in each of M column groups of LPR * VEC.  Each step
// takes UR rows per sub-wave; the next step's rows load while the current one
// is summed.  Partial limb sums are exact integers below 2^40 in FP64, so the
// combination order does not matter.  Chunks are taken in a grid-stride loop.
template <int VEC, int M, int LPR, bool DELTA, bool WEIGHTED>
__global__ __launch_bounds__(256) void cf_reduce_kernel(
    const float* __restrict__ X, int d, int64_t ldx, const float* __restrict__ w,
    const double* __restrict__ qrow, const int32_t* __restrict__ ent,
    const int32_t* __restrict__ base, const int32_t* __restrict__ chunk_base, int k,
    const double* __restrict__ cfs, double* __restrict__ partS, double* __restrict__ partWQ,
    const int* __restrict__ gate) {
  if (gate && *gate) return;
  constexpr int SUB = 64 / LPR;     // rows side by side in a wave
  constexpr int CB = LPR * VEC * M; // columns per pass
  constexpr int UR = 4;             // rows per sub-wave and step
  constexpr int RS = 4 * SUB;       // row stride between a sub-wave's rows
  __shared__ double sh[4][CB];
  __shared__ double shs[4][4];
  __shared__ int srow[kReduceRows];
  __shared__ float swt[kReduceRows];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int sub = lane / LPR, sl = lane % LPR;
  const int first = wv + 4 * sub;   // this sub-wave's rows: first, first + RS, ...
  const int nchunks = chunk_base[k];
  const double sW = cfs[2 * d], sQ = cfs[2 * d + 2];
  for (int cidx = blockIdx.x; cidx < nchunks; cidx += gridDim.x) {
    // cluster owning this chunk: last j with chunk_base[j] <= cidx
    int lo = 0, hi = k;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (chunk_base[mid] <= cidx) lo = mid; else hi = mid;
    }
    const int j = lo;
    const int64_t r0 = (int64_t)base[j] + (int64_t)(cidx - chunk_base[j]) * kReduceRows;
    const int64_t r1 = min((int64_t)base[j + 1], r0 + kReduceRows);
    const int nr = (int)(r1 - r0);
    double wh = 0.0, wm = 0.0, qh = 0.0, qm = 0.0;
    for (int t = threadIdx.x; t < nr; t += 256) {
      const int e = ent[r0 + t];
      const int i = DELTA ? (e >= 0 ? e : -e - 1) : e;
      const float wi = WEIGHTED ? w[i] : 1.0f;
      const float ws = (DELTA && e < 0) ? -wi : wi;
      srow[t] = i;
      swt[t] = ws;
      double h, m;
      cf_split((double)ws * sW, h, m);
      wh += h;
      wm += m;
      cf_split((double)ws * qrow[i] * sQ, h, m);
      qh += h;
      qm += m;
    }
    wh = wave_sum_f64(wh);
    wm = wave_sum_f64(wm);
    qh = wave_sum_f64(qh);
    qm = wave_sum_f64(qm);
    if (lane == 0) {
      shs[wv][0] = wh;
      shs[wv][1] = wm;
      shs[wv][2] = qh;
      shs[wv][3] = qm;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
      const int q = threadIdx.x;
      partWQ[(int64_t)cidx * 4 + q] = ((shs[0][q] + shs[1][q]) + shs[2][q]) + shs[3][q];
    }
    for (int cb = 0; cb < d; cb += CB) {
      double Sh[M][VEC], Sm[M][VEC], sc[M][VEC];
#pragma unroll
      for (int m = 0; m < M; ++m)
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
          const int c = cb + (m * LPR + sl) * VEC + v;
          sc[m][v] = (c < d) ? cfs[c] : 0.0;
          Sh[m][v] = Sm[m][v] = 0.0;
        }
      // rows t0 + RS u of one step, zeros past the chunk
      auto load_step = [&](int t0, float (&xv)[UR][M][VEC]) {
#pragma unroll
        for (int u = 0; u < UR; ++u) {
          const int t = t0 + RS * u;
          const bool rv = t < nr;
          const float* xr = X + (int64_t)(rv ? srow[t] : 0) * ldx + cb;
#pragma unroll
          for (int m = 0; m < M; ++m) {
            const int c0 = (m * LPR + sl) * VEC;
            if (VEC == 4 && rv && cb + c0 + 4 <= d) {
              const float4 t4 = *(const float4*)(xr + c0);
              xv[u][m][0] = t4.x;
              if (VEC == 4) { xv[u][m][1] = t4.y; xv[u][m][2] = t4.z; xv[u][m][3] = t4.w; }
            } else {
#pragma unroll
              for (int q = 0; q < VEC; ++q)
                xv[u][m][q] = (rv && cb + c0 + q < d) ? xr[c0 + q] : 0.0f;
            }
          }
        }
      };
      float xa[UR][M][VEC], xb[UR][M][VEC];
      load_step(first, xa);
      for (int t0 = first; t0 < nr; t0 += RS * UR) {
        const bool more = t0 + RS * UR < nr;
        if (more) load_step(t0 + RS * UR, xb);
#pragma unroll
        for (int u = 0; u < UR; ++u) {
          const int t = t0 + RS * u;
          // rows past the chunk carry x = 0 and weight 0: zero limbs
          const double wt = (t < nr) ? (double)swt[t] : 0.0;
#pragma unroll
          for (int m = 0; m < M; ++m)
#pragma unroll
            for (int q = 0; q < VEC; ++q) {
              const double xd = (double)xa[u][m][q];
              double h, l;
              if (WEIGHTED || DELTA) cf_split(wt * xd * sc[m][q], h, l);
              else cf_split(xd * sc[m][q], h, l);
              Sh[m][q] += h;
              Sm[m][q] += l;
            }
        }
        if (more) {
#pragma unroll
          for (int u = 0; u < UR; ++u)
#pragma unroll
            for (int m = 0; m < M; ++m)
#pragma unroll
              for (int q = 0; q < VEC; ++q) xa[u][m][q] = xb[u][m][q];
        }
      }
      // sub-waves, then waves (exact integer sums)
#pragma unroll
      for (int limb = 0; limb < 2; ++limb) {
#pragma unroll
        for (int m = 0; m < M; ++m)
#pragma unroll
          for (int q = 0; q < VEC; ++q) {
            double v = limb ? Sm[m][q] : Sh[m][q];
#pragma unroll
            for (int o = LPR; o < 64; o <<= 1) v += __shfl_xor(v, o, 64);
            if (sub == 0) sh[wv][(m * LPR + sl) * VEC + q] = v;
          }
        __syncthreads();
        for (int c = threadIdx.x; c < CB; c += 256) {
          if (cb + c < d)
            partS[((int64_t)cidx * d + cb + c) * 2 + limb] =
                ((sh[0][c] + sh[1][c]) + sh[2][c]) + sh[3][c];
        }
        __syncthreads();
      }
    }
  }
}

template <bool DELTA, bool WEIGHTED>
static void launch_cf_reduce_t(hipStream_t s, dim3 g, bool vec, const float* X, int d,
                               int64_t ldx, const float* w, const double* qrow,
                               const int32_t* ent, const int32_t* base,
                               const int32_t* chunk_base, int k, const double* cfs,
                               double* partS, double* partWQ, const int* gate) {
#define KMX_R(V, M, L)                                                                      \
  hipLaunchKernelGGL((cf_reduce_kernel<V, M, L, DELTA, WEIGHTED>), g, dim3(256), 0, s, X, d, \
                     ldx, w, qrow, ent, base, chunk_base, k, cfs, partS, partWQ, gate)
  // columns per pass: LPR * VEC * M, the smallest shape covering d (or 512)
  if (vec) {
    if (d > 256) KMX_R(4, 2, 64);
    else if (d > 128) KMX_R(4, 1, 64);
    else if (d > 64) KMX_R(4, 1, 32);
    else if (d > 32) KMX_R(4, 1, 16);
    else KMX_R(4, 1, 8);
  } else {
    if (d > 32) KMX_R(1, 1, 64);
    else if (d > 16) KMX_R(1, 1, 32);
    else KMX_R(1, 1, 16);
  }
#undef KMX_R
}

hipError_t launch_cf_prep(hipStream_t s, const float* X, int64_t n, int d, int64_t ldx,
                          unsigned* colmax, double* qrow, unsigned long long* qmax,
                          int num_cus) {
  hipError_t e = hipMemsetAsync(colmax, 0, (size_t)d * sizeof(unsigned), s);
  if (e != hipSuccess) return e;
  e = hipMemsetAsync(qmax, 0, sizeof(unsigned long long), s);
  if (e != hipSuccess) return e;
  const int tiles = (d + 255) / 256;
  int64_t slices = ((int64_t)num_cus * 8 + tiles - 1) / tiles;
  if (slices > n) slices = n;
  if (slices < 1) slices = 1;
  const int64_t rps = (n + slices - 1) / slices;
  hipLaunchKernelGGL(cf_colmax_kernel, dim3(tiles, (unsigned)slices), dim3(256), 0, s, X, n, d,
                     ldx, rps, colmax);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  int64_t blocks = (n + 3) / 4;
  if (blocks > (int64_t)num_cus * 16) blocks = (int64_t)num_cus * 16;
  hipLaunchKernelGGL(cf_rowq_kernel, dim3((unsigned)blocks), dim3(256), 0, s, X, n, d, ldx, qrow,
                     qmax);
  return hipGetLastError();
}

hipError_t launch_cf_scales(hipStream_t s, const unsigned* colmax, int d,
                            const unsigned long long* qmax, const float* w, int64_t n,
                            unsigned* wmax, double* cfs, int num_cus) {
  if (w) {
    hipError_t e = hipMemsetAsync(wmax, 0, sizeof(unsigned), s);
    if (e != hipSuccess) return e;
    int64_t blocks = (n + 255) / 256;
    if (blocks > (int64_t)num_cus * 4) blocks = (int64_t)num_cus * 4;
    hipLaunchKernelGGL(cf_wmax_kernel, dim3((unsigned)blocks), dim3(256), 0, s, w, n, wmax);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(cf_scales_kernel, dim3(1), dim3(256), 0, s, colmax, d, qmax,
                     w ? wmax : nullptr, cfs);
  return hipGetLastError();
}

hipError_t launch_reduce(hipStream_t s, const float* X, int64_t n, int d, int64_t ldx,
                         const float* w, const double* qrow, const int32_t* ent,
                         const int32_t* base, const int32_t* chunk_base, int k,
                         const double* cfs, double* partS, double* partWQ, int delta,
                         int num_cus, const int* gate) {
  const int64_t maxchunks = (n + kReduceRows - 1) / kReduceRows + k;
  const bool vec = ((((uintptr_t)X) & 15) == 0) && (ldx % 4 == 0);
  // the full reduction takes one workgroup per possible chunk; the delta one
  // (whose chunk count is only known on the device) a grid-stride loop
  int64_t blocks = maxchunks;
  if (delta && blocks > (int64_t)num_cus * 4) blocks = (int64_t)num_cus * 4;
  const dim3 g((unsigned)blocks);
  if (delta) {
    if (w) launch_cf_reduce_t<true, true>(s, g, vec, X, d, ldx, w, qrow, ent, base, chunk_base, k, cfs, partS, partWQ, gate);
    else launch_cf_reduce_t<true, false>(s, g, vec, X, d, ldx, w, qrow, ent, base, chunk_base, k, cfs, partS, partWQ, gate);
  } else {
    if (w) launch_cf_reduce_t<false, true>(s, g, vec, X, d, ldx, w, qrow, ent, base, chunk_base, k, cfs, partS, partWQ, gate);
    else launch_cf_reduce_t<false, false>(s, g, vec, X, d, ldx, w, qrow, ent, base, chunk_base, k, cfs, partS, partWQ, gate);
  }
  return hipGetLastError();
}

// ---- 7. per-cluster finalize: chunk sums (+ the carried features), new
// center, cost terms ----
// Limb sums of one feature: the chunks' exact FP64 integers summed in int64.
// acc (nullable) holds the cluster's features across calls of one Lloyd run:
// mode 1 stores the sums in it, mode 0 adds them to it (the chunks then hold
// the changes of a delta reduction).  *mode_p selects the mode and the chunk
// bases (chunk_base for mode 1, dchunk for mode 0); mode_p == nullptr: mode 1.
__device__ __forceinline__ double cf_value(long long H, long long Mlo, double inv) {
  // H 2^31 + Mlo with Mlo reduced to [0, 2^31), then one conversion
  const long long carry = Mlo >> 31;   // floor division (arithmetic shift)
  const long long ml = Mlo - carry * (1ll << 31);
  const long long hh = H + carry;
  return fma((double)hh, 0x1p31, (double)ml) * inv;
}

__global__ __launch_bounds__(256) void cf_finalize_kernel(
    const double* __restrict__ partS, const double* __restrict__ partWQ,
    const int32_t* __restrict__ chunk_base, const int32_t* __restrict__ dchunk,
    const int* __restrict__ mode_p, long long* __restrict__ acc, int k, int d,
    const double* __restrict__ cfs, const float* C_prev, float* C_out, double* __restrict__ W_out,
    double* __restrict__ termC, double* __restrict__ termMu, int write_c,
    LoopState* __restrict__ st, const int* __restrict__ gate) {
  if (gate && *gate) return;
  __shared__ double red[3][4];
  __shared__ double sWQ[2];
  __shared__ long long shWQ[4][4];
  __shared__ long long shS[256][2];
  const int j = blockIdx.x;
  const int mode = mode_p ? *mode_p : 1;
  const int32_t* cbp = mode ? chunk_base : dchunk;
  const int c0 = cbp[j], c1 = cbp[j + 1];
  long long* accS = acc ? acc + (int64_t)j * d * 2 : nullptr;
  long long* accWQ = acc ? acc + (int64_t)k * d * 2 + (int64_t)j * 4 : nullptr;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  // chunk partials are integers (exact in FP64 and int64): any summation
  // order gives the same sums, so every thread takes a strided share
  {
    long long w4[4] = {0, 0, 0, 0};
    for (int c = c0 + tid; c < c1; c += 256)
#pragma unroll
      for (int q = 0; q < 4; ++q) w4[q] += (long long)partWQ[(int64_t)c * 4 + q];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
#pragma unroll
      for (int m = 32; m >= 1; m >>= 1) w4[q] += __shfl_xor(w4[q], m, 64);
      if (lane == 0) shWQ[q][wv] = w4[q];
    }
  }
  __syncthreads();
  if (tid < 4) {
    const int q = tid;
    long long s = (!mode && accWQ) ? accWQ[q] : 0ll;
    s += ((shWQ[q][0] + shWQ[q][1]) + shWQ[q][2]) + shWQ[q][3];
    if (accWQ) accWQ[q] = s;
    // lanes 0 and 1 form W, lanes 2 and 3 form Q
    const long long o = __shfl_xor(s, 1, 64);
    if (q == 0) sWQ[0] = cf_value(s, o, cfs[2 * d + 1]);
    if (q == 2) sWQ[1] = cf_value(s, o, cfs[2 * d + 3]);
  }
  // columns: for d <= 128 the block's threads form G = 256 / d groups over
  // the chunks of each column, combined in LDS; thread col then owns column col
  const int G = (d <= 128) ? 256 / d : 1;
  long long gH = 0, gL = 0;
  if (G > 1 && tid < G * d) {
    const int col = tid % d, grp = tid / d;
    for (int c = c0 + grp; c < c1; c += G) {
      const double* p = partS + ((int64_t)c * d + col) * 2;
      gH += (long long)p[0];
      gL += (long long)p[1];
    }
    shS[tid][0] = gH;
    shS[tid][1] = gL;
  }
  __syncthreads();
  const double W = sWQ[0], Q = sWQ[1];
  double dotCS = 0.0, cn2 = 0.0, s2 = 0.0;
  for (int col = threadIdx.x; col < d; col += 256) {
    long long H = 0, L = 0;
    if (!mode && accS) {
      H = accS[col * 2];
      L = accS[col * 2 + 1];
    }
    if (G > 1) {
      for (int g = 0; g < G; ++g) {
        H += shS[g * d + col][0];
        L += shS[g * d + col][1];
      }
    } else {
      for (int c = c0; c < c1; ++c) {
        const double* p = partS + ((int64_t)c * d + col) * 2;
        H += (long long)p[0];
        L += (long long)p[1];
      }
    }
    if (accS) {
      accS[col * 2] = H;
      accS[col * 2 + 1] = L;
    }
    const double S = cf_value(H, L, cfs[d + col]);
    const float cp = C_prev[(int64_t)j * d + col];
    const double cpd = (double)cp;
    dotCS += cpd * S;
    cn2 += cpd * cpd;
    s2 += S * S;
    if (write_c) C_out[(int64_t)j * d + col] = (W > 0.0) ? (float)(S / W) : cp;
  }
  dotCS = wave_sum_f64(dotCS);
  cn2 = wave_sum_f64(cn2);
  s2 = wave_sum_f64(s2);
  if (lane == 0) {
    red[0][wv] = dotCS;
    red[1][wv] = cn2;
    red[2][wv] = s2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double a = ((red[0][0] + red[0][1]) + red[0][2]) + red[0][3];
    const double b = ((red[1][0] + red[1][1]) + red[1][2]) + red[1][3];
    const double e = ((red[2][0] + red[2][1]) + red[2][2]) + red[2][3];
    termC[j] = Q - 2.0 * a + W * b;
    termMu[j] = (W > 0.0) ? (Q - e / W) : 0.0;
    if (W_out) W_out[j] = W;
    if (acc && st && j == 0) st->acc_valid = 1;
  }
}

hipError_t launch_finalize(hipStream_t s, const double* partS, const double* partWQ,
                           const int32_t* chunk_base, const int32_t* dchunk, const int* mode_p,
                           long long* acc, int k, int d, const double* cfs, const float* C_prev,
                           float* C_out, double* W_out, double* termC, double* termMu,
                           int write_c, LoopState* st, const int* gate) {
  hipLaunchKernelGGL(cf_finalize_kernel, dim3(k), dim3(256), 0, s, partS, partWQ, chunk_base,
                     dchunk, mode_p, acc, k, d, cfs, C_prev, C_out, W_out, termC, termMu, write_c,
                     st, gate);
  return hipGetLastError();
}

// ---- delta update: the rows whose label changed ----
// A mark workgroup takes kMarkRows rows (32 per thread, one bit each in the
// change mask): its two same-address atomics (list position, change count)
// serialize across workgroups, so fewer, larger workgroups are faster
// (8192 rows: 43 -> 26 us at n = 4M).
constexpr int kMarkRows = 8192;
// mark: changed rows (label != previous label) are listed with their previous
// label (block-aggregated positions, any order), the per-cluster entry counts
// (one removal from the old cluster, one addition to the new) are added to
// ecount, the previous labels are brought up to date and the number of
// changes goes to st->changed (the stopping rule) and st->dcount (the list).
__global__ __launch_bounds__(256) void delta_mark_kernel(const int32_t* __restrict__ label,
                                                         int32_t* __restrict__ lab_prev, int64_t n,
                                                         int k, int32_t* __restrict__ ecount,
                                                         int32_t* __restrict__ clist,
                                                         int32_t* __restrict__ cold,
                                                         LoopState* __restrict__ st,
                                                         const int* __restrict__ gate) {
  if (gate && *gate) return;
  extern __shared__ int hsm[];
  __shared__ int wcnt[4];
  __shared__ int bbase;
  constexpr int PER = kMarkRows / 256;
  const int64_t r0 = (int64_t)blockIdx.x * kMarkRows;
  const int64_t r1 = min(n, r0 + kMarkRows);
  int lab[PER], prev[PER];
  unsigned chm = 0;
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int64_t i = r0 + threadIdx.x + 256 * q;
    lab[q] = (i < r1) ? label[i] : -1;
    prev[q] = (i < r1) ? lab_prev[i] : -1;
    if (i < r1 && lab[q] != prev[q]) chm |= 1u << q;
  }
  for (int j = threadIdx.x; j < k; j += blockDim.x) hsm[j] = 0;
  __syncthreads();
  const int cnt = __popc(chm);
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    if (chm & (1u << q)) {
      const int64_t i = r0 + threadIdx.x + 256 * q;
      if (lab[q] >= 0 && lab[q] < k) atomicAdd(&hsm[lab[q]], 1);
      if (prev[q] >= 0 && prev[q] < k) atomicAdd(&hsm[prev[q]], 1);
      lab_prev[i] = lab[q];
    }
  }
  // block-exclusive offsets of the changed rows
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int x = cnt;
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) {
    const int y = __shfl_up(x, m, 64);
    if (lane >= m) x += y;
  }
  if (lane == 63) wcnt[wv] = x;
  __syncthreads();
  int woff = 0;
  for (int v = 0; v < wv; ++v) woff += wcnt[v];
  if (threadIdx.x == 0) {
    const int tot = wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];
    bbase = tot ? (int)atomicAdd(&st->dcount, (unsigned long long)tot) : 0;
    if (tot) atomicAdd(&st->changed, (unsigned long long)tot);
  }
  __syncthreads();
  int pos = bbase + woff + x - cnt;
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    if (chm & (1u << q)) {
      clist[pos] = (int32_t)(r0 + threadIdx.x + 256 * q);
      cold[pos] = prev[q];
      ++pos;
    }
  }
  for (int j = threadIdx.x; j < k; j += blockDim.x)
    if (hsm[j]) atomicAdd(ecount + j, hsm[j]);
}

// plan (one workgroup of 1024): full reduction when the carried features are
// not valid or more than half of the rows changed, else the delta one; with
// the gate set (a stopped loop) both paths are skipped.
// flags[0] = skip the full path, flags[1] = skip the delta path, flags[2] =
// finalize mode (1 full, 0 delta).  The delta path gets its cluster segment
// bases (ebase, also the scatter cursors) and chunk bases (dchunk).  ecount
// is cleared for the next mark.
__global__ __launch_bounds__(1024) void delta_plan_kernel(int32_t* __restrict__ ecount, int k,
                                                          int64_t n, int32_t* __restrict__ ebase,
                                                          int32_t* __restrict__ cursor,
                                                          int32_t* __restrict__ dchunk,
                                                          int* __restrict__ flags,
                                                          LoopState* __restrict__ st,
                                                          const int* __restrict__ gate) {
  __shared__ int sh[64];
  __shared__ int sfull;
  if (threadIdx.x == 0) {
    const int done = gate ? *gate : 0;
    const int full = !st->acc_valid || (int64_t)st->dcount * 2 > n;
    sfull = done ? -1 : full;
    flags[0] = done ? 1 : !full;
    flags[1] = done ? 1 : full;
    flags[2] = full;
  }
  __syncthreads();
  const int f = sfull;
  if (f < 0) return;   // stopped: mark did not run, ecount is still clear
  const int per = (k + 1023) / 1024;
  const int j0 = threadIdx.x * per;
  int tot = 0, ch = 0;
  for (int q = 0; q < per; ++q) {
    const int j = j0 + q;
    if (j < k) {
      tot += ecount[j];
      ch += (ecount[j] + kReduceRows - 1) / kReduceRows;
    }
  }
  if (f) {
    for (int q = 0; q < per; ++q)
      if (j0 + q < k) ecount[j0 + q] = 0;
    return;
  }
  int total, totalc;
  int off = block_excl_scan_1024(tot, sh, total);
  int coff = block_excl_scan_1024(ch, sh, totalc);
  for (int q = 0; q < per; ++q) {
    const int j = j0 + q;
    if (j < k) {
      const int e = ecount[j];
      ebase[j] = off;
      cursor[j] = off;
      dchunk[j] = coff;
      off += e;
      coff += (e + kReduceRows - 1) / kReduceRows;
      ecount[j] = 0;
    }
  }
  if (threadIdx.x == 0) {
    ebase[k] = total;
    dchunk[k] = totalc;
  }
}

// scatter: every changed row becomes a removal entry in its old cluster's
// segment and an addition entry in its new one.  A workgroup takes a
// contiguous slice of the changed rows, counts its entries per cluster in LDS,
// reserves each cluster's range with one global atomic, and places the
// entries with LDS atomics (any order within a segment: the features are
// exact sums).  Per-row global atomics on the k cursors would serialize when
// many rows change and k is small.
__global__ __launch_bounds__(256) void delta_scatter_kernel(const int32_t* __restrict__ label,
                                                            const int32_t* __restrict__ clist,
                                                            const int32_t* __restrict__ cold, int k,
                                                            int32_t* __restrict__ cursor,
                                                            int32_t* __restrict__ ent,
                                                            const LoopState* __restrict__ st,
                                                            const int* __restrict__ gate) {
  if (gate && *gate) return;
  extern __shared__ int hs[];   // k counters: counts, then positions
  const int64_t cnt = (int64_t)st->dcount;
  const int64_t per = (cnt + gridDim.x - 1) / gridDim.x;
  const int64_t q0 = (int64_t)blockIdx.x * per;
  const int64_t q1 = min(cnt, q0 + per);
  if (q0 >= q1) return;   // uniform within the workgroup
  for (int j = threadIdx.x; j < k; j += blockDim.x) hs[j] = 0;
  __syncthreads();
  for (int64_t q = q0 + threadIdx.x; q < q1; q += blockDim.x) {
    const int o = cold[q];
    const int nw = label[clist[q]];
    if (o >= 0 && o < k) atomicAdd(&hs[o], 1);
    if (nw >= 0 && nw < k) atomicAdd(&hs[nw], 1);
  }
  __syncthreads();
  for (int j = threadIdx.x; j < k; j += blockDim.x) {
    const int c = hs[j];
    hs[j] = c ? atomicAdd(cursor + j, c) : 0;
  }
  __syncthreads();
  for (int64_t q = q0 + threadIdx.x; q < q1; q += blockDim.x) {
    const int i = clist[q];
    const int o = cold[q];
    const int nw = label[i];
    if (o >= 0 && o < k) ent[atomicAdd(&hs[o], 1)] = -i - 1;
    if (nw >= 0 && nw < k) ent[atomicAdd(&hs[nw], 1)] = i;
  }
}

hipError_t launch_delta_prepare(hipStream_t s, const int32_t* label, int32_t* lab_prev, int64_t n,
                                int k, int32_t* ecount, int32_t* clist, int32_t* cold,
                                int32_t* ebase, int32_t* cursor, int32_t* dchunk, int32_t* ent,
                                int* flags, LoopState* st, int num_cus, const int* gate) {
  const int nb = (int)((n + kMarkRows - 1) / kMarkRows);
  hipLaunchKernelGGL(delta_mark_kernel, dim3(nb), dim3(256), (size_t)k * sizeof(int), s, label,
                     lab_prev, n, k, ecount, clist, cold, st, gate);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(delta_plan_kernel, dim3(1), dim3(1024), 0, s, ecount, k, n, ebase, cursor,
                     dchunk, flags, st, gate);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  int64_t blocks = (n + 255) / 256;
  if (blocks > (int64_t)num_cus * 4) blocks = (int64_t)num_cus * 4;
  hipLaunchKernelGGL(delta_scatter_kernel, dim3((unsigned)blocks), dim3(256),
                     (size_t)k * sizeof(int), s, label, clist, cold, k, cursor, ent, st, flags + 1);
  return hipGetLastError();
}

// ---- 8. cost sums and loop control (one workgroup) ----
// mode 0: Lloyd iteration -> cost_hist[iter], stopping rule, iter += 1
// mode 1: final assignment -> cost_hist[iter]
// mode 2: store both sums in the state (standalone update / cost)
__global__ __launch_bounds__(256) void cost_sum_kernel(const double* __restrict__ termC,
                                                       const double* __restrict__ termMu, int k,
                                                       LoopState* __restrict__ st,
                                                       double* __restrict__ cost_hist, int mode,
                                                       const int* __restrict__ gate) {
  if (gate && *gate) return;
  __shared__ double red[2][4];
  double a = 0.0, b = 0.0;
  for (int j = threadIdx.x; j < k; j += 256) {
    a += termC[j];
    b += termMu[j];
  }
  a = wave_sum_f64(a);
  b = wave_sum_f64(b);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) {
    red[0][wv] = a;
    red[1][wv] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double cC = ((red[0][0] + red[0][1]) + red[0][2]) + red[0][3];
    const double cM = ((red[1][0] + red[1][1]) + red[1][2]) + red[1][3];
    st->cost_last = cC;
    st->cost_at_centroids = cM;
    if (mode == 0) {
      const int t = st->iter;
      cost_hist[t] = cC;
      st->iter = t + 1;
      if (st->tol >= 0.0 && t >= 1) {
        const double prev = cost_hist[t - 1];
        if (st->changed == 0ull || (prev - cC) <= st->tol * prev) st->done = 1;
      }
      if (t + 1 >= st->max_iter) st->done = 1;
      st->changed = 0ull;
    } else if (mode == 1) {
      cost_hist[st->iter] = cC;
    }
  }
}

hipError_t launch_cost_sum(hipStream_t s, const double* termC, const double* termMu, int k,
                           LoopState* st, double* cost_hist, int mode, const int* gate) {
  hipLaunchKernelGGL(cost_sum_kernel, dim3(1), dim3(256), 0, s, termC, termMu, k, st, cost_hist,
                     mode, gate);
  return hipGetLastError();
}

}  // namespace kmx
