// Update step of Lloyd's algorithm (Sec. 1: replace each center by the
// centroid of its subset) as a deterministic, HBM-bound segmented reduction.
//
// For every cluster j the kernels form the weighted clustering feature of
// Sec. 2.1 / Sec. 2.3.1: W_j = sum w_i, S_j = sum w_i x_i, Q_j = sum w_i ||x_i||^2
// in FP64 (w_i x_i is exact in FP64).  The cost of the partition against any
// center c follows from the identity of Sec. 2.1:
//     sum_{i in P_j} w_i ||x_i - c||^2 = Q_j - 2 c.S_j + W_j ||c||^2 .
//
// Mechanism: a stable counting sort of row ids by label (block histograms,
// column scans, in-block ranks from one ballot per label bit), then one workgroup
// per chunk of at most kReduceRows rows of one cluster gathers whole rows
// (coalesced) and accumulates FP64 partial features, and one workgroup per
// cluster sums its chunks in chunk order.  Every sum has a fixed order, so the
// results are bitwise reproducible.
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

// ---- 6. chunk reduction: FP64 (S, Q, W) over at most kReduceRows rows ----
// The chunk's row ids and weights are staged in LDS first.  Four waves walk
// the chunk's rows in an interleaved, fixed order (wave v: rows v, v + 4,
// ...).  A wave is split into SUB = 64 / LPR sub-waves of LPR lanes, each on
// its own row, so short rows still occupy every lane; a lane owns VEC
// consecutive columns in each of M column groups of LPR*VEC.  Each step takes
// UR rows per sub-wave; the next step's rows are loaded while the current
// step is summed.  The sub-waves' partial sums are combined by a butterfly
// (same bits on every lane), the waves in a fixed order.
template <int VEC, int M, int LPR>
__global__ __launch_bounds__(256) void reduce_kernel(const float* __restrict__ X, int d,
                                                     int64_t ldx, const float* __restrict__ w,
                                                     const int32_t* __restrict__ perm,
                                                     const int32_t* __restrict__ base,
                                                     const int32_t* __restrict__ chunk_base,
                                                     int k, double* __restrict__ partS,
                                                     double* __restrict__ partQ,
                                                     double* __restrict__ partW,
                                                     const int* __restrict__ gate) {
  if (gate && *gate) return;
  constexpr int SUB = 64 / LPR;     // rows side by side in a wave
  constexpr int CB = LPR * VEC * M; // columns per pass
  constexpr int UR = 4;             // rows per sub-wave and step
  constexpr int RS = 4 * SUB;       // row stride between a sub-wave's rows
  __shared__ double sh[4][CB];
  __shared__ double shq[4], shw[4];
  __shared__ int srow[kReduceRows];
  __shared__ float swt[kReduceRows];
  const int cidx = blockIdx.x;
  if (cidx >= chunk_base[k]) return;
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
  for (int t = threadIdx.x; t < nr; t += 256) {
    const int i = perm[r0 + t];
    srow[t] = i;
    swt[t] = w ? w[i] : 1.0f;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int sub = lane / LPR, sl = lane % LPR;
  const int first = wv + 4 * sub;   // this sub-wave's rows: first, first + RS, ...
  double qacc = 0.0, wacc = 0.0;
  for (int cb = 0; cb < d; cb += CB) {
    double S[M][VEC], Q[M][VEC];
#pragma unroll
    for (int m = 0; m < M; ++m)
#pragma unroll
      for (int v = 0; v < VEC; ++v) S[m][v] = Q[m][v] = 0.0;
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
        const double wt = (t < nr) ? (double)swt[t] : 0.0;
        if (cb == 0) wacc += wt;
#pragma unroll
        for (int m = 0; m < M; ++m)
#pragma unroll
          for (int q = 0; q < VEC; ++q) {
            const double xd = (double)xa[u][m][q];
            const double wx = wt * xd;
            S[m][q] += wx;
            Q[m][q] = fma(wx, xd, Q[m][q]);
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
    // sub-waves, then waves, in a fixed order
#pragma unroll
    for (int m = 0; m < M; ++m)
#pragma unroll
      for (int q = 0; q < VEC; ++q) {
        double v = S[m][q];
#pragma unroll
        for (int o = LPR; o < 64; o <<= 1) v += __shfl_xor(v, o, 64);
        if (sub == 0) sh[wv][(m * LPR + sl) * VEC + q] = v;
        qacc += Q[m][q];
      }
    __syncthreads();
    for (int c = threadIdx.x; c < CB; c += 256) {
      if (cb + c < d)
        partS[(int64_t)cidx * d + cb + c] = ((sh[0][c] + sh[1][c]) + sh[2][c]) + sh[3][c];
    }
    __syncthreads();
  }
  qacc = wave_sum_f64(qacc);
#pragma unroll
  for (int o = LPR; o < 64; o <<= 1) wacc += __shfl_xor(wacc, o, 64);
  if (lane == 0) {
    shq[wv] = qacc;
    shw[wv] = wacc;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    partQ[cidx] = ((shq[0] + shq[1]) + shq[2]) + shq[3];
    partW[cidx] = ((shw[0] + shw[1]) + shw[2]) + shw[3];
  }
}

hipError_t launch_reduce(hipStream_t s, const float* X, int64_t n, int d, int64_t ldx,
                         const float* w, const int32_t* perm, const int32_t* base,
                         const int32_t* chunk_base, int k, double* partS, double* partQ,
                         double* partW, const int* gate) {
  const int64_t maxchunks = (n + kReduceRows - 1) / kReduceRows + k;
  const bool vec = ((((uintptr_t)X) & 15) == 0) && (ldx % 4 == 0);
  dim3 g((unsigned)maxchunks);
#define KMX_R(V, M, L)                                                                         \
  hipLaunchKernelGGL((reduce_kernel<V, M, L>), g, dim3(256), 0, s, X, d, ldx, w, perm, base, \
                     chunk_base, k, partS, partQ, partW, gate)
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
  return hipGetLastError();
}

// ---- 7. per-cluster finalize: sum chunks, new center, cost terms ----
__global__ __launch_bounds__(256) void finalize_kernel(
    const double* __restrict__ partS, const double* __restrict__ partQ,
    const double* __restrict__ partW, const int32_t* __restrict__ chunk_base, int k, int d,
    const float* C_prev, float* C_out, double* __restrict__ W_out, double* __restrict__ termC,
    double* __restrict__ termMu, int write_c, const int* __restrict__ gate) {
  if (gate && *gate) return;
  __shared__ double red[3][4];
  const int j = blockIdx.x;
  const int c0 = chunk_base[j], c1 = chunk_base[j + 1];
  // chunk sums in chunk order; unrolled so that the loads issue together
  double W = 0.0, Q = 0.0;
#pragma unroll 8
  for (int c = c0; c < c1; ++c) {
    W += partW[c];
    Q += partQ[c];
  }
  double dotCS = 0.0, cn2 = 0.0, s2 = 0.0;
  for (int col = threadIdx.x; col < d; col += 256) {
    double S = 0.0;
#pragma unroll 8
    for (int c = c0; c < c1; ++c) S += partS[(int64_t)c * d + col];
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
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
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
  }
}

hipError_t launch_finalize(hipStream_t s, const double* partS, const double* partQ,
                           const double* partW, const int32_t* chunk_base, int k, int d,
                           const float* C_prev, float* C_out, double* W_out, double* termC,
                           double* termMu, int write_c, const int* gate) {
  hipLaunchKernelGGL(finalize_kernel, dim3(k), dim3(256), 0, s, partS, partQ, partW, chunk_base,
                     k, d, C_prev, C_out, W_out, termC, termMu, write_c, gate);
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
