// Exact re-check of the rows the assignment GEMM could not decide (Sec. 1:
// every point goes to its closest center; the squared Euclidean distance).
//   pair entry: the two or three listed candidates;
//   full entry: every center.
// Plain FP32 direct differences decide when their error bound separates the
// candidates; otherwise double-float (TwoSum / TwoProd) sums decide, so the
// labels agree with exact arithmetic except on ties closer than about 1e-13
// relative.  One wave per pair entry, one workgroup per full entry; the
// batched versions find the entry's bucket or instance by binary search.
#include "kmx_device.h"
#include "kmx_internal.h"

namespace kmx {

// Exact distance of one row pair with double-float sums, the G lanes of a
// group (lane = index within the group) splitting the coordinates.
template <int G = 64>
__device__ __forceinline__ void exact_dist(const float* __restrict__ x,
                                           const float* __restrict__ c, int d, int lane,
                                           float& hi, float& lo) {
  float s = 0.f, e = 0.f;
  for (int q = lane; q < d; q += G) df_acc_sqdiff(x[q], c[q], s, e);
  wave_sum_df<G>(s, e);
  df_norm(s, e, hi, lo);
}

// Short re-check: the listed 2 or 3 candidates, one group of G lanes per
// entry (64 / G entries per wave at once).  Plain FP32 distances first: each
// lane sums the squares of its own coordinates (four consecutive ones per
// 4G-column step, or one per G-column step when rows are not 16-byte aligned:
// at most ceil(d/G) + 3 terms), then a log2(G)-level butterfly, so the
// relative error is below (ceil(d/G) + 13) u.  When the best plain distance
// beats every other candidate by more than that bound the result is exact;
// otherwise the candidates are compared with double-float sums.  The next
// entry and its current label are fetched one entry ahead.
template <int G = 64>
__device__ __forceinline__ void plain_dist3(const float* __restrict__ x,
                                            const float* __restrict__ c0,
                                            const float* __restrict__ c1,
                                            const float* __restrict__ c2, int d, int lane,
                                            bool vec, float& p0, float& p1, float& p2) {
  float a0 = 0.f, a1 = 0.f, a2 = 0.f;
  if (vec) {
#pragma unroll 4
    for (int q = lane * 4; q < d; q += 4 * G) {
      const float4 xv = *(const float4*)(x + q);
      const float4 u0 = *(const float4*)(c0 + q);
      const float4 u1 = *(const float4*)(c1 + q);
      const float4 u2 = *(const float4*)(c2 + q);
      const float xs[4] = {xv.x, xv.y, xv.z, xv.w};
      const float v0[4] = {u0.x, u0.y, u0.z, u0.w};
      const float v1[4] = {u1.x, u1.y, u1.z, u1.w};
      const float v2[4] = {u2.x, u2.y, u2.z, u2.w};
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        float df = xs[e] - v0[e];
        a0 = __builtin_fmaf(df, df, a0);
        df = xs[e] - v1[e];
        a1 = __builtin_fmaf(df, df, a1);
        df = xs[e] - v2[e];
        a2 = __builtin_fmaf(df, df, a2);
      }
    }
  } else {
    for (int q = lane; q < d; q += G) {
      const float xq = x[q];
      float df = xq - c0[q];
      a0 = __builtin_fmaf(df, df, a0);
      df = xq - c1[q];
      a1 = __builtin_fmaf(df, df, a1);
      df = xq - c2[q];
      a2 = __builtin_fmaf(df, df, a2);
    }
  }
#pragma unroll
  for (int m = G / 2; m >= 1; m >>= 1) {
    a0 += __shfl_xor(a0, m, 64);
    a1 += __shfl_xor(a1, m, 64);
    a2 += __shfl_xor(a2, m, 64);
  }
  p0 = a0;
  p1 = a1;
  p2 = a2;
}

// Carried bounds of a re-checked row (when kept), from the plain distances
// (relative error below tol each, taken twice): the winner's upper bound, the
// closest other candidate as the runner-up, and a third candidate folded into
// the bound of the centers not listed (which the listing pass stored).
__device__ __forceinline__ void pair_bounds(const BoundsOut& bo, int row, const float* p,
                                            const int* cj, int nc, int best, float tol) {
  const double t2 = 2.0 * (double)tol;
  double ub2 = 0.0, ru2 = 1e308, th2 = 1e308;
  int ru = -1;
  for (int q = 0; q < nc; ++q) {
    const double v = (double)p[q];
    if (cj[q] == best) {
      ub2 = v;
    } else if (v < ru2) {
      th2 = ru2;
      ru2 = v;
      ru = cj[q];
    } else {
      th2 = fmin(th2, v);
    }
  }
  bo.ub[row] = dist_up(ub2 * (1.0 + t2));
  bo.sec[row] = ru;
  bo.l2[row] = dist_down(ru2 * (1.0 - t2));
  if (th2 < 1e300) bo.lb[row] = fminf(bo.lb[row], dist_down(th2 * (1.0 - t2)));
}

template <int G>
__global__ __launch_bounds__(256) void recheck_pair_kernel(
    const float* __restrict__ X, int64_t n, int d, int64_t ldx, const float* __restrict__ C,
    int k, int32_t* __restrict__ label, float* __restrict__ d1o,
    const FlagEntry* __restrict__ flags, const LoopState* __restrict__ st,
    const int* __restrict__ gate, BoundsOut bo) {
  if (gate && *gate) return;
  constexpr int SPW = 64 / G;          // entries per wave at once
  const int64_t cnt = (int64_t)st->flagged;
  const int lane = threadIdx.x & 63, gl = lane % G, grp = lane / G;
  const int64_t gw = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * SPW + grp;
  const int64_t nw = (int64_t)gridDim.x * 4 * SPW;
  const float tol = (float)((d + G - 1) / G + 13) * 5.9604645e-8f;
  const bool vec = ((((uintptr_t)X) & 15) == 0) && (ldx % 4 == 0) &&
                   ((((uintptr_t)C) & 15) == 0) && (d % 4 == 0);
  // entries each row appears in at most once, so a label fetched ahead is
  // never one this kernel writes before reading it
  FlagEntry fe_n = {-1, -1, -1, 0};
  int lab_n = 0;
  if (gw < cnt) {
    fe_n = flags[gw];
    lab_n = (fe_n.row >= 0 && fe_n.row < n) ? label[fe_n.row] : 0;
  }
  for (int64_t e = gw; e < cnt; e += nw) {   // uniform within a group
    const FlagEntry fe = fe_n;
    const int lab = lab_n;
    if (e + nw < cnt) {
      fe_n = flags[e + nw];
      lab_n = (fe_n.row >= 0 && fe_n.row < n) ? label[fe_n.row] : 0;
    }
    const int row = fe.row;
    if (row < 0 || row >= n) continue;
    const float* x = X + (int64_t)row * ldx;
    int cj[3];
    cj[0] = min(max(lab, 0), k - 1);
    cj[1] = min(max(fe.cand2, 0), k - 1);
    cj[2] = fe.cand3 >= 0 ? min(fe.cand3, k - 1) : -1;
    const int nc = (cj[2] >= 0) ? 3 : 2;
    float p[3];
    plain_dist3<G>(x, C + (int64_t)cj[0] * d, C + (int64_t)cj[1] * d,
                   C + (int64_t)(nc == 3 ? cj[2] : cj[1]) * d, d, gl, vec, p[0], p[1], p[2]);
    int b = 0;
    for (int q = 1; q < nc; ++q)
      if (p[q] < p[b] || (p[q] == p[b] && cj[q] < cj[b])) b = q;
    bool sure = true;
    for (int q = 0; q < nc; ++q)
      if (q != b && !(p[q] - p[b] > tol * (p[q] + p[b]))) sure = false;
    int best = cj[b];
    float bd = p[b];
    if (!sure) {
      float bh = 0.f, bl = 0.f;
      for (int q = 0; q < nc; ++q) {
        float h, l;
        exact_dist<G>(x, C + (int64_t)cj[q] * d, d, gl, h, l);
        if (q == 0 || df_less(h, l, bh, bl) || (h == bh && l == bl && cj[q] < best)) {
          bh = h; bl = l; best = cj[q];
        }
      }
      bd = bh;
    }
    if (gl == 0) {
      label[row] = best;
      if (d1o) d1o[row] = bd;
      if (bo.ub) pair_bounds(bo, row, p, cj, nc, best, tol);
    }
  }
}

// Pipelined short re-check for short, 16-byte aligned rows (at most 4 G NX
// columns): while entry e is decided, the label and the row of entry e + 1
// and the list entry e + 2 are in flight (a lane holds its NX row chunks of
// the next entry in registers).  Same per-lane summation order as
// plain_dist3, so the same plain distances.  Short rows make the plain
// re-check latency-bound; long ones are bandwidth-bound and use
// recheck_pair_kernel.
template <int G, int NX>
__device__ __forceinline__ void load_row_chunks(const float* __restrict__ x, int d, int lane,
                                                float4 (&xv)[NX]) {
#pragma unroll
  for (int i = 0; i < NX; ++i) {
    const int q = lane * 4 + 4 * G * i;
    xv[i] = (q < d) ? *(const float4*)(x + q) : make_float4(0.f, 0.f, 0.f, 0.f);
  }
}

template <int G, int NX>
__device__ __forceinline__ void plain_dist3_rows(const float4 (&xv)[NX],
                                                 const float* __restrict__ c0,
                                                 const float* __restrict__ c1,
                                                 const float* __restrict__ c2, int d, int lane,
                                                 float& p0, float& p1, float& p2) {
  float a0 = 0.f, a1 = 0.f, a2 = 0.f;
#pragma unroll
  for (int i = 0; i < NX; ++i) {
    const int q = lane * 4 + 4 * G * i;
    if (q < d) {
      const float4 u0 = *(const float4*)(c0 + q);
      const float4 u1 = *(const float4*)(c1 + q);
      const float4 u2 = *(const float4*)(c2 + q);
      const float xs[4] = {xv[i].x, xv[i].y, xv[i].z, xv[i].w};
      const float v0[4] = {u0.x, u0.y, u0.z, u0.w};
      const float v1[4] = {u1.x, u1.y, u1.z, u1.w};
      const float v2[4] = {u2.x, u2.y, u2.z, u2.w};
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        float df = xs[e] - v0[e];
        a0 = __builtin_fmaf(df, df, a0);
        df = xs[e] - v1[e];
        a1 = __builtin_fmaf(df, df, a1);
        df = xs[e] - v2[e];
        a2 = __builtin_fmaf(df, df, a2);
      }
    }
  }
#pragma unroll
  for (int m = G / 2; m >= 1; m >>= 1) {
    a0 += __shfl_xor(a0, m, 64);
    a1 += __shfl_xor(a1, m, 64);
    a2 += __shfl_xor(a2, m, 64);
  }
  p0 = a0;
  p1 = a1;
  p2 = a2;
}

template <int G, int NX>
__global__ __launch_bounds__(256) void recheck_pair_pipe_kernel(
    const float* __restrict__ X, int64_t n, int d, int64_t ldx, const float* __restrict__ C,
    int k, int32_t* __restrict__ label, float* __restrict__ d1o,
    const FlagEntry* __restrict__ flags, const LoopState* __restrict__ st,
    const int* __restrict__ gate, BoundsOut bo) {
  if (gate && *gate) return;
  constexpr int SPW = 64 / G;          // entries per wave at once
  const int64_t cnt = (int64_t)st->flagged;
  const int lane = threadIdx.x & 63, gl = lane % G, grp = lane / G;
  const int64_t gw = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * SPW + grp;
  const int64_t nw = (int64_t)gridDim.x * 4 * SPW;
  const float tol = (float)((d + G - 1) / G + 13) * 5.9604645e-8f;
  const FlagEntry none = {-1, -1, -1, 0};
  auto valid = [&](const FlagEntry& f) { return f.row >= 0 && f.row < n; };
  // entries each row appears in at most once, so a label fetched ahead is
  // never one this kernel writes before reading it
  FlagEntry fe_c = (gw < cnt) ? flags[gw] : none;
  FlagEntry fe_n = (gw + nw < cnt) ? flags[gw + nw] : none;
  int lab_c = valid(fe_c) ? label[fe_c.row] : 0;
  float4 xc[NX];
  load_row_chunks<G, NX>(X + (int64_t)(valid(fe_c) ? fe_c.row : 0) * ldx, valid(fe_c) ? d : 0,
                         gl, xc);
  for (int64_t e = gw; e < cnt; e += nw) {   // uniform within a group
    // stage 1: list entry e + 2; stage 2: label and row of entry e + 1
    const FlagEntry fe_nn = (e + 2 * nw < cnt) ? flags[e + 2 * nw] : none;
    const bool vn = valid(fe_n);
    const int lab_n = vn ? label[fe_n.row] : 0;
    float4 xn[NX];
    load_row_chunks<G, NX>(X + (int64_t)(vn ? fe_n.row : 0) * ldx, vn ? d : 0, gl, xn);
    // stage 3: decide entry e
    if (valid(fe_c)) {
      const int row = fe_c.row;
      int cj[3];
      cj[0] = min(max(lab_c, 0), k - 1);
      cj[1] = min(max(fe_c.cand2, 0), k - 1);
      cj[2] = fe_c.cand3 >= 0 ? min(fe_c.cand3, k - 1) : -1;
      const int nc = (cj[2] >= 0) ? 3 : 2;
      float p[3];
      plain_dist3_rows<G, NX>(xc, C + (int64_t)cj[0] * d, C + (int64_t)cj[1] * d,
                              C + (int64_t)(nc == 3 ? cj[2] : cj[1]) * d, d, gl, p[0], p[1],
                              p[2]);
      int b = 0;
      for (int q = 1; q < nc; ++q)
        if (p[q] < p[b] || (p[q] == p[b] && cj[q] < cj[b])) b = q;
      bool sure = true;
      for (int q = 0; q < nc; ++q)
        if (q != b && !(p[q] - p[b] > tol * (p[q] + p[b]))) sure = false;
      int best = cj[b];
      float bd = p[b];
      if (!sure) {
        const float* x = X + (int64_t)row * ldx;
        float bh = 0.f, bl = 0.f;
        for (int q = 0; q < nc; ++q) {
          float h, l;
          exact_dist<G>(x, C + (int64_t)cj[q] * d, d, gl, h, l);
          if (q == 0 || df_less(h, l, bh, bl) || (h == bh && l == bl && cj[q] < best)) {
            bh = h; bl = l; best = cj[q];
          }
        }
        bd = bh;
      }
      if (gl == 0) {
        label[row] = best;
        if (d1o) d1o[row] = bd;
        if (bo.ub) pair_bounds(bo, row, p, cj, nc, best, tol);
      }
    }
    fe_c = fe_n;
    lab_c = lab_n;
#pragma unroll
    for (int i = 0; i < NX; ++i) xc[i] = xn[i];
    fe_n = fe_nn;
  }
}

constexpr int kFullWaves = 16;   // waves per row of the every-center re-check
constexpr bool kRecheckPipe = true;   // pipelined short re-check for rows of d <= 128

// One workgroup per row that needs every center.  Each wave takes four
// centers at a time (centers 4(kFullWaves i + w) + 0..3 for wave w), its lanes splitting
// the coordinates as in the short re-check, so every plain distance has
// relative error below gamma = (ceil(d/64) + 13) u.  Pass 1: the plain
// distances (kept in LDS) and their minimum m.  Pass 2: exact double-float
// distances for the centers at most m (1 + gamma) / (1 - gamma) (the only
// ones that can be the minimum); lexicographic argmin with the lowest index
// on ties.
constexpr int kFullPer = 4;   // centers per wave and step (8 measured slower)
__device__ __forceinline__ void plain_dist_k(const float* __restrict__ x,
                                            const float* __restrict__ C, int j0, int k, int d,
                                            int lane, bool vec, float* p) {
  const float* c[kFullPer];
#pragma unroll
  for (int t = 0; t < kFullPer; ++t) c[t] = C + (int64_t)min(j0 + t, k - 1) * d;
  float a[kFullPer];
#pragma unroll
  for (int t = 0; t < kFullPer; ++t) a[t] = 0.f;
  if (vec) {
    for (int q = lane * 4; q < d; q += 256) {
      const float4 xv = *(const float4*)(x + q);
      const float xs[4] = {xv.x, xv.y, xv.z, xv.w};
#pragma unroll
      for (int t = 0; t < kFullPer; ++t) {
        const float4 u = *(const float4*)(c[t] + q);
        const float v[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const float df = xs[e] - v[e];
          a[t] = __builtin_fmaf(df, df, a[t]);
        }
      }
    }
  } else {
    for (int q = lane; q < d; q += 64) {
      const float xq = x[q];
#pragma unroll
      for (int t = 0; t < kFullPer; ++t) {
        const float df = xq - c[t][q];
        a[t] = __builtin_fmaf(df, df, a[t]);
      }
    }
  }
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
#pragma unroll
    for (int t = 0; t < kFullPer; ++t) a[t] += __shfl_xor(a[t], m, 64);
  }
#pragma unroll
  for (int t = 0; t < kFullPer; ++t) p[t] = (j0 + t < k) ? a[t] : __builtin_inff();
}

__global__ __launch_bounds__(kFullWaves * 64) void recheck_full_kernel(
    const float* __restrict__ X, int64_t n, int d, int64_t ldx, const float* __restrict__ C,
    int k, int32_t* __restrict__ label, float* __restrict__ d1o, const int* __restrict__ brute,
    const LoopState* __restrict__ st, const int* __restrict__ gate, BoundsOut bo,
    float* __restrict__ d2o) {
  if (gate && *gate) return;
  extern __shared__ float pl[];   // k plain distances of the current row
  __shared__ float redf[kFullWaves], redf2[kFullWaves];
  __shared__ int redfj[kFullWaves];
  __shared__ float redh[kFullWaves], redl[kFullWaves];
  __shared__ int redj[kFullWaves];
  const int64_t cnt = (int64_t)st->flagged_full;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const float gam = (float)((d + 63) / 64 + 13) * 5.9604645e-8f;
  const bool vec = ((((uintptr_t)X) & 15) == 0) && (ldx % 4 == 0) &&
                   ((((uintptr_t)C) & 15) == 0) && (d % 4 == 0);
  for (int64_t e = blockIdx.x; e < cnt; e += gridDim.x) {
    const int row = brute[e];
    if (row < 0 || row >= n) continue;   // uniform across the block
    const float* x = X + (int64_t)row * ldx;
    // pass 1: the smallest plain distance m (center jm) and the second
    // smallest m2 (for the carried lower bound)
    float m = __builtin_inff(), m2 = __builtin_inff();
    int jm = 0x7FFFFFFF;
    for (int j0 = kFullPer * wv; j0 < k; j0 += kFullPer * kFullWaves) {
      float p[kFullPer];
      plain_dist_k(x, C, j0, k, d, lane, vec, p);
#pragma unroll
      for (int t = 0; t < kFullPer; ++t) {
        if (lane == t && j0 + t < k) pl[j0 + t] = p[t];
        if (p[t] < m) { m2 = m; m = p[t]; jm = j0 + t; }
        else m2 = fminf(m2, p[t]);
      }
    }
    if (lane == 0) { redf[wv] = m; redf2[wv] = m2; redfj[wv] = jm; }
    __syncthreads();
    m = redf[0];
    m2 = redf2[0];
    jm = redfj[0];
    for (int w = 1; w < kFullWaves; ++w) {
      if (redf[w] < m) { m2 = fminf(m, redf2[w]); m = redf[w]; jm = redfj[w]; }
      else m2 = fminf(m2, fminf(redf[w], redf2[w]));
    }
    const float thr = m * (1.0f + gam) / (1.0f - gam) * 1.0001f + 1e-30f;
    float bh = __builtin_inff(), bl = 0.f;
    int best = 0x7FFFFFFF;
    for (int j0 = kFullPer * wv; j0 < k; j0 += kFullPer * kFullWaves) {
      float p[kFullPer];
#pragma unroll
      for (int t = 0; t < kFullPer; ++t) p[t] = (j0 + t < k) ? pl[j0 + t] : __builtin_inff();
#pragma unroll
      for (int t = 0; t < kFullPer; ++t) {
        if (p[t] <= thr) {   // wave-uniform
          float h, l;
          exact_dist(x, C + (int64_t)(j0 + t) * d, d, lane, h, l);
          if (df_less(h, l, bh, bl) || (h == bh && l == bl && j0 + t < best)) {
            bh = h; bl = l; best = j0 + t;
          }
        }
      }
    }
    if (lane == 0) { redh[wv] = bh; redl[wv] = bl; redj[wv] = best; }
    __syncthreads();
    if (tid == 0) {
      for (int w = 1; w < kFullWaves; ++w) {
        if (df_less(redh[w], redl[w], bh, bl) || (redh[w] == bh && redl[w] == bl && redj[w] < best)) {
          bh = redh[w]; bl = redl[w]; best = redj[w];
        }
      }
      if (best < k) {
        label[row] = best;
        if (d1o) d1o[row] = bh;
        // second smallest plain distance (+inf for k = 1)
        if (d2o) d2o[row] = (jm == best) ? m2 : m;
        if (bo.ub) {
          // the winner's exact distance; every other center's plain
          // distance is at least m2, or m when the plain minimum is not the
          // winner (no runner-up kept)
          const double g2 = 2.0 * (double)gam;
          bo.ub[row] = dist_up((double)bh + (double)bl + fabs((double)bh) * 0x1p-40);
          bo.sec[row] = -1;
          bo.lb[row] = dist_down((double)(jm == best ? m2 : m) * (1.0 - g2));
        }
      }
    }
    __syncthreads();
  }
}

// A short list for the FP32 GEMM pass goes to the every-center re-check
// instead: that pass costs one workgroup's walk over all k centers however
// few rows it has, while the re-check runs hundreds of rows side by side.
// Moves the list onto the every-center list and empties it (the pass then
// finds no rows); longer lists are left to the pass.
__global__ __launch_bounds__(1024) void route_small_kernel(unsigned long long* __restrict__ ctr,
                                                           const int* __restrict__ list,
                                                           int* __restrict__ brute,
                                                           LoopState* __restrict__ st,
                                                           unsigned long long limit,
                                                           const int* __restrict__ gate) {
  if (gate && *gate) return;
  const unsigned long long cnt = *ctr;
  if (cnt == 0ull || cnt > limit) return;
  const unsigned long long base = st->flagged_full;
  for (unsigned long long i = threadIdx.x; i < cnt; i += blockDim.x) brute[base + i] = list[i];
  __syncthreads();
  if (threadIdx.x == 0) {
    st->flagged_full = base + cnt;
    *ctr = 0ull;
  }
}

__global__ void list_all_kernel(int* __restrict__ brute, int64_t n, const int* __restrict__ rows,
                                const unsigned long long* __restrict__ row_count,
                                LoopState* __restrict__ st, const int* __restrict__ gate) {
  if (gate && *gate) return;
  const int64_t m = rows ? (int64_t)(*row_count) : n;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride)
    brute[i] = rows ? rows[i] : (int)i;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->flagged_full = (unsigned long long)m;
    st->undecided = (unsigned long long)m;
  }
}

hipError_t launch_list_all(hipStream_t s, int* brute, int64_t n, const int* rows,
                           const unsigned long long* row_count, LoopState* st, const int* gate) {
  int64_t blocks = (n + 255) / 256;
  if (blocks > 2048) blocks = 2048;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(list_all_kernel, dim3((unsigned)blocks), dim3(256), 0, s, brute, n, rows,
                     row_count, st, gate);
  return hipGetLastError();
}

hipError_t launch_route_small(hipStream_t s, unsigned long long* ctr, const int* list, int* brute,
                              LoopState* st, int k, int d, const int* gate) {
  const unsigned long long lim =
      ((int64_t)k * d >= kShortListMinKD) ? (unsigned long long)kShortList : 0ull;
  hipLaunchKernelGGL(route_small_kernel, dim3(1), dim3(1024), 0, s, ctr, list, brute, st, lim,
                     gate);
  return hipGetLastError();
}

hipError_t launch_recheck(hipStream_t s, const float* X, int64_t n, int d, int64_t ldx,
                          const float* C, int k, int32_t* label, float* d1,
                          const FlagEntry* flags, const int* brute, const LoopState* st,
                          int num_cus, const int* gate, BoundsOut bo, float* d2) {
  int64_t blocks = (n + 3) / 4;
  int64_t cap = (int64_t)num_cus * 8;
  if (blocks > cap) blocks = cap;
  if (blocks < 1) blocks = 1;
  // lanes per entry: enough to cover a row in a few 16-byte steps, more
  // entries in flight per wave for short rows; short aligned rows pipelined
  const bool vec = ((((uintptr_t)X) & 15) == 0) && (ldx % 4 == 0) &&
                   ((((uintptr_t)C) & 15) == 0) && (d % 4 == 0);
  if (kRecheckPipe && vec && d <= 64)
    hipLaunchKernelGGL((recheck_pair_pipe_kernel<16, 1>), dim3((unsigned)blocks), dim3(256), 0, s,
                       X, n, d, ldx, C, k, label, d1, flags, st, gate, bo);
  else if (kRecheckPipe && vec && d <= 128)
    hipLaunchKernelGGL((recheck_pair_pipe_kernel<16, 2>), dim3((unsigned)blocks), dim3(256), 0, s,
                       X, n, d, ldx, C, k, label, d1, flags, st, gate, bo);
  else if (d <= 256)
    hipLaunchKernelGGL(recheck_pair_kernel<16>, dim3((unsigned)blocks), dim3(256), 0, s, X, n,
                       d, ldx, C, k, label, d1, flags, st, gate, bo);
  else if (d <= 1024)
    hipLaunchKernelGGL(recheck_pair_kernel<32>, dim3((unsigned)blocks), dim3(256), 0, s, X, n,
                       d, ldx, C, k, label, d1, flags, st, gate, bo);
  else
    hipLaunchKernelGGL(recheck_pair_kernel<64>, dim3((unsigned)blocks), dim3(256), 0, s, X, n,
                       d, ldx, C, k, label, d1, flags, st, gate, bo);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  cap = (int64_t)num_cus * 4;
  blocks = n;
  if (blocks > cap) blocks = cap;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(recheck_full_kernel, dim3((unsigned)blocks), dim3(kFullWaves * 64),
                     (size_t)k * sizeof(float), s, X, n, d, ldx, C, k, label, d1, brute, st, gate,
                     bo, d2);
  return hipGetLastError();
}


// Re-check of a batched assignment: list rows are global; the bucket (pair
// entries) or the instance (every-center entries) is found by binary search.
__device__ __forceinline__ int find_bucket(const BatchBucket* __restrict__ b, int nb, int64_t g) {
  int lo = 0, hi = nb - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (b[mid].grow0 <= g) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ int find_inst(const BatchInst* __restrict__ in, int ni, int64_t g) {
  int lo = 0, hi = ni - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (in[mid].grow0 <= g) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Batched short re-check: G lanes per entry (64 / G entries per wave), the
// next list entry fetched one ahead; the bucket of a row is found by binary
// search over the buckets' first rows, staged in LDS when there are at most
// kBucketLds buckets.
constexpr int kBucketLds = 256;

template <int G>
__global__ __launch_bounds__(256) void recheck_pair_batched_kernel(
    const BatchBucket* __restrict__ buckets, int nb, int32_t* __restrict__ label,
    const FlagEntry* __restrict__ flags, const LoopState* __restrict__ st, int64_t nrows) {
  __shared__ int64_t sg0[kBucketLds];
  const bool staged = nb <= kBucketLds;
  if (staged)
    for (int i = threadIdx.x; i < nb; i += blockDim.x) sg0[i] = buckets[i].grow0;
  __syncthreads();
  constexpr int SPW = 64 / G;
  const int64_t cnt = (int64_t)st->flagged;
  const int lane = threadIdx.x & 63, gl = lane % G, grp = lane / G;
  const int64_t gw = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * SPW + grp;
  const int64_t nw = (int64_t)gridDim.x * 4 * SPW;
  const FlagEntry none = {-1, -1, -1, 0};
  FlagEntry fe_n = (gw < cnt) ? flags[gw] : none;
  for (int64_t e = gw; e < cnt; e += nw) {   // uniform within a group
    const FlagEntry fe = fe_n;
    if (e + nw < cnt) fe_n = flags[e + nw];
    const int64_t row = fe.row;
    if (row < 0 || row >= nrows) continue;
    int bi;
    if (staged) {
      int lo = 0, hi = nb - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (sg0[mid] <= row) lo = mid;
        else hi = mid - 1;
      }
      bi = lo;
    } else {
      bi = find_bucket(buckets, nb, row);
    }
    const BatchBucket B = buckets[bi];
    const int d = B.d;
    const float tol = (float)((d + G - 1) / G + 13) * 5.9604645e-8f;
    const float* x = B.X + (row - B.grow0) * d;
    const bool vec = ((((uintptr_t)B.X) & 15) == 0) && ((((uintptr_t)B.C) & 15) == 0) &&
                     (d % 4 == 0);
    int cj[3];
    cj[0] = min(max(label[row], 0), B.K - 1);
    cj[1] = min(max(fe.cand2, 0), B.K - 1);
    cj[2] = fe.cand3 >= 0 ? min(fe.cand3, B.K - 1) : -1;
    const int nc = (cj[2] >= 0) ? 3 : 2;
    float p[3];
    plain_dist3<G>(x, B.C + (int64_t)cj[0] * d, B.C + (int64_t)cj[1] * d,
                   B.C + (int64_t)(nc == 3 ? cj[2] : cj[1]) * d, d, gl, vec, p[0], p[1], p[2]);
    int b = 0;
    for (int q = 1; q < nc; ++q)
      if (p[q] < p[b] || (p[q] == p[b] && cj[q] < cj[b])) b = q;
    bool sure = true;
    for (int q = 0; q < nc; ++q)
      if (q != b && !(p[q] - p[b] > tol * (p[q] + p[b]))) sure = false;
    int best = cj[b];
    if (!sure) {
      float bh = 0.f, bl = 0.f;
      for (int q = 0; q < nc; ++q) {
        float h, l;
        exact_dist<G>(x, B.C + (int64_t)cj[q] * d, d, gl, h, l);
        if (q == 0 || df_less(h, l, bh, bl) || (h == bh && l == bl && cj[q] < best)) {
          bh = h;
          bl = l;
          best = cj[q];
        }
      }
    }
    if (gl == 0) label[row] = best;
  }
}

// One workgroup per row needing every center of its instance.
__global__ __launch_bounds__(kFullWaves * 64) void recheck_full_batched_kernel(
    const BatchInst* __restrict__ insts, int ni, int32_t* __restrict__ label,
    const int* __restrict__ brute, const LoopState* __restrict__ st, int64_t nrows) {
  __shared__ float redf[kFullWaves];
  __shared__ float redh[kFullWaves], redl[kFullWaves];
  __shared__ int redj[kFullWaves];
  const unsigned long long cnt = st->flagged_full;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int64_t e = blockIdx.x; e < (int64_t)cnt; e += gridDim.x) {
    const int64_t row = brute[e];
    if (row < 0 || row >= nrows) continue;   // uniform across the block
    const BatchInst& I = insts[find_inst(insts, ni, row)];
    const int d = I.d;
    const float gam = (float)((d + 63) / 64 + 13) * 5.9604645e-8f;
    const float* x = I.X + (I.row0 + (row - I.grow0)) * d;
    const float* C = I.C + (int64_t)I.koff * d;
    const bool vec = ((((uintptr_t)x) & 15) == 0) && ((((uintptr_t)C) & 15) == 0) && (d % 4 == 0);
    float m = __builtin_inff();
    for (int j0 = kFullPer * wv; j0 < I.k; j0 += kFullPer * kFullWaves) {
      float p[kFullPer];
      plain_dist_k(x, C, j0, I.k, d, lane, vec, p);
#pragma unroll
      for (int t = 0; t < kFullPer; ++t) m = fminf(m, p[t]);
    }
    if (lane == 0) redf[wv] = m;
    __syncthreads();
    m = redf[0];
    for (int w = 1; w < kFullWaves; ++w) m = fminf(m, redf[w]);
    const float thr = m * (1.0f + gam) / (1.0f - gam) * 1.0001f + 1e-30f;
    float bh = __builtin_inff(), bl = 0.f;
    int best = 0x7FFFFFFF;
    for (int j0 = kFullPer * wv; j0 < I.k; j0 += kFullPer * kFullWaves) {
      float p[kFullPer];
      plain_dist_k(x, C, j0, I.k, d, lane, vec, p);
#pragma unroll
      for (int t = 0; t < kFullPer; ++t) {
        if (p[t] <= thr) {   // wave-uniform
          float h, l;
          exact_dist(x, C + (int64_t)(j0 + t) * d, d, lane, h, l);
          if (df_less(h, l, bh, bl) || (h == bh && l == bl && j0 + t < best)) {
            bh = h;
            bl = l;
            best = j0 + t;
          }
        }
      }
    }
    if (lane == 0) {
      redh[wv] = bh;
      redl[wv] = bl;
      redj[wv] = best;
    }
    __syncthreads();
    if (tid == 0) {
      for (int w = 1; w < kFullWaves; ++w) {
        if (df_less(redh[w], redl[w], bh, bl) ||
            (redh[w] == bh && redl[w] == bl && redj[w] < best)) {
          bh = redh[w];
          bl = redl[w];
          best = redj[w];
        }
      }
      if (best < I.k) label[row] = I.koff + best;
    }
    __syncthreads();
  }
}

hipError_t launch_recheck_batched(hipStream_t s, const BatchBucket* buckets, int nbuckets,
                                  const BatchInst* insts, int ninst, int32_t* label,
                                  const FlagEntry* flags, const int* brute, const LoopState* st,
                                  int64_t nrows, int num_cus) {
  // 16 lanes per entry: bucket widths are at most 512 (8 steps of 16 bytes)
  hipLaunchKernelGGL(recheck_pair_batched_kernel<16>, dim3((unsigned)(num_cus * 8)), dim3(256), 0,
                     s, buckets, nbuckets, label, flags, st, nrows);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(recheck_full_batched_kernel, dim3((unsigned)(num_cus * 4)), dim3(kFullWaves * 64), 0, s,
                     insts, ninst, label, brute, st, nrows);
  return hipGetLastError();
}

}  // namespace kmx
