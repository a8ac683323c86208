// Bounds carried across Lloyd iterations (Hamerly's form of Elkan's
// triangle-inequality filtering): every row keeps an upper bound u of the
// distance to its assigned center c_a and a lower bound l of the distance to
// every other center.  When the centers move by delta_j = ||c_j' - c_j||, the
// triangle inequality gives ||x - c_a'|| <= u + delta_a and ||x - c_j'|| >=
// l - max_{j != a} delta_j, so a row whose new u stays strictly below its new
// l keeps its label without reading the row: no other center can be as close
// (Sec. 1, the assignment step, is unchanged; only the work is skipped).
// Rows that fail go on to the certificate and the GEMM, which set fresh
// bounds.  All bounds are rounded outward.
#include "kmx_device.h"
#include "kmx_internal.h"

namespace kmx {

// Drift of every center: delta_j = ||c_new_j - c_old_j|| rounded up (FP64
// sums of FP32 differences), one wave per center.
__global__ __launch_bounds__(1024) void drift_kernel(const float* __restrict__ Cold,
                                                     const float* __restrict__ Cnew, int k, int d,
                                                     float* __restrict__ drift,
                                                     const int* __restrict__ gate) {
  if (gate && *gate) return;
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * 16 + (threadIdx.x >> 6);
  if (j >= k) return;   // whole waves
  const float* a = Cold + (int64_t)j * d;
  const float* b = Cnew + (int64_t)j * d;
  double s = 0.0;
  for (int e = lane; e < d; e += 64) {
    const double df = (double)b[e] - (double)a[e];
    s += df * df;
  }
  s = wave_sum_f64(s);
  if (lane == 0) drift[j] = dist_up(s);
}

// The three largest drifts and the centers of the largest two (one workgroup):
// every thread keeps its own top three, then butterfly merges within the wave
// and across the waves.
struct Top3 {
  float v1, v2, v3;
  int i1, i2;
};

__device__ __forceinline__ void top3_add(Top3& t, float v, int j) {
  if (v > t.v1) { t.v3 = t.v2; t.v2 = t.v1; t.i2 = t.i1; t.v1 = v; t.i1 = j; }
  else if (v > t.v2) { t.v3 = t.v2; t.v2 = v; t.i2 = j; }
  else if (v > t.v3) { t.v3 = v; }
}

__device__ __forceinline__ void top3_merge(Top3& t, const Top3& o) {
  top3_add(t, o.v1, o.i1);
  top3_add(t, o.v2, o.i2);
  top3_add(t, o.v3, -1);
}

__global__ __launch_bounds__(1024) void drift_max_kernel(const float* __restrict__ drift, int k,
                                                         DriftStat* __restrict__ ds,
                                                         const int* __restrict__ gate) {
  if (gate && *gate) return;
  __shared__ Top3 red[16];
  Top3 t = {-1.0f, -1.0f, -1.0f, -1, -1};
  for (int j = threadIdx.x; j < k; j += 1024) top3_add(t, drift[j], j);
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    Top3 o;
    o.v1 = __shfl_xor(t.v1, m, 64);
    o.v2 = __shfl_xor(t.v2, m, 64);
    o.v3 = __shfl_xor(t.v3, m, 64);
    o.i1 = __shfl_xor(t.i1, m, 64);
    o.i2 = __shfl_xor(t.i2, m, 64);
    top3_merge(t, o);
  }
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 16; ++w) top3_merge(t, red[w]);
    ds->max1 = fmaxf(t.v1, 0.0f);
    ds->max2 = fmaxf(t.v2, 0.0f);
    ds->max3 = fmaxf(t.v3, 0.0f);
    ds->arg1 = t.i1;
    ds->arg2 = t.i2;
  }
}

// The bound test over all rows, for label a and runner-up b (sec, or -1):
// u += delta_a, l2 -= delta_b, lb -= the largest drift of a center other than
// a and b.  Rows with u < min(l2, lb) keep their label; rows with l2 <= u <
// lb can only go to b, and go to the short re-check as the pair (a, b); the
// others are listed in fail_rows (st->bound_fail).  A workgroup takes
// kBoundRows consecutive rows (kBoundPer per thread), counts with ballots and
// reserves its slices of both lists with one atomic each (same-address
// atomics from every wave would serialize).
constexpr int kBoundPer = 16;
constexpr int kBoundRows = 256 * kBoundPer;

__global__ __launch_bounds__(256) void bounds_test_kernel(int64_t n, const int32_t* __restrict__ label,
                                                          BoundsOut bo,
                                                          const float* __restrict__ drift,
                                                          const DriftStat* __restrict__ ds, int k,
                                                          int* __restrict__ fail_rows,
                                                          FlagEntry* __restrict__ flags,
                                                          LoopState* __restrict__ st,
                                                          const int* __restrict__ gate) {
  if (gate && *gate) return;
  __shared__ int wcnt[2][4];
  __shared__ unsigned long long wbase[2];
  const float m1 = ds->max1, m2 = ds->max2, m3 = ds->max3;
  const int j1 = ds->arg1, j2 = ds->arg2;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const unsigned long long below = (1ull << lane) - 1ull;
  const int64_t nchunks = (n + kBoundRows - 1) / kBoundRows;
  for (int64_t chk = blockIdx.x; chk < nchunks; chk += gridDim.x) {
    // row of slot q: chk * kBoundRows + q * 256 + threadIdx.x (coalesced)
    const int64_t r0 = chk * kBoundRows + threadIdx.x;
    unsigned fails = 0u, pairs = 0u;
    int secs[kBoundPer];
#pragma unroll 4
    for (int q = 0; q < kBoundPer; ++q) {
      const int64_t i = r0 + (int64_t)q * 256;
      secs[q] = -1;
      if (i < n) {
        const int a = label[i];
        int b = bo.sec[i];
        if (b < 0 || b >= k || b == a) b = -1;
        const bool ok = a >= 0 && a < k;
        const float da = ok ? drift[a] : __builtin_inff();
        const float dr = (j1 != a && j1 != b) ? m1 : ((j2 != a && j2 != b) ? m2 : m3);
        const float u = f64_to_f32_up((double)bo.ub[i] + (double)da);
        const float l = f64_to_f32_down((double)bo.lb[i] - (double)dr);
        const float l2 = b >= 0 ? f64_to_f32_down((double)bo.l2[i] - (double)drift[b])
                                : __builtin_inff();
        bo.ub[i] = u;
        bo.lb[i] = l;
        if (b >= 0) bo.l2[i] = l2;
        if (!(u < l)) fails |= 1u << q;
        else if (!(u < l2)) { pairs |= 1u << q; secs[q] = b; }
      }
    }
    int cf = 0, cp = 0;
#pragma unroll
    for (int q = 0; q < kBoundPer; ++q) {
      cf += __popcll(__ballot((fails >> q) & 1u));
      cp += __popcll(__ballot((pairs >> q) & 1u));
    }
    if (lane == 0) { wcnt[0][wave] = cf; wcnt[1][wave] = cp; }
    __syncthreads();
    if (threadIdx.x == 0) {
      const int tf = wcnt[0][0] + wcnt[0][1] + wcnt[0][2] + wcnt[0][3];
      const int tp = wcnt[1][0] + wcnt[1][1] + wcnt[1][2] + wcnt[1][3];
      wbase[0] = tf ? atomicAdd(&st->bound_fail, (unsigned long long)tf) : 0ull;
      wbase[1] = tp ? atomicAdd(&st->flagged, (unsigned long long)tp) : 0ull;
      if (tp) atomicAdd(&st->bound_pair, (unsigned long long)tp);
    }
    __syncthreads();
    unsigned long long of = wbase[0], op = wbase[1];
    for (int w = 0; w < wave; ++w) { of += wcnt[0][w]; op += wcnt[1][w]; }
#pragma unroll
    for (int q = 0; q < kBoundPer; ++q) {
      const int64_t i = r0 + (int64_t)q * 256;
      const unsigned long long bf = __ballot((fails >> q) & 1u);
      const unsigned long long bp = __ballot((pairs >> q) & 1u);
      if ((fails >> q) & 1u) fail_rows[of + __popcll(bf & below)] = (int)i;
      if ((pairs >> q) & 1u) {
        FlagEntry fe;
        fe.row = (int)i;
        fe.cand2 = secs[q];
        fe.cand3 = -1;
        fe.pad = 0;
        flags[op + __popcll(bp & below)] = fe;
      }
      of += __popcll(bf);
      op += __popcll(bp);
    }
    __syncthreads();
  }
}

// dst = src (count floats) unless the loop has stopped: the centers the
// drift is measured from.
__global__ void copy_f32_kernel(const float* __restrict__ src, float* __restrict__ dst,
                                int64_t count, const int* __restrict__ gate) {
  if (gate && *gate) return;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
    dst[i] = src[i];
}

// kept[slot] = rows the bound test kept (n - listed - paired), or 0 without st.
__global__ void record_kept_kernel(const LoopState* __restrict__ st, int64_t* __restrict__ kept,
                                   int slot, int64_t n, const int* __restrict__ gate) {
  if (gate && *gate) return;
  if (threadIdx.x == 0)
    kept[slot] = st ? n - (int64_t)st->bound_fail - (int64_t)st->bound_pair : 0;
}

hipError_t launch_copy_f32(hipStream_t s, const float* src, float* dst, int64_t count,
                           const int* gate) {
  int64_t blocks = (count + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(copy_f32_kernel, dim3((unsigned)blocks), dim3(256), 0, s, src, dst, count,
                     gate);
  return hipGetLastError();
}

hipError_t launch_record_kept(hipStream_t s, const LoopState* st, int64_t* kept, int slot,
                              int64_t n, const int* gate) {
  hipLaunchKernelGGL(record_kept_kernel, dim3(1), dim3(64), 0, s, st, kept, slot, n, gate);
  return hipGetLastError();
}

hipError_t launch_drift(hipStream_t s, const float* Cold, const float* Cnew, int k, int d,
                        float* drift, DriftStat* ds, const int* gate) {
  hipLaunchKernelGGL(drift_kernel, dim3((unsigned)((k + 15) / 16)), dim3(1024), 0, s, Cold, Cnew, k,
                     d, drift, gate);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(drift_max_kernel, dim3(1), dim3(1024), 0, s, drift, k, ds, gate);
  return hipGetLastError();
}

hipError_t launch_bounds_test(hipStream_t s, int64_t n, const int32_t* label, BoundsOut bo,
                              const float* drift, const DriftStat* ds, int k, int* fail_rows,
                              FlagEntry* flags, LoopState* st, const int* gate, int num_cus) {
  int64_t blocks = (n + kBoundRows - 1) / kBoundRows;
  const int64_t cap = (int64_t)num_cus * 8;
  if (blocks > cap) blocks = cap;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(bounds_test_kernel, dim3((unsigned)blocks), dim3(256), 0, s, n, label, bo,
                     drift, ds, k, fail_rows, flags, st, gate);
  return hipGetLastError();
}

}  // namespace kmx
