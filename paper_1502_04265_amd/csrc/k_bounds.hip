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
// sums of FP32 differences), and the largest two drifts with the index of the
// largest.  One workgroup.
__global__ __launch_bounds__(1024) void drift_kernel(const float* __restrict__ Cold,
                                                     const float* __restrict__ Cnew, int k, int d,
                                                     float* __restrict__ drift,
                                                     DriftStat* __restrict__ ds,
                                                     const int* __restrict__ gate) {
  if (gate && *gate) return;
  __shared__ float m1s[16], m2s[16];
  __shared__ int j1s[16];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  float m1 = 0.0f, m2 = 0.0f;
  int j1 = -1;
  for (int j = wave; j < k; j += 16) {
    const float* a = Cold + (int64_t)j * d;
    const float* b = Cnew + (int64_t)j * d;
    double s = 0.0;
    for (int e = lane; e < d; e += 64) {
      const double df = (double)b[e] - (double)a[e];
      s += df * df;
    }
    s = wave_sum_f64(s);
    const float dj = dist_up(s);
    if (lane == 0) drift[j] = dj;
    if (dj > m1) { m2 = m1; m1 = dj; j1 = j; }
    else m2 = fmaxf(m2, dj);
  }
  if (lane == 0) { m1s[wave] = m1; m2s[wave] = m2; j1s[wave] = j1; }
  __syncthreads();
  if (threadIdx.x == 0) {
    float a1 = m1s[0], a2 = m2s[0];
    int aj = j1s[0];
    for (int w = 1; w < 16; ++w) {
      if (m1s[w] > a1) { a2 = fmaxf(a1, m2s[w]); a1 = m1s[w]; aj = j1s[w]; }
      else a2 = fmaxf(a2, fmaxf(m1s[w], m2s[w]));
    }
    ds->max1 = a1;
    ds->max2 = a2;
    ds->arg1 = aj;
  }
}

// The bound test over all rows: u += delta_a, l -= (largest drift of a center
// other than a); rows with u < l keep their label, the others are listed in
// fail_rows (counter st->bound_fail; one atomic per wave).
__global__ __launch_bounds__(256) void bounds_test_kernel(int64_t n, const int32_t* __restrict__ label,
                                                          float* __restrict__ hub,
                                                          float* __restrict__ hlb,
                                                          const float* __restrict__ drift,
                                                          const DriftStat* __restrict__ ds, int k,
                                                          int* __restrict__ fail_rows,
                                                          LoopState* __restrict__ st,
                                                          const int* __restrict__ gate) {
  if (gate && *gate) return;
  const float m1 = ds->max1, m2 = ds->max2;
  const int j1 = ds->arg1;
  const int lane = threadIdx.x & 63;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const unsigned long long below = (1ull << lane) - 1ull;
  for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x; i0 < n; i0 += stride) {
    const int64_t i = i0 + threadIdx.x;
    bool fail = false;
    if (i < n) {
      const int a = label[i];
      const bool ok = a >= 0 && a < k;
      const float da = ok ? drift[a] : __builtin_inff();
      const float u = f64_to_f32_up((double)hub[i] + (double)da);
      const float l = f64_to_f32_down((double)hlb[i] - (double)(a == j1 ? m2 : m1));
      hub[i] = u;
      hlb[i] = l;
      fail = !(u < l);
    }
    const unsigned long long bal = __ballot(fail);
    unsigned long long base = 0;
    if (lane == 0 && bal) base = atomicAdd(&st->bound_fail, (unsigned long long)__popcll(bal));
    base = (unsigned long long)__shfl((long long)base, 0, 64);
    if (fail) fail_rows[base + __popcll(bal & below)] = (int)i;
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

// kept[slot] = rows the bound test kept (n - st->bound_fail), or 0 without st.
__global__ void record_kept_kernel(const LoopState* __restrict__ st, int64_t* __restrict__ kept,
                                   int slot, int64_t n, const int* __restrict__ gate) {
  if (gate && *gate) return;
  if (threadIdx.x == 0) kept[slot] = st ? n - (int64_t)st->bound_fail : 0;
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
  hipLaunchKernelGGL(drift_kernel, dim3(1), dim3(1024), 0, s, Cold, Cnew, k, d, drift, ds, gate);
  return hipGetLastError();
}

hipError_t launch_bounds_test(hipStream_t s, int64_t n, const int32_t* label, float* hub,
                              float* hlb, const float* drift, const DriftStat* ds, int k,
                              int* fail_rows, LoopState* st, const int* gate, int num_cus) {
  int64_t blocks = (n + 255) / 256;
  const int64_t cap = (int64_t)num_cus * 16;
  if (blocks > cap) blocks = cap;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(bounds_test_kernel, dim3((unsigned)blocks), dim3(256), 0, s, n, label, hub,
                     hlb, drift, ds, k, fail_rows, st, gate);
  return hipGetLastError();
}

}  // namespace kmx
