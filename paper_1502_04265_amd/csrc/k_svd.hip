// Device kernels of the randomized range finder (the best-fit subspace of
// Sec. 2.2, "Computation of the SVD": a random test matrix reduces the columns
// before a small SVD, after Halko, Martinsson and Tropp 2011; weighted points
// enter as rows scaled by sqrt(w), Sec. 2.3.2).
//
//   gauss_fill:  the Gaussian test matrix, a counter-based stream
//                (SplitMix64 outputs of the element's counter, Box-Muller);
//   scale_rows:  Y_i *= s_i (the sqrt(w) row scaling);
//   atb:         G = A^T diag(s) B for tall A (n x p) and B (n x q <= 128),
//                FP64 sums of FP32 products (exact), one partial per row
//                slice, then a fixed-order sum of the slices.
#include "kmx_device.h"
#include "kmx_internal.h"

namespace kmx {

__device__ __forceinline__ uint64_t splitmix_at(uint64_t seed, uint64_t r) {
  // the r-th output (r >= 0) of SplitMix64 started at state seed
  uint64_t z = seed + (r + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ void gauss_fill_kernel(float* __restrict__ out, int64_t count, uint64_t seed) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
    const double u1 = ((double)(splitmix_at(seed, 2 * (uint64_t)i) >> 11) + 0.5) * 0x1p-53;
    const double u2 = (double)(splitmix_at(seed, 2 * (uint64_t)i + 1) >> 11) * 0x1p-53;
    out[i] = (float)(sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2));
  }
}

__global__ void scale_rows_kernel(float* __restrict__ Y, int64_t n, int q, int64_t ldy,
                                  const float* __restrict__ w) {
  const int64_t total = n * (int64_t)q;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
    const int64_t r = i / q;
    Y[r * ldy + (i - r * q)] *= sqrtf(w[r]);
  }
}

// One workgroup: 64 columns of A (tile), rows [r0, r1) of one slice.  Thread
// t owns column t % 64 and outputs j = t / 64 + 4 m (m < q / 4 rounded up).
// Rows are staged in LDS RB at a time: A's tile columns and all q columns of B
// (with the row scale applied to B).
constexpr int kAtbRB = 32;
constexpr int kAtbMaxQ = 128;

__global__ __launch_bounds__(256) void atb_kernel(const float* __restrict__ A, int64_t n, int p,
                                                  int64_t lda, const float* __restrict__ B, int q,
                                                  int64_t ldb, const float* __restrict__ w,
                                                  int64_t rows_per_slice,
                                                  double* __restrict__ part) {
  __shared__ float sa[kAtbRB][64];
  __shared__ float sb[kAtbRB][kAtbMaxQ];
  const int t = threadIdx.x;
  const int c = t & 63, g = t >> 6;
  const int col0 = blockIdx.x * 64;
  const int64_t r0 = (int64_t)blockIdx.y * rows_per_slice;
  const int64_t r1 = min(n, r0 + rows_per_slice);
  constexpr int MQ = kAtbMaxQ / 4;
  double acc[MQ];
#pragma unroll
  for (int m = 0; m < MQ; ++m) acc[m] = 0.0;
  for (int64_t rb = r0; rb < r1; rb += kAtbRB) {
    const int nr = (int)min((int64_t)kAtbRB, r1 - rb);
    for (int e = t; e < kAtbRB * 64; e += 256) {
      const int rr = e >> 6, cc = e & 63;
      sa[rr][cc] = (rr < nr && col0 + cc < p) ? A[(rb + rr) * lda + col0 + cc] : 0.0f;
    }
    for (int e = t; e < kAtbRB * kAtbMaxQ; e += 256) {
      const int rr = e / kAtbMaxQ, jj = e % kAtbMaxQ;
      float v = 0.0f;
      if (rr < nr && jj < q) {
        v = B[(rb + rr) * ldb + jj];
        if (w) v *= sqrtf(w[rb + rr]);
      }
      sb[rr][jj] = v;
    }
    __syncthreads();
    for (int rr = 0; rr < nr; ++rr) {
      const double a = (double)sa[rr][c];
#pragma unroll
      for (int m = 0; m < MQ; ++m) acc[m] += a * (double)sb[rr][g + 4 * m];
    }
    __syncthreads();
  }
  double* out = part + (int64_t)blockIdx.y * p * q;
  if (col0 + c < p) {
#pragma unroll
    for (int m = 0; m < MQ; ++m) {
      const int j = g + 4 * m;
      if (j < q) out[(int64_t)(col0 + c) * q + j] = acc[m];
    }
  }
}

__global__ void atb_sum_kernel(const double* __restrict__ part, int slices, int64_t count,
                               double* __restrict__ out) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
    double s = 0.0;
    for (int sl = 0; sl < slices; ++sl) s += part[(int64_t)sl * count + i];
    out[i] = s;
  }
}

__global__ void f64_to_f32_kernel(const double* __restrict__ in, float* __restrict__ out,
                                  int64_t count) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
    out[i] = (float)in[i];
}

hipError_t launch_gauss_fill(hipStream_t s, float* out, int64_t count, uint64_t seed) {
  int64_t blocks = (count + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(gauss_fill_kernel, dim3((unsigned)blocks), dim3(256), 0, s, out, count, seed);
  return hipGetLastError();
}

hipError_t launch_scale_rows(hipStream_t s, float* Y, int64_t n, int q, int64_t ldy,
                             const float* w) {
  int64_t blocks = (n * q + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(scale_rows_kernel, dim3((unsigned)blocks), dim3(256), 0, s, Y, n, q, ldy, w);
  return hipGetLastError();
}

int atb_slices(int64_t n, int p, int num_cus) {
  const int tiles = (p + 63) / 64;
  int64_t slices = ((int64_t)num_cus * 2 + tiles - 1) / tiles;
  const int64_t maxs = (n + 255) / 256;   // at least 256 rows a slice
  if (slices > maxs) slices = maxs;
  if (slices < 1) slices = 1;
  return (int)slices;
}

hipError_t launch_atb(hipStream_t s, const float* A, int64_t n, int p, int64_t lda, const float* B,
                      int q, int64_t ldb, const float* w, double* part, int slices, double* out) {
  if (q < 1 || q > kAtbMaxQ) return hipErrorInvalidValue;
  const int64_t rps = (n + slices - 1) / slices;
  hipLaunchKernelGGL(atb_kernel, dim3((unsigned)((p + 63) / 64), (unsigned)slices), dim3(256), 0, s,
                     A, n, p, lda, B, q, ldb, w, rps, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t count = (int64_t)p * q;
  int64_t blocks = (count + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(atb_sum_kernel, dim3((unsigned)blocks), dim3(256), 0, s, part, slices, count,
                     out);
  return hipGetLastError();
}

hipError_t launch_f64_to_f32(hipStream_t s, const double* in, float* out, int64_t count) {
  int64_t blocks = (count + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(f64_to_f32_kernel, dim3((unsigned)blocks), dim3(256), 0, s, in, out, count);
  return hipGetLastError();
}

}  // namespace kmx
