// Projection of a chunk of rows onto a low-dimensional subspace (the
// dimension reduction of the streamed pipeline, Sec. 3: each row is replaced
// by its coordinates in the span of the top right singular vectors V, so
// that squared distances inside that span are preserved).
//
//   Y[r][j] = sum_i X[r][i] V[i][j],   X: rows x d_in, V: d_in x d_out (FP32)
//
// FP32 MFMA 16x16x4 with FP32 accumulation.  A = V^T (16 output columns x 4
// k, from LDS), B = X (4 k x 16 rows, registers, streamed from HBM once).
// Lane l holds output column 16j + 4(l/16) + i of row l%16 (a float4 store).
// Each lane reads 16 contiguous bytes of its row per 16-wide k step; A and B
// use the same lane-to-k mapping (k = 16s + 4(l/16) + e), so the order of
// the contraction inside a step does not change what is computed.
// Workgroup: 4 waves x 16 rows; V in chunks of 64 k, double-buffered.
#include "kmx_internal.h"

namespace kmx {

typedef __attribute__((ext_vector_type(4))) float pf32x4_t;

template <int NT, bool VEC>
__global__ __launch_bounds__(256) void project_kernel(const float* __restrict__ X, int64_t rows,
                                                      int d_in, int64_t ldx,
                                                      const float* __restrict__ V, int d_out,
                                                      float* __restrict__ Y, int64_t ldy) {
  constexpr int KC = 64;                 // k per LDS chunk
  constexpr int DO = NT * 16;            // output columns
  constexpr int PIT = DO + 4;            // LDS pitch (floats)
  __shared__ __attribute__((aligned(16))) float vs[2][KC * PIT];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int c = lane & 15, g = lane >> 4;
  const int64_t nblk = (rows + 63) / 64;
  const int nchunks = (d_in + KC - 1) / KC;

  auto load_v = [&](int ch, int buf) {
    const int k0 = ch * KC;
    for (int e = tid; e < KC * DO; e += 256) {
      const int kk = e / DO, j = e - kk * DO;
      const int k = k0 + kk;
      vs[buf][kk * PIT + j] = (k < d_in && j < d_out) ? V[(int64_t)k * d_out + j] : 0.0f;
    }
  };
  auto load_x = [&](const float* xr, bool valid, int ch, pf32x4_t* xv) {
#pragma unroll
    for (int s = 0; s < KC / 16; ++s) {
      const int k = ch * KC + 16 * s + 4 * g;
      pf32x4_t v = {0.f, 0.f, 0.f, 0.f};
      if (valid) {
        if (VEC && k + 4 <= d_in) {
          v = *(const pf32x4_t*)(xr + k);
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (k + e < d_in) v[e] = xr[k + e];
        }
      }
      xv[s] = v;
    }
  };

  for (int64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
    const int64_t row = blk * 64 + wave * 16 + c;
    const bool valid = row < rows;
    const float* xr = X + (valid ? row : 0) * ldx;
    pf32x4_t acc[NT];
#pragma unroll
    for (int j = 0; j < NT; ++j) acc[j] = (pf32x4_t){0.f, 0.f, 0.f, 0.f};
    pf32x4_t xv[KC / 16], xn[KC / 16];
    __syncthreads();                     // previous block done with vs
    load_v(0, 0);
    load_x(xr, valid, 0, xv);
    __syncthreads();
    for (int ch = 0; ch < nchunks; ++ch) {
      const int buf = ch & 1;
      if (ch + 1 < nchunks) {
        load_v(ch + 1, buf ^ 1);
        load_x(xr, valid, ch + 1, xn);
      }
      const float* vb = &vs[buf][0];
#pragma unroll
      for (int s = 0; s < KC / 16; ++s) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int kk = 16 * s + 4 * g + e;
#pragma unroll
          for (int j = 0; j < NT; ++j)
            acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(vb[kk * PIT + 16 * j + c], xv[s][e],
                                                          acc[j], 0, 0, 0);
        }
      }
      __syncthreads();
#pragma unroll
      for (int s = 0; s < KC / 16; ++s) xv[s] = xn[s];
    }
    // lane holds D[column 16j + 4g + i][row c of the wave's 16]
    const int64_t orow = blk * 64 + wave * 16 + c;
    if (orow < rows) {
#pragma unroll
      for (int j = 0; j < NT; ++j) {
        const int col = 16 * j + 4 * g;
        if (col + 4 <= d_out) *(pf32x4_t*)(Y + orow * ldy + col) = acc[j];
      }
    }
  }
}

hipError_t launch_project(hipStream_t s, const float* X, int64_t rows, int d_in, int64_t ldx,
                          const float* V, int d_out, float* Y, int64_t ldy, int num_cus) {
  if (d_out < 16 || d_out > 128 || d_out % 16 != 0 || ldy % 4 != 0 || (((uintptr_t)Y) & 15))
    return hipErrorInvalidValue;
  const bool vec = ((((uintptr_t)X) & 15) == 0) && (ldx % 4 == 0);
  int64_t blocks = (rows + 63) / 64;
  const int64_t cap = (int64_t)num_cus * 8;
  if (blocks > cap) blocks = cap;
  if (blocks < 1) blocks = 1;
  const int nt = d_out / 16;
#define KMX_P(NT_)                                                                              \
  do {                                                                                          \
    if (vec)                                                                                    \
      hipLaunchKernelGGL((project_kernel<NT_, true>), dim3((unsigned)blocks), dim3(256), 0, s, \
                         X, rows, d_in, ldx, V, d_out, Y, ldy);                                 \
    else                                                                                        \
      hipLaunchKernelGGL((project_kernel<NT_, false>), dim3((unsigned)blocks), dim3(256), 0,   \
                         s, X, rows, d_in, ldx, V, d_out, Y, ldy);                              \
    return hipGetLastError();                                                                   \
  } while (0)
  switch (nt) {
    case 1: KMX_P(1);
    case 2: KMX_P(2);
    case 3: KMX_P(3);
    case 4: KMX_P(4);
    case 5: KMX_P(5);
    case 6: KMX_P(6);
    case 7: KMX_P(7);
    case 8: KMX_P(8);
    default: break;
  }
#undef KMX_P
  return hipErrorInvalidValue;
}

}  // namespace kmx
