// Projection of a chunk of rows onto a low-dimensional subspace (the
// dimension reduction of the streamed pipeline, Sec. 2.2 "Using SVD to project
// to the best fit subspace": each row is replaced
// by its coordinates in the span of the top right singular vectors V, so
// that squared distances inside that span are preserved).
//
//   Y[r][j] = sum_i X[r][i] V[i][j],   X: rows x d_in, V: d_in x d_out (FP32)
//
// FP32 MFMA 16x16x4 with FP32 accumulation.  V is first transposed into a
// workspace Vt (d_out x dpad, dpad = d_in rounded up to 64, zero padding), so
// a lane reads the four k values it needs for four MFMAs with one 16-byte LDS
// read.  Per chunk of 64 k, lane (c, g) = (l % 16, l / 16) holds k0 + 16g ..
// k0 + 16g + 15 of its row (four 16-byte loads, 256 contiguous bytes per row
// across the four lane groups); MFMA e of step s contracts k = k0 + 16g +
// 4s + e on both operands, so every k meets its own V row exactly once.
// A = Vt (16 output columns x 4 k, from LDS), B = X (4 k x 16 rows), D holds
// output columns 16j + 4g + i of row c (one 16-byte store per column tile).
// Workgroup: 4 waves x RG groups of 16 rows; the next chunk's rows and Vt
// slice are loaded while the current chunk is contracted.
#include "kmx_internal.h"

namespace kmx {

typedef __attribute__((ext_vector_type(4))) float pf32x4_t;

// Vt[j][i] = V[i][j] for i < d_in, 0 for d_in <= i < dpad.
__global__ void transpose_v_kernel(const float* __restrict__ V, int d_in, int d_out, int dpad,
                                   float* __restrict__ Vt) {
  const int64_t total = (int64_t)d_out * dpad;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int j = (int)(e / dpad), i = (int)(e - (int64_t)j * dpad);
    Vt[e] = (i < d_in) ? V[(int64_t)i * d_out + j] : 0.0f;
  }
}

template <int NT, int RG, bool VEC>
__global__ __launch_bounds__(256) void project_kernel(const float* __restrict__ X, int64_t rows,
                                                      int d_in, int64_t ldx,
                                                      const float* __restrict__ Vt, int dpad,
                                                      float* __restrict__ Y, int64_t ldy) {
  constexpr int KC = 64;               // k per chunk
  constexpr int DO = NT * 16;          // output columns
  constexpr int PIT = KC + 4;          // LDS pitch (floats) of a Vt row
  constexpr int RPB = 4 * RG * 16;     // rows per workgroup
  constexpr int VPT = DO * KC / 4 / 256;  // 16-byte Vt pieces per thread and chunk
  __shared__ __attribute__((aligned(16))) float vs[2][DO * PIT];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int c = lane & 15, g = lane >> 4;
  const int64_t nblk = (rows + RPB - 1) / RPB;
  const int nchunks = dpad / KC;

  auto load_v = [&](int ch, pf32x4_t (&vr)[VPT > 0 ? VPT : 1]) {
#pragma unroll
    for (int q = 0; q < VPT; ++q) {
      const int piece = tid + 256 * q;          // (column, 16-byte unit of the chunk)
      const int j = piece / (KC / 4), u = piece - j * (KC / 4);
      vr[q] = *(const pf32x4_t*)(Vt + (int64_t)j * dpad + ch * KC + 4 * u);
    }
  };
  auto store_v = [&](int buf, const pf32x4_t (&vr)[VPT > 0 ? VPT : 1]) {
#pragma unroll
    for (int q = 0; q < VPT; ++q) {
      const int piece = tid + 256 * q;
      const int j = piece / (KC / 4), u = piece - j * (KC / 4);
      *(pf32x4_t*)(&vs[buf][j * PIT + 4 * u]) = vr[q];
    }
  };
  auto load_x = [&](const float* const (&xr)[RG], const bool (&valid)[RG], int ch,
                    pf32x4_t (&xv)[RG][4]) {
#pragma unroll
    for (int rg = 0; rg < RG; ++rg) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int k = ch * KC + 16 * g + 4 * q;
        pf32x4_t v = {0.f, 0.f, 0.f, 0.f};
        if (valid[rg]) {
          if (VEC && k + 4 <= d_in) {
            v = *(const pf32x4_t*)(xr[rg] + k);
          } else {
#pragma unroll
            for (int e = 0; e < 4; ++e)
              if (k + e < d_in) v[e] = xr[rg][k + e];
          }
        }
        xv[rg][q] = v;
      }
    }
  };

  for (int64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
    const float* xr[RG];
    bool valid[RG];
#pragma unroll
    for (int rg = 0; rg < RG; ++rg) {
      const int64_t row = blk * RPB + (int64_t)(wave * RG + rg) * 16 + c;
      valid[rg] = row < rows;
      xr[rg] = X + (valid[rg] ? row : 0) * ldx;
    }
    pf32x4_t acc[RG][NT];
#pragma unroll
    for (int rg = 0; rg < RG; ++rg)
#pragma unroll
      for (int j = 0; j < NT; ++j) acc[rg][j] = (pf32x4_t){0.f, 0.f, 0.f, 0.f};
    pf32x4_t xv[RG][4], xn[RG][4];
    pf32x4_t vr[VPT > 0 ? VPT : 1];
    __syncthreads();                   // previous block done with vs
    load_v(0, vr);
    load_x(xr, valid, 0, xv);
    store_v(0, vr);
    __syncthreads();
    for (int ch = 0; ch < nchunks; ++ch) {
      const int buf = ch & 1;
      const bool more = ch + 1 < nchunks;
      if (more) {
        load_v(ch + 1, vr);
        load_x(xr, valid, ch + 1, xn);
      }
      const float* vb = &vs[buf][0];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
#pragma unroll
        for (int j = 0; j < NT; ++j) {
          const pf32x4_t a = *(const pf32x4_t*)(vb + (16 * j + c) * PIT + 16 * g + 4 * s);
#pragma unroll
          for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int rg = 0; rg < RG; ++rg)
              acc[rg][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[e], xv[rg][s][e], acc[rg][j],
                                                                0, 0, 0);
        }
      }
      if (more) {
        store_v(buf ^ 1, vr);
#pragma unroll
        for (int rg = 0; rg < RG; ++rg)
#pragma unroll
          for (int q = 0; q < 4; ++q) xv[rg][q] = xn[rg][q];
      }
      __syncthreads();
    }
    // lane holds D[column 16j + 4g + i][row c of its row group]
#pragma unroll
    for (int rg = 0; rg < RG; ++rg) {
      const int64_t orow = blk * RPB + (int64_t)(wave * RG + rg) * 16 + c;
      if (orow < rows) {
#pragma unroll
        for (int j = 0; j < NT; ++j) *(pf32x4_t*)(Y + orow * ldy + 16 * j + 4 * g) = acc[rg][j];
      }
    }
  }
}

hipError_t launch_project(hipStream_t s, const float* X, int64_t rows, int d_in, int64_t ldx,
                          const float* V, int d_out, float* Y, int64_t ldy, float* Vt,
                          int num_cus) {
  if (d_out < 16 || d_out > 128 || d_out % 16 != 0 || ldy % 4 != 0 || (((uintptr_t)Y) & 15) ||
      (((uintptr_t)Vt) & 15))
    return hipErrorInvalidValue;
  const int dpad = project_dpad(d_in);
  {
    const int64_t total = (int64_t)d_out * dpad;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 2048) blocks = 2048;
    hipLaunchKernelGGL(transpose_v_kernel, dim3((unsigned)blocks), dim3(256), 0, s, V, d_in, d_out,
                       dpad, Vt);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const bool vec = ((((uintptr_t)X) & 15) == 0) && (ldx % 4 == 0);
  constexpr int RG = 2;
  int64_t blocks = (rows + 4 * RG * 16 - 1) / (4 * RG * 16);
  const int64_t cap = (int64_t)num_cus * 4;
  if (blocks > cap) blocks = cap;
  if (blocks < 1) blocks = 1;
  const int nt = d_out / 16;
#define KMX_P(NT_)                                                                                \
  do {                                                                                            \
    if (vec)                                                                                      \
      hipLaunchKernelGGL((project_kernel<NT_, RG, true>), dim3((unsigned)blocks), dim3(256), 0,  \
                         s, X, rows, d_in, ldx, Vt, dpad, Y, ldy);                                \
    else                                                                                          \
      hipLaunchKernelGGL((project_kernel<NT_, RG, false>), dim3((unsigned)blocks), dim3(256), 0, \
                         s, X, rows, d_in, ldx, Vt, dpad, Y, ldy);                                \
    return hipGetLastError();                                                                     \
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

int project_dpad(int d_in) { return (d_in + 63) / 64 * 64; }

// Lift of coordinates back to R^d (the rows of A_m = A V V^T in Sec. 2.2
// "Using SVD to project to the best fit subspace": a point keeps d
// coordinates, its intrinsic dimension is m):
//     Y[i][c] = sum_j Z[i][j] V[c][j],   Z: rows x m, V: d x m (FP32),
// FP32 FMAs in j order.  A workgroup stages 64 rows of Z and 64 rows of V
// (m <= 128 values each, padded against bank conflicts) in LDS; thread
// (ty, tx) accumulates rows 4 ty .. 4 ty + 3 and columns 4 tx .. 4 tx + 3 and
// writes them as 16-byte stores when the row allows.
constexpr int kLiftMaxM = 128;
constexpr int kLiftPitch = kLiftMaxM + 1;

__global__ __launch_bounds__(256) void lift_kernel(const float* __restrict__ Z, int64_t rows, int m,
                                                   int64_t ldz, const float* __restrict__ V, int d,
                                                   float* __restrict__ Y, int64_t ldy) {
  __shared__ float zs[64 * kLiftPitch];
  __shared__ float vs[64 * kLiftPitch];
  const int tid = threadIdx.x;
  const int ty = tid >> 4, tx = tid & 15;
  const int64_t r0 = (int64_t)blockIdx.y * 64;
  const int c0 = blockIdx.x * 64;
  for (int e = tid; e < 64 * m; e += 256) {
    const int r = e / m, j = e - r * m;
    zs[r * kLiftPitch + j] = (r0 + r < rows) ? Z[(r0 + r) * ldz + j] : 0.0f;
    vs[r * kLiftPitch + j] = (c0 + r < d) ? V[(int64_t)(c0 + r) * m + j] : 0.0f;
  }
  __syncthreads();
  float acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.0f;
  for (int j = 0; j < m; ++j) {
    float zv[4], vv[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) zv[a] = zs[(4 * ty + a) * kLiftPitch + j];
#pragma unroll
    for (int b = 0; b < 4; ++b) vv[b] = vs[(4 * tx + b) * kLiftPitch + j];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] = fmaf(zv[a], vv[b], acc[a][b]);
  }
  const int c = c0 + 4 * tx;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int64_t r = r0 + 4 * ty + a;
    if (r >= rows) continue;
    float* yr = Y + r * ldy + c;
    if (c + 4 <= d && ((((uintptr_t)yr) & 15) == 0)) {
      *(pf32x4_t*)yr = (pf32x4_t){acc[a][0], acc[a][1], acc[a][2], acc[a][3]};
    } else {
#pragma unroll
      for (int b = 0; b < 4; ++b)
        if (c + b < d) yr[b] = acc[a][b];
    }
  }
}

hipError_t launch_lift(hipStream_t s, const float* Z, int64_t rows, int m, int64_t ldz,
                       const float* V, int d, float* Y, int64_t ldy) {
  if (m < 1 || m > kLiftMaxM) return hipErrorInvalidValue;
  const int64_t rb = (rows + 63) / 64;
  if (rb > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(lift_kernel, dim3((unsigned)((d + 63) / 64), (unsigned)rb), dim3(256), 0, s,
                     Z, rows, m, ldz, V, d, Y, ldy);
  return hipGetLastError();
}

}  // namespace kmx
