// Training of the candidate router: mini-batch softmax cross-entropy over
// (point, label) pairs, gradients by the chain rule, Adam updates (Kingma &
// Ba 2015) of FP32 master weights with BF16 copies for the matrix cores.
//
// Per step, with B the batch, Xb its BF16 rows and y its labels:
//   Z1 = Xb W1^T + b1, Hb = bf16(relu(Z1))              (B x 256)
//   Z2 = Hb W2^T + b2, P = softmax(Z2)                   (B x k)
//   dZ = (P - onehot(y)) / B                             -> BF16
//   dW2 = dZ^T Hb, db2 = colsum(dZ), dH = dZ W2
//   dA = dH * [Hb > 0]                                   -> BF16
//   dW1 = dA^T Xb, db1 = colsum(dA)
// Every product runs on one BF16 MFMA GEMM kernel (FP32 accumulate) that
// reads each operand either K-contiguous or K-major, so no transposed copies
// are made.  Split-K partial products are summed in a fixed order by the
// consumer kernels: results do not depend on scheduling.
#include "kmx_device.h"
#include "kmx_internal.h"

namespace kmx {

typedef __attribute__((ext_vector_type(8))) __bf16 tbf16x8_t;
typedef __attribute__((ext_vector_type(4))) float tf32x4_t;
typedef __attribute__((ext_vector_type(4))) unsigned int tu32x4_t;

// ---- sample order ---------------------------------------------------------
__device__ __forceinline__ uint64_t t_mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Pseudo-random permutation of [0, N): a four-round balanced Feistel network
// on 2*hb bits (2^(2 hb) >= N) with SplitMix64 round functions, walked along
// its cycle until the value falls below N.
__device__ uint64_t feistel_index(uint64_t x, uint64_t N, int hb, uint64_t key) {
  const uint64_t hm = (hb >= 64) ? ~0ull : ((1ull << hb) - 1ull);
  do {
    uint64_t L = x >> hb, R = x & hm;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const uint64_t F = t_mix64(R ^ (key + (uint64_t)(r + 1) * 0x9E3779B97F4A7C15ull)) & hm;
      const uint64_t t = L ^ F;
      L = R;
      R = t;
    }
    x = (L << hb) | R;
  } while (x >= N);
  return x;
}

// One wave per batch row: sample s = first + i of the epoch (permuted when
// shuffle != 0) is pair p = (set, row) = (p / n, p % n).
__global__ __launch_bounds__(256) void gather_batch_kernel(
    const float* __restrict__ X, int64_t n, int d, int64_t ldx, const int32_t* __restrict__ labels,
    uint64_t total, int64_t first, int bsz, int d8, int shuffle, int hb, uint64_t key, int k,
    uint16_t* __restrict__ Xb, int32_t* __restrict__ yb) {
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= bsz) return;
  const uint64_t s = (uint64_t)first + (uint64_t)i;
  const uint64_t p = shuffle ? feistel_index(s, total, hb, key) : s;
  const int64_t r = (int64_t)(p % (uint64_t)n);
  const int64_t set = (int64_t)(p / (uint64_t)n);
  const float* x = X + r * ldx;
  for (int c = lane; c < d8; c += 64)
    Xb[(int64_t)i * d8 + c] = (c < d) ? f32_to_bf16_rne(x[c]) : (uint16_t)0;
  if (lane == 0) {
    const int y = labels[set * n + r];
    yb[i] = (y >= 0 && y < k) ? y : 0;
  }
}

hipError_t launch_gather_batch(hipStream_t s, const float* X, int64_t n, int d, int64_t ldx,
                               const int32_t* labels, uint64_t total, int64_t first, int bsz,
                               int d8, int shuffle, uint64_t key, int k, uint16_t* Xb,
                               int32_t* yb) {
  int bits = 1;
  while (bits < 64 && (1ull << bits) < total) ++bits;
  const int hb = (bits + 1) / 2;
  hipLaunchKernelGGL(gather_batch_kernel, dim3((unsigned)((bsz + 3) / 4)), dim3(256), 0, s, X, n,
                     d, ldx, labels, total, first, bsz, d8, shuffle, hb, key, k, Xb, yb);
  return hipGetLastError();
}

// ---- BF16 GEMM --------------------------------------------------------------
// Cp[z] (M x N, row-major, leading dimension N) = sum over k in split z of
// A(m, k) B(n, k), with A(m, k) = A[m*lda + k] (AK = false, K-contiguous) or
// A[k*lda + m] (AK = true, K-major); the same for B.  Tile 128 x 128 x 32,
// four waves of 64 x 64 (4 x 4 MFMA 16x16x32 tiles).  Requirements (checked
// by the launcher): 16-byte aligned bases, lda and ldb multiples of 8,
// K % 8 == 0 for a K-contiguous operand, M (N) % 8 == 0 for a K-major one,
// kchunk a multiple of 32.
template <bool AK, bool BK>
__global__ __launch_bounds__(256) void gemm_bf16_kernel(int M, int N, int K, int kchunk,
                                                        const uint16_t* __restrict__ A,
                                                        int64_t lda,
                                                        const uint16_t* __restrict__ B,
                                                        int64_t ldb, float* __restrict__ Cp) {
  constexpr int BM = 128, BN = 128, PIT = 40;  // LDS pitch in BF16 elements
  __shared__ __attribute__((aligned(16))) uint16_t As[BM * PIT];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[BN * PIT];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int prow = lane & 15, grp = lane >> 4;
  const int wm = wave >> 1, wn = wave & 1;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const int kb = blockIdx.z * kchunk;
  const int ke = min(K, kb + kchunk);
  float* Cz = Cp + (int64_t)blockIdx.z * M * N;

  tf32x4_t acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = (tf32x4_t){0.f, 0.f, 0.f, 0.f};

  tu32x4_t ra[2], rb[2];
  auto gload = [&](const uint16_t* S, int64_t ld, bool kmaj, int rows, int r0, int k0,
                   tu32x4_t* st) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int u = tid + 256 * q;
      tu32x4_t v = {0u, 0u, 0u, 0u};
      if (!kmaj) {
        const int row = u >> 2, kc = (u & 3) * 8;
        if (r0 + row < rows && k0 + kc < ke)
          v = *(const tu32x4_t*)(S + (int64_t)(r0 + row) * ld + k0 + kc);
      } else {
        const int kk = u >> 4, mc = (u & 15) * 8;
        if (k0 + kk < ke && r0 + mc < rows)
          v = *(const tu32x4_t*)(S + (int64_t)(k0 + kk) * ld + r0 + mc);
      }
      st[q] = v;
    }
  };
  auto sstore = [&](uint16_t* S, bool kmaj, const tu32x4_t* st) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int u = tid + 256 * q;
      if (!kmaj) {
        const int row = u >> 2, kc = (u & 3) * 8;
        *(tu32x4_t*)(S + row * PIT + kc) = st[q];
      } else {
        const int kk = u >> 4, mc = (u & 15) * 8;
#pragma unroll
        for (int e = 0; e < 8; ++e)
          S[(mc + e) * PIT + kk] = (uint16_t)(st[q][e >> 1] >> (16 * (e & 1)));
      }
    }
  };

  if (kb < ke) {
    gload(A, lda, AK, M, m0, kb, ra);
    gload(B, ldb, BK, N, n0, kb, rb);
  }
  for (int k0 = kb; k0 < ke; k0 += 32) {
    __syncthreads();
    sstore(As, AK, ra);
    sstore(Bs, BK, rb);
    __syncthreads();
    if (k0 + 32 < ke) {
      gload(A, lda, AK, M, m0, k0 + 32, ra);
      gload(B, ldb, BK, N, n0, k0 + 32, rb);
    }
    tu32x4_t af[4], bf[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) af[i] = *(const tu32x4_t*)(As + (wm * 64 + i * 16 + prow) * PIT + grp * 8);
#pragma unroll
    for (int j = 0; j < 4; ++j) bf[j] = *(const tu32x4_t*)(Bs + (wn * 64 + j * 16 + prow) * PIT + grp * 8);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
            __builtin_bit_cast(tbf16x8_t, af[i]), __builtin_bit_cast(tbf16x8_t, bf[j]), acc[i][j],
            0, 0, 0);
  }
  // lane holds D[m = 4 grp + e][n = prow] of each 16 x 16 tile
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int m = m0 + wm * 64 + i * 16 + grp * 4 + e;
        const int nn = n0 + wn * 64 + j * 16 + prow;
        if (m < M && nn < N) Cz[(int64_t)m * N + nn] = acc[i][j][e];
      }
}

// Splits of K so that the grid holds about two workgroups per compute unit,
// each split at least 128 deep.  Returns the number of splits; *kchunk is a
// multiple of 32.
int gemm_splits(int M, int N, int K, int num_cus, int* kchunk) {
  const int tiles = ((M + 127) / 128) * ((N + 127) / 128);
  int s = (2 * num_cus + tiles - 1) / tiles;
  const int maxs = (K + 127) / 128;
  if (s > maxs) s = maxs;
  if (s < 1) s = 1;
  int kc = (K + s - 1) / s;
  kc = (kc + 31) / 32 * 32;
  s = (K + kc - 1) / kc;
  if (s < 1) s = 1;
  *kchunk = kc;
  return s;
}

hipError_t launch_gemm_bf16(hipStream_t s, int M, int N, int K, const uint16_t* A, int64_t lda,
                            bool ak, const uint16_t* B, int64_t ldb, bool bk, float* Cp, int splits,
                            int kchunk) {
  if ((((uintptr_t)A) & 15) || (((uintptr_t)B) & 15) || (lda % 8) || (ldb % 8) ||
      (kchunk % 32) || (!ak && K % 8) || (!bk && K % 8) || (ak && M % 8) || (bk && N % 8))
    return hipErrorInvalidValue;
  const dim3 grid((unsigned)((N + 127) / 128), (unsigned)((M + 127) / 128), (unsigned)splits);
  if (!ak && !bk)
    hipLaunchKernelGGL((gemm_bf16_kernel<false, false>), grid, dim3(256), 0, s, M, N, K, kchunk, A,
                       lda, B, ldb, Cp);
  else if (!ak && bk)
    hipLaunchKernelGGL((gemm_bf16_kernel<false, true>), grid, dim3(256), 0, s, M, N, K, kchunk, A,
                       lda, B, ldb, Cp);
  else if (ak && !bk)
    hipLaunchKernelGGL((gemm_bf16_kernel<true, false>), grid, dim3(256), 0, s, M, N, K, kchunk, A,
                       lda, B, ldb, Cp);
  else
    hipLaunchKernelGGL((gemm_bf16_kernel<true, true>), grid, dim3(256), 0, s, M, N, K, kchunk, A,
                       lda, B, ldb, Cp);
  return hipGetLastError();
}

// ---- epilogues ---------------------------------------------------------------
// mode 0: Hb = bf16(relu(sum_z P + bias))      (P: S x M x N; out M x N)
// mode 1: dAb = bf16(sum_z P) where Hb > 0, else 0
__global__ void ep_hidden_kernel(const float* __restrict__ P, int S, int M, int N,
                                 const float* __restrict__ bias, const uint16_t* __restrict__ Hb,
                                 uint16_t* __restrict__ out, int mode) {
  const int64_t MN = (int64_t)M * N;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < MN;
       i += (int64_t)gridDim.x * blockDim.x) {
    float v = 0.0f;
    for (int z = 0; z < S; ++z) v += P[z * MN + i];
    if (mode == 0) {
      v = fmaxf(v + bias[i % N], 0.0f);
    } else {
      if (!(Hb[i] & 0x7FFFu) || (Hb[i] & 0x8000u)) v = 0.0f;
    }
    out[i] = f32_to_bf16_rne(v);
  }
}

hipError_t launch_ep_hidden(hipStream_t s, const float* P, int S, int M, int N, const float* bias,
                            const uint16_t* Hb, uint16_t* out, int mode) {
  int64_t blocks = ((int64_t)M * N + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(ep_hidden_kernel, dim3((unsigned)blocks), dim3(256), 0, s, P, S, M, N, bias,
                     Hb, out, mode);
  return hipGetLastError();
}

// One wave per batch row: logits z = P[row] + b2 (the k real columns of the
// k8-wide product), log-sum-exp, loss_row = lse - z_y, dZ = (softmax - onehot)
// / B stored as BF16 (zero in the padding columns).
__global__ __launch_bounds__(256) void softmax_ce_kernel(const float* __restrict__ P, int bsz,
                                                         int k, int k8,
                                                         const float* __restrict__ b2,
                                                         const int32_t* __restrict__ yb,
                                                         uint16_t* __restrict__ dZ,
                                                         float* __restrict__ lossrow) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= bsz) return;
  const float* z = P + (int64_t)row * k8;
  float mx = -__builtin_inff();
  for (int j = lane; j < k; j += 64) mx = fmaxf(mx, z[j] + b2[j]);
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) mx = fmaxf(mx, __shfl_xor(mx, m, 64));
  float se = 0.0f;
  for (int j = lane; j < k; j += 64) se += expf(z[j] + b2[j] - mx);
  se = wave_sum_f32(se);
  const int y = yb[row];
  const float inv = 1.0f / (float)bsz;
  const float lse = logf(se);
  for (int j = lane; j < k8; j += 64) {
    float g = 0.0f;
    if (j < k) {
      g = expf(z[j] + b2[j] - mx - lse);
      if (j == y) g -= 1.0f;
      g *= inv;
    }
    dZ[(int64_t)row * k8 + j] = f32_to_bf16_rne(g);
  }
  if (lane == 0) lossrow[row] = lse - (z[y] + b2[y] - mx);
}

hipError_t launch_softmax_ce(hipStream_t s, const float* P, int bsz, int k, int k8,
                             const float* b2, const int32_t* yb, uint16_t* dZ, float* lossrow) {
  hipLaunchKernelGGL(softmax_ce_kernel, dim3((unsigned)((bsz + 3) / 4)), dim3(256), 0, s, P, bsz,
                     k, k8, b2, yb, dZ, lossrow);
  return hipGetLastError();
}

// out[r*cols + c] = sum_z P[z][r*ldp + c] for r < rows, c < cols.
__global__ void sum_partials_kernel(const float* __restrict__ P, int S, int64_t zstride, int rows,
                                    int cols, int ldp, float* __restrict__ out) {
  const int64_t total = (int64_t)rows * cols;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / cols, c = i % cols;
    float v = 0.0f;
    for (int z = 0; z < S; ++z) v += P[z * zstride + r * ldp + c];
    out[i] = v;
  }
}

hipError_t launch_sum_partials(hipStream_t s, const float* P, int S, int64_t zstride, int rows,
                               int cols, int ldp, float* out) {
  int64_t blocks = ((int64_t)rows * cols + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(sum_partials_kernel, dim3((unsigned)blocks), dim3(256), 0, s, P, S, zstride,
                     rows, cols, ldp, out);
  return hipGetLastError();
}

// Column sums of a BF16 matrix (rows x cols, leading dimension ld): partial
// sums over row segments, then the sum of the segments in order.
__global__ void colsum_part_kernel(const uint16_t* __restrict__ Mx, int rows, int cols, int ld,
                                   int rps, float* __restrict__ part) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int sgm = blockIdx.y;
  if (c >= cols) return;
  const int r1 = min(rows, (sgm + 1) * rps);
  float v = 0.0f;
  for (int r = sgm * rps; r < r1; ++r) v += bf16_to_f32(Mx[(int64_t)r * ld + c]);
  part[(int64_t)sgm * cols + c] = v;
}

__global__ void colsum_final_kernel(const float* __restrict__ part, int S, int cols,
                                    float* __restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  float v = 0.0f;
  for (int z = 0; z < S; ++z) v += part[(int64_t)z * cols + c];
  out[c] = v;
}

hipError_t launch_colsum(hipStream_t s, const uint16_t* Mx, int rows, int cols, int ld,
                         float* part, float* out) {
  const int rps = 256;
  const int S = (rows + rps - 1) / rps;
  hipLaunchKernelGGL(colsum_part_kernel, dim3((unsigned)((cols + 255) / 256), (unsigned)S),
                     dim3(256), 0, s, Mx, rows, cols, ld, rps, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(colsum_final_kernel, dim3((unsigned)((cols + 255) / 256)), dim3(256), 0, s,
                     part, S, cols, out);
  return hipGetLastError();
}

int colsum_segments(int rows) { return (rows + 255) / 256; }

// Mean of the per-row losses of one step (fixed-order FP64 sum).
__global__ void loss_mean_kernel(const float* __restrict__ lossrow, int bsz,
                                 double* __restrict__ out) {
  __shared__ double red[256];
  double v = 0.0;
  for (int i = threadIdx.x; i < bsz; i += 256) v += (double)lossrow[i];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int h = 128; h >= 1; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0] / (double)bsz;
}

hipError_t launch_loss_mean(hipStream_t s, const float* lossrow, int bsz, double* out) {
  hipLaunchKernelGGL(loss_mean_kernel, dim3(1), dim3(256), 0, s, lossrow, bsz, out);
  return hipGetLastError();
}

// Adam on one parameter tensor of rows x cols FP32 values:
//   m = b1 m + (1 - b1) g,  v = b2 v + (1 - b2) g^2,
//   p -= lr (m / bc1) / (sqrt(v / bc2) + eps),  bc = 1 - beta^t;
// the BF16 copy (when given) is written at bf[r*ldb + c].
__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g,
                            float* __restrict__ m, float* __restrict__ v, int rows, int cols,
                            float lr, float beta1, float beta2, float eps, float bc1, float bc2,
                            uint16_t* __restrict__ bf, int ldb) {
  const int64_t total = (int64_t)rows * cols;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = beta1 * m[i] + (1.0f - beta1) * gi;
    const float vi = beta2 * v[i] + (1.0f - beta2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    p[i] = pi;
    if (bf) bf[(i / cols) * ldb + (i % cols)] = f32_to_bf16_rne(pi);
  }
}

hipError_t launch_adam(hipStream_t s, float* p, const float* g, float* m, float* v, int rows,
                       int cols, float lr, float beta1, float beta2, float eps, float bc1, float bc2,
                       uint16_t* bf, int ldb) {
  int64_t blocks = ((int64_t)rows * cols + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, g, m, v, rows, cols,
                     lr, beta1, beta2, eps, bc1, bc2, bf, ldb);
  return hipGetLastError();
}

// BF16 copy of a rows x cols FP32 matrix into a zero-padded buffer of
// prow x ldb (rows <= prow, cols <= ldb).
__global__ void to_bf16_pad_kernel(const float* __restrict__ src, int rows, int cols, int prow,
                                   int ldb, uint16_t* __restrict__ dst) {
  const int64_t total = (int64_t)prow * ldb;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / ldb, c = i % ldb;
    dst[i] = (r < rows && c < cols) ? f32_to_bf16_rne(src[r * cols + c]) : (uint16_t)0;
  }
}

hipError_t launch_to_bf16_pad(hipStream_t s, const float* src, int rows, int cols, int prow,
                              int ldb, uint16_t* dst) {
  int64_t blocks = ((int64_t)prow * ldb + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(to_bf16_pad_kernel, dim3((unsigned)blocks), dim3(256), 0, s, src, rows, cols,
                     prow, ldb, dst);
  return hipGetLastError();
}

}  // namespace kmx
