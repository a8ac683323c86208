// Input preparation: per-row statistics and the BF16 copy of X (once per
// dataset), per-iteration center preparation, and small fill kernels.
//
// Distances are squared Euclidean (Sec. 1).  The quantized copy feeds the
// distance GEMM only; every reported cost and centroid uses the FP32 input in
// FP64 arithmetic.  The statistics feed the rigorous error bound that decides
// which rows the assignment re-checks.
#include "kmx_internal.h"
#include "kmx_device.h"

namespace kmx {

// One wave per row.  Writes RowStats and, when Xq != nullptr, the BF16 row
// (round to nearest even) of dp elements: x~ in columns [0, d), zeros after.
// xq_max receives max_i ||x~_i||.
__device__ __forceinline__ unsigned block_max_u32(unsigned v, unsigned* sh) {
  // maxima of non-negative float bits over a 256-thread block (valid in thread 0)
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v = max(v, (unsigned)__shfl_xor((int)v, m, 64));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  v = max(max(sh[0], sh[1]), max(sh[2], sh[3]));
  __syncthreads();
  return v;
}

__global__ __launch_bounds__(256) void prep_rows_kernel(const float* __restrict__ X, int64_t n,
                                                        int d, int64_t ldx, int dp,
                                                        uint16_t* __restrict__ Xq,
                                                        RowStats* __restrict__ st,
                                                        unsigned* __restrict__ xq_max) {
  const int lane = threadIdx.x & 63;
  const int64_t wave0 = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x >> 6);
  unsigned local_max = 0u;
  for (int64_t row = wave0; row < n; row += nwaves) {
    const float* x = X + row * ldx;
    double s2 = 0.0, q2 = 0.0, r2 = 0.0;
    const int lim = Xq ? dp : d;
    for (int c = lane; c < lim; c += 64) {
      const float v = (c < d) ? x[c] : 0.0f;
      const double vd = (double)v;
      s2 += vd * vd;
      if (Xq) {
        const uint16_t b = f32_to_bf16_rne(v);
        Xq[row * dp + c] = b;
        if (c < d) {
          const double qd = (double)bf16_to_f32(b);
          q2 += qd * qd;
          r2 += (vd - qd) * (vd - qd);
        }
      }
    }
    s2 = wave_sum_f64(s2);
    q2 = wave_sum_f64(q2);
    r2 = wave_sum_f64(r2);
    if (lane == 0) {
      RowStats r;
      r.xn2 = (float)s2;
      r.nx = f64_to_f32_up(sqrt(s2));
      if (Xq) {
        r.nxq = f64_to_f32_up(sqrt(q2));
        r.rx = f64_to_f32_up(sqrt(r2));
      } else {
        r.nxq = r.nx;
        r.rx = 0.0f;
      }
      st[row] = r;
      local_max = max(local_max, __float_as_uint(r.nxq));
    }
  }
  // one atomic per block (same-address atomics from every XCD serialize)
  __shared__ unsigned shm[4];
  local_max = block_max_u32(local_max, shm);
  if (threadIdx.x == 0 && xq_max) atomicMax(xq_max, local_max);
}

hipError_t launch_prep_rows(hipStream_t s, const float* X, int64_t n, int d, int64_t ldx,
                            int dp, uint16_t* Xq, RowStats* st, unsigned* xq_max, int num_cus) {
  int64_t blocks = (n + 3) / 4;
  const int64_t cap = (int64_t)num_cus * 16;
  if (blocks > cap) blocks = cap;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(prep_rows_kernel, dim3((unsigned)blocks), dim3(256), 0, s, X, n, d, ldx,
                     dp, Xq, st, xq_max);
  return hipGetLastError();
}

// Pass A, one wave per (padded) center.  prec 0 (FP32): copy of c_j into a
// row of dp floats, ch[j] = ||c_j||^2 / 2 (+inf for padding rows, whose score
// is then never selected).  prec 1 (BF16): c~_j (round to nearest even) in
// columns [0, d), zeros elsewhere; hd[j] = ||c_j||^2 / 2 in FP64.
// prec kSplitBf16: a row of 2 dp BF16 values, the high parts hi = bf16(c)
// then the low parts bf16(c - hi) (c - hi is exact in FP32); ch as for FP32.
// Maxima of the norms go to cs.

// Each wave takes padded centers wave_id, wave_id + total_waves, ...; the
// norm maxima are reduced over the block and reach cs with one atomic per
// block and statistic (same-address atomics from every XCD serialize).
__global__ __launch_bounds__(256) void prep_centers_kernel(const float* __restrict__ C, int k,
                                                           int d, int dp, int kpad, int prec,
                                                           void* __restrict__ Cq,
                                                           float* __restrict__ ch,
                                                           double* __restrict__ hd,
                                                           CenterStats* __restrict__ cs) {
  __shared__ unsigned shm[4];
  const int lane = threadIdx.x & 63;
  const int wave = blockIdx.x * 4 + (threadIdx.x >> 6), nwaves = gridDim.x * 4;
  unsigned cqm = 0u, rcm = 0u, cnm = 0u;
  for (int j = wave; j < kpad; j += nwaves) {
    double s2 = 0.0, q2 = 0.0, r2 = 0.0;
    // unrolled so the loads of a row are in flight together
#pragma unroll 8
    for (int c = lane; c < dp; c += 64) {
      const float v = (j < k && c < d) ? C[(int64_t)j * d + c] : 0.0f;
      const double vd = (double)v;
      s2 += vd * vd;
      if (prec == 1) {
        const uint16_t b = f32_to_bf16_rne(v);
        ((uint16_t*)Cq)[(int64_t)j * dp + c] = b;
        const double qd = (double)bf16_to_f32(b);
        q2 += qd * qd;
        r2 += (vd - qd) * (vd - qd);
      } else if (prec == kSplitBf16) {
        // high part, then the low part of the exact remainder v - hi
        const uint16_t h = f32_to_bf16_rne(v);
        const uint16_t l = f32_to_bf16_rne(v - bf16_to_f32(h));
        ((uint16_t*)Cq)[(int64_t)j * 2 * dp + c] = h;
        ((uint16_t*)Cq)[(int64_t)j * 2 * dp + dp + c] = l;
      } else {
        ((float*)Cq)[(int64_t)j * dp + c] = v;
      }
    }
    s2 = wave_sum_f64(s2);
    q2 = wave_sum_f64(q2);
    r2 = wave_sum_f64(r2);
    if (lane == 0) {
      if (prec == 1) {
        hd[j] = 0.5 * s2;
      } else {
        ch[j] = (j < k) ? (float)(0.5 * s2) : __builtin_inff();
      }
    }
    if (j < k) {
      const float cn = f64_to_f32_up(sqrt(s2));
      const float cq = (prec == 1) ? f64_to_f32_up(sqrt(q2)) : cn;
      const float rc = (prec == 1) ? f64_to_f32_up(sqrt(r2)) : 0.0f;
      cqm = max(cqm, __float_as_uint(cq));
      rcm = max(rcm, __float_as_uint(rc));
      cnm = max(cnm, __float_as_uint(cn));
    }
  }
  cqm = block_max_u32(cqm, shm);
  rcm = block_max_u32(rcm, shm);
  cnm = block_max_u32(cnm, shm);
  if (threadIdx.x == 0) {
    atomicMax(&cs->cq_max, cqm);
    atomicMax(&cs->rc_max, rcm);
    atomicMax(&cs->cn_max, cnm);
  }
}

// ---------------------------------------------------------------------------
// FP8 E4M3 (OCP: bias 7, largest finite 448, subnormals m 2^-9, no
// infinities).  Round to nearest even; magnitudes above 448 saturate.  The
// error bounds use the residuals of the stored values, so they hold for any
// rounding; round-to-nearest only keeps them small.
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned f32_to_e4m3_rne(float v) {
  const unsigned u = __float_as_uint(v);
  const unsigned sgn = (u >> 24) & 0x80u;
  const unsigned a = u & 0x7FFFFFFFu;
  unsigned r;
  if (a >= 0x43E00000u) {              // >= 448, inf, NaN
    r = 0x7Eu;
  } else if (a < 0x3C800000u) {        // below 2^-6: multiples of 2^-9 (8 -> 2^-6 = 0x08)
    r = (unsigned)__builtin_rintf(__uint_as_float(a) * 512.0f);
  } else {                             // keep three mantissa bits, ties to even
    const unsigned rr = a + 0x7FFFFu + ((a >> 20) & 1u);
    r = (((rr >> 23) - 120u) << 3) | ((rr >> 20) & 7u);
    if (r > 0x7Eu) r = 0x7Eu;
  }
  return sgn | r;
}

__device__ __forceinline__ float e4m3_to_f32(unsigned b) {
  const unsigned e = (b >> 3) & 15u, m = b & 7u;
  const float v = e ? __uint_as_float(((e + 120u) << 23) | (m << 20)) : (float)m * 0.001953125f;
  return (b & 0x80u) ? -v : v;
}

// Exponent e of the power-of-two scale 2^e with amax / 2^e <= 448 (smallest
// such e, clamped to the E8M0 range).
__device__ __forceinline__ int e4m3_scale_exp(float amax) {
  if (!(amax > 0.0f)) return 0;
  int e;
  const float f = frexpf(amax / 448.0f, &e);   // amax/448 = f 2^e, f in [0.5, 1)
  if (f == 0.5f) e -= 1;
  while (ldexpf(448.0f, e) < amax) ++e;        // guard against the rounding of amax / 448
  return max(-127, min(127, e));
}

// One wave per row: FP8 row of dp bytes (q in [0, d), zeros after), its E8M0
// scale byte sx8[row] = e + 127, and RowStats with nxq = ||2^e q|| and
// rx = ||x - 2^e q||.  xq_max receives max_i nxq_i.
__global__ __launch_bounds__(256) void prep_rows_f8_kernel(const float* __restrict__ X, int64_t n,
                                                           int d, int64_t ldx, int dp,
                                                           uint8_t* __restrict__ Xq8,
                                                           uint8_t* __restrict__ sx8,
                                                           RowStats* __restrict__ st,
                                                           unsigned* __restrict__ xq_max) {
  const int lane = threadIdx.x & 63;
  const int64_t wave0 = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x >> 6);
  unsigned local_max = 0u;
  for (int64_t row = wave0; row < n; row += nwaves) {
    const float* x = X + row * ldx;
    float amax = 0.0f;
    for (int c = lane; c < d; c += 64) amax = fmaxf(amax, fabsf(x[c]));
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) amax = fmaxf(amax, __shfl_xor(amax, m, 64));
    const int e = e4m3_scale_exp(amax);
    const float inv = ldexpf(1.0f, -e);
    const double sc = ldexp(1.0, e);
    double s2 = 0.0, q2 = 0.0, r2 = 0.0;
    for (int c0 = 4 * lane; c0 < dp; c0 += 256) {
      unsigned word = 0u;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int c = c0 + t;
        const float v = (c < d) ? x[c] : 0.0f;
        const unsigned q = f32_to_e4m3_rne(v * inv);
        const double back = (double)e4m3_to_f32(q) * sc;
        s2 += (double)v * v;
        q2 += back * back;
        r2 += ((double)v - back) * ((double)v - back);
        word |= q << (8 * t);
      }
      *(unsigned*)(Xq8 + row * dp + c0) = word;
    }
    s2 = wave_sum_f64(s2);
    q2 = wave_sum_f64(q2);
    r2 = wave_sum_f64(r2);
    if (lane == 0) {
      RowStats r;
      r.xn2 = (float)s2;
      r.nx = f64_to_f32_up(sqrt(s2));
      r.nxq = f64_to_f32_up(sqrt(q2));
      r.rx = f64_to_f32_up(sqrt(r2));
      st[row] = r;
      sx8[row] = (uint8_t)(e + 127);
      local_max = max(local_max, __float_as_uint(r.nxq));
    }
  }
  __shared__ unsigned shm[4];
  local_max = block_max_u32(local_max, shm);
  if (threadIdx.x == 0 && xq_max) atomicMax(xq_max, local_max);
}

hipError_t launch_prep_rows_f8(hipStream_t s, const float* X, int64_t n, int d, int64_t ldx,
                               int dp, uint8_t* Xq8, uint8_t* sx8, RowStats* st,
                               unsigned* xq_max, int num_cus) {
  if (dp % 256 != 0 && dp % 128 != 0) return hipErrorInvalidValue;
  int64_t blocks = (n + 3) / 4;
  const int64_t cap = (int64_t)num_cus * 16;
  if (blocks > cap) blocks = cap;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(prep_rows_f8_kernel, dim3((unsigned)blocks), dim3(256), 0, s, X, n, d, ldx,
                     dp, Xq8, sx8, st, xq_max);
  return hipGetLastError();
}

// Centers, FP8: one scale for all centers.  Pass 1: max |c_ji|.  Pass 2 (one
// wave per padded center): the FP8 row (zeros for padding), hd = ||c||^2 / 2
// in FP64 and the norm maxima.  Then the offsets (prep_offsets_kernel).
__global__ __launch_bounds__(256) void center_amax_kernel(const float* __restrict__ C,
                                                          int64_t total,
                                                          CenterStats* __restrict__ cs) {
  __shared__ unsigned shm[4];
  float m = 0.0f;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x)
    m = fmaxf(m, fabsf(C[i]));
  const unsigned bm = block_max_u32(__float_as_uint(m), shm);
  if (threadIdx.x == 0) atomicMax(&cs->c_amax, bm);
}

__global__ __launch_bounds__(256) void prep_centers_f8_kernel(const float* __restrict__ C, int k,
                                                              int d, int dp, int kpad,
                                                              uint8_t* __restrict__ Cq8,
                                                              double* __restrict__ hd,
                                                              CenterStats* __restrict__ cs) {
  __shared__ unsigned shm[4];
  const int lane = threadIdx.x & 63;
  const int wave = blockIdx.x * 4 + (threadIdx.x >> 6), nwaves = gridDim.x * 4;
  const int e = e4m3_scale_exp(__uint_as_float(cs->c_amax));
  const float inv = ldexpf(1.0f, -e);
  const double sc = ldexp(1.0, e);
  unsigned cqm = 0u, rcm = 0u, cnm = 0u;
  for (int j = wave; j < kpad; j += nwaves) {
    double s2 = 0.0, q2 = 0.0, r2 = 0.0;
#pragma unroll 4
    for (int c0 = 4 * lane; c0 < dp; c0 += 256) {
      unsigned word = 0u;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int c = c0 + t;
        const float v = (j < k && c < d) ? C[(int64_t)j * d + c] : 0.0f;
        const unsigned q = f32_to_e4m3_rne(v * inv);
        const double back = (double)e4m3_to_f32(q) * sc;
        s2 += (double)v * v;
        q2 += back * back;
        r2 += ((double)v - back) * ((double)v - back);
        word |= q << (8 * t);
      }
      *(unsigned*)(Cq8 + (int64_t)j * dp + c0) = word;
    }
    s2 = wave_sum_f64(s2);
    q2 = wave_sum_f64(q2);
    r2 = wave_sum_f64(r2);
    if (lane == 0) hd[j] = 0.5 * s2;
    if (j < k) {
      cqm = max(cqm, __float_as_uint(f64_to_f32_up(sqrt(q2))));
      rcm = max(rcm, __float_as_uint(f64_to_f32_up(sqrt(r2))));
      cnm = max(cnm, __float_as_uint(f64_to_f32_up(sqrt(s2))));
    }
  }
  cqm = block_max_u32(cqm, shm);
  rcm = block_max_u32(rcm, shm);
  cnm = block_max_u32(cnm, shm);
  if (threadIdx.x == 0) {
    if (blockIdx.x == 0) cs->c_exp = e + 127;
    atomicMax(&cs->cq_max, cqm);
    atomicMax(&cs->rc_max, rcm);
    atomicMax(&cs->cn_max, cnm);
  }
}

// BF16 and FP8, one thread per padded center: the offset
// O = (max||x~|| max||c~|| + max||c||^2 / 2) * 1.001 + 1, which makes every
// score x~.c~_j - h_j + O positive, and the accumulator start values
// ch[j] = O - hd[j] rounded to FP32 (0 for padding: score 0, never selected).
__global__ void prep_offsets_kernel(int k, int kpad, const double* __restrict__ hd,
                                    CenterStats* __restrict__ cs,
                                    const unsigned* __restrict__ xq_max, float* __restrict__ ch) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const float xm = __uint_as_float(*xq_max);
  const float cqm = __uint_as_float(cs->cq_max);
  const float cnm = __uint_as_float(cs->cn_max);
  const float O = (xm * cqm + 0.5f * cnm * cnm) * 1.001f + 1.0f;
  if (j == 0) cs->O = O;
  if (j >= kpad) return;
  ch[j] = (j < k) ? (float)((double)O - hd[j]) : 0.0f;
}

hipError_t launch_prep_centers(hipStream_t s, const float* C, int k, int d, int kpad, int dp,
                               int prec, void* Cq, float* ch, double* hd, CenterStats* cs,
                               const unsigned* xq_max) {
  // four waves per block, a few centers per wave: few blocks, few atomics
  const int cblocks = min((kpad + 7) / 8, 128);
  if (prec == 2) {
    const int64_t total = (int64_t)k * d;
    int64_t blocks = (total + 4095) / 4096;
    if (blocks > 128) blocks = 128;
    hipLaunchKernelGGL(center_amax_kernel, dim3((unsigned)blocks), dim3(256), 0, s, C, total, cs);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(prep_centers_f8_kernel, dim3(cblocks), dim3(256), 0, s, C, k, d, dp, kpad,
                       (uint8_t*)Cq, hd, cs);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(prep_offsets_kernel, dim3((kpad + 255) / 256), dim3(256), 0, s, k, kpad,
                       hd, cs, xq_max, ch);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(prep_centers_kernel, dim3(cblocks), dim3(256), 0, s, C, k, d, dp, kpad, prec,
                     Cq, ch, hd, cs);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || prec != 1) return e;
  hipLaunchKernelGGL(prep_offsets_kernel, dim3((kpad + 255) / 256), dim3(256), 0, s, k, kpad, hd,
                     cs, xq_max, ch);
  return hipGetLastError();
}

__global__ void fill_i32_kernel(int32_t* p, int64_t n, int32_t v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

__global__ void fill_u8_kernel(uint8_t* p, int64_t n, uint8_t v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

hipError_t launch_fill_i32(hipStream_t s, int32_t* p, int64_t n, int32_t v) {
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(fill_i32_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_fill_u8(hipStream_t s, uint8_t* p, int64_t n, uint8_t v) {
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(fill_u8_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

// Argument checks that need the data (run before any work of a call):
// out[0] += rows with w_i > 0, out[1] += entries that are not finite or are
// negative (weights) / not finite (any other array).  One atomic per block.
__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += (unsigned long long)__shfl_xor((long long)v, m, 64);
  return v;
}

__global__ __launch_bounds__(256) void check_weights_kernel(const float* __restrict__ w, int64_t n,
                                                            unsigned long long* out) {
  unsigned long long pos = 0, bad = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const float v = w[i];
    pos += (v > 0.0f) ? 1u : 0u;
    bad += (!(v >= 0.0f) || !isfinite(v)) ? 1u : 0u;   // NaN, negative, +inf
  }
  pos = wave_sum_u64(pos);
  bad = wave_sum_u64(bad);
  if ((threadIdx.x & 63) == 0 && (pos | bad)) {
    atomicAdd(&out[0], pos);
    atomicAdd(&out[1], bad);
  }
}

__global__ __launch_bounds__(256) void scan_finite_kernel(const float* __restrict__ A, int64_t rows,
                                                          int cols, int64_t ld,
                                                          unsigned long long* out) {
  unsigned long long bad = 0;
  const int64_t total = rows * (int64_t)cols;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
    const int64_t r = i / cols;
    const float v = A[r * ld + (i - r * cols)];
    bad += isfinite(v) ? 0u : 1u;
  }
  bad = wave_sum_u64(bad);
  if ((threadIdx.x & 63) == 0 && bad) atomicAdd(&out[1], bad);
}

hipError_t launch_check_weights(hipStream_t s, const float* w, int64_t n, unsigned long long* out,
                                int num_cus) {
  int64_t blocks = (n + 255) / 256;
  if (blocks > (int64_t)num_cus * 8) blocks = (int64_t)num_cus * 8;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(check_weights_kernel, dim3((unsigned)blocks), dim3(256), 0, s, w, n, out);
  return hipGetLastError();
}

hipError_t launch_scan_finite(hipStream_t s, const float* A, int64_t rows, int cols, int64_t ld,
                              unsigned long long* out, int num_cus) {
  int64_t blocks = (rows * (int64_t)cols + 255) / 256;
  if (blocks > (int64_t)num_cus * 8) blocks = (int64_t)num_cus * 8;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(scan_finite_kernel, dim3((unsigned)blocks), dim3(256), 0, s, A, rows, cols,
                     ld, out);
  return hipGetLastError();
}

// Clears the center maxima and the per-assignment counters; with reset_iter
// also the loop state (done, iter, changed).
__global__ void reset_small_kernel(CenterStats* cs, CenterStats* cs2, CenterStats* cs3,
                                   LoopState* st, int reset_iter) {
  if (threadIdx.x == 0) {
    if (cs3) { cs3->cq_max = 0; cs3->rc_max = 0; cs3->cn_max = 0; cs3->O = 0.0f; cs3->c_amax = 0; cs3->c_exp = 127; }
    if (cs) { cs->cq_max = 0; cs->rc_max = 0; cs->cn_max = 0; cs->O = 0.0f; cs->c_amax = 0; cs->c_exp = 127; }
    if (cs2) { cs2->cq_max = 0; cs2->rc_max = 0; cs2->cn_max = 0; cs2->O = 0.0f; cs2->c_amax = 0; cs2->c_exp = 127; }
    if (st) {
      st->listed_total += st->flagged;
      st->full_total += st->flagged_full;
      st->flagged = 0;
      st->full_count = 0;
      st->full_count2 = 0;
      st->flagged_full = 0;
      st->undecided = 0;
      st->routed_fallback = 0;
      st->routed_listed = 0;
      st->bound_fail = 0;
      st->bound_pair = 0;
      st->dcount = 0;
      st->need_rows = 0;
      if (reset_iter) {
        st->done = 0;
        st->iter = 0;
        st->changed = 0;
      }
    }
  }
}

hipError_t launch_reset_small(hipStream_t s, CenterStats* cs, CenterStats* cs2, CenterStats* cs3,
                              LoopState* st, int reset_iter) {
  hipLaunchKernelGGL(reset_small_kernel, dim3(1), dim3(64), 0, s, cs, cs2, cs3, st, reset_iter);
  return hipGetLastError();
}

}  // namespace kmx
