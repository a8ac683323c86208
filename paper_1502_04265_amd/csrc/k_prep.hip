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
// (round to nearest even) zero-padded to dp elements.
__global__ __launch_bounds__(256) void prep_rows_kernel(const float* __restrict__ X, int64_t n,
                                                        int d, int64_t ldx, int dp,
                                                        uint16_t* __restrict__ Xq,
                                                        RowStats* __restrict__ st) {
  const int lane = threadIdx.x & 63;
  const int64_t wave0 = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t row = wave0; row < n; row += nwaves) {
    const float* x = X + row * ldx;
    double s2 = 0.0, q2 = 0.0, r2 = 0.0;
    const int lim = Xq ? dp : d;
    for (int c = lane; c < lim; c += 64) {
      float v = (c < d) ? x[c] : 0.0f;
      double vd = (double)v;
      s2 += vd * vd;
      if (Xq) {
        uint16_t b = f32_to_bf16_rne(v);
        Xq[row * dp + c] = b;
        double qd = (double)bf16_to_f32(b);
        q2 += qd * qd;
        r2 += (vd - qd) * (vd - qd);
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
    }
  }
}

hipError_t launch_prep_rows(hipStream_t s, const float* X, int64_t n, int d, int64_t ldx,
                            int dp, uint16_t* Xq, RowStats* st, int num_cus) {
  int64_t waves_needed = n;
  int64_t blocks = (waves_needed + 3) / 4;
  int64_t cap = (int64_t)num_cus * 16;
  if (blocks > cap) blocks = cap;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(prep_rows_kernel, dim3((unsigned)blocks), dim3(256), 0, s, X, n, d, ldx,
                     dp, Xq, st);
  return hipGetLastError();
}

// One wave per (padded) center.  prec 0: FP32 copy; prec 1: BF16 copy.
// ch[j] = 0.5 ||c_j||^2 rounded to nearest float (0 for padding rows).
__global__ __launch_bounds__(64) void prep_centers_kernel(const float* __restrict__ C, int k,
                                                          int d, int dp, int prec,
                                                          void* __restrict__ Cq,
                                                          float* __restrict__ ch,
                                                          CenterStats* __restrict__ cs) {
  const int j = blockIdx.x;
  const int lane = threadIdx.x;
  double s2 = 0.0, q2 = 0.0, r2 = 0.0;
  for (int c = lane; c < dp; c += 64) {
    float v = (j < k && c < d) ? C[(int64_t)j * d + c] : 0.0f;
    double vd = (double)v;
    s2 += vd * vd;
    if (prec == 1) {
      uint16_t b = f32_to_bf16_rne(v);
      ((uint16_t*)Cq)[(int64_t)j * dp + c] = b;
      double qd = (double)bf16_to_f32(b);
      q2 += qd * qd;
      r2 += (vd - qd) * (vd - qd);
    } else {
      ((float*)Cq)[(int64_t)j * dp + c] = v;
    }
  }
  s2 = wave_sum_f64(s2);
  q2 = wave_sum_f64(q2);
  r2 = wave_sum_f64(r2);
  if (lane == 0) {
    ch[j] = (float)(0.5 * s2);
    if (j < k) {
      float cn = f64_to_f32_up(sqrt(s2));
      float cq = (prec == 1) ? f64_to_f32_up(sqrt(q2)) : cn;
      float rc = (prec == 1) ? f64_to_f32_up(sqrt(r2)) : 0.0f;
      atomicMax(&cs->cq_max, __float_as_uint(cq));
      atomicMax(&cs->rc_max, __float_as_uint(rc));
      atomicMax(&cs->cn_max, __float_as_uint(cn));
    }
  }
}

hipError_t launch_prep_centers(hipStream_t s, const float* C, int k, int d, int kpad, int dp,
                               int prec, void* Cq, float* ch, CenterStats* cs) {
  hipLaunchKernelGGL(prep_centers_kernel, dim3(kpad), dim3(64), 0, s, C, k, d, dp, prec, Cq,
                     ch, cs);
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

// Clears the center maxima and the per-assignment counters; with reset_iter
// also the loop state (done, iter, changed).
__global__ void reset_small_kernel(CenterStats* cs, unsigned long long* ctr, LoopState* st,
                                   int reset_iter) {
  if (threadIdx.x == 0) {
    if (cs) { cs->cq_max = 0; cs->rc_max = 0; cs->cn_max = 0; cs->pad = 0; }
    if (ctr) { ctr[0] = 0; ctr[1] = 0; }
    if (st) {
      st->flagged = 0;
      st->flagged_full = 0;
      if (reset_iter) {
        st->done = 0;
        st->iter = 0;
        st->changed = 0;
      }
    }
  }
}

hipError_t launch_reset_small(hipStream_t s, CenterStats* cs, unsigned long long* ctr,
                              LoopState* st, int reset_iter) {
  hipLaunchKernelGGL(reset_small_kernel, dim3(1), dim3(64), 0, s, cs, ctr, st, reset_iter);
  return hipGetLastError();
}

}  // namespace kmx
