// Small kernels of the batched Lloyd loop (many independent instances):
// per-instance statistics reset, center preparation for all instances at
// once, per-instance cost (Sec. 2.1 clustering-feature identity, summed over
// the instance's own centers) and the scatter of labels to the callers'
// arrays.  The assignment itself is assign_batched_kernel (k_assign.hip).
#include "kmx_device.h"
#include "kmx_internal.h"

namespace kmx {

__global__ void batch_reset_kernel(const BatchInst* __restrict__ insts, int ninst,
                                   LoopState* __restrict__ st) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ninst) {
    CenterStats* cs = insts[i].cs;
    cs->cq_max = 0;
    cs->rc_max = 0;
    cs->cn_max = 0;
    cs->O = 0.0f;
    cs->c_amax = 0;
    cs->c_exp = 127;
  }
  if (i == 0) {
    st->flagged = 0;
    st->full_count = 0;
    st->full_count2 = 0;
    st->flagged_full = 0;
    st->undecided = 0;
  }
}

hipError_t launch_batch_reset(hipStream_t s, const BatchInst* insts, int ninst, LoopState* st,
                              unsigned* work_ctr) {
  (void)work_ctr;
  hipLaunchKernelGGL(batch_reset_kernel, dim3((unsigned)((ninst + 255) / 256)), dim3(256), 0, s,
                     insts, ninst, st);
  return hipGetLastError();
}

// Per-bucket delta-update states: the change counts start every iteration
// at zero; init also marks the carried features as not valid (a new call).
__global__ void bucket_states_kernel(LoopState* __restrict__ bst, int nb, int init) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < nb) {
    bst[b].dcount = 0;
    bst[b].changed = 0;
    if (init) bst[b].acc_valid = 0;
  }
}

hipError_t launch_bucket_states(hipStream_t s, LoopState* bst, int nb, int init) {
  hipLaunchKernelGGL(bucket_states_kernel, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, s,
                     bst, nb, init);
  return hipGetLastError();
}

// Pass A, one wave per padded center of any instance (global padded index g,
// instance cinst[g]): BF16 row of the center (zeros for padding), hd[g] =
// ||c||^2 / 2 in FP64, norm maxima of the instance.
__global__ __launch_bounds__(64) void batch_centers_a_kernel(const BatchInst* __restrict__ insts,
                                                             const int* __restrict__ cinst) {
  const int g = blockIdx.x;
  const int lane = threadIdx.x;
  const BatchInst& I = insts[cinst[g]];
  const int j = g - I.hd0;
  const bool real = j < I.k;
  const float* c = I.C + (int64_t)(I.koff + (real ? j : 0)) * I.d;
  uint16_t* q = I.cq + (int64_t)(I.cpad0 + j) * I.dp;
  double s2 = 0.0, q2 = 0.0, r2 = 0.0;
  for (int col = lane; col < I.dp; col += 64) {
    const float v = (real && col < I.d) ? c[col] : 0.0f;
    const uint16_t b = f32_to_bf16_rne(v);
    q[col] = b;
    const double vd = (double)v, qd = (double)bf16_to_f32(b);
    s2 += vd * vd;
    q2 += qd * qd;
    r2 += (vd - qd) * (vd - qd);
  }
  s2 = wave_sum_f64(s2);
  q2 = wave_sum_f64(q2);
  r2 = wave_sum_f64(r2);
  if (lane == 0) {
    I.hd[g] = 0.5 * s2;
    if (real) {
      atomicMax(&I.cs->cq_max, __float_as_uint(f64_to_f32_up(sqrt(q2))));
      atomicMax(&I.cs->rc_max, __float_as_uint(f64_to_f32_up(sqrt(r2))));
      atomicMax(&I.cs->cn_max, __float_as_uint(f64_to_f32_up(sqrt(s2))));
    }
  }
}

// Pass B, one thread per padded center: the instance's score offset O (as for
// a single problem, with the bucket's largest ||x~||) and the accumulator
// start values ch[g] = O - h_j in FP32 (zeros for padding).
__global__ void batch_centers_b_kernel(const BatchInst* __restrict__ insts,
                                       const int* __restrict__ cinst, int npad) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= npad) return;
  const BatchInst& I = insts[cinst[g]];
  const int j = g - I.hd0;
  const float xm = __uint_as_float(*I.xq_max);
  const float cqm = __uint_as_float(I.cs->cq_max);
  const float cnm = __uint_as_float(I.cs->cn_max);
  const float O = (xm * cqm + 0.5f * cnm * cnm) * 1.001f + 1.0f;
  if (j == 0) I.cs->O = O;
  I.ch[g] = (j < I.k) ? (float)((double)O - I.hd[g]) : 0.0f;
}

hipError_t launch_batch_prep_centers(hipStream_t s, const BatchInst* insts, const int* cinst,
                                     int npad) {
  hipLaunchKernelGGL(batch_centers_a_kernel, dim3((unsigned)npad), dim3(64), 0, s, insts, cinst);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(batch_centers_b_kernel, dim3((unsigned)((npad + 255) / 256)), dim3(256), 0,
                     s, insts, cinst, npad);
  return hipGetLastError();
}

// cost[i * stride + iter] = sum over the instance's centers of
// Q_j - 2 c_j.S_j + W_j ||c_j||^2 (termC, global center numbering), summed in
// center order; iter is the device-side count of completed assignments, which
// advances after the sums (a captured iteration replays unchanged).
__global__ __launch_bounds__(256) void batch_cost_kernel(const BatchInst* __restrict__ insts,
                                                         int ninst,
                                                         const double* __restrict__ termC,
                                                         double* __restrict__ cost, int stride,
                                                         LoopState* __restrict__ st,
                                                         int advance) {
  const int it = st->iter;
  for (int i = threadIdx.x; i < ninst; i += blockDim.x) {
    const BatchInst& I = insts[i];
    double c = 0.0;
    for (int j = 0; j < I.k; ++j) c += termC[I.kg0 + j];
    if (it < stride) cost[(int64_t)i * stride + it] = c;
  }
  __syncthreads();
  if (advance && threadIdx.x == 0) st->iter = it + 1;
}

hipError_t launch_batch_cost(hipStream_t s, const BatchInst* insts, int ninst,
                             const double* termC, double* cost, int stride, LoopState* st,
                             int advance) {
  hipLaunchKernelGGL(batch_cost_kernel, dim3(1), dim3(256), 0, s, insts, ninst, termC, cost,
                     stride, st, advance);
  return hipGetLastError();
}

__global__ void batch_labels_kernel(const int32_t* __restrict__ glabel, int64_t grow0, int n,
                                    int koff, int32_t* __restrict__ out) {
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x)
    out[r] = glabel[grow0 + r] - koff;
}

hipError_t launch_batch_labels(hipStream_t s, const int32_t* glabel, int64_t grow0, int n,
                               int koff, int32_t* out) {
  int blocks = (n + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(batch_labels_kernel, dim3((unsigned)blocks), dim3(256), 0, s, glabel, grow0,
                     n, koff, out);
  return hipGetLastError();
}

}  // namespace kmx
