// Host side of the candidate router: parameters and their Adam state, the
// training loop, proposals, and the Lloyd loop whose assignment step tries
// the certified proposals before the GEMM (k_router.hip explains the
// certificate; k_train.hip the training step).
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "host_util.h"

using namespace kmx;
using namespace kmx::host;

struct kmx_router {
  int device = 0;
  int d = 0, k = 0, d8 = 0, k8 = 0, kpad = 0;
  int64_t step = 0;                              // Adam steps taken
  Buf W1, b1, W2, b2;                            // FP32 parameters
  Buf mW1, vW1, mb1, vb1, mW2, vW2, mb2, vb2;    // Adam moments
  Buf gW1, gb1, gW2, gb2;                        // gradients of the last step
  Buf W1b, W2b;                                  // BF16 copies: H x d8, k8 x H
  Buf W1a, W2a, b2p;                             // inference layouts
  int r1 = 0;                                    // row length of W1a (elements)
  bool layout_ok = false;
  Buf Xb, yb, part, Hb, dZb, dAb, lossrow, cpart, lossdev;  // training workspace
};

namespace {

constexpr int H = kRouterH;

// SplitMix64 stream and Box-Muller normals for the initial weights.
struct InitRng {
  uint64_t z;
  uint64_t next() {
    z += 0x9E3779B97F4A7C15ull;
    uint64_t x = z;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
  }
  double uniform() { return ((double)(next() >> 11) + 0.5) * 0x1.0p-53; }
  double normal() {
    const double u1 = uniform(), u2 = uniform();
    return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
  }
};

kmx_status check_router(kmx_ctx* ctx, kmx_router* r) {
  if (!r) return fail(ctx, KMX_EINVAL, "router is NULL");
  if (r->device != ctx->device) return fail(ctx, KMX_EINVAL, "router belongs to another device");
  return KMX_OK;
}

// BF16 training copies from the FP32 parameters; clears the Adam state.
kmx_status refresh_copies(kmx_ctx* ctx, kmx_router* r, bool reset_adam) {
  KMX_HIP(ctx, launch_to_bf16_pad(ctx->stream, P<float>(r->W1), H, r->d, H, r->d8,
                                  P<uint16_t>(r->W1b)));
  KMX_HIP(ctx, launch_to_bf16_pad(ctx->stream, P<float>(r->W2), r->k, H, r->k8, H,
                                  P<uint16_t>(r->W2b)));
  if (reset_adam) {
    Buf* m[] = {&r->mW1, &r->vW1, &r->mb1, &r->vb1, &r->mW2, &r->vW2, &r->mb2, &r->vb2};
    for (Buf* b : m) KMX_HIP(ctx, hipMemsetAsync(b->p, 0, b->bytes, ctx->stream));
    r->step = 0;
  }
  r->layout_ok = false;
  return KMX_OK;
}

kmx_status ensure_layout(kmx_ctx* ctx, kmx_router* r, int dp) {
  const int units = router_units(r->d, dp);
  if (units < 0) return fail(ctx, KMX_EUNSUPPORTED, "no router kernel for this d");
  if (r->layout_ok && r->r1 == units * 32) return KMX_OK;
  r->r1 = units * 32;
  KMX_TRY(grow(ctx, r->W1a, (size_t)H * r->r1 * sizeof(uint16_t)));
  KMX_TRY(grow(ctx, r->W2a, (size_t)r->kpad * H * sizeof(uint16_t)));
  KMX_TRY(grow(ctx, r->b2p, (size_t)r->kpad * sizeof(float)));
  KMX_HIP(ctx, launch_router_layout(ctx->stream, P<float>(r->W1), P<float>(r->W2), P<float>(r->b2),
                                    r->d, r->k, r->kpad, r->r1, P<uint16_t>(r->W1a),
                                    P<uint16_t>(r->W2a), P<float>(r->b2p)));
  r->layout_ok = true;
  return KMX_OK;
}

// Workspace for batches of up to bsz rows.
kmx_status ensure_ws(kmx_ctx* ctx, kmx_router* r, int bsz) {
  int kc;
  size_t pmax = (size_t)bsz * r->k8;                                               // Z2
  pmax = std::max(pmax, (size_t)gemm_splits(bsz, H, r->d8, ctx->num_cus, &kc) * bsz * H);  // Z1
  pmax = std::max(pmax, (size_t)gemm_splits(bsz, H, r->k8, ctx->num_cus, &kc) * bsz * H);  // dH
  pmax = std::max(pmax, (size_t)gemm_splits(r->k8, H, bsz, ctx->num_cus, &kc) * r->k8 * H);  // dW2
  pmax = std::max(pmax, (size_t)gemm_splits(H, r->d8, bsz, ctx->num_cus, &kc) * H * r->d8);  // dW1
  KMX_TRY(grow(ctx, r->Xb, (size_t)bsz * r->d8 * sizeof(uint16_t)));
  KMX_TRY(grow(ctx, r->yb, (size_t)bsz * sizeof(int32_t)));
  KMX_TRY(grow(ctx, r->part, pmax * sizeof(float)));
  KMX_TRY(grow(ctx, r->Hb, (size_t)bsz * H * sizeof(uint16_t)));
  KMX_TRY(grow(ctx, r->dZb, (size_t)bsz * r->k8 * sizeof(uint16_t)));
  KMX_TRY(grow(ctx, r->dAb, (size_t)bsz * H * sizeof(uint16_t)));
  KMX_TRY(grow(ctx, r->lossrow, (size_t)bsz * sizeof(float)));
  KMX_TRY(grow(ctx, r->cpart,
               (size_t)colsum_segments(bsz) * std::max(r->k, H) * sizeof(float)));
  return KMX_OK;
}

// Forward and backward pass over the gathered batch (Xb, yb) of bsz rows;
// gradients into gW1..gb2, the mean loss into *loss_slot (device).
kmx_status fwd_bwd(kmx_ctx* ctx, kmx_router* r, int bsz, double* loss_slot) {
  hipStream_t s = ctx->stream;
  float* part = P<float>(r->part);
  const uint16_t* Xb = P<uint16_t>(r->Xb);
  uint16_t* Hb = P<uint16_t>(r->Hb);
  uint16_t* dZb = P<uint16_t>(r->dZb);
  uint16_t* dAb = P<uint16_t>(r->dAb);
  const int d8 = r->d8, k8 = r->k8;
  const size_t cap = r->part.bytes / sizeof(float);
  // split-K factor that also fits the partial-product buffer
  auto splits = [&](int M, int N, int K, int* kc) {
    int sp = gemm_splits(M, N, K, ctx->num_cus, kc);
    while (sp > 1 && (size_t)sp * M * N > cap) {
      --sp;
      *kc = ((K + sp - 1) / sp + 31) / 32 * 32;
      sp = (K + *kc - 1) / *kc;
    }
    return sp;
  };
  int kc;
  // Z1 -> Hb
  int sp = splits(bsz, H, d8, &kc);
  KMX_HIP(ctx, launch_gemm_bf16(s, bsz, H, d8, Xb, d8, false, P<uint16_t>(r->W1b), d8, false, part,
                                sp, kc));
  KMX_HIP(ctx, launch_ep_hidden(s, part, sp, bsz, H, P<float>(r->b1), nullptr, Hb, 0));
  // Z2 -> softmax cross-entropy, dZ
  KMX_HIP(ctx, launch_gemm_bf16(s, bsz, k8, H, Hb, H, false, P<uint16_t>(r->W2b), H, false, part, 1,
                                H));
  KMX_HIP(ctx, launch_softmax_ce(s, part, bsz, r->k, k8, P<float>(r->b2), P<int32_t>(r->yb), dZb,
                                 P<float>(r->lossrow)));
  // dH = dZ W2 -> dA
  sp = splits(bsz, H, k8, &kc);
  KMX_HIP(ctx, launch_gemm_bf16(s, bsz, H, k8, dZb, k8, false, P<uint16_t>(r->W2b), H, true, part,
                                sp, kc));
  KMX_HIP(ctx, launch_ep_hidden(s, part, sp, bsz, H, nullptr, Hb, dAb, 1));
  // dW2 = dZ^T Hb
  sp = splits(k8, H, bsz, &kc);
  KMX_HIP(ctx, launch_gemm_bf16(s, k8, H, bsz, dZb, k8, true, Hb, H, true, part, sp, kc));
  KMX_HIP(ctx, launch_sum_partials(s, part, sp, (int64_t)k8 * H, r->k, H, H, P<float>(r->gW2)));
  // dW1 = dA^T Xb
  sp = splits(H, d8, bsz, &kc);
  KMX_HIP(ctx, launch_gemm_bf16(s, H, d8, bsz, dAb, H, true, Xb, d8, true, part, sp, kc));
  KMX_HIP(ctx, launch_sum_partials(s, part, sp, (int64_t)H * d8, H, r->d, d8, P<float>(r->gW1)));
  // bias gradients, loss
  KMX_HIP(ctx, launch_colsum(s, dZb, bsz, r->k, k8, P<float>(r->cpart), P<float>(r->gb2)));
  KMX_HIP(ctx, launch_colsum(s, dAb, bsz, H, H, P<float>(r->cpart), P<float>(r->gb1)));
  KMX_HIP(ctx, launch_loss_mean(s, P<float>(r->lossrow), bsz, loss_slot));
  return KMX_OK;
}

kmx_status adam_step(kmx_ctx* ctx, kmx_router* r, float lr) {
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  r->step += 1;
  const float bc1 = (float)(1.0 - std::pow(0.9, (double)r->step));
  const float bc2 = (float)(1.0 - std::pow(0.999, (double)r->step));
  hipStream_t s = ctx->stream;
  KMX_HIP(ctx, launch_adam(s, P<float>(r->W1), P<float>(r->gW1), P<float>(r->mW1),
                           P<float>(r->vW1), H, r->d, lr, b1, b2, eps, bc1, bc2,
                           P<uint16_t>(r->W1b), r->d8));
  KMX_HIP(ctx, launch_adam(s, P<float>(r->b1), P<float>(r->gb1), P<float>(r->mb1),
                           P<float>(r->vb1), 1, H, lr, b1, b2, eps, bc1, bc2, nullptr, 0));
  KMX_HIP(ctx, launch_adam(s, P<float>(r->W2), P<float>(r->gW2), P<float>(r->mW2),
                           P<float>(r->vW2), r->k, H, lr, b1, b2, eps, bc1, bc2,
                           P<uint16_t>(r->W2b), H));
  KMX_HIP(ctx, launch_adam(s, P<float>(r->b2), P<float>(r->gb2), P<float>(r->mb2),
                           P<float>(r->vb2), 1, r->k, lr, b1, b2, eps, bc1, bc2, nullptr, 0));
  r->layout_ok = false;
  return KMX_OK;
}

kmx_status check_data(kmx_ctx* ctx, kmx_router* r, const float* X, int64_t n, int32_t d,
                      int64_t ldx) {
  if (!X) return fail(ctx, KMX_EINVAL, "X is NULL");
  if (d != r->d) return fail(ctx, KMX_EINVAL, "d differs from the router's input width");
  if (n < 1 || n > (int64_t)INT32_MAX - 1) return fail(ctx, KMX_EINVAL, "n out of range");
  if (ldx < d) return fail(ctx, KMX_EINVAL, "ldx must be >= d");
  return KMX_OK;
}

// Certificate pass (proposals `keys`, or the current labels when keys is
// null), then the GEMM assignment of the rows it could not certify.
kmx_status routed_assign(kmx_ctx* ctx, const float* X, int64_t n, int d, int64_t ldx,
                         const float* C, int k, int prec, int32_t* lab, const uint32_t* keys,
                         int kpad_r, const int* gate) {
  LoopState* st = ST(ctx);
  const int dp = assign_dpad(KMX_BF16, d);
  {
    Timed tm(ctx, T_CERT);
    KMX_HIP(ctx, launch_center_table(ctx->stream, C, k, d, P<float>(ctx->cdist),
                                     P<int32_t>(ctx->nbr), P<float>(ctx->nbd), gate));
    KMX_HIP(ctx, launch_router_cert(ctx->stream, P<uint16_t>(ctx->xq), dp, n, d, C, k,
                                    P<RowStats>(ctx->rowstats), keys, kpad_r, P<int32_t>(ctx->nbr),
                                    P<float>(ctx->nbd), lab, P<FlagEntry>(ctx->flags),
                                    P<int>(ctx->fb_rows), st, gate, ctx->num_cus));
  }
  return run_assign_gemm(ctx, X, n, d, ldx, C, k, prec, lab, nullptr, nullptr,
                         P<int>(ctx->fb_rows), &st->routed_fallback, gate);
}

}  // namespace

extern "C" {

kmx_status kmx_router_create(kmx_ctx* ctx, int32_t d, int32_t k, uint64_t init_seed,
                             kmx_router** out) {
  if (!ctx) return KMX_EINVAL;
  ctx->err.clear();
  if (!out) return fail(ctx, KMX_EINVAL, "out is NULL");
  *out = nullptr;
  if (d < 1 || d > 1024) return fail(ctx, KMX_EUNSUPPORTED, "router supports 1 <= d <= 1024");
  if (k < 1 || k > kRouterMaxK)
    return fail(ctx, KMX_EUNSUPPORTED, "router supports 1 <= k <= " + std::to_string(kRouterMaxK));
  KMX_TRY(set_device(ctx));
  kmx_router* r = new (std::nothrow) kmx_router();
  if (!r) return fail(ctx, KMX_ENOMEM, "out of host memory");
  r->device = ctx->device;
  r->d = d;
  r->k = k;
  r->d8 = (d + 7) / 8 * 8;
  r->k8 = (k + 7) / 8 * 8;
  r->kpad = (k + kRouterBN2 - 1) / kRouterBN2 * kRouterBN2;
  const size_t w1 = (size_t)H * d, w2 = (size_t)k * H;
  struct { Buf* b; size_t elems; } req[] = {
      {&r->W1, w1},  {&r->mW1, w1}, {&r->vW1, w1}, {&r->gW1, w1},
      {&r->b1, H},   {&r->mb1, H},  {&r->vb1, H},  {&r->gb1, H},
      {&r->W2, w2},  {&r->mW2, w2}, {&r->vW2, w2}, {&r->gW2, w2},
      {&r->b2, (size_t)k}, {&r->mb2, (size_t)k}, {&r->vb2, (size_t)k}, {&r->gb2, (size_t)k}};
  for (auto& q : req) {
    kmx_status st = grow(ctx, *q.b, q.elems * sizeof(float));
    if (st != KMX_OK) {
      kmx_router_destroy(ctx, r);
      return st;
    }
  }
  kmx_status st = grow(ctx, r->W1b, (size_t)H * r->d8 * sizeof(uint16_t));
  if (st == KMX_OK) st = grow(ctx, r->W2b, (size_t)r->k8 * H * sizeof(uint16_t));
  if (st != KMX_OK) {
    kmx_router_destroy(ctx, r);
    return st;
  }
  // He-normal first layer, variance 1/H second layer, zero biases.
  InitRng g{init_seed};
  std::vector<float> hw1(w1), hw2(w2), hb1(H, 0.0f), hb2((size_t)k, 0.0f);
  const double s1 = std::sqrt(2.0 / d), s2 = std::sqrt(1.0 / H);
  for (auto& v : hw1) v = (float)(s1 * g.normal());
  for (auto& v : hw2) v = (float)(s2 * g.normal());
  hipError_t e = hipMemcpy(r->W1.p, hw1.data(), w1 * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(r->W2.p, hw2.data(), w2 * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(r->b1.p, hb1.data(), H * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(r->b2.p, hb2.data(), (size_t)k * sizeof(float), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    kmx_router_destroy(ctx, r);
    return fail(ctx, KMX_EDEVICE, std::string("hipMemcpy: ") + hipGetErrorString(e));
  }
  st = refresh_copies(ctx, r, true);
  if (st != KMX_OK) {
    kmx_router_destroy(ctx, r);
    return st;
  }
  *out = r;
  return KMX_OK;
}

kmx_status kmx_router_destroy(kmx_ctx* ctx, kmx_router* r) {
  if (!r) return KMX_EINVAL;
  if (ctx) {
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
  }
  Buf* all[] = {&r->W1,  &r->b1,  &r->W2,  &r->b2,  &r->mW1, &r->vW1, &r->mb1, &r->vb1,
                &r->mW2, &r->vW2, &r->mb2, &r->vb2, &r->gW1, &r->gb1, &r->gW2, &r->gb2,
                &r->W1b, &r->W2b, &r->W1a, &r->W2a, &r->b2p, &r->Xb,  &r->yb,  &r->part,
                &r->Hb,  &r->dZb, &r->dAb, &r->lossrow, &r->cpart, &r->lossdev};
  for (Buf* b : all)
    if (b->p) (void)hipFree(b->p);
  delete r;
  return KMX_OK;
}

kmx_status kmx_router_set_params(kmx_ctx* ctx, kmx_router* r, const float* W1, const float* b1,
                                 const float* W2, const float* b2) {
  if (!ctx) return KMX_EINVAL;
  ctx->err.clear();
  KMX_TRY(check_router(ctx, r));
  if (!W1 || !b1 || !W2 || !b2) return fail(ctx, KMX_EINVAL, "NULL parameter");
  KMX_TRY(set_device(ctx));
  hipStream_t s = ctx->stream;
  KMX_HIP(ctx, hipMemcpyAsync(r->W1.p, W1, (size_t)H * r->d * 4, hipMemcpyDeviceToDevice, s));
  KMX_HIP(ctx, hipMemcpyAsync(r->b1.p, b1, (size_t)H * 4, hipMemcpyDeviceToDevice, s));
  KMX_HIP(ctx, hipMemcpyAsync(r->W2.p, W2, (size_t)r->k * H * 4, hipMemcpyDeviceToDevice, s));
  KMX_HIP(ctx, hipMemcpyAsync(r->b2.p, b2, (size_t)r->k * 4, hipMemcpyDeviceToDevice, s));
  return refresh_copies(ctx, r, true);
}

kmx_status kmx_router_get_params(kmx_ctx* ctx, kmx_router* r, float* W1, float* b1, float* W2,
                                 float* b2) {
  if (!ctx) return KMX_EINVAL;
  ctx->err.clear();
  KMX_TRY(check_router(ctx, r));
  KMX_TRY(set_device(ctx));
  hipStream_t s = ctx->stream;
  if (W1) KMX_HIP(ctx, hipMemcpyAsync(W1, r->W1.p, (size_t)H * r->d * 4, hipMemcpyDeviceToDevice, s));
  if (b1) KMX_HIP(ctx, hipMemcpyAsync(b1, r->b1.p, (size_t)H * 4, hipMemcpyDeviceToDevice, s));
  if (W2) KMX_HIP(ctx, hipMemcpyAsync(W2, r->W2.p, (size_t)r->k * H * 4, hipMemcpyDeviceToDevice, s));
  if (b2) KMX_HIP(ctx, hipMemcpyAsync(b2, r->b2.p, (size_t)r->k * 4, hipMemcpyDeviceToDevice, s));
  return KMX_OK;
}

kmx_status kmx_router_loss_grad(kmx_ctx* ctx, kmx_router* r, const float* X, int64_t n, int32_t d,
                                int64_t ldx, const int32_t* labels, double* loss, float* dW1,
                                float* db1, float* dW2, float* db2) {
  if (!ctx) return KMX_EINVAL;
  ctx->err.clear();
  KMX_TRY(check_router(ctx, r));
  KMX_TRY(check_data(ctx, r, X, n, d, ldx));
  if (!labels) return fail(ctx, KMX_EINVAL, "labels is NULL");
  if (n > kRouterMaxBatch)
    return fail(ctx, KMX_EINVAL, "n above the largest batch " + std::to_string(kRouterMaxBatch));
  KMX_TRY(set_device(ctx));
  const int bsz = (int)n;
  KMX_TRY(ensure_ws(ctx, r, bsz));
  KMX_TRY(grow(ctx, r->lossdev, sizeof(double)));
  hipStream_t s = ctx->stream;
  KMX_HIP(ctx, launch_gather_batch(s, X, n, d, ldx, labels, (uint64_t)n, 0, bsz, r->d8, 0, 0,
                                   r->k, P<uint16_t>(r->Xb), P<int32_t>(r->yb)));
  KMX_TRY(fwd_bwd(ctx, r, bsz, P<double>(r->lossdev)));
  if (dW1) KMX_HIP(ctx, hipMemcpyAsync(dW1, r->gW1.p, (size_t)H * d * 4, hipMemcpyDeviceToDevice, s));
  if (db1) KMX_HIP(ctx, hipMemcpyAsync(db1, r->gb1.p, (size_t)H * 4, hipMemcpyDeviceToDevice, s));
  if (dW2) KMX_HIP(ctx, hipMemcpyAsync(dW2, r->gW2.p, (size_t)r->k * H * 4, hipMemcpyDeviceToDevice, s));
  if (db2) KMX_HIP(ctx, hipMemcpyAsync(db2, r->gb2.p, (size_t)r->k * 4, hipMemcpyDeviceToDevice, s));
  if (loss) {
    KMX_HIP(ctx, hipMemcpyAsync(loss, r->lossdev.p, sizeof(double), hipMemcpyDeviceToHost, s));
    KMX_HIP(ctx, hipStreamSynchronize(s));
  }
  return KMX_OK;
}

kmx_status kmx_router_train(kmx_ctx* ctx, kmx_router* r, const float* X, int64_t n, int32_t d,
                            int64_t ldx, const int32_t* labels, int32_t n_sets, int32_t epochs,
                            int32_t batch, float lr, uint64_t shuffle_seed, double* loss_hist,
                            int64_t* steps_done) {
  if (!ctx) return KMX_EINVAL;
  ctx->err.clear();
  KMX_TRY(check_router(ctx, r));
  KMX_TRY(check_data(ctx, r, X, n, d, ldx));
  if (!labels) return fail(ctx, KMX_EINVAL, "labels is NULL");
  if (n_sets < 1 || epochs < 0) return fail(ctx, KMX_EINVAL, "n_sets >= 1 and epochs >= 0 required");
  if (batch < 1 || batch > kRouterMaxBatch)
    return fail(ctx, KMX_EINVAL, "batch must lie in [1, " + std::to_string(kRouterMaxBatch) + "]");
  if (!(lr > 0.0f) || !std::isfinite(lr)) return fail(ctx, KMX_EINVAL, "lr must be positive");
  KMX_TRY(set_device(ctx));
  const uint64_t total = (uint64_t)n * (uint64_t)n_sets;
  const int bsz_max = (int)std::min<uint64_t>((uint64_t)batch, total);
  const int64_t per_epoch = (int64_t)((total + (uint64_t)batch - 1) / (uint64_t)batch);
  const int64_t steps = per_epoch * epochs;
  KMX_TRY(ensure_ws(ctx, r, bsz_max));
  KMX_TRY(grow(ctx, r->lossdev, (size_t)std::max<int64_t>(steps, 1) * sizeof(double)));
  hipStream_t s = ctx->stream;
  {
    Timed tm(ctx, T_TRAIN);
    int64_t t = 0;
    for (int ep = 0; ep < epochs; ++ep) {
      const uint64_t key = shuffle_seed + (uint64_t)ep * 0xD1B54A32D192ED03ull;
      for (int64_t b = 0; b < per_epoch; ++b, ++t) {
        const int64_t first = b * (int64_t)batch;
        const int bsz = (int)std::min<uint64_t>((uint64_t)batch, total - (uint64_t)first);
        KMX_HIP(ctx, launch_gather_batch(s, X, n, d, ldx, labels, total, first, bsz, r->d8,
                                         shuffle_seed != 0, key, r->k, P<uint16_t>(r->Xb),
                                         P<int32_t>(r->yb)));
        KMX_TRY(fwd_bwd(ctx, r, bsz, P<double>(r->lossdev) + t));
        KMX_TRY(adam_step(ctx, r, lr));
      }
    }
  }
  if (loss_hist && steps > 0) {
    KMX_HIP(ctx, hipMemcpyAsync(loss_hist, r->lossdev.p, (size_t)steps * sizeof(double),
                                hipMemcpyDeviceToHost, s));
  }
  KMX_HIP(ctx, hipStreamSynchronize(s));
  if (steps_done) *steps_done = steps;
  return KMX_OK;
}

kmx_status kmx_router_propose(kmx_ctx* ctx, kmx_router* r, const float* X, int64_t n, int32_t d,
                              int64_t ldx, int32_t* cand_out) {
  if (!ctx) return KMX_EINVAL;
  ctx->err.clear();
  KMX_TRY(check_router(ctx, r));
  KMX_TRY(check_data(ctx, r, X, n, d, ldx));
  if (!cand_out) return fail(ctx, KMX_EINVAL, "cand_out is NULL");
  KMX_TRY(set_device(ctx));
  KMX_TRY(ensure_prep(ctx, X, n, d, ldx, KMX_BF16));
  const int dp = assign_dpad(KMX_BF16, d);
  KMX_TRY(ensure_layout(ctx, r, dp));
  KMX_TRY(grow(ctx, ctx->keys, (size_t)n * kRouterM * sizeof(uint32_t)));
  {
    Timed tm(ctx, T_ROUTER);
    KMX_HIP(ctx, launch_router_fwd(ctx->stream, P<uint16_t>(ctx->xq), dp, n, d,
                                   P<uint16_t>(r->W1a), P<float>(r->b1), P<uint16_t>(r->W2a),
                                   P<float>(r->b2p), r->kpad, P<uint32_t>(ctx->keys), nullptr,
                                   ctx->num_cus));
  }
  KMX_HIP(ctx, launch_router_decode(ctx->stream, P<uint32_t>(ctx->keys), n * kRouterM, r->k,
                                    r->kpad, cand_out));
  return KMX_OK;
}

kmx_status kmx_center_bounds(kmx_ctx* ctx, const float* C, int32_t k, int32_t d, float* D_out) {
  if (!ctx) return KMX_EINVAL;
  ctx->err.clear();
  if (!C || !D_out) return fail(ctx, KMX_EINVAL, "NULL C or D_out");
  if (k < 1 || k > kRouterMaxK)
    return fail(ctx, KMX_EINVAL, "k must lie in [1, " + std::to_string(kRouterMaxK) + "]");
  if (d < 1) return fail(ctx, KMX_EINVAL, "d must be >= 1");
  KMX_TRY(set_device(ctx));
  KMX_TRY(grow(ctx, ctx->nbr, (size_t)k * kNbrL * sizeof(int32_t)));
  KMX_TRY(grow(ctx, ctx->nbd, (size_t)k * (kNbrL + 1) * sizeof(float)));
  Timed tm(ctx, T_CERT);
  KMX_HIP(ctx, launch_center_table(ctx->stream, C, k, d, D_out, P<int32_t>(ctx->nbr),
                                   P<float>(ctx->nbd), nullptr));
  return KMX_OK;
}

// The routed Lloyd loop; with `bounded` the assignment first applies the
// carried bounds (k_bounds.hip) and only the rows they cannot keep go to the
// certificate and the GEMM.
static kmx_status lloyd_routed_impl(kmx_ctx* ctx, kmx_router* r, const float* X, int64_t n,
                                    int32_t d, int64_t ldx, const float* w, float* C_inout,
                                    int32_t k, int32_t max_iter, double tol, kmx_prec prec,
                                    int32_t* label_out, double* cost_hist, int32_t* iters_done,
                                    int64_t* gemm_rows, int bounded, int64_t* kept_rows) {
  if (!ctx) return KMX_EINVAL;
  ctx->err.clear();
  KMX_TRY(check_problem(ctx, X, n, d, ldx, k));
  KMX_TRY(check_prec(ctx, prec, d));
  if (r) {
    KMX_TRY(check_router(ctx, r));
    if (r->d != d || r->k != k) return fail(ctx, KMX_EINVAL, "router shape differs from (d, k)");
  }
  if (k > kRouterMaxK)
    return fail(ctx, KMX_EUNSUPPORTED, "routed assignment supports k <= " + std::to_string(kRouterMaxK));
  if (!C_inout || !cost_hist || !iters_done)
    return fail(ctx, KMX_EINVAL, "NULL C_inout, cost_hist or iters_done");
  if (max_iter < 0) return fail(ctx, KMX_EINVAL, "max_iter must be >= 0");
  KMX_TRY(set_device(ctx));
  KMX_TRY(check_data(ctx, X, n, d, ldx, w, 0, C_inout, k));
  KMX_TRY(ensure_common(ctx, n, d, k));
  KMX_TRY(ensure_prep(ctx, X, n, d, ldx, KMX_BF16));   // the certificate reads the BF16 rows
  if (prec == KMX_FP8E4M3) KMX_TRY(ensure_prep(ctx, X, n, d, ldx, KMX_FP8E4M3));
  KMX_TRY(grow(ctx, ctx->lab_prev, (size_t)n * sizeof(int32_t)));
  KMX_TRY(grow(ctx, ctx->hist, (size_t)(max_iter + 1) * sizeof(double)));
  KMX_TRY(grow(ctx, ctx->fb_rows, (size_t)n * sizeof(int)));
  KMX_TRY(grow(ctx, ctx->cdist, (size_t)k * k * sizeof(float)));
  KMX_TRY(grow(ctx, ctx->nbr, (size_t)k * kNbrL * sizeof(int32_t)));
  KMX_TRY(grow(ctx, ctx->nbd, (size_t)k * (kNbrL + 1) * sizeof(float)));
  KMX_TRY(grow(ctx, ctx->fbh, (size_t)(max_iter + 1) * sizeof(int64_t)));
  BoundsOut bo;
  if (bounded) {
    KMX_TRY(grow(ctx, ctx->hub, (size_t)n * sizeof(float)));
    KMX_TRY(grow(ctx, ctx->hlb, (size_t)n * sizeof(float)));
    KMX_TRY(grow(ctx, ctx->hl2, (size_t)n * sizeof(float)));
    KMX_TRY(grow(ctx, ctx->hsec, (size_t)n * sizeof(int)));
    KMX_TRY(grow(ctx, ctx->bl_rows, (size_t)n * sizeof(int)));
    KMX_TRY(grow(ctx, ctx->cprev, (size_t)k * d * sizeof(float)));
    KMX_TRY(grow(ctx, ctx->drift, (size_t)k * sizeof(float)));
    KMX_TRY(grow(ctx, ctx->dstat, sizeof(DriftStat)));
    KMX_TRY(grow(ctx, ctx->bkh, (size_t)(max_iter + 1) * sizeof(int64_t)));
    bo.ub = P<float>(ctx->hub);
    bo.lb = P<float>(ctx->hlb);
    bo.l2 = P<float>(ctx->hl2);
    bo.sec = P<int>(ctx->hsec);
  }
  const int dp = assign_dpad(KMX_BF16, d);
  const uint32_t* keys = nullptr;
  int kpad_r = (k + kRouterBN2 - 1) / kRouterBN2 * kRouterBN2;
  if (r) {
    KMX_TRY(ensure_layout(ctx, r, dp));
    KMX_TRY(grow(ctx, ctx->keys, (size_t)n * kRouterM * sizeof(uint32_t)));
    kpad_r = r->kpad;
  }
  KMX_TRY(ensure_cf(ctx, X, n, d, ldx, w));
  KMX_TRY(write_state(ctx, max_iter, tol));
  int32_t* lab = label_out ? label_out : P<int32_t>(ctx->lab_a);
  int32_t* prev = P<int32_t>(ctx->lab_prev);
  double* hist = P<double>(ctx->hist);
  int64_t* fbh = P<int64_t>(ctx->fbh);
  int64_t* bkh = bounded ? P<int64_t>(ctx->bkh) : nullptr;
  LoopState* st = ST(ctx);
  KMX_TRY(begin_lloyd(ctx, prev, n));
  if (r && !bounded) {
    // the proposals depend on the points only: one forward pass serves every iteration
    Timed tm(ctx, T_ROUTER);
    KMX_HIP(ctx, launch_router_fwd(ctx->stream, P<uint16_t>(ctx->xq), dp, n, d,
                                   P<uint16_t>(r->W1a), P<float>(r->b1), P<uint16_t>(r->W2a),
                                   P<float>(r->b2p), r->kpad, P<uint32_t>(ctx->keys), nullptr,
                                   ctx->num_cus));
  }
  if (r && bounded) {
    // with carried bounds only the rows the bounds cannot keep need proposals:
    // each row's are computed the first time it needs them and kept for the run
    KMX_TRY(grow(ctx, ctx->prop_have, (size_t)n));
    KMX_TRY(grow(ctx, ctx->prop_rows, (size_t)n * sizeof(int)));
    KMX_HIP(ctx, launch_fill_u8(ctx->stream, P<uint8_t>(ctx->prop_have), n, 0));
  }
  if (r) keys = P<uint32_t>(ctx->keys);
  // one assignment of iteration t (t == max_iter: the final one); gate: the stop flag
  auto assign_step = [&](int t, const int* gate) -> kmx_status {
    KMX_TRY(run_prep_centers(ctx, C_inout, k, d, prec));
    if (bounded && t > 0) {
      {
        Timed tm(ctx, T_BOUND);
        KMX_HIP(ctx, launch_bounds_test(ctx->stream, n, lab, bo, P<float>(ctx->drift),
                                        P<DriftStat>(ctx->dstat), k, P<int>(ctx->bl_rows),
                                        P<FlagEntry>(ctx->flags), st, gate, ctx->num_cus));
      }
      if (r) {
        Timed tm(ctx, T_ROUTER);
        KMX_HIP(ctx, launch_need_proposals(ctx->stream, P<int>(ctx->bl_rows), &st->bound_fail, n,
                                           P<uint8_t>(ctx->prop_have), P<int>(ctx->prop_rows),
                                           &st->need_rows, gate, ctx->num_cus));
        KMX_HIP(ctx, launch_router_fwd(ctx->stream, P<uint16_t>(ctx->xq), dp, n, d,
                                       P<uint16_t>(r->W1a), P<float>(r->b1),
                                       P<uint16_t>(r->W2a), P<float>(r->b2p), r->kpad,
                                       P<uint32_t>(ctx->keys), gate, ctx->num_cus,
                                       P<int>(ctx->prop_rows), &st->need_rows));
      }
      {
        Timed tm(ctx, T_CERT);
        KMX_HIP(ctx, launch_center_table(ctx->stream, C_inout, k, d, P<float>(ctx->cdist),
                                         P<int32_t>(ctx->nbr), P<float>(ctx->nbd), gate));
        KMX_HIP(ctx, launch_router_cert(ctx->stream, P<uint16_t>(ctx->xq), dp, n, d, C_inout, k,
                                        P<RowStats>(ctx->rowstats), keys, kpad_r,
                                        P<int32_t>(ctx->nbr), P<float>(ctx->nbd), lab,
                                        P<FlagEntry>(ctx->flags), P<int>(ctx->fb_rows), st, gate,
                                        ctx->num_cus, P<int>(ctx->bl_rows), &st->bound_fail, bo));
      }
      KMX_TRY(run_assign_gemm(ctx, X, n, d, ldx, C_inout, k, prec, lab, nullptr, nullptr,
                              P<int>(ctx->fb_rows), &st->routed_fallback, gate, bo));
      KMX_HIP(ctx, launch_record_fallback(ctx->stream, st, fbh, t, 0, n, gate));
      KMX_HIP(ctx, launch_record_kept(ctx->stream, st, bkh, t, n, gate));
    } else if (bounded || (!r && t == 0)) {
      // the first assignment of a bounded loop (or of the previous-label
      // loop): every row through the GEMM
      KMX_TRY(run_assign_gemm(ctx, X, n, d, ldx, C_inout, k, prec, lab, nullptr, nullptr, nullptr,
                              nullptr, gate, bo));
      KMX_HIP(ctx, launch_record_fallback(ctx->stream, st, fbh, t, 1, n, gate));
      if (bounded) KMX_HIP(ctx, launch_record_kept(ctx->stream, nullptr, bkh, t, 0, gate));
    } else {
      KMX_TRY(routed_assign(ctx, X, n, d, ldx, C_inout, k, prec, lab, keys, kpad_r, gate));
      KMX_HIP(ctx, launch_record_fallback(ctx->stream, st, fbh, t, 0, n, gate));
    }
    return KMX_OK;
  };
  for (int t = 0; t < max_iter; ++t) {
    KMX_TRY(assign_step(t, &st->done));
    // the centers before the update (not after the loop has stopped: then
    // they keep the last centers the bounds were moved from)
    if (bounded)
      KMX_HIP(ctx, launch_copy_f32(ctx->stream, C_inout, P<float>(ctx->cprev), (int64_t)k * d,
                                   &st->done));
    KMX_TRY(run_update(ctx, X, n, d, ldx, w, lab, k, C_inout, C_inout, nullptr, 1, prev, hist, 0,
                       &st->done));
    if (bounded) {
      // not gated: the update that sets the stop flag still moved the centers
      Timed tm(ctx, T_BOUND);
      KMX_HIP(ctx, launch_drift(ctx->stream, P<float>(ctx->cprev), C_inout, k, d,
                                P<float>(ctx->drift), P<DriftStat>(ctx->dstat), nullptr));
    }
  }
  KMX_TRY(assign_step(max_iter, nullptr));
  KMX_TRY(run_update(ctx, X, n, d, ldx, w, lab, k, C_inout, nullptr, nullptr, 0, prev, hist, 1,
                     nullptr));
  LoopState h;
  KMX_HIP(ctx, hipMemcpyAsync(&h, ctx->state.p, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
  KMX_HIP(ctx, hipStreamSynchronize(ctx->stream));
  const int it = h.iter;
  KMX_HIP(ctx, hipMemcpy(cost_hist, hist, (size_t)(it + 1) * sizeof(double), hipMemcpyDeviceToHost));
  auto copy_hist = [&](const int64_t* dev, int64_t* out) -> kmx_status {
    std::vector<int64_t> fb((size_t)max_iter + 1);
    KMX_HIP(ctx, hipMemcpy(fb.data(), dev, (size_t)(max_iter + 1) * sizeof(int64_t),
                           hipMemcpyDeviceToHost));
    for (int t = 0; t < it; ++t) out[t] = fb[t];
    out[it] = fb[max_iter];
    return KMX_OK;
  };
  if (gemm_rows) KMX_TRY(copy_hist(fbh, gemm_rows));
  if (kept_rows && bkh) KMX_TRY(copy_hist(bkh, kept_rows));
  *iters_done = it;
  return KMX_OK;
}

kmx_status kmx_lloyd_routed(kmx_ctx* ctx, kmx_router* r, const float* X, int64_t n, int32_t d,
                            int64_t ldx, const float* w, float* C_inout, int32_t k,
                            int32_t max_iter, double tol, kmx_prec prec, int32_t* label_out,
                            double* cost_hist, int32_t* iters_done, int64_t* gemm_rows) {
  return lloyd_routed_impl(ctx, r, X, n, d, ldx, w, C_inout, k, max_iter, tol, prec, label_out,
                           cost_hist, iters_done, gemm_rows, 0, nullptr);
}

kmx_status kmx_lloyd_bounded(kmx_ctx* ctx, kmx_router* r, const float* X, int64_t n, int32_t d,
                             int64_t ldx, const float* w, float* C_inout, int32_t k,
                             int32_t max_iter, double tol, kmx_prec prec, int32_t* label_out,
                             double* cost_hist, int32_t* iters_done, int64_t* gemm_rows,
                             int64_t* kept_rows) {
  return lloyd_routed_impl(ctx, r, X, n, d, ldx, w, C_inout, k, max_iter, tol, prec, label_out,
                           cost_hist, iters_done, gemm_rows, 1, kept_rows);
}

}  // extern "C"
