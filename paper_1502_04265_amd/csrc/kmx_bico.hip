// BICO summary on the host (bico_core.h: Sec. 2.1 clustering features in a
// tree of spheres, Sec. 2.3.1 weighted insertion), with the part the paper
// names as dominating insertion -- finding the closest reference point among
// the features of the first tree level -- offloaded to the device in blocks
// of points through the assignment step's distance GEMM with fused argmin.
//
// For a block of points, the device returns the closest reference among the
// first-level features that existed when the block started (FP32 distance
// GEMM, exact argmin) with the two smallest distances; bico_core.h re-measures
// that choice in FP64, scans the first-level features opened since, and scans
// all of them in FP64 when the two device distances are too near to order, so
// every decision is the one a sequential FP64 implementation takes.  A
// rebuild ends the block; the next block queries the new tree.  Rebuilds send
// their first-level searches to the device in blocks of 256 features.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "bico_core.h"
#include "host_util.h"
#include "kmx_internal.h"

using namespace kmx;
using namespace kmx::host;

struct kmx_bico {
  bico::Core core;
  int64_t gpu_rows = 0;
  // first-level references on the device (rows in roots order)
  Buf dref;
  int64_t dref_rows = 0;
  int64_t dref_rebuilds = -1;   // rebuild count at the last upload
  Buf dlab, dd1, dd2, dq;       // query results and a staging block
  int64_t block = 1024;         // points per device query (adapted)
};

namespace {

constexpr int64_t kBicoMinBlock = 64, kBicoMaxBlock = 8192;
constexpr int64_t kRebuildBlock = 256;

// Device query: closest first-level reference for rows [0, nq) of Q (device,
// leading dimension ldq) among roots[0, u); hints to the host.
kmx_status query(kmx_ctx* ctx, kmx_bico* b, const float* Q, int64_t nq, int64_t ldq, size_t u,
                 bico::Hint* hints) {
  bico::Core& c = b->core;
  const int d = c.d;
  const int64_t nr = (int64_t)u;
  if (b->dref_rebuilds != c.rebuilds || b->dref_rows > nr) b->dref_rows = 0;
  const size_t need = (size_t)std::max<int64_t>(nr, 1) * d * sizeof(float);
  if (b->dref.bytes < need) {
    // a new buffer holds none of the uploaded rows; grow by half again at least
    KMX_TRY(grow(ctx, b->dref, std::max(need, b->dref.bytes + b->dref.bytes / 2)));
    b->dref_rows = 0;
  }
  if (b->dref_rows < nr) {
    // append the references opened since the last upload
    std::vector<float> h((size_t)(nr - b->dref_rows) * d);
    for (int64_t q = b->dref_rows; q < nr; ++q)
      std::memcpy(&h[(size_t)(q - b->dref_rows) * d], &c.ref[(size_t)c.roots[q] * d],
                  (size_t)d * sizeof(float));
    KMX_HIP(ctx, hipMemcpyAsync(P<float>(b->dref) + (size_t)b->dref_rows * d, h.data(),
                                h.size() * sizeof(float), hipMemcpyHostToDevice, ctx->stream));
    KMX_HIP(ctx, hipStreamSynchronize(ctx->stream));
    b->dref_rows = nr;
  }
  b->dref_rebuilds = c.rebuilds;
  KMX_TRY(grow(ctx, b->dlab, (size_t)nq * sizeof(int32_t)));
  KMX_TRY(grow(ctx, b->dd1, (size_t)nq * sizeof(float)));
  KMX_TRY(grow(ctx, b->dd2, (size_t)nq * sizeof(float)));
  KMX_TRY(ensure_assign(ctx, nq, (int)nr));
  // the block's rows change from call to call at the same address: no cached
  // row statistics may survive the query
  ctx->cache_valid = false;
  KMX_TRY(ensure_prep(ctx, Q, nq, d, ldq, KMX_FP32));
  const kmx_status ks = run_assign(ctx, Q, nq, d, ldq, P<float>(b->dref), (int)nr, KMX_FP32,
                                   P<int32_t>(b->dlab), P<float>(b->dd1), P<float>(b->dd2),
                                   nullptr);
  ctx->cache_valid = false;
  KMX_TRY(ks);
  std::vector<int32_t> lab(nq);
  std::vector<float> d1(nq), d2(nq);
  KMX_HIP(ctx, hipMemcpyAsync(lab.data(), b->dlab.p, nq * sizeof(int32_t), hipMemcpyDeviceToHost,
                              ctx->stream));
  KMX_HIP(ctx, hipMemcpyAsync(d1.data(), b->dd1.p, nq * sizeof(float), hipMemcpyDeviceToHost,
                              ctx->stream));
  KMX_HIP(ctx, hipMemcpyAsync(d2.data(), b->dd2.p, nq * sizeof(float), hipMemcpyDeviceToHost,
                              ctx->stream));
  KMX_HIP(ctx, hipStreamSynchronize(ctx->stream));
  for (int64_t q = 0; q < nq; ++q) {
    hints[q].valid = true;
    hints[q].lab = lab[q];
    hints[q].d1 = d1[q];
    hints[q].d2 = d2[q];
    hints[q].u = u;
  }
  b->gpu_rows += nq;
  return KMX_OK;
}

// Rebuild with the first-level searches of each block of features on the device.
kmx_status rebuild(kmx_ctx* ctx, kmx_bico* b) {
  const int d = b->core.d;
  KMX_TRY(grow(ctx, b->dq, (size_t)kRebuildBlock * d * sizeof(float)));
  kmx_status st = KMX_OK;
  const bool ok = bico::rebuild(b->core, kRebuildBlock,
                                [&](const float* refs, int64_t nq, size_t u, bico::Hint* h) {
    const hipError_t e = hipMemcpyAsync(b->dq.p, refs, (size_t)nq * d * sizeof(float),
                                        hipMemcpyHostToDevice, ctx->stream);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      st = fail(ctx, KMX_EDEVICE, std::string("hipMemcpyAsync: ") + hipGetErrorString(e));
      return false;
    }
    st = query(ctx, b, P<float>(b->dq), nq, d, u, h);
    return st == KMX_OK;
  });
  if (!ok) return st != KMX_OK ? st : fail(ctx, KMX_EDEVICE, "rebuild failed");
  return KMX_OK;
}

}  // namespace

extern "C" {

kmx_status kmx_bico_create(kmx_ctx* ctx, int32_t d, int64_t m, double T0, kmx_bico** out) {
  if (!ctx || !out) return KMX_EINVAL;
  ctx->err.clear();
  *out = nullptr;
  if (d < 1) return fail(ctx, KMX_EINVAL, "d must be >= 1");
  if (m < 1) return fail(ctx, KMX_EINVAL, "m must be >= 1");
  if (!(T0 > 0.0) || !std::isfinite(T0))
    return fail(ctx, KMX_EINVAL, "the starting threshold T0 must be positive and finite");
  kmx_bico* b = new kmx_bico();
  b->core.d = d;
  b->core.m = m;
  b->core.T = T0;
  *out = b;
  return KMX_OK;
}

kmx_status kmx_bico_destroy(kmx_ctx* ctx, kmx_bico* b) {
  if (!ctx) return KMX_EINVAL;
  if (!b) return KMX_OK;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  for (Buf* p : {&b->dref, &b->dlab, &b->dd1, &b->dd2, &b->dq})
    if (p->p) (void)hipFree(p->p);
  delete b;
  return KMX_OK;
}

kmx_status kmx_bico_insert(kmx_ctx* ctx, kmx_bico* b, const float* X, int64_t n, int64_t ldx,
                           const float* w) {
  if (!ctx) return KMX_EINVAL;
  ctx->err.clear();
  if (!b) return fail(ctx, KMX_EINVAL, "b is NULL");
  if (!X) return fail(ctx, KMX_EINVAL, "X is NULL");
  bico::Core& c = b->core;
  if (n < 0 || ldx < c.d) return fail(ctx, KMX_EINVAL, "bad n or ldx");
  if (n == 0) return KMX_OK;
  KMX_TRY(set_device(ctx));
  const int d = c.d;
  std::vector<float> hx, hw;
  std::vector<bico::Hint> hints;
  int64_t i0 = 0;
  while (i0 < n) {
    const int64_t nb = std::min(b->block, n - i0);
    hx.resize((size_t)nb * d);
    KMX_HIP(ctx, hipMemcpy2DAsync(hx.data(), (size_t)d * sizeof(float), X + i0 * ldx,
                                  (size_t)ldx * sizeof(float), (size_t)d * sizeof(float),
                                  (size_t)nb, hipMemcpyDeviceToHost, ctx->stream));
    if (w) {
      hw.resize(nb);
      KMX_HIP(ctx, hipMemcpyAsync(hw.data(), w + i0, (size_t)nb * sizeof(float),
                                  hipMemcpyDeviceToHost, ctx->stream));
    }
    KMX_HIP(ctx, hipStreamSynchronize(ctx->stream));
    for (int64_t q = 0; q < nb; ++q) {
      const double wq = w ? (double)hw[q] : 1.0;
      if (!(wq >= 0.0) || !std::isfinite(wq))
        return fail(ctx, KMX_EINVAL, "w holds an entry that is negative or not finite");
    }
    hints.assign(nb, bico::Hint());
    if (!c.roots.empty()) KMX_TRY(query(ctx, b, X + i0 * ldx, nb, ldx, c.roots.size(), hints.data()));
    int64_t done = 0;
    const size_t opened0 = c.f.size();
    bool rebuilt = false;
    for (int64_t q = 0; q < nb; ++q) {
      const float* x = &hx[(size_t)q * d];
      const double wq = w ? (double)hw[q] : 1.0;
      done = q + 1;
      if (wq == 0.0) continue;
      int32_t best;
      double bd;
      bico::first_level(c, x, hints[q], best, bd);
      bico::insert_point(c, x, wq, best, bd);
      if ((int64_t)c.f.size() > c.m) {
        while ((int64_t)c.f.size() > c.m) KMX_TRY(rebuild(ctx, b));
        rebuilt = true;
        break;
      }
    }
    // block size: halve when many first-level features opened (their host
    // scans grow with the block), double when few did
    const size_t opened = c.f.size() >= opened0 ? c.f.size() - opened0 : 0;
    if (!rebuilt) {
      if ((int64_t)opened * 8 > done) b->block = std::max(kBicoMinBlock, b->block / 2);
      else if ((int64_t)opened * 64 < done) b->block = std::min(kBicoMaxBlock, b->block * 2);
    }
    i0 += done;
  }
  return KMX_OK;
}

kmx_status kmx_bico_stats(kmx_ctx* ctx, const kmx_bico* b, int64_t* count, double* T,
                          int64_t* rebuilds, int64_t* gpu_rows, int64_t* host_scans) {
  if (!ctx) return KMX_EINVAL;
  ctx->err.clear();
  if (!b) return fail(ctx, KMX_EINVAL, "b is NULL");
  if (count) *count = (int64_t)b->core.f.size();
  if (T) *T = b->core.T;
  if (rebuilds) *rebuilds = b->core.rebuilds;
  if (gpu_rows) *gpu_rows = b->gpu_rows;
  if (host_scans) *host_scans = b->core.host_scans;
  return KMX_OK;
}

kmx_status kmx_bico_features(kmx_ctx* ctx, const kmx_bico* b, double* W, double* S, double* Q,
                             float* ref, int32_t* level) {
  if (!ctx) return KMX_EINVAL;
  ctx->err.clear();
  if (!b) return fail(ctx, KMX_EINVAL, "b is NULL");
  const bico::Core& c = b->core;
  const int d = c.d;
  const std::vector<int32_t> order = bico::bfs(c);
  for (size_t q = 0; q < order.size(); ++q) {
    const int32_t id = order[q];
    if (W) W[q] = c.f[id].W;
    if (Q) Q[q] = c.f[id].Q;
    if (level) level[q] = c.f[id].level;
    if (S) std::memcpy(S + q * d, &c.S[(size_t)id * d], (size_t)d * sizeof(double));
    if (ref) std::memcpy(ref + q * d, &c.ref[(size_t)id * d], (size_t)d * sizeof(float));
  }
  return KMX_OK;
}

kmx_status kmx_bico_coreset(kmx_ctx* ctx, const kmx_bico* b, float* P_out, float* w_out) {
  if (!ctx) return KMX_EINVAL;
  ctx->err.clear();
  if (!b) return fail(ctx, KMX_EINVAL, "b is NULL");
  if (!P_out || !w_out) return fail(ctx, KMX_EINVAL, "NULL P_out or w_out");
  KMX_TRY(set_device(ctx));
  const bico::Core& c = b->core;
  const int d = c.d;
  const std::vector<int32_t> order = bico::bfs(c);
  std::vector<float> hp(order.size() * (size_t)d), hw(order.size());
  for (size_t q = 0; q < order.size(); ++q) {
    const int32_t id = order[q];
    const double W = c.f[id].W;
    hw[q] = (float)W;
    for (int j = 0; j < d; ++j) hp[q * d + j] = (float)(c.S[(size_t)id * d + j] / W);
  }
  KMX_HIP(ctx, hipMemcpyAsync(P_out, hp.data(), hp.size() * sizeof(float), hipMemcpyHostToDevice,
                              ctx->stream));
  KMX_HIP(ctx, hipMemcpyAsync(w_out, hw.data(), hw.size() * sizeof(float), hipMemcpyHostToDevice,
                              ctx->stream));
  KMX_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return KMX_OK;
}

}  // extern "C"
