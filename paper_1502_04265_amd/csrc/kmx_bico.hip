// BICO summary on the host (bico_core.h: Sec. 2.1 clustering features in a
// tree of spheres, Sec. 2.3.1 weighted insertion), with the part the paper
// names as dominating insertion -- finding the closest reference point among
// the children of a node, of which the first level is the largest -- offloaded
// to the device in blocks of points through the assignment step's distance
// GEMM with fused argmin.
//
// For a block of points, the device returns, for the root and for up to 15
// nodes with at least 32 children, the closest child that existed when the
// block started (FP32 distance GEMM, exact argmin) with the two smallest
// distances; bico_core.h re-measures that choice in FP64, scans the children
// added since, and scans all of them in FP64 when the two device distances are
// too near to order, so every decision is the one a sequential FP64
// implementation takes.  A rebuild ends the block; the next block queries the
// new tree.  Rebuilds send their searches to the device in blocks of 256
// features.  Each node's child references stay on the device between blocks
// and only the children added since are uploaded.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "bico_core.h"
#include "host_util.h"
#include "kmx_internal.h"

using namespace kmx;
using namespace kmx::host;

// Device copy of one node's child references (rows in child order).
struct NodeRefs {
  int32_t node = -2;
  Buf buf;
  int64_t rows = 0;
};

struct kmx_bico {
  bico::Core core;
  int64_t gpu_rows = 0, gpu_queries = 0;
  int64_t pairs = 0;            // (row, reference) distances the device searches computed
  std::vector<NodeRefs> refs;   // cached child lists, valid for one tree
  int64_t refs_rebuilds = -1;   // rebuild count the cache belongs to
  Buf dlab, dd1, dd2, dq;       // query results and a staging block
  int64_t block = 1024;         // points per device query (adapted, 512 to 8192)
};

namespace {

constexpr int64_t kBicoMinBlock = 512, kBicoMaxBlock = 8192;
constexpr int64_t kRebuildBlock = 256;

// The device copy of `node`'s children, uploading what was added since the
// last query (child lists only grow between rebuilds; a rebuild empties the
// cache, a reallocation uploads everything again).
kmx_status node_refs(kmx_ctx* ctx, kmx_bico* b, int32_t node, const float*& dev, int64_t& rows) {
  bico::Core& c = b->core;
  const int d = c.d;
  if (b->refs_rebuilds != c.rebuilds) {
    for (NodeRefs& r : b->refs) {
      r.node = -2;
      r.rows = 0;
    }
    b->refs_rebuilds = c.rebuilds;
  }
  NodeRefs* e = nullptr;
  for (NodeRefs& r : b->refs)
    if (r.node == node) e = &r;
  if (!e)
    for (NodeRefs& r : b->refs)
      if (r.node == -2) {
        e = &r;
        break;
      }
  if (!e) {
    b->refs.emplace_back();
    e = &b->refs.back();
  }
  e->node = node;
  const std::vector<int32_t>& kids = bico::kids_of(c, node);
  const int64_t nr = (int64_t)kids.size();
  const size_t need = (size_t)std::max<int64_t>(nr, 1) * d * sizeof(float);
  if (e->buf.bytes < need) {
    // a new buffer holds none of the uploaded rows; grow by half again at least
    KMX_TRY(grow(ctx, e->buf, std::max(need, e->buf.bytes + e->buf.bytes / 2)));
    e->rows = 0;
  }
  if (e->rows > nr) e->rows = 0;
  if (e->rows < nr) {
    std::vector<float> h((size_t)(nr - e->rows) * d);
    for (int64_t q = e->rows; q < nr; ++q)
      std::memcpy(&h[(size_t)(q - e->rows) * d], &c.ref[(size_t)kids[q] * d],
                  (size_t)d * sizeof(float));
    KMX_HIP(ctx, hipMemcpyAsync(P<float>(e->buf) + (size_t)e->rows * d, h.data(),
                                h.size() * sizeof(float), hipMemcpyHostToDevice, ctx->stream));
    KMX_HIP(ctx, hipStreamSynchronize(ctx->stream));
    e->rows = nr;
  }
  dev = P<float>(e->buf);
  rows = nr;
  return KMX_OK;
}

// Device search hints for rows [0, nq) of Q (device, leading dimension ldq)
// over the child lists of the nodes bico::hint_nodes names: per node, the
// closest child (FP32 distance GEMM with exact argmin) and the two smallest
// distances.
kmx_status query(kmx_ctx* ctx, kmx_bico* b, const float* Q, int64_t nq, int64_t ldq,
                 std::vector<bico::NodeHints>& hints) {
  bico::Core& c = b->core;
  const int d = c.d;
  hints.clear();
  const std::vector<int32_t> nodes = bico::hint_nodes(c);
  if (nodes.empty()) return KMX_OK;
  KMX_TRY(grow(ctx, b->dlab, (size_t)nq * sizeof(int32_t)));
  KMX_TRY(grow(ctx, b->dd1, (size_t)nq * sizeof(float)));
  KMX_TRY(grow(ctx, b->dd2, (size_t)nq * sizeof(float)));
  // the block's rows change from call to call at the same address: no cached
  // row statistics may survive the query
  ctx->cache_valid = false;
  for (int32_t node : nodes) {
    const float* R = nullptr;
    int64_t nr = 0;
    KMX_TRY(node_refs(ctx, b, node, R, nr));
    KMX_TRY(ensure_assign(ctx, nq, (int)nr));
    KMX_TRY(ensure_prep(ctx, Q, nq, d, ldq, KMX_FP32));
    const kmx_status ks = run_assign(ctx, Q, nq, d, ldq, R, (int)nr, KMX_FP32,
                                     P<int32_t>(b->dlab), P<float>(b->dd1), P<float>(b->dd2),
                                     nullptr);
    if (ks != KMX_OK) {
      ctx->cache_valid = false;
      return ks;
    }
    bico::NodeHints h;
    h.node = node;
    h.u = (size_t)nr;
    h.lab.resize(nq);
    h.d1.resize(nq);
    h.d2.resize(nq);
    KMX_HIP(ctx, hipMemcpyAsync(h.lab.data(), b->dlab.p, nq * sizeof(int32_t),
                                hipMemcpyDeviceToHost, ctx->stream));
    KMX_HIP(ctx, hipMemcpyAsync(h.d1.data(), b->dd1.p, nq * sizeof(float), hipMemcpyDeviceToHost,
                                ctx->stream));
    KMX_HIP(ctx, hipMemcpyAsync(h.d2.data(), b->dd2.p, nq * sizeof(float), hipMemcpyDeviceToHost,
                                ctx->stream));
    KMX_HIP(ctx, hipStreamSynchronize(ctx->stream));
    hints.push_back(std::move(h));
    b->gpu_queries++;
    b->pairs += nq * nr;
  }
  ctx->cache_valid = false;
  b->gpu_rows += nq;
  return KMX_OK;
}

// Rebuild with the searches of each block of features on the device.
kmx_status rebuild(kmx_ctx* ctx, kmx_bico* b) {
  const int d = b->core.d;
  KMX_TRY(grow(ctx, b->dq, (size_t)kRebuildBlock * d * sizeof(float)));
  kmx_status st = KMX_OK;
  const bool ok = bico::rebuild(b->core, kRebuildBlock,
                                [&](const float* refs, int64_t nq,
                                    std::vector<bico::NodeHints>& h) {
    const hipError_t e = hipMemcpyAsync(b->dq.p, refs, (size_t)nq * d * sizeof(float),
                                        hipMemcpyHostToDevice, ctx->stream);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      st = fail(ctx, KMX_EDEVICE, std::string("hipMemcpyAsync: ") + hipGetErrorString(e));
      return false;
    }
    st = query(ctx, b, P<float>(b->dq), nq, d, h);
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
  for (Buf* p : {&b->dlab, &b->dd1, &b->dd2, &b->dq})
    if (p->p) (void)hipFree(p->p);
  for (NodeRefs& r : b->refs)
    if (r.buf.p) (void)hipFree(r.buf.p);
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
  std::vector<bico::NodeHints> hints;
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
    KMX_TRY(query(ctx, b, X + i0 * ldx, nb, ldx, hints));
    int64_t done = 0;
    const size_t opened0 = c.f.size();
    bool rebuilt = false;
    for (int64_t q = 0; q < nb; ++q) {
      const float* x = &hx[(size_t)q * d];
      const double wq = w ? (double)hw[q] : 1.0;
      done = q + 1;
      if (wq == 0.0) continue;
      bico::insert_point(c, x, wq, &hints, q);
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
                          int64_t* rebuilds, int64_t* gpu_rows, int64_t* host_scans,
                          int64_t* pairs) {
  if (!ctx) return KMX_EINVAL;
  ctx->err.clear();
  if (!b) return fail(ctx, KMX_EINVAL, "b is NULL");
  if (count) *count = (int64_t)b->core.f.size();
  if (T) *T = b->core.T;
  if (rebuilds) *rebuilds = b->core.rebuilds;
  if (gpu_rows) *gpu_rows = b->gpu_rows;
  if (host_scans) *host_scans = b->core.host_scans;
  if (pairs) *pairs = b->pairs;
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
