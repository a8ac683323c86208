// Host side of the batched Lloyd loop: many independent weighted instances
// (Sec. 2.2 runs k-means++ and Lloyd on weighted summaries; here many such
// problems at once).  Instances of equal d form a bucket whose rows, centers
// and labels are concatenated; one persistent launch per width group assigns
// every instance of that group, the FP64 update runs per bucket, and one
// iteration is captured as a HIP graph and replayed.  The tile shape of each (d, k class)
// comes from the autotuner (kmx_batched_autotune) or the default shape.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "host_util.h"

using namespace kmx;
using namespace kmx::host;

namespace {

int kclass_of(int k) { return k <= 24 ? 0 : (k <= 96 ? 1 : 2); }

struct BucketPlan {
  int d = 0, dp = 0, K = 0, P = 0;
  int64_t n = 0, grow0 = 0;
  int64_t xoff = 0, xqoff = 0, coff = 0, cqoff = 0;   // offsets (elements) into bX, bXq, bC, bCq
  int kg0 = 0;
  int64_t acc_off = 0;                               // carried features (int64) of the bucket
  std::vector<int> members;                          // internal instance indices
};

// Widest row of the batched path: the stride of the per-bucket feature grids.
constexpr int kBatchCfD = 512;

struct Plan {
  std::vector<BatchInst> insts;   // internal order: bucket by bucket
  std::vector<int> user_of;       // internal -> caller's index
  std::vector<BatchItem> items;
  std::vector<BatchBucket> buckets;
  std::vector<int> cinst;         // padded center -> internal instance
  std::vector<BucketPlan> bk;
  int64_t N = 0, xsz = 0, xqsz = 0, csz = 0, cqsz = 0;
  int Ktot = 0, Ptot = 0;
  int64_t max_sort_counts = 0, max_n = 0, max_chunks_d = 0, max_chunks = 0;
  int64_t acc_tot = 0;                                // int64 values of all buckets' features
  int max_K = 0;
  int gbegin[7] = {0, 0, 0, 0, 0, 0, 0};   // items of width group g: [gbegin[g], gbegin[g+1])
};

kmx_status check_problems(kmx_ctx* ctx, const kmx_problem* probs, int count) {
  if (!probs || count < 1) return fail(ctx, KMX_EINVAL, "no problems");
  for (int i = 0; i < count; ++i) {
    const kmx_problem& q = probs[i];
    const std::string at = " (problem " + std::to_string(i) + ")";
    if (!q.X || !q.C) return fail(ctx, KMX_EINVAL, "NULL X or C" + at);
    if (q.n < 1 || q.n > (int64_t)INT32_MAX / 4) return fail(ctx, KMX_EINVAL, "n out of range" + at);
    if (q.d < 1 || q.ldx < q.d) return fail(ctx, KMX_EINVAL, "bad d or ldx" + at);
    if (q.k < 1 || (int64_t)q.k > q.n) return fail(ctx, KMX_EINVAL, "k must lie in [1, n]" + at);
    if (q.d > 512 || batched_variants(q.d) == 0)
      return fail(ctx, KMX_EUNSUPPORTED, "batched assignment supports d <= 512" + at);
    if (q.k > kMaxK) return fail(ctx, KMX_EUNSUPPORTED, "k too large" + at);
  }
  return KMX_OK;
}

// Data checks of every problem (weights finite and >= 0; with KMX_VALIDATE,
// X and C finite): all launched, then one synchronization.
kmx_status check_problem_data(kmx_ctx* ctx, const kmx_problem* probs, int count) {
  bool any = ctx->validate;
  for (int i = 0; i < count && !any; ++i) any = probs[i].w != nullptr;
  if (!any) return KMX_OK;
  KMX_TRY(grow(ctx, ctx->vcheck, (size_t)count * 6 * sizeof(unsigned long long)));
  unsigned long long* v = P<unsigned long long>(ctx->vcheck);
  KMX_HIP(ctx, launch_fill_i32(ctx->stream, P<int32_t>(ctx->vcheck), (int64_t)count * 12, 0));
  for (int i = 0; i < count; ++i) {
    const kmx_problem& q = probs[i];
    if (q.w) KMX_HIP(ctx, launch_check_weights(ctx->stream, q.w, q.n, v + 6 * i, ctx->num_cus));
    if (ctx->validate) {
      KMX_HIP(ctx, launch_scan_finite(ctx->stream, q.X, q.n, q.d, q.ldx, v + 6 * i + 2,
                                      ctx->num_cus));
      KMX_HIP(ctx, launch_scan_finite(ctx->stream, q.C, q.k, q.d, q.d, v + 6 * i + 4,
                                      ctx->num_cus));
    }
  }
  std::vector<unsigned long long> h((size_t)count * 6);
  KMX_HIP(ctx, hipMemcpyAsync(h.data(), v, h.size() * sizeof(unsigned long long),
                              hipMemcpyDeviceToHost, ctx->stream));
  KMX_HIP(ctx, hipStreamSynchronize(ctx->stream));
  for (int i = 0; i < count; ++i) {
    const std::string at = " (problem " + std::to_string(i) + ")";
    if (h[6 * i + 1] != 0)
      return fail(ctx, KMX_EINVAL, "w holds " + std::to_string(h[6 * i + 1]) +
                                       " entries that are negative or not finite" + at);
    if (h[6 * i + 3] != 0 || h[6 * i + 5] != 0)
      return fail(ctx, KMX_EINVAL, "X or C holds entries that are not finite (KMX_VALIDATE)" + at);
  }
  return KMX_OK;
}

int variant_for(const kmx_ctx* ctx, int d, int k) {
  auto it = ctx->tune.find({d, kclass_of(k)});
  return it == ctx->tune.end() ? 0 : it->second;
}

// Buckets (by d, split so that a bucket's centers fit the label histograms),
// offsets, items ordered by decreasing cost.  subset: caller indices to use
// (all when empty); force_variant >= 0 overrides the tuned shapes.
void build_plan(const kmx_ctx* ctx, const kmx_problem* probs, int count,
                const std::vector<int>& subset, int force_variant, Plan& pl) {
  std::vector<int> ids = subset;
  if (ids.empty())
    for (int i = 0; i < count; ++i) ids.push_back(i);
  std::stable_sort(ids.begin(), ids.end(), [&](int a, int b) { return probs[a].d < probs[b].d; });
  pl = Plan();
  for (size_t s = 0; s < ids.size();) {
    const int d = probs[ids[s]].d;
    size_t e = s;
    while (e < ids.size() && probs[ids[e]].d == d) ++e;
    // split the run [s, e) into buckets of at most kMaxK centers
    size_t a = s;
    while (a < e) {
      BucketPlan B;
      B.d = d;
      B.dp = batched_dpad(d);
      B.grow0 = pl.N;
      B.xoff = pl.xsz;
      B.xqoff = pl.xqsz;
      B.coff = pl.csz;
      B.cqoff = pl.cqsz;
      B.kg0 = pl.Ktot;
      size_t b = a;
      while (b < e && B.K + probs[ids[b]].k <= kMaxK) {
        const kmx_problem& q = probs[ids[b]];
        const int v = force_variant >= 0 ? force_variant : variant_for(ctx, d, q.k);
        const int tile = batched_variant_tile(d, v);
        BatchInst I;
        std::memset(&I, 0, sizeof(I));
        I.row0 = B.n;
        I.grow0 = pl.N + B.n;
        I.n = (int)q.n;
        I.d = d;
        I.dp = B.dp;
        I.k = q.k;
        I.kpad = (q.k + tile - 1) / tile * tile;
        I.koff = B.K;
        I.kg0 = pl.Ktot + B.K;
        I.cpad0 = B.P;
        I.variant = batched_variant_id(d, v);
        int ib = 1;
        while ((1 << ib) < I.kpad) ++ib;
        I.ib = ib;
        I.bucket = (int)pl.bk.size();
        I.hd0 = pl.Ptot + B.P;
        B.members.push_back((int)pl.insts.size());
        const int ppb = batched_variant_ppb(d, v);
        const int nblk = (I.n + ppb - 1) / ppb;
        for (int blk = 0; blk < nblk; ++blk) pl.items.push_back({(int)pl.insts.size(), blk});
        for (int j = 0; j < I.kpad; ++j) pl.cinst.push_back((int)pl.insts.size());
        pl.insts.push_back(I);
        pl.user_of.push_back(ids[b]);
        B.n += q.n;
        B.K += q.k;
        B.P += I.kpad;
        ++b;
      }
      pl.N += B.n;
      pl.Ktot += B.K;
      pl.Ptot += B.P;
      pl.xsz += B.n * B.d;
      pl.xqsz += B.n * B.dp;
      pl.csz += (int64_t)B.K * B.d;
      pl.cqsz += (int64_t)B.P * B.dp;
      const int64_t nb = (B.n + kSortRows - 1) / kSortRows;
      pl.max_sort_counts = std::max(pl.max_sort_counts, nb * B.K);
      pl.max_n = std::max(pl.max_n, B.n);
      const int64_t chunks = (B.n + kReduceRows - 1) / kReduceRows + B.K;
      pl.max_chunks = std::max(pl.max_chunks, chunks);
      pl.max_chunks_d = std::max(pl.max_chunks_d, chunks * B.d);
      pl.max_K = std::max(pl.max_K, B.K);
      B.acc_off = pl.acc_tot;
      pl.acc_tot += (int64_t)B.K * B.d * 2 + 4 * (int64_t)B.K;
      pl.bk.push_back(B);
      a = b;
    }
    s = e;
  }
  // by width group (one launch each), costliest items first within a group;
  // workgroups take them round-robin
  auto group = [&](const BatchItem& it) { return batched_group(pl.insts[it.inst].d); };
  auto cost = [&](const BatchItem& it) {
    const BatchInst& I = pl.insts[it.inst];
    return (double)I.kpad * I.dp;
  };
  std::stable_sort(pl.items.begin(), pl.items.end(), [&](const BatchItem& x, const BatchItem& y) {
    const int gx = group(x), gy = group(y);
    return gx != gy ? gx < gy : cost(x) > cost(y);
  });
  for (int g = 0; g <= 6; ++g) pl.gbegin[g] = (int)pl.items.size();
  for (int i = (int)pl.items.size() - 1; i >= 0; --i) pl.gbegin[group(pl.items[i])] = i;
  for (int g = 5; g >= 0; --g) pl.gbegin[g] = std::min(pl.gbegin[g], pl.gbegin[g + 1]);
}

hipError_t launch_groups(kmx_ctx* ctx, const Plan& pl, hipStream_t s) {
  for (int g = 0; g < 6; ++g) {
    const hipError_t e = launch_assign_batched(
        s, g, P<BatchItem>(ctx->bitems), pl.gbegin[g], pl.gbegin[g + 1], P<BatchInst>(ctx->binsts),
        P<FlagEntry>(ctx->flags), P<int>(ctx->brute), ST(ctx), P<int32_t>(ctx->blab),
        ctx->num_cus);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Allocations, descriptor pointers, copies of the inputs, row preparation.
kmx_status setup(kmx_ctx* ctx, const kmx_problem* probs, Plan& pl, int stride) {
  const int ni = (int)pl.insts.size(), nb = (int)pl.bk.size();
  KMX_TRY(grow(ctx, ctx->bX, (size_t)pl.xsz * sizeof(float)));
  KMX_TRY(grow(ctx, ctx->bXq, (size_t)pl.xqsz * sizeof(uint16_t)));
  KMX_TRY(grow(ctx, ctx->brs, (size_t)pl.N * sizeof(RowStats)));
  KMX_TRY(grow(ctx, ctx->bw, (size_t)pl.N * sizeof(float)));
  KMX_TRY(grow(ctx, ctx->bC, (size_t)pl.csz * sizeof(float)));
  KMX_TRY(grow(ctx, ctx->bCq, (size_t)pl.cqsz * sizeof(uint16_t)));
  KMX_TRY(grow(ctx, ctx->bhd, (size_t)pl.Ptot * sizeof(double)));
  KMX_TRY(grow(ctx, ctx->bch, (size_t)pl.Ptot * sizeof(float)));
  KMX_TRY(grow(ctx, ctx->bcs, (size_t)ni * sizeof(CenterStats)));
  KMX_TRY(grow(ctx, ctx->blab, (size_t)pl.N * sizeof(int32_t)));
  KMX_TRY(grow(ctx, ctx->bitems, pl.items.size() * sizeof(BatchItem)));
  KMX_TRY(grow(ctx, ctx->binsts, (size_t)ni * sizeof(BatchInst)));
  KMX_TRY(grow(ctx, ctx->bbuckets, (size_t)nb * sizeof(BatchBucket)));
  KMX_TRY(grow(ctx, ctx->bcinst, pl.cinst.size() * sizeof(int)));
  KMX_TRY(grow(ctx, ctx->bxstats, (size_t)nb * sizeof(unsigned)));
  KMX_TRY(grow(ctx, ctx->btermC, (size_t)pl.Ktot * sizeof(double)));
  KMX_TRY(grow(ctx, ctx->btermMu, (size_t)pl.Ktot * sizeof(double)));
  KMX_TRY(grow(ctx, ctx->bW, (size_t)pl.Ktot * sizeof(double)));
  KMX_TRY(grow(ctx, ctx->bcost, (size_t)ni * stride * sizeof(double)));
  KMX_TRY(grow(ctx, ctx->flags, (size_t)pl.N * sizeof(FlagEntry)));
  KMX_TRY(grow(ctx, ctx->brute, (size_t)pl.N * sizeof(int)));
  KMX_TRY(grow(ctx, ctx->state, sizeof(LoopState)));
  KMX_TRY(grow(ctx, ctx->counts, (size_t)pl.max_sort_counts * sizeof(int32_t)));
  KMX_TRY(grow(ctx, ctx->segsum, (size_t)kScanSegs * pl.max_K * sizeof(int32_t)));
  KMX_TRY(grow(ctx, ctx->base, (size_t)(pl.max_K + 1) * sizeof(int32_t)));
  KMX_TRY(grow(ctx, ctx->chunk_base, (size_t)(pl.max_K + 1) * sizeof(int32_t)));
  KMX_TRY(grow(ctx, ctx->perm, (size_t)pl.max_n * sizeof(int32_t)));
  KMX_TRY(grow(ctx, ctx->partS, (size_t)pl.max_chunks_d * 2 * sizeof(double)));
  KMX_TRY(grow(ctx, ctx->partWQ, (size_t)pl.max_chunks * 4 * sizeof(double)));
  KMX_TRY(grow(ctx, ctx->bcf_colmax, (size_t)nb * kBatchCfD * sizeof(unsigned)));
  KMX_TRY(grow(ctx, ctx->bcf_q, (size_t)pl.N * sizeof(double)));
  KMX_TRY(grow(ctx, ctx->bcf_qmax, (size_t)nb * sizeof(unsigned long long)));
  KMX_TRY(grow(ctx, ctx->bcf_wmax, (size_t)nb * sizeof(unsigned)));
  KMX_TRY(grow(ctx, ctx->bcfs, (size_t)nb * (2 * kBatchCfD + 4) * sizeof(double)));
  // delta update: per-bucket states, previous labels and carried features;
  // the mark / plan / scatter buffers are shared (the buckets run in order)
  KMX_TRY(grow(ctx, ctx->bstate, (size_t)nb * sizeof(LoopState)));
  KMX_TRY(grow(ctx, ctx->blab_prev, (size_t)pl.N * sizeof(int32_t)));
  KMX_TRY(grow(ctx, ctx->bacc, (size_t)pl.acc_tot * sizeof(long long)));
  KMX_TRY(grow(ctx, ctx->ecount, (size_t)(pl.max_K + 1) * sizeof(int32_t)));
  KMX_TRY(grow(ctx, ctx->ebase, (size_t)(pl.max_K + 1) * sizeof(int32_t)));
  KMX_TRY(grow(ctx, ctx->ecursor, (size_t)(pl.max_K + 1) * sizeof(int32_t)));
  KMX_TRY(grow(ctx, ctx->dchunk, (size_t)(pl.max_K + 1) * sizeof(int32_t)));
  KMX_TRY(grow(ctx, ctx->clist, (size_t)pl.max_n * sizeof(int32_t)));
  KMX_TRY(grow(ctx, ctx->cold, (size_t)pl.max_n * sizeof(int32_t)));
  KMX_TRY(grow(ctx, ctx->dent, (size_t)pl.max_n * sizeof(int32_t)));
  KMX_TRY(grow(ctx, ctx->cfflag, 16));

  float* bX = P<float>(ctx->bX);
  float* bC = P<float>(ctx->bC);
  uint16_t* bXq = P<uint16_t>(ctx->bXq);
  uint16_t* bCq = P<uint16_t>(ctx->bCq);
  unsigned* xst = P<unsigned>(ctx->bxstats);
  pl.buckets.clear();
  for (int b = 0; b < nb; ++b) {
    const BucketPlan& B = pl.bk[b];
    BatchBucket bb;
    bb.grow0 = B.grow0;
    bb.n = B.n;
    bb.d = B.d;
    bb.K = B.K;
    bb.X = bX + B.xoff;
    bb.C = bC + B.coff;
    pl.buckets.push_back(bb);
  }
  for (int i = 0; i < ni; ++i) {
    BatchInst& I = pl.insts[i];
    const BucketPlan& B = pl.bk[I.bucket];
    I.xq = bXq + B.xqoff;
    I.rs = P<RowStats>(ctx->brs) + B.grow0;
    I.cq = bCq + B.cqoff;
    I.hd = P<double>(ctx->bhd);
    I.ch = P<float>(ctx->bch);
    I.cs = P<CenterStats>(ctx->bcs) + i;
    I.X = bX + B.xoff;
    I.C = bC + B.coff;
    I.xq_max = xst + I.bucket;
  }
  // The grouped rows, weights, row statistics and feature grids depend only
  // on the problems' X and w (pointers, sizes; contents as the caller
  // promises until kmx_invalidate) and on the layout: a call with the same
  // key as the previous one reuses them.
  std::vector<int64_t> key;
  key.push_back(ni);
  key.push_back(nb);
  for (int b = 0; b < nb; ++b) {
    const BucketPlan& B = pl.bk[b];
    for (int64_t v : {(int64_t)B.d, (int64_t)B.dp, B.n, B.grow0, B.xoff, B.xqoff}) key.push_back(v);
  }
  for (int i = 0; i < ni; ++i) {
    const BatchInst& I = pl.insts[i];
    const kmx_problem& q = probs[pl.user_of[i]];
    for (int64_t v : {(int64_t)(uintptr_t)q.X, q.n, (int64_t)q.d, q.ldx, (int64_t)(uintptr_t)q.w,
                      (int64_t)I.bucket, I.row0, I.grow0})
      key.push_back(v);
  }
  for (const Buf* b : {&ctx->bX, &ctx->bXq, &ctx->brs, &ctx->bw, &ctx->bxstats, &ctx->bcf_colmax,
                       &ctx->bcf_q, &ctx->bcf_qmax, &ctx->bcf_wmax, &ctx->bcfs})
    key.push_back((int64_t)(uintptr_t)b->p);
  const bool reuse = (key == ctx->batch_key);
  ctx->batch_key.clear();   // set again once the buffers hold these problems
  hipStream_t s = ctx->stream;
  KMX_HIP(ctx, hipMemcpy(ctx->binsts.p, pl.insts.data(), (size_t)ni * sizeof(BatchInst),
                         hipMemcpyHostToDevice));
  KMX_HIP(ctx, hipMemcpy(ctx->bitems.p, pl.items.data(), pl.items.size() * sizeof(BatchItem),
                         hipMemcpyHostToDevice));
  KMX_HIP(ctx, hipMemcpy(ctx->bbuckets.p, pl.buckets.data(), (size_t)nb * sizeof(BatchBucket),
                         hipMemcpyHostToDevice));
  KMX_HIP(ctx, hipMemcpy(ctx->bcinst.p, pl.cinst.data(), pl.cinst.size() * sizeof(int),
                         hipMemcpyHostToDevice));
  for (int i = 0; i < ni; ++i) {
    const BatchInst& I = pl.insts[i];
    const BucketPlan& B = pl.bk[I.bucket];
    const kmx_problem& q = probs[pl.user_of[i]];
    if (!reuse) {
      KMX_HIP(ctx, hipMemcpy2DAsync(bX + B.xoff + I.row0 * I.d, (size_t)I.d * sizeof(float), q.X,
                                    (size_t)q.ldx * sizeof(float), (size_t)I.d * sizeof(float),
                                    (size_t)I.n, hipMemcpyDeviceToDevice, s));
      float* w = P<float>(ctx->bw) + I.grow0;
      if (q.w)
        KMX_HIP(ctx, hipMemcpyAsync(w, q.w, (size_t)I.n * sizeof(float), hipMemcpyDeviceToDevice,
                                    s));
      else
        KMX_HIP(ctx, launch_fill_i32(s, (int32_t*)w, I.n, 0x3F800000));   // 1.0f
    }
    KMX_HIP(ctx, hipMemcpyAsync(bC + B.coff + (int64_t)I.koff * I.d, q.C,
                                (size_t)I.k * I.d * sizeof(float), hipMemcpyDeviceToDevice, s));
  }
  if (!reuse) KMX_HIP(ctx, launch_fill_i32(s, (int32_t*)xst, nb, 0));
  for (int b = 0; b < nb && !reuse; ++b) {
    const BucketPlan& B = pl.bk[b];
    Timed tm(ctx, T_PREP);
    KMX_HIP(ctx, launch_prep_rows(s, bX + B.xoff, B.n, B.d, B.d, B.dp, bXq + B.xqoff,
                                  P<RowStats>(ctx->brs) + B.grow0, xst + b, ctx->num_cus));
    // the bucket's feature grids (one bound for all of its instances)
    unsigned* cm = P<unsigned>(ctx->bcf_colmax) + (int64_t)b * kBatchCfD;
    unsigned long long* qm = P<unsigned long long>(ctx->bcf_qmax) + b;
    KMX_HIP(ctx, launch_cf_prep(s, bX + B.xoff, B.n, B.d, B.d, cm, P<double>(ctx->bcf_q) + B.grow0,
                                qm, ctx->num_cus));
    KMX_HIP(ctx, launch_cf_scales(s, cm, B.d, qm, P<float>(ctx->bw) + B.grow0, B.n,
                                  P<unsigned>(ctx->bcf_wmax) + b,
                                  P<double>(ctx->bcfs) + (int64_t)b * (2 * kBatchCfD + 4),
                                  ctx->num_cus));
  }
  // a new call: no carried features, every previous label unknown
  KMX_HIP(ctx, launch_bucket_states(s, P<LoopState>(ctx->bstate), nb, 1));
  KMX_HIP(ctx, launch_fill_i32(s, P<int32_t>(ctx->blab_prev), pl.N, -1));
  KMX_HIP(ctx, launch_fill_i32(s, P<int32_t>(ctx->ecount), pl.max_K + 1, 0));
  ctx->batch_key = std::move(key);
  return KMX_OK;
}

// One Lloyd iteration of every instance on stream s (kernels only, so it can
// be captured): centers, one assignment launch, re-check, per-bucket update,
// per-instance cost.  write_c = 0: cost of the current centers only.
hipError_t enqueue_iteration(kmx_ctx* ctx, const Plan& pl, hipStream_t s, int write_c,
                             int stride) {
  const int ni = (int)pl.insts.size(), nb = (int)pl.bk.size();
  const BatchInst* insts = P<BatchInst>(ctx->binsts);
  LoopState* st = ST(ctx);
  hipError_t e;
  if ((e = launch_batch_reset(s, insts, ni, st, nullptr)) != hipSuccess) return e;
  if ((e = launch_bucket_states(s, P<LoopState>(ctx->bstate), nb, 0)) != hipSuccess) return e;
  if ((e = launch_batch_prep_centers(s, insts, P<int>(ctx->bcinst), pl.Ptot)) != hipSuccess)
    return e;
  if ((e = launch_groups(ctx, pl, s)) != hipSuccess) return e;
  if ((e = launch_recheck_batched(s, P<BatchBucket>(ctx->bbuckets), nb, insts, ni,
                                  P<int32_t>(ctx->blab), P<FlagEntry>(ctx->flags),
                                  P<int>(ctx->brute), st, pl.N, ctx->num_cus)) != hipSuccess)
    return e;
  // per bucket: the delta plan (the rows whose label changed since the
  // previous update, added to the carried features) or, on the first update
  // of a call or when more than half of the rows changed, the full sort and
  // reduction; both paths are decided on the device (flags), so the captured
  // iteration replays either
  int* flags = P<int>(ctx->cfflag);
  for (int b = 0; b < nb; ++b) {
    const BucketPlan& B = pl.bk[b];
    const int32_t* lab = P<int32_t>(ctx->blab) + B.grow0;
    float* Xb = P<float>(ctx->bX) + B.xoff;
    float* Cb = P<float>(ctx->bC) + B.coff;
    LoopState* bst = P<LoopState>(ctx->bstate) + b;
    const float* wb = P<float>(ctx->bw) + B.grow0;
    const double* qb = P<double>(ctx->bcf_q) + B.grow0;
    if ((e = launch_delta_prepare(s, lab, P<int32_t>(ctx->blab_prev) + B.grow0, B.n, B.K,
                                  P<int32_t>(ctx->ecount), P<int32_t>(ctx->clist),
                                  P<int32_t>(ctx->cold), P<int32_t>(ctx->ebase),
                                  P<int32_t>(ctx->ecursor), P<int32_t>(ctx->dchunk),
                                  P<int32_t>(ctx->dent), flags, bst, ctx->num_cus, nullptr)) !=
        hipSuccess)
      return e;
    if ((e = launch_sort(s, lab, nullptr, B.n, B.K, P<int32_t>(ctx->counts),
                         P<int32_t>(ctx->segsum), P<int32_t>(ctx->base),
                         P<int32_t>(ctx->chunk_base), P<int32_t>(ctx->perm), st, 0, flags)) !=
        hipSuccess)
      return e;
    const double* cfs = P<double>(ctx->bcfs) + (int64_t)b * (2 * kBatchCfD + 4);
    if ((e = launch_reduce(s, Xb, B.n, B.d, B.d, wb, qb, P<int32_t>(ctx->perm),
                           P<int32_t>(ctx->base), P<int32_t>(ctx->chunk_base), B.K, cfs,
                           P<double>(ctx->partS), P<double>(ctx->partWQ), 0, ctx->num_cus,
                           flags)) != hipSuccess)
      return e;
    if ((e = launch_reduce(s, Xb, B.n, B.d, B.d, wb, qb, P<int32_t>(ctx->dent),
                           P<int32_t>(ctx->ebase), P<int32_t>(ctx->dchunk), B.K, cfs,
                           P<double>(ctx->partS), P<double>(ctx->partWQ), 1, ctx->num_cus,
                           flags + 1)) != hipSuccess)
      return e;
    if ((e = launch_finalize(s, P<double>(ctx->partS), P<double>(ctx->partWQ),
                             P<int32_t>(ctx->chunk_base), P<int32_t>(ctx->dchunk), flags + 2,
                             P<long long>(ctx->bacc) + B.acc_off, B.K, B.d, cfs, Cb,
                             write_c ? Cb : nullptr, P<double>(ctx->bW) + B.kg0,
                             P<double>(ctx->btermC) + B.kg0, P<double>(ctx->btermMu) + B.kg0,
                             write_c, bst, nullptr)) != hipSuccess)
      return e;
  }
  return launch_batch_cost(s, insts, ni, P<double>(ctx->btermC), P<double>(ctx->bcost), stride,
                           st, 1);
}

kmx_status ensure_cap_stream(kmx_ctx* ctx) {
  if (!ctx->cap_stream) KMX_HIP(ctx, hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
  return KMX_OK;
}

std::string device_name(kmx_ctx* ctx) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, ctx->device) != hipSuccess) {
    (void)hipGetLastError();
    return "unknown";
  }
  return std::string(prop.gcnArchName) + "/" + std::to_string(prop.multiProcessorCount) + "cu";
}

}  // namespace

extern "C" {

kmx_status kmx_lloyd_batched(kmx_ctx* ctx, const kmx_problem* probs, int32_t count,
                             int32_t iters, kmx_prec prec, double* cost_hist) {
  if (!ctx) return KMX_EINVAL;
  ctx->err.clear();
  KMX_TRY(check_problems(ctx, probs, count));
  if (prec != KMX_BF16) return fail(ctx, KMX_EUNSUPPORTED, "batched Lloyd runs the BF16 GEMM");
  if (iters < 0) return fail(ctx, KMX_EINVAL, "iters must be >= 0");
  if (!cost_hist) return fail(ctx, KMX_EINVAL, "cost_hist is NULL");
  KMX_TRY(set_device(ctx));
  KMX_TRY(check_problem_data(ctx, probs, count));
  Plan pl;
  build_plan(ctx, probs, count, {}, -1, pl);
  const int stride = iters + 1;
  KMX_TRY(setup(ctx, probs, pl, stride));
  KMX_TRY(write_state(ctx, iters, -1.0));
  KMX_TRY(ensure_cap_stream(ctx));
  hipStream_t cs = ctx->cap_stream;
  EventGuard ev;
  KMX_HIP(ctx, hipEventCreateWithFlags(&ev.e, hipEventDisableTiming));
  KMX_HIP(ctx, hipEventRecord(ev.e, ctx->stream));
  KMX_HIP(ctx, hipStreamWaitEvent(cs, ev.e, 0));
  {
    Timed tm(ctx, T_ASSIGN);   // whole batched iterations (timing brackets the replays)
    if (iters > 0) {
      GraphGuard gg;
      KMX_HIP(ctx, hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
      const hipError_t ce = enqueue_iteration(ctx, pl, cs, 1, stride);
      const hipError_t ee = hipStreamEndCapture(cs, &gg.g);
      if (ce != hipSuccess || ee != hipSuccess) {
        (void)hipGetLastError();
        return fail(ctx, KMX_EDEVICE, std::string("capture of the batched iteration failed: ") +
                                          hipGetErrorString(ce != hipSuccess ? ce : ee));
      }
      KMX_HIP(ctx, hipGraphInstantiate(&gg.e, gg.g, nullptr, nullptr, 0));
      for (int t = 0; t < iters; ++t) KMX_HIP(ctx, hipGraphLaunch(gg.e, cs));
      KMX_HIP(ctx, hipStreamSynchronize(cs));
    }
    KMX_HIP(ctx, enqueue_iteration(ctx, pl, cs, 0, stride));
    KMX_HIP(ctx, hipEventRecord(ev.e, cs));
    KMX_HIP(ctx, hipStreamWaitEvent(ctx->stream, ev.e, 0));
  }
  // outputs
  const int ni = (int)pl.insts.size();
  for (int i = 0; i < ni; ++i) {
    const BatchInst& I = pl.insts[i];
    const BucketPlan& B = pl.bk[I.bucket];
    const kmx_problem& q = probs[pl.user_of[i]];
    KMX_HIP(ctx, hipMemcpyAsync(q.C, P<float>(ctx->bC) + B.coff + (int64_t)I.koff * I.d,
                                (size_t)I.k * I.d * sizeof(float), hipMemcpyDeviceToDevice,
                                ctx->stream));
    if (q.label)
      KMX_HIP(ctx, launch_batch_labels(ctx->stream, P<int32_t>(ctx->blab), I.grow0, I.n, I.koff,
                                       q.label));
  }
  std::vector<double> hc((size_t)ni * stride);
  KMX_HIP(ctx, hipMemcpyAsync(hc.data(), ctx->bcost.p, hc.size() * sizeof(double),
                              hipMemcpyDeviceToHost, ctx->stream));
  KMX_HIP(ctx, hipStreamSynchronize(ctx->stream));
  for (int i = 0; i < ni; ++i)
    std::memcpy(cost_hist + (size_t)pl.user_of[i] * stride, hc.data() + (size_t)i * stride,
                stride * sizeof(double));
  return KMX_OK;
}

kmx_status kmx_batched_autotune(kmx_ctx* ctx, const kmx_problem* probs, int32_t count,
                                kmx_prec prec, const char* cache_path, int32_t* loaded) {
  if (!ctx) return KMX_EINVAL;
  ctx->err.clear();
  KMX_TRY(check_problems(ctx, probs, count));
  if (prec != KMX_BF16) return fail(ctx, KMX_EUNSUPPORTED, "batched Lloyd runs the BF16 GEMM");
  KMX_TRY(set_device(ctx));
  if (loaded) *loaded = 0;
  const std::string dev = device_name(ctx);
  // the cache: one entry per line, {"device": ..., "d": .., "kclass": .., "variant": ..}
  if (cache_path) {
    std::ifstream in(cache_path);
    std::string line;
    int got = 0;
    while (in && std::getline(in, line)) {
      const size_t p = line.find("\"device\": \"" + dev + "\"");
      if (p == std::string::npos) continue;
      int d = 0, kc = 0, v = 0;
      const size_t q = line.find("\"d\":");
      if (q == std::string::npos) continue;
      if (std::sscanf(line.c_str() + q, "\"d\": %d, \"kclass\": %d, \"variant\": %d", &d, &kc,
                      &v) == 3 &&
          v >= 0 && v < batched_variants(d)) {
        ctx->tune[{d, kc}] = v;
        ++got;
      }
    }
    if (got > 0) {
      if (loaded) *loaded = 1;
      return KMX_OK;
    }
  }
  // classes present
  std::map<std::pair<int, int>, std::vector<int>> classes;
  for (int i = 0; i < count; ++i) classes[{probs[i].d, kclass_of(probs[i].k)}].push_back(i);
  std::ostringstream out;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  KMX_HIP(ctx, hipEventCreate(&e0));
  KMX_HIP(ctx, hipEventCreate(&e1));
  for (auto& kv : classes) {
    const int d = kv.first.first;
    const int nv = batched_variants(d);
    double best_ms = 1e300;
    int best = 0;
    std::vector<double> times;
    for (int v = 0; v < nv; ++v) {
      Plan pl;
      build_plan(ctx, probs, count, kv.second, v, pl);
      KMX_TRY(setup(ctx, probs, pl, 1));
      LoopState* st = ST(ctx);
      const BatchInst* insts = P<BatchInst>(ctx->binsts);
      auto run = [&]() -> hipError_t {
        hipError_t e = launch_batch_reset(ctx->stream, insts, (int)pl.insts.size(), st, nullptr);
        if (e == hipSuccess)
          e = launch_batch_prep_centers(ctx->stream, insts, P<int>(ctx->bcinst), pl.Ptot);
        if (e == hipSuccess) e = launch_groups(ctx, pl, ctx->stream);
        return e;
      };
      KMX_HIP(ctx, run());
      KMX_HIP(ctx, hipEventRecord(e0, ctx->stream));
      const int reps = 5;
      for (int r = 0; r < reps; ++r) KMX_HIP(ctx, run());
      KMX_HIP(ctx, hipEventRecord(e1, ctx->stream));
      KMX_HIP(ctx, hipEventSynchronize(e1));
      float ms = 0.f;
      KMX_HIP(ctx, hipEventElapsedTime(&ms, e0, e1));
      times.push_back(ms / reps);
      if (ms / reps < best_ms) {
        best_ms = ms / reps;
        best = v;
      }
    }
    ctx->tune[kv.first] = best;
    out << "{\"device\": \"" << dev << "\", \"d\": " << d << ", \"kclass\": " << kv.first.second
        << ", \"variant\": " << best << ", \"tile\": " << batched_variant_tile(d, best)
        << ", \"points_per_block\": " << batched_variant_ppb(d, best) << ", \"ms\": [";
    for (size_t t = 0; t < times.size(); ++t) out << (t ? ", " : "") << times[t];
    out << "]}\n";
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (cache_path) {
    std::ofstream f(cache_path, std::ios::app);
    if (!f) return fail(ctx, KMX_EINVAL, std::string("cannot write ") + cache_path);
    f << out.str();
  }
  return KMX_OK;
}

kmx_status kmx_batched_tiles(kmx_ctx* ctx, int32_t d, int32_t k, int32_t* tile,
                             int32_t* points_per_block) {
  if (!ctx) return KMX_EINVAL;
  ctx->err.clear();
  if (d < 1 || d > 512 || batched_variants(d) == 0 || k < 1)
    return fail(ctx, KMX_EUNSUPPORTED, "no batched shape for this (d, k)");
  const int v = variant_for(ctx, d, k);
  if (tile) *tile = batched_variant_tile(d, v);
  if (points_per_block) *points_per_block = batched_variant_ppb(d, v);
  return KMX_OK;
}

}  // extern "C"
