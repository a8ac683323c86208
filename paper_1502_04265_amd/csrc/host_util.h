// Host-side helpers shared by the kmx translation units: error reporting,
// the grow-only workspace, event timing and the launch sequences that the
// plain and the routed Lloyd loops have in common.  Not installed.
#pragma once

#include <string>

#include "kmx_internal.h"

namespace kmx {
namespace host {

extern thread_local std::string g_create_err;

inline kmx_status fail(kmx_ctx* ctx, kmx_status st, const std::string& msg) {
  if (ctx) ctx->err = msg;
  else g_create_err = msg;
  return st;
}

#define KMX_HIP(ctx, call)                                                              \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess) {                                                             \
      (void)hipGetLastError();                                                          \
      return ::kmx::host::fail(ctx, KMX_EDEVICE,                                        \
                               std::string(#call) + ": " + hipGetErrorString(e_));      \
    }                                                                                   \
  } while (0)

#define KMX_TRY(expr)            \
  do {                           \
    kmx_status s_ = (expr);      \
    if (s_ != KMX_OK) return s_; \
  } while (0)

// Grow-only device buffer: reallocates (after draining the stream) only when
// the request exceeds the current size.
inline kmx_status grow(kmx_ctx* ctx, Buf& b, size_t bytes) {
  if (bytes == 0) bytes = 16;
  if (b.bytes >= bytes) return KMX_OK;
  if (b.p) {
    KMX_HIP(ctx, hipStreamSynchronize(ctx->stream));
    KMX_HIP(ctx, hipFree(b.p));
    b.p = nullptr;
    b.bytes = 0;
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(ctx, KMX_ENOMEM,
                "hipMalloc of " + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(e));
  }
  b.p = p;
  b.bytes = bytes;
  ctx->ws_gen++;   // captured graphs that used the old buffer are stale
  return KMX_OK;
}

template <typename T>
inline T* P(const Buf& b) {
  return reinterpret_cast<T*>(b.p);
}

inline hipEvent_t take_event(kmx_ctx* c) {
  if (!c->pool.empty()) {
    hipEvent_t e = c->pool.back();
    c->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return e;
}

// HIP events around one kernel class on the context stream (when enabled).
struct Timed {
  kmx_ctx* c;
  int cls;
  hipEvent_t a = nullptr;
  Timed(kmx_ctx* c_, int cls_) : c(c_), cls(cls_) {
    if (c->timing) {
      a = take_event(c);
      if (a) (void)hipEventRecord(a, c->stream);
    }
  }
  ~Timed() {
    if (c->timing && a) {
      hipEvent_t b = take_event(c);
      if (b) {
        (void)hipEventRecord(b, c->stream);
        c->recs.push_back({cls, a, b});
      } else {
        c->pool.push_back(a);
      }
    }
  }
};

// Owners of a graph, its executable and an event: released on every return.
struct GraphGuard {
  hipGraph_t g = nullptr;
  hipGraphExec_t e = nullptr;
  ~GraphGuard() {
    if (e) (void)hipGraphExecDestroy(e);
    if (g) (void)hipGraphDestroy(g);
  }
};
struct EventGuard {
  hipEvent_t e = nullptr;
  ~EventGuard() {
    if (e) (void)hipEventDestroy(e);
  }
};

inline kmx_status set_device(kmx_ctx* ctx) {
  KMX_HIP(ctx, hipSetDevice(ctx->device));
  return KMX_OK;
}

inline LoopState* ST(kmx_ctx* ctx) { return P<LoopState>(ctx->state); }

kmx_status check_problem(kmx_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx,
                         int32_t k);
// allow_wide: rows wider than kGemmMaxD are taken (the exact every-center path)
kmx_status check_prec(kmx_ctx* ctx, int prec, int d, bool allow_wide = false);
// Weights finite and >= 0 with at least min_pos positive; with KMX_VALIDATE
// also X and C finite.  Synchronizes when it checks anything.
kmx_status check_data(kmx_ctx* ctx, const float* X, int64_t n, int d, int64_t ldx, const float* w,
                      int64_t min_pos, const float* C, int k);
kmx_status ensure_prep(kmx_ctx* ctx, const float* X, int64_t n, int d, int64_t ldx, int prec);
kmx_status ensure_assign(kmx_ctx* ctx, int64_t n, int k);
kmx_status ensure_common(kmx_ctx* ctx, int64_t n, int d, int k);
kmx_status write_state(kmx_ctx* ctx, int max_iter, double tol);
// Grids of the exactly summed clustering features for X and w (the dataset
// part cached like the quantized copies).
kmx_status ensure_cf(kmx_ctx* ctx, const float* X, int64_t n, int d, int64_t ldx, const float* w);
// Start of a Lloyd run: previous labels unknown (-1), delta entry counts clear.
kmx_status begin_lloyd(kmx_ctx* ctx, int32_t* prev, int64_t n);

// Per-iteration center preparation: resets the per-assignment counters,
// writes the FP32 GEMM copy of C and, for BF16, the quantized copy.
kmx_status run_prep_centers(kmx_ctx* ctx, const float* C, int k, int d, int prec);
// GEMM assignment over all rows (rows == nullptr) or over the rows listed in
// rows[0 .. *row_count), then the FP32 pass and the re-check.
// bo (nullable pointers): carried bounds written for the rows decided here.
kmx_status run_assign_gemm(kmx_ctx* ctx, const float* X, int64_t n, int d, int64_t ldx,
                           const float* C, int k, int prec, int32_t* label, float* d1,
                           float* d2, const int* rows, const unsigned long long* row_count,
                           const int* gate, BoundsOut bo = {});
// run_prep_centers + run_assign_gemm over all rows.
kmx_status run_assign(kmx_ctx* ctx, const float* X, int64_t n, int d, int64_t ldx, const float* C,
                      int k, int prec, int32_t* label, float* d1, float* d2, const int* gate);
kmx_status run_update(kmx_ctx* ctx, const float* X, int64_t n, int d, int64_t ldx, const float* w,
                      const int32_t* label, int k, const float* C_prev, float* C_out,
                      double* W_out, int write_c, int32_t* lab_prev, double* hist, int mode,
                      const int* gate);

}  // namespace host
}  // namespace kmx
