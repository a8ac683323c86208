// Allocation-free assignment: kmx_assign_noalloc.
//
// The same FP32 assignment as kmx_assign with KMX_FP32 (FP32 MFMA distance
// GEMM with the fused argmin, the rigorous flag and the exact re-check of the
// flagged rows; Sec. 1, assignment to the closest center), for callers that
// cannot allocate device memory.  Its working memory is one file-scope device
// array per GPU, `scratch`, that lives until the process ends; the rows are
// taken in chunks of kNaRows so that the per-row part of that memory does not
// grow with n.  Each row's label and distances depend only on that row and the
// centers, so chunking gives the bits kmx_assign gives.
//
// Host code never passes `scratch` itself to a kernel: in host code the name
// is a host-side stand-in.  Its device address is looked up once per device
// with hipGetSymbolAddress (noalloc_init, called by kmx_create with the device
// current) and kept in a per-device table.
#include <cstring>
#include <mutex>
#include <string>

#include "host_util.h"

using namespace kmx;
using namespace kmx::host;

namespace kmx {

constexpr size_t kNaBytes = (size_t)32 << 20;   // the whole array: 32 MiB per GPU
constexpr int64_t kNaRows = 262144;             // rows per chunk
constexpr size_t kNaHead = 4096;                // loop state, center statistics
constexpr size_t kNaRowBytes =
    (size_t)kNaRows * (sizeof(RowStats) + sizeof(FlagEntry) + sizeof(int));
constexpr size_t kNaCenterBytes = kNaBytes - kNaHead - kNaRowBytes;

__device__ __align__(256) unsigned char scratch[kNaBytes];

namespace {
constexpr int kNaMaxDev = 64;
std::mutex g_na_mu;
void* g_na_ptr[kNaMaxDev] = {nullptr};
}  // namespace

// Looks up (once per device; the caller has made `device` current) the device
// address of this device's copy of the array.
hipError_t noalloc_init(int device, void** ptr) {
  *ptr = nullptr;
  if (device < 0 || device >= kNaMaxDev) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_na_mu);
  if (!g_na_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_na_ptr[device] = p;
  }
  *ptr = g_na_ptr[device];
  return hipSuccess;
}

}  // namespace kmx

extern "C" kmx_status kmx_assign_noalloc(kmx_ctx* ctx, const float* X, int64_t n, int32_t d,
                                         int64_t ldx, const float* C, int32_t k,
                                         int32_t* label_out, float* d1_out, float* d2_out) {
  if (!ctx) return KMX_EINVAL;
  ctx->err.clear();
  KMX_TRY(check_problem(ctx, X, n, d, ldx, k));
  KMX_TRY(check_prec(ctx, KMX_FP32, d));
  if (!C) return fail(ctx, KMX_EINVAL, "C is NULL");
  if (!label_out) return fail(ctx, KMX_EINVAL, "label_out is NULL");
  if (!ctx->na_scratch)
    return fail(ctx, KMX_EDEVICE, "the static scratch array has no device address");
  const int dp32 = assign_dpad(KMX_FP32, d);
  const int bn32 = assign_tile_n(KMX_FP32, d, k);
  const int64_t kpad32 = ((int64_t)k + bn32 - 1) / bn32 * bn32;
  const size_t cbytes = (size_t)kpad32 * dp32 * sizeof(float);
  const size_t hbytes = ((size_t)kpad32 * sizeof(float) + 255) / 256 * 256;
  if (cbytes + hbytes > kNaCenterBytes)
    return fail(ctx, KMX_EINVAL,
                "kmx_assign_noalloc: the padded centers need " + std::to_string(cbytes + hbytes) +
                    " bytes of static scratch, more than the " + std::to_string(kNaCenterBytes) +
                    " available (k * d too large)");
  KMX_TRY(set_device(ctx));

  // carve the array (all offsets are multiples of 256 bytes)
  unsigned char* base = static_cast<unsigned char*>(ctx->na_scratch);
  LoopState* st = reinterpret_cast<LoopState*>(base);
  CenterStats* cs = reinterpret_cast<CenterStats*>(base + 256);
  unsigned* xmax = reinterpret_cast<unsigned*>(base + 512);
  RowStats* rs = reinterpret_cast<RowStats*>(base + kNaHead);
  FlagEntry* flags = reinterpret_cast<FlagEntry*>(rs + kNaRows);
  int* brute = reinterpret_cast<int*>(flags + kNaRows);
  float* ch = reinterpret_cast<float*>(base + kNaHead + kNaRowBytes);
  float* cq = reinterpret_cast<float*>(reinterpret_cast<unsigned char*>(ch) + hbytes);

  hipStream_t s = ctx->stream;
  // the loop state and the center statistics start from zero on every call
  KMX_HIP(ctx, launch_fill_i32(s, reinterpret_cast<int32_t*>(base), 1024 / 4, 0));
  KMX_HIP(ctx, launch_reset_small(s, cs, nullptr, nullptr, st, 1));
  KMX_HIP(ctx, launch_prep_centers(s, C, k, d, (int)kpad32, dp32, KMX_FP32, cq, ch, nullptr, cs,
                                   nullptr));
  for (int64_t r0 = 0; r0 < n; r0 += kNaRows) {
    const int64_t m = (n - r0 < kNaRows) ? n - r0 : kNaRows;
    const float* Xc = X + r0 * ldx;
    int32_t* lab = label_out + r0;
    float* d1 = d1_out ? d1_out + r0 : nullptr;
    float* d2 = d2_out ? d2_out + r0 : nullptr;
    // per-chunk counters of the flag lists
    KMX_HIP(ctx, launch_reset_small(s, nullptr, nullptr, nullptr, st, 0));
    KMX_HIP(ctx, launch_prep_rows(s, Xc, m, d, ldx, dp32, nullptr, rs, xmax, ctx->num_cus));
    KMX_HIP(ctx, launch_assign(s, KMX_FP32, Xc, ldx, nullptr, nullptr, m, nullptr, nullptr, d,
                               dp32, rs, cq, ch, k, (int)kpad32, cs, lab, d1, d2, flags, nullptr,
                               nullptr, 0, brute, st, nullptr, ctx->num_cus));
    KMX_HIP(ctx, launch_recheck(s, Xc, m, d, ldx, C, k, lab, d1, flags, brute, st, ctx->num_cus,
                                nullptr));
  }
  return KMX_OK;
}
