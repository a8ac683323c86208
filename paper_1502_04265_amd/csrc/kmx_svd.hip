// Host side of the randomized range finder: kmx_range_basis.
//
// The top-r right singular vectors of A' = diag(sqrt(w)) A (Sec. 2.2,
// "Computation of the SVD": a randomized truncated SVD that multiplies A with
// a random matrix to reduce its columns before computing the SVD, after
// Halko, Martinsson and Tropp 2011; Sec. 2.3.2: a point of weight w enters
// as its row scaled by sqrt(w), which gives the best-fit subspace of the
// point set with w copies of each point).  Randomized subspace iteration
// (HMT Alg. 4.4) and the direct SVD of the small projected matrix (Alg. 5.1):
//
//   Omega (d x l) Gaussian, l = r + oversampling rounded up to 16;
//   Q = orth(A' Omega);   q times: Z = orth(A'^T Q), Q = orth(A' Z);
//   Z = A'^T Q (d x l, = B^T for B = Q^T A');
//   B B^T = Z^T Z = U diag(sigma^2) U^T (l x l, host Jacobi in FP64);
//   V_r = Z U_r diag(1 / sigma_r)  (the top-r right singular vectors of B).
//
// On the device: the products with A (the projection kernel for A X, the
// FP64-accumulated A^T B kernel for A^T Q and the Gram matrices).  On the
// host, in FP64: the l x l Cholesky factors of the orthonormalisations
// (CholeskyQR2, the first pass shifted so that a rank-deficient block still
// factors; any invertible factor keeps the span) and the l x l eigenproblem.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "host_util.h"

using namespace kmx;
using namespace kmx::host;

namespace {

// G = R^T R for symmetric positive definite G (l x l, row-major), R upper
// triangular; false if a pivot is not positive.
bool cholesky_upper(const std::vector<double>& G, int l, std::vector<double>& R) {
  R.assign((size_t)l * l, 0.0);
  for (int i = 0; i < l; ++i) {
    double s = G[(size_t)i * l + i];
    for (int k = 0; k < i; ++k) s -= R[(size_t)k * l + i] * R[(size_t)k * l + i];
    if (!(s > 0.0)) return false;
    const double rii = std::sqrt(s);
    R[(size_t)i * l + i] = rii;
    for (int j = i + 1; j < l; ++j) {
      double t = G[(size_t)i * l + j];
      for (int k = 0; k < i; ++k) t -= R[(size_t)k * l + i] * R[(size_t)k * l + j];
      R[(size_t)i * l + j] = t / rii;
    }
  }
  return true;
}

// Inverse of an upper triangular matrix (back substitution, column by column).
std::vector<double> upper_inverse(const std::vector<double>& R, int l) {
  std::vector<double> X((size_t)l * l, 0.0);
  for (int j = 0; j < l; ++j) {
    X[(size_t)j * l + j] = 1.0 / R[(size_t)j * l + j];
    for (int i = j - 1; i >= 0; --i) {
      double s = 0.0;
      for (int k = i + 1; k <= j; ++k) s += R[(size_t)i * l + k] * X[(size_t)k * l + j];
      X[(size_t)i * l + j] = -s / R[(size_t)i * l + i];
    }
  }
  return X;
}

// Eigenvalues (descending) and eigenvectors (columns of U) of a symmetric
// l x l matrix by cyclic Jacobi rotations.
void jacobi_eig(std::vector<double> S, int l, std::vector<double>& lam, std::vector<double>& U) {
  U.assign((size_t)l * l, 0.0);
  for (int i = 0; i < l; ++i) U[(size_t)i * l + i] = 1.0;
  double fro = 0.0;
  for (double v : S) fro += v * v;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < l; ++p)
      for (int q = p + 1; q < l; ++q) off += S[(size_t)p * l + q] * S[(size_t)p * l + q];
    if (off <= 1e-30 * fro || off == 0.0) break;
    for (int p = 0; p < l; ++p) {
      for (int q = p + 1; q < l; ++q) {
        const double apq = S[(size_t)p * l + q];
        if (std::fabs(apq) < 1e-300) continue;
        const double app = S[(size_t)p * l + p], aqq = S[(size_t)q * l + q];
        const double tau = (aqq - app) / (2.0 * apq);
        const double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
        const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
        for (int k = 0; k < l; ++k) {   // rows p, q
          const double a = S[(size_t)p * l + k], b = S[(size_t)q * l + k];
          S[(size_t)p * l + k] = c * a - s * b;
          S[(size_t)q * l + k] = s * a + c * b;
        }
        for (int k = 0; k < l; ++k) {   // columns p, q
          const double a = S[(size_t)k * l + p], b = S[(size_t)k * l + q];
          S[(size_t)k * l + p] = c * a - s * b;
          S[(size_t)k * l + q] = s * a + c * b;
        }
        for (int k = 0; k < l; ++k) {
          const double a = U[(size_t)k * l + p], b = U[(size_t)k * l + q];
          U[(size_t)k * l + p] = c * a - s * b;
          U[(size_t)k * l + q] = s * a + c * b;
        }
      }
    }
  }
  std::vector<int> order(l);
  for (int i = 0; i < l; ++i) order[i] = i;
  std::sort(order.begin(), order.end(),
            [&](int a, int b) { return S[(size_t)a * l + a] > S[(size_t)b * l + b]; });
  lam.resize(l);
  std::vector<double> Us((size_t)l * l);
  for (int j = 0; j < l; ++j) {
    lam[j] = S[(size_t)order[j] * l + order[j]];
    for (int i = 0; i < l; ++i) Us[(size_t)i * l + j] = U[(size_t)i * l + order[j]];
  }
  U.swap(Us);
}

struct Svd {
  kmx_ctx* ctx;
  int l;
  double* part;
  double* G;      // l x l (or d x l) FP64 results
  float* Rinv;    // l x l
  float* Vt;      // projection workspace
  int64_t part_elems;
};

// G (p x q, FP64, device) = M1^T diag(sqrt w) M2 for tall M1 (rows x p), M2 (rows x q)
kmx_status atb(Svd& S, const float* M1, int64_t rows, int p, int64_t ld1, const float* M2, int q,
               int64_t ld2, const float* w, double* out) {
  kmx_ctx* ctx = S.ctx;
  int sl = atb_slices(rows, p, ctx->num_cus);
  while ((int64_t)sl * p * q > S.part_elems && sl > 1) --sl;
  KMX_HIP(ctx, launch_atb(ctx->stream, M1, rows, p, ld1, M2, q, ld2, w, S.part, sl, out));
  return KMX_OK;
}

// M (rows x l, leading dimension l) <- an orthonormal basis of its span
// (CholeskyQR2; tmp holds rows x l floats).
kmx_status orth(Svd& S, float* M, int64_t rows, float* tmp) {
  kmx_ctx* ctx = S.ctx;
  const int l = S.l;
  std::vector<double> G((size_t)l * l), R;
  for (int pass = 0; pass < 2; ++pass) {
    KMX_TRY(atb(S, M, rows, l, l, M, l, l, nullptr, S.G));
    KMX_HIP(ctx, hipMemcpyAsync(G.data(), S.G, G.size() * sizeof(double), hipMemcpyDeviceToHost,
                                ctx->stream));
    KMX_HIP(ctx, hipStreamSynchronize(ctx->stream));
    double tr = 0.0;
    for (int i = 0; i < l; ++i) tr += G[(size_t)i * l + i];
    if (!(tr > 0.0) || !std::isfinite(tr))
      return fail(ctx, KMX_EINVAL, "the sample spans no direction (zero or non-finite data)");
    // first pass shifted (FP32 data): a rank-deficient block still factors
    const double shift = pass == 0 ? 1e-6 * tr / l : 0.0;
    for (int i = 0; i < l; ++i) G[(size_t)i * l + i] += shift;
    if (!cholesky_upper(G, l, R)) {
      for (int i = 0; i < l; ++i) G[(size_t)i * l + i] += 1e-6 * tr / l;
      if (!cholesky_upper(G, l, R))
        return fail(ctx, KMX_EDEVICE, "Cholesky factor of the sample block failed");
    }
    const std::vector<double> Ri = upper_inverse(R, l);
    std::vector<float> Rf(Ri.size());
    for (size_t i = 0; i < Ri.size(); ++i) Rf[i] = (float)Ri[i];
    KMX_HIP(ctx, hipMemcpyAsync(S.Rinv, Rf.data(), Rf.size() * sizeof(float),
                                hipMemcpyHostToDevice, ctx->stream));
    KMX_HIP(ctx, launch_project(ctx->stream, M, rows, l, l, S.Rinv, l, tmp, l, S.Vt,
                                ctx->num_cus));
    KMX_HIP(ctx, hipMemcpyAsync(M, tmp, (size_t)rows * l * sizeof(float), hipMemcpyDeviceToDevice,
                                ctx->stream));
    KMX_HIP(ctx, hipStreamSynchronize(ctx->stream));   // Rf is read before it goes
  }
  return KMX_OK;
}

}  // namespace

extern "C" kmx_status kmx_range_basis(kmx_ctx* ctx, const float* A, int64_t n, int32_t d,
                                      int64_t lda, const float* w, int32_t r,
                                      int32_t oversample, int32_t power_iters, uint64_t seed,
                                      float* V_out, double* sigma_out) {
  if (!ctx) return KMX_EINVAL;
  ctx->err.clear();
  if (!A || !V_out) return fail(ctx, KMX_EINVAL, "NULL A or V_out");
  if (n < 1 || d < 1 || lda < d) return fail(ctx, KMX_EINVAL, "bad n, d or lda");
  if (r < 1 || oversample < 0 || power_iters < 0 || power_iters > 64)
    return fail(ctx, KMX_EINVAL, "bad r, oversample or power_iters");
  const int l = (r + oversample + 15) / 16 * 16;
  if (l > 128)
    return fail(ctx, KMX_EUNSUPPORTED, "r + oversample (rounded up to 16) must be <= 128");
  if ((int64_t)l > n || l > d)
    return fail(ctx, KMX_EINVAL, "r + oversample (rounded up to 16 = " + std::to_string(l) +
                                     ") exceeds n or d");
  KMX_TRY(set_device(ctx));
  KMX_TRY(check_data(ctx, A, n, d, lda, w, 1, nullptr, 0));
  const int r16 = (r + 15) / 16 * 16;
  const int64_t pmax = std::max<int64_t>(d, l);
  const int slmax = std::max(atb_slices(n, d, ctx->num_cus), atb_slices(d, l, ctx->num_cus));
  const int64_t part_elems = (int64_t)slmax * pmax * l;
  KMX_TRY(grow(ctx, ctx->sv_om, (size_t)d * l * sizeof(float)));
  KMX_TRY(grow(ctx, ctx->sv_y, (size_t)n * l * sizeof(float)));
  KMX_TRY(grow(ctx, ctx->sv_y2, (size_t)std::max<int64_t>(n, d) * l * sizeof(float)));
  KMX_TRY(grow(ctx, ctx->sv_z, (size_t)d * l * sizeof(float)));
  KMX_TRY(grow(ctx, ctx->sv_g, (size_t)pmax * l * sizeof(double)));
  KMX_TRY(grow(ctx, ctx->sv_part, (size_t)part_elems * sizeof(double)));
  KMX_TRY(grow(ctx, ctx->sv_r, (size_t)l * std::max(l, r16) * sizeof(float)));
  KMX_TRY(grow(ctx, ctx->vt, (size_t)std::max(l, r16) * project_dpad((int)pmax) * sizeof(float)));
  KMX_TRY(grow(ctx, ctx->sv_v, (size_t)d * r16 * sizeof(float)));
  Svd S{ctx, l, P<double>(ctx->sv_part), P<double>(ctx->sv_g), P<float>(ctx->sv_r),
        P<float>(ctx->vt), part_elems};
  float* Om = P<float>(ctx->sv_om);
  float* Y = P<float>(ctx->sv_y);
  float* T = P<float>(ctx->sv_y2);
  float* Z = P<float>(ctx->sv_z);
  hipStream_t s = ctx->stream;
  Timed tm(ctx, T_PROJECT);
  auto sample = [&](const float* V) -> kmx_status {   // Y = diag(sqrt w) A V, orthonormalised
    KMX_HIP(ctx, launch_project(s, A, n, d, lda, V, l, Y, l, S.Vt, ctx->num_cus));
    if (w) KMX_HIP(ctx, launch_scale_rows(s, Y, n, l, l, w));
    return orth(S, Y, n, T);
  };
  auto back = [&]() -> kmx_status {                    // Z = A^T diag(sqrt w) Y
    KMX_TRY(atb(S, A, n, d, lda, Y, l, l, w, S.G));
    KMX_HIP(ctx, launch_f64_to_f32(s, S.G, Z, (int64_t)d * l));
    return KMX_OK;
  };
  KMX_HIP(ctx, launch_gauss_fill(s, Om, (int64_t)d * l, seed));
  KMX_TRY(sample(Om));
  for (int it = 0; it < power_iters; ++it) {
    KMX_TRY(back());
    KMX_TRY(orth(S, Z, d, T));
    KMX_TRY(sample(Z));
  }
  KMX_TRY(back());
  // B B^T = Z^T Z (l x l) on the host: its eigenvectors are B's left
  // singular vectors, the square roots of its eigenvalues the singular values
  std::vector<double> Gh((size_t)l * l), lam, U;
  KMX_TRY(atb(S, Z, d, l, l, Z, l, l, nullptr, S.G));
  KMX_HIP(ctx, hipMemcpyAsync(Gh.data(), S.G, Gh.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  KMX_HIP(ctx, hipStreamSynchronize(s));
  jacobi_eig(Gh, l, lam, U);
  std::vector<float> M((size_t)l * r16, 0.0f);
  for (int j = 0; j < r; ++j) {
    const double sj = std::sqrt(std::max(lam[j], 0.0));
    if (sigma_out) sigma_out[j] = sj;
    if (!(sj > 0.0))
      return fail(ctx, KMX_EINVAL, "the data has fewer than r directions with positive variance");
    for (int i = 0; i < l; ++i) M[(size_t)i * r16 + j] = (float)(U[(size_t)i * l + j] / sj);
  }
  KMX_HIP(ctx, hipMemcpyAsync(S.Rinv, M.data(), M.size() * sizeof(float), hipMemcpyHostToDevice, s));
  float* Vp = P<float>(ctx->sv_v);
  KMX_HIP(ctx, launch_project(s, Z, d, l, l, S.Rinv, r16, Vp, r16, S.Vt, ctx->num_cus));
  KMX_HIP(ctx, hipMemcpy2DAsync(V_out, (size_t)r * sizeof(float), Vp, (size_t)r16 * sizeof(float),
                                (size_t)r * sizeof(float), (size_t)d, hipMemcpyDeviceToDevice, s));
  KMX_HIP(ctx, hipStreamSynchronize(s));   // M is read before it goes
  return KMX_OK;
}
