// Float64 eigendecomposition of the mixture covariances at setup (Sec. 2.1:
// the eigenspace formulation needs Sigma_k = U_k S_k U_k^t), by the cyclic
// Jacobi method: plane rotations that zero one off-diagonal pair at a time,
// swept over all pairs until the off-diagonal mass is at rounding level.
// Each rotation is exactly orthogonal up to rounding, so U stays
// orthonormal to ~1e-15 and the eigenvalues are accurate relative to the
// largest one.  Host code: it runs once per mixture.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "fepll.h"
#include "internal.h"

using namespace fepll;

namespace {

// Symmetric a (n x n, row-major, overwritten) -> eigenvalues in w (any
// order) and eigenvectors as the columns of v.  Returns false if the sweeps
// do not converge.
bool jacobi(std::vector<double>& a, int n, std::vector<double>& w, std::vector<double>& v) {
  v.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) v[(size_t)i * n + i] = 1.0;
  double norm2 = 0.0;
  for (double x : a) norm2 += x * x;
  const double tol2 = norm2 * 1e-32;  // (1e-16 ||A||_F)^2
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) off += a[(size_t)p * n + q] * a[(size_t)p * n + q];
    if (off <= tol2) {
      w.resize(n);
      for (int i = 0; i < n; ++i) w[i] = a[(size_t)i * n + i];
      return true;
    }
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = a[(size_t)p * n + q];
        if (apq == 0.0) continue;
        const double app = a[(size_t)p * n + p], aqq = a[(size_t)q * n + q];
        // rotation angle: tan of the smaller root of t^2 + 2 theta t - 1 = 0
        const double theta = (aqq - app) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int r = 0; r < n; ++r) {
          if (r == p || r == q) continue;
          const double arp = a[(size_t)r * n + p], arq = a[(size_t)r * n + q];
          const double np_ = c * arp - s * arq, nq = s * arp + c * arq;
          a[(size_t)r * n + p] = a[(size_t)p * n + r] = np_;
          a[(size_t)r * n + q] = a[(size_t)q * n + r] = nq;
        }
        a[(size_t)p * n + p] = app - t * apq;
        a[(size_t)q * n + q] = aqq + t * apq;
        a[(size_t)p * n + q] = a[(size_t)q * n + p] = 0.0;
        for (int r = 0; r < n; ++r) {
          const double vrp = v[(size_t)r * n + p], vrq = v[(size_t)r * n + q];
          v[(size_t)r * n + p] = c * vrp - s * vrq;
          v[(size_t)r * n + q] = s * vrp + c * vrq;
        }
      }
  }
  return false;
}

}  // namespace

extern "C" {

fepll_status fepll_cov_eig(const double* Sigma, int32_t K, int32_t d, double* U, double* lambda) {
  clear_error();
  if (!Sigma || !U || !lambda) return fail(FEPLL_EINVAL, "Sigma, U and lambda must be non-NULL");
  if (K < 1 || K > 1024 || d < 1 || d > 1024) return fail(FEPLL_EINVAL, "K or d out of range");
  const size_t dd = (size_t)d * d;
  std::vector<double> a(dd), w, v;
  for (int k = 0; k < K; ++k) {
    const double* S = Sigma + (size_t)k * dd;
    double mx = 0.0;
    for (size_t i = 0; i < dd; ++i) {
      if (!std::isfinite(S[i]))
        return fail(FEPLL_EINVAL, "Sigma_" + std::to_string(k) + " has a non-finite entry");
      mx = std::max(mx, std::fabs(S[i]));
    }
    for (int i = 0; i < d; ++i)
      for (int j = i + 1; j < d; ++j)
        if (std::fabs(S[(size_t)i * d + j] - S[(size_t)j * d + i]) > 1e-9 * mx)
          return fail(FEPLL_EINVAL, "Sigma_" + std::to_string(k) + " is not symmetric (1e-9)");
    // the symmetric part
    for (int i = 0; i < d; ++i)
      for (int j = 0; j < d; ++j)
        a[(size_t)i * d + j] = 0.5 * (S[(size_t)i * d + j] + S[(size_t)j * d + i]);
    if (!jacobi(a, d, w, v))
      return fail(FEPLL_EINVAL, "Sigma_" + std::to_string(k) + ": eigenvalues did not converge");
    // decreasing order (Sec. 2.1); eigenvalues below zero by rounding are
    // clamped to zero, below by more the matrix is not a covariance
    std::vector<int> ord(d);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return w[x] > w[y]; });
    const double wmax = std::max(std::fabs(w[ord[0]]), mx);
    for (int j = 0; j < d; ++j) {
      double l = w[ord[j]];
      if (l < -1e-10 * wmax)
        return fail(FEPLL_EINVAL, "Sigma_" + std::to_string(k) + " is not positive semidefinite");
      lambda[(size_t)k * d + j] = std::max(l, 0.0);
      for (int p = 0; p < d; ++p) U[(size_t)k * dd + (size_t)p * d + j] = v[(size_t)p * d + ord[j]];
    }
  }
  return FEPLL_OK;
}

fepll_status fepll_gmm_create_from_cov(const double* Sigma, const double* w, int32_t K, int32_t d,
                                       fepll_gmm** out) {
  clear_error();
  if (!out) return fail(FEPLL_EINVAL, "out is NULL");
  if (d != 64) return fail(FEPLL_EINVAL, "d must be 64 (8x8 patches)");
  if (K < 1 || K > 1024) return fail(FEPLL_EINVAL, "K must be in 1..1024");
  std::vector<double> U((size_t)K * d * d), lam((size_t)K * d);
  fepll_status s = fepll_cov_eig(Sigma, K, d, U.data(), lam.data());
  if (s != FEPLL_OK) return s;
  return fepll_gmm_create(U.data(), lam.data(), w, K, d, out);
}

}  // extern "C"
