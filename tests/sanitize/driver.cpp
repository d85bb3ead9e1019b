// Host-side checks of libfepll under AddressSanitizer and
// UndefinedBehaviorSanitizer (built with the whole library, host code
// instrumented; runs without a GPU): the float64 eigendecomposition of the
// setup on random covariances, and the argument validation and error paths
// of the C ABI, none of which may touch memory out of bounds or hit
// undefined behaviour.  Exit status 0 when every check holds.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "fepll.h"

static int failures = 0;
#define CHECK(cond)                                                       \
  do {                                                                    \
    if (!(cond)) {                                                        \
      std::fprintf(stderr, "check failed at line %d: %s (%s)\n", __LINE__, \
                   #cond, fepll_last_error());                            \
      ++failures;                                                         \
    }                                                                     \
  } while (0)

int main() {
  const int d = 64, K = 3;
  std::mt19937_64 rng(7);
  std::normal_distribution<double> nrm(0.0, 1.0);
  // random covariances B B^t / d + small ridge
  std::vector<double> S((size_t)K * d * d), U((size_t)K * d * d), lam((size_t)K * d);
  for (int k = 0; k < K; ++k) {
    std::vector<double> B((size_t)d * d);
    for (double& v : B) v = nrm(rng);
    for (int i = 0; i < d; ++i)
      for (int j = 0; j < d; ++j) {
        double s = 0.0;
        for (int l = 0; l < d; ++l) s += B[(size_t)i * d + l] * B[(size_t)j * d + l];
        S[((size_t)k * d + i) * d + j] = s / d + (i == j ? 1e-3 : 0.0);
      }
  }
  CHECK(fepll_cov_eig(S.data(), K, d, U.data(), lam.data()) == FEPLL_OK);
  // Sigma U = U diag(lambda), U orthonormal
  double res = 0.0, orth = 0.0;
  for (int k = 0; k < K; ++k)
    for (int i = 0; i < d; ++i)
      for (int j = 0; j < d; ++j) {
        double su = 0.0, uu = 0.0;
        for (int l = 0; l < d; ++l) {
          su += S[((size_t)k * d + i) * d + l] * U[((size_t)k * d + l) * d + j];
          uu += U[((size_t)k * d + l) * d + i] * U[((size_t)k * d + l) * d + j];
        }
        res = std::fmax(res, std::fabs(su - U[((size_t)k * d + i) * d + j] * lam[(size_t)k * d + j]));
        orth = std::fmax(orth, std::fabs(uu - (i == j ? 1.0 : 0.0)));
      }
  CHECK(res < 1e-10);
  CHECK(orth < 1e-12);
  // eigendecomposition: bad input
  CHECK(fepll_cov_eig(nullptr, K, d, U.data(), lam.data()) == FEPLL_EINVAL);
  CHECK(fepll_cov_eig(S.data(), 0, d, U.data(), lam.data()) == FEPLL_EINVAL);
  std::vector<double> bad = S;
  bad[1] += 1.0;  // not symmetric
  CHECK(fepll_cov_eig(bad.data(), K, d, U.data(), lam.data()) == FEPLL_EINVAL);
  bad = S;
  bad[5 * d + 5] = NAN;
  CHECK(fepll_cov_eig(bad.data(), K, d, U.data(), lam.data()) == FEPLL_EINVAL);
  // mixture creation: validation before any device work
  std::vector<double> w(K, 1.0 / K);
  fepll_gmm* g = nullptr;
  CHECK(fepll_gmm_create(U.data(), lam.data(), w.data(), K, 63, &g) == FEPLL_EINVAL);
  CHECK(fepll_gmm_create(U.data(), lam.data(), w.data(), 0, d, &g) == FEPLL_EINVAL);
  CHECK(fepll_gmm_create(U.data(), lam.data(), w.data(), K, d, nullptr) == FEPLL_EINVAL);
  std::vector<double> w2 = w;
  w2[0] += 0.1;  // weights do not sum to one
  CHECK(fepll_gmm_create(U.data(), lam.data(), w2.data(), K, d, &g) == FEPLL_EINVAL);
  std::vector<double> lam2 = lam;
  lam2[3] = -1.0;
  CHECK(fepll_gmm_create(U.data(), lam2.data(), w.data(), K, d, &g) == FEPLL_EINVAL);
  std::vector<double> U2 = U;
  U2[0] *= 2.0;  // not orthonormal
  CHECK(fepll_gmm_create(U2.data(), lam.data(), w.data(), K, d, &g) == FEPLL_EINVAL);
  CHECK(fepll_gmm_create_from_cov(nullptr, w.data(), K, d, &g) == FEPLL_EINVAL);
  // calls on a NULL handle or with NULL buffers
  float px[64 * 64] = {0};
  fepll_image im{px, 64, 64, 64, 0};
  fepll_options o;
  fepll_options_default(&o);
  CHECK(fepll_restore(nullptr, &im, nullptr, 10.0, nullptr, 5, &im, &o, nullptr) == FEPLL_EINVAL);
  CHECK(fepll_select_static(nullptr, &im, 1.0, nullptr, nullptr, nullptr, nullptr, nullptr) ==
        FEPLL_EINVAL);
  CHECK(fepll_restore_batch(nullptr, 1, &im, nullptr, &im, &o) == FEPLL_EINVAL);
  CHECK(fepll_set_tuning(nullptr, nullptr) == FEPLL_EINVAL);
  CHECK(fepll_gmm_load_proposal(nullptr, nullptr, 0) == FEPLL_EINVAL);
  CHECK(fepll_profile(nullptr, nullptr, nullptr, 0) == FEPLL_EINVAL);
  CHECK(fepll_mlp_param_count(200) == 65 * 256 + 256 + 256 * 256 + 256 + 256 * 200 + 200);
  CHECK(fepll_mlp_param_count(0) < 0);
  fepll_mlp* m = nullptr;
  CHECK(fepll_mlp_create(200, nullptr, 16, &m) == FEPLL_EINVAL);
  fepll_gmm_destroy(nullptr);
  // the memory cap and counter
  CHECK(fepll_set_memory_limit(1 << 20) == FEPLL_OK);
  CHECK(fepll_memory_in_use() == 0);
  CHECK(fepll_set_memory_limit(0) == FEPLL_OK);
  CHECK(fepll_version() != nullptr && fepll_last_error() != nullptr);
  if (failures) std::fprintf(stderr, "%d check(s) failed\n", failures);
  else std::printf("sanitized host checks passed\n");
  return failures ? 1 : 0;
}
