// Host-only driver for ash_principal_modes, built with the address and
// undefined-behaviour sanitizers by tests/test_host_sanitizers.py.  Checks
// shapes, orthogonality of the new coefficient columns and the error codes
// on a few cases; exits non-zero on a failed check.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include <vector>

#include "ash.h"

static int fails = 0;
#define CHECK(c)                                              \
  do {                                                        \
    if (!(c)) {                                               \
      fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
      ++fails;                                                \
    }                                                         \
  } while (0)

static double urand(unsigned* s) {
  *s = *s * 1664525u + 1013904223u;
  return (*s >> 8) * (1.0 / 16777216.0) - 0.5;
}

static void run_case(int N, int K, unsigned seed) {
  // basis: piston, x and y tilt, then 6 modes with degree-2 and degree-3
  // monomials (1, x, y, x^2, xy, y^2, x^3, y^3)
  const int n_mono = 8, D = 9;
  const int32_t pw[2 * n_mono] = {0, 0, 1, 0, 0, 1, 2, 0, 1, 1, 0, 2, 3, 0, 0, 3};
  std::vector<double> cf(D * n_mono, 0.0);
  cf[0 * n_mono + 0] = 1.0;
  cf[1 * n_mono + 1] = 2.0;
  cf[2 * n_mono + 2] = 2.0;
  for (int d = 3; d < D; ++d)
    for (int k = 0; k < n_mono; ++k) cf[d * n_mono + k] = k >= 3 ? urand(&seed) : 0.1 * urand(&seed);
  std::vector<double> w(N * D);
  for (auto& x : w) x = urand(&seed);
  int Dk = -1;
  std::vector<double> sigma(D, -1.0), mono(D * n_mono, 0.0), wk(N * D, 0.0);
  const int rc = ash_principal_modes(N, D, n_mono, pw, cf.data(), w.data(), K,
                                     &Dk, sigma.data(), mono.data(), wk.data());
  CHECK(rc == ASH_OK);
  if (rc != ASH_OK) return;
  CHECK(Dk == 3 + K);
  for (int j = 1; j < 6; ++j) CHECK(sigma[j] <= sigma[j - 1]);
  // new columns are orthogonal with norms sigma_j
  for (int a = 0; a < K; ++a)
    for (int b = 0; b < K; ++b) {
      double dot = 0.0;
      for (int n = 0; n < N; ++n) dot += wk[n * Dk + 3 + a] * wk[n * Dk + 3 + b];
      const double ref = a == b ? sigma[a] * sigma[a] : 0.0;
      CHECK(fabs(dot - ref) <= 1e-9 * (1.0 + sigma[0] * sigma[0]));
    }
  // kept modes unchanged
  for (int n = 0; n < N; ++n)
    for (int d = 0; d < 3; ++d) CHECK(wk[n * Dk + d] == w[n * D + d]);
}

int main() {
  run_case(40, 3, 1u);
  run_case(4, 6, 2u);     // fewer spots than rotated modes
  run_case(200, 0, 3u);
  run_case(1, 1, 4u);
  // errors
  int Dk = 0;
  double sig[9], mono[72], wk[9];
  const int32_t pw[2] = {2, 0};
  const double cf[9] = {1, 1, 1, 1, 1, 1, 1, 1, 1};
  const double w[9] = {1, 2, 3, 4, 5, 6, 7, 8, 9};
  CHECK(ash_principal_modes(1, 9, 1, pw, cf, w, 10, &Dk, sig, mono, wk) == ASH_EINVAL);
  CHECK(ash_principal_modes(1, 9, 1, pw, cf, w, -1, &Dk, sig, mono, wk) == ASH_EINVAL);
  CHECK(ash_principal_modes(0, 9, 1, pw, cf, w, 1, &Dk, sig, mono, wk) == ASH_EINVAL);
  CHECK(ash_principal_modes(1, ASH_MAX_PRINCIPAL_MODES + 1, 1, pw, cf, w, 1, &Dk,
                            sig, mono, wk) == ASH_EUNSUPPORTED);
  double wn[9] = {1, 2, 3, 4, NAN, 6, 7, 8, 9};
  CHECK(ash_principal_modes(1, 9, 1, pw, cf, wn, 1, &Dk, sig, mono, wk) == ASH_EINVAL);
  if (fails) return 1;
  printf("principal driver ok\n");
  return 0;
}
