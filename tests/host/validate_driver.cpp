// Driver of the host-only argument checks (csrc/validate.cpp) for the
// sanitizer build: valid and invalid set-ups of several sizes, each code
// checked, including inputs whose arrays end exactly where the checks stop
// reading.
#include <math.h>
#include <stdint.h>
#include <stdio.h>

#include <vector>

#include "ash.h"

static int failures = 0;

static void expect(int got, int want, const char* what) {
  if (got != want) {
    printf("FAIL %s: got %d want %d\n", what, got, want);
    ++failures;
  }
}

int main() {
  const char* why = nullptr;
  // a basis of D modes over n monomials, exactly sized arrays
  for (int D = 1; D <= ASH_MAX_MODES; D += 7) {
    for (int n = 1; n <= 40; n += 13) {
      std::vector<int32_t> pw(2 * n);
      for (int k = 0; k < n; ++k) {
        pw[2 * k] = k % 5;
        pw[2 * k + 1] = k / 5;
      }
      std::vector<double> cf((size_t)D * n, 0.5);
      expect(ash_check_basis(64, 48, 32.0, 24.0, 24.0, D, n, pw.data(),
                             cf.data(), &why),
             ASH_OK, "valid basis");
      cf.back() = NAN;
      expect(ash_check_basis(64, 48, 32.0, 24.0, 24.0, D, n, pw.data(),
                             cf.data(), &why),
             ASH_EINVAL, "NaN in the last coefficient");
      if (n > 1) {
        pw[2 * (n - 1)] = pw[0];
        pw[2 * (n - 1) + 1] = pw[1];
        cf.back() = 0.5;
        expect(ash_check_basis(64, 48, 32.0, 24.0, 24.0, D, n, pw.data(),
                               cf.data(), &why),
               ASH_EINVAL, "repeated last monomial");
      }
    }
  }
  std::vector<int32_t> pw1 = {1, 0};
  std::vector<double> cf1 = {1.0};
  expect(ash_check_basis(0, 48, 0, 0, 1, 1, 1, pw1.data(), cf1.data(), &why),
         ASH_EINVAL, "nx 0");
  expect(ash_check_basis(ASH_MAX_SIDE + 1, 48, 0, 0, 1, 1, 1, pw1.data(),
                         cf1.data(), nullptr),
         ASH_EUNSUPPORTED, "nx too large, no detail pointer");
  expect(ash_check_basis(64, 48, 0, 0, 1, 1, 1, nullptr, nullptr, &why),
         ASH_EINVAL, "null tables");
  std::vector<int32_t> high = {ASH_MAX_DEGREE, 1};
  expect(ash_check_basis(64, 48, 0, 0, 1, 1, 1, high.data(), cf1.data(), &why),
         ASH_EUNSUPPORTED, "degree too high");
  // spots: exactly N x D coefficients and N targets
  for (int N = 1; N <= 4097; N += 1024) {
    for (int D = 1; D <= ASH_MAX_MODES; D += 10) {
      std::vector<double> w((size_t)N * D, 0.25);
      std::vector<float> t(N, 1.0f);
      expect(ash_check_spots(N, D, w.data(), t.data(), &why), ASH_OK,
             "valid spots");
      expect(ash_check_spots(N, D, w.data(), nullptr, &why), ASH_OK,
             "valid spots, unit targets");
      w.back() = INFINITY;
      expect(ash_check_spots(N, D, w.data(), t.data(), &why), ASH_EINVAL,
             "inf in the last coefficient");
      w.back() = 0.25;
      t.back() = 0.0f;
      expect(ash_check_spots(N, D, w.data(), t.data(), &why), ASH_EINVAL,
             "zero last target");
    }
  }
  expect(ash_check_spots(ASH_MAX_SPOTS + 1, 3, nullptr, nullptr, &why),
         ASH_EINVAL, "null w");
  double w1 = 0.0;
  expect(ash_check_spots(ASH_MAX_SPOTS + 1, 1, &w1, nullptr, &why),
         ASH_EUNSUPPORTED, "too many spots");
  if (failures) return 1;
  printf("validate driver ok\n");
  return 0;
}
