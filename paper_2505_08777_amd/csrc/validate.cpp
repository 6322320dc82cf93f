// Argument checks of the set-up calls, host-only: ash_set_basis and
// ash_set_spots run them before touching the device, and they build without
// HIP (g++ alone), so CPU tests and the host sanitizers exercise every
// error code of those calls without a GPU.
#include <math.h>
#include <stdint.h>

#include "ash.h"

namespace {

int reject(const char** detail, int code, const char* msg) {
  if (detail) *detail = msg;
  return code;
}

}  // namespace

extern "C" {

int ash_check_basis(int nx, int ny, double cx, double cy, double R, int D,
                    int n_mono, const int32_t* mono_pow,
                    const double* mono_coef, const char** detail) {
  if (detail) *detail = "";
  if (nx < 1 || ny < 1)
    return reject(detail, ASH_EINVAL, "nx, ny out of range");
  if (nx > ASH_MAX_SIDE || ny > ASH_MAX_SIDE)
    return reject(detail, ASH_EUNSUPPORTED, "nx, ny out of range");
  if (!isfinite(cx) || !isfinite(cy) || !isfinite(R) || !(R > 0.0))
    return reject(detail, ASH_EINVAL, "cx, cy must be finite and R > 0");
  if (D < 1 || n_mono < 1 || !mono_pow || !mono_coef)
    return reject(detail, ASH_EINVAL,
                  "D, n_mono must be >= 1, tables non-null");
  if (D > ASH_MAX_MODES || n_mono > ASH_MAX_MONOMIALS)
    return reject(detail, ASH_EUNSUPPORTED, "too many modes or monomials");
  for (int k = 0; k < n_mono; ++k) {
    const int p = mono_pow[2 * k], q = mono_pow[2 * k + 1];
    if (p < 0 || q < 0) return reject(detail, ASH_EINVAL, "negative exponent");
    if (p + q > ASH_MAX_DEGREE)
      return reject(detail, ASH_EUNSUPPORTED, "monomial degree too high");
    for (int k2 = 0; k2 < k; ++k2)
      if (mono_pow[2 * k2] == p && mono_pow[2 * k2 + 1] == q)
        return reject(detail, ASH_EINVAL, "repeated monomial");
  }
  for (long k = 0; k < (long)D * n_mono; ++k)
    if (!isfinite(mono_coef[k]))
      return reject(detail, ASH_EINVAL, "non-finite basis coefficient");
  return ASH_OK;
}

int ash_check_spots(int N, int D, const double* w, const float* target,
                    const char** detail) {
  if (detail) *detail = "";
  if (N < 1 || !w) return reject(detail, ASH_EINVAL, "N >= 1 and w required");
  if (N > ASH_MAX_SPOTS)
    return reject(detail, ASH_EUNSUPPORTED, "too many spots");
  if (D < 1 || D > ASH_MAX_MODES)
    return reject(detail, ASH_EINVAL, "D out of range");
  const long nw = (long)N * D;
  for (long k = 0; k < nw; ++k)
    if (!isfinite(w[k]))
      return reject(detail, ASH_EINVAL, "non-finite spot coefficient");
  if (target)
    for (int k = 0; k < N; ++k)
      if (!isfinite(target[k]) || !(target[k] > 0.0f))
        return reject(detail, ASH_EINVAL, "targets must be finite and > 0");
  return ASH_OK;
}

}  // extern "C"
