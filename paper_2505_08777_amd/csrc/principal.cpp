// Principal isoplanatic modes: the basis rotation of the paper's Methods,
// "Anisoplanatic Singular Value Decomposition".  The N x D spot-coefficient
// matrix is factored W = U S V^T; the columns of V turn the basis into modes
// ordered by singular value, and keeping the K largest gives the truncated
// correction.  Only the modes with a term of total degree >= 2 are rotated:
// piston and tilts carry each spot's constant and farfield position and
// pass through unchanged.  Host-only FP64 work on N x D numbers; no device
// memory is touched.
#include <math.h>

#include <algorithm>
#include <vector>

#include "ash.h"

namespace {

// One-sided (Hestenes) Jacobi SVD of the column-major m x n matrix a:
// plane rotations of column pairs until all columns are orthogonal; the
// column norms are then the singular values and the accumulated rotations
// the right singular vectors (v, column-major n x n).
void jacobi_svd(int m, int n, std::vector<double>& a, std::vector<double>& v) {
  v.assign((size_t)n * n, 0.0);
  for (int j = 0; j < n; ++j) v[(size_t)j * n + j] = 1.0;
  for (int sweep = 0; sweep < 80; ++sweep) {
    bool rotated = false;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        double* ap = &a[(size_t)p * m];
        double* aq = &a[(size_t)q * m];
        double alpha = 0.0, beta = 0.0, gamma = 0.0;
        for (int i = 0; i < m; ++i) {
          alpha += ap[i] * ap[i];
          beta += aq[i] * aq[i];
          gamma += ap[i] * aq[i];
        }
        if (gamma == 0.0 || fabs(gamma) <= 1e-15 * sqrt(alpha * beta))
          continue;
        rotated = true;
        // rotation angle that zeroes the pair's off-diagonal Gram entry
        const double zeta = (beta - alpha) / (2.0 * gamma);
        const double t = (zeta >= 0.0 ? 1.0 : -1.0) /
                         (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
        for (int i = 0; i < m; ++i) {
          const double x = ap[i], y = aq[i];
          ap[i] = c * x - s * y;
          aq[i] = s * x + c * y;
        }
        double* vp = &v[(size_t)p * n];
        double* vq = &v[(size_t)q * n];
        for (int i = 0; i < n; ++i) {
          const double x = vp[i], y = vq[i];
          vp[i] = c * x - s * y;
          vq[i] = s * x + c * y;
        }
      }
    if (!rotated) break;
  }
}

}  // namespace

extern "C" int ash_principal_modes(int N, int D, int n_mono,
                                   const int32_t* mono_pow,
                                   const double* mono_coef, const double* w,
                                   int K, int* D_out, double* sigma,
                                   double* mono_out, double* w_out) {
  if (N < 1 || D < 1 || n_mono < 1 || !mono_pow || !mono_coef || !w ||
      !D_out || !sigma || !mono_out || !w_out)
    return ASH_EINVAL;
  if (D > ASH_MAX_PRINCIPAL_MODES || n_mono > ASH_MAX_MONOMIALS ||
      N > ASH_MAX_SPOTS)
    return ASH_EUNSUPPORTED;
  for (long k = 0; k < (long)D * n_mono; ++k)
    if (!isfinite(mono_coef[k])) return ASH_EINVAL;
  for (long k = 0; k < (long)N * D; ++k)
    if (!isfinite(w[k])) return ASH_EINVAL;
  for (int k = 0; k < n_mono; ++k)
    if (mono_pow[2 * k] < 0 || mono_pow[2 * k + 1] < 0) return ASH_EINVAL;

  std::vector<int> keep, rot;
  for (int d = 0; d < D; ++d) {
    bool nonlin = false;
    for (int k = 0; k < n_mono; ++k)
      if (mono_pow[2 * k] + mono_pow[2 * k + 1] >= 2 &&
          mono_coef[(long)d * n_mono + k] != 0.0)
        nonlin = true;
    (nonlin ? rot : keep).push_back(d);
  }
  const int nr = (int)rot.size(), nk = (int)keep.size();
  if (K < 0 || K > nr) return ASH_EINVAL;

  // W_R, column-major N x nr
  std::vector<double> a((size_t)N * nr), v;
  for (int j = 0; j < nr; ++j)
    for (int n = 0; n < N; ++n)
      a[(size_t)j * N + n] = w[(long)n * D + rot[j]];
  jacobi_svd(N, nr, a, v);
  std::vector<double> s(nr);
  for (int j = 0; j < nr; ++j) {
    double ss = 0.0;
    for (int n = 0; n < N; ++n) ss += a[(size_t)j * N + n] * a[(size_t)j * N + n];
    s[j] = sqrt(ss);
  }
  std::vector<int> order(nr);
  for (int j = 0; j < nr; ++j) order[j] = j;
  std::stable_sort(order.begin(), order.end(),
                   [&](int x, int y) { return s[x] > s[y]; });
  // Sign of each singular vector: its largest entry positive (the products
  // that the transforms use do not depend on it).
  std::vector<double> V((size_t)nr * K);  // [rot index][principal j]
  for (int j = 0; j < K; ++j) {
    const double* col = &v[(size_t)order[j] * nr];
    int big = 0;
    for (int i = 1; i < nr; ++i)
      if (fabs(col[i]) > fabs(col[big])) big = i;
    const double sg = col[big] < 0.0 ? -1.0 : 1.0;
    for (int i = 0; i < nr; ++i) V[(size_t)i * K + j] = sg * col[i];
  }

  for (int j = 0; j < nr; ++j) sigma[j] = s[order[j]];
  *D_out = nk + K;
  const int Do = nk + K;
  for (int j = 0; j < nk; ++j)
    for (int k = 0; k < n_mono; ++k)
      mono_out[(long)j * n_mono + k] = mono_coef[(long)keep[j] * n_mono + k];
  for (int j = 0; j < K; ++j)
    for (int k = 0; k < n_mono; ++k) {
      double acc = 0.0;
      for (int i = 0; i < nr; ++i)
        acc += V[(size_t)i * K + j] * mono_coef[(long)rot[i] * n_mono + k];
      mono_out[(long)(nk + j) * n_mono + k] = acc;
    }
  for (int n = 0; n < N; ++n) {
    for (int j = 0; j < nk; ++j) w_out[(long)n * Do + j] = w[(long)n * D + keep[j]];
    for (int j = 0; j < K; ++j) {
      double acc = 0.0;
      for (int i = 0; i < nr; ++i)
        acc += w[(long)n * D + rot[i]] * V[(size_t)i * K + j];
      w_out[(long)n * Do + nk + j] = acc;
    }
  }
  return ASH_OK;
}
