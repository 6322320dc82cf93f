// Host side of libash: the C ABI declared in include/ash.h, argument
// validation, device memory management and the Zernike -> monomial
// expansion used to hand a basis to ash_set_basis.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "ash.h"
#include "internal.h"

using namespace ash;

namespace {

// Detail of the last failed ash_create on this thread (no context exists).
thread_local std::string g_create_err;

int create_fail(int code, const std::string& msg) {
  g_create_err = msg;
  return code;
}

int fail(ash_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

int hip_fail(ash_ctx* c, hipError_t e, const char* what) {
  if (c) c->err = std::string(what) + ": " + hipGetErrorString(e);
  return ASH_EHIP;
}

#define HIPCHK(ctx, expr, what)                        \
  do {                                                 \
    hipError_t e_ = (expr);                            \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, what); \
  } while (0)

// Select the context's device for this host thread.
int use_device(ash_ctx* c) {
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return hip_fail(c, e, "hipGetDevice");
  if (cur != c->device) {
    e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
  }
  return ASH_OK;
}

hipEvent_t prof_event(ash_ctx* c) {
  if (!c->prof_pool.empty()) {
    hipEvent_t e = c->prof_pool.back();
    c->prof_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return e;
}

// Enqueue `launch` bracketed by events of category `cat` when profiling.
template <typename F>
hipError_t timed(ash_ctx* c, int cat, F&& launch) {
  if (!c->prof_on) return launch();
  hipEvent_t a = prof_event(c), b = prof_event(c);
  if (a) (void)hipEventRecord(a, c->stream);
  hipError_t e = launch();
  if (a && b) {
    (void)hipEventRecord(b, c->stream);
    c->prof.push_back({cat, a, b});
  } else {
    if (a) c->prof_pool.push_back(a);
    if (b) c->prof_pool.push_back(b);
  }
  return e;
}

void prof_release(ash_ctx* c) {
  for (auto& r : c->prof) {
    c->prof_pool.push_back(r.start);
    c->prof_pool.push_back(r.stop);
  }
  c->prof.clear();
}

template <typename T>
void dfree(T*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

template <typename T>
int dalloc(ash_ctx* c, T** p, size_t count, const char* what) {
  *p = nullptr;
  if (count == 0) count = 1;
  hipError_t e = hipMalloc(reinterpret_cast<void**>(p), count * sizeof(T));
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    c->err = std::string("out of device memory allocating ") + what;
    return ASH_ENOMEM;
  }
  return ASH_OK;
}

void free_spots(ash_ctx* c) {
  Buffers& b = c->buf;
  dfree(b.spotrec);
  dfree(b.offtab);
  dfree(b.target);
  dfree(b.y);
  dfree(b.Ebuf);
  dfree(b.w64);
  dfree(b.spot64);
  dfree(b.partial);
  dfree(b.red);
  b.cap_spots = b.cap_w = b.cap_off = b.cap_partial = b.cap_red = 0;
  c->has_spots = false;
  c->spots = Spots();
}

void free_basis(ash_ctx* c) {
  free_spots(c);
  Buffers& b = c->buf;
  dfree(b.pixtab);
  dfree(b.amp_t);
  dfree(b.field_t);
  dfree(b.aff_dev);
  dfree(b.nlmode_dev);
  dfree(b.tilez);
  c->has_basis = false;
  c->basis = Basis();
}

// binomial coefficient (exact in double for the degrees allowed)
double binom(int n, int k) {
  if (k < 0 || k > n) return 0.0;
  double r = 1.0;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}

double fact(int n) {
  double r = 1.0;
  for (int i = 2; i <= n; ++i) r *= i;
  return r;
}

}  // namespace

extern "C" {

int ash_version(void) { return 100; }

const char* ash_strerror(int code) {
  switch (code) {
    case ASH_OK: return "ok";
    case ASH_EINVAL: return "invalid argument";
    case ASH_ESHAPE: return "shape mismatch";
    case ASH_ENOTREADY: return "basis or spots not set";
    case ASH_EUNSUPPORTED: return "unsupported size or configuration";
    case ASH_ENOMEM: return "out of memory";
    case ASH_EHIP: return "HIP runtime error";
    default: return "unknown error";
  }
}

const char* ash_last_error(const ash_ctx* ctx) {
  return ctx ? ctx->err.c_str() : g_create_err.c_str();
}

int ash_zernike_monomials(int ansi, int cap, int32_t* pow_out,
                          double* coef_out) {
  if (ansi < 0 || cap < 0 || (cap > 0 && (!pow_out || !coef_out)))
    return ASH_EINVAL;
  // ANSI index -> (n, m)
  int n = 0;
  while ((n + 1) * (n + 2) / 2 <= ansi) ++n;
  const int m = 2 * ansi - n * (n + 2);
  if (n > ASH_MAX_DEGREE) return ASH_EUNSUPPORTED;
  const int am = m < 0 ? -m : m;
  // Z = N * sum_s r_s rho^(n-2s) * {cos, sin}(am * angle), and
  // rho^(n-2s) cos(am angle) = (x^2+y^2)^q Re((x+iy)^am), q = (n-2s-am)/2
  // (Im for the sine).  Accumulate coefficients of x^p y^q in a grid.
  std::vector<double> grid((n + 1) * (n + 1), 0.0);
  const double N = sqrt(2.0 * (n + 1) / (m == 0 ? 2.0 : 1.0));
  for (int s = 0; s <= (n - am) / 2; ++s) {
    const double rs = ((s % 2) ? -1.0 : 1.0) * fact(n - s) /
                      (fact(s) * fact((n + am) / 2 - s) * fact((n - am) / 2 - s));
    const int q = (n - 2 * s - am) / 2;
    for (int t = 0; t <= am; ++t) {
      // i^t: real part for cos (t even), imaginary part for sin (t odd)
      double part;
      if (m >= 0) {
        if (t % 2) continue;
        part = (t % 4 == 0) ? 1.0 : -1.0;
      } else {
        if (!(t % 2)) continue;
        part = (t % 4 == 1) ? 1.0 : -1.0;
      }
      const double bt = binom(am, t) * part;  // x^(am-t) y^t
      for (int r = 0; r <= q; ++r) {
        const double br = binom(q, r);  // x^(2(q-r)) y^(2r)
        const int px = am - t + 2 * (q - r);
        const int py = t + 2 * r;
        grid[px * (n + 1) + py] += N * rs * bt * br;
      }
    }
  }
  int count = 0;
  for (int px = 0; px <= n; ++px)
    for (int py = 0; py + px <= n; ++py) {
      const double v = grid[px * (n + 1) + py];
      if (v != 0.0) {
        if (count >= cap) return ASH_EUNSUPPORTED;
        pow_out[2 * count] = px;
        pow_out[2 * count + 1] = py;
        coef_out[count] = v;
        ++count;
      }
    }
  return count;
}

int ash_create(ash_ctx** out, int device, void* stream) {
  g_create_err = "null context";
  if (!out) return ASH_EINVAL;
  *out = nullptr;
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return create_fail(ASH_EHIP, std::string("hipGetDeviceCount: ") +
                                     hipGetErrorString(e));
  }
  if (ndev <= 0) return create_fail(ASH_EHIP, "no HIP device");
  if (device < 0 || device >= ndev)
    return create_fail(ASH_EINVAL, "device index out of range");
  char arch[64] = {0};
  hipDevice_t dev;
  e = hipDeviceGet(&dev, device);
  if (e == hipSuccess) {
    int major = 0, minor = 0;
    e = hipDeviceGetAttribute(&major, hipDeviceAttributeComputeCapabilityMajor,
                              device);
    if (e == hipSuccess)
      e = hipDeviceGetAttribute(
          &minor, hipDeviceAttributeComputeCapabilityMinor, device);
    // gfx950 reports compute capability 9.5
    if (e == hipSuccess) snprintf(arch, sizeof arch, "%d.%d", major, minor);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return create_fail(ASH_EHIP, std::string("device query: ") +
                                     hipGetErrorString(e));
  }
  if (strcmp(arch, "9.5") != 0)
    return create_fail(ASH_EUNSUPPORTED,
                       std::string("needs gfx950, device reports ") + arch);
  int n_cu = 0;
  e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount,
                            device);
  if (e != hipSuccess || n_cu <= 0) {
    (void)hipGetLastError();
    return create_fail(ASH_EHIP, "device query: compute unit count");
  }
  ash_ctx* c = new (std::nothrow) ash_ctx();
  if (!c) return create_fail(ASH_ENOMEM, "host allocation");
  g_create_err.clear();
  c->device = device;
  c->n_cu = n_cu;
  c->stream = reinterpret_cast<hipStream_t>(stream);
  *out = c;
  return ASH_OK;
}

int ash_destroy(ash_ctx* c) {
  if (!c) return ASH_EINVAL;
  if (use_device(c) == ASH_OK) (void)hipStreamSynchronize(c->stream);
  prof_release(c);
  for (hipEvent_t e : c->prof_pool) (void)hipEventDestroy(e);
  c->prof_pool.clear();
  free_basis(c);
  delete c;
  return ASH_OK;
}

int ash_set_stream(ash_ctx* c, void* stream) {
  if (!c) return ASH_EINVAL;
  c->stream = reinterpret_cast<hipStream_t>(stream);
  return ASH_OK;
}

int ash_sync(ash_ctx* c) {
  if (!c) return ASH_EINVAL;
  int rc = use_device(c);
  if (rc) return rc;
  HIPCHK(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  return ASH_OK;
}

int ash_set_basis(ash_ctx* c, int nx, int ny, double cx, double cy, double R,
                  int D, int n_mono, const int32_t* mono_pow,
                  const double* mono_coef, const float* amp_dev) {
  if (!c) return ASH_EINVAL;
  c->err.clear();
  if (nx < 1 || ny < 1 || nx > ASH_MAX_SIDE || ny > ASH_MAX_SIDE)
    return fail(c, nx < 1 || ny < 1 ? ASH_EINVAL : ASH_EUNSUPPORTED,
                "nx, ny out of range");
  if (!isfinite(cx) || !isfinite(cy) || !isfinite(R) || !(R > 0.0))
    return fail(c, ASH_EINVAL, "cx, cy must be finite and R > 0");
  if (D < 1 || n_mono < 1 || !mono_pow || !mono_coef)
    return fail(c, ASH_EINVAL, "D, n_mono must be >= 1, tables non-null");
  if (D > ASH_MAX_MODES || n_mono > ASH_MAX_MONOMIALS)
    return fail(c, ASH_EUNSUPPORTED, "too many modes or monomials");
  for (int k = 0; k < n_mono; ++k) {
    const int p = mono_pow[2 * k], q = mono_pow[2 * k + 1];
    if (p < 0 || q < 0) return fail(c, ASH_EINVAL, "negative exponent");
    if (p + q > ASH_MAX_DEGREE)
      return fail(c, ASH_EUNSUPPORTED, "monomial degree too high");
    for (int k2 = 0; k2 < k; ++k2)
      if (mono_pow[2 * k2] == p && mono_pow[2 * k2 + 1] == q)
        return fail(c, ASH_EINVAL, "repeated monomial");
  }
  for (long k = 0; k < (long)D * n_mono; ++k)
    if (!isfinite(mono_coef[k]))
      return fail(c, ASH_EINVAL, "non-finite basis coefficient");

  Basis b;
  b.nx = nx;
  b.ny = ny;
  b.cx = cx;
  b.cy = cy;
  b.R = R;
  b.D = D;
  b.aff.assign(3 * D, 0.0);
  std::vector<double> nlcoef;  // [nl][n_mono], affine terms zeroed
  for (int d = 0; d < D; ++d) {
    bool nonlin = false;
    for (int k = 0; k < n_mono; ++k) {
      const int p = mono_pow[2 * k], q = mono_pow[2 * k + 1];
      const double v = mono_coef[(long)d * n_mono + k];
      if (p + q == 0) b.aff[3 * d] += v;
      else if (p == 1 && q == 0) b.aff[3 * d + 1] += v;
      else if (p == 0 && q == 1) b.aff[3 * d + 2] += v;
      else if (v != 0.0) nonlin = true;
    }
    if (nonlin) {
      b.nl_mode.push_back(d);
      for (int k = 0; k < n_mono; ++k) {
        const int p = mono_pow[2 * k], q = mono_pow[2 * k + 1];
        nlcoef.push_back(p + q >= 2 ? mono_coef[(long)d * n_mono + k] : 0.0);
      }
    }
  }
  b.nl = (int)b.nl_mode.size();
  if (b.nl > ASH_MAX_NONLINEAR)
    return fail(c, ASH_EUNSUPPORTED, "too many non-linear modes");
  b.kh = half_k(b.nl);
  b.rec = 2 * b.kh;
  b.tiles_x = (nx + kTileW - 1) / kTileW;
  b.tiles_y = (ny + kTileH - 1) / kTileH;
  b.n_tiles = b.tiles_x * b.tiles_y;

  int rc = use_device(c);
  if (rc) return rc;
  // amplitude: validate and sum A^2 on the host (one-time copy)
  const size_t P = (size_t)nx * ny;
  double s2 = 0.0;
  if (amp_dev) {
    std::vector<float> h(P);
    hipError_t e = hipMemcpyAsync(h.data(), amp_dev, P * sizeof(float),
                                  hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "reading amplitude");
    for (size_t k = 0; k < P; ++k) {
      if (!isfinite(h[k]) || h[k] < 0.0f)
        return fail(c, ASH_EINVAL, "amplitude must be finite and >= 0");
      s2 += (double)h[k] * h[k];
    }
  } else {
    s2 = (double)P;
  }
  b.amp_sum2 = s2;

  free_basis(c);
  Buffers& B = c->buf;
  const size_t npix = (size_t)b.n_tiles * kTile;
  if ((rc = dalloc(c, &B.pixtab, npix * b.rec, "basis table")) ||
      (rc = dalloc(c, &B.amp_t, npix, "amplitude")) ||
      (rc = dalloc(c, &B.field_t, 2 * npix, "nearfield")) ||
      (rc = dalloc(c, &B.aff_dev, 3 * (size_t)D, "basis affine terms")) ||
      (rc = dalloc(c, &B.nlmode_dev, (size_t)std::max(b.nl, 1), "modes")) ||
      (rc = dalloc(c, &B.tilez, 3 * (size_t)b.n_tiles * std::max(b.nl, 1),
                   "tile basis"))) {
    free_basis(c);
    return rc;
  }
  int32_t* d_pow = nullptr;
  double* d_nl = nullptr;
  if ((rc = dalloc(c, &d_pow, 2 * (size_t)n_mono, "monomials")) ||
      (rc = dalloc(c, &d_nl, nlcoef.size(), "monomial coefficients"))) {
    dfree(d_pow);
    free_basis(c);
    return rc;
  }
  hipError_t e = hipMemcpyAsync(d_pow, mono_pow, 2 * n_mono * sizeof(int32_t),
                                hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess && !nlcoef.empty())
    e = hipMemcpyAsync(d_nl, nlcoef.data(), nlcoef.size() * sizeof(double),
                       hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(B.aff_dev, b.aff.data(), 3 * D * sizeof(double),
                       hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess && b.nl > 0)
    e = hipMemcpyAsync(B.nlmode_dev, b.nl_mode.data(), b.nl * sizeof(int),
                       hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess)
    e = launch_build_pixtab(b, d_pow, d_nl, n_mono, amp_dev, B.pixtab,
                            B.amp_t, B.tilez, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  dfree(d_pow);
  dfree(d_nl);
  if (e != hipSuccess) {
    free_basis(c);
    return hip_fail(c, e, "building basis table");
  }
  c->basis = b;
  c->has_basis = true;
  return ASH_OK;
}

int ash_set_spots(ash_ctx* c, int N, const double* w_host,
                  const float* target_host) {
  if (!c) return ASH_EINVAL;
  c->err.clear();
  if (!c->has_basis) return fail(c, ASH_ENOTREADY, "set the basis first");
  if (N < 1 || !w_host) return fail(c, ASH_EINVAL, "N >= 1 and w required");
  if (N > ASH_MAX_SPOTS) return fail(c, ASH_EUNSUPPORTED, "too many spots");
  const Basis& b = c->basis;
  const size_t nw = (size_t)N * b.D;
  for (size_t k = 0; k < nw; ++k)
    if (!isfinite(w_host[k]))
      return fail(c, ASH_EINVAL, "non-finite spot coefficient");
  std::vector<float> t(N, 1.0f);
  double tn2 = 0.0;
  for (int k = 0; k < N; ++k) {
    if (target_host) t[k] = target_host[k];
    if (!isfinite(t[k]) || !(t[k] > 0.0f))
      return fail(c, ASH_EINVAL, "targets must be finite and > 0");
    tn2 += (double)t[k] * t[k];
  }
  int rc = use_device(c);
  if (rc) return rc;
  const FwdPlan plan = plan_forward(b.n_tiles, N,
                                    forward_blocks_per_cu(b.kh), c->n_cu);
  Buffers& B = c->buf;
  const size_t n_off = (size_t)b.n_tiles * N * 4;
  const size_t n_part = (size_t)plan.groups * N * 2;
  const size_t n_red = (size_t)plan.slices * N * 2;
  // grow-only allocations (state is rebuilt below in any case)
  if ((size_t)N > B.cap_spots) {
    dfree(B.spotrec);
    dfree(B.target);
    dfree(B.y);
    dfree(B.Ebuf);
    dfree(B.spot64);
    B.cap_spots = 0;
    if ((rc = dalloc(c, &B.spotrec, (size_t)N * b.rec, "spot records")) ||
        (rc = dalloc(c, &B.target, (size_t)N, "targets")) ||
        (rc = dalloc(c, &B.y, 2 * (size_t)N, "spot fields")) ||
        (rc = dalloc(c, &B.Ebuf, 2 * (size_t)N, "spot fields")) ||
        (rc = dalloc(c, &B.spot64, 3 * (size_t)N, "spot offsets"))) {
      free_spots(c);
      return rc;
    }
    B.cap_spots = N;
  }
  if (nw > B.cap_w) {
    dfree(B.w64);
    B.cap_w = 0;
    if ((rc = dalloc(c, &B.w64, nw, "coefficients"))) {
      free_spots(c);
      return rc;
    }
    B.cap_w = nw;
  }
  if (n_off > B.cap_off) {
    dfree(B.offtab);
    B.cap_off = 0;
    if ((rc = dalloc(c, &B.offtab, n_off, "tile offsets"))) {
      free_spots(c);
      return rc;
    }
    B.cap_off = n_off;
  }
  if (n_part > B.cap_partial) {
    dfree(B.partial);
    B.cap_partial = 0;
    if ((rc = dalloc(c, &B.partial, n_part, "partial sums"))) {
      free_spots(c);
      return rc;
    }
    B.cap_partial = n_part;
  }
  if (n_red > B.cap_red) {
    dfree(B.red);
    B.cap_red = 0;
    if ((rc = dalloc(c, &B.red, n_red, "partial sums"))) {
      free_spots(c);
      return rc;
    }
    B.cap_red = n_red;
  }
  hipError_t e = hipMemcpyAsync(B.w64, w_host, nw * sizeof(double),
                                hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(B.target, t.data(), N * sizeof(float),
                       hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess)
    e = launch_prep_spots(b, N, B.w64, B.aff_dev, B.nlmode_dev, B.tilez,
                          B.spotrec, B.offtab, B.spot64, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    c->has_spots = false;
    return hip_fail(c, e, "preparing spots");
  }
  c->spots.N = N;
  c->spots.srec = b.rec;
  c->spots.t_norm2 = tn2;
  c->plan = plan;
  c->has_spots = true;
  return ASH_OK;
}

int ash_forward(ash_ctx* c, const float* phase_dev, const float* field_dev,
                float* E_dev) {
  if (!c) return ASH_EINVAL;
  c->err.clear();
  if (!c->has_basis || !c->has_spots)
    return fail(c, ASH_ENOTREADY, "basis and spots must be set");
  if ((phase_dev == nullptr) == (field_dev == nullptr) || !E_dev)
    return fail(c, ASH_EINVAL, "exactly one of phase/field, and E, required");
  int rc = use_device(c);
  if (rc) return rc;
  const Basis& b = c->basis;
  Buffers& B = c->buf;
  const int N = c->spots.N;
  HIPCHK(c, timed(c, ASH_PROF_FIELD, [&] {
           return launch_make_field(b, phase_dev, field_dev, B.amp_t,
                                    B.field_t, c->stream);
         }), "make_field");
  HIPCHK(c, timed(c, ASH_PROF_FORWARD, [&] {
           return launch_forward(b, N, c->plan, B.pixtab, B.field_t,
                                 B.spotrec, B.offtab, B.partial, c->stream);
         }), "forward");
  HIPCHK(c, timed(c, ASH_PROF_REDUCE, [&] {
           return launch_reduce(N, c->plan, B.partial, B.red, c->stream);
         }), "reduce");
  HIPCHK(c, timed(c, ASH_PROF_REDUCE, [&] {
           return launch_finish_E(N, c->plan, B.red, E_dev, c->stream);
         }), "finish");
  return ASH_OK;
}

int ash_adjoint(ash_ctx* c, const float* y_dev, float* g_dev,
                float* phase_out_dev) {
  if (!c) return ASH_EINVAL;
  c->err.clear();
  if (!c->has_basis || !c->has_spots)
    return fail(c, ASH_ENOTREADY, "basis and spots must be set");
  if (!y_dev || (!g_dev && !phase_out_dev))
    return fail(c, ASH_EINVAL, "y and at least one output required");
  int rc = use_device(c);
  if (rc) return rc;
  const int outs = (g_dev ? kOutG : 0) | (phase_out_dev ? kOutPhase : 0);
  HIPCHK(c, timed(c, ASH_PROF_REDUCE, [&] {
           return launch_to_polar(c->spots.N, y_dev, c->buf.y, c->stream);
         }), "to_polar");
  HIPCHK(c, timed(c, ASH_PROF_ADJOINT, [&] {
           return launch_adjoint(c->basis, c->spots.N, c->buf.pixtab,
                                 c->buf.spotrec, c->buf.offtab, c->buf.y,
                                 c->buf.amp_t, outs, g_dev, phase_out_dev,
                                 nullptr, c->stream);
         }), "adjoint");
  return ASH_OK;
}

int ash_wgs_iterate(ash_ctx* c, float* phase_dev, float* weights_dev,
                    int n_iter, const ash_wgs_params* params, float* E_dev,
                    float* stats_dev) {
  if (!c) return ASH_EINVAL;
  c->err.clear();
  if (!c->has_basis || !c->has_spots)
    return fail(c, ASH_ENOTREADY, "basis and spots must be set");
  if (!phase_dev || !weights_dev || n_iter < 0)
    return fail(c, ASH_EINVAL, "phase, weights and n_iter >= 0 required");
  const float power = params ? params->power : 1.0f;
  if (!isfinite(power)) return fail(c, ASH_EINVAL, "power must be finite");
  if (n_iter == 0) return ASH_OK;
  int rc = use_device(c);
  if (rc) return rc;
  const Basis& b = c->basis;
  Buffers& B = c->buf;
  const int N = c->spots.N;
  const float t_norm = (float)sqrt(c->spots.t_norm2);
  const float eff_denom = (float)((double)b.nx * b.ny * b.amp_sum2);
  HIPCHK(c, timed(c, ASH_PROF_FIELD, [&] {
           return launch_make_field(b, phase_dev, nullptr, B.amp_t,
                                    B.field_t, c->stream);
         }), "make_field");
  for (int it = 0; it < n_iter; ++it) {
    const bool last = it == n_iter - 1;
    HIPCHK(c, timed(c, ASH_PROF_FORWARD, [&] {
             return launch_forward(b, N, c->plan, B.pixtab, B.field_t,
                                   B.spotrec, B.offtab, B.partial, c->stream);
           }), "forward");
    HIPCHK(c, timed(c, ASH_PROF_REDUCE, [&] {
             return launch_reduce(N, c->plan, B.partial, B.red, c->stream);
           }), "reduce");
    HIPCHK(c, timed(c, ASH_PROF_REDUCE, [&] {
             return launch_wgs_update(
                 N, c->plan, B.red, B.target, t_norm, weights_dev, power,
                 eff_denom, B.y, B.Ebuf, last ? E_dev : nullptr,
                 stats_dev ? stats_dev + 4 * (size_t)it : nullptr, c->stream);
           }), "wgs_update");
    HIPCHK(c, timed(c, ASH_PROF_ADJOINT, [&] {
             return launch_adjoint(b, N, B.pixtab, B.spotrec, B.offtab, B.y,
                                   B.amp_t, last ? kOutPhase : kOutField,
                                   nullptr, last ? phase_dev : nullptr,
                                   last ? nullptr : B.field_t, c->stream);
           }), "adjoint");
  }
  return ASH_OK;
}

int ash_profile_enable(ash_ctx* c, int enable) {
  if (!c) return ASH_EINVAL;
  c->prof_on = enable != 0;
  return ASH_OK;
}

int ash_profile_read(ash_ctx* c, double* ms_out, int64_t* launches_out) {
  if (!c) return ASH_EINVAL;
  int rc = use_device(c);
  if (rc) return rc;
  double ms[4] = {0, 0, 0, 0};
  int64_t n[4] = {0, 0, 0, 0};
  hipError_t e = hipStreamSynchronize(c->stream);
  for (auto& r : c->prof) {
    float t = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, r.start, r.stop);
    if (r.cat >= 0 && r.cat < 4) {
      ms[r.cat] += t;
      n[r.cat] += 1;
    }
  }
  prof_release(c);
  if (e != hipSuccess) return hip_fail(c, e, "reading kernel timings");
  for (int k = 0; k < 4; ++k) {
    if (ms_out) ms_out[k] = ms[k];
    if (launches_out) launches_out[k] = n[k];
  }
  return ASH_OK;
}

}  // extern "C"
