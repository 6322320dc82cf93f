// Host side of libash: the C ABI declared in include/ash.h, argument
// validation, device memory management and the Zernike -> monomial
// expansion used to hand a basis to ash_set_basis.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <map>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "ash.h"
#include "internal.h"

using namespace ash;

namespace {

// Armed failure injections (ash_inject_failure), process-wide.
std::atomic<int> g_inject_alloc{0};
std::atomic<int> g_inject_barrier{0};

bool consume(std::atomic<int>& armed) {
  int n = armed.load();
  while (n > 0 && !armed.compare_exchange_weak(n, n - 1)) {
  }
  return n > 0;
}

}  // namespace

namespace ash {
bool injected_alloc_failure() { return consume(g_inject_alloc); }
bool injected_barrier_failure() { return consume(g_inject_barrier); }
}  // namespace ash

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
  if (hipEventCreateWithFlags(&e, kProfEventFlags) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return e;
}

// Enqueue `launch` bracketed by events of category `cat` when profiling.
template <typename F>
hipError_t timed(ash_ctx* c, int cat, F&& launch) {
  if (!(c->prof_mask & (1 << cat))) return launch();
  if (c->prof_seen[cat]++ % c->prof_stride != 0) return launch();
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
  if (injected_alloc_failure()) {
    c->err = std::string("out of device memory allocating ") + what +
             " (injected)";
    return ASH_ENOMEM;
  }
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
  dfree(b.bound);
  dfree(b.partial);
  dfree(b.red);
  dfree(b.mom_partial);
  dfree(b.fixph);
  b.cap_spots = b.cap_spotrec = b.cap_w = b.cap_off = b.cap_partial =
      b.cap_red = b.cap_mom = 0;
  c->has_spots = false;
  c->has_fixed = false;
  c->spots = Spots();
}

void free_basis(ash_ctx* c) {
  free_spots(c);
  Buffers& b = c->buf;
  dfree(b.pixtab);
  dfree(b.amp_t);
  dfree(b.field_t);
  dfree(b.fmag_t);
  dfree(b.aff_dev);
  dfree(b.nlmode_dev);
  dfree(b.tilez);
  dfree(b.rmax);
  dfree(b.d_pow);
  dfree(b.d_nlcoef);
  dfree(b.d_coef);
  dfree(b.momtab);
  dfree(b.grad);
  dfree(b.tvp);
  dfree(b.lossbuf);
  b.cap_pixtab = 0;
  c->has_basis = false;
  c->basis = Basis();
}

// (Re)build the pixel table for the geometry's record shape; the tile-order
// amplitude is written only when `with_amp` (from amp_dev, or 1 if NULL).
int build_pixtab(ash_ctx* c, const float* amp_dev, bool with_amp) {
  Buffers& B = c->buf;
  const Geom& g = c->basis.g;
  const size_t need = (size_t)g.n_tiles * g.groups * 2 * kTile * 8;
  if (need > B.cap_pixtab) {
    dfree(B.pixtab);
    B.cap_pixtab = 0;
    int rc = dalloc(c, &B.pixtab, need, "basis table");
    if (rc) return rc;
    B.cap_pixtab = need;
  }
  HIPCHK(c, launch_build_pixtab(g, B.d_pow, B.d_nlcoef, c->basis.n_mono,
                                amp_dev, B.pixtab,
                                with_amp ? B.amp_t : nullptr, c->stream),
         "building basis table");
  return ASH_OK;
}

template <typename T>
int grow(ash_ctx* c, T** p, size_t* cap, size_t need, const char* what) {
  if (need <= *cap) return ASH_OK;
  dfree(*p);
  *cap = 0;
  int rc = dalloc(c, p, need, what);
  if (rc) return rc;
  *cap = need;
  return ASH_OK;
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

// Remainder phases below this bound (turns) use 2 bf16 pieces: the dropped
// piece products stay below 2^-16 of it, 7.6e-6 turns.
constexpr float kTwoPieceBound = 0.5f;

// Phases bounded by this many turns skip the explicit range reduction: the
// hardware sine and cosine reduce exactly over |x| <= 256 turns.
constexpr float kNoReduceBound = 64.0f;

// Largest in-tile phase (turns) the FP32 accumulation of the phase keeps
// within the field bar: its rounding error grows about 2e-7 relative per
// turn of the bound (measured: 4.9e-5 at 215 turns, 8.6e-5 at 425, 1.2e-4
// at 845).  A bound above this means kernel phases that change by several
// turns between neighbouring pixels of a 32 x 16 tile: kernels aliased many
// times over, which are refused rather than computed inaccurately.
constexpr float kMaxPhaseBound = 256.0f;

}  // namespace

extern "C" {

int ash_version(void) { return 100; }

int ash_inject_failure(int what, int count) {
  if (count < 0) return ASH_EINVAL;
  switch (what) {
    case ASH_INJECT_ALLOC:
      g_inject_alloc.store(count);
      return ASH_OK;
    case ASH_INJECT_BARRIER:
      g_inject_barrier.store(count);
      return ASH_OK;
    default:
      return ASH_EINVAL;
  }
}

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
  // the device address of the allocation-free forward's scratch
  e = resolve_static_scratch(device);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return create_fail(ASH_EHIP, std::string("resolving the static scratch: ") +
                                     hipGetErrorString(e));
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
  {
    const char* why = "";
    const int rc0 = ash_check_basis(nx, ny, cx, cy, R, D, n_mono, mono_pow,
                                    mono_coef, &why);
    if (rc0) return fail(c, rc0, why);
  }

  Basis b;
  Geom& g = b.g;
  g.nx = nx;
  g.ny = ny;
  g.cx = cx;
  g.cy = cy;
  g.R = R;
  g.D = D;
  b.n_mono = n_mono;
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
  g.nl = (int)b.nl_mode.size();
  if (g.nl > ASH_MAX_NONLINEAR)
    return fail(c, ASH_EUNSUPPORTED, "too many non-linear modes");
  g.pieces = 2;
  g.groups = groups_for(g.nl, g.pieces);
  g.tiles_x = (nx + kTileW - 1) / kTileW;
  g.tiles_y = (ny + kTileH - 1) / kTileH;
  g.n_tiles = g.tiles_x * g.tiles_y;

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
  c->basis = b;
  Buffers& B = c->buf;
  const size_t npix = (size_t)g.n_tiles * kTile;
  const size_t nl1 = (size_t)std::max(g.nl, 1);
  if ((rc = dalloc(c, &B.amp_t, npix, "amplitude")) ||
      (rc = dalloc(c, &B.field_t, 8 * npix, "nearfield")) ||
      (rc = dalloc(c, &B.fmag_t, npix, "nearfield magnitudes")) ||
      (rc = dalloc(c, &B.aff_dev, 3 * (size_t)D, "basis affine terms")) ||
      (rc = dalloc(c, &B.nlmode_dev, nl1, "modes")) ||
      (rc = dalloc(c, &B.tilez, 3 * (size_t)g.n_tiles * nl1, "tile basis")) ||
      (rc = dalloc(c, &B.rmax, (size_t)g.n_tiles * nl1, "tile bounds")) ||
      (rc = dalloc(c, &B.d_pow, 2 * (size_t)n_mono, "monomials")) ||
      (rc = dalloc(c, &B.d_nlcoef, std::max(nlcoef.size(), (size_t)1),
                   "monomial coefficients")) ||
      (rc = dalloc(c, &B.d_coef, (size_t)D * n_mono, "basis coefficients")) ||
      (rc = dalloc(c, &B.momtab, npix * 2 * (size_t)D, "moment table")) ||
      (rc = dalloc(c, &B.grad, P, "gradient")) ||
      (rc = dalloc(c, &B.tvp, (size_t)g.n_tiles * kBlkPerTile, "TV sums")) ||
      (rc = dalloc(c, &B.lossbuf, 1, "loss"))) {
    free_basis(c);
    return rc;
  }
  hipError_t e = hipMemcpyAsync(B.d_pow, mono_pow,
                                2 * n_mono * sizeof(int32_t),
                                hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess && !nlcoef.empty())
    e = hipMemcpyAsync(B.d_nlcoef, nlcoef.data(),
                       nlcoef.size() * sizeof(double), hipMemcpyHostToDevice,
                       c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(B.aff_dev, b.aff.data(), 3 * D * sizeof(double),
                       hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(B.d_coef, mono_coef, (size_t)D * n_mono * sizeof(double),
                       hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess && g.nl > 0)
    e = hipMemcpyAsync(B.nlmode_dev, b.nl_mode.data(), g.nl * sizeof(int),
                       hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess)
    e = launch_build_tilebasis(g, B.d_pow, B.d_nlcoef, n_mono, B.tilez,
                               B.rmax, c->stream);
  if (e != hipSuccess) {
    free_basis(c);
    return hip_fail(c, e, "building basis table");
  }
  rc = build_pixtab(c, amp_dev, true);
  if (rc == ASH_OK) {
    e = launch_build_momtab(g, B.d_pow, B.d_coef, n_mono, B.amp_t, B.momtab,
                            c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) rc = hip_fail(c, e, "building basis table");
  }
  if (rc) {
    std::string msg = c->err;
    free_basis(c);
    c->err = msg;
    return rc;
  }
  c->has_basis = true;
  return ASH_OK;
}

int ash_set_precision(ash_ctx* c, int mode) {
  if (!c) return ASH_EINVAL;
  if (mode != ASH_PRECISION_AUTO && mode != ASH_PRECISION_FULL)
    return fail(c, ASH_EINVAL, "unknown precision mode");
  c->precision = mode;
  return ASH_OK;
}

int ash_get_info(const ash_ctx* c, ash_info* out) {
  if (!c || !out) return ASH_EINVAL;
  out->n_tiles = c->basis.g.n_tiles;
  out->nonlinear = c->basis.g.nl;
  out->pieces = c->basis.g.pieces;
  out->groups = c->basis.g.groups;
  out->fwd_ranges = c->plan.groups;
  out->rm_bound = c->spots.rm_bound;
  out->theta_bound = c->spots.theta_bound;
  out->range_reduce = c->basis.g.reduce;
  return ASH_OK;
}

int ash_set_spots(ash_ctx* c, int N, const double* w_host,
                  const float* target_host) {
  if (!c) return ASH_EINVAL;
  c->err.clear();
  if (!c->has_basis) return fail(c, ASH_ENOTREADY, "set the basis first");
  Geom& g = c->basis.g;
  const char* why = "";
  int rc = ash_check_spots(N, g.D, w_host, target_host, &why);
  if (rc) return fail(c, rc, why);
  const size_t nw = (size_t)N * g.D;
  std::vector<float> t(N, 1.0f);
  double tn2 = 0.0;
  for (int k = 0; k < N; ++k) {
    if (target_host) t[k] = target_host[k];
    tn2 += (double)t[k] * t[k];
  }
  rc = use_device(c);
  if (rc) return rc;
  c->has_spots = false;
  Buffers& B = c->buf;
  const size_t n_blk32 = ((size_t)N + 31) / 32, n_pad = n_blk32 * 32;
  if ((size_t)N > B.cap_spots) {  // per-spot buffers share one capacity
    dfree(B.target);
    dfree(B.y);
    dfree(B.Ebuf);
    dfree(B.spot64);
    dfree(B.fixph);
    B.cap_spots = 0;
    if ((rc = dalloc(c, &B.target, (size_t)N, "targets")) ||
        (rc = dalloc(c, &B.y, 9 * n_pad, "spot fields")) ||
        (rc = dalloc(c, &B.fixph, n_pad, "fixed phases")) ||
        (rc = dalloc(c, &B.Ebuf, 2 * (size_t)N, "spot fields")) ||
        (rc = dalloc(c, &B.spot64, 3 * (size_t)N, "spot offsets")))
      goto fail_alloc;
    B.cap_spots = N;
  }
  if (!B.bound && (rc = dalloc(c, &B.bound, 2, "bound"))) goto fail_alloc;
  if ((rc = grow(c, &B.w64, &B.cap_w, nw, "coefficients")) ||
      (rc = grow(c, &B.offtab, &B.cap_off, (size_t)g.n_tiles * 2 * n_pad * 4,
                 "tile offsets")) ||
      (rc = grow(c, &B.spotrec, &B.cap_spotrec,
                 n_blk32 * kMaxGroups * 2 * 32 * 8, "spot records")))
    goto fail_alloc;
  {
    hipError_t e = hipMemcpyAsync(B.w64, w_host, nw * sizeof(double),
                                  hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(B.target, t.data(), N * sizeof(float),
                         hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(B.bound, 0, 8, c->stream);
    // spot-field records: the padding past N stays zero
    if (e == hipSuccess)
      e = hipMemsetAsync(B.y, 0, 9 * n_pad * sizeof(unsigned), c->stream);
    if (e == hipSuccess)
      e = launch_prep_spots(g, N, B.w64, B.aff_dev, B.nlmode_dev, B.tilez,
                            B.rmax, B.spotrec, B.spot64, B.offtab, B.bound,
                            c->stream);
    unsigned bound_bits[2] = {0u, 0u};
    if (e == hipSuccess)
      e = hipMemcpyAsync(bound_bits, B.bound, 8, hipMemcpyDeviceToHost,
                         c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "preparing spots");
    float bound, theta_bound;
    memcpy(&bound, &bound_bits[0], 4);
    memcpy(&theta_bound, &bound_bits[1], 4);
    c->spots.rm_bound = bound;
    c->spots.theta_bound = theta_bound;
    if (!(theta_bound <= kMaxPhaseBound))
      return fail(c, ASH_EUNSUPPORTED,
                  "in-tile phase bound " + std::to_string(theta_bound) +
                      " turns exceeds " + std::to_string(kMaxPhaseBound) +
                      ": kernels aliased between neighbouring pixels "
                      "(lower the coefficients or raise R)");
    g.reduce = theta_bound <= kNoReduceBound ? 0 : 1;
    const int pieces =
        (c->precision == ASH_PRECISION_AUTO && bound <= kTwoPieceBound) ? 2
                                                                        : 3;
    if (pieces != g.pieces) {
      // a different record shape: rebuild the basis table and the records
      Geom g2 = g;
      g2.pieces = pieces;
      g2.groups = groups_for(g.nl, pieces);
      if (g2.groups > kMaxGroups)
        return fail(c, ASH_EUNSUPPORTED, "record too long");
      const Geom old = g;
      g = g2;
      if ((rc = build_pixtab(c, nullptr, false))) {
        g = old;
        return rc;
      }
      e = launch_prep_spots(g, N, B.w64, B.aff_dev, B.nlmode_dev, B.tilez,
                            B.rmax, B.spotrec, B.spot64, B.offtab, B.bound,
                            c->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
      if (e != hipSuccess) return hip_fail(c, e, "preparing spots");
    }
  }
  {
    FwdPlan plan = plan_forward(g.n_tiles, N, forward_blocks_per_cu(g.groups),
                                c->n_cu);
    plan.mom_groups = plan_moment_ranges(
        g.n_tiles, N, moments_blocks_per_cu(g.groups, g.D), c->n_cu);
    if ((rc = grow(c, &B.partial, &B.cap_partial,
                   (size_t)plan.groups * N * 2, "partial sums")) ||
        (rc = grow(c, &B.red, &B.cap_red, (size_t)plan.slices * N * 2,
                   "partial sums")) ||
        (rc = grow(c, &B.mom_partial, &B.cap_mom,
                   (size_t)plan.mom_groups * 2 * g.D * n_pad * 2,
                   "moment sums")))
      goto fail_alloc;
    c->plan = plan;
  }
  c->spots.N = N;
  c->spots.t_norm2 = tn2;
  c->has_spots = true;
  c->has_fixed = false;  // stored farfield phases belong to the old spots
  return ASH_OK;
fail_alloc:
  free_spots(c);
  return rc;
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
  const Geom& g = c->basis.g;
  Buffers& B = c->buf;
  const int N = c->spots.N;
  HIPCHK(c, timed(c, ASH_PROF_FIELD, [&] {
           return launch_make_field(g, phase_dev, field_dev, B.amp_t,
                                    B.pixtab, B.field_t,
                                    field_dev ? B.fmag_t : nullptr, c->stream);
         }), "make_field");
  HIPCHK(c, timed(c, ASH_PROF_FORWARD, [&] {
           return launch_forward(g, N, c->plan, B.pixtab, B.field_t,
                                 field_dev ? B.fmag_t : B.amp_t, B.spotrec,
                                 B.offtab, B.partial, c->stream);
         }), "forward");
  HIPCHK(c, timed(c, ASH_PROF_REDUCE, [&] {
           return launch_reduce(N, c->plan, B.partial, B.red, c->stream);
         }), "reduce");
  HIPCHK(c, timed(c, ASH_PROF_REDUCE, [&] {
           return launch_finish_E(N, c->plan, B.red, E_dev, c->stream);
         }), "finish");
  return ASH_OK;
}

int ash_forward_noalloc(ash_ctx* c, const float* phase_dev,
                        const float* field_dev, float* E_dev) {
  if (!c) return ASH_EINVAL;
  c->err.clear();
  if (!c->has_basis || !c->has_spots)
    return fail(c, ASH_ENOTREADY, "basis and spots must be set");
  if ((phase_dev == nullptr) == (field_dev == nullptr) || !E_dev)
    return fail(c, ASH_EINVAL, "exactly one of phase/field, and E, required");
  const int N = c->spots.N;
  // partial sums [ranges][N] and their reduction [N], both float2, the
  // reduction starting on a 256-byte boundary
  const size_t part_bytes = (size_t)c->plan.groups * N * 2 * sizeof(float);
  const size_t red_off = (part_bytes + 255) / 256 * 256;
  const size_t need = red_off + (size_t)N * 2 * sizeof(float);
  if (need > kStaticScratchBytes)
    return fail(c, ASH_EUNSUPPORTED,
                "the static scratch holds " +
                    std::to_string(kStaticScratchBytes) + " bytes; this "
                    "set-up's partial sums need " + std::to_string(need));
  unsigned char* scr = static_cast<unsigned char*>(static_scratch(c->device));
  if (!scr) return fail(c, ASH_EHIP, "static scratch not resolved");
  int rc = use_device(c);
  if (rc) return rc;
  const Geom& g = c->basis.g;
  Buffers& B = c->buf;
  float* partial = reinterpret_cast<float*>(scr);
  float* red = reinterpret_cast<float*>(scr + red_off);
  HIPCHK(c, timed(c, ASH_PROF_FIELD, [&] {
           return launch_make_field(g, phase_dev, field_dev, B.amp_t,
                                    B.pixtab, B.field_t,
                                    field_dev ? B.fmag_t : nullptr, c->stream);
         }), "make_field");
  HIPCHK(c, timed(c, ASH_PROF_FORWARD, [&] {
           return launch_forward(g, N, c->plan, B.pixtab, B.field_t,
                                 field_dev ? B.fmag_t : B.amp_t, B.spotrec,
                                 B.offtab, partial, c->stream);
         }), "forward");
  HIPCHK(c, timed(c, ASH_PROF_REDUCE, [&] {
           return launch_reduce(N, c->plan, partial, red, c->stream);
         }), "reduce");
  HIPCHK(c, timed(c, ASH_PROF_REDUCE, [&] {
           return launch_finish_E(N, c->plan, red, E_dev, c->stream);
         }), "finish");
  return ASH_OK;
}

// Basis moments of the forward, and with G the coefficient gradient; both
// take the phase with the context's amplitude.
static int moments(ash_ctx* c, const float* phase_dev, const float* G_dev,
                   float* M_dev, float* grad_dev) {
  int rc = use_device(c);
  if (rc) return rc;
  const Geom& g = c->basis.g;
  Buffers& B = c->buf;
  const int N = c->spots.N;
  HIPCHK(c, timed(c, ASH_PROF_FIELD, [&] {
           return launch_make_field(g, phase_dev, nullptr, B.amp_t, B.pixtab,
                                    B.field_t, nullptr, c->stream);
         }), "make_field");
  HIPCHK(c, timed(c, ASH_PROF_FORWARD, [&] {
           return launch_moments(g, N, c->plan.mom_groups, B.pixtab,
                                 B.field_t, B.spotrec, B.offtab, B.momtab,
                                 B.mom_partial, c->stream);
         }), "moments");
  HIPCHK(c, timed(c, ASH_PROF_REDUCE, [&] {
           return launch_moments_finish(N, g.D, c->plan.mom_groups,
                                        B.mom_partial, G_dev, M_dev, grad_dev,
                                        c->stream);
         }), "moments finish");
  return ASH_OK;
}

int ash_forward_moments(ash_ctx* c, const float* phase_dev, float* M_dev) {
  if (!c) return ASH_EINVAL;
  c->err.clear();
  if (!c->has_basis || !c->has_spots)
    return fail(c, ASH_ENOTREADY, "basis and spots must be set");
  if (!phase_dev || !M_dev) return fail(c, ASH_EINVAL, "phase and M required");
  return moments(c, phase_dev, nullptr, M_dev, nullptr);
}

int ash_coef_grad(ash_ctx* c, const float* phase_dev, const float* G_dev,
                  float* grad_dev) {
  if (!c) return ASH_EINVAL;
  c->err.clear();
  if (!c->has_basis || !c->has_spots)
    return fail(c, ASH_ENOTREADY, "basis and spots must be set");
  if (!phase_dev || !G_dev || !grad_dev)
    return fail(c, ASH_EINVAL, "phase, G and grad required");
  return moments(c, phase_dev, G_dev, nullptr, grad_dev);
}

int ash_window_coefficients(int N, int D, const double* w, int ix, int iy,
                            int nx, int ny, double R, double step, int win,
                            double* w_out) {
  if (N < 1 || D < 1 || !w || !w_out || win < 1 || win % 2 == 0 || ix < 0 ||
      iy < 0 || ix >= D || iy >= D || ix == iy || nx < 1 || ny < 1 ||
      !isfinite(R) || !(R > 0.0) || !isfinite(step))
    return ASH_EINVAL;
  if ((long)N * win * win > ASH_MAX_SPOTS) return ASH_EUNSUPPORTED;
  // one DFT bin along x is a phase slope of 2 pi / nx per pixel; the tilt
  // Z = 2 xh = 2 (i - cx) / R has slope 2 / R per unit coefficient
  const double dwx = M_PI * step * R / nx, dwy = M_PI * step * R / ny;
  const int h = win / 2;
  for (int k = 0; k < N; ++k)
    for (int b = 0; b < win; ++b)
      for (int a = 0; a < win; ++a) {
        double* row = w_out + (((long)k * win + b) * win + a) * D;
        for (int d = 0; d < D; ++d) row[d] = w[(long)k * D + d];
        row[ix] += (a - h) * dwx;
        row[iy] += (b - h) * dwy;
      }
  return ASH_OK;
}

int ash_window_strehl(ash_ctx* c, const float* phase_dev, int n_windows,
                      int win, float* S_dev) {
  if (!c) return ASH_EINVAL;
  c->err.clear();
  if (!c->has_basis || !c->has_spots)
    return fail(c, ASH_ENOTREADY, "basis and spots must be set");
  if (!phase_dev || !S_dev || n_windows < 1 || win < 1)
    return fail(c, ASH_EINVAL, "phase, S, n_windows >= 1 and win >= 1 required");
  if ((long)n_windows * win * win != c->spots.N)
    return fail(c, ASH_ESHAPE, "spots must be n_windows * win * win");
  int rc = use_device(c);
  if (rc) return rc;
  const Geom& g = c->basis.g;
  Buffers& B = c->buf;
  const int N = c->spots.N;
  HIPCHK(c, timed(c, ASH_PROF_FIELD, [&] {
           return launch_make_field(g, phase_dev, nullptr, B.amp_t, B.pixtab,
                                    B.field_t, nullptr, c->stream);
         }), "make_field");
  HIPCHK(c, timed(c, ASH_PROF_FORWARD, [&] {
           return launch_forward(g, N, c->plan, B.pixtab, B.field_t, B.amp_t,
                                 B.spotrec, B.offtab, B.partial, c->stream);
         }), "forward");
  HIPCHK(c, timed(c, ASH_PROF_REDUCE, [&] {
           return launch_reduce(N, c->plan, B.partial, B.red, c->stream);
         }), "reduce");
  HIPCHK(c, timed(c, ASH_PROF_REDUCE, [&] {
           return launch_finish_E(N, c->plan, B.red, B.Ebuf, c->stream);
         }), "finish");
  HIPCHK(c, timed(c, ASH_PROF_REDUCE, [&] {
           return launch_window_strehl(n_windows, win * win, B.Ebuf, S_dev,
                                       c->stream);
         }), "window strehl");
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
  Buffers& B = c->buf;
  const int outs = (g_dev ? kOutG : 0) | (phase_out_dev ? kOutPhase : 0);
  HIPCHK(c, timed(c, ASH_PROF_REDUCE, [&] {
           return launch_to_polar(c->spots.N, y_dev, B.y, c->stream);
         }), "to_polar");
  HIPCHK(c, timed(c, ASH_PROF_ADJOINT, [&] {
           AdjOut o;
           o.outs = outs;
           o.g = g_dev;
           o.phase = phase_out_dev;
           return launch_adjoint(c->basis.g, c->spots.N, B.pixtab, B.spotrec,
                                 B.offtab, B.y, B.amp_t, o, c->stream);
         }), "adjoint");
  return ASH_OK;
}

// n_iter weighted-GS iterations; meas (one iteration) replaces |E| in the
// weight update.
static int wgs_loop(ash_ctx* c, float* phase_dev, float* weights_dev,
                    int n_iter, const ash_wgs_params* params, float* E_dev,
                    float* stats_dev, const float* meas_dev) {
  if (!c) return ASH_EINVAL;
  c->err.clear();
  if (!c->has_basis || !c->has_spots)
    return fail(c, ASH_ENOTREADY, "basis and spots must be set");
  if (!phase_dev || !weights_dev || n_iter < 0)
    return fail(c, ASH_EINVAL, "phase, weights and n_iter >= 0 required");
  const float power = params ? params->power : 1.0f;
  const int fix_after = params ? params->fix_phase_after : 0;
  if (!isfinite(power)) return fail(c, ASH_EINVAL, "power must be finite");
  if (fix_after < 0 && !c->has_fixed)
    return fail(c, ASH_ENOTREADY, "no stored farfield phases to fix");
  if (n_iter == 0) return ASH_OK;
  int rc = use_device(c);
  if (rc) return rc;
  const Geom& g = c->basis.g;
  Buffers& B = c->buf;
  const int N = c->spots.N;
  const float t_norm = (float)sqrt(c->spots.t_norm2);
  const float eff_denom = (float)((double)g.nx * g.ny * c->basis.amp_sum2);
  HIPCHK(c, timed(c, ASH_PROF_FIELD, [&] {
           return launch_make_field(g, phase_dev, nullptr, B.amp_t,
                                    B.pixtab, B.field_t, nullptr, c->stream);
         }), "make_field");
  for (int it = 0; it < n_iter; ++it) {
    const bool last = it == n_iter - 1;
    // fix_phase_after = n > 0: iterations 0 .. n-1 free, n-1 stores its
    // phases, n .. use them; < 0: every iteration uses stored phases
    const int mode = fix_after < 0        ? kPhaseFixed
                     : fix_after == 0     ? kPhaseFree
                     : it < fix_after - 1 ? kPhaseFree
                     : it == fix_after - 1 ? kPhaseStore
                                           : kPhaseFixed;
    HIPCHK(c, timed(c, ASH_PROF_FORWARD, [&] {
             return launch_forward(g, N, c->plan, B.pixtab, B.field_t, B.amp_t,
                                   B.spotrec, B.offtab, B.partial, c->stream);
           }), "forward");
    HIPCHK(c, timed(c, ASH_PROF_REDUCE, [&] {
             return launch_reduce(N, c->plan, B.partial, B.red, c->stream);
           }), "reduce");
    HIPCHK(c, timed(c, ASH_PROF_REDUCE, [&] {
             return launch_wgs_update(
                 N, c->plan, B.red, B.target, t_norm, weights_dev, power,
                 eff_denom, B.y, B.Ebuf, last ? E_dev : nullptr,
                 stats_dev ? stats_dev + 4 * (size_t)it : nullptr, meas_dev,
                 B.fixph, mode, c->stream);
           }), "wgs_update");
    if (mode == kPhaseStore) c->has_fixed = true;
    HIPCHK(c, timed(c, ASH_PROF_ADJOINT, [&] {
             AdjOut o;
             o.outs = last ? kOutPhase : kOutField;
             o.phase = last ? phase_dev : nullptr;
             o.nf_t = last ? nullptr : B.field_t;
             return launch_adjoint(g, N, B.pixtab, B.spotrec, B.offtab, B.y,
                                   B.amp_t, o, c->stream);
           }), "adjoint");
  }
  return ASH_OK;
}

int ash_wgs_iterate(ash_ctx* c, float* phase_dev, float* weights_dev,
                    int n_iter, const ash_wgs_params* params, float* E_dev,
                    float* stats_dev) {
  return wgs_loop(c, phase_dev, weights_dev, n_iter, params, E_dev, stats_dev,
                  nullptr);
}

int ash_get_fixed_phases(ash_ctx* c, float* psi_dev) {
  if (!c) return ASH_EINVAL;
  c->err.clear();
  if (!psi_dev) return fail(c, ASH_EINVAL, "psi required");
  if (!c->has_spots || !c->has_fixed)
    return fail(c, ASH_ENOTREADY, "no stored farfield phases");
  int rc = use_device(c);
  if (rc) return rc;
  HIPCHK(c, hipMemcpyAsync(psi_dev, c->buf.fixph, c->spots.N * sizeof(float),
                           hipMemcpyDeviceToDevice, c->stream),
         "copying phases");
  return ASH_OK;
}

int ash_set_fixed_phases(ash_ctx* c, const float* psi_dev) {
  if (!c) return ASH_EINVAL;
  c->err.clear();
  if (!psi_dev) return fail(c, ASH_EINVAL, "psi required");
  if (!c->has_spots) return fail(c, ASH_ENOTREADY, "spots must be set");
  int rc = use_device(c);
  if (rc) return rc;
  HIPCHK(c, hipMemcpyAsync(c->buf.fixph, psi_dev, c->spots.N * sizeof(float),
                           hipMemcpyDeviceToDevice, c->stream),
         "copying phases");
  c->has_fixed = true;
  return ASH_OK;
}

int ash_wgs_feedback(ash_ctx* c, float* phase_dev, float* weights_dev,
                     const float* measured_dev, const ash_wgs_params* params,
                     float* E_dev, float* stats_dev) {
  if (c && !measured_dev) {
    c->err.clear();
    return fail(c, ASH_EINVAL, "measured amplitudes required");
  }
  return wgs_loop(c, phase_dev, weights_dev, 1, params, E_dev, stats_dev,
                  measured_dev);
}

int ash_phase_grad(ash_ctx* c, const float* phase_dev, const float* G_dev,
                   float* grad_dev) {
  if (!c) return ASH_EINVAL;
  c->err.clear();
  if (!c->has_basis || !c->has_spots)
    return fail(c, ASH_ENOTREADY, "basis and spots must be set");
  if (!phase_dev || !G_dev || !grad_dev)
    return fail(c, ASH_EINVAL, "phase, G and grad required");
  int rc = use_device(c);
  if (rc) return rc;
  Buffers& B = c->buf;
  HIPCHK(c, timed(c, ASH_PROF_REDUCE, [&] {
           return launch_to_polar(c->spots.N, G_dev, B.y, c->stream);
         }), "to_polar");
  HIPCHK(c, timed(c, ASH_PROF_ADJOINT, [&] {
           AdjOut o;
           o.outs = kOutGrad;
           o.phase_in = phase_dev;
           o.grad = grad_dev;
           return launch_adjoint(c->basis.g, c->spots.N, B.pixtab, B.spotrec,
                                 B.offtab, B.y, B.amp_t, o, c->stream);
         }), "adjoint");
  return ASH_OK;
}

int ash_adam_iterate(ash_ctx* c, float* phase_dev, float* m_dev, float* v_dev,
                     int step0, int n_steps, const ash_adam_params* params,
                     float* loss_dev, float* E_dev) {
  if (!c) return ASH_EINVAL;
  c->err.clear();
  if (!c->has_basis || !c->has_spots)
    return fail(c, ASH_ENOTREADY, "basis and spots must be set");
  if (!phase_dev || !m_dev || !v_dev || n_steps < 0 || step0 < 0)
    return fail(c, ASH_EINVAL,
                "phase, m, v required; n_steps and step0 must be >= 0");
  ash_adam_params pr = {0.05f, 0.9f, 0.999f, 1e-8f, 1e-3f, 1e-3f};
  if (params) pr = *params;
  if (!isfinite(pr.lr) || !(pr.beta1 >= 0.0f && pr.beta1 < 1.0f) ||
      !(pr.beta2 >= 0.0f && pr.beta2 < 1.0f) || !(pr.eps > 0.0f) ||
      !isfinite(pr.eps) || !isfinite(pr.tv_weight) || pr.tv_weight < 0.0f ||
      !(pr.tv_eps > 0.0f) || !isfinite(pr.tv_eps))
    return fail(c, ASH_EINVAL, "Adam parameters out of range");
  if (n_steps == 0) return ASH_OK;
  int rc = use_device(c);
  if (rc) return rc;
  const Geom& g = c->basis.g;
  Buffers& B = c->buf;
  const int N = c->spots.N;
  const double P = (double)g.nx * g.ny;
  if (!(c->basis.amp_sum2 > 0.0))
    return fail(c, ASH_EINVAL, "the source amplitude is zero everywhere");
  const float inv_s = (float)(1.0 / sqrt(P * c->basis.amp_sum2 / N));
  const int n_tvp = g.n_tiles * kBlkPerTile;
  HIPCHK(c, timed(c, ASH_PROF_FIELD, [&] {
           return launch_make_field(g, phase_dev, nullptr, B.amp_t,
                                    B.pixtab, B.field_t, nullptr, c->stream);
         }), "make_field");
  for (int it = 0; it < n_steps; ++it) {
    const int step = step0 + it + 1;
    const bool last = it == n_steps - 1;
    HIPCHK(c, timed(c, ASH_PROF_FORWARD, [&] {
             return launch_forward(g, N, c->plan, B.pixtab, B.field_t, B.amp_t,
                                   B.spotrec, B.offtab, B.partial, c->stream);
           }), "forward");
    HIPCHK(c, timed(c, ASH_PROF_REDUCE, [&] {
             return launch_reduce(N, c->plan, B.partial, B.red, c->stream);
           }), "reduce");
    HIPCHK(c, timed(c, ASH_PROF_REDUCE, [&] {
             return launch_spot_loss(N, c->plan, B.red, B.target, inv_s, B.y,
                                     last ? E_dev : nullptr, B.lossbuf,
                                     c->stream);
           }), "spot_loss");
    HIPCHK(c, timed(c, ASH_PROF_ADJOINT, [&] {
             AdjOut o;
             o.outs = kOutGrad;
             o.phase_in = phase_dev;
             o.grad = B.grad;
             o.tv_scale = (float)(pr.tv_weight / P);
             o.tv_eps = pr.tv_eps;
             o.tvp = loss_dev ? B.tvp : nullptr;
             return launch_adjoint(g, N, B.pixtab, B.spotrec, B.offtab, B.y,
                                   B.amp_t, o, c->stream);
           }), "adjoint");
    if (loss_dev)
      HIPCHK(c, timed(c, ASH_PROF_REDUCE, [&] {
               return launch_loss_finish(n_tvp, B.tvp,
                                         (float)(pr.tv_weight / P), B.lossbuf,
                                         loss_dev + it, c->stream);
             }), "loss");
    const float bc1 = (float)(1.0 - pow((double)pr.beta1, step));
    const float bc2 = (float)(1.0 - pow((double)pr.beta2, step));
    HIPCHK(c, timed(c, ASH_PROF_FIELD, [&] {
             return launch_adam(g, phase_dev, m_dev, v_dev, B.grad, pr.lr,
                                pr.beta1, pr.beta2, pr.eps, bc1, bc2, B.pixtab,
                                B.field_t, c->stream);
           }), "adam");
  }
  return ASH_OK;
}

int ash_profile_enable(ash_ctx* c, int mask) {
  if (!c) return ASH_EINVAL;
  if (mask & ~ASH_PROF_ALL) return fail(c, ASH_EINVAL, "unknown category bits");
  c->prof_mask = mask;
  for (long& n : c->prof_seen) n = 0;
  return ASH_OK;
}

int ash_profile_stride(ash_ctx* c, int stride) {
  if (!c) return ASH_EINVAL;
  if (stride < 1) return fail(c, ASH_EINVAL, "stride must be >= 1");
  c->prof_stride = stride;
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
