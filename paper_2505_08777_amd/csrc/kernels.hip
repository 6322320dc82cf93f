// Device kernels of libash: basis table, spot preparation, forward and
// adjoint spot transforms, reductions and the weighted-GS farfield update.
//
// Phases are carried in turns (1 turn = 2 pi rad).  Let Z^nl_s be the part
// of basis function s made of monomials of total degree >= 2.  For pixel x
// in tile t with anchor x0 (the pixel nearest the tile centre) and offsets
// (di, dj) = x - x0, each Z^nl_s is split, in FP64, into its value and
// gradient at x0 plus a remainder
//
//   Z^nl_s(x) = Z^nl_s(x0) + dZ/di(x0) di + dZ/dj(x0) dj + Rm_s(x),
//
// and the kernel phase of spot k becomes
//
//   tau_k(x) = off[t][k] + a[t][k] di + b[t][k] dj + sum_s c_k,s Rm_s(x)
//
// where off (wrapped into [0, 1) in FP64), a and b collect every constant
// and linear term at the anchor.  Only the small in-tile quantities
// enter FP32, so the FP32 phase stays within a few tens of turns wherever
// the kernels respect the Nyquist limit.  The hardware v_sin_f32 and
// v_cos_f32 take their argument in turns; tau is reduced to [0, 1) first.
#include <math.h>

#include "internal.h"

namespace ash {

int pad_nonlinear(int nl) {
  if (nl <= 16) return nl;
  if (nl <= 20) return 20;
  if (nl <= 24) return 24;
  return 28;
}

__host__ __device__ constexpr int rec_of(int nl) { return (nl + 2 + 3) & ~3; }

// Anchor of a tile: offsets di in [-32, 31], dj in [-8, 7].
constexpr int kAnchorI = kTileW / 2;
constexpr int kAnchorJ = kTileH / 2;

__device__ __forceinline__ void kahan_add(float& s, float& c, float x) {
  const float yv = x - c;
  const float t = s + yv;
  c = (t - s) - yv;
  s = t;
}

__device__ __forceinline__ double ipow(double x, int p) {
  double r = 1.0;
  for (int q = 0; q < p; ++q) r *= x;
  return r;
}

// ---------------------------------------------------------------------------
// Basis table, FP64 evaluation rounded once to FP32.
// ---------------------------------------------------------------------------
// Value and pixel-index gradient of the non-linear part of slot s at (x, y)
// (normalised coordinates).
__device__ void eval_nl(int s, int n_mono, const int32_t* __restrict__ pw,
                        const double* __restrict__ nlcoef, double invR,
                        double x, double y, double* v, double* di,
                        double* dj) {
  double sv = 0.0, sx = 0.0, sy = 0.0;
  for (int m = 0; m < n_mono; ++m) {
    const double c = nlcoef[s * n_mono + m];
    if (c == 0.0) continue;
    const int p = pw[2 * m], q = pw[2 * m + 1];
    const double xp = ipow(x, p), yq = ipow(y, q);
    sv += c * xp * yq;
    if (p > 0) sx += c * p * ipow(x, p - 1) * yq;
    if (q > 0) sy += c * q * xp * ipow(y, q - 1);
  }
  *v = sv;
  *di = sx * invR;
  *dj = sy * invR;
}

__global__ void k_build_pixtab(int nx, int ny, double cx, double cy,
                               double invR, int tiles_x, long total, int rec,
                               int nl, int n_mono,
                               const int32_t* __restrict__ pw,
                               const double* __restrict__ nlcoef,
                               const float* __restrict__ amp,
                               float* __restrict__ pixtab,
                               float* __restrict__ amp_t) {
  const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= total) return;
  const int tile = (int)(gid / kTile), pix = (int)(gid % kTile);
  const int i0 = (tile % tiles_x) * kTileW + kAnchorI;
  const int j0 = (tile / tiles_x) * kTileH + kAnchorJ;
  const int di = pix % kTileW - kAnchorI, dj = pix / kTileW - kAnchorJ;
  const int i = i0 + di, j = j0 + dj;
  const bool valid = i < nx && j < ny;
  float* r = pixtab + gid * rec;
  r[0] = (float)di;
  r[1] = (float)dj;
  const double xh = (i - cx) * invR, yh = (j - cy) * invR;
  const double x0 = (i0 - cx) * invR, y0 = (j0 - cy) * invR;
  for (int s = 0; s < rec - 2; ++s) {
    double rem = 0.0;
    if (s < nl && valid) {
      double v, gx, gy, v0, g0x, g0y;
      eval_nl(s, n_mono, pw, nlcoef, invR, xh, yh, &v, &gx, &gy);
      eval_nl(s, n_mono, pw, nlcoef, invR, x0, y0, &v0, &g0x, &g0y);
      rem = v - v0 - g0x * di - g0y * dj;
    }
    r[2 + s] = (float)rem;
  }
  amp_t[gid] = valid ? (amp ? amp[(long)j * nx + i] : 1.0f) : 0.0f;
}

// Value and gradient of every non-linear slot at every tile origin (FP64).
__global__ void k_build_tilebasis(double cx, double cy, double invR,
                                  int tiles_x, int n_tiles, int nl, int n_mono,
                                  const int32_t* __restrict__ pw,
                                  const double* __restrict__ nlcoef,
                                  double* __restrict__ tilez) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= n_tiles * nl) return;
  const int tile = gid / nl, s = gid % nl;
  const double x0 = ((tile % tiles_x) * kTileW + kAnchorI - cx) * invR;
  const double y0 = ((tile / tiles_x) * kTileH + kAnchorJ - cy) * invR;
  double v, gx, gy;
  eval_nl(s, n_mono, pw, nlcoef, invR, x0, y0, &v, &gx, &gy);
  tilez[3 * (long)gid] = v;
  tilez[3 * (long)gid + 1] = gx;
  tilez[3 * (long)gid + 2] = gy;
}

hipError_t launch_build_pixtab(const Basis& b, const int32_t* d_pow,
                               const double* d_nlcoef, int n_mono,
                               const float* amp_dev, float* pixtab,
                               float* amp_t, double* tilez, hipStream_t s) {
  const long total = (long)b.n_tiles * kTile;
  const int threads = 256;
  const long blocks = (total + threads - 1) / threads;
  hipLaunchKernelGGL(k_build_pixtab, dim3((unsigned)blocks), dim3(threads), 0,
                     s, b.nx, b.ny, b.cx, b.cy, 1.0 / b.R, b.tiles_x, total,
                     b.rec, b.nl, n_mono, d_pow, d_nlcoef, amp_dev, pixtab,
                     amp_t);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || b.nl == 0) return e;
  const int nt = b.n_tiles * b.nl;
  hipLaunchKernelGGL(k_build_tilebasis, dim3((nt + 255) / 256), dim3(256), 0,
                     s, b.cx, b.cy, 1.0 / b.R, b.tiles_x, b.n_tiles, b.nl,
                     n_mono, d_pow, d_nlcoef, tilez);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Spot preparation (FP64): per-spot non-linear coefficients in turns, and
// for every (tile, spot) the wrapped phase and the phase slopes of all
// constant and linear terms at the tile origin.
// ---------------------------------------------------------------------------
__global__ void k_spot_records(int N, int D, int nl, int rec, double invR,
                               const double* __restrict__ w,
                               const double* __restrict__ aff,
                               const int* __restrict__ nlmode,
                               float* __restrict__ spotrec,
                               double* __restrict__ spot64) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N) return;
  const double inv2pi = 0.15915494309189533577;
  double o = 0.0, a = 0.0, bb = 0.0;
  for (int d = 0; d < D; ++d) {
    const double wd = w[(long)k * D + d];
    o += wd * aff[3 * d];
    a += wd * aff[3 * d + 1];
    bb += wd * aff[3 * d + 2];
  }
  float* r = spotrec + (long)k * rec;
  r[0] = 0.0f;
  r[1] = 0.0f;
  for (int s = 0; s < rec - 2; ++s)
    r[2 + s] = s < nl ? (float)(w[(long)k * D + nlmode[s]] * inv2pi) : 0.0f;
  spot64[3 * (long)k] = o * inv2pi;
  spot64[3 * (long)k + 1] = a * inv2pi * invR;
  spot64[3 * (long)k + 2] = bb * inv2pi * invR;
}

__global__ void k_spot_offsets(int N, int D, int nl, int tiles_x, long total,
                               double cx, double cy,
                               const double* __restrict__ spot64,
                               const double* __restrict__ w,
                               const int* __restrict__ nlmode,
                               const double* __restrict__ tilez,
                               float4* __restrict__ offtab) {
  const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= total) return;
  const int tile = (int)(gid / N), k = (int)(gid % N);
  const double inv2pi = 0.15915494309189533577;
  const double i0 = (double)((tile % tiles_x) * kTileW + kAnchorI) - cx;
  const double j0 = (double)((tile / tiles_x) * kTileH + kAnchorJ) - cy;
  const double al = spot64[3 * (long)k + 1], be = spot64[3 * (long)k + 2];
  double t = spot64[3 * (long)k] + al * i0 + be * j0;
  double a = al, b = be;
  const double* tz = tilez + 3 * (long)tile * nl;
  for (int s = 0; s < nl; ++s) {
    const double c = w[(long)k * D + nlmode[s]] * inv2pi;
    t += c * tz[3 * s];
    a += c * tz[3 * s + 1];
    b += c * tz[3 * s + 2];
  }
  t -= floor(t);
  offtab[gid] = make_float4((float)t, (float)a, (float)b, 0.0f);
}

hipError_t launch_prep_spots(const Basis& b, int N, const double* d_w,
                             const double* d_aff, const int* d_nlmode,
                             const double* tilez, float* spotrec,
                             float* offtab, double* spot64, hipStream_t s) {
  hipLaunchKernelGGL(k_spot_records, dim3((N + 255) / 256), dim3(256), 0, s,
                     N, b.D, b.nl, b.rec, 1.0 / b.R, d_w, d_aff, d_nlmode,
                     spotrec, spot64);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const long total = (long)b.n_tiles * N;
  hipLaunchKernelGGL(k_spot_offsets, dim3((unsigned)((total + 255) / 256)),
                     dim3(256), 0, s, N, b.D, b.nl, b.tiles_x, total, b.cx,
                     b.cy, spot64, d_w, d_nlmode, tilez,
                     reinterpret_cast<float4*>(offtab));
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Nearfield in tile-major order: f = A exp(i phase), or a copied field.
// ---------------------------------------------------------------------------
__global__ void k_make_field(int nx, int ny, int tiles_x, long total,
                             const float* __restrict__ phase,
                             const float2* __restrict__ field,
                             const float* __restrict__ amp_t,
                             float2* __restrict__ field_t) {
  const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= total) return;
  const int tile = (int)(gid / kTile), pix = (int)(gid % kTile);
  const int i = (tile % tiles_x) * kTileW + pix % kTileW;
  const int j = (tile / tiles_x) * kTileH + pix / kTileW;
  float2 v = make_float2(0.0f, 0.0f);
  if (i < nx && j < ny) {
    const long p = (long)j * nx + i;
    if (phase) {
      float sn, cs;
      sincosf(phase[p], &sn, &cs);
      const float a = amp_t[gid];
      v = make_float2(a * cs, a * sn);
    } else {
      v = field[p];
    }
  }
  field_t[gid] = v;
}

hipError_t launch_make_field(const Basis& b, const float* phase,
                             const float* field, const float* amp_t,
                             float* field_t, hipStream_t s) {
  const long total = (long)b.n_tiles * kTile;
  hipLaunchKernelGGL(k_make_field, dim3((unsigned)((total + 255) / 256)),
                     dim3(256), 0, s, b.nx, b.ny, b.tiles_x, total, phase,
                     reinterpret_cast<const float2*>(field), amp_t,
                     reinterpret_cast<float2*>(field_t));
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Forward transform.  One lane per spot, 64 spots per wave; the pixel record
// and the nearfield value are wave-uniform and come through scalar loads.
// Each wave walks `tpg` consecutive tiles; per 64 pixels the block sum is
// added into a Kahan-compensated running total.  Output: partial[g][k].
// ---------------------------------------------------------------------------
template <int NL>
__global__ __launch_bounds__(kBlock) void k_forward(
    int N, int n_tiles, int tpg, const float* __restrict__ pixtab,
    const float2* __restrict__ field_t, const float* __restrict__ spotrec,
    const float4* __restrict__ offtab, float2* __restrict__ partial) {
  constexpr int E = NL + 2;
  constexpr int REC = rec_of(NL);
  const int lane = threadIdx.x & (kWave - 1);
  const int sg = blockIdx.y * (kBlock / kWave) + (threadIdx.x / kWave);
  if (sg * kWave >= N) return;  // wave-uniform exit; no barriers below
  const int k = sg * kWave + lane;
  const int kc = k < N ? k : N - 1;
  float c[E];
#pragma unroll
  for (int e = 0; e < E; ++e) c[e] = spotrec[(long)kc * REC + e];
  const int g = blockIdx.x;
  const int t0 = g * tpg;
  const int t1 = min(t0 + tpg, n_tiles);
  float sr = 0.0f, si = 0.0f, cr = 0.0f, ci = 0.0f;
  for (int t = t0; t < t1; ++t) {
    const float4 ot = offtab[(long)t * N + kc];
    c[0] = ot.y;  // tile slopes take the di, dj slots of the record
    c[1] = ot.z;
    const float off = ot.x;
    const float* __restrict__ rt = pixtab + (long)t * kTile * REC;
    const float2* __restrict__ ft = field_t + (long)t * kTile;
    for (int pb = 0; pb < kTile; pb += 64) {
      float br = 0.0f, bi = 0.0f;
#pragma unroll 4
      for (int p = pb; p < pb + 64; ++p) {
        const float* __restrict__ r = rt + p * REC;
        float tau = off;
#pragma unroll
        for (int e = 0; e < E; ++e) tau = fmaf(c[e], r[e], tau);
        tau = __builtin_amdgcn_fractf(tau);
        const float sn = __builtin_amdgcn_sinf(tau);
        const float cs = __builtin_amdgcn_cosf(tau);
        const float2 f = ft[p];
        // f * exp(-i theta) = (fr c + fi s) + i (fi c - fr s)
        br = fmaf(f.x, cs, br);
        br = fmaf(f.y, sn, br);
        bi = fmaf(f.y, cs, bi);
        bi = fmaf(-f.x, sn, bi);
      }
      kahan_add(sr, cr, br);
      kahan_add(si, ci, bi);
    }
  }
  if (k < N) partial[(long)g * N + k] = make_float2(sr, si);
}

template <int NL>
static hipError_t fwd_nl(dim3 grid, hipStream_t s, int N, int n_tiles, int tpg,
                         const float* pixtab, const float* field_t,
                         const float* spotrec, const float* offtab,
                         float* partial) {
  hipLaunchKernelGGL(k_forward<NL>, grid, dim3(kBlock), 0, s, N, n_tiles, tpg,
                     pixtab, reinterpret_cast<const float2*>(field_t), spotrec,
                     reinterpret_cast<const float4*>(offtab),
                     reinterpret_cast<float2*>(partial));
  return hipGetLastError();
}

#define ASH_NL_CASES(X) \
  X(0) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) \
  X(14) X(15) X(16) X(20) X(24) X(28)

hipError_t launch_forward(const Basis& b, int N, const FwdPlan& p,
                          const float* pixtab, const float* field_t,
                          const float* spotrec, const float* offtab,
                          float* partial, hipStream_t s) {
  const int n_sg = (N + kWave - 1) / kWave;
  const int waves_per_block = kBlock / kWave;
  dim3 grid(p.groups, (n_sg + waves_per_block - 1) / waves_per_block);
  switch (b.nl_pad) {
#define X(n)                                                                 \
  case n:                                                                    \
    return fwd_nl<n>(grid, s, N, b.n_tiles, p.tiles_per_group, pixtab,       \
                     field_t, spotrec, offtab, partial);
    ASH_NL_CASES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------------------
// Reductions of the forward partials (fixed order, compensated).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_reduce(int N, int groups, int rows,
                                               const float2* __restrict__ part,
                                               float2* __restrict__ red) {
  const int k = blockIdx.x * 64 + threadIdx.x;
  if (k >= N) return;
  const int g0 = blockIdx.y * rows;
  const int g1 = min(g0 + rows, groups);
  float sr = 0.0f, si = 0.0f, cr = 0.0f, ci = 0.0f;
  for (int g = g0; g < g1; ++g) {
    const float2 v = part[(long)g * N + k];
    kahan_add(sr, cr, v.x);
    kahan_add(si, ci, v.y);
  }
  red[(long)blockIdx.y * N + k] = make_float2(sr, si);
}

hipError_t launch_reduce(int N, const FwdPlan& p, const float* partial,
                         float* red, hipStream_t s) {
  dim3 grid((N + 63) / 64, p.slices);
  hipLaunchKernelGGL(k_reduce, grid, dim3(64), 0, s, N, p.groups,
                     p.rows_per_slice,
                     reinterpret_cast<const float2*>(partial),
                     reinterpret_cast<float2*>(red));
  return hipGetLastError();
}

__device__ __forceinline__ float2 sum_slices(const float2* __restrict__ red,
                                             int slices, int N, int k) {
  float sr = 0.0f, si = 0.0f, cr = 0.0f, ci = 0.0f;
  for (int q = 0; q < slices; ++q) {
    const float2 v = red[(long)q * N + k];
    kahan_add(sr, cr, v.x);
    kahan_add(si, ci, v.y);
  }
  return make_float2(sr, si);
}

__global__ void k_finish_E(int N, int slices, const float2* __restrict__ red,
                           float2* __restrict__ E) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < N) E[k] = sum_slices(red, slices, N, k);
}

hipError_t launch_finish_E(int N, const FwdPlan& p, const float* red, float* E,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_finish_E, dim3((N + 255) / 256), dim3(256), 0, s, N,
                     p.slices, reinterpret_cast<const float2*>(red),
                     reinterpret_cast<float2*>(E));
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Weighted-GS farfield update (one block).
// ---------------------------------------------------------------------------
constexpr int kUpd = 1024;

template <typename Op>
__device__ float block_reduce(float v, float* sh, Op op) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int w = kUpd / 2; w > 0; w >>= 1) {
    if (tid < w) sh[tid] = op(sh[tid], sh[tid + w]);
    __syncthreads();
  }
  const float r = sh[0];
  __syncthreads();
  return r;
}

struct OpSum {
  __device__ float operator()(float a, float b) const { return a + b; }
};
struct OpMax {
  __device__ float operator()(float a, float b) const { return fmaxf(a, b); }
};
struct OpMin {
  __device__ float operator()(float a, float b) const { return fminf(a, b); }
};

__global__ __launch_bounds__(kUpd) void k_wgs_update(
    int N, int slices, const float2* __restrict__ red,
    const float* __restrict__ t, float t_norm, float* __restrict__ W,
    float power, float eff_denom, float2* __restrict__ y,
    float2* __restrict__ Ebuf, float2* __restrict__ E_extra,
    float* __restrict__ stats) {
  __shared__ float sh[kUpd];
  const int tid = threadIdx.x;
  // pass 1: fields, |E|^2 and normalised intensities I = |E|^2 / t^2
  float s_a2 = 0.0f, s_I = 0.0f, mx = 0.0f, mn = INFINITY;
  for (int k = tid; k < N; k += kUpd) {
    const float2 e = sum_slices(red, slices, N, k);
    Ebuf[k] = e;
    if (E_extra) E_extra[k] = e;
    const float a2 = e.x * e.x + e.y * e.y;
    const float I = a2 / (t[k] * t[k]);
    s_a2 += a2;
    s_I += I;
    mx = fmaxf(mx, I);
    mn = fminf(mn, I);
  }
  const float sum_a2 = block_reduce(s_a2, sh, OpSum());
  const float sum_I = block_reduce(s_I, sh, OpSum());
  const float maxI = block_reduce(mx, sh, OpMax());
  const float minI = block_reduce(mn, sh, OpMin());
  const float norm_a = sqrtf(sum_a2);
  const float meanI = sum_I / (float)N;
  // pass 2: spread of I, unnormalised weight update
  float s_v = 0.0f, s_w = 0.0f;
  for (int k = tid; k < N; k += kUpd) {
    const float2 e = Ebuf[k];
    const float a2 = e.x * e.x + e.y * e.y;
    const float dI = a2 / (t[k] * t[k]) - meanI;
    s_v += dI * dI;
    const float a = sqrtf(a2);
    float wk = W[k];
    if (a > 0.0f && norm_a > 0.0f) {
      const float r = (a / norm_a) / (t[k] / t_norm);
      wk = (power == 1.0f) ? wk / r : wk * powf(r, -power);
    }
    W[k] = wk;
    s_w += wk;
  }
  const float var = block_reduce(s_v, sh, OpSum()) / (float)N;
  const float mean_w = block_reduce(s_w, sh, OpSum()) / (float)N;
  // pass 3: normalise weights, farfield projection y = W t E / |E|
  for (int k = tid; k < N; k += kUpd) {
    const float wk = W[k] / mean_w;
    W[k] = wk;
    const float2 e = Ebuf[k];
    const float a = sqrtf(e.x * e.x + e.y * e.y);
    const float amp = wk * t[k];
    y[k] = a > 0.0f ? make_float2(amp * (e.x / a), amp * (e.y / a))
                    : make_float2(amp, 0.0f);
  }
  if (stats && tid == 0) {
    stats[0] = eff_denom > 0.0f ? sum_a2 / eff_denom : 0.0f;
    stats[1] = (maxI + minI) > 0.0f ? 1.0f - (maxI - minI) / (maxI + minI)
                                    : 0.0f;
    stats[2] = meanI > 0.0f ? sqrtf(var) / meanI : 0.0f;
    stats[3] = sum_a2;
  }
}

hipError_t launch_wgs_update(int N, const FwdPlan& p, const float* red,
                             const float* target, float t_norm, float* W,
                             float power, float eff_denom, float* y,
                             float* Ebuf, float* E_extra, float* stats_row,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_wgs_update, dim3(1), dim3(kUpd), 0, s, N, p.slices,
                     reinterpret_cast<const float2*>(red), target, t_norm, W,
                     power, eff_denom, reinterpret_cast<float2*>(y),
                     reinterpret_cast<float2*>(Ebuf),
                     reinterpret_cast<float2*>(E_extra), stats_row);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Adjoint transform.  One block per tile, four pixels per lane; the spot
// record, y_k and the tile offset are wave-uniform (scalar loads).  Per 64
// spots the block sum is added into a Kahan-compensated total.  Epilogue:
// g, arg g, and/or the next nearfield A g/|g| in tile order.
// ---------------------------------------------------------------------------
constexpr int kAdjPx = kTile / kBlock;  // 4

template <int NL>
__global__ __launch_bounds__(kBlock) void k_adjoint(
    int N, int nx, int ny, int tiles_x, const float* __restrict__ pixtab,
    const float* __restrict__ spotrec, const float4* __restrict__ offtab,
    const float2* __restrict__ y, const float* __restrict__ amp_t, int outs,
    float2* __restrict__ g, float* __restrict__ phase,
    float2* __restrict__ field_t) {
  constexpr int E = NL + 2;
  constexpr int REC = rec_of(NL);
  const int tile = blockIdx.x;
  const int tid = threadIdx.x;
  float z[kAdjPx][E];
#pragma unroll
  for (int q = 0; q < kAdjPx; ++q) {
    const float* r = pixtab + ((long)tile * kTile + tid + kBlock * q) * REC;
#pragma unroll
    for (int e = 0; e < E; ++e) z[q][e] = r[e];
  }
  float gr[kAdjPx], gi[kAdjPx], cr[kAdjPx], ci[kAdjPx];
#pragma unroll
  for (int q = 0; q < kAdjPx; ++q) gr[q] = gi[q] = cr[q] = ci[q] = 0.0f;
  const float4* __restrict__ offrow = offtab + (long)tile * N;
  for (int k0 = 0; k0 < N; k0 += 64) {
    const int k1 = min(k0 + 64, N);
    float br[kAdjPx], bi[kAdjPx];
#pragma unroll
    for (int q = 0; q < kAdjPx; ++q) br[q] = bi[q] = 0.0f;
#pragma unroll 2
    for (int k = k0; k < k1; ++k) {
      const float* __restrict__ sr = spotrec + (long)k * REC;
      const float2 yk = y[k];
      const float4 ot = offrow[k];
#pragma unroll
      for (int q = 0; q < kAdjPx; ++q) {
        float tau = fmaf(ot.y, z[q][0], ot.x);
        tau = fmaf(ot.z, z[q][1], tau);
#pragma unroll
        for (int e = 2; e < E; ++e) tau = fmaf(sr[e], z[q][e], tau);
        tau = __builtin_amdgcn_fractf(tau);
        const float sn = __builtin_amdgcn_sinf(tau);
        const float cs = __builtin_amdgcn_cosf(tau);
        // y * exp(+i theta) = (yr c - yi s) + i (yr s + yi c)
        br[q] = fmaf(yk.x, cs, br[q]);
        br[q] = fmaf(-yk.y, sn, br[q]);
        bi[q] = fmaf(yk.x, sn, bi[q]);
        bi[q] = fmaf(yk.y, cs, bi[q]);
      }
    }
#pragma unroll
    for (int q = 0; q < kAdjPx; ++q) {
      kahan_add(gr[q], cr[q], br[q]);
      kahan_add(gi[q], ci[q], bi[q]);
    }
  }
  const int tx = tile % tiles_x, ty = tile / tiles_x;
#pragma unroll
  for (int q = 0; q < kAdjPx; ++q) {
    const int pix = tid + kBlock * q;
    const int i = tx * kTileW + pix % kTileW;
    const int j = ty * kTileH + pix / kTileW;
    if (outs & kOutField) {
      const float a = amp_t[(long)tile * kTile + pix];
      const float m = hypotf(gr[q], gi[q]);
      field_t[(long)tile * kTile + pix] =
          m > 0.0f ? make_float2(a * (gr[q] / m), a * (gi[q] / m))
                   : make_float2(a, 0.0f);
    }
    if (i < nx && j < ny) {
      const long p = (long)j * nx + i;
      if (outs & kOutG) g[p] = make_float2(gr[q], gi[q]);
      if (outs & kOutPhase) phase[p] = atan2f(gi[q], gr[q]);
    }
  }
}

template <int NL>
static hipError_t adj_nl(const Basis& b, int N, const float* pixtab,
                         const float* spotrec, const float* offtab,
                         const float* y, const float* amp_t, int outs, float* g,
                         float* phase, float* field_t, hipStream_t s) {
  hipLaunchKernelGGL(k_adjoint<NL>, dim3(b.n_tiles), dim3(kBlock), 0, s, N,
                     b.nx, b.ny, b.tiles_x, pixtab, spotrec,
                     reinterpret_cast<const float4*>(offtab),
                     reinterpret_cast<const float2*>(y), amp_t, outs,
                     reinterpret_cast<float2*>(g), phase,
                     reinterpret_cast<float2*>(field_t));
  return hipGetLastError();
}

hipError_t launch_adjoint(const Basis& b, int N, const float* pixtab,
                          const float* spotrec, const float* offtab,
                          const float* y, const float* amp_t, int outs,
                          float* g, float* phase, float* field_t,
                          hipStream_t s) {
  switch (b.nl_pad) {
#define X(n)                                                                  \
  case n:                                                                     \
    return adj_nl<n>(b, N, pixtab, spotrec, offtab, y, amp_t, outs, g, phase, \
                     field_t, s);
    ASH_NL_CASES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}

FwdPlan plan_forward(int n_tiles, int N) {
  FwdPlan p;
  const int n_sg = (N + kWave - 1) / kWave;
  // about 8192 waves in flight: 8 per SIMD on 256 CUs x 4 SIMDs
  long want = 8192 / (long)n_sg;
  if (want < 1) want = 1;
  if (want > n_tiles) want = n_tiles;
  p.tiles_per_group = (int)((n_tiles + want - 1) / want);
  p.groups = (n_tiles + p.tiles_per_group - 1) / p.tiles_per_group;
  p.rows_per_slice = 32;
  p.slices = (p.groups + p.rows_per_slice - 1) / p.rows_per_slice;
  return p;
}

}  // namespace ash
