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
// v_cos_f32 take their argument in turns; phases are reduced to [0, 1)
// first.
//
// Nearfield values and spot fields are kept in polar form (magnitude,
// phase in turns).  The phase of the multiplier joins the contraction as
// one more term, so the forward sums A(x) exp(-2 pi i (tau - phi(x))) and
// the adjoint |y_k| exp(2 pi i (tau + psi_k)), two FMAs per evaluation:
//
//   theta = sum_k S[spot][k] X[k][pixel],  k = 0 .. 2 KH - 1, with
//     k = 0            S: off        X: 1
//     k = 1, 2         S: a, b       X: di, dj
//     k = 3 .. 2+nl    S: c_s        X: Rm_s
//     k = 2 KH - 1     S: -1 | psi   X: phi | 1     (forward | adjoint)
//   and zeros in between.
#include <math.h>

#include "internal.h"

namespace ash {

int half_k(int nl) {
  // anchor offset, two slopes, the non-linear modes and the multiplier phase
  const int k = 4 + nl;
  return (k + 1) / 2;
}

// Records hold k = 0 .. 2 KH - 1 split by parity: entry (k & 1) KH + k / 2.
__host__ __device__ constexpr int slot(int k, int kh) {
  return (k & 1) * kh + (k >> 1);
}

constexpr float kInv2Pi = 0.15915494309189533577f;

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
  const int kh = rec / 2;
  float* r = pixtab + gid * rec;
  for (int k = 0; k < rec; ++k) r[k] = 0.0f;
  r[slot(0, kh)] = 1.0f;
  r[slot(1, kh)] = (float)di;
  r[slot(2, kh)] = (float)dj;
  r[slot(2 * kh - 1, kh)] = 1.0f;  // multiplier phase term (adjoint)
  const double xh = (i - cx) * invR, yh = (j - cy) * invR;
  const double x0 = (i0 - cx) * invR, y0 = (j0 - cy) * invR;
  for (int s = 0; s < nl && valid; ++s) {
    double v, gx, gy, v0, g0x, g0y;
    eval_nl(s, n_mono, pw, nlcoef, invR, xh, yh, &v, &gx, &gy);
    eval_nl(s, n_mono, pw, nlcoef, invR, x0, y0, &v0, &g0x, &g0y);
    r[slot(3 + s, kh)] = (float)(v - v0 - g0x * di - g0y * dj);
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
  const int kh = rec / 2;
  float* r = spotrec + (long)k * rec;
  for (int e = 0; e < rec; ++e) r[e] = 0.0f;  // slots 0..2: per tile
  for (int s = 0; s < nl; ++s)
    r[slot(3 + s, kh)] = (float)(w[(long)k * D + nlmode[s]] * inv2pi);
  r[slot(2 * kh - 1, kh)] = -1.0f;  // multiplier phase term (forward)
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
// Nearfield in tile-major polar form (A, phi in turns) from a phase with the
// basis amplitude, or from a complex field; spot fields in polar form.
// ---------------------------------------------------------------------------
__global__ void k_make_field(int nx, int ny, int tiles_x, long total,
                             const float* __restrict__ phase,
                             const float2* __restrict__ field,
                             const float* __restrict__ amp_t,
                             float2* __restrict__ nf_t) {
  const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= total) return;
  const int tile = (int)(gid / kTile), pix = (int)(gid % kTile);
  const int i = (tile % tiles_x) * kTileW + pix % kTileW;
  const int j = (tile / tiles_x) * kTileH + pix / kTileW;
  float2 v = make_float2(0.0f, 0.0f);
  if (i < nx && j < ny) {
    const long p = (long)j * nx + i;
    if (phase) {
      v = make_float2(amp_t[gid], phase[p] * kInv2Pi);
    } else {
      const float2 f = field[p];
      v = make_float2(hypotf(f.x, f.y), atan2f(f.y, f.x) * kInv2Pi);
    }
  }
  nf_t[gid] = v;
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

__global__ void k_to_polar(int N, const float2* __restrict__ y,
                           float2* __restrict__ ypol) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N) return;
  const float2 v = y[k];
  ypol[k] = make_float2(hypotf(v.x, v.y), atan2f(v.y, v.x) * kInv2Pi);
}

hipError_t launch_to_polar(int N, const float* y, float* ypol,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_to_polar, dim3((N + 255) / 256), dim3(256), 0, s, N,
                     reinterpret_cast<const float2*>(y),
                     reinterpret_cast<float2*>(ypol));
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Transforms on the matrix cores.
//
// For a block of 32 spots x 32 pixels the phases form the product
// theta = S X of the spot records S[32][2 KH] and the pixel records
// X[2 KH][32] (layout at the top of this file), one
// v_mfma_f32_32x32x2_f32 per pair of k.  Operand lane l carries item l%32
// and k = 2j + l/32, which is why records are stored split by the parity of
// k.  Result lane l holds the 16 phases of column n = l%32 and rows
// m = 8(i/4) + 4(l/32) + i%4, i = 0..15.  The VALU then range-reduces,
// takes the hardware sine and cosine and multiply-accumulates: the forward
// keeps 16 spots per lane and sums over pixel columns, the adjoint
// (theta^T = X^T S^T) keeps 16 pixels per lane and sums over spot columns.
// At the end a butterfly over the 32 lanes of each half-wave finishes the
// column sums, leaving one (re, im) result in every pair of lanes.
// ---------------------------------------------------------------------------
typedef float floatx16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ floatx16 mfma32(float a, float b, floatx16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

// One butterfly step over lane bit `mask` (< 32): of the 2*half complex
// values per lane keep the lower or upper `half` (by the lane's bit) and add
// the partner's copy of them.
template <int HALF>
__device__ __forceinline__ void bfly_step(float* re, float* im, int q,
                                          int mask) {
  const bool up = (q & mask) != 0;
#pragma unroll
  for (int i = 0; i < HALF; ++i) {
    const float sr = up ? re[i] : re[i + HALF];
    const float si = up ? im[i] : im[i + HALF];
    const float kr = up ? re[i + HALF] : re[i];
    const float ki = up ? im[i + HALF] : im[i];
    re[i] = kr + __shfl_xor(sr, mask, kWave);
    im[i] = ki + __shfl_xor(si, mask, kWave);
  }
}

// Sum 16 complex values per lane over the 32 lanes of the half-wave.  On
// return re[0], im[0] hold the total of value index bfly_index(q).
__device__ __forceinline__ void bfly_reduce(float* re, float* im, int q) {
  bfly_step<8>(re, im, q, 16);
  bfly_step<4>(re, im, q, 8);
  bfly_step<2>(re, im, q, 4);
  bfly_step<1>(re, im, q, 2);
  re[0] += __shfl_xor(re[0], 1, kWave);
  im[0] += __shfl_xor(im[0], 1, kWave);
}

__device__ __forceinline__ int bfly_index(int q) {
  return 8 * ((q >> 4) & 1) + 4 * ((q >> 3) & 1) + 2 * ((q >> 2) & 1) +
         ((q >> 1) & 1);
}

// row of the 32x32 result held in value i by a lane of half h
__device__ __forceinline__ int mfma_row(int i, int h) {
  return 8 * (i >> 2) + 4 * h + (i & 3);
}

// Range reduction, hardware sine / cosine and the multiply-accumulate of
// one 32x32 block of phases (16 per lane) with the lane's magnitude m:
// sr += m cos(2 pi theta), si += sgn m sin(2 pi theta).
template <bool kNegSin>
__device__ __forceinline__ void accumulate(const floatx16& th, float m,
                                           float* sr, float* si) {
  const float ms = kNegSin ? -m : m;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const float r = __builtin_amdgcn_fractf(th[i]);
    sr[i] = fmaf(m, __builtin_amdgcn_cosf(r), sr[i]);
    si[i] = fmaf(ms, __builtin_amdgcn_sinf(r), si[i]);
  }
}

template <int KH>
__device__ __forceinline__ floatx16 phase_block(const float* a,
                                                const float* b) {
  floatx16 acc;
#pragma unroll
  for (int i = 0; i < 16; ++i) acc[i] = 0.0f;
#pragma unroll
  for (int j = 0; j < KH; ++j) acc = mfma32(a[j], b[j], acc);
  return acc;
}

// Forward: wave = 32 spots x a contiguous range of 32-pixel blocks (tile
// order); the ranges split the pixel blocks of the SLM evenly over the
// groups.  E_k = sum_x A(x) exp(-2 pi i (tau_k(x) - phi(x))).
template <int KH>
__global__ __launch_bounds__(kBlock) void k_forward(
    int N, long n_blk, int groups, const float* __restrict__ pixtab,
    const float2* __restrict__ nf_t, const float* __restrict__ spotrec,
    const float4* __restrict__ offtab, float2* __restrict__ partial) {
  constexpr int R2 = 2 * KH;
  const int lane = threadIdx.x & (kWave - 1);
  const int h = lane >> 5, q = lane & 31;
  const int mb = blockIdx.y * (kBlock / kWave) + (threadIdx.x / kWave);
  if (mb * 32 >= N) return;  // wave-uniform exit; no barriers below
  const int k = mb * 32 + q;
  const bool live = k < N;
  const int kc = live ? k : N - 1;
  float S[KH];
#pragma unroll
  for (int j = 0; j < KH; ++j)
    S[j] = live ? spotrec[(long)kc * R2 + h * KH + j] : 0.0f;
  const float s1 = S[1];
  const int g = blockIdx.x;
  const long b0 = n_blk * g / groups;
  const long b1 = n_blk * (g + 1) / groups;
  float er[16], ei[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) er[i] = ei[i] = 0.0f;
  long tcur = -1;
  for (long b = b0; b < b1; ++b) {
    const long t = b >> 5;  // 32 blocks per tile
    if (t != tcur) {        // wave-uniform
      tcur = t;
      const float4 ot = offtab[t * N + kc];
      S[0] = live ? (h ? ot.y : ot.x) : 0.0f;
      S[1] = h ? s1 : (live ? ot.z : 0.0f);
    }
    const long px = b * 32 + q;  // tile-major pixel of this lane's column
    float X[KH];
    const float* __restrict__ xr = pixtab + px * R2 + h * KH;
#pragma unroll
    for (int j = 0; j < KH; ++j) X[j] = xr[j];
    const float2 nf = nf_t[px];
    if (h) X[KH - 1] = nf.y;  // k = 2 KH - 1: the nearfield phase
    const floatx16 th = phase_block<KH>(S, X);
    accumulate<true>(th, nf.x, er, ei);
  }
  bfly_reduce(er, ei, q);
  const int ko = mb * 32 + mfma_row(bfly_index(q), h);
  if ((q & 1) == 0 && ko < N)
    partial[(long)g * N + ko] = make_float2(er[0], ei[0]);
}

template <int KH>
static hipError_t fwd_kh(int n_mb, int groups, hipStream_t s, int N,
                         long n_blk, const float* pixtab, const float* field_t,
                         const float* spotrec, const float* offtab,
                         float* partial) {
  const int waves_per_block = kBlock / kWave;
  dim3 grid(groups, (n_mb + waves_per_block - 1) / waves_per_block);
  hipLaunchKernelGGL(k_forward<KH>, grid, dim3(kBlock), 0, s, N, n_blk,
                     groups, pixtab, reinterpret_cast<const float2*>(field_t),
                     spotrec, reinterpret_cast<const float4*>(offtab),
                     reinterpret_cast<float2*>(partial));
  return hipGetLastError();
}

template <int KH>
static int fwd_blocks_per_cu() {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_forward<KH>, kBlock,
                                                   0) != hipSuccess) {
    (void)hipGetLastError();
    return 1;
  }
  return n > 0 ? n : 1;
}

#define ASH_KH_CASES(X) \
  X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) \
  X(15) X(16)

int forward_blocks_per_cu(int kh) {
  switch (kh) {
#define X(n) \
  case n:    \
    return fwd_blocks_per_cu<n>();
    ASH_KH_CASES(X)
#undef X
    default:
      return 1;
  }
}

hipError_t launch_forward(const Basis& b, int N, const FwdPlan& p,
                          const float* pixtab, const float* field_t,
                          const float* spotrec, const float* offtab,
                          float* partial, hipStream_t s) {
  const int n_mb = (N + 31) / 32;
  const long n_blk = (long)b.n_tiles * (kTile / 32);
  switch (b.kh) {
#define X(n)                                                                \
  case n:                                                                   \
    return fwd_kh<n>(n_mb, p.groups, s, N, n_blk, pixtab, field_t, spotrec, \
                     offtab, partial);
    ASH_KH_CASES(X)
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
    // y = W t E/|E| in polar form (W t, arg E / 2 pi); arg 0 = 0
    y[k] = make_float2(wk * t[k], atan2f(e.y, e.x) * kInv2Pi);
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

// Adjoint: wave = 32 pixels of one tile x all spots.
// g(x) = sum_k |y_k| exp(2 pi i (tau_k(x) + psi_k)); the epilogue writes g,
// arg g and/or the next nearfield (A, arg g / 2 pi) in tile order.
constexpr int kAdjWavesPerTile = kTile / 32;  // 32

template <int KH>
__global__ __launch_bounds__(kBlock) void k_adjoint(
    int N, int nx, int ny, int tiles_x, const float* __restrict__ pixtab,
    const float* __restrict__ spotrec, const float4* __restrict__ offtab,
    const float2* __restrict__ ypol, const float* __restrict__ amp_t,
    int outs, float2* __restrict__ g, float* __restrict__ phase,
    float2* __restrict__ nf_t) {
  constexpr int R2 = 2 * KH;
  const int lane = threadIdx.x & (kWave - 1);
  const int h = lane >> 5, q = lane & 31;
  const int wv = blockIdx.x * (kBlock / kWave) + (threadIdx.x / kWave);
  const int tile = wv / kAdjWavesPerTile;
  const int p0 = (wv % kAdjWavesPerTile) * 32;  // first pixel of the block
  float X[KH];
  const float* __restrict__ xr =
      pixtab + ((long)tile * kTile + p0 + q) * R2 + h * KH;
#pragma unroll
  for (int j = 0; j < KH; ++j) X[j] = xr[j];
  const float4* __restrict__ orow = offtab + (long)tile * N;
  float gr[16], gi[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) gr[i] = gi[i] = 0.0f;
  for (int n0 = 0; n0 < N; n0 += 32) {
    const int n = n0 + q;
    const bool live = n < N;
    const int nc = live ? n : N - 1;
    float S[KH];
    const float* __restrict__ sr = spotrec + (long)nc * R2 + h * KH;
#pragma unroll
    for (int j = 0; j < KH; ++j) S[j] = sr[j];
    const float4 ot = orow[nc];
    const float2 yp = ypol[nc];
    S[0] = h ? ot.y : ot.x;
    if (!h) S[1] = ot.z;
    if (h) S[KH - 1] = yp.y;  // k = 2 KH - 1: the spot-field phase
    const floatx16 th = phase_block<KH>(X, S);
    accumulate<false>(th, live ? yp.x : 0.0f, gr, gi);
  }
  bfly_reduce(gr, gi, q);
  if (q & 1) return;  // the pair partner holds the same result
  const int pix = p0 + mfma_row(bfly_index(q), h);
  const int i = (tile % tiles_x) * kTileW + pix % kTileW;
  const int j = (tile / tiles_x) * kTileH + pix / kTileW;
  const float vr = gr[0], vi = gi[0];
  const float ang = atan2f(vi, vr);  // atan2(0, 0) = 0
  if (outs & kOutField)
    nf_t[(long)tile * kTile + pix] =
        make_float2(amp_t[(long)tile * kTile + pix], ang * kInv2Pi);
  if (i < nx && j < ny) {
    const long p = (long)j * nx + i;
    if (outs & kOutG) g[p] = make_float2(vr, vi);
    if (outs & kOutPhase) phase[p] = ang;
  }
}

template <int KH>
static hipError_t adj_kh(const Basis& b, int N, const float* pixtab,
                         const float* spotrec, const float* offtab,
                         const float* ypol, const float* amp_t, int outs,
                         float* g, float* phase, float* field_t,
                         hipStream_t s) {
  const int blocks = b.n_tiles * kAdjWavesPerTile / (kBlock / kWave);
  hipLaunchKernelGGL(k_adjoint<KH>, dim3(blocks), dim3(kBlock), 0, s, N, b.nx,
                     b.ny, b.tiles_x, pixtab, spotrec,
                     reinterpret_cast<const float4*>(offtab),
                     reinterpret_cast<const float2*>(ypol), amp_t, outs,
                     reinterpret_cast<float2*>(g), phase,
                     reinterpret_cast<float2*>(field_t));
  return hipGetLastError();
}

hipError_t launch_adjoint(const Basis& b, int N, const float* pixtab,
                          const float* spotrec, const float* offtab,
                          const float* ypol, const float* amp_t, int outs,
                          float* g, float* phase, float* field_t,
                          hipStream_t s) {
  switch (b.kh) {
#define X(n)                                                              \
  case n:                                                                 \
    return adj_kh<n>(b, N, pixtab, spotrec, offtab, ypol, amp_t, outs, g, \
                     phase, field_t, s);
    ASH_KH_CASES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}

FwdPlan plan_forward(int n_tiles, int N, int blocks_per_cu, int n_cu) {
  FwdPlan p;
  const int n_mb = (N + 31) / 32;
  const long n_blk = (long)n_tiles * (kTile / 32);
  // one full round of resident waves, each wave a range of pixel blocks
  const long waves = (long)blocks_per_cu * (kBlock / kWave) * n_cu;
  long want = waves / n_mb;
  if (want < 1) want = 1;
  if (want > n_blk) want = n_blk;
  p.groups = (int)want;
  p.rows_per_slice = 32;
  p.slices = (p.groups + p.rows_per_slice - 1) / p.rows_per_slice;
  return p;
}

}  // namespace ash
