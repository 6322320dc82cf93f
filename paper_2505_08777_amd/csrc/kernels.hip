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
// and linear term at the anchor.  Only the small in-tile quantities enter
// the single-precision sum, so it stays within a few tens of turns wherever
// the kernels respect the Nyquist limit.
//
// Nearfield values and spot fields are kept in polar form (magnitude,
// phase in turns); the phase of the multiplier joins the sum, so the
// forward adds A(x) exp(-2 pi i (tau - phi(x))) and the adjoint
// |y_k| exp(2 pi i (tau + psi_k)): two FMAs per evaluation after the
// hardware v_sin_f32 / v_cos_f32 (argument in turns, reduced to [0, 1)).
//
// The sum is a dot product theta = sum_f S[spot][f] X[f][pixel] over slots
// f, evaluated on the matrix cores in bf16 with FP32 accumulation.  Every
// FP32 / FP64 quantity is carried as an exact sum of bf16 pieces
// (v = v_h + v_m + v_l, each the bf16 rounding of what remains), and each
// product becomes a few products of pieces:
//   mode s, 2 pieces:  c_h Rm_h + c_h Rm_m + c_m Rm_h               (3 slots)
//   mode s, 3 pieces:  + c_h Rm_l + c_l Rm_h + c_m Rm_m              (6 slots)
//   fixed 12 slots at the end of the last 16-slot group:
//     p 4..6    S: -1 -1 -1 | psi_h psi_m psi_l   X: phi_h phi_m phi_l | 1 1 1
//               (forward | adjoint)
//     p 7..9    S: off_h off_m off_l              X: 1 1 1
//     p 10..12  S: a_h a_m a_l                    X: di di di
//     p 13..15  S: b_h b_m b_l                    X: dj dj dj
// Products of 8-bit-mantissa pieces are exact, so the error is that of the
// FP32 accumulation plus the dropped piece products: below 2^-16 |c Rm|
// with 2 pieces (used only while that stays negligible) and ~2^-24
// otherwise.  One v_mfma_f32_32x32x16_bf16 takes 16 slots.
#include <math.h>

#include <mutex>
#include <type_traits>

#include "internal.h"

namespace ash {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr float kInv2Pi = 0.15915494309189533577f;
constexpr double kInv2PiD = 0.15915494309189533577;
constexpr float kPiF = 3.14159265358979323846f;
constexpr float k2PiF = 6.28318530717958647692f;

// Anchor of a tile: offsets di in [-16, 15], dj in [-8, 7].
constexpr int kAnchorI = kTileW / 2;
constexpr int kAnchorJ = kTileH / 2;

constexpr unsigned kBf16One = 0x3F80u;
constexpr unsigned kBf16MinusOne = 0xBF80u;

// Global-memory pointers.  The transforms take their tables through
// pointers in the global address space, so that the compiler emits global
// loads with scalar base addresses; pointers read from memory (the batch's
// descriptors) are generic and are converted with as_global.
#define GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ GLOBAL T* as_global(T* p) {
  return (GLOBAL T*)p;
}

// Buffer loads for the transforms' inner loops: a resource over a
// wave-uniform base and extent (bytes), a per-lane offset fixed for the loop
// and a wave-uniform offset stepped by scalar instructions, so that the loop
// spends no vector instructions on addresses.  Reads past the extent return
// zeros.
typedef __amdgpu_buffer_rsrc_t rsrc_t;
constexpr int kRsrcWord3 = 0x00020000;  // raw 32-bit dword access
// A lane offset past every resource's extent (extents stay below 2^31
// bytes): its buffer loads return zeros.
constexpr unsigned kOutOfRange = 0x80000000u;

template <typename T>
__device__ __forceinline__ rsrc_t make_rsrc(const GLOBAL T* base,
                                            unsigned long bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(
      (void*)(const T*)base, (short)0,
      (int)(bytes < 0x7FFFFFFFul ? bytes : 0x7FFFFFFFul), kRsrcWord3);
}

__device__ __forceinline__ u32x4 bload4(rsrc_t r, unsigned voff,
                                        unsigned soff) {
  return __builtin_bit_cast(
      u32x4, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
}

__device__ __forceinline__ float bload1f(rsrc_t r, unsigned voff,
                                         unsigned soff) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}

__host__ __device__ int slots_per_mode(int pieces) {
  return pieces == 2 ? 3 : 6;
}

int groups_for(int nl, int pieces) {
  const int f = slots_per_mode(pieces) * nl + 12;
  return (f + 15) / 16;
}

// ---------------------------------------------------------------------------
// bf16 pieces
// ---------------------------------------------------------------------------
__device__ inline unsigned bf16_bits(float x) {  // round to nearest even
  unsigned u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return u >> 16;
}

__device__ inline float bf16_val(unsigned b) { return __uint_as_float(b << 16); }

// v = h + m + l + O(2^-27 |v|); each piece is the bf16 rounding of the rest
__device__ inline void split3(double v, unsigned* p) {
  p[0] = bf16_bits((float)v);
  const double r1 = v - (double)bf16_val(p[0]);
  p[1] = bf16_bits((float)r1);
  const double r2 = r1 - (double)bf16_val(p[1]);
  p[2] = bf16_bits((float)r2);
}

__device__ inline void split3f(float v, unsigned* p) {
  p[0] = bf16_bits(v);
  const float r1 = v - bf16_val(p[0]);  // exact (Sterbenz)
  p[1] = bf16_bits(r1);
  const float r2 = r1 - bf16_val(p[1]);
  p[2] = bf16_bits(r2);
}

// The dynamic per-pixel and per-spot data are laid out so that a wave
// fetches what both lane halves of a matrix-core operand need in one load:
// the vector-memory data path, not the arithmetic, is what these loads
// contend for.
//
// Nearfield of the tile-ordered pixels, per 32-pixel block (tile row)
// [tile * kBlkPerTile + row][half][32] u32x4.  Half 0: the words of half 0
// of the pixel record's last group (its nonlinear slots p 0..3, the phase
// pieces and a 1 at p 4..7).  Half 1: the words of half 1 of the last
// group, {1 | 1, di | di, di | dj, dj | dj} as bf16 (p 8..15).  The
// magnitudes are a separate per-pixel array in the same tile order.
__host__ __device__ inline long nf_index(long tile, int pix, int half) {
  return ((tile * kBlkPerTile + pix / 32) * 2 + half) * 32 + pix % 32;
}
// Phase (radians) to turns in [-1/2, 1/2]: a rounded multiply that is
// never fused into a later operation, then the nearest whole turn removed,
// so that every path writing a nearfield record from a phase (input phase,
// WGS projection, Adam update) writes the same bits for the same phase.
__device__ __forceinline__ float rad_to_turns(float rad) {
  const float t = __fmul_rn(rad, kInv2Pi);
  return t - rintf(t);
}

// Record of a pixel from its table nonlinear words and phase (turns).
__device__ inline u32x4 nearfield_record(u32x2 nl, float turns) {
  unsigned p[3];
  split3f(turns, p);
  return u32x4{nl.x, nl.y, p[0] | (p[1] << 16), p[2] | (kBf16One << 16)};
}
// The nonlinear words (p 0..3 of the last group, half 0) of pixel `pix` of
// `tile` in the pixel table.
__device__ inline u32x2 pixel_nl_words(const u32x4* pixtab, int G, long tile,
                                       int pix) {
  return *reinterpret_cast<const u32x2*>(
      pixtab + ((tile * G + G - 1) * 2) * kTile + pix);
}

// Spot fields of the adjoint, [NP / 32][half][32] u32x4 like the spot
// records: half 0 {the phase pieces at p 4..6 of the spot record's last
// group (words 2..3 of half 0), magnitude bits, 0}, half 1 {0, 0,
// magnitude bits, 0}, so that each lane half ORs its words in and reads the
// magnitude without selecting; then the magnitudes once more as a dense
// array of NP floats (words 8 NP + k), for kernels that need one per spot
// row of a lane.  Entries past N stay zero.
__device__ inline void put_spot_field(unsigned* y, int N, int k, float mag,
                                      float turns) {
  unsigned p[3];
  split3f(turns, p);
  u32x4* y4 = reinterpret_cast<u32x4*>(y) + (long)(k / 32) * 64 + k % 32;
  y4[0] = u32x4{p[0] | (p[1] << 16), p[2], __float_as_uint(mag), 0u};
  y4[32] = u32x4{0u, 0u, __float_as_uint(mag), 0u};
  reinterpret_cast<float*>(y)[(long)(N + 31) / 32 * 32 * 8 + k] = mag;
}

// Slot f of a record of 16-slot groups: group f / 16, lane half (f % 16)/8,
// entry f % 8.
__device__ inline void put_slot(unsigned short* rec, int f, unsigned v) {
  rec[(f / 16) * 16 + ((f % 16) / 8) * 8 + (f % 8)] = (unsigned short)v;
}

__device__ __forceinline__ double ipow(double x, int p) {
  double r = 1.0;
  for (int q = 0; q < p; ++q) r *= x;
  return r;
}

__device__ __forceinline__ void kahan_add(float& s, float& c, float x) {
  const float yv = x - c;
  const float t = s + yv;
  c = (t - s) - yv;
  s = t;
}

// Compensated sum of the n complex values p[0], p[stride], ... in index
// order.  The loads go out eight at a time, so their latencies overlap; the
// additions keep the serial order, so the result does not depend on it.
// A value written by another block of the same launch, read at device
// scope: the load goes to the level where the accelerator dies' caches are
// coherent and invalidates nothing.
__device__ __forceinline__ float2 load_device_scope(const float2* p) {
  const unsigned long long u =
      __hip_atomic_load(reinterpret_cast<const unsigned long long*>(p),
                        __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return __builtin_bit_cast(float2, u);
}

template <bool kDeviceScope = false>
__device__ __forceinline__ float2 kahan_sum_strided(
    const float2* __restrict__ p, long stride, int n) {
  float sr = 0.0f, si = 0.0f, cr = 0.0f, ci = 0.0f;
  for (int q = 0; q < n; q += 8) {
    float2 v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const float2* a = p + (long)(q + u) * stride;
      v[u] = q + u >= n     ? make_float2(0.0f, 0.0f)
             : kDeviceScope ? load_device_scope(a)
                            : *a;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if (q + u < n) {
        kahan_add(sr, cr, v[u].x);
        kahan_add(si, ci, v[u].y);
      }
    }
  }
  return make_float2(sr, si);
}

// ---------------------------------------------------------------------------
// Basis table (FP64, rounded once into bf16 pieces).
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

__device__ inline bool pixel_ij(const Geom& b, int tile, int pix, int* i,
                                int* j) {
  *i = (tile % b.tiles_x) * kTileW + pix % kTileW;
  *j = (tile / b.tiles_x) * kTileH + pix / kTileW;
  return *i < b.nx && *j < b.ny;
}

// Remainder Rm_s at one pixel of a tile (FP64); 0 outside the SLM.
__device__ double remainder_at(const Geom& b, int s, int n_mono,
                               const int32_t* __restrict__ pw,
                               const double* __restrict__ nlcoef, int tile,
                               int pix) {
  int i, j;
  if (!pixel_ij(b, tile, pix, &i, &j)) return 0.0;
  const double invR = 1.0 / b.R;
  const int i0 = (tile % b.tiles_x) * kTileW + kAnchorI;
  const int j0 = (tile / b.tiles_x) * kTileH + kAnchorJ;
  double v, gx, gy, v0, g0x, g0y;
  eval_nl(s, n_mono, pw, nlcoef, invR, (i - b.cx) * invR, (j - b.cy) * invR,
          &v, &gx, &gy);
  eval_nl(s, n_mono, pw, nlcoef, invR, (i0 - b.cx) * invR,
          (j0 - b.cy) * invR, &v0, &g0x, &g0y);
  return v - v0 - g0x * (i - i0) - g0y * (j - j0);
}

// One thread per pixel: the pixel's record, scattered as
// [tile][group][half][pixel][8 bf16] so that lanes read 16 consecutive bytes.
__global__ void k_build_pixtab(Geom b, long total, int n_mono,
                               const int32_t* __restrict__ pw,
                               const double* __restrict__ nlcoef,
                               const float* __restrict__ amp,
                               unsigned short* __restrict__ pixtab,
                               float* __restrict__ amp_t) {
  const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= total) return;
  const int tile = (int)(gid / kTile), pix = (int)(gid % kTile);
  const int G = b.groups;
  unsigned short rec[16 * kMaxGroups];
  for (int e = 0; e < 16 * G; ++e) rec[e] = 0;
  const int spm = slots_per_mode(b.pieces);
  for (int s = 0; s < b.nl; ++s) {
    unsigned p[3];
    split3(remainder_at(b, s, n_mono, pw, nlcoef, tile, pix), p);
    const int f = spm * s;  // pixel side of the piece products
    put_slot(rec, f + 0, p[0]);
    put_slot(rec, f + 1, p[1]);
    put_slot(rec, f + 2, p[0]);
    if (spm == 6) {
      put_slot(rec, f + 3, p[2]);
      put_slot(rec, f + 4, p[0]);
      put_slot(rec, f + 5, p[1]);
    }
  }
  const int di = pix % kTileW - kAnchorI, dj = pix / kTileW - kAnchorJ;
  const int base = 16 * (G - 1);
  const unsigned bdi = bf16_bits((float)di), bdj = bf16_bits((float)dj);
  for (int r = 0; r < 3; ++r) {
    put_slot(rec, base + 4 + r, kBf16One);  // multiplier phase (adjoint)
    put_slot(rec, base + 7 + r, kBf16One);
    put_slot(rec, base + 10 + r, bdi);
    put_slot(rec, base + 13 + r, bdj);
  }
  for (int g = 0; g < G; ++g)
    for (int h = 0; h < 2; ++h) {
      unsigned short* dst =
          pixtab + ((((long)tile * G + g) * 2 + h) * kTile + pix) * 8;
      for (int e = 0; e < 8; ++e) dst[e] = rec[g * 16 + h * 8 + e];
    }
  if (amp_t) {
    int i, j;
    const bool valid = pixel_ij(b, tile, pix, &i, &j);
    amp_t[gid] = valid ? (amp ? amp[(long)j * b.nx + i] : 1.0f) : 0.0f;
  }
}

// Value and gradient of every non-linear slot at every tile anchor, and the
// largest |Rm_s| over the tile's pixels (one block of 256 per tile).
__global__ __launch_bounds__(256) void k_build_tilebasis(
    Geom b, int n_mono, const int32_t* __restrict__ pw,
    const double* __restrict__ nlcoef, double* __restrict__ tilez,
    float* __restrict__ rmax) {
  __shared__ double sh[256];
  const int tile = blockIdx.x;
  const double invR = 1.0 / b.R;
  const double x0 = ((tile % b.tiles_x) * kTileW + kAnchorI - b.cx) * invR;
  const double y0 = ((tile / b.tiles_x) * kTileH + kAnchorJ - b.cy) * invR;
  for (int s = 0; s < b.nl; ++s) {
    if (threadIdx.x == 0) {
      double v, gx, gy;
      eval_nl(s, n_mono, pw, nlcoef, invR, x0, y0, &v, &gx, &gy);
      tilez[3 * ((long)tile * b.nl + s)] = v;
      tilez[3 * ((long)tile * b.nl + s) + 1] = gx;
      tilez[3 * ((long)tile * b.nl + s) + 2] = gy;
    }
    double m = 0.0;
    for (int pix = threadIdx.x; pix < kTile; pix += 256)
      m = fmax(m, fabs(remainder_at(b, s, n_mono, pw, nlcoef, tile, pix)));
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (threadIdx.x < w)
        sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + w]);
      __syncthreads();
    }
    if (threadIdx.x == 0) rmax[(long)tile * b.nl + s] = (float)sh[0];
    __syncthreads();
  }
}

hipError_t launch_build_tilebasis(const Geom& b, const int32_t* d_pow,
                                  const double* d_nlcoef, int n_mono,
                                  double* tilez, float* rmax, hipStream_t s) {
  if (b.nl == 0) return hipSuccess;
  hipLaunchKernelGGL(k_build_tilebasis, dim3(b.n_tiles), dim3(256), 0, s, b,
                     n_mono, d_pow, d_nlcoef, tilez, rmax);
  return hipGetLastError();
}

hipError_t launch_build_pixtab(const Geom& b, const int32_t* d_pow,
                               const double* d_nlcoef, int n_mono,
                               const float* amp_dev, unsigned short* pixtab,
                               float* amp_t, hipStream_t s) {
  const long total = (long)b.n_tiles * kTile;
  hipLaunchKernelGGL(k_build_pixtab, dim3((unsigned)((total + 255) / 256)),
                     dim3(256), 0, s, b, total, n_mono, d_pow, d_nlcoef,
                     amp_dev, pixtab, amp_t);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Spot preparation (FP64): per-spot records of the non-linear coefficients
// (turns, in pieces), and for every (tile, spot) the wrapped phase and the
// phase slopes of all constant and linear terms at the tile anchor.
// ---------------------------------------------------------------------------
__global__ void k_spot_records(Geom b, int N, const double* __restrict__ w,
                               const double* __restrict__ aff,
                               const int* __restrict__ nlmode,
                               unsigned short* __restrict__ spotrec,
                               double* __restrict__ spot64) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int G = b.groups;
  const long blk = k / 32, q = k % 32;
  if (k >= N) {  // padding to a whole spot block: zero records
    if (k < (N + 31) / 32 * 32)
      for (int g = 0; g < G; ++g)
        for (int h = 0; h < 2; ++h) {
          unsigned short* dst =
              spotrec + (((blk * G + g) * 2 + h) * 32 + q) * 8;
          for (int e = 0; e < 8; ++e) dst[e] = 0;
        }
    return;
  }
  const int D = b.D;
  double o = 0.0, a = 0.0, bb = 0.0;
  for (int d = 0; d < D; ++d) {
    const double wd = w[(long)k * D + d];
    o += wd * aff[3 * d];
    a += wd * aff[3 * d + 1];
    bb += wd * aff[3 * d + 2];
  }
  unsigned short rec[16 * kMaxGroups];
  for (int e = 0; e < 16 * G; ++e) rec[e] = 0;
  const int spm = slots_per_mode(b.pieces);
  for (int s = 0; s < b.nl; ++s) {
    unsigned p[3];
    split3(w[(long)k * D + nlmode[s]] * kInv2PiD, p);
    const int f = spm * s;  // spot side of the piece products
    put_slot(rec, f + 0, p[0]);
    put_slot(rec, f + 1, p[0]);
    put_slot(rec, f + 2, p[1]);
    if (spm == 6) {
      put_slot(rec, f + 3, p[0]);
      put_slot(rec, f + 4, p[2]);
      put_slot(rec, f + 5, p[1]);
    }
  }
  const int base = 16 * (G - 1);
  for (int r = 0; r < 3; ++r) put_slot(rec, base + 4 + r, kBf16MinusOne);
  // scatter: [spot block of 32][group][half][32 spots][8]
  for (int g = 0; g < G; ++g)
    for (int h = 0; h < 2; ++h) {
      unsigned short* dst = spotrec + (((blk * G + g) * 2 + h) * 32 + q) * 8;
      for (int e = 0; e < 8; ++e) dst[e] = rec[g * 16 + h * 8 + e];
    }
  spot64[3 * (long)k] = o * kInv2PiD;
  spot64[3 * (long)k + 1] = a * kInv2PiD / b.R;
  spot64[3 * (long)k + 2] = bb * kInv2PiD / b.R;
}

// One thread per (tile, spot).  Output [tile][half][NP] u32x4: the last
// 16-slot group of the spot record with its per-tile slots (half 0: the
// record's nonlinear slots p 0..3 and p 7; half 1: p 8..15), spots padded
// with zero records to NP, a whole number of 32-spot blocks.  Also the
// largest bound sum_s |c_s| max|Rm_s| (turns) of the in-tile remainder
// phase, and a bound on |theta|.
__global__ __launch_bounds__(256) void k_spot_offsets(Geom b, int N, long total,
                               const double* __restrict__ spot64,
                               const double* __restrict__ w,
                               const int* __restrict__ nlmode,
                               const double* __restrict__ tilez,
                               const float* __restrict__ rmax,
                               const u32x4* __restrict__ spotrec,
                               unsigned* __restrict__ offtab,
                               unsigned* __restrict__ bound_bits) {
  const int NP = (N + 31) / 32 * 32;  // spots padded to whole blocks
  float bnd = 0.0f, mg = 0.0f;  // this thread's bounds (0: none)
  for (long gid = (long)blockIdx.x * blockDim.x + threadIdx.x; gid < total;
       gid += (long)gridDim.x * blockDim.x) {
    const int tile = (int)(gid / NP), k = (int)(gid % NP);
    u32x4* __restrict__ ot = reinterpret_cast<u32x4*>(offtab);
    if (k >= N) {
      const u32x4 z = {0u, 0u, 0u, 0u};
      ot[((long)tile * 2 + 0) * NP + k] = z;
      ot[((long)tile * 2 + 1) * NP + k] = z;
    } else {
      const int nl = b.nl;
      const double i0 =
          (double)((tile % b.tiles_x) * kTileW + kAnchorI) - b.cx;
      const double j0 =
          (double)((tile / b.tiles_x) * kTileH + kAnchorJ) - b.cy;
      const double al = spot64[3 * (long)k + 1], be = spot64[3 * (long)k + 2];
      double t = spot64[3 * (long)k] + al * i0 + be * j0;
      double a = al, bs = be, bound = 0.0;
      const double* tz = tilez + 3 * (long)tile * nl;
      for (int s = 0; s < nl; ++s) {
        const double c = w[(long)k * b.D + nlmode[s]] * kInv2PiD;
        t += c * tz[3 * s];
        a += c * tz[3 * s + 1];
        bs += c * tz[3 * s + 2];
        bound += fabs(c) * (double)rmax[(long)tile * nl + s];
      }
      t -= floor(t);
      // |theta| over the tile: offset, slopes times the largest distance
      // from the anchor, remainder, and the two record phases of at most
      // 1/2 each
      const double mag = 2.0 + kAnchorI * fabs(a) + kAnchorJ * fabs(bs) + bound;
      unsigned po[3], pa[3], pb[3];
      split3(t, po);
      split3(a, pa);
      split3(bs, pb);
      // half 0: the spot record's nonlinear slots p 0..3 (so that the
      // adjoint need not read the record's last group), and p 7
      const u32x2 nlw = *reinterpret_cast<const u32x2*>(
          spotrec +
          ((((long)k / 32) * b.groups + b.groups - 1) * 2) * 32 + k % 32);
      u32x4 h0, h1;
      h0[0] = nlw.x;
      h0[1] = nlw.y;
      h0[2] = 0u;
      h0[3] = po[0] << 16;            // p 7
      h1[0] = po[1] | (po[2] << 16);  // p 8, 9
      h1[1] = pa[0] | (pa[1] << 16);  // p 10, 11
      h1[2] = pa[2] | (pb[0] << 16);  // p 12, 13
      h1[3] = pb[1] | (pb[2] << 16);  // p 14, 15
      ot[((long)tile * 2 + 0) * NP + k] = h0;
      ot[((long)tile * 2 + 1) * NP + k] = h1;
      bnd = fmaxf(bnd, (float)bound);
      mg = fmaxf(mg, (float)mag);
    }
  }
  // the block's largest bounds, then one atomic per block: atomics on one
  // address serialise, so they are kept to a few thousand per launch
  // (non-negative floats order like their bit patterns)
  __shared__ float sh[2][256 / kWave];
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    bnd = fmaxf(bnd, __shfl_xor(bnd, m, kWave));
    mg = fmaxf(mg, __shfl_xor(mg, m, kWave));
  }
  if ((threadIdx.x & (kWave - 1)) == 0) {
    sh[0][threadIdx.x / kWave] = bnd;
    sh[1][threadIdx.x / kWave] = mg;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < (int)(blockDim.x / kWave); ++i) {
      bnd = fmaxf(bnd, sh[0][i]);
      mg = fmaxf(mg, sh[1][i]);
    }
    atomicMax(bound_bits, __float_as_uint(bnd));
    atomicMax(bound_bits + 1, __float_as_uint(mg));
  }
}

hipError_t launch_prep_spots(const Geom& b, int N, const double* d_w,
                             const double* d_aff, const int* d_nlmode,
                             const double* tilez, const float* rmax,
                             unsigned short* spotrec, double* spot64,
                             unsigned* offtab, unsigned* bound_bits,
                             hipStream_t s) {
  const int n_pad = (N + 31) / 32 * 32;
  hipLaunchKernelGGL(k_spot_records, dim3((n_pad + 255) / 256), dim3(256), 0,
                     s, b, N, d_w, d_aff, d_nlmode, spotrec, spot64);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const long total = (long)b.n_tiles * n_pad;
  const long blocks = (total + 255) / 256 < 8192 ? (total + 255) / 256 : 8192;
  hipLaunchKernelGGL(k_spot_offsets, dim3((unsigned)blocks),
                     dim3(256), 0, s, b, N, total, spot64, d_w, d_nlmode,
                     tilez, rmax, reinterpret_cast<const u32x4*>(spotrec),
                     offtab, bound_bits);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Nearfield records in tile order, {A, phase pieces | 1 (p 7)}, from a phase
// with the basis amplitude or from a complex field; spot-field records
// {|y|, phase pieces}.
// ---------------------------------------------------------------------------
// Nearfield record of pixel `pix` of `tile` (tile-order index gid).
__device__ __forceinline__ void make_field_at(
    int nx, int ny, int tiles_x, int G, long gid,
    const float* __restrict__ phase, const float2* __restrict__ field,
    const float* __restrict__ amp_t, const u32x4* __restrict__ pixtab,
    u32x4* __restrict__ nf, float* __restrict__ fmag) {
  const int tile = (int)(gid / kTile), pix = (int)(gid % kTile);
  const int i = (tile % tiles_x) * kTileW + pix % kTileW;
  const int j = (tile / tiles_x) * kTileH + pix / kTileW;
  float mag = 0.0f, turns = 0.0f;
  if (i < nx && j < ny) {
    const long p = (long)j * nx + i;
    if (phase) {
      mag = amp_t[gid];
      turns = rad_to_turns(phase[p]);  // any phase: reduced to [-1/2, 1/2]
    } else {
      const float2 f = field[p];
      mag = hypotf(f.x, f.y);
      turns = rad_to_turns(atan2f(f.y, f.x));
    }
  }
  nf[nf_index(tile, pix, 0)] =
      nearfield_record(pixel_nl_words(pixtab, G, tile, pix), turns);
  const unsigned bdi = bf16_bits((float)(pix % kTileW - kAnchorI));
  const unsigned bdj = bf16_bits((float)(pix / kTileW - kAnchorJ));
  nf[nf_index(tile, pix, 1)] =
      u32x4{kBf16One | (kBf16One << 16), bdi | (bdi << 16), bdi | (bdj << 16),
            bdj | (bdj << 16)};
  if (fmag) fmag[gid] = mag;
}

__global__ void k_make_field(Geom b, long total,
                             const float* __restrict__ phase,
                             const float2* __restrict__ field,
                             const float* __restrict__ amp_t,
                             const u32x4* __restrict__ pixtab,
                             u32x4* __restrict__ nf, float* __restrict__ fmag) {
  const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= total) return;
  make_field_at(b.nx, b.ny, b.tiles_x, b.groups, gid, phase, field, amp_t,
                pixtab, nf, fmag);
}

hipError_t launch_make_field(const Geom& b, const float* phase,
                             const float* field, const float* amp_t,
                             const unsigned short* pixtab, unsigned* nf_t,
                             float* fmag, hipStream_t s) {
  const long total = (long)b.n_tiles * kTile;
  hipLaunchKernelGGL(k_make_field, dim3((unsigned)((total + 255) / 256)),
                     dim3(256), 0, s, b, total, phase,
                     reinterpret_cast<const float2*>(field), amp_t,
                     reinterpret_cast<const u32x4*>(pixtab),
                     reinterpret_cast<u32x4*>(nf_t), fmag);
  return hipGetLastError();
}

__global__ void k_to_polar(int N, const float2* __restrict__ y,
                           unsigned* __restrict__ ypol) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N) return;
  const float2 v = y[k];
  put_spot_field(ypol, N, k, hypotf(v.x, v.y), atan2f(v.y, v.x) * kInv2Pi);
}

hipError_t launch_to_polar(int N, const float* y, unsigned* ypol,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_to_polar, dim3((N + 255) / 256), dim3(256), 0, s, N,
                     reinterpret_cast<const float2*>(y), ypol);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Transforms on the matrix cores.
//
// For a block of 32 spots x 32 pixels the phases form the product
// theta = S X of the spot records S[32][16 G] and the pixel records
// X[16 G][32]: G v_mfma_f32_32x32x16_bf16.  Operand lane l carries item
// l%32 and slots 8 (l/32) .. 8 (l/32) + 7 of each 16-slot group.  Result
// lane l holds the 16 phases of column n = l%32 and rows
// m = 8(i/4) + 4(l/32) + i%4, i = 0..15.  The VALU then range-reduces,
// takes the hardware sine and cosine and multiply-accumulates: the forward
// keeps 16 spots per lane and sums over pixel columns, the adjoint
// (theta^T = X^T S^T) keeps 16 pixels per lane and sums over spot columns.
// At the end a butterfly over the 32 lanes of each half-wave finishes the
// column sums, leaving one (re, im) result in every pair of lanes.
// ---------------------------------------------------------------------------
__device__ __forceinline__ floatx16 mfma_bf16(u32x4 a, u32x4 b, floatx16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(
      __builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0, 0,
      0);
}

template <int G>
__device__ __forceinline__ floatx16 phase_block(const u32x4* a,
                                                const u32x4* b) {
  floatx16 acc;
#pragma unroll
  for (int i = 0; i < 16; ++i) acc[i] = 0.0f;
#pragma unroll
  for (int g = 0; g < G; ++g) acc = mfma_bf16(a[g], b[g], acc);
  return acc;
}

// Value of lane-permuted x through DPP control CTRL (all lanes active).
template <int CTRL>
__device__ __forceinline__ float dpp(float x) {
  return __int_as_float(
      __builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}

// One butterfly step: each lane keeps the lower or upper HALF of its
// 2*HALF complex values (by its own bit `up`) and adds the partner lane's
// copy of them; the partner, reached through DPP control CTRL, has the
// opposite bit.
template <int HALF, int CTRL>
__device__ __forceinline__ void bfly_step(float* re, float* im, bool up) {
#pragma unroll
  for (int i = 0; i < HALF; ++i) {
    const float kr = up ? re[i + HALF] : re[i], sr = up ? re[i] : re[i + HALF];
    const float ki = up ? im[i + HALF] : im[i], si = up ? im[i] : im[i + HALF];
    re[i] = kr + dpp<CTRL>(sr);
    im[i] = ki + dpp<CTRL>(si);
  }
}

// Sum 16 complex values per lane over the 32 lanes of the half-wave.  On
// return re[0], im[0] hold the total of value index bfly_index(q).  The
// partners of the five steps are lanes 16 apart (a row swap: the lower
// values of the odd row trade places with the upper values of the even
// row, so one add finishes each pair), 8 apart (rotation by 8 in a row),
// mirrored in 8 lanes (bit 2 flipped), 2 apart and 1 apart; together they
// pair every lane with all 31 others exactly once.  No LDS.
__device__ __forceinline__ void bfly_reduce(float* re, float* im, int q) {
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const auto r = __builtin_amdgcn_permlane16_swap(
        __float_as_uint(re[i]), __float_as_uint(re[i + 8]), false, false);
    re[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    const auto m = __builtin_amdgcn_permlane16_swap(
        __float_as_uint(im[i]), __float_as_uint(im[i + 8]), false, false);
    im[i] = __uint_as_float(m[0]) + __uint_as_float(m[1]);
  }
  bfly_step<4, 0x128>(re, im, (q & 8) != 0);  // row_ror:8
  bfly_step<2, 0x141>(re, im, (q & 4) != 0);  // row_half_mirror
  bfly_step<1, 0x4E>(re, im, (q & 2) != 0);   // quad_perm [2, 3, 0, 1]
  re[0] += dpp<0xB1>(re[0]);                   // quad_perm [1, 0, 3, 2]
  im[0] += dpp<0xB1>(im[0]);
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
// sr += m cos(2 pi theta), si += sgn m sin(2 pi theta).  The hardware
// sine and cosine take turns and reduce exactly by themselves over
// |theta| <= 256; kReduce = false skips the explicit fract where the host
// has bounded every phase of the set-up well inside that domain.
// kInit: the sums start here (sr = m cos, si = sgn m sin: the same
// roundings as adding to zeros, without the zeroing moves).
template <bool kNegSin, bool kReduce, bool kInit = false>
__device__ __forceinline__ void accumulate(const floatx16& th, float m,
                                           float* sr, float* si) {
  const float ms = kNegSin ? -m : m;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const float r = kReduce ? __builtin_amdgcn_fractf(th[i]) : th[i];
    if (kInit) {
      sr[i] = m * __builtin_amdgcn_cosf(r);
      si[i] = ms * __builtin_amdgcn_sinf(r);
    } else {
      sr[i] = fmaf(m, __builtin_amdgcn_cosf(r), sr[i]);
      si[i] = fmaf(ms, __builtin_amdgcn_sinf(r), si[i]);
    }
  }
}


// Forward sum of one wave: the 32 spots of spot block mb over the pixel
// blocks [b0, b1) (tile rows, tile order).  Operand A is the spot record,
// B the pixel record of a block; each lane keeps 16 spot rows, and a
// butterfly over the 32 lanes of each half-wave finishes the pixel sums,
// written to row[k] for the block's spots k < N.  One load brings each
// lane half its part of the nearfield record's last group, another the
// magnitude of the lane's pixel (the same for both halves).
// E_k = sum_x A(x) exp(-2 pi i (tau_k(x) - phi(x))).
template <int G, bool kReduce, bool kTwoSets>
__device__ __forceinline__ void forward_range(
    int N, int mb, long b0, long b1, const GLOBAL u32x4* __restrict__ pixtab,
    const GLOBAL u32x4* __restrict__ nf, const GLOBAL float* __restrict__ mag,
    const GLOBAL u32x4* __restrict__ spotrec,
    const GLOBAL u32x4* __restrict__ offtab, float2* __restrict__ row) {
  const int lane = threadIdx.x & (kWave - 1);
  const int h = lane >> 5, q = lane & 31;
  const int NP = (N + 31) / 32 * 32;  // spot stride of the per-tile slots
  // the record's last group is the per-tile slots (which carry its
  // nonlinear slots p 0..3) with -1 at p 4..6 against the nearfield phase
  // addresses: a wave-uniform base plus a 32-bit lane offset, so that
  // loads take the scalar-base form
  const unsigned lane_pix = h * kTile + q, lane_spot = h * 32 + q;
  const unsigned off_pix = lane_pix * 16u, off_spot = lane_spot * 16u,
                 off_q = q * 4u;
  u32x4 S[G];
  const GLOBAL u32x4* __restrict__ sb = spotrec + (long)mb * G * 64;
#pragma unroll
  for (int g = 0; g < G - 1; ++g) S[g] = sb[lane_spot + g * 64];
  const unsigned m2 = h ? 0u : (kBf16MinusOne | (kBf16MinusOne << 16));
  const unsigned m3 = h ? 0u : kBf16MinusOne;
  float er[16], ei[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) er[i] = ei[i] = 0.0f;
  const unsigned lane_ot = h * NP + q;
  const GLOBAL u32x4* __restrict__ ot_k = offtab + (long)mb * 32;
  // tiles of the range; the tile slots of the lane's spot once per tile
  for (long b = b0; b < b1;) {
    const long t = b / kBlkPerTile;
    const int r0 = (int)(b - t * kBlkPerTile);
    const int r1 = (int)min((long)kBlkPerTile, r0 + (b1 - b));
    S[G - 1] = (ot_k + t * 2 * NP)[lane_ot];
    S[G - 1][2] |= m2;
    S[G - 1][3] |= m3;
    const rsrc_t rx = make_rsrc(pixtab + t * G * 2 * kTile,
                                (unsigned long)G * 2 * kTile * 16);
    const rsrc_t rn = make_rsrc(nf + t * kBlkPerTile * 64,
                                (unsigned long)kBlkPerTile * 64 * 16);
    const rsrc_t rm = make_rsrc(mag + t * kTile, (unsigned long)kTile * 4);
    // kTwoSets: two register sets take turns, one block's products running
    // while the next block's records load into the other set; otherwise
    // (where the second set would cost a wave per SIMD) each block's loads
    // go out before its products
    u32x4 XA[G], XB[G];
    float mA, mB;
    auto load = [&](u32x4* X, float& m, int r) {
#pragma unroll
      for (int g = 0; g < G - 1; ++g)
        X[g] = bload4(rx, off_pix, (unsigned)(g * 2 * kTile + r * 32) * 16u);
      X[G - 1] = bload4(rn, off_spot, (unsigned)r * 64u * 16u);
      m = bload1f(rm, off_q, (unsigned)r * 32u * 4u);
    };
    if constexpr (kTwoSets) {
      load(XA, mA, r0);
      for (int r = r0; r < r1; r += 2) {
        load(XB, mB, min(r + 1, r1 - 1));
        __builtin_amdgcn_sched_barrier(0);
        accumulate<true, kReduce>(phase_block<G>(S, XA), mA, er, ei);
        if (r + 1 < r1) {
          load(XA, mA, min(r + 2, r1 - 1));
          __builtin_amdgcn_sched_barrier(0);
          accumulate<true, kReduce>(phase_block<G>(S, XB), mB, er, ei);
        }
      }
    } else {
      for (int r = r0; r < r1; ++r) {
        load(XA, mA, r);
        __builtin_amdgcn_sched_barrier(0);
        accumulate<true, kReduce>(phase_block<G>(S, XA), mA, er, ei);
      }
    }
    b += r1 - r0;
  }
  bfly_reduce(er, ei, q);
  const int ko = mb * 32 + mfma_row(bfly_index(q), h);
  if ((q & 1) == 0 && ko < N) row[ko] = make_float2(er[0], ei[0]);
}

// Forward of one hologram: wave = 32 spots x a contiguous range of pixel
// blocks; the ranges split the pixel blocks of the SLM evenly.  Blocks are
// handed to the XCDs round-robin by linear id; range r belongs to XCD r % 8,
// and the waves of one XCD enumerate (range, spot block) pairs with the
// spot block fastest, so all spot blocks of a range run on one XCD at
// neighbouring slots and its L2 serves the range's records to all of them.
template <int G, bool kReduce>
__global__ __launch_bounds__(kBlock) void k_forward(
    int N, long n_blk, int groups, const u32x4* __restrict__ pixtab,
    const unsigned* __restrict__ nf_t, const float* __restrict__ mag,
    const u32x4* __restrict__ spotrec, const unsigned* __restrict__ offtab,
    float2* __restrict__ partial) {
  const int n_mb = (N + 31) / 32;
  const int xcd = blockIdx.x % kXcds, slot = blockIdx.x / kXcds;
  // the wave index is uniform over the wave; say so, so that the range
  // bounds and record addresses live in scalar registers
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const long v = (long)slot * (kBlock / kWave) + wave;
  if (v >= (long)(groups / kXcds) * n_mb) return;  // wave-uniform exit
  const int gi = (int)(v / n_mb) * kXcds + xcd;  // pixel range
  const int mb = (int)(v % n_mb);                // spot block
  // two register sets where they keep this kernel's waves per SIMD
  forward_range<G, kReduce, G == 3 || G == 6>(N, mb, n_blk * gi / groups,
                            n_blk * (gi + 1) / groups, as_global(pixtab),
                            as_global(reinterpret_cast<const u32x4*>(nf_t)),
                            as_global(mag), as_global(spotrec),
                            as_global(reinterpret_cast<const u32x4*>(offtab)),
                            partial + (long)gi * N);
}

template <int G>
static hipError_t fwd_g(bool reduce, int n_mb, int groups, hipStream_t s,
                        int N, long n_blk, const unsigned short* pixtab,
                        const unsigned* nf_t, const float* mag,
                        const unsigned short* spotrec,
                        const unsigned* offtab, float* partial) {
  // groups is a multiple of kXcds (plan_forward); waves per XCD:
  const long per_xcd = (long)(groups / kXcds) * n_mb;
  const long blocks_per_xcd = (per_xcd + kBlock / kWave - 1) / (kBlock / kWave);
  auto* const kern = reduce ? k_forward<G, true> : k_forward<G, false>;
  hipLaunchKernelGGL(kern, dim3((unsigned)(blocks_per_xcd * kXcds)),
                     dim3(kBlock), 0, s, N, n_blk, groups,
                     reinterpret_cast<const u32x4*>(pixtab), nf_t, mag,
                     reinterpret_cast<const u32x4*>(spotrec), offtab,
                     reinterpret_cast<float2*>(partial));
  return hipGetLastError();
}

template <int G>
static int fwd_blocks_per_cu() {
  int n = 0;
  // both variants: the plan must fit the larger register footprint
  int n2 = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_forward<G, true>,
                                                   kBlock, 0) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&n2, k_forward<G, false>,
                                                   kBlock, 0) != hipSuccess) {
    (void)hipGetLastError();
    return 1;
  }
  n = n < n2 ? n : n2;
  return n > 0 ? n : 1;
}

#define ASH_G_CASES(X) \
  X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12)

int forward_blocks_per_cu(int groups) {
  switch (groups) {
#define X(n) \
  case n:    \
    return fwd_blocks_per_cu<n>();
    ASH_G_CASES(X)
#undef X
    default:
      return 1;
  }
}

hipError_t launch_forward(const Geom& b, int N, const FwdPlan& p,
                          const unsigned short* pixtab, const unsigned* nf_t,
                          const float* mag, const unsigned short* spotrec,
                          const unsigned* offtab, float* partial,
                          hipStream_t s) {
  const int n_mb = (N + 31) / 32;
  const long n_blk = (long)b.n_tiles * kBlkPerTile;
  switch (b.groups) {
#define X(n)                                                            \
  case n:                                                               \
    return fwd_g<n>(b.reduce != 0, n_mb, p.groups, s, N, n_blk, pixtab, \
                    nf_t, mag, spotrec, offtab, partial);
    ASH_G_CASES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------------------
// Basis moments of the forward,
//   M[k][d] = sum_x Z_d(x) f(x) exp(-i theta_k(x)),  dE_k/dw[k][d] = -i M[k][d].
// The phases come from the forward's records with the matrix-core operands
// swapped (rows: 32 pixels, column: the lane's spot), so that every lane holds
// one spot and 16 pixels.  Their cosines and sines, split into two bf16
// pieces, are the B operand of a second product whose A operand is the
// moment table (rows: the hi and lo bf16 pieces of A(x) Z_d(x); K: pixels);
// the matrix cores then sum over the pixels of the block.
// ---------------------------------------------------------------------------
typedef float float2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// Two values as bf16 pieces, packed two per word (x0 in the low half):
// hi rounds to nearest even, the remainder x - hi is exact, and lo is its
// rounding, so x = hi + lo + O(2^-17 |x|).  Each remainder is one bf16 dot
// product, x + (-1) hi + 0 hi': its products are exact and its result is
// representable, so it carries no rounding.  The selector pairs {-1, 0}
// and {0, -1} (n0, n1: bf16 bits 0x0000BF80, 0xBF800000) are held in
// registers by the caller, never folded into the instruction as constants.
__device__ __forceinline__ void split2(float x0, float x1, unsigned n0,
                                       unsigned n1, unsigned& hi,
                                       unsigned& lo) {
  const bf16x2 h = __builtin_convertvector(float2v{x0, x1}, bf16x2);
  const float r0 = __builtin_amdgcn_fdot2_f32_bf16(
      h, __builtin_bit_cast(bf16x2, n0), x0, false);
  const float r1 = __builtin_amdgcn_fdot2_f32_bf16(
      h, __builtin_bit_cast(bf16x2, n1), x1, false);
  hi = __builtin_bit_cast(unsigned, h);
  lo = __builtin_bit_cast(unsigned,
                          __builtin_convertvector(float2v{r0, r1}, bf16x2));
}

// Moment-table slot of pixel p (0..31) of a 32-pixel block: K block kb
// (16 pixels), lane half h and element e, such that element e of half h in
// K block kb is the pixel of phase value 8 kb + e of a lane of half h.
__device__ __forceinline__ void mom_slot(int p, int* kb, int* h, int* e) {
  *kb = p >> 4;
  *h = (p >> 2) & 1;
  *e = ((p >> 3) & 1) * 4 + (p & 3);
}

// One thread per pixel: A(x) Z_d(x) for every mode in FP64, stored as two
// bf16 pieces in rows d (hi) and D + d (lo) of [block][kb][h][2D][8].
__global__ void k_build_momtab(Geom b, long total, int n_mono,
                               const int32_t* __restrict__ pw,
                               const double* __restrict__ coef,
                               const float* __restrict__ amp_t,
                               unsigned short* __restrict__ momtab) {
  const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= total) return;
  const int tile = (int)(gid / kTile), pix = (int)(gid % kTile);
  const int D = b.D, D2 = 2 * b.D;
  int i, j;
  const bool valid = pixel_ij(b, tile, pix, &i, &j);
  const double invR = 1.0 / b.R;
  const double x = (i - b.cx) * invR, y = (j - b.cy) * invR;
  const double a = valid ? (double)amp_t[gid] : 0.0;
  const long blk = gid / 32;
  int kb, h, e;
  mom_slot((int)(gid % 32), &kb, &h, &e);
  unsigned short* dst = momtab + ((blk * 2 + kb) * 2 + h) * D2 * 8 + e;
  for (int d = 0; d < D; ++d) {
    double z = 0.0;
    for (int m = 0; m < n_mono; ++m) {
      const double c = coef[d * n_mono + m];
      if (c != 0.0) z += c * ipow(x, pw[2 * m]) * ipow(y, pw[2 * m + 1]);
    }
    unsigned pc[3];
    split3(a * z, pc);
    dst[d * 8] = (unsigned short)pc[0];
    dst[(D + d) * 8] = (unsigned short)pc[1];
  }
}

hipError_t launch_build_momtab(const Geom& b, const int32_t* d_pow,
                               const double* d_coef, int n_mono,
                               const float* amp_t, unsigned short* momtab,
                               hipStream_t s) {
  const long total = (long)b.n_tiles * kTile;
  hipLaunchKernelGGL(k_build_momtab, dim3((unsigned)((total + 255) / 256)),
                     dim3(256), 0, s, b, total, n_mono, d_pow, d_coef, amp_t,
                     momtab);
  return hipGetLastError();
}

// Moments of one wave: the 32 spots of spot block mb over pixel blocks
// [b0, b1).  RT tiles of 32 moment rows; out: [2D][NP] (re, -im) sums.
// kReduce as for the transforms.
template <int G, int RT, bool kReduce>
__device__ __forceinline__ void moments_range(
    int N, int D2, int mb, long b0, long b1,
    const GLOBAL u32x4* __restrict__ pixtab, const GLOBAL u32x4* __restrict__ nf,
    const GLOBAL u32x4* __restrict__ spotrec,
    const GLOBAL u32x4* __restrict__ offtab,
    const GLOBAL u32x4* __restrict__ momtab, float2* __restrict__ out) {
  const int lane = threadIdx.x & (kWave - 1);
  const int h = lane >> 5, q = lane & 31;
  const int NP = (N + 31) / 32 * 32;
  const unsigned lane_pix = h * kTile + q, lane_spot = h * 32 + q;
  u32x4 S[G];
  const GLOBAL u32x4* __restrict__ sb = spotrec + (long)mb * G * 64;
#pragma unroll
  for (int g = 0; g < G - 1; ++g) S[g] = sb[lane_spot + g * 64];
  const unsigned m2 = h ? 0u : (kBf16MinusOne | (kBf16MinusOne << 16));
  const unsigned m3 = h ? 0u : kBf16MinusOne;
  // split2's selector pairs, in vector registers (an empty asm statement
  // hides their values from constant folding)
  unsigned sel0 = kBf16MinusOne, sel1 = kBf16MinusOne << 16;
  asm volatile("" : "+v"(sel0), "+v"(sel1));
  floatx16 are[RT], aim[RT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int i = 0; i < 16; ++i) are[rt][i] = aim[rt][i] = 0.0f;
  const unsigned lane_ot = h * NP + q;
  const GLOBAL u32x4* __restrict__ ot_k = offtab + (long)mb * 32;
  for (long b = b0; b < b1;) {
    const long t = b / kBlkPerTile;
    const int r0 = (int)(b - t * kBlkPerTile);
    const int r1 = (int)min((long)kBlkPerTile, r0 + (b1 - b));
    S[G - 1] = (ot_k + t * 2 * NP)[lane_ot];
    S[G - 1][2] |= m2;
    S[G - 1][3] |= m3;
    const rsrc_t rx = make_rsrc(pixtab + t * G * 2 * kTile,
                                (unsigned long)G * 2 * kTile * 16);
    const rsrc_t rn = make_rsrc(nf + t * kBlkPerTile * 64,
                                (unsigned long)kBlkPerTile * 64 * 16);
    const rsrc_t rm = make_rsrc(momtab + t * kBlkPerTile * 4 * D2,
                                (unsigned long)kBlkPerTile * 4 * D2 * 16);
    // where it costs no occupancy (one moment tile, 3 or 4 groups), two
    // register sets take turns: one block's products run while the next
    // block's records and moment rows load into the other set
    u32x4 XA[G], XB[G], AA[RT][2], AB[RT][2];
    auto load = [&](u32x4* X, u32x4 (*A)[2], int r) {
#pragma unroll
      for (int g = 0; g < G - 1; ++g)
        X[g] = bload4(rx, lane_pix * 16u,
                      (unsigned)(g * 2 * kTile + r * 32) * 16u);
      X[G - 1] = bload4(rn, lane_spot * 16u, (unsigned)r * 64u * 16u);
      // moment rows 32 rt + q of this lane; rows past 2D load zeros
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int kb = 0; kb < 2; ++kb) {
          const int row = 32 * rt + q;
          A[rt][kb] = bload4(
              rm, row < D2 ? (unsigned)((kb * 2 + h) * D2 + row) * 16u : kOutOfRange,
              (unsigned)r * 4u * D2 * 16u);
        }
    };
    auto block = [&](const u32x4* X, u32x4 (*A)[2]) {
      const floatx16 th = phase_block<G>(X, S);
      u32x4 ch[2], cl[2], sh[2], sl[2];
#pragma unroll
      for (int kb = 0; kb < 2; ++kb)
#pragma unroll
        for (int w = 0; w < 4; ++w) {
          float t0 = th[8 * kb + 2 * w], t1 = th[8 * kb + 2 * w + 1];
          if (kReduce) {
            t0 = __builtin_amdgcn_fractf(t0);
            t1 = __builtin_amdgcn_fractf(t1);
          }
          unsigned a0, a1, b0w, b1w;
          split2(__builtin_amdgcn_cosf(t0), __builtin_amdgcn_cosf(t1), sel0,
                 sel1, a0, a1);
          split2(__builtin_amdgcn_sinf(t0), __builtin_amdgcn_sinf(t1), sel0,
                 sel1, b0w, b1w);
          ch[kb][w] = a0;
          cl[kb][w] = a1;
          sh[kb][w] = b0w;
          sl[kb][w] = b1w;
        }
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int kb = 0; kb < 2; ++kb) {
          are[rt] = mfma_bf16(A[rt][kb], ch[kb], are[rt]);
          are[rt] = mfma_bf16(A[rt][kb], cl[kb], are[rt]);
          aim[rt] = mfma_bf16(A[rt][kb], sh[kb], aim[rt]);
          aim[rt] = mfma_bf16(A[rt][kb], sl[kb], aim[rt]);
        }
    };
    if constexpr (RT == 1 && G >= 3 && G <= 4) {
      load(XA, AA, r0);
      for (int r = r0; r < r1; r += 2) {
        load(XB, AB, min(r + 1, r1 - 1));
        __builtin_amdgcn_sched_barrier(0);
        block(XA, AA);
        if (r + 1 < r1) {
          load(XA, AA, min(r + 2, r1 - 1));
          __builtin_amdgcn_sched_barrier(0);
          block(XB, AB);
        }
      }
    } else {
      for (int r = r0; r < r1; ++r) {
        load(XA, AA, r);
        block(XA, AA);
      }
    }
    b += r1 - r0;
  }
  const long k = (long)mb * 32 + q;
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int row = 32 * rt + mfma_row(i, h);
      if (row < D2) out[(long)row * NP + k] = make_float2(are[rt][i], aim[rt][i]);
    }
}

// Waves and ranges are laid out over the XCDs as in k_forward.
template <int G, int RT, bool kReduce>
__global__ __launch_bounds__(kBlock) void k_moments(
    int N, int D2, long n_blk, int groups,
    const u32x4* __restrict__ pixtab, const unsigned* __restrict__ nf_t,
    const u32x4* __restrict__ spotrec, const unsigned* __restrict__ offtab,
    const u32x4* __restrict__ momtab, float2* __restrict__ partial) {
  const int n_mb = (N + 31) / 32;
  const int NP = n_mb * 32;
  const int xcd = blockIdx.x % kXcds, slot = blockIdx.x / kXcds;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const long v = (long)slot * (kBlock / kWave) + wave;
  if (v >= (long)(groups / kXcds) * n_mb) return;  // wave-uniform exit
  const int gi = (int)(v / n_mb) * kXcds + xcd;
  const int mb = (int)(v % n_mb);
  moments_range<G, RT, kReduce>(N, D2, mb, n_blk * gi / groups,
                                n_blk * (gi + 1) / groups,
                       as_global(pixtab),
                       as_global(reinterpret_cast<const u32x4*>(nf_t)),
                       as_global(spotrec),
                       as_global(reinterpret_cast<const u32x4*>(offtab)),
                       as_global(momtab), partial + (long)gi * D2 * NP);
}

template <int G, int RT>
static hipError_t mom_g(const Geom& b, int N, int groups, hipStream_t s,
                        const unsigned short* pixtab, const unsigned* nf_t,
                        const unsigned short* spotrec, const unsigned* offtab,
                        const unsigned short* momtab, float* partial) {
  const int n_mb = (N + 31) / 32;
  const long n_blk = (long)b.n_tiles * kBlkPerTile;
  const long per_xcd = (long)(groups / kXcds) * n_mb;
  const long blocks_per_xcd =
      (per_xcd + kBlock / kWave - 1) / (kBlock / kWave);
  auto* const kern =
      b.reduce ? k_moments<G, RT, true> : k_moments<G, RT, false>;
  hipLaunchKernelGGL(kern, dim3((unsigned)(blocks_per_xcd * kXcds)),
                     dim3(kBlock), 0, s, N, 2 * b.D, n_blk, groups,
                     reinterpret_cast<const u32x4*>(pixtab), nf_t,
                     reinterpret_cast<const u32x4*>(spotrec), offtab,
                     reinterpret_cast<const u32x4*>(momtab),
                     reinterpret_cast<float2*>(partial));
  return hipGetLastError();
}

hipError_t launch_moments(const Geom& b, int N, int groups,
                          const unsigned short* pixtab, const unsigned* nf_t,
                          const unsigned short* spotrec,
                          const unsigned* offtab,
                          const unsigned short* momtab, float* partial,
                          hipStream_t s) {
  const bool two = 2 * b.D > 32;
  switch (b.groups) {
#define X(n)                                                               \
  case n:                                                                  \
    return two ? mom_g<n, 2>(b, N, groups, s, pixtab, nf_t, spotrec,       \
                             offtab, momtab, partial)                      \
               : mom_g<n, 1>(b, N, groups, s, pixtab, nf_t, spotrec,       \
                             offtab, momtab, partial);
    ASH_G_CASES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}

template <int G, int RT>
static int mom_blocks_per_cu() {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &n, k_moments<G, RT, false>, kBlock, 0) != hipSuccess) {
    (void)hipGetLastError();
    return 1;
  }
  return n > 0 ? n : 1;
}

int moments_blocks_per_cu(int groups, int D) {
  const bool two = 2 * D > 32;
  switch (groups) {
#define X(n) \
  case n:    \
    return two ? mom_blocks_per_cu<n, 2>() : mom_blocks_per_cu<n, 1>();
    ASH_G_CASES(X)
#undef X
    default:
      return 1;
  }
}

// Sum of the range partials of moment rows d (hi pieces) and D + d (lo
// pieces) in a fixed order; M = (re, -im) and, with G, the coefficient
// gradient Im(conj(G_k) M[k][d]).  One thread per (d, k), k fastest.
__global__ void k_moments_finish(int N, int D, int ranges,
                                 const float2* __restrict__ partial,
                                 const float2* __restrict__ Gk,
                                 float2* __restrict__ M,
                                 float* __restrict__ grad) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)N * D) return;
  const int d = (int)(t / N), k = (int)(t % N);
  const int NP = (N + 31) / 32 * 32;
  const long stride = (long)2 * D * NP;
  const float2 a = kahan_sum_strided(partial + (long)d * NP + k, stride, ranges);
  const float2 c =
      kahan_sum_strided(partial + (long)(D + d) * NP + k, stride, ranges);
  const float mr = a.x + c.x, mi = -(a.y + c.y);
  if (M) M[(long)k * D + d] = make_float2(mr, mi);
  if (grad) {
    const float2 g = Gk[k];
    grad[(long)k * D + d] = g.x * mi - g.y * mr;
  }
}

hipError_t launch_moments_finish(int N, int D, int ranges,
                                 const float* partial, const float* G,
                                 float* M, float* grad, hipStream_t s) {
  const long total = (long)N * D;
  hipLaunchKernelGGL(k_moments_finish, dim3((unsigned)((total + 255) / 256)),
                     dim3(256), 0, s, N, D, ranges,
                     reinterpret_cast<const float2*>(partial),
                     reinterpret_cast<const float2*>(G),
                     reinterpret_cast<float2*>(M), grad);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Windowed Strehl proxy S' = max |E|^2 / sum |E|^2 over each window of win^2
// consecutive spot fields (one wave per window; fixed-order reductions).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_window_strehl(
    int n_windows, int win2, const float2* __restrict__ E,
    float* __restrict__ S) {
  const int lane = threadIdx.x & (kWave - 1);
  const long wnd = (long)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  if (wnd >= n_windows) return;  // wave-uniform
  const float2* __restrict__ e = E + wnd * win2;
  float mx = 0.0f, sum = 0.0f;
  for (int j = lane; j < win2; j += kWave) {
    const float I = e[j].x * e[j].x + e[j].y * e[j].y;
    mx = fmaxf(mx, I);
    sum += I;
  }
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    mx = fmaxf(mx, __shfl_xor(mx, m, kWave));
    sum += __shfl_xor(sum, m, kWave);
  }
  if (lane == 0) S[wnd] = sum > 0.0f ? mx / sum : 0.0f;
}

hipError_t launch_window_strehl(int n_windows, int win2, const float* E,
                                float* S, hipStream_t s) {
  const int per_block = 256 / kWave;
  hipLaunchKernelGGL(k_window_strehl,
                     dim3((unsigned)((n_windows + per_block - 1) / per_block)),
                     dim3(256), 0, s, n_windows, win2,
                     reinterpret_cast<const float2*>(E), S);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Reductions of the forward partials (fixed order, compensated).
// ---------------------------------------------------------------------------
// Threads of the single-block kernels (reduction, weighted-GS update, loss).
constexpr int kUpd = 1024;

// One block of kUpd threads per kRedSpots spots: thread t takes spot
// k0 + t % kRedSpots and the rows t / kRedSpots + j * kRedPhases, so
// consecutive threads read consecutive spots of one row; each thread sums
// its rows in order (compensated), then the kRedPhases row phases of a
// spot combine in a fixed order: two butterfly steps over the four phases
// in a wave, then the waves' sums in wave order.
constexpr int kRedSpots = 16, kRedPhases = kUpd / kRedSpots;

__global__ __launch_bounds__(kUpd) void k_reduce(
    int N, int groups, const float2* __restrict__ part,
    float2* __restrict__ red) {
  __shared__ float2 sh[kUpd / kWave][kRedSpots];
  const int sp = threadIdx.x % kRedSpots, rp = threadIdx.x / kRedSpots;
  const int k = blockIdx.x * kRedSpots + sp;
  const int rows = rp < groups ? (groups - 1 - rp) / kRedPhases + 1 : 0;
  float2 v = make_float2(0.0f, 0.0f);
  if (k < N)
    v = kahan_sum_strided(part + (long)rp * N + k, (long)kRedPhases * N,
                          rows);
#pragma unroll
  for (int w = kRedSpots; w < kWave; w <<= 1) {
    v.x += __shfl_xor(v.x, w, kWave);
    v.y += __shfl_xor(v.y, w, kWave);
  }
  const int wave = threadIdx.x / kWave;
  if ((threadIdx.x & (kWave - 1)) < kRedSpots) sh[wave][sp] = v;
  __syncthreads();
  if (threadIdx.x < kRedSpots && k < N) {
    float2 r = sh[0][sp];
#pragma unroll
    for (int i = 1; i < kUpd / kWave; ++i) {
      r.x += sh[i][sp].x;
      r.y += sh[i][sp].y;
    }
    red[k] = r;
  }
}

hipError_t launch_reduce(int N, const FwdPlan& p, const float* partial,
                         float* red, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce, dim3((N + kRedSpots - 1) / kRedSpots),
                     dim3(kUpd), 0, s, N, p.groups,
                     reinterpret_cast<const float2*>(partial),
                     reinterpret_cast<float2*>(red));
  return hipGetLastError();
}

template <bool kDeviceScope = false>
__device__ __forceinline__ float2 sum_slices(const float2* __restrict__ red,
                                             int slices, int N, int k) {
  return kahan_sum_strided<kDeviceScope>(red + k, N, slices);
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

// Reduction over a block of NT threads (sh: one float per wave): a
// butterfly within each wave, then the waves' results in wave order; every
// thread returns the same value.  The wave count is a constant, so the LDS
// reads all go out before the first combine.
template <int NT = kUpd, typename Op>
__device__ float block_reduce(float v, float* sh, Op op) {
  constexpr int nw = NT / kWave;
#pragma unroll
  for (int w = 32; w >= 1; w >>= 1) v = op(v, __shfl_xor(v, w, kWave));
  if ((threadIdx.x & (kWave - 1)) == 0) sh[threadIdx.x / kWave] = v;
  __syncthreads();
  float r = sh[0];
#pragma unroll
  for (int i = 1; i < nw; ++i) r = op(r, sh[i]);
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

// Several block reductions in one LDS pass over a block of NT threads
// (sh: NV floats per wave): value i is combined with Op_i, in the order of
// block_reduce.
template <typename Op0, typename Op1, typename Op2, typename Op3,
          int NT = kUpd>
__device__ void block_reduce4(float* v, float* sh) {
  constexpr int NV = 4;
  const Op0 o0;
  const Op1 o1;
  const Op2 o2;
  const Op3 o3;
  auto op = [&](int i, float a, float b) {
    return i == 0 ? o0(a, b) : i == 1 ? o1(a, b) : i == 2 ? o2(a, b) : o3(a, b);
  };
#pragma unroll
  for (int i = 0; i < NV; ++i)
#pragma unroll
    for (int w = 32; w >= 1; w >>= 1) v[i] = op(i, v[i], __shfl_xor(v[i], w, kWave));
  constexpr int nw = NT / kWave;
  const int wave = threadIdx.x / kWave;
  if ((threadIdx.x & (kWave - 1)) == 0)
#pragma unroll
    for (int i = 0; i < NV; ++i) sh[i * nw + wave] = v[i];
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    float r = sh[i * nw];
#pragma unroll
    for (int j = 1; j < nw; ++j) r = op(i, r, sh[i * nw + j]);
    v[i] = r;
  }
  __syncthreads();
}

// The weighted-GS farfield update of one hologram by one block of NT
// threads (sh: four floats of LDS per wave).  W and Ebuf may be global or
// LDS (generic) pointers.
// meas: amplitudes that replace |E_k| in the weight update (experimental
// feedback), or null.  phase_mode: kPhaseFree projects onto arg E_k;
// kPhaseStore also stores arg E_k (turns) in fixph; kPhaseFixed projects
// onto the stored phases (phase-fixed weighted GS).  kDeviceScope: red was
// written by other blocks of the same launch (read at device scope).
template <int NT = kUpd, bool kDeviceScope = false>
__device__ __forceinline__ void wgs_update_block(
    int N, int slices, const float2* __restrict__ red,
    const float* __restrict__ t, float t_norm, float* __restrict__ W,
    float power, float eff_denom, unsigned* __restrict__ ypol,
    float2* __restrict__ Ebuf, float2* __restrict__ E_extra,
    float* __restrict__ stats, float* sh, const float* __restrict__ meas,
    float* __restrict__ fixph, int phase_mode) {
  const int tid = threadIdx.x;
  // with at most one spot per thread the spot's field and weight stay in
  // registers between the passes
  const bool one = N <= (int)blockDim.x;
  float2 e1 = make_float2(0.0f, 0.0f);
  float w1 = 0.0f, t1 = 0.0f;
  // pass 1: fields, |E|^2 and normalised intensities I = |E|^2 / t^2, and
  // the norm of the amplitudes that drive the weights
  float s_a2 = 0.0f, s_I = 0.0f, mx = 0.0f, mn = INFINITY, s_m2 = 0.0f;
  for (int k = tid; k < N; k += blockDim.x) {
    const float tk = t[k];
    const float2 e = sum_slices<kDeviceScope>(red, slices, N, k);
    if (one) {
      e1 = e;
      t1 = tk;
      w1 = W[k];
    } else {
      Ebuf[k] = e;
    }
    if (E_extra) E_extra[k] = e;
    const float a2 = e.x * e.x + e.y * e.y;
    const float I = a2 / (tk * tk);
    s_a2 += a2;
    s_I += I;
    mx = fmaxf(mx, I);
    mn = fminf(mn, I);
    if (meas) {
      const float m = fmaxf(meas[k], 0.0f);  // NaN and negatives: dark
      s_m2 += m * m;
    }
  }
  float r1[4] = {s_a2, s_I, mx, mn};
  block_reduce4<OpSum, OpSum, OpMax, OpMin, NT>(r1, sh);
  const float sum_a2 = r1[0], sum_I = r1[1], maxI = r1[2], minI = r1[3];
  const float norm_a =
      sqrtf(meas ? block_reduce<NT>(s_m2, sh, OpSum()) : sum_a2);
  const float meanI = sum_I / (float)N;
  // pass 2: spread of I, unnormalised weight update
  float s_v = 0.0f, s_w = 0.0f;
  for (int k = tid; k < N; k += blockDim.x) {
    const float2 e = one ? e1 : Ebuf[k];
    const float tk = one ? t1 : t[k];
    const float a2 = e.x * e.x + e.y * e.y;
    const float dI = a2 / (tk * tk) - meanI;
    s_v += dI * dI;
    const float a = meas ? fmaxf(meas[k], 0.0f) : sqrtf(a2);
    float wk = one ? w1 : W[k];
    if (a > 0.0f && norm_a > 0.0f) {
      const float r = (a / norm_a) / (tk / t_norm);
      wk = (power == 1.0f) ? wk / r : wk * powf(r, -power);
    }
    if (one)
      w1 = wk;
    else
      W[k] = wk;
    s_w += wk;
  }
  float r2[4] = {s_v, s_w, 0.0f, 0.0f};
  block_reduce4<OpSum, OpSum, OpSum, OpSum, NT>(r2, sh);
  const float var = r2[0] / (float)N;
  const float mean_w = r2[1] / (float)N;
  // pass 3: normalise weights, farfield projection y = W t exp(i psi) with
  // psi = arg E (arg 0 = 0) or the stored phase, in polar form (W t,
  // psi / 2 pi in pieces)
  for (int k = tid; k < N; k += blockDim.x) {
    const float wk = (one ? w1 : W[k]) / mean_w;
    const float tk = one ? t1 : t[k];
    W[k] = wk;
    float turns;
    if (phase_mode == kPhaseFixed) {
      turns = fixph[k];
    } else {
      const float2 e = one ? e1 : Ebuf[k];
      turns = atan2f(e.y, e.x) * kInv2Pi;
      if (phase_mode == kPhaseStore) fixph[k] = turns;
    }
    put_spot_field(ypol, N, k, wk * tk, turns);
  }
  if (stats && tid == 0) {
    stats[0] = eff_denom > 0.0f ? sum_a2 / eff_denom : 0.0f;
    stats[1] = (maxI + minI) > 0.0f ? 1.0f - (maxI - minI) / (maxI + minI)
                                    : 0.0f;
    stats[2] = meanI > 0.0f ? sqrtf(var) / meanI : 0.0f;
    stats[3] = sum_a2;
  }
}

__global__ __launch_bounds__(kUpd) void k_wgs_update(
    int N, int slices, const float2* __restrict__ red,
    const float* __restrict__ t, float t_norm, float* __restrict__ W,
    float power, float eff_denom, unsigned* __restrict__ ypol,
    float2* __restrict__ Ebuf, float2* __restrict__ E_extra,
    float* __restrict__ stats, const float* __restrict__ meas,
    float* __restrict__ fixph, int phase_mode) {
  __shared__ float sh[4 * kUpd / kWave];
  wgs_update_block(N, slices, red, t, t_norm, W, power, eff_denom, ypol, Ebuf,
                   E_extra, stats, sh, meas, fixph, phase_mode);
}

hipError_t launch_wgs_update(int N, const FwdPlan& p, const float* red,
                             const float* target, float t_norm, float* W,
                             float power, float eff_denom, unsigned* ypol,
                             float* Ebuf, float* E_extra, float* stats_row,
                             const float* meas, float* fixph, int phase_mode,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_wgs_update, dim3(1), dim3(kUpd), 0, s, N, p.slices,
                     reinterpret_cast<const float2*>(red), target, t_norm, W,
                     power, eff_denom, ypol,
                     reinterpret_cast<float2*>(Ebuf),
                     reinterpret_cast<float2*>(E_extra), stats_row, meas,
                     fixph, phase_mode);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Differentiable form: spot-amplitude loss and its field gradient (one
// block).  With Eh = E / s, d_k = |Eh_k|^2 - t_k:
//   L_spot = sum_k d_k^2,   G_k = dL/dRe E_k + i dL/dIm E_k = 4 d_k Eh_k / s,
// stored as spot-field records (|G_k|, arg G_k) for the adjoint.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void spot_loss_block(int N, int slices,
                                const float2* __restrict__ red,
                                const float* __restrict__ t, float inv_s,
                                unsigned* __restrict__ ypol,
                                float2* __restrict__ E_extra,
                                float* __restrict__ lossbuf, float* sh) {
  const int tid = threadIdx.x;
  float acc = 0.0f, comp = 0.0f;
  for (int k = tid; k < N; k += blockDim.x) {
    const float2 e = sum_slices(red, slices, N, k);
    if (E_extra) E_extra[k] = e;
    const float hr = e.x * inv_s, hi = e.y * inv_s;
    const float d = hr * hr + hi * hi - t[k];
    kahan_add(acc, comp, d * d);
    const float c = 4.0f * d * inv_s;
    put_spot_field(ypol, N, k, fabsf(c) * hypotf(hr, hi),
                   atan2f(c * hi, c * hr) * kInv2Pi);
  }
  const float L = block_reduce(acc, sh, OpSum());
  if (tid == 0) lossbuf[0] = L;
}

__global__ __launch_bounds__(kUpd) void k_spot_loss(
    int N, int slices, const float2* __restrict__ red,
    const float* __restrict__ t, float inv_s, unsigned* __restrict__ ypol,
    float2* __restrict__ E_extra, float* __restrict__ lossbuf) {
  __shared__ float sh[kUpd / kWave];
  spot_loss_block(N, slices, red, t, inv_s, ypol, E_extra, lossbuf, sh);
}

hipError_t launch_spot_loss(int N, const FwdPlan& p, const float* red,
                            const float* target, float inv_s, unsigned* ypol,
                            float* E_extra, float* lossbuf, hipStream_t s) {
  hipLaunchKernelGGL(k_spot_loss, dim3(1), dim3(kUpd), 0, s, N, p.slices,
                     reinterpret_cast<const float2*>(red), target, inv_s,
                     ypol,
                     reinterpret_cast<float2*>(E_extra), lossbuf);
  return hipGetLastError();
}

// loss = L_spot + tv_sum_scale * (sum of the per-wave TV sums, fixed order)
__global__ __launch_bounds__(kUpd) void k_loss_finish(
    int n, const float* __restrict__ tvp, float tv_sum_scale,
    const float* __restrict__ lossbuf, float* __restrict__ loss_out) {
  __shared__ float sh[kUpd / kWave];
  // this thread's values in index order, eight loads in flight
  float acc = 0.0f, comp = 0.0f;
  for (int k0 = threadIdx.x; k0 < n; k0 += 8 * kUpd) {
    float v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int k = k0 + u * kUpd;
      v[u] = k < n ? tvp[k] : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (k0 + u * kUpd < n) kahan_add(acc, comp, v[u]);
  }
  const float tv = block_reduce(acc, sh, OpSum());
  if (threadIdx.x == 0) loss_out[0] = lossbuf[0] + tv_sum_scale * tv;
}

hipError_t launch_loss_finish(int n_tvp, const float* tvp, float tv_sum_scale,
                              const float* lossbuf, float* loss_out,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_loss_finish, dim3(1), dim3(kUpd), 0, s, n_tvp, tvp,
                     tv_sum_scale, lossbuf, loss_out);
  return hipGetLastError();
}

// One Adam update per pixel (tile order), and the pixel's next nearfield
// record.  bc1 = 1 - beta1^step, bc2 = 1 - beta2^step.
__global__ void k_adam(Geom b, long total, float* __restrict__ phase,
                       float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ grad, float lr, float beta1,
                       float beta2, float eps, float bc1, float bc2,
                       const u32x4* __restrict__ pixtab,
                       u32x4* __restrict__ nf_rec) {
  const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= total) return;
  const int tile = (int)(gid / kTile), pix = (int)(gid % kTile);
  int i, j;
  if (!pixel_ij(b, tile, pix, &i, &j)) return;  // padding stays zero
  const long p = (long)j * b.nx + i;
  const float g = grad[p];
  const float mk = beta1 * m[p] + (1.0f - beta1) * g;
  const float vk = beta2 * v[p] + (1.0f - beta2) * g * g;
  m[p] = mk;
  v[p] = vk;
  const float ph = phase[p] - lr * (mk / bc1) / (sqrtf(vk / bc2) + eps);
  phase[p] = ph;
  const float turns = rad_to_turns(ph);
  // next nearfield record; the magnitudes stay
  nf_rec[nf_index(tile, pix, 0)] = nearfield_record(
      pixel_nl_words(pixtab, b.groups, tile, pix), turns);
}

hipError_t launch_adam(const Geom& b, float* phase, float* m, float* v,
                       const float* grad, float lr, float beta1, float beta2,
                       float eps, float bc1, float bc2,
                       const unsigned short* pixtab, unsigned* nf_t,
                       hipStream_t s) {
  const long total = (long)b.n_tiles * kTile;
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((total + 255) / 256)), dim3(256),
                     0, s, b, total, phase, m, v, grad, lr, beta1, beta2, eps,
                     bc1, bc2, reinterpret_cast<const u32x4*>(pixtab),
                     reinterpret_cast<u32x4*>(nf_t));
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Phase-gradient total variation.  With forward differences of the wrapped
// phase, dx(j, i) = wrap(phi[j][i+1] - phi[j][i]) (0 in the last column),
// dy(j, i) likewise along j (0 in the last row), wrap into (-pi, pi], the
// term of pixel (i, j) is q(j, i) = sqrt(dx^2 + dy^2 + eps^2).  Returns the
// derivative of sum q over the whole SLM by phi[j][i] (each root through
// the differences it contains; wrap has unit slope) and sets *term to
// q(j, i).
// ---------------------------------------------------------------------------
__device__ inline float wrap_pi(float d) {
  const float r = (kPiF - d) - k2PiF * floorf((kPiF - d) * kInv2Pi);
  return kPiF - r;
}

__device__ inline void tv_diffs(const float* __restrict__ ph, int nx, int ny,
                                int i, int j, float* dx, float* dy) {
  const float c = ph[(long)j * nx + i];
  *dx = i + 1 < nx ? wrap_pi(ph[(long)j * nx + i + 1] - c) : 0.0f;
  *dy = j + 1 < ny ? wrap_pi(ph[(long)(j + 1) * nx + i] - c) : 0.0f;
}

__device__ inline float tv_grad_at(const float* __restrict__ ph, int nx,
                                   int ny, int i, int j, float eps,
                                   float* term) {
  const float e2 = eps * eps;
  float dx, dy;
  tv_diffs(ph, nx, ny, i, j, &dx, &dy);
  const float q = sqrtf(dx * dx + dy * dy + e2);
  *term = q;
  float g = -(dx + dy) / q;
  if (i > 0) {  // the root of (i - 1, j) holds dx(j, i - 1)
    float ex, ey;
    tv_diffs(ph, nx, ny, i - 1, j, &ex, &ey);
    g += ex / sqrtf(ex * ex + ey * ey + e2);
  }
  if (j > 0) {  // the root of (i, j - 1) holds dy(j - 1, i)
    float ex, ey;
    tv_diffs(ph, nx, ny, i, j - 1, &ex, &ey);
    g += ey / sqrtf(ex * ex + ey * ey + e2);
  }
  return g;
}

// ---------------------------------------------------------------------------
// Adjoint of one wave: the 32 pixels of one tile row (first pixel p0 of
// tile `tile`) over all spots.  g(x) = sum_k |y_k| exp(2 pi i (tau_k(x) +
// psi_k)); the epilogue writes g, arg g, the next nearfield record in tile
// order, or the phase gradient (see AdjOut).  `wv` indexes the per-wave TV
// sums.
// ---------------------------------------------------------------------------
// Epilogue of an adjoint row: the butterfly over the spot columns leaves
// h = g(x) of pixel p0 + (row of the lane) in every even lane, which writes
// what `o` asks for.
template <int G>
__device__ __forceinline__ void adjoint_epilogue(
    float* gr, float* gi, int nx, int ny, int tiles_x, int tile, int p0,
    long wv, const GLOBAL u32x4* __restrict__ pixtab,
    const GLOBAL float* __restrict__ amp_t, const AdjOut& o) {
  const int lane = threadIdx.x & (kWave - 1);
  const int h = lane >> 5, q = lane & 31;
  bfly_reduce(gr, gi, q);
  // one result per lane pair; the odd lane of a pair idles in the epilogue
  const bool lead = (q & 1) == 0;
  const int pix = p0 + mfma_row(bfly_index(q), h);
  const int i = (tile % tiles_x) * kTileW + pix % kTileW;
  const int j = (tile / tiles_x) * kTileH + pix / kTileW;
  const bool inside = lead && i < nx && j < ny;
  const long p = (long)j * nx + i;
  const float vr = gr[0], vi = gi[0];
  if (lead && (o.outs & (kOutField | kOutPhase))) {
    const float ang = atan2f(vi, vr);  // atan2(0, 0) = 0
    if (o.outs & kOutField)  // next nearfield: the magnitudes stay
      reinterpret_cast<u32x4*>(o.nf_t)[nf_index(tile, pix, 0)] =
          nearfield_record(
              pixel_nl_words((const u32x4*)pixtab, G, tile, pix),
              rad_to_turns(ang));
    if (inside && (o.outs & kOutPhase)) o.phase[p] = ang;
  }
  if (inside && (o.outs & kOutG))
    reinterpret_cast<float2*>(o.g)[p] = make_float2(vr, vi);
  if (o.outs & kOutGrad) {
    float term = 0.0f;
    if (inside) {
      // Im(conj(f) h) with f = A exp(i phi)
      float sn, cs;
      sincosf(o.phase_in[p], &sn, &cs);
      float gv = amp_t[(long)tile * kTile + pix] * (cs * vi - sn * vr);
      if (o.tv_scale != 0.0f)
        gv += o.tv_scale * tv_grad_at(o.phase_in, nx, ny, i, j, o.tv_eps, &term);
      o.grad[p] = gv;
    }
    if (o.tvp) {  // this wave's TV terms, in a fixed order
#pragma unroll
      for (int w = 32; w >= 1; w >>= 1) term += __shfl_xor(term, w, kWave);
      if (lane == 0) o.tvp[wv] = term;
    }
  }
}

template <int G, bool kReduce>
__device__ __forceinline__ void adjoint_row(
    int N, int nx, int ny, int tiles_x, int tile, int p0, long wv,
    const GLOBAL u32x4* __restrict__ pixtab,
    const GLOBAL u32x4* __restrict__ spotrec,
    const GLOBAL u32x4* __restrict__ offtab,
    const GLOBAL u32x4* __restrict__ yrec,
    const GLOBAL float* __restrict__ amp_t, const AdjOut& o) {
  const int lane = threadIdx.x & (kWave - 1);
  const int h = lane >> 5, q = lane & 31;
  u32x4 X[G];
  const unsigned lane_spot = h * 32 + q;
#pragma unroll
  for (int gg = 0; gg < G; ++gg)
    X[gg] = (pixtab + (((long)tile * G + gg) * 2 + h) * kTile + p0)[q];
  const int NB = (N + 31) / 32, NP = NB * 32;
  const unsigned lane_ot = h * NP + q;
  // per spot block: the lane's spot record, groups 0..G-2 from the record
  // and the last group from the per-tile slots, with the spot-field phase
  // (p 4..6) OR-ed in from half 0's spot-field entry (half 1's entry has
  // zeros there); both carry the magnitude.  Spot tables are padded to
  // whole blocks with zero records.
  const GLOBAL u32x4* __restrict__ ot_t = offtab + (long)tile * 2 * NP;
  float gr[16], gi[16];
  const unsigned off_spot = lane_spot * 16u, off_ot = lane_ot * 16u;
  const rsrc_t rs = make_rsrc(spotrec, (unsigned long)NB * G * 64 * 16);
  const rsrc_t ro = make_rsrc(ot_t, (unsigned long)2 * NP * 16);
  const rsrc_t ry = make_rsrc(yrec, (unsigned long)NB * 64 * 16);
  // spot block nb; the first one starts the sums
  auto block = [&](int nb, auto init) {
    u32x4 S[G];
#pragma unroll
    for (int gg = 0; gg < G - 1; ++gg)
      S[gg] = bload4(rs, off_spot, (unsigned)(nb * G + gg) * 64u * 16u);
    u32x4 last = bload4(ro, off_ot, (unsigned)nb * 32u * 16u);
    const u32x4 yv = bload4(ry, off_spot, (unsigned)nb * 64u * 16u);
    __builtin_amdgcn_sched_barrier(0);  // loads before the products
    last[2] |= yv[0];
    last[3] |= yv[1];
    S[G - 1] = last;
    const float m = __uint_as_float(yv[2]);
    const floatx16 th = phase_block<G>(X, S);
    accumulate<false, kReduce, decltype(init)::value>(th, m, gr, gi);
  };
  block(0, std::true_type());
  for (int nb = 1; nb < NB; ++nb) block(nb, std::false_type());
  adjoint_epilogue<G>(gr, gi, nx, ny, tiles_x, tile, p0, wv, pixtab, amp_t, o);
}

// Adjoint of one hologram: the four waves of a block are four rows of one
// tile; blocks reach the XCDs round-robin, so each XCD gets a contiguous run
// of blocks in tile order and the blocks of one tile share its L2.
template <int G, bool kReduce>
__global__ __launch_bounds__(kBlock) void k_adjoint(
    int N, int nx, int ny, int tiles_x, const u32x4* __restrict__ pixtab,
    const u32x4* __restrict__ spotrec, const unsigned* __restrict__ offtab,
    const unsigned* __restrict__ ypol, const float* __restrict__ amp_t,
    AdjOut o) {
  const int nblk = gridDim.x, per = nblk / kXcds, extra = nblk % kXcds;
  const int xcd = blockIdx.x % kXcds, slot = blockIdx.x / kXcds;
  const int lin = xcd * per + min(xcd, extra) + slot;
  const int wv = lin * (kBlock / kWave) +
                 __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  adjoint_row<G, kReduce>(N, nx, ny, tiles_x, wv / kBlkPerTile,
                          (wv % kBlkPerTile) * 32, wv, as_global(pixtab),
                          as_global(spotrec),
                          as_global(reinterpret_cast<const u32x4*>(offtab)),
                          as_global(reinterpret_cast<const u32x4*>(ypol)),
                          as_global(amp_t), o);
}

template <int G>
static hipError_t adj_g(const Geom& b, int N, const unsigned short* pixtab,
                        const unsigned short* spotrec, const unsigned* offtab,
                        const unsigned* ypol, const float* amp_t,
                        const AdjOut& o, hipStream_t s) {
  const int blocks = b.n_tiles * kBlkPerTile / (kBlock / kWave);
  auto* const kern = b.reduce ? k_adjoint<G, true> : k_adjoint<G, false>;
  hipLaunchKernelGGL(kern, dim3(blocks), dim3(kBlock), 0, s, N, b.nx,
                     b.ny, b.tiles_x, reinterpret_cast<const u32x4*>(pixtab),
                     reinterpret_cast<const u32x4*>(spotrec), offtab, ypol,
                     amp_t, o);
  return hipGetLastError();
}

hipError_t launch_adjoint(const Geom& b, int N, const unsigned short* pixtab,
                          const unsigned short* spotrec,
                          const unsigned* offtab, const unsigned* ypol,
                          const float* amp_t, const AdjOut& o, hipStream_t s) {
  switch (b.groups) {
#define X(n)      \
  case n:         \
    return adj_g<n>(b, N, pixtab, spotrec, offtab, ypol, amp_t, o, s);
    ASH_G_CASES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------------------
// Batched form: persistent launches over the work items of many holograms.
// Each wave takes items from its XCD's queue (block id mod 8, as blocks
// reach the XCDs round-robin), then from the other queues in turn; it asks
// for the next item before computing the current one so that the atomic's
// latency is hidden.  Before its first take from a queue a wave reads the
// queue's counter and passes over a queue already drained: counters only
// grow, so a stale read costs one take and never skips an item, while the
// many waves that find every queue drained at the end cost loads, not
// serialised atomics.  Every wave stops after the eighth queue.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int wave_take(int* ctr) {
  int v = 0;
  if ((threadIdx.x & (kWave - 1)) == 0) v = atomicAdd(ctr, 1);
  return __builtin_amdgcn_readfirstlane(v);
}

__device__ __forceinline__ int4 uniform_item(const int4* items, long i) {
  const int4 it = items[i];
  return make_int4(__builtin_amdgcn_readfirstlane(it.x),
                   __builtin_amdgcn_readfirstlane(it.y),
                   __builtin_amdgcn_readfirstlane(it.z), 0);
}

template <typename F>
__device__ __forceinline__ void drain_queues(const int4* __restrict__ items,
                                             const int* __restrict__ qoff,
                                             int* __restrict__ ctr, F&& work) {
  const int home = blockIdx.x % kXcds;
  for (int qi = 0; qi < kXcds; ++qi) {
    const int x = (home + qi) % kXcds;
    int* const c = ctr + x * kCtrPad;
    const int base = qoff[x], cnt = qoff[x + 1] - base;
    const int seen = __builtin_amdgcn_readfirstlane(
        __hip_atomic_load(c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    if (seen >= cnt) continue;
    int idx = wave_take(c);
    while (idx < cnt) {
      const int4 it = uniform_item(items, (long)base + idx);
      const int nxt = wave_take(c);
      work(it);
      idx = nxt;
    }
  }
}

template <int G, bool kReduce>
__global__ __launch_bounds__(kBlock) void k_batch_forward(
    const HoloDesc* __restrict__ hd, const int4* __restrict__ items,
    const int* __restrict__ qoff, int* __restrict__ ctr) {
  drain_queues(items, qoff, ctr, [&](const int4& it) {
    const HoloDesc& d = hd[it.x];
    const long b0 = (long)it.y * d.L;
    const long b1 = min(b0 + d.L, d.n_blk);
    // two register sets where they keep this kernel's waves per SIMD
    forward_range<G, kReduce, G <= 3 || G == 5 || G == 9>(
        d.N, it.z, b0, b1, as_global(d.pixtab),
        as_global(reinterpret_cast<const u32x4*>(d.nf_t)), as_global(d.amp_t),
        as_global(d.spotrec),
        as_global(reinterpret_cast<const u32x4*>(d.offtab)),
        d.partial + (long)it.y * d.N);
  });
}

// Adjoint of a batch: one block per quarter tile {holo, tile * 4 +
// quarter} of the item list (negative holo: idle padding), four rows, one
// per wave; the hardware hands the blocks out as slots free up.
template <int G, bool kReduce>
__global__ __launch_bounds__(kBlock) void k_batch_adjoint(
    const HoloDesc* __restrict__ hd, const int4* __restrict__ items,
    int last) {
  const int4 it = uniform_item(items, blockIdx.x);
  if (it.x < 0) return;
  const HoloDesc& d = hd[it.x];
  AdjOut o;
  o.outs = last ? kOutPhase : kOutField;
  o.phase = d.phase;
  o.nf_t = d.nf_t;
  const int wv = it.y * (kBlock / kWave) +
                 __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  adjoint_row<G, kReduce>(d.N, d.nx, d.ny, d.tiles_x, wv / kBlkPerTile,
                          (wv % kBlkPerTile) * 32, wv, as_global(d.pixtab),
                          as_global(d.spotrec),
                          as_global(reinterpret_cast<const u32x4*>(d.offtab)),
                          as_global(reinterpret_cast<const u32x4*>(d.ypol)),
                          as_global(d.amp_t), o);
}

// one block per {holo, 64 spots, slice of kRowsPerSlice forward ranges}
__global__ __launch_bounds__(64) void k_batch_reduce(
    const HoloDesc* __restrict__ hd, const int4* __restrict__ blocks) {
  const int4 bl = blocks[blockIdx.x];
  const HoloDesc& d = hd[bl.x];
  const int k = bl.y + threadIdx.x;
  if (k >= d.N) return;
  const int r0 = bl.z * kRowsPerSlice;
  const int r1 = min(r0 + kRowsPerSlice, d.n_ranges);
  d.red[(long)bl.z * d.N + k] =
      kahan_sum_strided(d.partial + (long)r0 * d.N + k, d.N, r1 - r0);
}

__global__ __launch_bounds__(kUpd) void k_batch_update(
    const HoloDesc* __restrict__ hd, float power) {
  __shared__ float sh[4 * kUpd / kWave];
  const HoloDesc& d = hd[blockIdx.x];
  wgs_update_block(d.N, d.slices, d.red, d.target, d.t_norm, d.W, power,
                   d.eff_denom, d.ypol, d.Ebuf, nullptr, nullptr, sh, nullptr,
                   nullptr, kPhaseFree);
}

// ---------------------------------------------------------------------------
// Fused adjoint and next forward.  Inside a weighted-GS loop the adjoint of
// iteration n gives each pixel its phase of iteration n + 1, and that pixel's
// terms of the next forward need nothing else; so one pass over a range of
// pixel blocks (tile rows) runs, per block, the adjoint over all spots, the
// projection onto the phase, and the block's share of the next forward, from
// one load of the pixel records.  The pixel table, the dominant memory
// stream of holograms with few spots, is then read once per iteration
// instead of twice, and no nearfield records are written.
//
// Both halves keep their sums inside the lanes.  The adjoint takes the
// forward's operand order (rows: 16 spots per lane, lane: pixel) and weights
// each spot row by its magnitude from a table staged in LDS; the forward
// takes the adjoint's order (rows: 16 pixels per lane, lane: spot) and
// weights each pixel row by its basis amplitude.  Lane l and lane l + 32
// hold the two row halves of one column, joined by one permlane32 swap, so
// the per-block butterfly of the separate kernels disappears.  The
// forward's running sums of the range, one per lane and spot block, live in
// LDS.
// ---------------------------------------------------------------------------
// LDS floats per wave: the spot magnitudes [NP], the forward sums
// [NP / 32][64] complex.
__host__ __device__ inline long fused_lds_floats(int np_max) {
  return (long)np_max * 5;
}

// Lane-half join: in every lane, the value of lane l % 32 plus the value of
// lane l % 32 + 32 (the same order in both halves).
__device__ __forceinline__ float join_halves(float x) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x),
                                                  __float_as_uint(x), false,
                                                  false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// The values of a lane that hold spot rows below n_valid (1..32): value i
// holds row 8 (i / 4) + 4h + i % 4 in lane half h, so values i < 4k hold
// rows < 8k in both halves.
__device__ __forceinline__ int valid_values(int n_valid) {
  return 4 * ((min(n_valid, 32) + 7) / 8);
}

// Sum, with per-value weights w, of w cos(2 pi theta) and w sin(2 pi theta)
// over one 32x32 block of phases (16 per lane) into four running pairs;
// kN < 16: the first kN values only, for a block whose later rows are
// padding (spots past N).
template <bool kReduce, int kN = 16>
__device__ __forceinline__ void accumulate_rows(const floatx16& th,
                                                const floatx4* w, float* sr,
                                                float* si) {
#pragma unroll
  for (int i = 0; i < kN; ++i) {
    const float r = kReduce ? __builtin_amdgcn_fractf(th[i]) : th[i];
    const float m = w[i >> 2][i & 3];
    sr[i & 3] = fmaf(m, __builtin_amdgcn_cosf(r), sr[i & 3]);
    si[i & 3] = fmaf(m, __builtin_amdgcn_sinf(r), si[i & 3]);
  }
}


// Adjoint of a pair of pixel blocks (records X0: row r, X1: row r + 1)
// over NB spot blocks: on return lane half h holds g(x) of pixel q of row
// r + h.  The magnitudes of the spot rows come from ym4 (LDS).  nv_last:
// the values of the last spot block that hold spots (valid_values).
template <int G, bool kReduce>
__device__ __forceinline__ float2 adjoint_pair(
    int NB, int nv_last, const u32x4* X0, const u32x4* X1, rsrc_t rs,
    rsrc_t ro, rsrc_t ry, const floatx4* ym4, unsigned off_spot,
    unsigned off_ot, int h) {
  float ar[4] = {0.0f, 0.0f, 0.0f, 0.0f}, ai[4] = {0.0f, 0.0f, 0.0f, 0.0f};
  float br[4] = {0.0f, 0.0f, 0.0f, 0.0f}, bi[4] = {0.0f, 0.0f, 0.0f, 0.0f};
  // spot block nb, its first kN values (the rest are padding rows)
  auto block = [&](int nb, auto kn) {
    constexpr int kN = decltype(kn)::value;
    u32x4 S[G];
#pragma unroll
    for (int g = 0; g < G - 1; ++g)
      S[g] = bload4(rs, off_spot, (unsigned)(nb * G + g) * 64u * 16u);
    u32x4 last = bload4(ro, off_ot, (unsigned)nb * 32u * 16u);
    const u32x4 yv = bload4(ry, off_spot, (unsigned)nb * 64u * 16u);
    floatx4 w[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) w[j] = ym4[nb * 8 + 2 * j + h];
    __builtin_amdgcn_sched_barrier(0);  // loads before the products
    last[2] |= yv[0];
    last[3] |= yv[1];
    S[G - 1] = last;
    const floatx16 th0 = phase_block<G>(S, X0);
    const floatx16 th1 = phase_block<G>(S, X1);
    accumulate_rows<kReduce, kN>(th0, w, ar, ai);
    accumulate_rows<kReduce, kN>(th1, w, br, bi);
  };
  for (int nb = 0; nb < NB - 1; ++nb)
    block(nb, std::integral_constant<int, 16>());
  // the last block: only the values that hold spots
  if (nv_last == 16)
    block(NB - 1, std::integral_constant<int, 16>());
  else if (nv_last == 12)
    block(NB - 1, std::integral_constant<int, 12>());
  else if (nv_last == 8)
    block(NB - 1, std::integral_constant<int, 8>());
  else
    block(NB - 1, std::integral_constant<int, 4>());
  const auto jr = __builtin_amdgcn_permlane32_swap(
      __float_as_uint((ar[0] + ar[1]) + (ar[2] + ar[3])),
      __float_as_uint((br[0] + br[1]) + (br[2] + br[3])), false, false);
  const auto ji = __builtin_amdgcn_permlane32_swap(
      __float_as_uint((ai[0] + ai[1]) + (ai[2] + ai[3])),
      __float_as_uint((bi[0] + bi[1]) + (bi[2] + bi[3])), false, false);
  return make_float2(__uint_as_float(jr[0]) + __uint_as_float(jr[1]),
                     __uint_as_float(ji[0]) + __uint_as_float(ji[1]));
}

// Forward terms of a pair of pixel blocks (records with their phases, X0:
// row r, X1: row r + 1 of the tile whose amplitudes ra covers) over NB spot
// blocks, added to the lane's running sums acc_s[nb][lane] (LDS): the sums
// over the lane's 16 pixel rows of both blocks of A(x) cos(2 pi theta) and
// A(x) sin(2 pi theta), theta = tau_k(x) - phi(x).
template <int G, bool kReduce>
__device__ __forceinline__ void forward_pair(
    int NB, int r, const u32x4* X0, const u32x4* X1, rsrc_t rs, rsrc_t ro,
    rsrc_t ra, unsigned off_spot, unsigned off_ot, unsigned off_amp,
    unsigned m2, unsigned m3, float2* acc_s, int lane) {
  floatx4 a0[4], a1[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    a0[j] = __builtin_bit_cast(
        floatx4, bload4(ra, off_amp, (unsigned)(r * 32 + 8 * j) * 4u));
    a1[j] = __builtin_bit_cast(
        floatx4, bload4(ra, off_amp, (unsigned)(r * 32 + 32 + 8 * j) * 4u));
  }
  for (int nb = 0; nb < NB; ++nb) {
    u32x4 S[G];
#pragma unroll
    for (int g = 0; g < G - 1; ++g)
      S[g] = bload4(rs, off_spot, (unsigned)(nb * G + g) * 64u * 16u);
    u32x4 last = bload4(ro, off_ot, (unsigned)nb * 32u * 16u);
    float2 o = acc_s[nb * kWave + lane];
    __builtin_amdgcn_sched_barrier(0);
    last[2] |= m2;
    last[3] |= m3;
    S[G - 1] = last;
    const floatx16 th0 = phase_block<G>(X0, S);
    const floatx16 th1 = phase_block<G>(X1, S);
    float fr[4] = {0.0f, 0.0f, 0.0f, 0.0f}, fi[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    accumulate_rows<kReduce>(th0, a0, fr, fi);
    accumulate_rows<kReduce>(th1, a1, fr, fi);
    o.x += (fr[0] + fr[1]) + (fr[2] + fr[3]);
    o.y += (fi[0] + fi[1]) + (fi[2] + fi[3]);
    acc_s[nb * kWave + lane] = o;
  }
}

// One wave: pixel blocks [b0, b1) of a hologram with N spots, two blocks
// (rows r and r + 1 of a tile) at a time; b0 and b1 are even, so a pair
// never leaves its tile.  yrec: the spot-field records of this iteration
// (the dense magnitudes follow them); ymag_s, acc_s: the wave's LDS; row:
// the range's forward sums of the next iteration, E_k for k < N.  Each
// spot block's records are loaded once for both rows, whose products form
// two independent matrix-core chains; after the adjoint's join, lane half
// h holds row r + h, so the phase of each of the 64 pixels is taken once.
// Modes (a template parameter, so that each kernel holds only its own
// path's registers): kFusedMid as above; kFusedFirst takes the phases from
// `phase` ([ny][nx], radians: the loop's start) and runs the forward only;
// kFusedLast runs the adjoint only and writes arg g to `phase`.
template <int G, bool kReduce, int kMode>
__device__ __forceinline__ void fused_range(
    int N, int nx, int ny, int tiles_x, float* __restrict__ phase,
    long b0, long b1, const GLOBAL u32x4* __restrict__ pixtab,
    const GLOBAL u32x4* __restrict__ spotrec,
    const GLOBAL u32x4* __restrict__ offtab,
    const GLOBAL u32x4* __restrict__ yrec,
    const GLOBAL float* __restrict__ amp_t, float* ymag_s, float2* acc_s,
    float2* __restrict__ row) {
  const int lane = threadIdx.x & (kWave - 1);
  const int h = lane >> 5, q = lane & 31;
  const int NB = (N + 31) / 32, NP = NB * 32;
  const int nv_last =
      __builtin_amdgcn_readfirstlane(valid_values(N - (NB - 1) * 32));
  const GLOBAL float* __restrict__ ymag =
      reinterpret_cast<const GLOBAL float*>(yrec + (long)NB * 64);
  for (int k = lane; k < NP; k += kWave) ymag_s[k] = ymag[k];
  for (int nb = 0; nb < NB; ++nb)
    acc_s[nb * kWave + lane] = make_float2(0.0f, 0.0f);
  // a wave's LDS operations complete in order; the fences keep the
  // compiler from moving the table's reads above its writes
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const floatx4* ym4 = reinterpret_cast<const floatx4*>(ymag_s);
  const unsigned off_pix = (unsigned)(h * kTile + q) * 16u;
  const unsigned off_spot = (unsigned)(h * 32 + q) * 16u;
  const unsigned off_ot = (unsigned)(h * NP + q) * 16u;
  const unsigned off_amp = (unsigned)h * 16u;
  // -1 at p 4..6 of the spot record's last group against the pixel phase
  const unsigned m2 = h ? 0u : (kBf16MinusOne | (kBf16MinusOne << 16));
  const unsigned m3 = h ? 0u : kBf16MinusOne;
  const rsrc_t rs = make_rsrc(spotrec, (unsigned long)NB * G * 64 * 16);
  const rsrc_t ry = make_rsrc(yrec, (unsigned long)NB * 64 * 16);
  // tile column and row of the current tile, stepped with it
  int tx = (int)((b0 / kBlkPerTile) % tiles_x);
  int ty = (int)((b0 / kBlkPerTile) / tiles_x);
  for (long b = b0; b < b1; b += 2) {
    const long t = b / kBlkPerTile;
    const int r = (int)(b - t * kBlkPerTile);
    if (r == 0 && b != b0 && ++tx == tiles_x) {
      tx = 0;
      ++ty;
    }
    const rsrc_t rx = make_rsrc(pixtab + t * G * 2 * kTile,
                                (unsigned long)G * 2 * kTile * 16);
    const rsrc_t ro = make_rsrc(offtab + t * 2 * NP, (unsigned long)2 * NP * 16);
    const rsrc_t ra = make_rsrc(amp_t + t * kTile, (unsigned long)kTile * 4);
    u32x4 X0[G], X1[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      X0[g] = bload4(rx, off_pix, (unsigned)(g * 2 * kTile + r * 32) * 16u);
      X1[g] = bload4(rx, off_pix, (unsigned)(g * 2 * kTile + r * 32 + 32) * 16u);
    }
    // the lane's pixel after the adjoint's join: row r + h, column q
    const int pix = (r + h) * 32 + q;
    const int pi = tx * kTileW + pix % kTileW;
    const int pj = ty * kTileH + pix / kTileW;
    const bool inside = pi < nx && pj < ny;
    const long pp = (long)pj * nx + pi;
    float turns = 0.0f;
    if (kMode == kFusedFirst) {
      if (inside) turns = rad_to_turns(phase[pp]);
    } else {
      const float2 gv = adjoint_pair<G, kReduce>(NB, nv_last, X0, X1, rs, ro,
                                                 ry, ym4, off_spot, off_ot, h);
      const float ang = atan2f(gv.y, gv.x);  // atan2(0, 0) = 0
      if (kMode == kFusedLast) {
        if (inside) phase[pp] = ang;
        continue;
      }
      turns = rad_to_turns(ang);
    }
    // the pixel's phase (as the adjoint's epilogue writes it) in the last
    // group of its record: half 0's words for row r stay, row r + 1's move
    // from half 1 to half 0
    unsigned ph[3];
    split3f(turns, ph);
    const unsigned w2 = ph[0] | (ph[1] << 16), w3 = ph[2] | (kBf16One << 16);
    const auto s2 = __builtin_amdgcn_permlane32_swap(w2, w2, false, false);
    const auto s3 = __builtin_amdgcn_permlane32_swap(w3, w3, false, false);
    if (h == 0) {
      X0[G - 1][2] = w2;
      X0[G - 1][3] = w3;
      X1[G - 1][2] = s2[1];
      X1[G - 1][3] = s3[1];
    }
    // forward of the next iteration over the pair's 64 pixels
    forward_pair<G, kReduce>(NB, r, X0, X1, rs, ro, ra, off_spot, off_ot,
                             off_amp, m2, m3, acc_s, lane);
  }
  if (kMode == kFusedLast) return;
  // E_k = sum_x A(x) exp(-2 pi i (tau_k(x) - phi(x))) of the range
  for (int nb = 0; nb < NB; ++nb) {
    const float2 o = acc_s[nb * kWave + lane];
    const float er = join_halves(o.x), ei = -join_halves(o.y);
    const int k = nb * 32 + q;
    if (h == 0 && k < N) row[k] = make_float2(er, ei);
  }
}

// Fused launch of a batch: each wave takes units {holo, range} from the
// queues (as the forward) and runs fused_range over the range, writing the
// range's row of forward partial sums (mode: see fused_range).
// Waves per SIMD the register allocator must allow the fused launches and
// the one-launch kernel, which runs the same rows: 4 up to G = 3, 3 up to
// G = 6; left to itself the compiler lands one step lower.  At these
// targets a few values spill at some G (the one-launch kernel at G = 2, 3,
// 5 and 6, the fused middle launch at G = 3 and 6), outside the loops over
// spot blocks.
constexpr int fused_waves(int G) { return G <= 3 ? 4 : G <= 6 ? 3 : 1; }

template <int G, bool kReduce, int kMode>
__global__ __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu(fused_waves(G)))) void k_batch_fused(
    const HoloDesc* __restrict__ hd, const int4* __restrict__ items,
    const int* __restrict__ qoff, int* __restrict__ ctr, int np_max) {
  extern __shared__ float lds[];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  float* const base = lds + (long)wave * fused_lds_floats(np_max);
  drain_queues(items, qoff, ctr, [&](const int4& it) {
    const HoloDesc& d = hd[it.x];
    const long b0 = (long)it.y * d.L;
    const long b1 = min(b0 + d.L, d.n_blk);
    fused_range<G, kReduce, kMode>(
        d.N, d.nx, d.ny, d.tiles_x, d.phase, b0, b1,
        as_global(d.pixtab), as_global(d.spotrec),
        as_global(reinterpret_cast<const u32x4*>(d.offtab)),
        as_global(reinterpret_cast<const u32x4*>(d.ypol)), as_global(d.amp_t),
        base, reinterpret_cast<float2*>(base + np_max),
        d.partial + (long)it.y * d.N);
  });
}

template <int G, bool kReduce>
static hipError_t bfus_g(int grid, int np_max, int mode, const HoloDesc* d,
                         const int4* items, const int* qoff, int* ctr,
                         hipStream_t s) {
  const size_t lds = (size_t)(kBlock / kWave) * fused_lds_floats(np_max) * 4;
  auto* const kern = mode == kFusedFirst ? k_batch_fused<G, kReduce, kFusedFirst>
                     : mode == kFusedMid ? k_batch_fused<G, kReduce, kFusedMid>
                                         : k_batch_fused<G, kReduce, kFusedLast>;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(kBlock), lds, s, d, items, qoff,
                     ctr, np_max);
  return hipGetLastError();
}

template <int G, bool kReduce>
static int fus_blocks_per_cu(int np_max) {
  const size_t lds = (size_t)(kBlock / kWave) * fused_lds_floats(np_max) * 4;
  int n = 0;
  // the middle mode's kernel, which runs every iteration but the last
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &n, k_batch_fused<G, kReduce, kFusedMid>, kBlock, lds) != hipSuccess) {
    (void)hipGetLastError();
    return 1;
  }
  return n > 0 ? n : 1;
}

hipError_t launch_batch_fused(int G, bool reduce, int grid, int np_max,
                              int mode, const HoloDesc* d, const int4* items,
                              const int* qoff, int* ctr, hipStream_t s) {
  if (np_max < 32 || np_max > kFusedSpots || np_max % 32 ||
      mode < kFusedFirst || mode > kFusedLast)
    return hipErrorInvalidValue;
  switch (G) {
#define X(n)                                                              \
  case n:                                                                 \
    return reduce                                                         \
               ? bfus_g<n, true>(grid, np_max, mode, d, items, qoff, ctr, s) \
               : bfus_g<n, false>(grid, np_max, mode, d, items, qoff, ctr, s);
    ASH_G_CASES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}

int fused_blocks_per_cu(int G, bool reduce, int np_max) {
  switch (G) {
#define X(n)                                                  \
  case n:                                                     \
    return reduce ? fus_blocks_per_cu<n, true>(np_max)        \
                  : fus_blocks_per_cu<n, false>(np_max);
    ASH_G_CASES(X)
#undef X
    default:
      return 1;
  }
}

template <int G, bool kReduce>
static hipError_t bfwd_g(int grid, const HoloDesc* d, const int4* items,
                         const int* qoff, int* ctr, hipStream_t s) {
  hipLaunchKernelGGL((k_batch_forward<G, kReduce>), dim3(grid), dim3(kBlock),
                     0, s, d, items, qoff, ctr);
  return hipGetLastError();
}

template <int G, bool kReduce>
static hipError_t badj_g(int grid, const HoloDesc* d, const int4* items,
                         int last, hipStream_t s) {
  hipLaunchKernelGGL((k_batch_adjoint<G, kReduce>), dim3(grid), dim3(kBlock),
                     0, s, d, items, last);
  return hipGetLastError();
}

hipError_t launch_batch_forward(int G, bool reduce, int grid,
                                const HoloDesc* d, const int4* items,
                                const int* qoff, int* ctr, hipStream_t s) {
  switch (G) {
#define X(n)                                                       \
  case n:                                                          \
    return reduce ? bfwd_g<n, true>(grid, d, items, qoff, ctr, s)  \
                  : bfwd_g<n, false>(grid, d, items, qoff, ctr, s);
    ASH_G_CASES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_batch_adjoint(int G, bool reduce, int grid,
                                const HoloDesc* d, const int4* items,
                                int last, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  switch (G) {
#define X(n)                                                        \
  case n:                                                           \
    return reduce ? badj_g<n, true>(grid, d, items, last, s)        \
                  : badj_g<n, false>(grid, d, items, last, s);
    ASH_G_CASES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_batch_reduce(const HoloDesc* d, const int4* blocks,
                               int n_blocks, hipStream_t s) {
  if (n_blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch_reduce, dim3(n_blocks), dim3(64), 0, s, d,
                     blocks);
  return hipGetLastError();
}

hipError_t launch_batch_update(int H, const HoloDesc* d, float power,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_batch_update, dim3(H), dim3(kUpd), 0, s, d, power);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Batched form in one launch.  The blocks of a hologram meet once per
// iteration at a barrier (a counter per hologram).  A block's partial sums
// are released to device scope (its accelerator die's L2 written back)
// before it counts itself in; the counter is polled, and the other blocks'
// sums read after it, with device-scope loads, which are coherent across
// the dies and invalidate no cache, so the L2s keep the records that the
// blocks still computing read.  The loads of the sums are issued after the
// poll that saw the full count returned (they follow it in program order
// behind a workgroup barrier), so they see the sums.  The launch is
// cooperative, so all blocks are resident and every block reaches every
// barrier; a barrier that waits longer than kBarrierTicks sets *err and
// every block leaves, so the kernel ends in any case.
// ---------------------------------------------------------------------------
constexpr unsigned long long kBarrierTicks = 1000000000ull;  // 10 s at 100 MHz

size_t persist_lds_bytes(int N) {
  const int NP = (N + 31) / 32 * 32;
  // per-wave forward sums [4][NP] float2 (reused for the fields E in the
  // update), the weights [NP], and each wave's fused-range LDS
  return (size_t)NP * (4 * 8 + 4) +
         (size_t)(kBlock / kWave) * fused_lds_floats(NP) * 4;
}

// Wait until the counter reaches `target` (thread 0); false on error.
__device__ __forceinline__ bool persist_barrier(int* ctr, int target,
                                                int* err) {
  __shared__ int ok;
  __syncthreads();  // the block's writes are done
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_fetch_add(ctr, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int good = 1;
    const unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
    while (__hip_atomic_load(ctr, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
        good = 0;
        break;
      }
      if (__builtin_amdgcn_s_memrealtime() - t0 > kBarrierTicks) {
        __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        good = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    ok = good;
  }
  __syncthreads();
  return ok != 0;
}


template <int G, bool kReduce>
__global__ __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu(fused_waves(G)))) void k_batch_persist(
    const PHolo* __restrict__ hd, const PBlock* __restrict__ blks, int n_iter,
    float power, int np_max, int* __restrict__ err) {
  extern __shared__ float lds[];
  __shared__ float sh[4 * kBlock / kWave];
  const int bi = blockIdx.x;
  const int holo = __builtin_amdgcn_readfirstlane(blks[bi].holo);
  const int j = __builtin_amdgcn_readfirstlane(blks[bi].j);
  const long b0 = blks[bi].b0, b1 = blks[bi].b1;
  const PHolo& d = hd[holo];
  const int N = d.N, NP = (N + 31) / 32 * 32;
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid / kWave);
  float2* wrow = reinterpret_cast<float2*>(lds);  // [4][NP]
  float* Ws = lds + 8 * NP;                         // [NP]
  // each wave's fused-range LDS (spot magnitudes, running forward sums)
  float* const fl = lds + 9 * np_max + (long)wave * fused_lds_floats(np_max);
  unsigned* yb = d.yblk + (long)j * NP * 9;
  // the block's weights and its spot-field records past N (zero)
  for (int k = tid; k < N; k += kBlock) Ws[k] = d.W[k];
  for (int k = N + tid; k < NP; k += kBlock) {
    u32x4* y4 = reinterpret_cast<u32x4*>(yb) + (long)(k / 32) * 64 + k % 32;
    y4[0] = u32x4{0u, 0u, 0u, 0u};
    y4[32] = u32x4{0u, 0u, 0u, 0u};
    reinterpret_cast<float*>(yb)[(long)NP * 8 + k] = 0.0f;
  }
  __threadfence_block();
  __syncthreads();
  // the wave's share of the block's pixel blocks, in whole pairs
  const long pairs = (b1 - b0) / 2;
  const long w0 = b0 + 2 * (pairs * wave / (kBlock / kWave));
  const long w1 = b0 + 2 * (pairs * (wave + 1) / (kBlock / kWave));
  float2* const my_row = wrow + (long)wave * NP;
  const GLOBAL u32x4* const ycur = as_global(reinterpret_cast<const u32x4*>(yb));
  for (int it = 0; it <= n_iter; ++it) {
    // fused ranges over the wave's pixel blocks: the forward of the start
    // phases; then each iteration's adjoint with the next forward; after
    // the last update the adjoint alone, which writes the phases
#define FUSED_ARGS                                                         \
  N, d.nx, d.ny, d.tiles_x, d.phase, w0, w1, as_global(d.pixtab),          \
      as_global(d.spotrec),                                                \
      as_global(reinterpret_cast<const u32x4*>(d.offtab)), ycur,           \
      as_global(d.amp_t), fl, reinterpret_cast<float2*>(fl + np_max), my_row
    if (it == n_iter) {
      fused_range<G, kReduce, kFusedLast>(FUSED_ARGS);
      break;
    }
    if (it == 0)
      fused_range<G, kReduce, kFusedFirst>(FUSED_ARGS);
    else
      fused_range<G, kReduce, kFusedMid>(FUSED_ARGS);
#undef FUSED_ARGS
    __syncthreads();
    float2* rows_it = d.rows + (long)(it & 1) * d.n_blocks * N;
    for (int k = tid; k < N; k += kBlock) {  // the waves' sums in order
      float2 v = wrow[k];
#pragma unroll
      for (int w = 1; w < kBlock / kWave; ++w) {
        v.x += wrow[(long)w * NP + k].x;
        v.y += wrow[(long)w * NP + k].y;
      }
      rows_it[(long)j * N + k] = v;
    }
    if (!persist_barrier(d.ctr, d.n_blocks * (it + 1), err)) return;
    // the weight update of the whole hologram from all blocks' sums, into
    // this block's weights and spot-field records
    wgs_update_block<kBlock, true>(N, d.n_blocks, rows_it, d.target,
                                   d.t_norm, Ws, power, 0.0f, yb, wrow,
                                   nullptr, nullptr, sh, nullptr, nullptr,
                                   kPhaseFree);
    __threadfence_block();
    __syncthreads();
  }
  if (j == 0)
    for (int k = tid; k < N; k += kBlock) d.W[k] = Ws[k];
}

template <int G, bool kReduce>
static hipError_t bpersist_g(int grid, size_t lds, const PHolo* hd,
                             const PBlock* blks, int n_iter, float power,
                             int np_max, int* err, hipStream_t s) {
  void* args[] = {(void*)&hd, (void*)&blks, (void*)&n_iter, (void*)&power,
                  (void*)&np_max, (void*)&err};
  return hipLaunchCooperativeKernel(
      reinterpret_cast<const void*>(&k_batch_persist<G, kReduce>),
      dim3(grid), dim3(kBlock), args, (unsigned)lds, s);
}

hipError_t launch_batch_persist(int G, bool reduce, int grid, size_t lds,
                                const PHolo* hd, const PBlock* blks,
                                int n_iter, float power, int np_max, int* err,
                                hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  if (n_iter < 1 || np_max < 32 || np_max > kPersistSpots || np_max % 32 ||
      lds < persist_lds_bytes(np_max))
    return hipErrorInvalidValue;
  switch (G) {
#define X(n)                                                                \
  case n:                                                                   \
    return reduce ? bpersist_g<n, true>(grid, lds, hd, blks, n_iter, power, \
                                        np_max, err, s)                     \
                  : bpersist_g<n, false>(grid, lds, hd, blks, n_iter, power,\
                                         np_max, err, s);
    ASH_G_CASES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}

template <int G, bool kReduce>
static int persist_occ(size_t lds) {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &n, k_batch_persist<G, kReduce>, kBlock, lds) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return n;
}

int persist_blocks_per_cu(int G, bool reduce, size_t lds) {
  switch (G) {
#define X(n) \
  case n:    \
    return reduce ? persist_occ<n, true>(lds) : persist_occ<n, false>(lds);
    ASH_G_CASES(X)
#undef X
    default:
      return 0;
  }
}

template <typename K>
static int occupancy(K kern) {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kern, kBlock, 0) !=
      hipSuccess) {
    (void)hipGetLastError();
    return 1;
  }
  return n > 0 ? n : 1;
}

int batch_blocks_per_cu(int G, bool reduce, bool forward) {
  switch (G) {
#define X(n)                                                          \
  case n:                                                             \
    return forward ? (reduce ? occupancy(k_batch_forward<n, true>)    \
                             : occupancy(k_batch_forward<n, false>))  \
                   : (reduce ? occupancy(k_batch_adjoint<n, true>)    \
                             : occupancy(k_batch_adjoint<n, false>));
    ASH_G_CASES(X)
#undef X
    default:
      return 1;
  }
}

// ---------------------------------------------------------------------------
// Device-resident scratch of the allocation-free forward
// (ash_forward_noalloc): the forward's partial sums and their reduction live
// in this file-scope array instead of context buffers.  Host code never
// passes `scratch` itself to a kernel (in host code the name is a host-side
// stand-in, not a device address): its device address is resolved once per
// device with hipGetSymbolAddress, with that device current, and kept here.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxScratchDevices] = {};
}  // namespace

hipError_t resolve_static_scratch(int device) {
  if (device < 0 || device >= kMaxScratchDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_addr[device]) return hipSuccess;
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return e;
  if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
  void* p = nullptr;
  e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (cur != device) {
    const hipError_t e2 = hipSetDevice(cur);
    if (e == hipSuccess) e = e2;
  }
  if (e != hipSuccess) return e;
  if (!p) return hipErrorInvalidSymbol;
  g_scratch_addr[device] = p;
  return hipSuccess;
}

void* static_scratch(int device) {
  if (device < 0 || device >= kMaxScratchDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_addr[device];
}

FwdPlan plan_forward(int n_tiles, int N, int blocks_per_cu, int n_cu) {
  FwdPlan p;
  const int n_mb = (N + 31) / 32;
  const long n_blk = (long)n_tiles * kBlkPerTile;
  // About eight rounds of resident waves, each wave a range of pixel
  // blocks: with several rounds the waves of a SIMD start at different
  // times, so their matrix-core and vector phases interleave (one round of
  // long waves runs in lockstep and measured 15-20 % slower; at 1920x1200
  // with 2000 spots eight rounds beat four by 3 %).  Ranges of at least 32
  // blocks keep the per-range work (tile slots, butterfly, partial sums)
  // small.
  const long waves = (long)blocks_per_cu * (kBlock / kWave) * n_cu;
  long want = 8 * waves / n_mb;
  // ranges of at least 32 blocks, or of down to 8 where fewer spots would
  // otherwise leave resident slots idle
  long cap = waves / n_mb < n_blk / 8 ? waves / n_mb : n_blk / 8;
  if (cap < n_blk / 32) cap = n_blk / 32;
  if (want > cap) want = cap;
  want = want / kXcds * kXcds;     // whole rounds over the XCDs
  if (want < kXcds) want = kXcds;  // (empty ranges give zeros)
  p.groups = (int)want;
  return p;
}

// Ranges of the moment transform: about two rounds of resident waves (its
// partial sums carry 2D rows per spot, and the finish sums all ranges).
int plan_moment_ranges(int n_tiles, int N, int blocks_per_cu, int n_cu) {
  const int n_mb = (N + 31) / 32;
  const long n_blk = (long)n_tiles * kBlkPerTile;
  const long waves = (long)blocks_per_cu * (kBlock / kWave) * n_cu;
  long want = 2 * waves / n_mb;
  if (want > n_blk / 32) want = n_blk / 32;
  want = want / kXcds * kXcds;
  if (want < kXcds) want = kXcds;
  return (int)want;
}

}  // namespace ash
