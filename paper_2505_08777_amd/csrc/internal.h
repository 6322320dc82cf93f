// Internal state and kernel launchers of libash (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "ash.h"

namespace ash {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

// Pixel tile: 32 columns x 16 rows.  Tiles are stored tile-major, pixels
// row-major inside a tile, ragged tiles padded with zero-amplitude pixels.
// A 32-pixel block (one tile row) is the column block of one matrix-core
// product.
constexpr int kTileW = 32;
constexpr int kTileH = 16;
constexpr int kTile = kTileW * kTileH;
constexpr int kBlkPerTile = kTile / 32;
constexpr int kBlock = 256;  // threads per block for the transforms
constexpr int kWave = 64;
constexpr int kMaxGroups = 12;  // 16-slot groups per record (compiled)
constexpr int kXcds = 8;        // accelerator dies (separate L2s) on MI355X

// Geometry and record shape, passed to kernels by value.
struct Geom {
  int nx = 0, ny = 0;
  double cx = 0, cy = 0, R = 1;
  int D = 0;
  int nl = 0;      // modes with a monomial of total degree >= 2
  int pieces = 2;  // bf16 pieces per remainder / coefficient (2 or 3)
  int groups = 1;  // 16-slot groups per record = MFMAs per 32x32 block
  int reduce = 1;  // range-reduce phases before the hardware sine/cosine
  int tiles_x = 0, tiles_y = 0, n_tiles = 0;
};

__host__ __device__ int slots_per_mode(int pieces);
int groups_for(int nl, int pieces);

struct Basis {
  Geom g;
  std::vector<int> nl_mode;  // [nl] original mode index of nonlinear slot
  std::vector<double> aff;   // [D][3] coefficient of 1, xh, yh in Z_d
  double amp_sum2 = 0;       // sum over pixels of A^2 (host, FP64)
  int n_mono = 0;
};

struct Spots {
  int N = 0;
  double t_norm2 = 0;  // sum t^2 (host, FP64)
  float rm_bound = 0;  // max over tiles and spots of sum_s |c_s| max|Rm_s|
  float theta_bound = 0;  // max |phase| in turns of any spot-pixel pair
};

struct Buffers {
  // basis
  unsigned short* pixtab = nullptr;  // [tile][group][half][kTile][8] bf16
  float* amp_t = nullptr;            // [n_tiles][kTile]
  unsigned* field_t = nullptr;  // nearfield [n_tiles * 16][half][32] u32x4
  float* fmag_t = nullptr;      // [n_tiles][kTile] |f| of a complex input
  double* aff_dev = nullptr;         // [D][3]
  int* nlmode_dev = nullptr;         // [nl]
  double* tilez = nullptr;           // [n_tiles][nl][3] Z^nl, d/di, d/dj
  float* rmax = nullptr;             // [n_tiles][nl] max |Rm_s| in a tile
  int32_t* d_pow = nullptr;          // [n_mono][2]
  double* d_nlcoef = nullptr;        // [nl][n_mono]
  double* d_coef = nullptr;          // [D][n_mono] whole basis
  unsigned short* momtab = nullptr;  // [block][kb][h][2D][8] bf16 A Z_d
  size_t cap_pixtab = 0;             // in unsigned shorts
  // spots (NP: N padded to whole 32-spot blocks, padding zero)
  unsigned short* spotrec = nullptr;  // [N/32][group][half][32][8] bf16
  unsigned* offtab = nullptr;   // [n_tiles][half][NP] u32x4 last-group slots
  float* target = nullptr;            // [N]
  unsigned* y = nullptr;        // spot fields [NP] u32x4 (phase words, |y|)
  float* Ebuf = nullptr;              // [N][2] fields of the last forward
  double* w64 = nullptr;              // [N][D] coefficients (radians)
  double* spot64 = nullptr;           // [N][3] constant, alpha, beta (turns)
  unsigned* bound = nullptr;          // [2] float bits: remainder, |phase|
  float* partial = nullptr;           // [groups][N][2]
  float* red = nullptr;               // [N][2] reduced forward sums
  // differentiable form
  float* grad = nullptr;              // [P] phase gradient
  float* tvp = nullptr;               // [n_tiles * kBlkPerTile] TV sums
  float* lossbuf = nullptr;           // [1] spot term of the loss
  float* mom_partial = nullptr;  // [ranges][2D][NP] moment range sums
  float* fixph = nullptr;        // [NP] stored farfield phases (turns)
  size_t cap_spots = 0, cap_spotrec = 0, cap_w = 0, cap_off = 0,
         cap_partial = 0, cap_red = 0, cap_mom = 0;
};

// Phase of the weighted-GS farfield projection: arg E (free), arg E also
// stored (store), or the stored phases (fixed).
enum : int { kPhaseFree = 0, kPhaseStore = 1, kPhaseFixed = 2 };

// Timing events: read only after a stream synchronisation, so they need no
// system-scope fence (which writes back and invalidates caches at every
// record and slows the work between them).
constexpr unsigned kProfEventFlags = hipEventDisableSystemFence;

struct FwdPlan {
  int groups = 0;  // pixel-block ranges (forward partial rows)
  int slices = 1;  // rows of red per spot: k_reduce sums all ranges at once
  int mom_groups = 0;  // pixel-block ranges of the moment transform
};

// Size of the device-resident scratch of the allocation-free forward.
constexpr size_t kStaticScratchBytes = size_t(16) << 20;
// Resolve (once per device; that device is made current for the call) and
// look up the device address of that scratch.  static_scratch returns null
// for a device whose address was never resolved.
hipError_t resolve_static_scratch(int device);
void* static_scratch(int device);

// Resident forward blocks per CU for a compiled record length.
int forward_blocks_per_cu(int groups);
FwdPlan plan_forward(int n_tiles, int N, int blocks_per_cu, int n_cu);

// ---- launchers (kernels.hip) ----
hipError_t launch_build_pixtab(const Geom& b, const int32_t* d_pow,
                               const double* d_nlcoef, int n_mono,
                               const float* amp_dev, unsigned short* pixtab,
                               float* amp_t, hipStream_t s);
hipError_t launch_build_tilebasis(const Geom& b, const int32_t* d_pow,
                                  const double* d_nlcoef, int n_mono,
                                  double* tilez, float* rmax, hipStream_t s);
hipError_t launch_prep_spots(const Geom& b, int N, const double* d_w,
                             const double* d_aff, const int* d_nlmode,
                             const double* tilez, const float* rmax,
                             unsigned short* spotrec, double* spot64,
                             unsigned* offtab, unsigned* bound_bits,
                             hipStream_t s);
hipError_t launch_make_field(const Geom& b, const float* phase,
                             const float* field, const float* amp_t,
                             const unsigned short* pixtab, unsigned* nf_t,
                             float* fmag, hipStream_t s);
hipError_t launch_to_polar(int N, const float* y, unsigned* ypol,
                           hipStream_t s);
hipError_t launch_forward(const Geom& b, int N, const FwdPlan& p,
                          const unsigned short* pixtab, const unsigned* nf_t,
                          const float* mag, const unsigned short* spotrec,
                          const unsigned* offtab, float* partial,
                          hipStream_t s);
hipError_t launch_reduce(int N, const FwdPlan& p, const float* partial,
                         float* red, hipStream_t s);
hipError_t launch_build_momtab(const Geom& b, const int32_t* d_pow,
                               const double* d_coef, int n_mono,
                               const float* amp_t, unsigned short* momtab,
                               hipStream_t s);
int moments_blocks_per_cu(int groups, int D);
int plan_moment_ranges(int n_tiles, int N, int blocks_per_cu, int n_cu);
hipError_t launch_moments(const Geom& b, int N, int groups,
                          const unsigned short* pixtab, const unsigned* nf_t,
                          const unsigned short* spotrec,
                          const unsigned* offtab,
                          const unsigned short* momtab, float* partial,
                          hipStream_t s);
hipError_t launch_window_strehl(int n_windows, int win2, const float* E,
                                float* S, hipStream_t s);
hipError_t launch_moments_finish(int N, int D, int ranges,
                                 const float* partial, const float* G,
                                 float* M, float* grad, hipStream_t s);
hipError_t launch_finish_E(int N, const FwdPlan& p, const float* red,
                           float* E, hipStream_t s);
hipError_t launch_wgs_update(int N, const FwdPlan& p, const float* red,
                             const float* target, float t_norm, float* W,
                             float power, float eff_denom, unsigned* ypol,
                             float* Ebuf, float* E_extra, float* stats_row,
                             const float* meas, float* fixph, int phase_mode,
                             hipStream_t s);
enum AdjOutFlags { kOutG = 1, kOutPhase = 2, kOutField = 4, kOutGrad = 8 };
// What the adjoint's epilogue writes for its pixel x, with h = g(x):
struct AdjOut {
  int outs = 0;
  float* g = nullptr;            // kOutG: [P][2] h
  float* phase = nullptr;        // kOutPhase: [P] arg h
  unsigned* nf_t = nullptr;      // kOutField: next nearfield A exp(i arg h)
  const float* phase_in = nullptr;  // kOutGrad: [P] phase of f = A e^{i phi}
  float* grad = nullptr;         // kOutGrad: [P] Im(conj(f) h) + TV term
  float tv_scale = 0.0f;         // lambda / P; 0 leaves out the TV term
  float tv_eps = 0.0f;
  float* tvp = nullptr;          // [n_tiles * kBlkPerTile] per-wave TV sums
};
hipError_t launch_adjoint(const Geom& b, int N, const unsigned short* pixtab,
                          const unsigned short* spotrec,
                          const unsigned* offtab, const unsigned* ypol,
                          const float* amp_t, const AdjOut& o, hipStream_t s);
hipError_t launch_spot_loss(int N, const FwdPlan& p, const float* red,
                            const float* target, float inv_s, unsigned* ypol,
                            float* E_extra, float* lossbuf, hipStream_t s);
hipError_t launch_loss_finish(int n_tvp, const float* tvp, float tv_sum_scale,
                              const float* lossbuf, float* loss_out,
                              hipStream_t s);
hipError_t launch_adam(const Geom& b, float* phase, float* m, float* v,
                       const float* grad, float lr, float beta1, float beta2,
                       float eps, float bc1, float bc2,
                       const unsigned short* pixtab, unsigned* nf_t,
                       hipStream_t s);

// ---- batched form ----
constexpr int kRowsPerSlice = 32;  // forward partial rows per reduce slice

// One hologram of a batch as the batched kernels see it (device copy).
struct HoloDesc {
  const u32x4* pixtab;
  unsigned* nf_t;    // nearfield records
  const u32x4* spotrec;
  unsigned* offtab;  // per-tile slot planes
  unsigned* ypol;    // spot-field records
  const float* amp_t;
  float2* partial;  // [n_ranges][N]
  float2* red;      // [slices][N]
  const float* target;
  float* W;      // spot weights (caller's)
  float* phase;  // phase (caller's): written by the last adjoint
  float2* Ebuf;
  long n_blk;
  int N, nx, ny, tiles_x;
  int L;         // pixel blocks per forward range
  int n_ranges;  // ceil(n_blk / L)
  int slices;    // ceil(n_ranges / kRowsPerSlice)
  float t_norm, eff_denom;
};

// Work items: forward {holo, range, spot block, 0} in 8 per-XCD queues
// items[qoff[x] .. qoff[x+1]) of a persistent launch, with take counters
// ctr[x * kCtrPad] (one counter per 256 bytes: atomics on one cache line
// serialise, so the queues' counters do not share lines); adjoint blocks
// {holo, tile * 4 + quarter, 0, 0} (holo < 0: idle); reduce blocks {holo,
// first spot, slice, 0}.
constexpr int kCtrPad = 64;
hipError_t launch_batch_forward(int G, bool reduce, int grid,
                                const HoloDesc* d, const int4* items,
                                const int* qoff, int* ctr, hipStream_t s);
hipError_t launch_batch_adjoint(int G, bool reduce, int grid,
                                const HoloDesc* d, const int4* items,
                                int last, hipStream_t s);
hipError_t launch_batch_reduce(const HoloDesc* d, const int4* blocks,
                               int n_blocks, hipStream_t s);
hipError_t launch_batch_update(int H, const HoloDesc* d, float power,
                               hipStream_t s);
// Resident blocks per CU of the persistent kernels.
int batch_blocks_per_cu(int G, bool reduce, bool forward);
// Armed failure injections (ash_inject_failure): each call consumes one
// armed failure of its kind if any is left and then returns true.
bool injected_alloc_failure();
bool injected_barrier_failure();

// Fused adjoint and next forward (per-phase form, members of at most
// kFusedSpots spots): units {holo, range, 0, 0} in 8 per-XCD queues like the
// forward's; np_max is the largest padded spot count of the launch's
// holograms (a multiple of 32), which sizes the LDS of each wave.
// Modes: the first forward (phase from the descriptors' phase arrays),
// an adjoint and the next forward, the last adjoint (writes the phase).
constexpr int kFusedSpots = 512;
constexpr int kFusedFirst = 0, kFusedMid = 1, kFusedLast = 2;
hipError_t launch_batch_fused(int G, bool reduce, int grid, int np_max,
                              int mode, const HoloDesc* d, const int4* items,
                              const int* qoff, int* ctr, hipStream_t s);
int fused_blocks_per_cu(int G, bool reduce, int np_max);

// ---- batched form in one launch (holograms of at most kPersistSpots) ----
// Every block owns a contiguous range of one hologram's 32-pixel blocks and
// runs all iterations: fused rows over its range (the adjoint of the last
// spot fields, then the forward of the new phases, partial sums per block),
// a barrier with the hologram's other blocks, and the weight update of the
// whole hologram from all blocks' partial sums (every block computes it,
// the same way, so no second barrier is needed).  After the last update a
// pass of adjoint rows writes the phase.
constexpr int kPersistSpots = 512;

struct PHolo {
  const u32x4* pixtab;
  const u32x4* spotrec;
  const unsigned* offtab;
  const float* amp_t;
  const float* target;
  float* W;                // spot weights (caller's), in/out
  float* phase;            // phase (caller's), in/out
  float2* rows;            // [2][n_blocks][N] per-block forward sums
  unsigned* yblk;          // [n_blocks][NP * 9] per-block spot-field records
  int* ctr;                // barrier counter (zero at launch)
  long n_blk;              // 32-pixel blocks (tile rows)
  int N, nx, ny, tiles_x, groups, n_blocks;
  float t_norm;
};
// Block `j` of hologram `holo` owns pixel blocks [b0, b1).
struct PBlock {
  int holo, j;
  long b0, b1;
};
// Each block's pixel-block range (an even number of pixel blocks) is split
// over its four waves in pairs; every iteration is one pass of fused rows
// (adjoint of the last fields, forward of the new phases).  `np_max` is the
// batch's largest spot count rounded up to 32.  `err` is set when a barrier
// waits longer than its time limit (then every block leaves the loop).
hipError_t launch_batch_persist(int G, bool reduce, int grid, size_t lds,
                                const PHolo* hd, const PBlock* blks,
                                int n_iter, float power, int np_max, int* err,
                                hipStream_t s);
// Resident blocks per CU of the persistent kernel with `lds` bytes of
// dynamic LDS, and its LDS need for N spots.
int persist_blocks_per_cu(int G, bool reduce, size_t lds);
size_t persist_lds_bytes(int N);

}  // namespace ash

struct ash_prof_rec {
  int cat;
  hipEvent_t start, stop;
};

struct ash_ctx {
  int device = 0;
  int n_cu = 0;
  int precision = ASH_PRECISION_AUTO;
  int prof_mask = 0;  // categories timed with events (bit 1 << category)
  int prof_stride = 1;          // time one launch in every prof_stride
  long prof_seen[4] = {0, 0, 0, 0};  // launches per category since enable
  std::vector<ash_prof_rec> prof;     // recorded pairs (in use)
  std::vector<hipEvent_t> prof_pool;  // free events
  hipStream_t stream = nullptr;
  std::string err;
  bool has_basis = false, has_spots = false;
  bool has_fixed = false;  // farfield phases stored since the last set_spots
  ash::Basis basis;
  ash::Spots spots;
  ash::Buffers buf;
  ash::FwdPlan plan;
};
