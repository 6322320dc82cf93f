// Internal state and kernel launchers of libash (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "ash.h"

namespace ash {

// Pixel tile: 64 columns x 16 rows.  Tiles are stored tile-major, pixels
// row-major inside a tile, ragged tiles padded with zero-amplitude pixels.
constexpr int kTileW = 64;
constexpr int kTileH = 16;
constexpr int kTile = kTileW * kTileH;
constexpr int kBlock = 256;  // threads per block for the transforms
constexpr int kWave = 64;

// Half of the padded contraction length 2 KH >= 4 + nl (one MFMA per pair).
int half_k(int nl);

struct Basis {
  int nx = 0, ny = 0;
  double cx = 0, cy = 0, R = 1;
  int D = 0;
  int nl = 0;      // modes with a monomial of total degree >= 2
  int kh = 0;      // half_k(nl): MFMAs per 32x32 block
  int rec = 0;     // floats per pixel / spot record: 2 kh
  int tiles_x = 0, tiles_y = 0, n_tiles = 0;
  std::vector<int> nl_mode;   // [nl] original mode index of nonlinear slot
  std::vector<double> aff;    // [D][3] coefficient of 1, xh, yh in Z_d
  double amp_sum2 = 0;        // sum over pixels of A^2 (host, FP64)
};

struct Spots {
  int N = 0;
  int srec = 0;        // floats per spot record (== basis rec)
  double t_norm2 = 0;  // sum t^2 (host, FP64)
};

struct Buffers {
  float* pixtab = nullptr;   // [n_tiles][kTile][rec]: 1, di, dj, Rm_s (split)
  float* amp_t = nullptr;    // [n_tiles][kTile]
  float* field_t = nullptr;  // [n_tiles][kTile][2] nearfield (A, phi turns)
  double* tilez = nullptr;   // [n_tiles][nl][3] Z^nl, d/di, d/dj at origins
  float* spotrec = nullptr;  // [N][rec]: 0, 0, 0, c_s in turns (split)
  float* offtab = nullptr;   // [n_tiles][N][4] wrapped offset, a, b, 0
  float* target = nullptr;   // [N]
  float* y = nullptr;        // [N][2] spot fields (|y|, psi turns)
  float* Ebuf = nullptr;     // [N][2] fields of the last WGS forward
  double* w64 = nullptr;     // [N][D] staged coefficients (radians)
  double* spot64 = nullptr;  // [N][3] FP64 constant, alpha, beta (turns)
  double* aff_dev = nullptr; // [D][3] affine coefficients of each mode
  int* nlmode_dev = nullptr; // [nl]
  float* partial = nullptr;  // [groups][N][2]
  float* red = nullptr;      // [slices][N][2]
  size_t cap_spots = 0, cap_w = 0, cap_off = 0, cap_partial = 0, cap_red = 0;
};

struct FwdPlan {
  int groups = 0;           // pixel-block ranges (forward partial rows)
  int slices = 0;           // second-level reduction rows
  int rows_per_slice = 0;
};

// Resident forward blocks per CU for a compiled contraction length.
int forward_blocks_per_cu(int kh);
FwdPlan plan_forward(int n_tiles, int N, int blocks_per_cu, int n_cu);

// ---- launchers (kernels.hip) ----
hipError_t launch_build_pixtab(const Basis& b, const int32_t* d_pow,
                               const double* d_nlcoef, int n_mono,
                               const float* amp_dev, float* pixtab,
                               float* amp_t, double* tilez, hipStream_t s);
hipError_t launch_prep_spots(const Basis& b, int N, const double* d_w,
                             const double* d_aff, const int* d_nlmode,
                             const double* tilez, float* spotrec,
                             float* offtab, double* spot64, hipStream_t s);
hipError_t launch_make_field(const Basis& b, const float* phase,
                             const float* field, const float* amp_t,
                             float* field_t, hipStream_t s);
hipError_t launch_to_polar(int N, const float* y, float* ypol,
                           hipStream_t s);
hipError_t launch_forward(const Basis& b, int N, const FwdPlan& p,
                          const float* pixtab, const float* field_t,
                          const float* spotrec, const float* offtab,
                          float* partial, hipStream_t s);
hipError_t launch_reduce(int N, const FwdPlan& p, const float* partial,
                         float* red, hipStream_t s);
hipError_t launch_finish_E(int N, const FwdPlan& p, const float* red,
                           float* E, hipStream_t s);
hipError_t launch_wgs_update(int N, const FwdPlan& p, const float* red,
                             const float* target, float t_norm, float* W,
                             float power, float eff_denom, float* y,
                             float* Ebuf, float* E_extra, float* stats_row,
                             hipStream_t s);
enum AdjOut { kOutG = 1, kOutPhase = 2, kOutField = 4 };
hipError_t launch_adjoint(const Basis& b, int N, const float* pixtab,
                          const float* spotrec, const float* offtab,
                          const float* ypol, const float* amp_t, int outs,
                          float* g, float* phase, float* field_t,
                          hipStream_t s);

}  // namespace ash

struct ash_prof_rec {
  int cat;
  hipEvent_t start, stop;
};

struct ash_ctx {
  int device = 0;
  int n_cu = 0;
  bool prof_on = false;
  std::vector<ash_prof_rec> prof;    // recorded pairs (in use)
  std::vector<hipEvent_t> prof_pool; // free events
  hipStream_t stream = nullptr;
  std::string err;
  bool has_basis = false, has_spots = false;
  ash::Basis basis;
  ash::Spots spots;
  ash::Buffers buf;
  ash::FwdPlan plan;
};
