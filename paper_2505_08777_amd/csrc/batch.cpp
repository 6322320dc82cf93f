// Host side of the batched form: many holograms' WGS loops run together,
// each phase of an iteration one persistent launch over the work items of
// all holograms (per record shape), with per-XCD work queues.  When every
// member has at most kFusedSpots spots, each iteration's adjoint and the
// next iteration's forward are one fused launch.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "ash.h"
#include "internal.h"

using namespace ash;

namespace {

constexpr int kDefaultRange = 64;  // pixel blocks per forward item (untuned)
constexpr int kTuneCandidates[] = {16, 32, 64, 128, 256, 512};
// Fused launches: pixel blocks per unit of a hologram of one 32-spot block
// (one of B blocks takes about 1/B of it), untuned and the candidates.
constexpr int kDefaultFusedRange = 16;
constexpr int kFusedCandidates[] = {4, 8, 16, 32, 64, 128};
// The tuner's two run lengths (iterations) per one-launch candidate and
// per form.  The long run is as long as a typical call: the one-launch
// form's cost per iteration grows with the run (its holograms fall out of
// step, and the slowest one's barriers set the end), so that a short run
// would favour it.
constexpr int kTuneItersShort = 2, kTuneItersLong = 22;
// Relative cost of a pixel block's adjoint epilogue (butterfly over the
// spots, arg g, next nearfield record) in 32 x 32 evaluation blocks.
constexpr double kEpilogueBlocks = 1.25;

// One record shape (matrix-core groups, range reduction) of the batch.
struct Cls {
  int G = 0;
  int reduce = 0;
  int L = kDefaultRange;
  std::vector<int> holos;
  size_t fwd_off = 0, adj_off = 0, fus_off = 0;  // first item of each phase
  int qoff_fwd = 0, qoff_fus = 0;  // index of its 9 queue offsets in qoff
  int fwd_grid = 0, adj_grid = 0, fus_grid = 0;
  int np_max = 32;  // largest padded spot count of its holograms
  // one-launch form
  int bpc = 0;                // resident blocks per CU (0: as many as fit)
  int p_grid = 0;             // blocks of its launch
  size_t p_lds = 0;           // dynamic LDS per block
  size_t p_holo = 0, p_blk = 0;  // first descriptor and block of its arrays
};

struct Snap {  // what the batch's plan depends on, per member
  int N, n_tiles, groups, reduce;
  const void *pixtab, *spotrec, *offtab, *y, *field_t;
};

}  // namespace

struct ash_batch {
  int device = 0;
  int n_cu = 0;
  hipStream_t stream = nullptr;
  std::string err;
  std::vector<ash_ctx*> m;
  std::vector<Snap> snap;
  std::vector<Cls> cls;
  std::vector<HoloDesc> desc;
  std::vector<int4> items, rblk;
  std::vector<int> qoff;
  double evals_per_transform = 0.0;
  // every member has at most kFusedSpots spots: an iteration's adjoint and
  // the next forward run as one fused launch
  bool fused = false;
  // device
  HoloDesc* d_desc = nullptr;
  float2* d_partial = nullptr;
  float2* d_red = nullptr;
  int4* d_items = nullptr;
  int4* d_rblk = nullptr;
  int* d_qoff = nullptr;
  int* d_ctr = nullptr;
  size_t cap_partial = 0, cap_red = 0, cap_items = 0, cap_rblk = 0,
         cap_qoff = 0, cap_ctr = 0;
  // one-launch form (possible when every member has at most kPersistSpots
  // spots and the device launches cooperative grids); one_launch selects it
  bool persist = false;
  bool one_launch = false;
  std::vector<PHolo> pholo;  // per member, in class order
  std::vector<PBlock> pblk;
  std::vector<int> pmember;  // member of each pholo entry
  PHolo* d_pholo = nullptr;
  PBlock* d_pblk = nullptr;
  float2* d_prows = nullptr;
  unsigned* d_pyblk = nullptr;
  int* d_pctr = nullptr;  // per member barrier counter, then the error flag
  bool pholo_on_device = false;  // d_pholo holds pholo as it stands
  int* h_flag = nullptr;         // pinned host copy of the error flag
  size_t cap_pholo = 0, cap_pblk = 0, cap_prows = 0, cap_pyblk = 0,
         cap_pctr = 0;
  // timing
  int prof_mask = 0;
  std::vector<ash_prof_rec> prof;
  std::vector<hipEvent_t> pool;
};

namespace {

int bfail(ash_batch* b, int code, const std::string& msg) {
  if (b) b->err = msg;
  return code;
}

int bhip(ash_batch* b, hipError_t e, const char* what) {
  if (b) b->err = std::string(what) + ": " + hipGetErrorString(e);
  return ASH_EHIP;
}

#define BCHK(b, expr, what)                           \
  do {                                                \
    hipError_t e_ = (expr);                           \
    if (e_ != hipSuccess) return bhip(b, e_, what);   \
  } while (0)

int buse(ash_batch* b) {
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return bhip(b, e, "hipGetDevice");
  if (cur != b->device && (e = hipSetDevice(b->device)) != hipSuccess)
    return bhip(b, e, "hipSetDevice");
  return ASH_OK;
}

template <typename T>
void bfree(T*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

template <typename T>
int bgrow(ash_batch* b, T** p, size_t* cap, size_t need, const char* what) {
  if (need == 0) need = 1;
  if (need <= *cap) return ASH_OK;
  bfree(*p);
  *cap = 0;
  if (injected_alloc_failure() ||
      hipMalloc(reinterpret_cast<void**>(p), need * sizeof(T)) != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return bfail(b, ASH_ENOMEM, std::string("out of device memory for ") + what);
  }
  *cap = need;
  return ASH_OK;
}

template <typename F>
hipError_t btimed(ash_batch* b, int cat, F&& launch) {
  if (!(b->prof_mask & (1 << cat))) return launch();
  hipEvent_t ev[2] = {nullptr, nullptr};
  for (auto& e : ev) {
    if (!b->pool.empty()) {
      e = b->pool.back();
      b->pool.pop_back();
    } else if (hipEventCreateWithFlags(&e, kProfEventFlags) != hipSuccess) {
      (void)hipGetLastError();
      e = nullptr;
    }
  }
  if (ev[0]) (void)hipEventRecord(ev[0], b->stream);
  hipError_t r = launch();
  if (ev[0] && ev[1]) {
    (void)hipEventRecord(ev[1], b->stream);
    b->prof.push_back({cat, ev[0], ev[1]});
  } else {
    for (auto e : ev)
      if (e) b->pool.push_back(e);
  }
  return r;
}

Snap snapshot(const ash_ctx* c) {
  const Buffers& B = c->buf;
  return {c->spots.N, c->basis.g.n_tiles, c->basis.g.groups, c->basis.g.reduce,
          B.pixtab, B.spotrec, B.offtab, B.y, B.field_t};
}

bool same(const Snap& a, const Snap& b) {
  return a.N == b.N && a.n_tiles == b.n_tiles && a.groups == b.groups &&
         a.reduce == b.reduce && a.pixtab == b.pixtab &&
         a.spotrec == b.spotrec && a.offtab == b.offtab && a.y == b.y &&
         a.field_t == b.field_t;
}

// Assign units of work to the 8 XCD queues, largest first to the least
// loaded queue (longest-processing-time order), keeping each unit's items
// together; returns, per queue, the units in assignment order.
std::vector<std::vector<int>> lpt(const std::vector<double>& work) {
  std::vector<int> order(work.size());
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int c) { return work[a] > work[c]; });
  std::vector<std::vector<int>> q(kXcds);
  double load[kXcds] = {0};
  for (int u : order) {
    int best = 0;
    for (int x = 1; x < kXcds; ++x)
      if (load[x] < load[best]) best = x;
    q[best].push_back(u);
    load[best] += work[u];
  }
  return q;
}

// The one-launch plan: per record shape, the resident blocks of its launch
// shared out over its holograms in proportion to their work per iteration
// (forward and adjoint blocks of evaluations and the adjoint's per-row
// epilogue), each block a contiguous range of its hologram's 32-pixel
// blocks; the blocks' partial-sum rows, spot-field records and barrier
// counters.
int plan_persist(ash_batch* b) {
  b->pholo.clear();
  b->pholo_on_device = false;
  b->pblk.clear();
  b->pmember.clear();
  size_t rows = 0, yblk = 0;
  for (auto& c : b->cls) {
    int maxN = 1;
    for (int h : c.holos) maxN = std::max(maxN, b->m[h]->spots.N);
    c.np_max = std::max(32, (maxN + 31) / 32 * 32);
    c.p_lds = persist_lds_bytes(c.np_max);
    int occ = persist_blocks_per_cu(c.G, c.reduce != 0, c.p_lds);
    if (occ <= 0) return bfail(b, ASH_EUNSUPPORTED, "no resident block fits");
    if (c.bpc > 0) occ = std::min(occ, c.bpc);
    c.p_grid = occ * b->n_cu;
    std::vector<double> work;
    double total = 0.0;
    for (int h : c.holos) {
      const ash_ctx* m = b->m[h];
      const double n_blk = (double)m->basis.g.n_tiles * kBlkPerTile;
      const double n_mb = (m->spots.N + 31) / 32;
      work.push_back(n_blk * (2.0 * n_mb + kEpilogueBlocks));
      total += work.back();
    }
    const int Hc = (int)c.holos.size();
    if (Hc > c.p_grid)
      return bfail(b, ASH_EUNSUPPORTED, "more holograms than resident blocks");
    // blocks per hologram: at least one, at most one per pair of pixel
    // blocks (the fused rows take them in pairs), the rest by largest
    // remainder of the proportional share
    std::vector<long> nb(Hc, 1);
    std::vector<std::pair<double, int>> rem;
    long given = Hc;
    for (int i = 0; i < Hc; ++i) {
      const long cap = (long)b->m[c.holos[i]]->basis.g.n_tiles * kBlkPerTile / 2;
      const double share = (double)(c.p_grid - Hc) * work[i] / total;
      const long extra = std::min(cap - 1, (long)floor(share));
      nb[i] += extra;
      given += extra;
      rem.push_back({share - floor(share), i});
    }
    std::sort(rem.begin(), rem.end(), [](const std::pair<double, int>& x,
                                         const std::pair<double, int>& y) {
      return x.first > y.first || (x.first == y.first && x.second < y.second);
    });
    for (size_t r = 0; r < rem.size() && given < c.p_grid; ++r) {
      const int i = rem[r].second;
      const long cap = (long)b->m[c.holos[i]]->basis.g.n_tiles * kBlkPerTile / 2;
      if (nb[i] < cap) {
        ++nb[i];
        ++given;
      }
    }
    c.p_grid = (int)given;
    c.p_holo = b->pholo.size();
    c.p_blk = b->pblk.size();
    for (int i = 0; i < Hc; ++i) {
      const int h = c.holos[i];
      ash_ctx* m = b->m[h];
      const Geom& g = m->basis.g;
      Buffers& B = m->buf;
      PHolo d;
      d.pixtab = reinterpret_cast<const u32x4*>(B.pixtab);
      d.spotrec = reinterpret_cast<const u32x4*>(B.spotrec);
      d.offtab = B.offtab;
      d.amp_t = B.amp_t;
      d.target = B.target;
      d.W = nullptr;
      d.phase = nullptr;
      d.n_blk = (long)g.n_tiles * kBlkPerTile;
      d.N = m->spots.N;
      d.nx = g.nx;
      d.ny = g.ny;
      d.tiles_x = g.tiles_x;
      d.groups = g.groups;
      d.n_blocks = (int)nb[i];
      d.t_norm = (float)sqrt(m->spots.t_norm2);
      const int NP = (d.N + 31) / 32 * 32;
      d.rows = reinterpret_cast<float2*>(rows);  // offsets for now
      d.yblk = reinterpret_cast<unsigned*>(yblk);
      d.ctr = reinterpret_cast<int*>((size_t)b->pholo.size() * kCtrPad);
      rows += (size_t)2 * nb[i] * d.N;
      yblk += (size_t)nb[i] * NP * 9;
      const long pairs = d.n_blk / 2;  // n_blk is a whole number of tiles
      for (long j = 0; j < nb[i]; ++j) {
        PBlock pb;
        pb.holo = i;
        pb.j = (int)j;
        pb.b0 = 2 * (pairs * j / nb[i]);
        pb.b1 = 2 * (pairs * (j + 1) / nb[i]);
        b->pblk.push_back(pb);
      }
      b->pholo.push_back(d);
      b->pmember.push_back(h);
    }
  }
  int rc;
  const size_t n_ctr = (b->pholo.size() + 1) * kCtrPad;
  if ((rc = bgrow(b, &b->d_pholo, &b->cap_pholo, b->pholo.size(),
                  "descriptors")) ||
      (rc = bgrow(b, &b->d_pblk, &b->cap_pblk, b->pblk.size(), "blocks")) ||
      (rc = bgrow(b, &b->d_prows, &b->cap_prows, rows, "partial sums")) ||
      (rc = bgrow(b, &b->d_pyblk, &b->cap_pyblk, yblk, "spot fields")) ||
      (rc = bgrow(b, &b->d_pctr, &b->cap_pctr, n_ctr, "barrier counters")))
    return rc;
  for (auto& d : b->pholo) {
    d.rows = b->d_prows + reinterpret_cast<size_t>(d.rows);
    d.yblk = b->d_pyblk + reinterpret_cast<size_t>(d.yblk);
    d.ctr = b->d_pctr + reinterpret_cast<size_t>(d.ctr);
  }
  BCHK(b, hipMemcpy(b->d_pblk, b->pblk.data(), b->pblk.size() * sizeof(PBlock),
                    hipMemcpyHostToDevice),
       "uploading the batch plan");
  return ASH_OK;
}

// Build descriptors (without the per-call phase and weight pointers),
// work items, queues and reduction blocks for the current range lengths.
int plan(ash_batch* b) {
  // launches of an earlier plan may still read the buffers rewritten here
  BCHK(b, hipStreamSynchronize(b->stream), "hipStreamSynchronize");
  const int H = (int)b->m.size();
  b->desc.assign(H, HoloDesc());
  size_t part = 0, red = 0;
  b->evals_per_transform = 0.0;
  // range lengths: the class's; fused, the class's divided by the
  // hologram's spot blocks, so that units hold about equal work, and even
  // (the fused kernel takes pixel blocks in pairs)
  std::vector<int> L_of(H, kDefaultRange);
  for (auto& c : b->cls) {
    if (b->fused) c.L += c.L & 1;
    for (int h : c.holos) {
      const int nb = (b->m[h]->spots.N + 31) / 32;
      L_of[h] = b->fused ? std::max(2, (c.L / nb + 1) & ~1) : c.L;
    }
  }
  for (int h = 0; h < H; ++h) {
    ash_ctx* c = b->m[h];
    const Geom& g = c->basis.g;
    Buffers& B = c->buf;
    HoloDesc& d = b->desc[h];
    d.pixtab = reinterpret_cast<const u32x4*>(B.pixtab);
    d.nf_t = B.field_t;
    d.spotrec = reinterpret_cast<const u32x4*>(B.spotrec);
    d.offtab = B.offtab;
    d.ypol = B.y;
    d.amp_t = B.amp_t;
    d.target = B.target;
    d.Ebuf = reinterpret_cast<float2*>(B.Ebuf);
    d.n_blk = (long)g.n_tiles * kBlkPerTile;
    d.N = c->spots.N;
    d.nx = g.nx;
    d.ny = g.ny;
    d.tiles_x = g.tiles_x;
    d.L = L_of[h];
    d.n_ranges = (int)((d.n_blk + d.L - 1) / d.L);
    d.slices = (d.n_ranges + kRowsPerSlice - 1) / kRowsPerSlice;
    d.t_norm = (float)sqrt(c->spots.t_norm2);
    d.eff_denom = (float)((double)g.nx * g.ny * c->basis.amp_sum2);
    d.partial = reinterpret_cast<float2*>(part);  // offsets for now
    d.red = reinterpret_cast<float2*>(red);
    part += (size_t)d.n_ranges * d.N;
    red += (size_t)d.slices * d.N;
    b->evals_per_transform += (double)d.N * g.nx * g.ny;
  }
  int rc;
  if ((rc = bgrow(b, &b->d_partial, &b->cap_partial, part, "partial sums")) ||
      (rc = bgrow(b, &b->d_red, &b->cap_red, red, "partial sums")))
    return rc;
  for (auto& d : b->desc) {
    d.partial = b->d_partial + reinterpret_cast<size_t>(d.partial);
    d.red = b->d_red + reinterpret_cast<size_t>(d.red);
  }
  // work items and queues, per record shape
  b->items.clear();
  b->qoff.clear();
  for (auto& c : b->cls) {
    // forward: unit = (holo, range), items = its spot blocks
    std::vector<int2> units;
    std::vector<double> work;
    for (int h : c.holos) {
      const HoloDesc& d = b->desc[h];
      const int n_mb = (d.N + 31) / 32;
      for (int r = 0; r < d.n_ranges; ++r) {
        const long len = std::min<long>(d.L, d.n_blk - (long)r * d.L);
        units.push_back(make_int2(h, r));
        work.push_back((double)len * n_mb);
      }
    }
    std::vector<std::vector<int>> q = lpt(work);
    c.np_max = 32;
    for (int h : c.holos)
      c.np_max = std::max(c.np_max, (b->desc[h].N + 31) / 32 * 32);
    if (b->fused) {
      // every launch fused: one item per unit (holo, range)
      c.fus_off = b->items.size();
      c.qoff_fus = (int)b->qoff.size();
      for (int x = 0; x < kXcds; ++x) {
        b->qoff.push_back((int)(b->items.size() - c.fus_off));
        for (int u : q[x])
          b->items.push_back(make_int4(units[u].x, units[u].y, 0, 0));
      }
      b->qoff.push_back((int)(b->items.size() - c.fus_off));
      c.fus_grid = std::max(
          kXcds, fused_blocks_per_cu(c.G, c.reduce != 0, c.np_max) * b->n_cu /
                     kXcds * kXcds);
      continue;
    }
    c.fwd_off = b->items.size();
    c.qoff_fwd = (int)b->qoff.size();
    for (int x = 0; x < kXcds; ++x) {
      b->qoff.push_back((int)(b->items.size() - c.fwd_off));
      for (int u : q[x]) {
        const int h = units[u].x, r = units[u].y;
        const int n_mb = (b->desc[h].N + 31) / 32;
        for (int mb = 0; mb < n_mb; ++mb)
          b->items.push_back(make_int4(h, r, mb, 0));
      }
    }
    b->qoff.push_back((int)(b->items.size() - c.fwd_off));
    // adjoint: unit = (holo, tile), one block per quarter tile (four rows,
    // one per wave).  Blocks reach the XCDs round-robin, so block j * 8 + x
    // takes the j-th block of XCD x's list (longest first); shorter lists
    // are padded with idle blocks.
    units.clear();
    work.clear();
    for (int h : c.holos) {
      const HoloDesc& d = b->desc[h];
      const int n_tiles = (int)(d.n_blk / kBlkPerTile);
      for (int t = 0; t < n_tiles; ++t) {
        units.push_back(make_int2(h, t));
        work.push_back((double)kBlkPerTile * ((d.N + 31) / 32));
      }
    }
    q = lpt(work);
    constexpr int kQuarters = kBlkPerTile / (kBlock / kWave);
    size_t longest = 0;
    for (int x = 0; x < kXcds; ++x)
      longest = std::max(longest, q[x].size() * kQuarters);
    c.adj_off = b->items.size();
    b->items.resize(c.adj_off + longest * kXcds, make_int4(-1, 0, 0, 0));
    for (int x = 0; x < kXcds; ++x) {
      size_t j = 0;
      for (int u : q[x])
        for (int qt = 0; qt < kQuarters; ++qt, ++j)
          b->items[c.adj_off + j * kXcds + x] =
              make_int4(units[u].x, units[u].y * kQuarters + qt, 0, 0);
    }
    c.fwd_grid = std::max(
        kXcds, batch_blocks_per_cu(c.G, c.reduce != 0, true) * b->n_cu /
                   kXcds * kXcds);
    c.adj_grid = (int)(longest * kXcds);
  }
  if (b->items.size() > (size_t)INT32_MAX)
    return bfail(b, ASH_EUNSUPPORTED, "too many work items");
  // reduction blocks: {holo, first spot, slice}
  b->rblk.clear();
  for (int h = 0; h < H; ++h) {
    const HoloDesc& d = b->desc[h];
    for (int sl = 0; sl < d.slices; ++sl)
      for (int k0 = 0; k0 < d.N; k0 += 64)
        b->rblk.push_back(make_int4(h, k0, sl, 0));
  }
  if ((rc = bgrow(b, &b->d_items, &b->cap_items, b->items.size(), "items")) ||
      (rc = bgrow(b, &b->d_rblk, &b->cap_rblk, b->rblk.size(), "items")) ||
      (rc = bgrow(b, &b->d_qoff, &b->cap_qoff, b->qoff.size(), "queues")))
    return rc;
  hipError_t e = hipMemcpy(b->d_items, b->items.data(),
                           b->items.size() * sizeof(int4),
                           hipMemcpyHostToDevice);
  if (e == hipSuccess && !b->rblk.empty())
    e = hipMemcpy(b->d_rblk, b->rblk.data(), b->rblk.size() * sizeof(int4),
                  hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(b->d_qoff, b->qoff.data(), b->qoff.size() * sizeof(int),
                  hipMemcpyHostToDevice);
  if (e != hipSuccess) return bhip(b, e, "uploading the batch plan");
  return b->persist ? plan_persist(b) : ASH_OK;
}

// Upload the descriptors with this call's phase and weight pointers.
int upload_desc(ash_batch* b, float* const* phase, float* const* W) {
  for (size_t h = 0; h < b->desc.size(); ++h) {
    b->desc[h].phase = phase ? phase[h] : nullptr;
    b->desc[h].W = W ? W[h] : nullptr;
  }
  // synchronous: the host copy is rewritten by the next call
  BCHK(b, hipStreamSynchronize(b->stream), "hipStreamSynchronize");
  BCHK(b, hipMemcpy(b->d_desc, b->desc.data(),
                    b->desc.size() * sizeof(HoloDesc), hipMemcpyHostToDevice),
       "uploading descriptors");
  return ASH_OK;
}

int check_members(ash_batch* b) {
  for (size_t h = 0; h < b->m.size(); ++h)
    if (!b->m[h]->has_basis || !b->m[h]->has_spots ||
        !same(b->snap[h], snapshot(b->m[h])))
      return bfail(b, ASH_ENOTREADY,
                   "member " + std::to_string(h) +
                       " changed since the batch was made; make it again");
  return ASH_OK;
}

// Enqueue one forward phase (all record shapes) with counters
// ctr[cls][8][kCtrPad], timed under category `cat`.
int enqueue_forward(ash_batch* b, int* ctr, int cat = ASH_PROF_FORWARD) {
  for (size_t k = 0; k < b->cls.size(); ++k) {
    const Cls& c = b->cls[k];
    BCHK(b, btimed(b, cat, [&] {
           return launch_batch_forward(c.G, c.reduce != 0, c.fwd_grid,
                                       b->d_desc, b->d_items + c.fwd_off,
                                       b->d_qoff + c.qoff_fwd,
                                       ctr + (size_t)k * kXcds * kCtrPad,
                                       b->stream);
         }), "batch forward");
  }
  return ASH_OK;
}

int enqueue_reduce_update(ash_batch* b, float power, bool update) {
  BCHK(b, btimed(b, ASH_PROF_REDUCE, [&] {
         return launch_batch_reduce(b->d_desc, b->d_rblk, (int)b->rblk.size(),
                                    b->stream);
       }), "batch reduce");
  if (update)
    BCHK(b, btimed(b, ASH_PROF_REDUCE, [&] {
           return launch_batch_update((int)b->m.size(), b->d_desc, power,
                                      b->stream);
         }), "batch update");
  return ASH_OK;
}

int enqueue_adjoint(ash_batch* b, int last, int cat = ASH_PROF_ADJOINT) {
  for (size_t k = 0; k < b->cls.size(); ++k) {
    const Cls& c = b->cls[k];
    BCHK(b, btimed(b, cat, [&] {
           return launch_batch_adjoint(c.G, c.reduce != 0, c.adj_grid,
                                       b->d_desc, b->d_items + c.adj_off,
                                       last, b->stream);
         }), "batch adjoint");
  }
  return ASH_OK;
}

int make_fields(ash_batch* b, float* const* phase) {
  for (size_t h = 0; h < b->m.size(); ++h) {
    ash_ctx* c = b->m[h];
    BCHK(b, btimed(b, ASH_PROF_FIELD, [&] {
           return launch_make_field(c->basis.g, phase[h], nullptr,
                                    c->buf.amp_t, c->buf.pixtab,
                                    c->buf.field_t, nullptr, b->stream);
         }), "make_field");
  }
  return ASH_OK;
}

// Enqueue one fused launch per record shape (mode: the first forward, an
// adjoint and the next forward, the last adjoint) with counters
// ctr[cls][8][kCtrPad].
int enqueue_fused(ash_batch* b, int mode, int* ctr) {
  for (size_t k = 0; k < b->cls.size(); ++k) {
    const Cls& c = b->cls[k];
    BCHK(b, btimed(b, ASH_PROF_ADJOINT, [&] {
           return launch_batch_fused(c.G, c.reduce != 0, c.fus_grid, c.np_max,
                                     mode, b->d_desc, b->d_items + c.fus_off,
                                     b->d_qoff + c.qoff_fus,
                                     ctr + (size_t)k * kXcds * kCtrPad,
                                     b->stream);
         }), "batch fused adjoint and forward");
  }
  return ASH_OK;
}

// The launches of n_iter >= 1 iterations from the phases in the
// descriptors, with take counters for n_iter + 1 queue launches.  Fused:
// the first forward, then per iteration the update and a fused launch (the
// adjoint and the next forward; after the last iteration the adjoint
// alone), all timed under ASH_PROF_ADJOINT.  Otherwise the nearfield
// records, then per iteration forward, update and adjoint.
int enqueue_iterations(ash_batch* b, float* const* phase, int n_iter,
                       float power, int* ctr) {
  const size_t per = b->cls.size() * kXcds * kCtrPad;
  int rc = ASH_OK;
  if (!b->fused) {
    if ((rc = make_fields(b, phase))) return rc;
    for (int it = 0; it < n_iter && !rc; ++it)
      if (!(rc = enqueue_forward(b, ctr + it * per)) &&
          !(rc = enqueue_reduce_update(b, power, true)))
        rc = enqueue_adjoint(b, it == n_iter - 1);
    return rc;
  }
  if ((rc = enqueue_fused(b, kFusedFirst, ctr))) return rc;
  for (int it = 0; it < n_iter && !rc; ++it) {
    if ((rc = enqueue_reduce_update(b, power, true))) break;
    rc = enqueue_fused(b, it + 1 < n_iter ? kFusedMid : kFusedLast,
                       ctr + (it + 1) * per);
  }
  return rc;
}


// Zeroed take counters for `launches` persistent launches of 8 queues per
// record shape, kCtrPad ints apart.
int counters(ash_batch* b, size_t launches, int** out) {
  const size_t n = launches * b->cls.size() * kXcds * kCtrPad;
  int rc = bgrow(b, &b->d_ctr, &b->cap_ctr, n, "queue counters");
  if (rc) return rc;
  BCHK(b, hipMemsetAsync(b->d_ctr, 0, n * sizeof(int), b->stream),
       "clearing queue counters");
  *out = b->d_ctr;
  return ASH_OK;
}

// Upload the one-launch descriptors with this call's phase and weight
// pointers, and zero the barrier counters and the error flag.
int upload_persist(ash_batch* b, float* const* phase, float* const* W) {
  bool same = b->pholo_on_device;
  for (size_t i = 0; i < b->pholo.size(); ++i) {
    const int h = b->pmember[i];
    same = same && b->pholo[i].phase == phase[h] && b->pholo[i].W == W[h];
    b->pholo[i].phase = phase[h];
    b->pholo[i].W = W[h];
  }
  if (same) return ASH_OK;  // the last call's arrays: nothing to send
  BCHK(b, hipStreamSynchronize(b->stream), "hipStreamSynchronize");
  BCHK(b, hipMemcpy(b->d_pholo, b->pholo.data(),
                    b->pholo.size() * sizeof(PHolo), hipMemcpyHostToDevice),
       "uploading descriptors");
  b->pholo_on_device = true;
  return ASH_OK;
}

// One launch per record shape runs all n_iter iterations of its holograms;
// then the stream is synchronised and the barriers' error flag read.
int run_persist(ash_batch* b, int n_iter, float power) {
  if (!b->h_flag &&
      (injected_alloc_failure() ||
       hipHostMalloc(reinterpret_cast<void**>(&b->h_flag), sizeof(int),
                     hipHostMallocDefault) != hipSuccess)) {
    (void)hipGetLastError();
    b->h_flag = nullptr;
    return bfail(b, ASH_ENOMEM, "out of pinned host memory for the flag");
  }
  const size_t n_ctr = (b->pholo.size() + 1) * kCtrPad;
  int* err = b->d_pctr + b->pholo.size() * kCtrPad;
  BCHK(b, hipMemsetAsync(b->d_pctr, 0, n_ctr * sizeof(int), b->stream),
       "clearing barrier counters");
  if (injected_barrier_failure())  // the flag set: every barrier gives up
    BCHK(b, hipMemsetAsync(err, 0x01, sizeof(int), b->stream),
         "setting the barrier flag");
  for (const Cls& c : b->cls) {
    BCHK(b, btimed(b, ASH_PROF_FORWARD, [&] {
           return launch_batch_persist(c.G, c.reduce != 0, c.p_grid, c.p_lds,
                                       b->d_pholo + c.p_holo,
                                       b->d_pblk + c.p_blk, n_iter, power,
                                       c.np_max, err, b->stream);
         }), "batch launch");
  }
  BCHK(b, hipMemcpyAsync(b->h_flag, err, sizeof(int), hipMemcpyDeviceToHost,
                         b->stream), "reading the barrier flag");
  BCHK(b, hipStreamSynchronize(b->stream), "hipStreamSynchronize");
  if (*b->h_flag)
    return bfail(b, ASH_EHIP, "a barrier of the one-launch batch gave up "
                              "(its time limit, or an injected failure); "
                              "results are incomplete");
  return ASH_OK;
}

// Tuner of the one-launch form: per record shape, every count of resident
// blocks per CU is timed on copies of the caller's phases (unit weights),
// and the cheapest kept; then the launches per phase are timed the same
// way and the cheaper form is kept.  A cost is the time of one more
// iteration: the difference of runs of kTuneItersShort and kTuneItersLong
// iterations over their difference, so that the first forward and the
// last adjoint, which both forms add once per call, weigh nothing.
int tune_persist(ash_batch* b, float* const* phase_dev,
                 std::vector<float>* best_ms) {
  const size_t H = b->m.size();
  std::vector<float*> ph(H, nullptr), W(H, nullptr);
  int rc = ASH_OK;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto cleanup = [&]() {
    for (size_t h = 0; h < H; ++h) {
      bfree(ph[h]);
      bfree(W[h]);
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  };
  for (size_t h = 0; h < H && !rc; ++h) {
    const size_t P = (size_t)b->m[h]->basis.g.nx * b->m[h]->basis.g.ny;
    if (injected_alloc_failure() ||
        hipMalloc(reinterpret_cast<void**>(&ph[h]), P * sizeof(float)) !=
            hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&W[h]),
                  b->m[h]->spots.N * sizeof(float)) != hipSuccess) {
      (void)hipGetLastError();
      rc = bfail(b, ASH_ENOMEM, "out of device memory for tuning copies");
    }
  }
  if (!rc && (hipEventCreate(&e0) != hipSuccess ||
              hipEventCreate(&e1) != hipSuccess))
    rc = bfail(b, ASH_EHIP, "hipEventCreate");
  const std::vector<float> ones(kPersistSpots, 1.0f);
  // fresh copies of the caller's phases and unit weights
  auto copy_inputs = [&]() {
    for (size_t h = 0; h < H; ++h) {
      const size_t P = (size_t)b->m[h]->basis.g.nx * b->m[h]->basis.g.ny;
      if (hipMemcpyAsync(ph[h], phase_dev[h], P * sizeof(float),
                         hipMemcpyDeviceToDevice, b->stream) != hipSuccess ||
          hipMemcpyAsync(W[h], ones.data(), b->m[h]->spots.N * sizeof(float),
                         hipMemcpyHostToDevice, b->stream) != hipSuccess)
        return bfail(b, ASH_EHIP, "copying tuning inputs");
    }
    return (int)ASH_OK;
  };
  auto elapsed = [&](float* ms) {
    if (hipEventRecord(e1, b->stream) != hipSuccess ||
        hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(ms, e0, e1) != hipSuccess) {
      (void)hipGetLastError();
      return bfail(b, ASH_EHIP, "timing a tuning run");
    }
    return (int)ASH_OK;
  };
  // one launch of record shape c for n iterations (planned and uploaded)
  auto time_one = [&](const Cls& c, int n, float* ms) {
    int r = copy_inputs();
    if (r) return r;
    int* err = b->d_pctr + b->pholo.size() * kCtrPad;
    if (hipMemsetAsync(b->d_pctr, 0,
                       (b->pholo.size() + 1) * kCtrPad * sizeof(int),
                       b->stream) != hipSuccess ||
        hipEventRecord(e0, b->stream) != hipSuccess ||
        launch_batch_persist(c.G, c.reduce != 0, c.p_grid, c.p_lds,
                             b->d_pholo + c.p_holo, b->d_pblk + c.p_blk, n,
                             1.0f, c.np_max, err, b->stream) != hipSuccess) {
      (void)hipGetLastError();
      return bfail(b, ASH_EHIP, "launching a one-launch candidate");
    }
    if ((r = elapsed(ms))) return r;
    int flag = 0;
    if (hipMemcpy(&flag, err, sizeof(int), hipMemcpyDeviceToHost) !=
            hipSuccess || flag)
      return bfail(b, ASH_EHIP, "a tuning launch's barrier timed out");
    return (int)ASH_OK;
  };
  // the launches per phase of every record shape for n iterations
  auto time_phase = [&](int n, float* ms) {
    int r = copy_inputs();
    int* ctr = nullptr;
    if (!r) r = upload_desc(b, ph.data(), W.data());
    if (!r) r = counters(b, n + 1, &ctr);
    if (!r && hipEventRecord(e0, b->stream) != hipSuccess)
      r = bfail(b, ASH_EHIP, "hipEventRecord");
    if (!r) r = enqueue_iterations(b, ph.data(), n, 1.0f, ctr);
    if (!r) r = elapsed(ms);
    return r;
  };
  constexpr int kShort = kTuneItersShort, kLong = kTuneItersLong;
  best_ms->assign(b->cls.size(), 0.0f);
  for (size_t k = 0; k < b->cls.size() && !rc; ++k) {
    Cls& c = b->cls[k];
    const int max_bpc = persist_blocks_per_cu(
        c.G, c.reduce != 0, c.p_lds ? c.p_lds : persist_lds_bytes(kPersistSpots));
    int best_bpc = c.bpc;
    float best_t = -1.0f;
    for (int bpc = 1; bpc <= max_bpc && !rc; ++bpc) {
      c.bpc = bpc;
      // an untimed launch first: the first launch of a kernel also loads
      // its code, which would inflate the short run
      float t0 = 0.0f, t1 = 0.0f;
      if ((rc = plan_persist(b)) ||
          (rc = upload_persist(b, ph.data(), W.data())) ||
          (rc = time_one(c, 1, &t0)) || (rc = time_one(c, kShort, &t0)) ||
          (rc = time_one(c, kLong, &t1)))
        break;
      const float t = (t1 - t0) / (kLong - kShort);
      if (best_t < 0.0f || t < best_t) {
        best_t = t;
        best_bpc = bpc;
      }
    }
    c.bpc = best_bpc;
    (*best_ms)[k] = best_t;
  }
  // the same iterations in launches per phase, with the range lengths
  // tuned before: the cheaper form is kept
  float p0 = 0.0f, p1 = 0.0f;
  if (!rc) rc = time_phase(1, &p0);  // untimed, as above
  if (!rc) rc = time_phase(kShort, &p0);
  if (!rc) rc = time_phase(kLong, &p1);
  if (!rc) {
    float ms_one = 0.0f;
    for (float x : *best_ms) ms_one += x;
    const float ms_phase = (p1 - p0) / (kLong - kShort);
    b->one_launch = ms_one <= ms_phase;
    best_ms->push_back(ms_phase);
  }
  cleanup();
  return rc;
}

}  // namespace

extern "C" {

int ash_batch_create(ash_batch** out, int H, ash_ctx* const* members,
                     void* stream) {
  if (!out) return ASH_EINVAL;
  *out = nullptr;
  if (H < 1 || !members) return ASH_EINVAL;
  for (int h = 0; h < H; ++h)
    if (!members[h] || !members[h]->has_basis || !members[h]->has_spots ||
        members[h]->device != members[0]->device)
      return ASH_EINVAL;
  ash_batch* b = new (std::nothrow) ash_batch();
  if (!b) return ASH_ENOMEM;
  b->device = members[0]->device;
  b->n_cu = members[0]->n_cu;
  b->stream = reinterpret_cast<hipStream_t>(stream);
  b->m.assign(members, members + H);
  for (int h = 0; h < H; ++h) {
    b->snap.push_back(snapshot(members[h]));
    const Geom& g = members[h]->basis.g;
    auto it = std::find_if(b->cls.begin(), b->cls.end(), [&](const Cls& c) {
      return c.G == g.groups && c.reduce == g.reduce;
    });
    if (it == b->cls.end()) {
      Cls c;
      c.G = g.groups;
      c.reduce = g.reduce;
      b->cls.push_back(c);
      it = b->cls.end() - 1;
    }
    it->holos.push_back(h);
  }
  int rc = buse(b);
  // every member small enough for the one-launch form, and a device that
  // launches cooperative grids
  int coop = 0;
  if (!rc && hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch,
                                   b->device) != hipSuccess) {
    (void)hipGetLastError();
    coop = 0;
  }
  b->persist = coop != 0;
  for (int h = 0; h < H; ++h)
    if (members[h]->spots.N > kPersistSpots) b->persist = false;
  b->one_launch = b->persist;
  b->fused = true;
  for (int h = 0; h < H; ++h)
    if (members[h]->spots.N > kFusedSpots) b->fused = false;
  for (auto& c : b->cls) c.L = b->fused ? kDefaultFusedRange : kDefaultRange;
  if (!rc) {
    if (injected_alloc_failure() ||
        hipMalloc(reinterpret_cast<void**>(&b->d_desc),
                  H * sizeof(HoloDesc)) != hipSuccess) {
      (void)hipGetLastError();
      b->d_desc = nullptr;
      rc = ASH_ENOMEM;
    }
  }
  if (!rc) rc = plan(b);
  if (rc) {
    ash_batch_destroy(b);
    return rc;
  }
  *out = b;
  return ASH_OK;
}

int ash_batch_destroy(ash_batch* b) {
  if (!b) return ASH_EINVAL;
  (void)buse(b);
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  bfree(b->d_desc);
  bfree(b->d_partial);
  bfree(b->d_red);
  bfree(b->d_items);
  bfree(b->d_rblk);
  bfree(b->d_qoff);
  bfree(b->d_ctr);
  bfree(b->d_pholo);
  bfree(b->d_pblk);
  bfree(b->d_prows);
  bfree(b->d_pyblk);
  bfree(b->d_pctr);
  if (b->h_flag) (void)hipHostFree(b->h_flag);
  for (auto& r : b->prof) {
    (void)hipEventDestroy(r.start);
    (void)hipEventDestroy(r.stop);
  }
  for (auto e : b->pool) (void)hipEventDestroy(e);
  delete b;
  return ASH_OK;
}

const char* ash_batch_last_error(const ash_batch* b) {
  return b ? b->err.c_str() : "";
}

int ash_batch_set_stream(ash_batch* b, void* stream) {
  if (!b) return ASH_EINVAL;
  b->stream = reinterpret_cast<hipStream_t>(stream);
  return ASH_OK;
}

int ash_batch_wgs(ash_batch* b, float* const* phase_dev,
                  float* const* weights_dev, int n_iter,
                  const ash_wgs_params* params) {
  if (!b) return ASH_EINVAL;
  b->err.clear();
  if (!phase_dev || !weights_dev || n_iter < 0)
    return bfail(b, ASH_EINVAL, "phases, weights and n_iter >= 0 required");
  for (size_t h = 0; h < b->m.size(); ++h)
    if (!phase_dev[h] || !weights_dev[h])
      return bfail(b, ASH_EINVAL, "null phase or weights");
  const float power = params ? params->power : 1.0f;
  if (!isfinite(power)) return bfail(b, ASH_EINVAL, "power must be finite");
  if (params && params->fix_phase_after != 0)
    return bfail(b, ASH_EUNSUPPORTED, "phase fixing runs per hologram");
  if (n_iter == 0) return ASH_OK;
  int rc;
  if (b->one_launch) {
    if ((rc = buse(b)) || (rc = check_members(b)) ||
        (rc = upload_persist(b, phase_dev, weights_dev)))
      return rc;
    return run_persist(b, n_iter, power);
  }
  if ((rc = buse(b)) || (rc = check_members(b)) ||
      (rc = upload_desc(b, phase_dev, weights_dev)))
    return rc;
  int* ctr = nullptr;
  if ((rc = counters(b, (size_t)n_iter + 1, &ctr))) return rc;
  return enqueue_iterations(b, phase_dev, n_iter, power, ctr);
}

int ash_batch_tune(ash_batch* b, float* const* phase_dev,
                   const char* table_out) {
  if (!b) return ASH_EINVAL;
  b->err.clear();
  if (!phase_dev) return bfail(b, ASH_EINVAL, "phases required");
  int rc;
  if ((rc = buse(b)) || (rc = check_members(b))) return rc;
  if ((rc = upload_desc(b, phase_dev, nullptr))) return rc;
  if (!b->fused && (rc = make_fields(b, phase_dev))) return rc;
  const int* const cand = b->fused ? kFusedCandidates : kTuneCandidates;
  const int n_cand = b->fused
                         ? (int)(sizeof(kFusedCandidates) / sizeof(int))
                         : (int)(sizeof(kTuneCandidates) / sizeof(int));
  constexpr int kWarm = 1, kTimed = 3;
  std::vector<float> best_ms(b->cls.size(), 0.0f);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  BCHK(b, hipEventCreate(&e0), "hipEventCreate");
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return bfail(b, ASH_EHIP, "hipEventCreate");
  }
  const int saved_mask = b->prof_mask;
  b->prof_mask = 0;
  for (size_t k = 0; k < b->cls.size() && !rc; ++k) {
    int best = b->cls[k].L;
    float best_t = -1.0f;
    for (int ci = 0; ci < n_cand && !rc; ++ci) {
      b->cls[k].L = cand[ci];
      if ((rc = plan(b)) || (rc = upload_desc(b, phase_dev, nullptr))) break;
      int* ctr = nullptr;
      if ((rc = counters(b, kWarm + kTimed, &ctr))) break;
      float ms = 0.0f;
      for (int r = 0; r < kWarm + kTimed && !rc; ++r) {
        if (r == kWarm && hipEventRecord(e0, b->stream) != hipSuccess)
          rc = bfail(b, ASH_EHIP, "hipEventRecord");
        // the launch that dominates an iteration: the fused adjoint and
        // forward (on the spot fields the members hold), else the forward
        const Cls& c = b->cls[k];
        int* const cr = ctr + ((size_t)r * b->cls.size() + k) * kXcds * kCtrPad;
        hipError_t e =
            b->fused
                ? launch_batch_fused(c.G, c.reduce != 0, c.fus_grid, c.np_max,
                                     kFusedMid, b->d_desc,
                                     b->d_items + c.fus_off,
                                     b->d_qoff + c.qoff_fus, cr, b->stream)
                : launch_batch_forward(c.G, c.reduce != 0, c.fwd_grid,
                                       b->d_desc, b->d_items + c.fwd_off,
                                       b->d_qoff + c.qoff_fwd, cr, b->stream);
        if (e != hipSuccess) rc = bhip(b, e, "tuning forward");
        if (!rc && (rc = enqueue_reduce_update(b, 1.0f, false))) break;
      }
      if (!rc && (hipEventRecord(e1, b->stream) != hipSuccess ||
                  hipEventSynchronize(e1) != hipSuccess ||
                  hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        rc = bfail(b, ASH_EHIP, "timing");
      if (!rc && (best_t < 0.0f || ms < best_t)) {
        best_t = ms;
        best = cand[ci];
      }
    }
    b->cls[k].L = best;
    best_ms[k] = best_t / kTimed;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (!rc) rc = plan(b);
  // the one-launch form: its blocks per CU, then the faster of the two
  // forms
  std::vector<float> pms;
  if (!rc && b->persist) {
    rc = tune_persist(b, phase_dev, &pms);
    if (!rc) rc = plan(b);
  }
  b->prof_mask = saved_mask;
  if (rc) return rc;
  if (table_out) {
    FILE* f = fopen(table_out, "w");
    if (!f) return bfail(b, ASH_EINVAL, std::string("cannot write ") + table_out);
    fprintf(f, "# groups range_reduce range_blocks %s_plus_reduce_ms\n",
            b->fused ? "fused" : "forward");
    for (size_t k = 0; k < b->cls.size(); ++k)
      fprintf(f, "%d %d %d %.4f\n", b->cls[k].G, b->cls[k].reduce,
              b->cls[k].L, best_ms[k]);
    if (b->persist) {
      fprintf(f, "# one_launch groups range_reduce blocks_per_cu "
                 "ms_per_iteration\n");
      for (size_t k = 0; k < b->cls.size(); ++k)
        fprintf(f, "one_launch %d %d %d %.4f\n", b->cls[k].G,
                b->cls[k].reduce, b->cls[k].bpc, pms[k]);
      fprintf(f, "# form (1: one launch, 0: launches per phase), "
                 "ms_per_iteration of the launches per phase\n");
      fprintf(f, "form %d %.4f\n", b->one_launch ? 1 : 0, pms.back());
    }
    fclose(f);
  }
  return ASH_OK;
}

int ash_batch_load_tuning(ash_batch* b, const char* table_in) {
  if (!b || !table_in) return ASH_EINVAL;
  b->err.clear();
  FILE* f = fopen(table_in, "r");
  if (!f) return bfail(b, ASH_EINVAL, std::string("cannot read ") + table_in);
  char line[256];
  int n_set = 0;
  while (fgets(line, sizeof line, f)) {
    if (line[0] == '#') continue;
    int G = 0, red = 0, L = 0, bpc = 0;
    if (sscanf(line, "form %d", &L) == 1) {
      b->one_launch = b->persist && L == 1;
      continue;
    }
    if (sscanf(line, "one_launch %d %d %d", &G, &red, &bpc) == 3) {
      if (bpc < 0 || bpc > 64) continue;
      for (auto& c : b->cls)
        if (c.G == G && c.reduce == red) {
          c.bpc = bpc;
          ++n_set;
        }
      continue;
    }
    if (sscanf(line, "%d %d %d", &G, &red, &L) != 3) continue;
    if (L < 1 || L > (1 << 20)) continue;
    for (auto& c : b->cls)
      if (c.G == G && c.reduce == red) {
        c.L = L;
        ++n_set;
      }
  }
  fclose(f);
  int rc = buse(b);
  if (!rc) rc = plan(b);
  return rc ? rc : ASH_OK;
}

int ash_batch_set_form(ash_batch* b, int one_launch) {
  if (!b || (one_launch != 0 && one_launch != 1)) return ASH_EINVAL;
  b->err.clear();
  if (one_launch && !b->persist)
    return bfail(b, ASH_EUNSUPPORTED,
                 "the one-launch form needs members of at most 512 spots "
                 "and a device with cooperative launches");
  b->one_launch = one_launch != 0;
  return ASH_OK;
}

int ash_batch_get_info(const ash_batch* b, ash_batch_info* out) {
  if (!b || !out) return ASH_EINVAL;
  memset(out, 0, sizeof *out);
  out->holograms = (int32_t)b->m.size();
  out->shapes = (int32_t)b->cls.size();
  for (size_t k = 0; k < b->cls.size() && k < 4; ++k) {
    out->groups[k] = b->cls[k].G;
    out->range_blocks[k] = b->cls[k].L;
  }
  out->items = (int64_t)b->items.size();
  out->evals_per_transform = b->evals_per_transform;
  out->one_launch = b->one_launch ? 1 : 0;
  out->fused = b->fused ? 1 : 0;
  for (size_t k = 0; k < b->cls.size() && k < 4; ++k) {
    out->blocks_per_cu[k] = b->one_launch ? b->cls[k].p_grid / b->n_cu : 0;
    out->grid[k] = b->one_launch ? b->cls[k].p_grid : 0;
  }
  return ASH_OK;
}

int ash_batch_profile_enable(ash_batch* b, int mask) {
  if (!b) return ASH_EINVAL;
  if (mask & ~ASH_PROF_ALL) return bfail(b, ASH_EINVAL, "unknown category bits");
  b->prof_mask = mask;
  return ASH_OK;
}

int ash_batch_profile_read(ash_batch* b, double* ms_out,
                           int64_t* launches_out) {
  if (!b) return ASH_EINVAL;
  int rc = buse(b);
  if (rc) return rc;
  double ms[4] = {0, 0, 0, 0};
  int64_t n[4] = {0, 0, 0, 0};
  hipError_t e = hipStreamSynchronize(b->stream);
  for (auto& r : b->prof) {
    float t = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, r.start, r.stop);
    ms[r.cat] += t;
    n[r.cat] += 1;
    b->pool.push_back(r.start);
    b->pool.push_back(r.stop);
  }
  b->prof.clear();
  if (e != hipSuccess) return bhip(b, e, "reading kernel timings");
  for (int k = 0; k < 4; ++k) {
    if (ms_out) ms_out[k] = ms[k];
    if (launches_out) launches_out[k] = n[k];
  }
  return ASH_OK;
}

}  // extern "C"
