// Host side of libss: the C ABI declared in include/ss.h.
//
// Parameters are resolved and validated before any device work (Sec. 3.1),
// the caller's workspace is carved into the flow's buffers (fields, velocity,
// RK stage arrays, reduction partials, a device status block), and the flow
// passes are queued on the caller's stream. ss_minimise captures a HIP graph
// of K flow steps once per context and replays it; the stop decision is taken
// on the device, so the host only reads a small status block between replays.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <new>
#include <string>
#include <vector>
#include <algorithm>
#include <mutex>

#include "../../include/ss.h"
#include "ss_kernels.hpp"
#include "ss_demag.hpp"
#include "ss_bec.hpp"

using namespace ss;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

#define SS_HIP(call)                                                                          \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess)                                                                     \
      return fail(SS_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));                \
  } while (0)

// Tile shapes compiled into the library: a workgroup covers TX x TY sites,
// each thread RY rows of one column. ss_autotune times them on the caller's
// lattice; SS_TILE (environment) or ss_set_tile force one.
struct TileCfg {
  int TX, TY, RY;
};
constexpr TileCfg kTiles[] = {{64, 16, 2}, {64, 8, 2}, {64, 16, 4}, {64, 32, 4}};
constexpr int kNumTiles = 4;
constexpr int kDefaultTile = 0;
constexpr int kDefaultPlanF32 = SS_PLAN_FUSED;
static_assert(kTiles[0].TX == kExTX && kTiles[0].TY == kExTY, "the exact-gradient passes use the layout of tile 0");
static_assert(kTiles[0].TX == 64 && kTiles[0].TY == 16 && kTiles[1].TX == 64 && kTiles[1].TY == 8,
              "the fused passes use the layouts of tiles 0 (64 x 16) and 1 (64 x 8)");
constexpr int kDefaultGraphSteps = 16;
constexpr long kMaxGroups = 2048;  // persistent launch: at most 8 workgroups per CU

int lower_eq(const char* a, const char* b) {
  for (; *a && *b; ++a, ++b) {
    char x = *a, y = *b;
    if (x >= 'A' && x <= 'Z') x = char(x - 'A' + 'a');
    if (y >= 'A' && y <= 'Z') y = char(y - 'A' + 'a');
    if (x == '_' || x == '-') x = ' ';
    if (y == '_' || y == '-') y = ' ';
    if (x != y) return 0;
  }
  return *a == 0 && *b == 0;
}

long round_up(long x, long m) { return (x + m - 1) / m * m; }

constexpr int kMaxVortices = 8192;

struct Layout {
  long pitch, plane;        // elements
  long col0;                // element offset of padded column 0 from the set base
  size_t set_bytes;         // bytes of one C-plane field set (256-B aligned)
  size_t status_off, partial_off, init_off, total;
  int ntx, nty, nlaunch;    // for the selected tile shape
  int seg;                  // tiles per work unit of the stage launches
};

void set_tiles(Layout& L, int Nx, int Ny, int tile) {
  const TileCfg tc = kTiles[tile];
  L.ntx = (Nx + tc.TX - 1) / tc.TX;
  L.nty = (Ny + tc.TY - 1) / tc.TY;
  L.nlaunch = (int)std::min<long>(round_up((long)L.ntx * L.nty, 8), kMaxGroups);
  // one unit per workgroup where there are enough tiles, else single tiles
  L.seg = (int)std::max<long>(1, ((long)L.ntx * L.nty) / L.nlaunch);
  L.seg = std::min(L.seg, L.nty);
}

Layout make_layout(int C, int Nx, int Ny, int esize) {
  Layout L;
  // 16-byte staging loads of a tile row may run up to roundup(Nx, TX) + 4
  // columns for any tile width TX dividing 256; keep them inside the row
  // Interior column 0 of every row sits on a 128-byte line: padded column 0
  // (the first halo column) is at element col0 = 128 / esize - 2 of the row, so
  // a wave's row of loads or stores covers whole lines. The kernels address a
  // set through a base pointer shifted by col0.
  L.col0 = 128 / esize - 2;
  L.pitch = round_up(L.col0 + round_up(Nx, 256) + 4, 64);
  L.plane = round_up(L.pitch * (Ny + 4), 64);
  L.set_bytes = (size_t)round_up(((long)C * L.plane + L.col0) * esize, 256);
  set_tiles(L, Nx, Ny, kDefaultTile);
  L.status_off = 7 * L.set_bytes;
  L.partial_off = L.status_off + (size_t)round_up(sizeof(DevStatus), 256);
  // partials: 4 doubles per stage-pass workgroup, 5 per observable workgroup
  const long nobs = 1024;
  const long nparts = std::max<long>(4L * kMaxGroups, 5L * nobs);
  L.init_off = L.partial_off + (size_t)round_up(nparts * 8, 256);
  // staging of ansatz centres and windings for ss_init_ansatz
  L.total = L.init_off + (size_t)round_up(3L * kMaxVortices * 8, 256);
  return L;
}

// BEC work region (after the flow's buffers): stage point and gradient sets,
// kBecGroups * 4 partials and eight scalars. With base == nullptr only the size.
size_t bec_region(const Layout& L, char* base, void** ptrs) {
  const size_t sizes[6] = {L.set_bytes, L.set_bytes, (size_t)round_up(kBecGroups * 4 * 8, 256), 256,
                           (size_t)round_up(kBecGroups * 8, 256), (size_t)round_up(kBecGroups * 4 * 8, 256)};
  size_t off = 0;
  for (int k = 0; k < 6; ++k) {
    if (ptrs) ptrs[k] = base + off;
    off += sizes[k];
  }
  return off;
}

}  // namespace

struct ss_batch;

struct ss_ctx {
  int theory, dtype, grad_mode, C, Nx, Ny;
  double h, courant;
  double p[kNumParams];
  hipStream_t stream;
  hipStream_t cap_stream;
  char* ws;
  Layout L;
  void* phi[2];
  void* vel[2];
  void* a1;
  void* a2;
  void* q;
  DevStatus* st;
  double* partials;
  hipGraphExec_t graph;
  int graph_steps;
  int tile;
  int plan;   // SS_PLAN_*: how stages 2-4 of a step are launched
  int integ;  // SS_INTEG_*: the flow's integrator
  int vv_form;  // SS_VV_*: how velocity Verlet keeps its state between steps
  size_t ws_total;  // bytes of the workspace in use
  // demagnetising potential (chiral magnet with params.i[2] = 1)
  struct Demag {
    int on;
    int iters_flow, iters_eval;  // conjugate-gradient iterations per solve
    void* S;                     // stage point (C planes, flow layout)
    DmVecs v;
    int nlev;
    DmLevel lv[kDmMaxLevels];
    double* cinv;  // inverse of Laplace_h on the coarsest level (cn x cn), or cn = 0
    int cn;
  } dm;
  // BEC work buffers (theory SS_THEORY_BEC): stage point, gradient, partials, scalars
  void* bec_S;
  void* bec_G;
  double* bec_part;
  double* bec_sc;
  double* bec_ps;  // stage-point norm partials
  double* bec_pg;  // gradient-sum partials
};

namespace {

template <class T>
Bufs<T> bufs_of(const ss_ctx* c) {
  Bufs<T> B;
  B.phi[0] = (T*)c->phi[0];
  B.phi[1] = (T*)c->phi[1];
  B.vel[0] = (T*)c->vel[0];
  B.vel[1] = (T*)c->vel[1];
  B.a1 = (T*)c->a1;
  B.a2 = (T*)c->a2;
  B.q = (T*)c->q;
  B.pitch = c->L.pitch;
  B.plane = c->L.plane;
  B.Nx = c->Nx;
  B.Ny = c->Ny;
  B.psi = c->dm.on ? c->dm.v.x : nullptr;
  B.psi_pitch = c->Nx + 4;
  return B;
}

Coeffs coeffs_of(const ss_ctx* c) {
  Coeffs cf;
  cf.h = c->h;
  cf.dt = c->courant * c->h;
  for (int k = 0; k < kNumParams; ++k) cf.p[k] = c->p[k];
  return cf;
}

template <class T>
PassArgs<T> pass_args(const ss_ctx* c) {
  PassArgs<T> a;
  a.B = bufs_of<T>(c);
  a.cf = coeffs_of(c);
  a.st = c->st;
  a.partials = c->partials;
  a.src = nullptr;
  a.out = nullptr;
  a.out_pitch = a.out_plane = 0;
  a.ntx = c->L.ntx;
  a.nty = c->L.nty;
  a.seg = c->L.seg;
  return a;
}

constexpr long kNumCUs = 256;

// Workgroups of one stage-pass instantiation resident on the whole GPU at
// once: the runtime's occupancy for one CU, rounded down to a power of two (so
// units still split evenly over the eight XCD bands), times the CUs. Queried
// once per instantiation on the first device that launches it.
template <class T, int TH, int PASS, int TX, int TY, int RY>
long resident_groups() {
  static const long n = [] {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, reinterpret_cast<const void*>(&stage_pass<T, TH, PASS, TX, TY, RY>), TX * (TY / RY), 0) !=
            hipSuccess ||
        per_cu < 1) {
      (void)hipGetLastError();  // a failed query must not surface as a launch error
      return kMaxGroups;
    }
    int p2 = 1;
    while (2 * p2 <= per_cu) p2 *= 2;
    return std::min(kMaxGroups, kNumCUs * p2);
  }();
  return n;
}

// Launches a pass and returns its workgroup count. P1 runs with at most its
// resident workgroups, each walking longer column segments (on 4096^2 with
// 64 x 16 tiles: 512 groups, 0.184 -> 0.177 ms against 2048).
template <class T, int TH, int PASS, int CFG>
int launch_cfg(const PassArgs<T>& a, int nlaunch, hipStream_t s) {
  constexpr TileCfg tc = kTiles[CFG];
  PassArgs<T> b = a;
  if constexpr (PASS == kP1 || PASS == kPrime || advances_first(PASS) || fixed_tile(PASS) || PASS == kGD) {
    const long r = resident_groups<T, TH, PASS, tc.TX, tc.TY, tc.RY>();
    if (nlaunch > r) {
      nlaunch = (int)r;
      b.seg = (int)std::min<long>(std::max<long>(1, ((long)a.ntx * a.nty) / nlaunch), a.nty);
    }
  }
  hipLaunchKernelGGL((stage_pass<T, TH, PASS, tc.TX, tc.TY, tc.RY>), dim3(nlaunch), dim3(tc.TX, tc.TY / tc.RY), 0,
                     s, b);
  return nlaunch;
}

template <class T, int TH, int PASS>
int launch_pass_t(int tile, const PassArgs<T>& a, int nlaunch, hipStream_t s) {
  switch (tile) {
    case 0: return launch_cfg<T, TH, PASS, 0>(a, nlaunch, s);
    case 1: return launch_cfg<T, TH, PASS, 1>(a, nlaunch, s);
    case 2: return launch_cfg<T, TH, PASS, 2>(a, nlaunch, s);
    default: return launch_cfg<T, TH, PASS, 3>(a, nlaunch, s);
  }
}

int dm_groups(long n) { return (int)std::max<long>(1, std::min<long>((n + 255) / 256, 4096)); }

// One V-cycle from level l (the level's psi and rhs are set): smoothing, the
// residual restricted to the next level, its correction, smoothing; on the
// coarsest level an even number of sweeps from zero.
void dm_vcycle(const ss_ctx::Demag& d, int l, const DevStatus* skip, hipStream_t s) {
  const DmLevel& L = d.lv[l];
  const long small = dm_small_bytes(d.lv, d.nlev, l);
  if (small <= kDmSmallLds) {
    // this level and the coarser ones in one workgroup, in LDS
    DmHierarchy H;
    for (int k = 0; k < d.nlev; ++k) H.lv[k] = d.lv[k];
    H.nlev = d.nlev;
    H.cinv = d.cinv;
    H.cn = d.cn;
    hipLaunchKernelGGL(dm_vcycle_small, dim3(1), dim3(256), (unsigned)small, s, H, l, skip);
    return;
  }
  if (l == d.nlev - 1) {
    hipLaunchKernelGGL(dm_coarse_solve, dim3(1), dim3(256), 0, s, L, skip);
    return;
  }
  // two sweeps psi -> tmp, the residual of tmp restricted, the coarse
  // correction, then tmp + P c smoothed by two sweeps into psi
  static_assert(kDmSmooth == 2, "one launch smooths twice");
  const DmLevel& Cl = d.lv[l + 1];
  const int gt = std::min(dm_tiles(L), 2048);
  hipLaunchKernelGGL(dm_jacobi2, dim3(gt), dim3(256), 0, s, L, (const double*)L.psi, L.tmp, Cl, 0, skip);
  hipLaunchKernelGGL(dm_restrict_res, dim3(std::min(dm_rtiles(Cl), 2048)), dim3(256), 0, s, L,
                     (const double*)L.tmp, Cl, skip);
  dm_vcycle(d, l + 1, skip, s);
  hipLaunchKernelGGL(dm_jacobi2, dim3(gt), dim3(256), 0, s, L, (const double*)L.tmp, L.psi, Cl, 1, skip);
}

// Demagnetising potential of the stage point of pass PASS (Sec. 4.2, eq. (6)),
// queued before the pass: the stage point, then `iters` iterations of
// multigrid-preconditioned conjugate gradients from the last potential. A flow's
// solves stop with the flow (its status block); an evaluation's always run.
template <class T, int PASS>
void demag_solve(const ss_ctx* c, const PassArgs<T>& a, hipStream_t s) {
  const ss_ctx::Demag& d = c->dm;
  const DevStatus* skip = PASS == kEval ? nullptr : c->st;
  const int iters = PASS == kEval ? d.iters_eval : d.iters_flow;
  const DmLevel& L0 = d.lv[0];
  Bufs<T> B = a.B;
  T* S = (T*)d.S;
  hipLaunchKernelGGL((dm_stage_point<T, PASS>), dim3(dm_groups((long)(c->Nx + 4) * (c->Ny + 4))), dim3(256), 0, s, B,
                     a.cf, (const DevStatus*)c->st, a.src, S);
  const int g = dm_groups((long)c->Nx * c->Ny);
  hipLaunchKernelGGL((dm_begin<T>), dim3(g), dim3(256), 0, s, B, (const T*)S, L0, d.v, skip);
  for (int it = 0; it < iters; ++it) {
    const int first = it == 0 ? 1 : 0;
    dm_vcycle(d, 0, skip, s);
    // r.z partials; beta and the direction; Ad with the d.Ad partials; alpha and the update
    hipLaunchKernelGGL(dm_dot, dim3(kDmRedGroups), dim3(256), 0, s, L0, (const double*)d.v.r, (const double*)L0.psi,
                       d.v.part, skip);
    hipLaunchKernelGGL(dm_dir, dim3(g), dim3(256), 0, s, L0, d.v, first, skip);
    hipLaunchKernelGGL(dm_matvec, dim3(kDmRedGroups), dim3(256), 0, s, L0, d.v, skip);
    hipLaunchKernelGGL(dm_update, dim3(g), dim3(256), 0, s, L0, d.v, skip);
  }
}

// A BEC pass (RK4 stages, the one-pass steps, the check, the prime pass and the
// evaluation) in three launches: the stage point and its norm partials; its scale
// to the atom number, G and the partials for mu; mu, the force and the pass's
// update. P4 ends with the step's constraint, velocity Verlet with the projection
// of v', a reducing pass with the status update.
template <class T, int PASS>
void bec_pass(const ss_ctx* c, const PassArgs<T>& a, hipStream_t s) {
  BecBufs<T> W;
  W.S = (T*)c->bec_S;
  W.G = (T*)c->bec_G;
  W.part = c->bec_part;
  W.sc = c->bec_sc;
  W.ps = c->bec_ps;
  W.pg = c->bec_pg;
  const dim3 g(kBecGroups), b(256), b1(256);
  hipLaunchKernelGGL((bec_stage<T, PASS>), g, b, 0, s, a.B, a.cf, (const DevStatus*)c->st, a.src, W);
  hipLaunchKernelGGL((bec_grad<T, PASS>), g, b, 0, s, a.B, a.cf, (const DevStatus*)c->st, W);
  hipLaunchKernelGGL((bec_apply<T, PASS>), g, b, 0, s, a.B, a.cf, (const DevStatus*)c->st, W, (const double*)W.sc,
                     a.out, a.out_pitch, a.out_plane);
  if constexpr (PASS == kP4 || PASS == kVVA) {
    hipLaunchKernelGGL(bec_fix_scalars, dim3(1), b1, 0, s, (const double*)W.part, W.sc, a.cf,
                       (const DevStatus*)c->st);
    if constexpr (PASS == kP4)
      hipLaunchKernelGGL((bec_fix<T>), g, b, 0, s, a.B, (const DevStatus*)c->st, (const double*)W.sc);
    else
      hipLaunchKernelGGL((bec_vproj<T>), g, b, 0, s, a.B, (const DevStatus*)c->st, (const double*)W.sc);
  }
  if constexpr (reduces(PASS))
    hipLaunchKernelGGL((bec_finalise<PASS>), dim3(1), b1, 0, s, c->st, (const double*)W.part, (const double*)W.sc);
}

template <class T, int PASS>
void launch_lattice_pass(const ss_ctx* c, const PassArgs<T>& a, hipStream_t s);

// A pass; a reducing pass (P1, evaluation, check) is followed by its finalise
// launch, which sums the workgroup partials and updates the status. With
// demagnetisation the pass is preceded by the solve for its stage point.
template <class T, int PASS>
void launch_pass(const ss_ctx* c, const PassArgs<T>& a, hipStream_t s) {
  if constexpr (PASS == kGF) {
    // only the BEC keeps the force between gradient-flow steps (the lattice
    // theories run kGD)
    bec_pass<T, PASS>(c, a, s);
    return;
  } else {
    if constexpr (!fixed_tile(PASS) && PASS != kGD) {
      if (c->theory == SS_THEORY_BEC) {
        bec_pass<T, PASS>(c, a, s);
        return;
      }
    }
    launch_lattice_pass<T, PASS>(c, a, s);
  }
}

// A pass of the lattice theories (everything but the BEC).
template <class T, int PASS>
void launch_lattice_pass(const ss_ctx* c, const PassArgs<T>& a, hipStream_t s) {
  // velocity Verlet's restart and end of run evaluate the current field, whose
  // potential the step that made it has solved for
  if (c->dm.on && PASS != kVVRestart && PASS != kVVEnd) demag_solve<T, PASS>(c, a, s);
  int groups = c->L.nlaunch;  // workgroups launched = partials written
  if (c->grad_mode == SS_GRAD_EXACT) {
    // exact-gradient passes: one tile shape (64 x 16), the layout of tile 0
    if (c->theory == SS_THEORY_AH)
      hipLaunchKernelGGL((stage_pass_exact<T, kAH, PASS>), dim3(groups), dim3(kExTX, kExTY / kExRY), 0, s, a);
    else if (c->theory == SS_THEORY_CM)
      hipLaunchKernelGGL((stage_pass_exact<T, kCM, PASS>), dim3(groups), dim3(kExTX, kExTY / kExRY), 0, s, a);
    else
      hipLaunchKernelGGL((stage_pass_exact<T, kBS, PASS>), dim3(groups), dim3(kExTX, kExTY / kExRY), 0, s, a);
  } else if constexpr (fixed_tile(PASS)) {
    // once per run, or after an arrest: one tile shape (64 x 16) whatever the
    // context's tile
    constexpr int kFixedTile = 0;
    PassArgs<T> b = a;
    Layout L = c->L;
    set_tiles(L, c->Nx, c->Ny, kFixedTile);
    b.ntx = L.ntx;
    b.nty = L.nty;
    b.seg = L.seg;
    if (c->theory == SS_THEORY_AH) groups = launch_cfg<T, kAH, PASS, kFixedTile>(b, L.nlaunch, s);
    else if (c->theory == SS_THEORY_CM) groups = launch_cfg<T, kCM, PASS, kFixedTile>(b, L.nlaunch, s);
    else groups = launch_cfg<T, kBS, PASS, kFixedTile>(b, L.nlaunch, s);
  } else if (c->theory == SS_THEORY_AH) {
    groups = launch_pass_t<T, kAH, PASS>(c->tile, a, groups, s);
  } else if (c->theory == SS_THEORY_CM) {
    groups = launch_pass_t<T, kCM, PASS>(c->tile, a, groups, s);
  } else {
    groups = launch_pass_t<T, kBS, PASS>(c->tile, a, groups, s);
  }
  if constexpr (reduces(PASS))
    hipLaunchKernelGGL((pass_finalise<PASS>), dim3(1), dim3(256), 0, s, a.st, (const double*)a.partials, groups,
                       a.cf.h);
}

// Fused stages 2-4 run on 64 x 16 tiles (tile 0) or 64 x 8 tiles (tile 1), two
// rows per thread. FP32 follows the context's tile when it is one of these two
// (so the autotuner can pick either) and uses 64 x 16 otherwise; FP64 always
// uses 64 x 8 (its LDS planes are twice as large).
template <class T>
int fused_layout_tile(int tile) {
  if (sizeof(T) == 8) return 1;
  return tile == 1 ? 1 : 0;
}

template <class T, int TH>
void launch_fused_t(int layout_tile, const PassArgs<T>& a, int nlaunch, hipStream_t s) {
  if constexpr (sizeof(T) == 4) {
    if (layout_tile == 0) {
      hipLaunchKernelGGL((stage_pass_fused<T, TH, 64, 16, 2>), dim3(nlaunch), dim3(64, 8), 0, s, a);
      return;
    }
  }
  hipLaunchKernelGGL((stage_pass_fused<T, TH, 64, 8, 2>), dim3(nlaunch), dim3(64, 4), 0, s, a);
}

// Workgroups of a fused launch: as many as are resident at once (one per CU
// for 512-thread groups at two waves per SIMD, two for 256-thread groups; one
// in FP64), each walking longer column segments, so no workgroup waits for a
// free CU. On 4096^2 (64 x 16, FP32) this took the pass from 0.622 to 0.610 ms
// against 2048 groups.

template <class T>
long fused_groups(int layout_tile) {
  const int threads = (sizeof(T) == 4 && layout_tile == 0) ? 512 : 256;
  const int waves_per_cu = 4 * FusedWaves<T>::value;
  return kNumCUs * std::max(1, waves_per_cu * 64 / threads);
}

template <class T>
void launch_fused(const ss_ctx* c, hipStream_t s) {
  PassArgs<T> a = pass_args<T>(c);
  Layout L = c->L;
  const int lt = fused_layout_tile<T>(c->tile);
  set_tiles(L, c->Nx, c->Ny, lt);
  const long groups = fused_groups<T>(lt);
  if (L.nlaunch > groups) {
    L.nlaunch = (int)groups;
    L.seg = (int)std::min<long>(std::max<long>(1, ((long)L.ntx * L.nty) / groups), L.nty);
  }
  a.ntx = L.ntx;
  a.nty = L.nty;
  a.seg = L.seg;
  if (c->theory == SS_THEORY_AH) launch_fused_t<T, kAH>(lt, a, L.nlaunch, s);
  else if (c->theory == SS_THEORY_CM) launch_fused_t<T, kCM>(lt, a, L.nlaunch, s);
  else launch_fused_t<T, kBS>(lt, a, L.nlaunch, s);
}

// Velocity Verlet's form (SS_VV_AUTO): kick-drift-kick from kKdkMinSites
// interior sites up, where its two fewer field sets per step outweigh the
// launch of its restart pass (about 3 us whether or not it works); the stored
// force below, and always for the BEC.
constexpr long kKdkMinSites = 1L << 20;
bool vv_kdk_form(const ss_ctx* c) {
  if (c->theory == SS_THEORY_BEC) return false;
  if (c->vv_form != SS_VV_AUTO) return c->vv_form == SS_VV_HALF_STEP;
  return (long)c->Nx * c->Ny >= kKdkMinSites;
}
bool vv_kdk(const ss_ctx* c) { return c->integ == SS_INTEG_VV && vv_kdk_form(c); }
// Gradient flow keeping only the field (the lattice theories; the BEC keeps the
// force of the current field between steps).
bool gd_form(const ss_ctx* c) { return c->integ == SS_INTEG_GF && c->theory != SS_THEORY_BEC; }

template <class T>
void enqueue_steps(const ss_ctx* c, int n, hipStream_t s) {
  PassArgs<T> a = pass_args<T>(c);
  if (c->integ != SS_INTEG_RK4) {
    // one pass (and its finalise) per step; velocity Verlet's restart pass
    // before it returns at once unless the last step was arrested
    for (int k = 0; k < n; ++k) {
      if (gd_form(c)) {
        launch_pass<T, kGD>(c, a, s);
      } else if (c->integ == SS_INTEG_GF) {
        launch_pass<T, kGF>(c, a, s);
      } else if (vv_kdk(c)) {
        launch_pass<T, kVVRestart>(c, a, s);
        launch_pass<T, kVV>(c, a, s);
      } else {
        launch_pass<T, kVVA>(c, a, s);
      }
    }
    return;
  }
  for (int k = 0; k < n; ++k) {
    launch_pass<T, kP1>(c, a, s);
    if (c->plan != SS_PLAN_STAGES) {
      launch_fused<T>(c, s);
      continue;
    }
    launch_pass<T, kP2>(c, a, s);
    launch_pass<T, kP3>(c, a, s);
    launch_pass<T, kP4>(c, a, s);
  }
}

void enqueue_steps_any(const ss_ctx* c, int n, hipStream_t s) {
  if (c->dtype == SS_F32) enqueue_steps<float>(c, n, s);
  else enqueue_steps<double>(c, n, s);
}

template <class T>
void enqueue_check(const ss_ctx* c, hipStream_t s) {
  PassArgs<T> a = pass_args<T>(c);
  launch_pass<T, kCheck>(c, a, s);
  hipLaunchKernelGGL((apply_arrest<T>), dim3(1024), dim3(256), 0, s, a.B, c->st, c->C);
}

void enqueue_check_any(const ss_ctx* c, hipStream_t s) {
  if (c->dtype == SS_F32) enqueue_check<float>(c, s);
  else enqueue_check<double>(c, s);
}

// Start of a run of a one-pass integrator: the arrest test of the current field
// (as a check pass) and its force stored in the buffer of the step's parity, or
// for velocity Verlet in kick-drift-kick form u = v + dt/2 a in place of v.
void enqueue_prime_any(const ss_ctx* c, hipStream_t s) {
  if (gd_form(c)) return;  // its first step tests the current field
  if (vv_kdk(c)) {
    if (c->dtype == SS_F32) launch_pass<float, kVVStart>(c, pass_args<float>(c), s);
    else launch_pass<double, kVVStart>(c, pass_args<double>(c), s);
    return;
  }
  if (c->dtype == SS_F32) launch_pass<float, kPrime>(c, pass_args<float>(c), s);
  else launch_pass<double, kPrime>(c, pass_args<double>(c), s);
}

template <class T>
void enqueue_apply_arrest(const ss_ctx* c, hipStream_t s) {
  hipLaunchKernelGGL((apply_arrest<T>), dim3(1024), dim3(256), 0, s, bufs_of<T>(c), c->st, c->C);
}

// End of a run of a one-pass integrator: the velocity of the current field,
// zero if the last test arrested the flow (kick-drift-kick velocity Verlet
// turns u back into v).
void enqueue_settle_any(const ss_ctx* c, hipStream_t s) {
  if (vv_kdk(c)) {
    if (c->dtype == SS_F32) launch_pass<float, kVVEnd>(c, pass_args<float>(c), s);
    else launch_pass<double, kVVEnd>(c, pass_args<double>(c), s);
  } else if (c->dtype == SS_F32) {
    enqueue_apply_arrest<float>(c, s);
  } else {
    enqueue_apply_arrest<double>(c, s);
  }
}

// End of a run of steps: the arrest test of the final field where the
// integrator has not taken it already, then the velocity zeroed if it fired.
void enqueue_end_of_run_any(const ss_ctx* c, hipStream_t s) {
  if (c->integ == SS_INTEG_RK4) {
    enqueue_check_any(c, s);
  } else if (gd_form(c)) {
    // the last field is untested: its energy and gradient
    if (c->dtype == SS_F32) launch_pass<float, kGDCheck>(c, pass_args<float>(c), s);
    else launch_pass<double, kGDCheck>(c, pass_args<double>(c), s);
  } else {
    enqueue_settle_any(c, s);
  }
}

int read_status(ss_ctx* c, DevStatus* out) {
  SS_HIP(hipMemcpyAsync(out, c->st, sizeof(DevStatus), hipMemcpyDeviceToHost, c->stream));
  SS_HIP(hipStreamSynchronize(c->stream));
  return SS_OK;
}

void fill_info(const DevStatus& d, ss_step_info* info) {
  info->energy = d.E;
  info->energy_prev = d.E_prev;
  info->gnorm_inf = d.gmax;
  info->step = d.step;
  info->n_arrests = d.n_arrests;
  info->arrested = d.arrest;
  info->nonfinite = d.nonfinite;
}

size_t esize_of(int dtype) { return dtype == SS_F32 ? 4 : 8; }

// Start from rest (Sec. 3.2): zero velocity and stage arrays, reset counters.
int reset_state(ss_ctx* c) {
  SS_HIP(hipMemsetAsync(c->ws + 2 * c->L.set_bytes, 0, 5 * c->L.set_bytes, c->stream));
  // the demagnetising potential (warm start of the solves) restarts from zero
  if (c->dm.on)
    SS_HIP(hipMemsetAsync(c->dm.v.x, 0, (size_t)(c->Nx + 4) * (c->Ny + 4) * sizeof(double), c->stream));
  DevStatus s;
  std::memset(&s, 0, sizeof(s));
  s.E = s.E_prev = std::numeric_limits<double>::infinity();
  s.gmax = std::numeric_limits<double>::infinity();
  s.e_target = -std::numeric_limits<double>::infinity();
  SS_HIP(hipMemcpyAsync(c->st, &s, sizeof(s), hipMemcpyHostToDevice, c->stream));
  SS_HIP(hipStreamSynchronize(c->stream));
  return SS_OK;
}

}  // namespace

namespace {

// Noise stream key of a seed: mix(seed * golden + stream), stream 1 = interior
// noise; 0 (amplitude <= 0) marks "no noise".
unsigned long long noise_key(uint64_t seed, double amp) {
  if (!(amp > 0.0)) return 0ULL;
  unsigned long long z = (unsigned long long)seed * 0x9E3779B97F4A7C15ULL + 1ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  z ^= z >> 31;
  return z ? z : 1ULL;
}

}  // namespace

namespace {
// Theory, lattice and parameters of a problem, resolved and validated before
// any device work (Sec. 3.1: parameters are resolved first, then packed).
struct Problem {
  int theory, dtype, grad_mode, C, nf_need;
  int dmi_kind, demag;  // chiral magnet: SS_DMI_*, demagnetisation on/off
  double courant;
  double p[kNumParams];
};

int resolve_problem(const char* theory, int Nx, int Ny, double h, const ss_params* params, int dtype, Problem* pb);

}  // namespace

extern "C" {

int ss_theory_id(const char* name) {
  if (!name) return SS_ETHEORY;
  static const char* ah[] = {"abelian_higgs", "abelian higgs", "ginzburg-landau", "gl", "ah", "ginzburg landau"};
  static const char* cm[] = {"chiral_magnet", "chiral magnet", "cm"};
  static const char* bs[] = {"baby_skyrme", "baby skyrme", "bs"};
  static const char* bec[] = {"bec", "bose_einstein", "bose-einstein condensate", "bose einstein condensate",
                              "rotating bec"};
  for (const char* a : ah)
    if (lower_eq(name, a)) return SS_THEORY_AH;
  for (const char* a : cm)
    if (lower_eq(name, a)) return SS_THEORY_CM;
  for (const char* a : bs)
    if (lower_eq(name, a)) return SS_THEORY_BS;
  for (const char* a : bec)
    if (lower_eq(name, a)) return SS_THEORY_BEC;
  return SS_ETHEORY;
}

int ss_components(const char* theory) {
  const int t = ss_theory_id(theory);
  if (t < 0) return t;
  return t == SS_THEORY_AH ? 4 : t == SS_THEORY_BEC ? 2 : 3;
}

int ss_workspace_bytes(const char* theory, int Nx, int Ny, int dtype, size_t* bytes) {
  const int C = ss_components(theory);
  if (C < 0) return fail(SS_ETHEORY, std::string("unknown theory '") + (theory ? theory : "(null)") + "'");
  if (dtype != SS_F32 && dtype != SS_F64) return fail(SS_EINVAL, "dtype must be SS_F32 or SS_F64");
  if (Nx < 8 || Ny < 8 || Nx > 65536 || Ny > 65536) return fail(SS_ESHAPE, "Nx, Ny must lie in [8, 65536]");
  if (!bytes) return fail(SS_EINVAL, "bytes is NULL");
  const Layout L = make_layout(C, Nx, Ny, (int)esize_of(dtype));
  *bytes = L.total + (ss_theory_id(theory) == SS_THEORY_BEC ? bec_region(L, nullptr, nullptr) : 0);
  return SS_OK;
}

}  // extern "C"

namespace {

int resolve_problem(const char* theory, int Nx, int Ny, double h, const ss_params* params, int dtype, Problem* pb) {
  const int th = ss_theory_id(theory);
  if (th < 0) return fail(SS_ETHEORY, std::string("unknown theory '") + (theory ? theory : "(null)") + "'");
  if (dtype != SS_F32 && dtype != SS_F64) return fail(SS_EINVAL, "dtype must be SS_F32 or SS_F64");
  if (Nx < 8 || Ny < 8 || Nx > 65536 || Ny > 65536) return fail(SS_ESHAPE, "Nx, Ny must lie in [8, 65536]");
  if (!(h > 0.0) || !std::isfinite(h)) return fail(SS_EINVAL, "lattice spacing h must be positive and finite");
  if (!params) return fail(SS_EINVAL, "params is NULL");
  // integer options: {grad_mode, dmi_kind, demag}
  int opt[3] = {SS_GRAD_EL, SS_DMI_BULK, 0};
  if (params->ni > 3) return fail(SS_EINVAL, "params.i holds at most {grad_mode, dmi_kind, demag}");
  if (params->ni > 0) {
    if (!params->i) return fail(SS_EINVAL, "params.i is NULL with ni > 0");
    for (int k = 0; k < params->ni; ++k) opt[k] = params->i[k];
  }
  const int grad_mode = opt[0], dmi_kind = opt[1], demag = opt[2];
  if (grad_mode != SS_GRAD_EL && grad_mode != SS_GRAD_EXACT) return fail(SS_EINVAL, "unknown grad_mode");
  if (dmi_kind != SS_DMI_BULK && dmi_kind != SS_DMI_HEUSLER) return fail(SS_EINVAL, "unknown dmi_kind");
  if (demag != 0 && demag != 1) return fail(SS_EINVAL, "demag must be 0 or 1");
  if (th != SS_THEORY_CM && (dmi_kind != SS_DMI_BULK || demag))
    return fail(SS_EINVAL, "DMI variants and demagnetisation belong to the chiral magnet");
  if (demag && grad_mode != SS_GRAD_EL)
    return fail(SS_EINVAL, "the demagnetising term runs with the Euler-Lagrange gradient (grad_mode SS_GRAD_EL)");
  if (th == SS_THEORY_BEC && grad_mode != SS_GRAD_EL)
    return fail(SS_EINVAL, "the BEC runs with the Euler-Lagrange gradient (grad_mode SS_GRAD_EL)");
  const int nf_need = th == SS_THEORY_AH ? 1 : th == SS_THEORY_CM ? 4 + demag : th == SS_THEORY_BEC ? 3 : 2;
  if (!params->f || params->nf < nf_need || params->nf > nf_need + 1)
    return fail(SS_EINVAL, th == SS_THEORY_AH ? "abelian_higgs needs params.f = {lambda [, courant]}"
                           : th == SS_THEORY_CM
                               ? (demag ? "chiral_magnet with demagnetisation needs params.f = {J, D, K, B, mu_d [, courant]}"
                                        : "chiral_magnet needs params.f = {J, D, K, B [, courant]}")
                           : th == SS_THEORY_BEC ? "bec needs params.f = {g, Omega, N [, courant]}"
                                                 : "baby_skyrme needs params.f = {kappa, mu^2 [, courant]}");
  for (int k = 0; k < params->nf; ++k)
    if (!std::isfinite(params->f[k])) return fail(SS_EINVAL, "non-finite parameter");
  const double courant = params->nf > nf_need ? params->f[nf_need] : 0.5;
  if (!(courant > 0.0 && courant < 1.0)) return fail(SS_EINVAL, "courant number C must lie in (0, 1)");
  if (demag && !(params->f[4] > 0.0)) return fail(SS_EINVAL, "mu_d must be positive");
  if (th == SS_THEORY_BEC && !(params->f[2] > 0.0)) return fail(SS_EINVAL, "the atom number N must be positive");
  pb->theory = th;
  pb->dtype = dtype;
  pb->grad_mode = grad_mode;
  pb->dmi_kind = dmi_kind;
  pb->demag = demag;
  pb->C = th == SS_THEORY_AH ? 4 : th == SS_THEORY_BEC ? 2 : 3;
  pb->nf_need = nf_need;
  pb->courant = courant;
  for (int k = 0; k < kNumParams; ++k) pb->p[k] = 0.0;
  for (int k = 0; k < std::min(nf_need, 4); ++k) pb->p[k] = params->f[k];  // BEC: {g, Omega, N}
  if (th == SS_THEORY_CM) {
    // d_1 = e_1 always; d_2 = e_2 (bulk) or -e_2 (Heusler): the y-derivative DMI coefficient
    pb->p[4] = dmi_kind == SS_DMI_HEUSLER ? -params->f[1] : params->f[1];
    pb->p[5] = demag ? params->f[4] : 0.0;
  }
  return SS_OK;
}

// Demagnetisation region of a workspace (after the flow's own buffers): the
// stage point, level 0 of the solver (x, r, d, Ad and the V-cycle's psi, tmp,
// rhs), three planes per coarser level, the reduction partials and scalars.
// With base == nullptr only the size is computed.
size_t demag_region(int Nx, int Ny, double h, const Layout& L, int esize, char* base, ss_ctx::Demag* d) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* p = base ? base + off : nullptr;
    off += (size_t)round_up((long)bytes, 256);
    return p;
  };
  char* S = take(L.set_bytes);
  if (d) d->S = S ? S + L.col0 * esize : nullptr;
  int nx = Nx, ny = Ny, nlev = 0;
  double hl = h;
  for (;;) {
    const size_t pb = (size_t)(nx + 4) * (ny + 4) * sizeof(double);
    DmLevel lv;
    lv.Nx = nx;
    lv.Ny = ny;
    lv.pitch = nx + 4;
    lv.h = hl;
    if (nlev == 0) {
      double* x = (double*)take(pb);
      double* r = (double*)take(pb);
      double* dd = (double*)take(pb);
      double* ad = (double*)take(pb);
      if (d) {
        d->v.x = x;
        d->v.r = r;
        d->v.d = dd;
        d->v.Ad = ad;
      }
    }
    lv.psi = (double*)take(pb);
    lv.tmp = (double*)take(pb);
    lv.rhs = (double*)take(pb);
    if (d) d->lv[nlev] = lv;
    ++nlev;
    if (std::min(nx, ny) < 8 || nlev == kDmMaxLevels) break;
    nx = (nx + 1) / 2;
    ny = (ny + 1) / 2;
    hl *= 2.0;
  }
  double* part = (double*)take(kDmRedGroups * sizeof(double));
  double* pmv = (double*)take(kDmRedGroups * sizeof(double));
  double* sc = (double*)take(8 * sizeof(double));
  const int cn = (long)nx * ny <= kDmExactMax ? nx * ny : 0;
  double* cinv = cn ? (double*)take((size_t)cn * cn * sizeof(double)) : nullptr;
  if (d) {
    d->nlev = nlev;
    d->v.part = part;
    d->v.pmv = pmv;
    d->v.sc = sc;
    d->cinv = cinv;
    d->cn = cn;
  }
  return off;
}

// Inverse of Laplace_h (eq. (2) along both axes, zero outside the interior) on
// an nx x ny level of spacing h, sites numbered row-major: Gauss-Jordan
// elimination with partial pivoting in FP64 on the host. out holds n x n, n = nx ny.
void dm_coarse_inverse(int nx, int ny, double h, std::vector<double>& out) {
  const int n = nx * ny;
  std::vector<double> a((size_t)n * n, 0.0);
  out.assign((size_t)n * n, 0.0);
  const double w = 1.0 / (12.0 * h * h);
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      const int m = j * nx + i;
      a[(size_t)m * n + m] = -60.0 * w;
      const int dj[8] = {0, 0, 0, 0, -1, 1, -2, 2}, di[8] = {-1, 1, -2, 2, 0, 0, 0, 0};
      const double cw[8] = {16.0, 16.0, -1.0, -1.0, 16.0, 16.0, -1.0, -1.0};
      for (int q = 0; q < 8; ++q) {
        const int jj = j + dj[q], ii = i + di[q];
        if (jj >= 0 && jj < ny && ii >= 0 && ii < nx) a[(size_t)m * n + jj * nx + ii] += cw[q] * w;
      }
      out[(size_t)m * n + m] = 1.0;
    }
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(a[(size_t)r * n + c]) > std::fabs(a[(size_t)piv * n + c])) piv = r;
    if (piv != c)
      for (int k = 0; k < n; ++k) {
        std::swap(a[(size_t)c * n + k], a[(size_t)piv * n + k]);
        std::swap(out[(size_t)c * n + k], out[(size_t)piv * n + k]);
      }
    const double inv = 1.0 / a[(size_t)c * n + c];
    for (int k = 0; k < n; ++k) {
      a[(size_t)c * n + k] *= inv;
      out[(size_t)c * n + k] *= inv;
    }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      const double f = a[(size_t)r * n + c];
      if (f == 0.0) continue;
      for (int k = 0; k < n; ++k) {
        a[(size_t)r * n + k] -= f * a[(size_t)c * n + k];
        out[(size_t)r * n + k] -= f * out[(size_t)c * n + k];
      }
    }
  }
}

}  // namespace

extern "C" {

int ss_workspace_bytes_for(const char* theory, int Nx, int Ny, const ss_params* params, int dtype, size_t* bytes) {
  Problem pb;
  int rc = resolve_problem(theory, Nx, Ny, 1.0, params, dtype, &pb);
  if (rc) return rc;
  if (!bytes) return fail(SS_EINVAL, "bytes is NULL");
  const Layout L = make_layout(pb.C, Nx, Ny, (int)esize_of(dtype));
  *bytes = L.total + (pb.demag ? demag_region(Nx, Ny, 1.0, L, (int)esize_of(dtype), nullptr, nullptr) : 0) +
           (pb.theory == SS_THEORY_BEC ? bec_region(L, nullptr, nullptr) : 0);
  return SS_OK;
}

int ss_create(const char* theory, int Nx, int Ny, double h, const ss_params* params, int dtype, void* workspace,
              size_t ws_bytes, void* stream, ss_ctx** out) {
  if (!out) return fail(SS_EINVAL, "out is NULL");
  *out = nullptr;
  Problem pb;
  int rc = resolve_problem(theory, Nx, Ny, h, params, dtype, &pb);
  if (rc) return rc;
  size_t need = 0;
  rc = ss_workspace_bytes_for(theory, Nx, Ny, params, dtype, &need);
  if (rc) return rc;
  if (!workspace || ws_bytes < need) return fail(SS_EINVAL, "workspace missing or smaller than ss_workspace_bytes");
  if (((uintptr_t)workspace) % 256 != 0) return fail(SS_EINVAL, "workspace must be 256-byte aligned");
  const int th = pb.theory, grad_mode = pb.grad_mode;

  ss_ctx* c = new (std::nothrow) ss_ctx();
  if (!c) return fail(SS_EINVAL, "out of host memory");
  c->theory = th;
  c->dtype = dtype;
  c->grad_mode = grad_mode;
  c->C = pb.C;
  c->Nx = Nx;
  c->Ny = Ny;
  c->h = h;
  c->courant = pb.courant;
  for (int k = 0; k < kNumParams; ++k) c->p[k] = pb.p[k];
  c->stream = (hipStream_t)stream;
  c->ws = (char*)workspace;
  c->L = make_layout(c->C, Nx, Ny, (int)esize_of(dtype));
  void** sets[7] = {&c->phi[0], &c->phi[1], &c->vel[0], &c->vel[1], &c->a1, &c->a2, &c->q};
  for (int k = 0; k < 7; ++k) *sets[k] = c->ws + k * c->L.set_bytes + c->L.col0 * esize_of(dtype);
  c->st = (DevStatus*)(c->ws + c->L.status_off);
  c->partials = (double*)(c->ws + c->L.partial_off);
  c->graph = nullptr;
  c->graph_steps = 0;
  c->tile = kDefaultTile;
  if (const char* env = std::getenv("SS_TILE")) {
    const int t = std::atoi(env);
    if (t >= 0 && t < kNumTiles) c->tile = t;
  }
  if (grad_mode == SS_GRAD_EXACT) c->tile = 0;
  set_tiles(c->L, Nx, Ny, c->tile);
  c->plan = (grad_mode == SS_GRAD_EL && dtype == SS_F32 && !pb.demag && th != SS_THEORY_BEC) ? kDefaultPlanF32
                                                                                          : SS_PLAN_STAGES;
  c->integ = SS_INTEG_RK4;
  c->vv_form = SS_VV_AUTO;
  c->ws_total = need;
  std::memset(&c->dm, 0, sizeof(c->dm));
  c->bec_S = c->bec_G = nullptr;
  c->bec_part = c->bec_sc = c->bec_ps = c->bec_pg = nullptr;
  if (th == SS_THEORY_BEC) {
    void* ptrs[6];
    bec_region(c->L, c->ws + c->L.total, ptrs);
    c->bec_S = (char*)ptrs[0] + c->L.col0 * esize_of(dtype);
    c->bec_G = (char*)ptrs[1] + c->L.col0 * esize_of(dtype);
    c->bec_part = (double*)ptrs[2];
    c->bec_sc = (double*)ptrs[3];
    c->bec_ps = (double*)ptrs[4];
    c->bec_pg = (double*)ptrs[5];
  }
  if (pb.demag) {
    c->dm.on = 1;
    c->dm.iters_flow = 2;
    c->dm.iters_eval = 40;
    demag_region(Nx, Ny, h, c->L, (int)esize_of(dtype), c->ws + c->L.total, &c->dm);
  }
  hipError_t e = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    delete c;
    return fail(SS_EHIP, std::string("hipStreamCreateWithFlags: ") + hipGetErrorString(e));
  }
  // zero the whole workspace once: halos of velocity and stage arrays stay 0
  e = hipMemsetAsync(c->ws, 0, c->ws_total, c->stream);
  if (e == hipSuccess && c->dm.on && c->dm.cn > 0) {
    // the demagnetisation solver's coarsest-level inverse
    const DmLevel& B = c->dm.lv[c->dm.nlev - 1];
    std::vector<double> inv;
    dm_coarse_inverse(B.Nx, B.Ny, B.h, inv);
    e = hipMemcpyAsync(c->dm.cinv, inv.data(), inv.size() * sizeof(double), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  }
  if (e != hipSuccess) {
    (void)hipStreamDestroy(c->cap_stream);
    delete c;
    return fail(SS_EHIP, std::string("workspace set-up: ") + hipGetErrorString(e));
  }
  *out = c;
  return SS_OK;
}

void ss_destroy(ss_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  if (c->graph) (void)hipGraphExecDestroy(c->graph);
  (void)hipStreamDestroy(c->cap_stream);
  delete c;
}

int ss_set_field(ss_ctx* c, const void* field) {
  if (!c || !field) return fail(SS_EINVAL, "ctx or field is NULL");
  const size_t es = esize_of(c->dtype);
  const size_t upitch = (size_t)(c->Nx + 4) * es;
  const size_t uplane = upitch * (c->Ny + 4);
  for (int b = 0; b < 2; ++b)
    for (int comp = 0; comp < c->C; ++comp)
      SS_HIP(hipMemcpy2DAsync((char*)c->phi[b] + comp * c->L.plane * es, c->L.pitch * es,
                              (const char*)field + comp * uplane, upitch, upitch, c->Ny + 4,
                              hipMemcpyDeviceToDevice, c->stream));
  return reset_state(c);
}

int ss_init_ansatz(ss_ctx* c, int kind, int n, const double* xy, const double* w, const double* shape,
                   uint64_t seed, double noise_amp) {
  if (!c) return fail(SS_EINVAL, "ctx is NULL");
  const int want = c->theory == SS_THEORY_AH    ? SS_ANSATZ_VORTICES
                   : c->theory == SS_THEORY_BEC ? SS_ANSATZ_BEC
                                                : SS_ANSATZ_SKYRMION;
  if (kind != want) return fail(SS_EINVAL, "ansatz kind does not match the theory");
  if (kind == SS_ANSATZ_BEC && (!shape || !(shape[0] > 0.0) || !(shape[1] > 0.0)))
    return fail(SS_EINVAL, "the BEC ansatz needs shape = {R > 0, xi > 0}");
  if (n < 0 || n > kMaxVortices || (n > 0 && !xy)) return fail(SS_EINVAL, "bad vortex list");
  if (kind == SS_ANSATZ_SKYRMION && (n != 1 || !shape)) return fail(SS_EINVAL, "skyrmion needs n = 1 and shape");
  if (kind == SS_ANSATZ_SKYRMION && w && !(w[0] != 0.0 && w[0] == std::nearbyint(w[0]) && std::fabs(w[0]) <= 64.0))
    return fail(SS_EINVAL, "skyrmion vorticity w[0] must be a nonzero integer");
  if (!(noise_amp >= 0.0) || !std::isfinite(noise_amp)) return fail(SS_EINVAL, "bad noise amplitude");
  std::vector<double> host(3 * (size_t)std::max(n, 1), 0.0);
  for (int k = 0; k < n; ++k) {
    host[2 * k] = xy[2 * k];
    host[2 * k + 1] = xy[2 * k + 1];
    host[2 * (size_t)n + k] = w ? w[k] : 1.0;
  }
  double* dev = (double*)(c->ws + c->L.init_off);
  SS_HIP(hipMemcpyAsync(dev, host.data(), host.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
  InitArgs ia;
  ia.kind = kind == SS_ANSATZ_VORTICES ? 0 : kind == SS_ANSATZ_SKYRMION ? 1 : 2;
  ia.n = n;
  ia.xy = dev;
  ia.w = dev + 2 * (size_t)n;
  ia.R = shape ? shape[0] : 0.0;
  ia.gamma = shape ? shape[1] : 0.0;
  ia.amp = noise_amp;
  ia.key = noise_key(seed, noise_amp);
  const long sites = (long)(c->Nx + 4) * (c->Ny + 4);
  const int nb = (int)((sites + 255) / 256);
  if (c->dtype == SS_F32)
    hipLaunchKernelGGL((init_ansatz<float>), dim3(nb), dim3(256), 0, c->stream, bufs_of<float>(c), coeffs_of(c), ia);
  else
    hipLaunchKernelGGL((init_ansatz<double>), dim3(nb), dim3(256), 0, c->stream, bufs_of<double>(c), coeffs_of(c), ia);
  SS_HIP(hipGetLastError());
  return reset_state(c);
}

int ss_time_passes(ss_ctx* c, int n_steps, double* ms) {
  if (!c || !ms || n_steps <= 0) return fail(SS_EINVAL, "bad arguments");
  hipEvent_t ev[5];
  for (int k = 0; k < 5; ++k) SS_HIP(hipEventCreate(&ev[k]));
  double acc[5] = {0, 0, 0, 0, 0};
  hipLaunchKernelGGL(arm_status, dim3(1), dim3(64), 0, c->stream, c->st, 0, 0.0, 0.0, 0, 0LL);
  if (c->integ != SS_INTEG_RK4) enqueue_prime_any(c, c->stream);
  for (int s = 0; s < n_steps; ++s) {
    SS_HIP(hipEventRecord(ev[0], c->stream));
    if (c->integ != SS_INTEG_RK4) {
      // one pass per step: its time (with its finalise) in ms[0]; velocity
      // Verlet's restart pass (timed as launched, also where it returns at
      // once) in ms[1]
      if (vv_kdk(c)) {
        if (c->dtype == SS_F32) launch_pass<float, kVVRestart>(c, pass_args<float>(c), c->stream);
        else launch_pass<double, kVVRestart>(c, pass_args<double>(c), c->stream);
      }
      SS_HIP(hipEventRecord(ev[1], c->stream));
      if (c->dtype == SS_F32) {
        if (gd_form(c)) launch_pass<float, kGD>(c, pass_args<float>(c), c->stream);
        else if (c->integ == SS_INTEG_GF) launch_pass<float, kGF>(c, pass_args<float>(c), c->stream);
        else if (vv_kdk(c)) launch_pass<float, kVV>(c, pass_args<float>(c), c->stream);
        else launch_pass<float, kVVA>(c, pass_args<float>(c), c->stream);
      } else {
        if (gd_form(c)) launch_pass<double, kGD>(c, pass_args<double>(c), c->stream);
        else if (c->integ == SS_INTEG_GF) launch_pass<double, kGF>(c, pass_args<double>(c), c->stream);
        else if (vv_kdk(c)) launch_pass<double, kVV>(c, pass_args<double>(c), c->stream);
        else launch_pass<double, kVVA>(c, pass_args<double>(c), c->stream);
      }
      for (int k = 2; k < 5; ++k) SS_HIP(hipEventRecord(ev[k], c->stream));
    } else if (c->plan != SS_PLAN_STAGES) {
      // stages 2-4 in one pass: its time in ms[1], zero in ms[2] and ms[3]
      if (c->dtype == SS_F32) {
        PassArgs<float> a = pass_args<float>(c);
        launch_pass<float, kP1>(c, a, c->stream); SS_HIP(hipEventRecord(ev[1], c->stream));
        launch_fused<float>(c, c->stream);
      } else {
        PassArgs<double> a = pass_args<double>(c);
        launch_pass<double, kP1>(c, a, c->stream); SS_HIP(hipEventRecord(ev[1], c->stream));
        launch_fused<double>(c, c->stream);
      }
      SS_HIP(hipEventRecord(ev[2], c->stream));
      SS_HIP(hipEventRecord(ev[3], c->stream));
      SS_HIP(hipEventRecord(ev[4], c->stream));
    } else if (c->dtype == SS_F32) {
      PassArgs<float> a = pass_args<float>(c);
      launch_pass<float, kP1>(c, a, c->stream); SS_HIP(hipEventRecord(ev[1], c->stream));
      launch_pass<float, kP2>(c, a, c->stream); SS_HIP(hipEventRecord(ev[2], c->stream));
      launch_pass<float, kP3>(c, a, c->stream); SS_HIP(hipEventRecord(ev[3], c->stream));
      launch_pass<float, kP4>(c, a, c->stream); SS_HIP(hipEventRecord(ev[4], c->stream));
    } else {
      PassArgs<double> a = pass_args<double>(c);
      launch_pass<double, kP1>(c, a, c->stream); SS_HIP(hipEventRecord(ev[1], c->stream));
      launch_pass<double, kP2>(c, a, c->stream); SS_HIP(hipEventRecord(ev[2], c->stream));
      launch_pass<double, kP3>(c, a, c->stream); SS_HIP(hipEventRecord(ev[3], c->stream));
      launch_pass<double, kP4>(c, a, c->stream); SS_HIP(hipEventRecord(ev[4], c->stream));
    }
    SS_HIP(hipEventSynchronize(ev[4]));
    for (int k = 0; k < 4; ++k) {
      float t = 0.f;
      SS_HIP(hipEventElapsedTime(&t, ev[k], ev[k + 1]));
      // one-pass: the step's pass runs between events 1 and 2, the restart before
      const int slot = c->integ == SS_INTEG_RK4 ? k : k == 0 ? 1 : k == 1 ? 0 : k;
      acc[slot] += t;
    }
    float t = 0.f;
    SS_HIP(hipEventElapsedTime(&t, ev[0], ev[4]));
    acc[4] += t;
  }
  enqueue_end_of_run_any(c, c->stream);
  SS_HIP(hipStreamSynchronize(c->stream));
  for (int k = 0; k < 5; ++k) {
    ms[k] = acc[k] / n_steps;
    (void)hipEventDestroy(ev[k]);
  }
  return SS_OK;
}

int ss_get_field(ss_ctx* c, void* field, void* velocity) {
  if (!c || !field) return fail(SS_EINVAL, "ctx or field is NULL");
  DevStatus d;
  int rc = read_status(c, &d);
  if (rc) return rc;
  const int cur = int(d.step & 1);
  const size_t es = esize_of(c->dtype);
  const size_t upitch = (size_t)(c->Nx + 4) * es;
  const size_t uplane = upitch * (c->Ny + 4);
  for (int comp = 0; comp < c->C; ++comp) {
    SS_HIP(hipMemcpy2DAsync((char*)field + comp * uplane, upitch, (char*)c->phi[cur] + comp * c->L.plane * es,
                            c->L.pitch * es, upitch, c->Ny + 4, hipMemcpyDeviceToDevice, c->stream));
    if (velocity)
      SS_HIP(hipMemcpy2DAsync((char*)velocity + comp * uplane, upitch, (char*)c->vel[cur] + comp * c->L.plane * es,
                              c->L.pitch * es, upitch, c->Ny + 4, hipMemcpyDeviceToDevice, c->stream));
  }
  SS_HIP(hipStreamSynchronize(c->stream));
  return SS_OK;
}

// Checkpoint blob: a header that names the problem, then the device status.
struct StateBlob {
  unsigned magic;
  unsigned bytes;
  int theory, dtype, grad_mode, Nx, Ny, pad_;
  DevStatus st;
};
constexpr unsigned kStateMagic = 0x53535354u;  // "SSST"

size_t ss_state_bytes(void) { return sizeof(StateBlob); }

int ss_get_state(ss_ctx* c, void* field, void* velocity, void* state) {
  if (!c || !field || !velocity || !state) return fail(SS_EINVAL, "ctx, field, velocity or state is NULL");
  int rc = ss_get_field(c, field, velocity);
  if (rc) return rc;
  StateBlob b;
  std::memset(&b, 0, sizeof(b));
  b.magic = kStateMagic;
  b.bytes = (unsigned)sizeof(StateBlob);
  b.theory = c->theory;
  b.dtype = c->dtype;
  b.grad_mode = c->grad_mode;
  b.Nx = c->Nx;
  b.Ny = c->Ny;
  rc = read_status(c, &b.st);
  if (rc) return rc;
  std::memcpy(state, &b, sizeof(b));
  return SS_OK;
}

int ss_set_state(ss_ctx* c, const void* field, const void* velocity, const void* state) {
  if (!c || !field || !velocity || !state) return fail(SS_EINVAL, "ctx, field, velocity or state is NULL");
  StateBlob b;
  std::memcpy(&b, state, sizeof(b));
  if (b.magic != kStateMagic || b.bytes != (unsigned)sizeof(StateBlob)) return fail(SS_EINVAL, "not a state blob");
  if (b.theory != c->theory || b.dtype != c->dtype || b.grad_mode != c->grad_mode || b.Nx != c->Nx ||
      b.Ny != c->Ny)
    return fail(SS_ESHAPE, "state was taken on another theory, dtype, gradient form or lattice");
  if (b.st.counter != 0u || b.st.counter_obs != 0u) return fail(SS_EINVAL, "state blob is inconsistent");
  // both ping-pong buffers get the field and the velocity (the halo of the
  // buffer the next step writes must hold the boundary values too)
  const size_t es = esize_of(c->dtype);
  const size_t upitch = (size_t)(c->Nx + 4) * es;
  const size_t uplane = upitch * (c->Ny + 4);
  for (int buf = 0; buf < 2; ++buf)
    for (int comp = 0; comp < c->C; ++comp) {
      SS_HIP(hipMemcpy2DAsync((char*)c->phi[buf] + comp * c->L.plane * es, c->L.pitch * es,
                              (const char*)field + comp * uplane, upitch, upitch, c->Ny + 4,
                              hipMemcpyDeviceToDevice, c->stream));
      SS_HIP(hipMemcpy2DAsync((char*)c->vel[buf] + comp * c->L.plane * es, c->L.pitch * es,
                              (const char*)velocity + comp * uplane, upitch, upitch, c->Ny + 4,
                              hipMemcpyDeviceToDevice, c->stream));
    }
  SS_HIP(hipMemcpyAsync(c->st, &b.st, sizeof(DevStatus), hipMemcpyHostToDevice, c->stream));
  SS_HIP(hipStreamSynchronize(c->stream));
  return SS_OK;
}

int ss_energy_grad(ss_ctx* c, const void* field, void* grad, double* energy, double* gnorm_inf) {
  if (!c) return fail(SS_EINVAL, "ctx is NULL");
  const size_t es = esize_of(c->dtype);
  const size_t upitch = (size_t)(c->Nx + 4) * es;
  const size_t uplane = upitch * (c->Ny + 4);
  if (grad) SS_HIP(hipMemsetAsync(grad, 0, (size_t)c->C * uplane, c->stream));
  // a caller's field is first copied into the q stage array (internal layout);
  // q is rewritten by every third stage pass before it is read, so the flow
  // state is not disturbed
  if (field)
    for (int comp = 0; comp < c->C; ++comp)
      SS_HIP(hipMemcpy2DAsync((char*)c->q + comp * c->L.plane * es, c->L.pitch * es,
                              (const char*)field + comp * uplane, upitch, upitch, c->Ny + 4,
                              hipMemcpyDeviceToDevice, c->stream));
  if (c->dtype == SS_F32) {
    PassArgs<float> a = pass_args<float>(c);
    a.src = field ? (const float*)c->q : nullptr;
    a.out = (float*)grad;
    a.out_pitch = c->Nx + 4;
    a.out_plane = (long)(c->Nx + 4) * (c->Ny + 4);
    launch_pass<float, kEval>(c, a, c->stream);
  } else {
    PassArgs<double> a = pass_args<double>(c);
    a.src = field ? (const double*)c->q : nullptr;
    a.out = (double*)grad;
    a.out_pitch = c->Nx + 4;
    a.out_plane = (long)(c->Nx + 4) * (c->Ny + 4);
    launch_pass<double, kEval>(c, a, c->stream);
  }
  SS_HIP(hipGetLastError());
  DevStatus d;
  int rc = read_status(c, &d);
  if (rc) return rc;
  if (energy) *energy = d.eval_E;
  if (gnorm_inf) *gnorm_inf = d.eval_gmax;
  if (d.nonfinite) return fail(SS_ENONFINITE, "non-finite energy or gradient");
  return SS_OK;
}

}  // extern "C"

// ------------------------------------------------ allocation-free evaluation
// ss_energy_grad_noalloc keeps its status block and workgroup partials in this
// file-scope array instead of a caller's workspace. Every GPU holds its own
// copy; the host reaches it only through the address hipGetSymbolAddress gives
// on that device (the array's name is not a device address in host code).
namespace {

constexpr size_t kScratchStatus = (sizeof(DevStatus) + 255) / 256 * 256;
constexpr size_t kScratchBytes = kScratchStatus + 4 * kMaxGroups * sizeof(double);
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];

// Address of the calling thread's current device's copy of `scratch`, looked up
// once per device.
int scratch_of_current_device(void** out) {
  int dev = -1;
  SS_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(SS_EINVAL, "device index beyond the library's device table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    SS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(SS_EHIP, "hipGetSymbolAddress returned no address for the scratch array");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return SS_OK;
}

template <class T>
__global__ void __launch_bounds__(256) fill_zero(T* __restrict__ p, long n) {
  for (long k = blockIdx.x * 256L + threadIdx.x; k < n; k += (long)gridDim.x * 256L) p[k] = T(0);
}

template <class T>
void enqueue_noalloc_eval(const ss_ctx* c, const void* field, void* grad, hipStream_t s) {
  const long pitch = c->Nx + 4, plane = pitch * (c->Ny + 4);
  if (grad) {
    const long n = (long)c->C * plane;
    const int nb = (int)std::min<long>(1024, (n + 255) / 256);
    hipLaunchKernelGGL((fill_zero<T>), dim3(nb), dim3(256), 0, s, (T*)grad, n);
  }
  PassArgs<T> a;
  std::memset(&a, 0, sizeof(a));
  // the evaluation pass reads only the source field, here in the caller's layout
  a.B.phi[0] = a.B.phi[1] = (T*)field;
  a.B.pitch = pitch;
  a.B.plane = plane;
  a.B.Nx = c->Nx;
  a.B.Ny = c->Ny;
  a.cf = coeffs_of(c);
  a.st = c->st;
  a.partials = c->partials;
  a.src = (const T*)field;
  a.out = (T*)grad;
  a.out_pitch = pitch;
  a.out_plane = plane;
  a.ntx = c->L.ntx;
  a.nty = c->L.nty;
  a.seg = c->L.seg;
  launch_pass<T, kEval>(c, a, s);
}

}  // namespace

extern "C" {

int ss_energy_grad_noalloc(const char* theory, int Nx, int Ny, double h, const ss_params* params, int dtype,
                           const void* field, void* grad, double* energy, double* gnorm_inf, void* stream) {
  Problem pb;
  int rc = resolve_problem(theory, Nx, Ny, h, params, dtype, &pb);
  if (rc) return rc;
  if (!field) return fail(SS_EINVAL, "field is NULL");
  if (pb.demag) return fail(SS_EINVAL, "the demagnetising term needs a context's workspace (use ss_energy_grad)");
  if (pb.theory == SS_THEORY_BEC) return fail(SS_EINVAL, "the BEC's constraint needs a context's workspace (use ss_energy_grad)");
  void* sp = nullptr;
  rc = scratch_of_current_device(&sp);
  if (rc) return rc;
  // a host-side description of the problem; no workspace behind it
  ss_ctx c;
  std::memset(&c, 0, sizeof(c));
  c.theory = pb.theory;
  c.dtype = dtype;
  c.grad_mode = pb.grad_mode;
  c.C = pb.C;
  c.Nx = Nx;
  c.Ny = Ny;
  c.h = h;
  c.courant = pb.courant;
  for (int k = 0; k < kNumParams; ++k) c.p[k] = pb.p[k];
  c.stream = (hipStream_t)stream;
  c.tile = kDefaultTile;
  set_tiles(c.L, Nx, Ny, c.tile);
  if (c.L.nlaunch > kMaxGroups) return fail(SS_ESHAPE, "more workgroup partials than the scratch array holds");
  c.st = (DevStatus*)sp;
  c.partials = (double*)((char*)sp + kScratchStatus);
  if (dtype == SS_F32) enqueue_noalloc_eval<float>(&c, field, grad, c.stream);
  else enqueue_noalloc_eval<double>(&c, field, grad, c.stream);
  SS_HIP(hipGetLastError());
  static_assert(offsetof(DevStatus, eval_gmax) == offsetof(DevStatus, eval_E) + sizeof(double),
                "eval_E and eval_gmax are read back as one pair");
  double vals[2];
  int nonfinite = 0;
  SS_HIP(hipMemcpyAsync(vals, &c.st->eval_E, sizeof(vals), hipMemcpyDeviceToHost, c.stream));
  SS_HIP(hipMemcpyAsync(&nonfinite, &c.st->nonfinite, sizeof(int), hipMemcpyDeviceToHost, c.stream));
  SS_HIP(hipStreamSynchronize(c.stream));
  if (energy) *energy = vals[0];
  if (gnorm_inf) *gnorm_inf = vals[1];
  if (nonfinite) return fail(SS_ENONFINITE, "non-finite energy or gradient");
  return SS_OK;
}

int ss_flow_step(ss_ctx* c, int n_steps, ss_step_info* info) {
  if (!c) return fail(SS_EINVAL, "ctx is NULL");
  if (n_steps < 0) return fail(SS_EINVAL, "n_steps < 0");
  hipLaunchKernelGGL(arm_status, dim3(1), dim3(64), 0, c->stream, c->st, 0, 0.0, 0.0, 0, 0LL);
  if (c->integ != SS_INTEG_RK4) enqueue_prime_any(c, c->stream);
  enqueue_steps_any(c, n_steps, c->stream);
  enqueue_end_of_run_any(c, c->stream);
  SS_HIP(hipGetLastError());
  if (info) {
    DevStatus d;
    int rc = read_status(c, &d);
    if (rc) return rc;
    fill_info(d, info);
    if (d.done == 4) return fail(SS_ENONFINITE, "non-finite value in the flow");
  }
  return SS_OK;
}

int ss_minimise(ss_ctx* c, const ss_stop* stop, ss_min_info* info) {
  if (!c || !stop) return fail(SS_EINVAL, "ctx or stop is NULL");
  if (stop->window < 0 || stop->window > kMaxWindow) return fail(SS_EINVAL, "window must lie in [0, 128]");
  if (stop->max_steps < 0) return fail(SS_EINVAL, "max_steps < 0");
  int K = stop->graph_steps > 0 ? stop->graph_steps : kDefaultGraphSteps;
  if (K % 2) ++K;
  if (c->graph && c->graph_steps != K) {
    (void)hipGraphExecDestroy(c->graph);
    c->graph = nullptr;
  }
  if (!c->graph) {
    hipGraph_t g;
    SS_HIP(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed));
    enqueue_steps_any(c, K, c->cap_stream);
    hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
    if (e != hipSuccess) return fail(SS_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&c->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      c->graph = nullptr;
      return fail(SS_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
    c->graph_steps = K;
  }
  hipLaunchKernelGGL(arm_status, dim3(1), dim3(64), 0, c->stream, c->st, 1, stop->grad_tol, stop->rel_e_tol,
                     stop->window, (long long)stop->max_steps);
  // a one-pass run starts by testing the current field and storing its force
  if (c->integ != SS_INTEG_RK4) enqueue_prime_any(c, c->stream);
  SS_HIP(hipGetLastError());
  DevStatus d;
  for (;;) {
    // a few replays between status reads keep the queue busy
    for (int r = 0; r < 4; ++r) SS_HIP(hipGraphLaunch(c->graph, c->stream));
    int rc = read_status(c, &d);
    if (rc) return rc;
    if (d.done) break;
  }
  if (c->integ == SS_INTEG_RK4) {
    if (c->dtype == SS_F32) enqueue_apply_arrest<float>(c, c->stream);
    else enqueue_apply_arrest<double>(c, c->stream);
  } else {
    enqueue_settle_any(c, c->stream);
  }
  int rc = read_status(c, &d);
  if (rc) return rc;
  if (info) {
    fill_info(d, &info->last);
    info->reason = d.done;
    info->converged = (d.done == SS_STOP_GRAD || d.done == SS_STOP_STALL || d.done == SS_STOP_TARGET) ? 1 : 0;
  }
  if (d.done == SS_STOP_NONFINITE) return fail(SS_ENONFINITE, "non-finite value in the flow");
  if (d.done == SS_STOP_MAXSTEPS) return SS_NOT_CONVERGED;
  return SS_OK;
}

}  // extern "C"

namespace {

// Observable passes of one context, enqueued on its stream; obs_collect reads them back.
template <class T>
void obs_enqueue_t(ss_ctx* c, int nobs) {
  Bufs<T> B = bufs_of<T>(c);
  if (c->theory == SS_THEORY_AH) {
    hipLaunchKernelGGL((obs_sites<T, kAH>), dim3(nobs), dim3(256), 0, c->stream, B, coeffs_of(c), c->st, c->partials,
                       nobs);
    hipLaunchKernelGGL((obs_winding<T>), dim3(1), dim3(256), 0, c->stream, B, c->st);
    return;
  }
  if (c->theory == SS_THEORY_BEC) {
    hipLaunchKernelGGL((bec_obs<T>), dim3(nobs), dim3(256), 0, c->stream, B, coeffs_of(c), c->st, c->partials, nobs);
    return;
  }
  if (c->theory == SS_THEORY_CM) {
    // the potential of the current field, for the demagnetising energy
    if (c->dm.on) demag_solve<T, kEval>(c, pass_args<T>(c), c->stream);
    hipLaunchKernelGGL((obs_sites<T, kCM>), dim3(nobs), dim3(256), 0, c->stream, B, coeffs_of(c), c->st, c->partials,
                       nobs);
  }
  else
    hipLaunchKernelGGL((obs_sites<T, kBS>), dim3(nobs), dim3(256), 0, c->stream, B, coeffs_of(c), c->st, c->partials,
                       nobs);
  hipLaunchKernelGGL((obs_berg_luscher<T>), dim3(nobs), dim3(256), 0, c->stream, B, c->st, c->partials, nobs);
}

int obs_enqueue(ss_ctx* c) {
  const int nobs = 1024;
  if (c->dtype == SS_F32) obs_enqueue_t<float>(c, nobs);
  else obs_enqueue_t<double>(c, nobs);
  SS_HIP(hipGetLastError());
  return SS_OK;
}

}  // namespace

extern "C" {

static int obs_collect(ss_ctx* c, ss_obs* out) {
  DevStatus d;
  int rc = read_status(c, &d);
  if (rc) return rc;
  const double h2 = c->h * c->h;
  std::memset(out, 0, sizeof(*out));
  out->energy = h2 * d.obs[0];
  out->gnorm_inf = d.gmax;
  if (c->theory == SS_THEORY_BEC) {
    out->atoms = h2 * d.obs[1];
    out->lz = h2 * d.obs[2];
  } else if (c->theory == SS_THEORY_AH) {
    out->flux = h2 * d.obs[1];
    out->n_rho = h2 * d.obs[2];
    out->bogo_r1 = h2 * d.obs[3];
    out->bogo_r2 = h2 * d.obs[4];
    out->n_wind = d.obs[6];
  } else {
    out->q_fd = h2 * d.obs[1] / (4.0 * M_PI);
    out->q_bl = d.obs[5] / (4.0 * M_PI);
  }
  return SS_OK;
}

int ss_observables(ss_ctx* c, ss_obs* out) {
  if (!c || !out) return fail(SS_EINVAL, "ctx or out is NULL");
  int rc = obs_enqueue(c);
  return rc ? rc : obs_collect(c, out);
}

int ss_set_tile(ss_ctx* c, int tile) {
  if (!c) return fail(SS_EINVAL, "ctx is NULL");
  if (tile < 0 || tile >= kNumTiles) return fail(SS_EINVAL, "tile index out of range");
  if (c->grad_mode == SS_GRAD_EXACT && tile != 0) return fail(SS_EINVAL, "the exact-gradient passes use tile 0 only");
  SS_HIP(hipStreamSynchronize(c->stream));
  c->tile = tile;
  set_tiles(c->L, c->Nx, c->Ny, tile);
  if (c->graph) {
    (void)hipGraphExecDestroy(c->graph);
    c->graph = nullptr;
  }
  return SS_OK;
}

int ss_set_plan(ss_ctx* c, int plan) {
  if (!c) return fail(SS_EINVAL, "ctx is NULL");
  if (plan < 0 || plan >= SS_NUM_PLANS) return fail(SS_EINVAL, "unknown plan");
  if (plan != SS_PLAN_STAGES && c->grad_mode != SS_GRAD_EL)
    return fail(SS_EINVAL, "the fused plans evaluate the Euler-Lagrange gradient only");
  if (plan != SS_PLAN_STAGES && c->dm.on)
    return fail(SS_EINVAL, "demagnetisation runs with SS_PLAN_STAGES (one solve per stage point)");
  if (plan != SS_PLAN_STAGES && c->theory == SS_THEORY_BEC)
    return fail(SS_EINVAL, "the BEC runs with SS_PLAN_STAGES (its constraint needs whole-lattice sums per stage)");
  SS_HIP(hipStreamSynchronize(c->stream));
  c->plan = plan;
  if (c->graph) {
    (void)hipGraphExecDestroy(c->graph);
    c->graph = nullptr;
  }
  return SS_OK;
}

int ss_get_plan(ss_ctx* c) { return c ? c->plan : SS_EINVAL; }

int ss_set_integrator(ss_ctx* c, int integ) {
  if (!c) return fail(SS_EINVAL, "ctx is NULL");
  if (integ != SS_INTEG_RK4 && integ != SS_INTEG_VV && integ != SS_INTEG_GF)
    return fail(SS_EINVAL, "unknown integrator");
  SS_HIP(hipStreamSynchronize(c->stream));
  c->integ = integ;
  if (c->graph) {
    (void)hipGraphExecDestroy(c->graph);
    c->graph = nullptr;
  }
  return SS_OK;
}

int ss_get_integrator(ss_ctx* c) { return c ? c->integ : SS_EINVAL; }

int ss_set_vv_form(ss_ctx* c, int form) {
  if (!c) return fail(SS_EINVAL, "ctx is NULL");
  if (form != SS_VV_AUTO && form != SS_VV_STORED_FORCE && form != SS_VV_HALF_STEP)
    return fail(SS_EINVAL, "unknown velocity Verlet form");
  if (form == SS_VV_HALF_STEP && c->theory == SS_THEORY_BEC)
    return fail(SS_EINVAL, "the BEC runs velocity Verlet in its stored-force form");
  SS_HIP(hipStreamSynchronize(c->stream));
  c->vv_form = form;
  if (c->graph) {
    (void)hipGraphExecDestroy(c->graph);
    c->graph = nullptr;
  }
  return SS_OK;
}

int ss_get_vv_form(ss_ctx* c) {
  if (!c) return SS_EINVAL;
  return vv_kdk_form(c) ? SS_VV_HALF_STEP : SS_VV_STORED_FORCE;
}

int ss_set_demag_iters(ss_ctx* c, int iters_flow, int iters_eval) {
  if (!c) return fail(SS_EINVAL, "ctx is NULL");
  if (!c->dm.on) return fail(SS_EINVAL, "the context has no demagnetising term");
  if (iters_flow < 1 || iters_flow > 1000 || iters_eval < 1 || iters_eval > 1000)
    return fail(SS_EINVAL, "iteration counts must lie in [1, 1000]");
  SS_HIP(hipStreamSynchronize(c->stream));
  c->dm.iters_flow = iters_flow;
  c->dm.iters_eval = iters_eval;
  if (c->graph) {
    (void)hipGraphExecDestroy(c->graph);
    c->graph = nullptr;
  }
  return SS_OK;
}

int ss_tile_count(void) { return kNumTiles; }

int ss_tile_shape(int tile, int* tx, int* ty, int* ry) {
  if (tile < 0 || tile >= kNumTiles || !tx || !ty || !ry) return fail(SS_EINVAL, "bad tile query");
  *tx = kTiles[tile].TX;
  *ty = kTiles[tile].TY;
  *ry = kTiles[tile].RY;
  return SS_OK;
}

}  // extern "C"

namespace {

// Autotune cache: a text file (path in SS_AUTOTUNE_CACHE) of lines
// "theory dtype grad_mode Nx Ny tiles integrator plan tile", one per tuned problem; the
// last line for a problem wins. "tiles" is the number of compiled tile shapes,
// so entries from a library with other shapes are not used.
std::string tune_key(const ss_ctx* c) {
  char buf[128];
  std::snprintf(buf, sizeof(buf), "%d %d %d %d %d %d %d %d", c->theory, c->dtype, c->grad_mode, c->Nx, c->Ny,
                kNumTiles, c->integ, c->dm.on);
  return buf;
}

bool tune_lookup(const ss_ctx* c, int* plan, int* tile) {
  const char* path = std::getenv("SS_AUTOTUNE_CACHE");
  if (!path || !*path) return false;
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  const std::string key = tune_key(c);
  bool found = false;
  char line[256];
  while (std::fgets(line, sizeof(line), f)) {
    int th, dt, gm, nx, ny, nt, ig, dm, p, t;
    if (std::sscanf(line, "%d %d %d %d %d %d %d %d %d %d", &th, &dt, &gm, &nx, &ny, &nt, &ig, &dm, &p, &t) != 10)
      continue;
    char k[128];
    std::snprintf(k, sizeof(k), "%d %d %d %d %d %d %d %d", th, dt, gm, nx, ny, nt, ig, dm);
    if (key == k && p >= 0 && p < SS_NUM_PLANS && t >= 0 && t < kNumTiles) {
      *plan = p;
      *tile = t;
      found = true;
    }
  }
  std::fclose(f);
  return found;
}

void tune_store(const ss_ctx* c, int plan, int tile) {
  const char* path = std::getenv("SS_AUTOTUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;  // an unwritable cache only costs the next run its timing
  std::fprintf(f, "%s %d %d\n", tune_key(c).c_str(), plan, tile);
  std::fclose(f);
}

}  // namespace

extern "C" {

int ss_autotune(ss_ctx* c, int n_steps, double* ms_out) {
  if (!c || n_steps <= 0) return fail(SS_EINVAL, "bad arguments");
  if (ms_out)
    for (int k = 0; k < SS_NUM_PLANS * kNumTiles; ++k) ms_out[k] = -1.0;
  if (c->grad_mode == SS_GRAD_EXACT || c->theory == SS_THEORY_BEC) {
    if (ms_out) ms_out[0] = 0.0;
    return 0;
  }
  int cached_p = 0, cached_t = 0;
  if (tune_lookup(c, &cached_p, &cached_t)) {
    int rc = ss_set_plan(c, cached_p);
    if (rc) return rc;
    rc = ss_set_tile(c, cached_t);
    if (rc) return rc;
    return cached_t;  // nothing timed: ms_out stays -1 throughout
  }
  // a uniform vacuum (psi = 1, A = 0; n = e_3) keeps every pass finite
  const double zero[2] = {0.0, 0.0};
  const double shape[2] = {0.0, 0.0};
  int rc = c->theory == SS_THEORY_AH ? ss_init_ansatz(c, SS_ANSATZ_VORTICES, 0, nullptr, nullptr, nullptr, 0, 0.0)
                                     : ss_init_ansatz(c, SS_ANSATZ_SKYRMION, 1, zero, nullptr, shape, 0, 0.0);
  if (rc) return rc;
  int best_t = c->tile, best_p = c->plan;
  double best_ms = 1e300;
  const int nplans = c->dm.on ? 1 : SS_NUM_PLANS;
  for (int p = 0; p < nplans; ++p) {
    rc = ss_set_plan(c, p);
    if (rc) return rc;
    for (int t = 0; t < kNumTiles; ++t) {
      rc = ss_set_tile(c, t);
      if (rc) return rc;
      double ms[5];
      rc = ss_time_passes(c, 2, ms);  // warm-up
      if (rc) return rc;
      rc = ss_time_passes(c, n_steps, ms);
      if (rc) return rc;
      if (ms_out) ms_out[p * kNumTiles + t] = ms[4];
      if (ms[4] < best_ms) {
        best_ms = ms[4];
        best_t = t;
        best_p = p;
      }
    }
  }
  rc = ss_set_plan(c, best_p);
  if (rc) return rc;
  rc = ss_set_tile(c, best_t);
  if (rc) return rc;
  tune_store(c, best_p, best_t);
  return reset_state(c) ? SS_EHIP : best_t;
}

int ss_get_tile(ss_ctx* c) { return c ? c->tile : SS_EINVAL; }

int ss_set_energy_target(ss_ctx* c, double e_target) {
  if (!c) return fail(SS_EINVAL, "ctx is NULL");
  SS_HIP(hipMemcpyAsync(&c->st->e_target, &e_target, sizeof(double), hipMemcpyHostToDevice, c->stream));
  SS_HIP(hipStreamSynchronize(c->stream));
  return SS_OK;
}

namespace {
// copy centres (and windings, default +1) into the workspace staging area
int stage_centres(ss_ctx* c, int n, const double* xy, const double* w, double** dxy, double** dw) {
  if (n < 0 || n > kMaxVortices || (n > 0 && !xy)) return fail(SS_EINVAL, "bad vortex list");
  std::vector<double> host(3 * (size_t)std::max(n, 1), 0.0);
  for (int k = 0; k < n; ++k) {
    host[2 * k] = xy[2 * k];
    host[2 * k + 1] = xy[2 * k + 1];
    host[2 * (size_t)n + k] = w ? w[k] : 1.0;
  }
  double* dev = (double*)(c->ws + c->L.init_off);
  SS_HIP(hipMemcpyAsync(dev, host.data(), host.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
  *dxy = dev;
  *dw = dev + 2 * (size_t)n;
  return SS_OK;
}
}  // namespace

int ss_learned_input(ss_ctx* c, int n, const double* xy, double kappa, float* out) {
  if (!c || !out) return fail(SS_EINVAL, "ctx or out is NULL");
  double *dxy, *dw;
  int rc = stage_centres(c, n, xy, nullptr, &dxy, &dw);
  if (rc) return rc;
  const long sites = (long)c->Nx * c->Ny;
  hipLaunchKernelGGL(learned_input, dim3((unsigned)((sites + 255) / 256)), dim3(256), 0, c->stream, c->Nx, c->Ny,
                     c->h, (const double*)dxy, n, kappa, out);
  SS_HIP(hipGetLastError());
  SS_HIP(hipStreamSynchronize(c->stream));
  return SS_OK;
}

int ss_learned_targets(ss_ctx* c, int n, const double* xy, const double* w, float* out) {
  if (!c || !out) return fail(SS_EINVAL, "ctx or out is NULL");
  if (c->theory != SS_THEORY_AH) return fail(SS_EINVAL, "learned targets exist for the Abelian Higgs model only");
  double *dxy, *dw;
  int rc = stage_centres(c, n, xy, w, &dxy, &dw);
  if (rc) return rc;
  const long sites = (long)c->Nx * c->Ny;
  const dim3 g((unsigned)((sites + 255) / 256));
  if (c->dtype == SS_F32)
    hipLaunchKernelGGL((learned_targets<float>), g, dim3(256), 0, c->stream, bufs_of<float>(c), coeffs_of(c), c->st,
                       (const double*)dxy, (const double*)dw, n, out);
  else
    hipLaunchKernelGGL((learned_targets<double>), g, dim3(256), 0, c->stream, bufs_of<double>(c), coeffs_of(c), c->st,
                       (const double*)dxy, (const double*)dw, n, out);
  SS_HIP(hipGetLastError());
  SS_HIP(hipStreamSynchronize(c->stream));
  return SS_OK;
}

int ss_init_learned(ss_ctx* c, int n, const double* xy, const double* w, const float* corr, double sigma,
                    double pin, uint64_t seed, double noise_amp) {
  if (!c || !corr) return fail(SS_EINVAL, "ctx or corrections are NULL");
  if (!std::isfinite(sigma) || !std::isfinite(pin)) return fail(SS_EINVAL, "sigma and pin must be finite");
  if (!std::isfinite(noise_amp) || noise_amp < 0.0) return fail(SS_EINVAL, "noise_amp must be finite and >= 0");
  const unsigned long long key = noise_key(seed, noise_amp);
  if (c->theory != SS_THEORY_AH) return fail(SS_EINVAL, "the learned start exists for the Abelian Higgs model only");
  double *dxy, *dw;
  int rc = stage_centres(c, n, xy, w, &dxy, &dw);
  if (rc) return rc;
  const long sites = (long)(c->Nx + 4) * (c->Ny + 4);
  const dim3 g((unsigned)((sites + 255) / 256));
  if (c->dtype == SS_F32)
    hipLaunchKernelGGL((init_learned<float>), g, dim3(256), 0, c->stream, bufs_of<float>(c), coeffs_of(c),
                       (const double*)dxy, (const double*)dw, n, corr, sigma, pin, key, noise_amp);
  else
    hipLaunchKernelGGL((init_learned<double>), g, dim3(256), 0, c->stream, bufs_of<double>(c), coeffs_of(c),
                       (const double*)dxy, (const double*)dw, n, corr, sigma, pin, key, noise_amp);
  SS_HIP(hipGetLastError());
  return reset_state(c);
}

int ss_get_info(ss_ctx* c, ss_step_info* info) {
  if (!c || !info) return fail(SS_EINVAL, "ctx or info is NULL");
  DevStatus d;
  int rc = read_status(c, &d);
  if (rc) return rc;
  fill_info(d, info);
  return SS_OK;
}

const char* ss_status_string(int code) {
  switch (code) {
    case SS_OK: return "ok";
    case SS_NOT_CONVERGED: return "not converged";
    case SS_EINVAL: return "invalid argument";
    case SS_ETHEORY: return "unknown theory";
    case SS_ESHAPE: return "bad lattice shape";
    case SS_EHIP: return "HIP runtime error";
    case SS_ENONFINITE: return "non-finite value";
    case SS_ESTATE: return "invalid state";
  }
  return "unknown status";
}

const char* ss_last_error(void) { return g_last_error.c_str(); }

double ss_gl_lambda_from_kappa(double kappa) { return 2.0 * kappa * kappa; }

}  // extern "C"

// Lattice and theory of a context, for the network's one-call learned start
// (C++ linkage: not part of the C interface).
namespace ss_detail {
int ctx_shape(const ss_ctx* c, int* Nx, int* Ny, int* theory) {
  if (!c) return SS_EINVAL;
  *Nx = c->Nx;
  *Ny = c->Ny;
  *theory = c->theory;
  return SS_OK;
}
}  // namespace ss_detail

// ======================================================================= batch

struct ss_batch {
  int theory, dtype, C, n, tile;
  int plan;   // SS_PLAN_*; the fused pass runs on tiles 0 and 1 only (see batch_fused)
  int integ;  // SS_INTEG_*
  hipStream_t stream;
  hipStream_t cap_stream;
  std::vector<ss_ctx*> members;
  std::vector<int> ntiles_of;   // tiles per member (current tile shape)
  std::vector<int> unit0_of;    // first unit of each member
  std::vector<int> nunits_of;   // units per member
  int ntiles_total;
  int nunits_total;
  // device tables (inside the workspace)
  char* tables;
  void* inst;          // BatchInst<T>[n]
  DevStatus** st_ptrs; // [n]
  BatchUnit* units;    // [max tiles] (a unit holds at least one tile)
  int* work;           // [max tiles]
  int* nwork;          // [1]
  int* done_flags;     // [n]
  double* partials;    // [4 * max tiles]
  int max_tiles;
  hipGraphExec_t graph;
  int graph_steps;
};

namespace {

size_t batch_table_bytes(int n, int max_tiles) {
  size_t b = 0;
  b += (size_t)round_up((long)n * (long)sizeof(BatchInst<double>), 256);
  b += (size_t)round_up((long)n * 8, 256);
  b += (size_t)round_up((long)max_tiles * (long)sizeof(BatchUnit), 256);
  b += (size_t)round_up((long)max_tiles * 4, 256);
  b += 256;
  b += (size_t)round_up((long)n * 4, 256);
  b += (size_t)round_up((long)max_tiles * 32, 256);
  return b;
}

// upper bound of tiles over all tile shapes
int batch_max_tiles(const int* Nx, const int* Ny, int n) {
  long mx = 0;
  for (int t = 0; t < kNumTiles; ++t) {
    long sum = 0;
    for (int i = 0; i < n; ++i)
      sum += (long)((Nx[i] + kTiles[t].TX - 1) / kTiles[t].TX) * ((Ny[i] + kTiles[t].TY - 1) / kTiles[t].TY);
    mx = std::max(mx, sum);
  }
  return (int)mx;
}

template <class T>
BatchInst<T> batch_inst_of(const ss_ctx* c, int unit0, int nunits) {
  BatchInst<T> I;
  Bufs<T> B = bufs_of<T>(c);
  Coeffs cf = coeffs_of(c);
  I.V.phi[0] = B.phi[0]; I.V.phi[1] = B.phi[1];
  I.V.vel[0] = B.vel[0]; I.V.vel[1] = B.vel[1];
  I.V.a1 = B.a1; I.V.a2 = B.a2; I.V.q = B.q;
  I.V.pitch = B.pitch; I.V.plane = B.plane;
  I.V.Nx = B.Nx; I.V.Ny = B.Ny;
  I.V.h = cf.h; I.V.dt = cf.dt;
  for (int k = 0; k < kNumParams; ++k) I.V.p[k] = cf.p[k];
  I.V.psi = nullptr;  // batches run local theories only
  I.V.psi_pitch = 0;
  I.st = c->st;
  I.unit0 = unit0;
  I.nunits = nunits;
  return I;
}

// Workgroups of a batch launch (persistent, at most 8 per CU).
int batch_nlaunch(const ss_batch* b) { return (int)std::min<long>(round_up(b->nunits_total, 8), kMaxGroups); }

// (Re)build, for the batch's tile shape, the per-member tile and unit counts,
// the units, the member descriptors and a full work list. Units are column
// segments: seg is half the tile count per workgroup of the launch (two or
// more units per workgroup balance uneven members better than one; measured),
// and each member's tile columns are cut into ceil(nty / seg) segments of
// near-equal length, so that units differ little in work. A member's units are
// numbered row-major over (segment row, tile column).
int batch_build_tables(ss_batch* b) {
  b->ntiles_of.assign(b->n, 0);
  b->unit0_of.assign(b->n, 0);
  b->nunits_of.assign(b->n, 0);
  long tot = 0;
  for (int i = 0; i < b->n; ++i) {
    ss_ctx* c = b->members[i];
    c->tile = b->tile;
    set_tiles(c->L, c->Nx, c->Ny, b->tile);
    b->ntiles_of[i] = c->L.ntx * c->L.nty;
    tot += b->ntiles_of[i];
  }
  if (tot > b->max_tiles) return fail(SS_EINVAL, "batch tile table overflow");
  b->ntiles_total = (int)tot;
  const long groups = std::min<long>(round_up(tot, 8), kMaxGroups);
  const int seg = (int)std::max<long>(1, tot / (2 * groups));
  std::vector<BatchUnit> un;
  un.reserve(tot);
  for (int i = 0; i < b->n; ++i) {
    const Layout& L = b->members[i]->L;
    const int nseg = (L.nty + seg - 1) / seg;
    const int base = L.nty / nseg, rem = L.nty % nseg;
    b->unit0_of[i] = (int)un.size();
    for (int k = 0, ty0 = 0; k < nseg; ++k) {
      const int len = base + (k < rem ? 1 : 0);
      for (int tx = 0; tx < L.ntx; ++tx) un.push_back(BatchUnit{i, tx, ty0, len});
      ty0 += len;
    }
    b->nunits_of[i] = (int)un.size() - b->unit0_of[i];
  }
  const int nu = (int)un.size();
  b->nunits_total = nu;
  std::vector<int> wk(nu);
  for (int u = 0; u < nu; ++u) wk[u] = u;
  SS_HIP(hipMemcpyAsync(b->units, un.data(), nu * sizeof(BatchUnit), hipMemcpyHostToDevice, b->stream));
  SS_HIP(hipMemcpyAsync(b->work, wk.data(), nu * sizeof(int), hipMemcpyHostToDevice, b->stream));
  SS_HIP(hipMemcpyAsync(b->nwork, &nu, sizeof(int), hipMemcpyHostToDevice, b->stream));
  std::vector<DevStatus*> sp(b->n);
  for (int i = 0; i < b->n; ++i) sp[i] = b->members[i]->st;
  SS_HIP(hipMemcpyAsync(b->st_ptrs, sp.data(), b->n * sizeof(DevStatus*), hipMemcpyHostToDevice, b->stream));
  if (b->dtype == SS_F32) {
    std::vector<BatchInst<float>> I(b->n);
    for (int i = 0; i < b->n; ++i) I[i] = batch_inst_of<float>(b->members[i], b->unit0_of[i], b->nunits_of[i]);
    SS_HIP(hipMemcpyAsync(b->inst, I.data(), I.size() * sizeof(I[0]), hipMemcpyHostToDevice, b->stream));
  } else {
    std::vector<BatchInst<double>> I(b->n);
    for (int i = 0; i < b->n; ++i) I[i] = batch_inst_of<double>(b->members[i], b->unit0_of[i], b->nunits_of[i]);
    SS_HIP(hipMemcpyAsync(b->inst, I.data(), I.size() * sizeof(I[0]), hipMemcpyHostToDevice, b->stream));
  }
  SS_HIP(hipStreamSynchronize(b->stream));
  if (b->graph) {
    (void)hipGraphExecDestroy(b->graph);
    b->graph = nullptr;
  }
  return SS_OK;
}

// Work list of the members that have not stopped.
int batch_compact(ss_batch* b, const std::vector<int>& done) {
  std::vector<int> wk;
  wk.reserve(b->nunits_total);
  for (int i = 0; i < b->n; ++i)
    if (!done[i])
      for (int k = 0; k < b->nunits_of[i]; ++k) wk.push_back(b->unit0_of[i] + k);
  const int nw = (int)wk.size();
  if (nw) SS_HIP(hipMemcpyAsync(b->work, wk.data(), nw * sizeof(int), hipMemcpyHostToDevice, b->stream));
  SS_HIP(hipMemcpyAsync(b->nwork, &nw, sizeof(int), hipMemcpyHostToDevice, b->stream));
  SS_HIP(hipStreamSynchronize(b->stream));
  return SS_OK;
}

template <class T, int TH, int PASS, int CFG>
void batch_launch_cfg(const BatchArgs<T>& a, int nlaunch, hipStream_t s) {
  constexpr TileCfg tc = kTiles[CFG];
  hipLaunchKernelGGL((batch_pass<T, TH, PASS, tc.TX, tc.TY, tc.RY>), dim3(nlaunch), dim3(tc.TX, tc.TY / tc.RY), 0,
                     s, a);
}

template <class T, int TH, int PASS>
void batch_launch_t(int tile, const BatchArgs<T>& a, int nlaunch, hipStream_t s) {
  switch (tile) {
    case 0: batch_launch_cfg<T, TH, PASS, 0>(a, nlaunch, s); break;
    case 1: batch_launch_cfg<T, TH, PASS, 1>(a, nlaunch, s); break;
    case 2: batch_launch_cfg<T, TH, PASS, 2>(a, nlaunch, s); break;
    default: batch_launch_cfg<T, TH, PASS, 3>(a, nlaunch, s); break;
  }
}

template <class T, int PASS>
void batch_launch(const ss_batch* b, hipStream_t s) {
  BatchArgs<T> a;
  a.inst = (const BatchInst<T>*)b->inst;
  a.work = b->work;
  a.units = b->units;
  a.nwork = b->nwork;
  a.partials = b->partials;
  const int nlaunch = batch_nlaunch(b);
  if (b->theory == SS_THEORY_AH) batch_launch_t<T, 0, PASS>(b->tile, a, nlaunch, s);
  else batch_launch_t<T, 1, PASS>(b->tile, a, nlaunch, s);
  if constexpr (reduces(PASS))
    hipLaunchKernelGGL((batch_finalise<T, PASS>), dim3(b->n), dim3(256), 0, s, a.inst, (const double*)b->partials);
}

template <class T>
bool batch_fused(const ss_batch* b) {
  return b->plan == SS_PLAN_FUSED && b->tile == fused_layout_tile<T>(b->tile);
}

template <class T>
void batch_launch_fused(const ss_batch* b, hipStream_t s) {
  BatchArgs<T> a;
  a.inst = (const BatchInst<T>*)b->inst;
  a.work = b->work;
  a.units = b->units;
  a.nwork = b->nwork;
  a.partials = b->partials;
  const int nlaunch = batch_nlaunch(b);
  // the batch's tile is 64 x 16 (tile 0, FP32 only) or 64 x 8 (tile 1); see batch_fused
  if constexpr (sizeof(T) == 4) {
    if (b->tile == 0) {
      if (b->theory == SS_THEORY_AH)
        hipLaunchKernelGGL((batch_pass_fused<T, 0, 64, 16, 2>), dim3(nlaunch), dim3(64, 8), 0, s, a);
      else
        hipLaunchKernelGGL((batch_pass_fused<T, 1, 64, 16, 2>), dim3(nlaunch), dim3(64, 8), 0, s, a);
      return;
    }
  }
  if (b->theory == SS_THEORY_AH)
    hipLaunchKernelGGL((batch_pass_fused<T, 0, 64, 8, 2>), dim3(nlaunch), dim3(64, 4), 0, s, a);
  else
    hipLaunchKernelGGL((batch_pass_fused<T, 1, 64, 8, 2>), dim3(nlaunch), dim3(64, 4), 0, s, a);
}

template <class T>
void batch_enqueue_steps(const ss_batch* b, int n, hipStream_t s) {
  if (b->integ != SS_INTEG_RK4) {
    // one pass (and the members' finalise) per step; velocity Verlet (in
    // kick-drift-kick form, as for one lattice) restarts the arrested members first
    for (int k = 0; k < n; ++k) {
      if (b->integ == SS_INTEG_VV) {
        batch_launch<T, kVVRestart>(b, s);
        batch_launch<T, kVV>(b, s);
      } else {
        batch_launch<T, kGD>(b, s);
      }
    }
    return;
  }
  const bool fused = batch_fused<T>(b);
  for (int k = 0; k < n; ++k) {
    batch_launch<T, kP1>(b, s);
    if (fused) {
      batch_launch_fused<T>(b, s);
      continue;
    }
    batch_launch<T, kP2>(b, s);
    batch_launch<T, kP3>(b, s);
    batch_launch<T, kP4>(b, s);
  }
}

void batch_enqueue_steps_any(const ss_batch* b, int n, hipStream_t s) {
  if (b->dtype == SS_F32) batch_enqueue_steps<float>(b, n, s);
  else batch_enqueue_steps<double>(b, n, s);
}

// First pass of a velocity Verlet run: each member's current field tested and
// its u formed.
void batch_enqueue_prime(const ss_batch* b, hipStream_t s) {
  // RK4 and gradient flow test the current field in their first step
  if (b->integ != SS_INTEG_VV) return;
  if (b->dtype == SS_F32) batch_launch<float, kVVStart>(b, s);
  else batch_launch<double, kVVStart>(b, s);
}

void batch_enqueue_apply_arrest(const ss_batch* b, hipStream_t s);

// End of a one-pass run: each member's velocity (velocity Verlet turns u back
// into v, or 0 after an arrest; gradient flow has none). The work list must
// hold every member's units.
void batch_enqueue_settle(const ss_batch* b, hipStream_t s) {
  if (b->integ != SS_INTEG_VV) {
    batch_enqueue_apply_arrest(b, s);
  } else if (b->dtype == SS_F32) {
    batch_launch<float, kVVEnd>(b, s);
  } else {
    batch_launch<double, kVVEnd>(b, s);
  }
}

// End of a run: RK4 and gradient flow test the last field (their check passes);
// velocity Verlet has tested it already and turns u back into v.
void batch_enqueue_check(const ss_batch* b, hipStream_t s) {
  if (b->integ == SS_INTEG_GF) {
    // the last fields are untested: their energies and gradients
    if (b->dtype == SS_F32) batch_launch<float, kGDCheck>(b, s);
    else batch_launch<double, kGDCheck>(b, s);
    return;
  }
  if (b->integ != SS_INTEG_RK4) {
    batch_enqueue_settle(b, s);
    return;
  }
  if (b->dtype == SS_F32) {
    batch_launch<float, kCheck>(b, s);
    hipLaunchKernelGGL((batch_apply_arrest<float>), dim3(b->n), dim3(256), 0, s,
                       (const BatchInst<float>*)b->inst, b->C);
  } else {
    batch_launch<double, kCheck>(b, s);
    hipLaunchKernelGGL((batch_apply_arrest<double>), dim3(b->n), dim3(256), 0, s,
                       (const BatchInst<double>*)b->inst, b->C);
  }
}

void batch_enqueue_apply_arrest(const ss_batch* b, hipStream_t s) {
  if (b->dtype == SS_F32)
    hipLaunchKernelGGL((batch_apply_arrest<float>), dim3(b->n), dim3(256), 0, s, (const BatchInst<float>*)b->inst,
                       b->C);
  else
    hipLaunchKernelGGL((batch_apply_arrest<double>), dim3(b->n), dim3(256), 0, s, (const BatchInst<double>*)b->inst,
                       b->C);
}

int batch_read_done(ss_batch* b, std::vector<int>& done) {
  hipLaunchKernelGGL(batch_done_flags, dim3((b->n + 255) / 256), dim3(256), 0, b->stream, b->st_ptrs, b->n,
                     b->done_flags);
  SS_HIP(hipGetLastError());
  done.assign(b->n, 0);
  SS_HIP(hipMemcpyAsync(done.data(), b->done_flags, b->n * sizeof(int), hipMemcpyDeviceToHost, b->stream));
  SS_HIP(hipStreamSynchronize(b->stream));
  return SS_OK;
}

}  // namespace

extern "C" {

int ss_batch_workspace_bytes(const char* theory, int n, const ss_instance* inst, int dtype, size_t* bytes) {
  if (n <= 0 || !inst || !bytes) return fail(SS_EINVAL, "bad batch description");
  size_t tot = 0;
  std::vector<int> nx(n), ny(n);
  for (int i = 0; i < n; ++i) {
    size_t b = 0;
    int rc = ss_workspace_bytes(theory, inst[i].Nx, inst[i].Ny, dtype, &b);
    if (rc) return rc;
    tot += (size_t)round_up((long)b, 256);
    nx[i] = inst[i].Nx;
    ny[i] = inst[i].Ny;
  }
  tot += batch_table_bytes(n, batch_max_tiles(nx.data(), ny.data(), n));
  *bytes = tot;
  return SS_OK;
}

int ss_batch_create(const char* theory, int n, const ss_instance* inst, int dtype, void* workspace, size_t ws_bytes,
                    void* stream, ss_batch** out) {
  if (!out) return fail(SS_EINVAL, "out is NULL");
  *out = nullptr;
  size_t need = 0;
  int rc = ss_batch_workspace_bytes(theory, n, inst, dtype, &need);
  if (rc) return rc;
  if (!workspace || ws_bytes < need) return fail(SS_EINVAL, "workspace missing or smaller than ss_batch_workspace_bytes");
  if (((uintptr_t)workspace) % 256 != 0) return fail(SS_EINVAL, "workspace must be 256-byte aligned");
  if (ss_theory_id(theory) == SS_THEORY_BS || ss_theory_id(theory) == SS_THEORY_BEC)
    return fail(SS_ETHEORY, "batches run the abelian_higgs and chiral_magnet theories");
  ss_batch* b = new (std::nothrow) ss_batch();
  if (!b) return fail(SS_EINVAL, "out of host memory");
  b->theory = ss_theory_id(theory);
  b->dtype = dtype;
  b->C = b->theory == SS_THEORY_AH ? 4 : 3;
  b->n = n;
  b->tile = kDefaultTile;
  b->plan = SS_PLAN_FUSED;
  b->integ = SS_INTEG_RK4;
  b->stream = (hipStream_t)stream;
  b->graph = nullptr;
  b->graph_steps = 0;
  char* p = (char*)workspace;
  for (int i = 0; i < n; ++i) {
    size_t wb = 0;
    ss_workspace_bytes(theory, inst[i].Nx, inst[i].Ny, dtype, &wb);
    wb = (size_t)round_up((long)wb, 256);
    ss_params prm;
    prm.f = inst[i].f;
    prm.nf = inst[i].nf;
    prm.i = nullptr;
    prm.ni = 0;
    ss_ctx* c = nullptr;
    rc = ss_create(theory, inst[i].Nx, inst[i].Ny, inst[i].h, &prm, dtype, p, wb, stream, &c);
    if (rc) {
      for (ss_ctx* m : b->members) ss_destroy(m);
      delete b;
      return rc;
    }
    b->members.push_back(c);
    p += wb;
  }
  std::vector<int> nx(n), ny(n);
  for (int i = 0; i < n; ++i) {
    nx[i] = inst[i].Nx;
    ny[i] = inst[i].Ny;
  }
  b->max_tiles = batch_max_tiles(nx.data(), ny.data(), n);
  char* t = p;
  b->inst = t; t += round_up((long)n * (long)sizeof(BatchInst<double>), 256);
  b->st_ptrs = (DevStatus**)t; t += round_up((long)n * 8, 256);
  b->units = (BatchUnit*)t; t += round_up((long)b->max_tiles * (long)sizeof(BatchUnit), 256);
  b->work = (int*)t; t += round_up((long)b->max_tiles * 4, 256);
  b->nwork = (int*)t; t += 256;
  b->done_flags = (int*)t; t += round_up((long)n * 4, 256);
  b->partials = (double*)t;
  hipError_t e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    for (ss_ctx* m : b->members) ss_destroy(m);
    delete b;
    return fail(SS_EHIP, std::string("hipStreamCreateWithFlags: ") + hipGetErrorString(e));
  }
  if (const char* env = std::getenv("SS_TILE")) {
    const int tl = std::atoi(env);
    if (tl >= 0 && tl < kNumTiles) b->tile = tl;
  }
  rc = batch_build_tables(b);
  if (rc) {
    ss_batch_destroy(b);
    return rc;
  }
  *out = b;
  return SS_OK;
}

void ss_batch_destroy(ss_batch* b) {
  if (!b) return;
  (void)hipStreamSynchronize(b->stream);
  if (b->graph) (void)hipGraphExecDestroy(b->graph);
  (void)hipStreamDestroy(b->cap_stream);
  for (ss_ctx* m : b->members) ss_destroy(m);
  delete b;
}

ss_ctx* ss_batch_member(ss_batch* b, int i) {
  if (!b || i < 0 || i >= b->n) {
    fail(SS_EINVAL, "member index out of range");
    return nullptr;
  }
  return b->members[i];
}

int ss_batch_size(ss_batch* b) { return b ? b->n : SS_EINVAL; }

int ss_batch_set_tile(ss_batch* b, int tile) {
  if (!b) return fail(SS_EINVAL, "batch is NULL");
  if (tile < 0 || tile >= kNumTiles) return fail(SS_EINVAL, "tile index out of range");
  SS_HIP(hipStreamSynchronize(b->stream));
  b->tile = tile;
  return batch_build_tables(b);
}

int ss_batch_set_plan(ss_batch* b, int plan) {
  if (!b) return fail(SS_EINVAL, "batch is NULL");
  if (plan < 0 || plan >= SS_NUM_PLANS) return fail(SS_EINVAL, "unknown plan");
  SS_HIP(hipStreamSynchronize(b->stream));
  b->plan = plan;
  if (b->graph) {
    (void)hipGraphExecDestroy(b->graph);
    b->graph = nullptr;
  }
  return SS_OK;
}

int ss_batch_get_plan(ss_batch* b) { return b ? b->plan : SS_EINVAL; }

int ss_batch_set_integrator(ss_batch* b, int integ) {
  if (!b) return fail(SS_EINVAL, "batch is NULL");
  if (integ != SS_INTEG_RK4 && integ != SS_INTEG_VV && integ != SS_INTEG_GF)
    return fail(SS_EINVAL, "unknown integrator");
  SS_HIP(hipStreamSynchronize(b->stream));
  b->integ = integ;
  if (b->graph) {
    (void)hipGraphExecDestroy(b->graph);
    b->graph = nullptr;
  }
  return SS_OK;
}

int ss_batch_get_integrator(ss_batch* b) { return b ? b->integ : SS_EINVAL; }

int ss_batch_observables(ss_batch* b, ss_obs* out) {
  if (!b || !out) return fail(SS_EINVAL, "batch or out is NULL");
  // Every member's passes go on the batch stream first, so the first read-back
  // waits for all of them and the rest find their results ready.
  for (ss_ctx* m : b->members) {
    int rc = obs_enqueue(m);
    if (rc) return rc;
  }
  for (int i = 0; i < b->n; ++i) {
    int rc = obs_collect(b->members[i], &out[i]);
    if (rc) return rc;
  }
  return SS_OK;
}

int ss_batch_flow_step(ss_batch* b, int n_steps, ss_step_info* infos) {
  if (!b || n_steps < 0) return fail(SS_EINVAL, "bad arguments");
  hipLaunchKernelGGL(batch_arm, dim3((b->n + 255) / 256), dim3(256), 0, b->stream, b->st_ptrs, b->n, 0, 0.0, 0.0, 0,
                     0LL);
  std::vector<int> none(b->n, 0);
  int rc = batch_compact(b, none);
  if (rc) return rc;
  batch_enqueue_prime(b, b->stream);
  batch_enqueue_steps_any(b, n_steps, b->stream);
  batch_enqueue_check(b, b->stream);
  SS_HIP(hipGetLastError());
  if (infos) {
    for (int i = 0; i < b->n; ++i) {
      rc = ss_get_info(b->members[i], &infos[i]);
      if (rc) return rc;
    }
  }
  return SS_OK;
}

int ss_batch_minimise(ss_batch* b, const ss_stop* stop, ss_min_info* infos) {
  if (!b || !stop) return fail(SS_EINVAL, "batch or stop is NULL");
  if (stop->window < 0 || stop->window > kMaxWindow) return fail(SS_EINVAL, "window must lie in [0, 128]");
  int K = stop->graph_steps > 0 ? stop->graph_steps : kDefaultGraphSteps;
  if (b->graph && b->graph_steps != K) {
    (void)hipGraphExecDestroy(b->graph);
    b->graph = nullptr;
  }
  std::vector<int> done(b->n, 0);
  int rc = batch_compact(b, done);
  if (rc) return rc;
  if (!b->graph) {
    hipGraph_t g;
    SS_HIP(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeRelaxed));
    batch_enqueue_steps_any(b, K, b->cap_stream);
    hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
    if (e != hipSuccess) return fail(SS_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      b->graph = nullptr;
      return fail(SS_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
    b->graph_steps = K;
  }
  hipLaunchKernelGGL(batch_arm, dim3((b->n + 255) / 256), dim3(256), 0, b->stream, b->st_ptrs, b->n, 1,
                     stop->grad_tol, stop->rel_e_tol, stop->window, (long long)stop->max_steps);
  batch_enqueue_prime(b, b->stream);
  SS_HIP(hipGetLastError());
  int ndone = 0;
  for (;;) {
    for (int r = 0; r < 2; ++r) SS_HIP(hipGraphLaunch(b->graph, b->stream));
    std::vector<int> now;
    rc = batch_read_done(b, now);
    if (rc) return rc;
    int nd = 0;
    for (int i = 0; i < b->n; ++i) nd += now[i] != 0;
    if (nd == b->n) break;
    if (nd != ndone) {
      rc = batch_compact(b, now);  // drop the tiles of stopped members
      if (rc) return rc;
      ndone = nd;
    }
  }
  rc = batch_compact(b, std::vector<int>(b->n, 0));
  if (rc) return rc;
  if (b->integ == SS_INTEG_RK4) batch_enqueue_apply_arrest(b, b->stream);
  else batch_enqueue_settle(b, b->stream);
  int worst = SS_OK;
  for (int i = 0; i < b->n; ++i) {
    DevStatus d;
    rc = read_status(b->members[i], &d);
    if (rc) return rc;
    if (infos) {
      fill_info(d, &infos[i].last);
      infos[i].reason = d.done;
      infos[i].converged = (d.done == SS_STOP_GRAD || d.done == SS_STOP_STALL || d.done == SS_STOP_TARGET) ? 1 : 0;
    }
    if (d.done == SS_STOP_NONFINITE) worst = SS_ENONFINITE;
    else if (d.done == SS_STOP_MAXSTEPS && worst == SS_OK) worst = SS_NOT_CONVERGED;
  }
  if (worst == SS_ENONFINITE) return fail(SS_ENONFINITE, "non-finite value in a batch member");
  return worst;
}

int ss_batch_autotune(ss_batch* b, int n_steps, double* ms_out) {
  if (!b || n_steps <= 0) return fail(SS_EINVAL, "bad arguments");
  for (ss_ctx* c : b->members) {
    int rc = c->theory == SS_THEORY_AH ? ss_init_ansatz(c, SS_ANSATZ_VORTICES, 0, nullptr, nullptr, nullptr, 0, 0.0)
                                       : 0;
    if (c->theory != SS_THEORY_AH) {
      const double zero[2] = {0.0, 0.0}, shape[2] = {0.0, 0.0};
      rc = ss_init_ansatz(c, SS_ANSATZ_SKYRMION, 1, zero, nullptr, shape, 0, 0.0);
    }
    if (rc) return rc;
  }
  if (ms_out)
    for (int k = 0; k < SS_NUM_PLANS * kNumTiles; ++k) ms_out[k] = -1.0;

  int best = b->tile, best_plan = b->plan;
  double best_ms = 1e300;
  hipEvent_t e0, e1;
  SS_HIP(hipEventCreate(&e0));
  SS_HIP(hipEventCreate(&e1));
  for (int p = 0; p < SS_NUM_PLANS; ++p) {
    for (int t = 0; t < kNumTiles; ++t) {
      // the fused pass runs on tiles 0 and 1 in FP32 and tile 1 in FP64
      if (p == SS_PLAN_FUSED && t != (b->dtype == SS_F32 ? fused_layout_tile<float>(t) : fused_layout_tile<double>(t)))
        continue;
      int rc = ss_batch_set_plan(b, p);
      if (rc) return rc;
      rc = ss_batch_set_tile(b, t);
      if (rc) return rc;
      hipLaunchKernelGGL(batch_arm, dim3((b->n + 255) / 256), dim3(256), 0, b->stream, b->st_ptrs, b->n, 0, 0.0,
                         0.0, 0, 0LL);
      batch_enqueue_prime(b, b->stream);
      batch_enqueue_steps_any(b, 2, b->stream);
      SS_HIP(hipEventRecord(e0, b->stream));
      batch_enqueue_steps_any(b, n_steps, b->stream);
      SS_HIP(hipEventRecord(e1, b->stream));
      if (b->integ != SS_INTEG_RK4) batch_enqueue_settle(b, b->stream);
      SS_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      SS_HIP(hipEventElapsedTime(&ms, e0, e1));
      const double per = ms / n_steps;
      if (ms_out) ms_out[p * kNumTiles + t] = per;
      if (per < best_ms) {
        best_ms = per;
        best = t;
        best_plan = p;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  int rc = ss_batch_set_plan(b, best_plan);
  if (rc) return rc;
  rc = ss_batch_set_tile(b, best);
  if (rc) return rc;
  for (ss_ctx* c : b->members) {
    rc = reset_state(c);
    if (rc) return rc;
  }
  return best;
}

}  // extern "C"
