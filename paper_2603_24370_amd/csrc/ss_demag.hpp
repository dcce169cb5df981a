// Demagnetising potential of the chiral magnet (Sec. 4.2, eq. (5)-(6)).
//
// In units where mu_0 M_s^2 is the coefficient mu_d, the potential psi of a field
// n solves Laplace_h psi = d_x n_1 + d_y n_2 on the interior, with psi = 0 outside
// it: the divergence by eq. (1), the Laplacian by eq. (2) along each axis. The
// energy density gains mu_d/2 |grad_h psi|^2 and the Euler-Lagrange gradient
// mu_d grad_h psi (eq. (1) derivatives of psi); the stage passes add both terms
// from the potential of the stage point they evaluate, solved just before.
//
// Solver: conjugate gradients on the symmetric positive definite A = -Laplace_h,
// preconditioned by one multigrid V-cycle, all in FP64. The hierarchy coarsens
// by two per axis (a coarse cell covers two fine sites, N_c = ceil(N / 2)) down
// to a level with fewer than eight sites along an axis; each level rediscretises
// eq. (2) at its spacing 2^l h with a zero halo of width two. The V-cycle is
// symmetric, as the preconditioner of conjugate gradients must be: two weighted
// Jacobi sweeps before and after the coarse correction, bilinear prolongation P
// (weights 3/4 and 1/4 per axis), restriction P^T / 4, and on the coarsest level
// an exact solve by its inverse (computed once on the host; up to kDmExactMax
// sites) or else an even number of Jacobi sweeps from zero. A solve runs a fixed number of
// iterations, warm-started from the last potential (stage points change little
// from one pass to the next), so that it can be captured in a graph. Dot
// products are summed per workgroup and then in workgroup order (deterministic).
#pragma once

#include "ss_internal.hpp"

namespace ss {

constexpr int kDmMaxLevels = 20;
constexpr int kDmRedGroups = 256;  // workgroups of the dot-product launches (one partial per thread of the sum)
constexpr double kDmOmega = 0.8;   // Jacobi weight (stable below 15/16 for this operator)
constexpr int kDmSmooth = 2;       // sweeps before and after the coarse correction
constexpr int kDmCoarse = 40;      // sweeps on the coarsest level (even) where it has no inverse
constexpr int kDmExactMax = 256;   // coarsest levels up to this many sites are solved exactly

// One level of the hierarchy: padded planes of (Ny + 4) rows of pitch = Nx + 4 doubles.
struct DmLevel {
  double* psi;  // solution (the preconditioned residual z on level 0)
  double* tmp;  // Jacobi partner of psi; holds the residual before a restriction
  double* rhs;
  int Nx, Ny;
  long pitch;
  double h;
};

// Level-0 vectors of conjugate gradients, the reduction partials and the scalars
// {r.z, beta, alpha, d.Ad}.
struct DmVecs {
  double* x;  // the potential psi
  double* r;
  double* d;
  double* Ad;
  double* part;  // kDmRedGroups partials of r.z
  double* pmv;   // kDmRedGroups partials of d.Ad
  double* sc;    // {r.z of the last iteration, beta, alpha, d.Ad}
};

__device__ __forceinline__ bool dm_skip(const DevStatus* st) { return st != nullptr && st->done != 0; }

__device__ __forceinline__ long dm_at(const DmLevel& L, int j, int i) { return (long)(j + 2) * L.pitch + (i + 2); }

// Laplace_h of a padded plane at interior site (j, i): eq. (2) along both axes.
__device__ __forceinline__ double dm_lap(const double* __restrict__ x, long p, int j, int i, double h) {
  const double* c = x + (long)(j + 2) * p + (i + 2);
  const double sx = -(c[-2] + c[2]) + 16.0 * (c[-1] + c[1]);
  const double sy = -(c[-2 * p] + c[2 * p]) + 16.0 * (c[-p] + c[p]);
  return (sx + sy - 60.0 * c[0]) / (12.0 * h * h);
}

#define DM_SITES(L)                                                                        \
  for (long k_ = blockIdx.x * 256L + threadIdx.x; k_ < (long)(L).Nx * (L).Ny;              \
       k_ += (long)gridDim.x * 256L)

// The coarsest level: kDmCoarse Jacobi sweeps (psi -> tmp -> psi ...) from the
// zero start the restriction left, in one workgroup, with a barrier between sweeps
// (one launch instead of kDmCoarse). Global memory is coherent within a workgroup
// across the barrier.
__global__ void __launch_bounds__(256) dm_coarse_solve(DmLevel L, const DevStatus* st) {
  if (dm_skip(st)) return;
  const double s = kDmOmega * L.h * L.h / 5.0;
  const long n = (long)L.Nx * L.Ny;
  for (int sweep = 0; sweep < kDmCoarse; ++sweep) {
    const double* __restrict__ src = (sweep & 1) ? L.tmp : L.psi;
    double* __restrict__ dst = (sweep & 1) ? L.psi : L.tmp;
    for (long k = threadIdx.x; k < n; k += 256) {
      const int j = (int)(k / L.Nx), i = (int)(k - (long)j * L.Nx);
      const long o = dm_at(L, j, i);
      dst[o] = src[o] - s * (L.rhs[o] - dm_lap(src, L.pitch, j, i, L.h));
    }
    __syncthreads();
  }
}

// 1-D weight of fine index f in coarse cell J (transpose of the prolongation):
// f = 2J - 1 and 2J + 2 carry 1/4, f = 2J and 2J + 1 carry 3/4.
__device__ __forceinline__ double dm_w(int f, int J) {
  const int d = f - 2 * J;
  return (d == 0 || d == 1) ? 0.75 : 0.25;
}

// (P c)(j, i): the bilinear correction at fine site (j, i) from the coarse plane
// c of level C (cell-centred positions; coarse cells outside the level count as zero).
__device__ __forceinline__ double dm_prolong_at(const DmLevel& C, const double* __restrict__ c, int j, int i) {
  const int J = j >> 1, I = i >> 1;
  const int J2 = J + ((j & 1) ? 1 : -1), I2 = I + ((i & 1) ? 1 : -1);
  auto cv = [&](int jj, int ii) -> double {
    return (ii >= 0 && ii < C.Nx && jj >= 0 && jj < C.Ny) ? c[dm_at(C, jj, ii)] : 0.0;
  };
  return 0.5625 * cv(J, I) + 0.1875 * (cv(J, I2) + cv(J2, I)) + 0.0625 * cv(J2, I2);
}

// ---- the small levels of a V-cycle in one workgroup, in LDS
// The coarse levels of a V-cycle cost a few microseconds per launch and almost
// nothing to compute. From the first level whose planes and those of every
// coarser level fit in kDmSmallLds bytes, the V-cycle down to the coarsest level
// and back up runs in one workgroup on LDS copies of those planes, phase by phase
// with a barrier between phases: the same updates in the same order of phases as
// the per-level launches, so the result is the same bit for bit. The level's rhs
// and psi are read from global memory at the start and psi written back at the end.
constexpr int kDmSmallLds = 64 * 1024;

struct DmHierarchy {
  DmLevel lv[kDmMaxLevels];
  int nlev;
  // inverse of Laplace_h on the coarsest level (cn x cn, row-major, sites
  // numbered row-major over the interior), or cn = 0 for Jacobi sweeps there
  const double* cinv;
  int cn;
};

// LDS bytes of levels l .. nlev - 1 (three padded planes each)
__host__ __device__ inline long dm_small_bytes(const DmLevel* lv, int nlev, int l) {
  long n = 0;
  for (int k = l; k < nlev; ++k) n += 3L * (lv[k].Nx + 4) * (lv[k].Ny + 4);
  return 8 * n;
}

__device__ __forceinline__ void dm_wg_jacobi(const DmLevel& L, const double* __restrict__ src,
                                             double* __restrict__ dst) {
  const double s = kDmOmega * L.h * L.h / 5.0;
  const long n = (long)L.Nx * L.Ny;
  for (long k = threadIdx.x; k < n; k += 256) {
    const int j = (int)(k / L.Nx), i = (int)(k - (long)j * L.Nx);
    const long o = dm_at(L, j, i);
    dst[o] = src[o] - s * (L.rhs[o] - dm_lap(src, L.pitch, j, i, L.h));
  }
  __syncthreads();
}

__global__ void __launch_bounds__(256) dm_vcycle_small(DmHierarchy H, int l0, const DevStatus* st) {
  if (dm_skip(st)) return;
  extern __shared__ double smem[];
  const int last = H.nlev - 1;
  // the LDS copy of level l (its planes follow those of levels l0 .. l - 1); a
  // value built per use, so that no array of levels is indexed at run time
  auto lds_level = [&](int l) {
    long off = 0;
    for (int k = l0; k < l; ++k) off += 3L * (H.lv[k].Nx + 4) * (H.lv[k].Ny + 4);
    DmLevel L = H.lv[l];
    const long pl = (long)(L.Nx + 4) * (L.Ny + 4);
    L.psi = smem + off;
    L.tmp = smem + off + pl;
    L.rhs = smem + off + 2 * pl;
    return L;
  };
  // every plane zero (halos included) before the interior of level l0 is read in
  const long total = dm_small_bytes(H.lv, H.nlev, l0) / 8;
  for (long k = threadIdx.x; k < total; k += 256) smem[k] = 0.0;
  __syncthreads();
  const DmLevel L0 = lds_level(l0);
  {
    const DmLevel& G = H.lv[l0];
    const long n = (long)G.Nx * G.Ny;
    for (long k = threadIdx.x; k < n; k += 256) {
      const int j = (int)(k / G.Nx), i = (int)(k - (long)j * G.Nx);
      const long o = dm_at(G, j, i);
      L0.rhs[o] = G.rhs[o];
      L0.psi[o] = G.psi[o];
    }
    __syncthreads();
  }
  for (int l = l0; l < last; ++l) {
    const DmLevel F = lds_level(l);
    const DmLevel C = lds_level(l + 1);
    for (int k = 0; k < kDmSmooth; k += 2) {
      dm_wg_jacobi(F, F.psi, F.tmp);
      dm_wg_jacobi(F, F.tmp, F.psi);
    }
    const long nf = (long)F.Nx * F.Ny;
    for (long k = threadIdx.x; k < nf; k += 256) {
      const int j = (int)(k / F.Nx), i = (int)(k - (long)j * F.Nx);
      const long o = dm_at(F, j, i);
      F.tmp[o] = F.rhs[o] - dm_lap(F.psi, F.pitch, j, i, F.h);
    }
    __syncthreads();
    const long nc = (long)C.Nx * C.Ny;
    for (long k = threadIdx.x; k < nc; k += 256) {
      const int J = (int)(k / C.Nx), I = (int)(k - (long)J * C.Nx);
      double acc = 0.0;
      for (int j = max(2 * J - 1, 0); j <= min(2 * J + 2, F.Ny - 1); ++j) {
        double row = 0.0;
        for (int i = max(2 * I - 1, 0); i <= min(2 * I + 2, F.Nx - 1); ++i) row += dm_w(i, I) * F.tmp[dm_at(F, j, i)];
        acc += dm_w(j, J) * row;
      }
      const long o = dm_at(C, J, I);
      C.rhs[o] = 0.25 * acc;
      C.psi[o] = 0.0;
    }
    __syncthreads();
  }
  const DmLevel B = lds_level(last);
  if (H.cn > 0) {
    // the coarsest level solved exactly: psi = (Laplace_h)^-1 rhs, each row summed in site order
    for (int k = threadIdx.x; k < H.cn; k += 256) {
      double acc = 0.0;
      for (int m = 0; m < H.cn; ++m) {
        const int jm = m / B.Nx, im = m - jm * B.Nx;
        acc += H.cinv[(long)k * H.cn + m] * B.rhs[dm_at(B, jm, im)];
      }
      const int jk = k / B.Nx, ik = k - jk * B.Nx;
      B.psi[dm_at(B, jk, ik)] = acc;
    }
    __syncthreads();
  } else {
    for (int k = 0; k < kDmCoarse; k += 2) {
      dm_wg_jacobi(B, B.psi, B.tmp);
      dm_wg_jacobi(B, B.tmp, B.psi);
    }
  }
  for (int l = last - 1; l >= l0; --l) {
    const DmLevel F = lds_level(l);
    const DmLevel C = lds_level(l + 1);
    const long nf = (long)F.Nx * F.Ny;
    for (long k = threadIdx.x; k < nf; k += 256) {
      const int j = (int)(k / F.Nx), i = (int)(k - (long)j * F.Nx);
      F.psi[dm_at(F, j, i)] += dm_prolong_at(C, C.psi, j, i);
    }
    __syncthreads();
    for (int k = 0; k < kDmSmooth; k += 2) {
      dm_wg_jacobi(F, F.psi, F.tmp);
      dm_wg_jacobi(F, F.tmp, F.psi);
    }
  }
  {
    const DmLevel& G = H.lv[l0];
    const long n = (long)G.Nx * G.Ny;
    for (long k = threadIdx.x; k < n; k += 256) {
      const int j = (int)(k / G.Nx), i = (int)(k - (long)j * G.Nx);
      const long o = dm_at(G, j, i);
      G.psi[o] = L0.psi[o];
    }
  }
}

// ---- the large levels: three launches per level and V-cycle
// Pre-smoothing (two sweeps, psi -> tmp), the residual restricted to the next
// level, and prolongation with post-smoothing (tmp + P c -> psi, two sweeps).
// Weighted Jacobi: x' = x - omega h^2/5 (rhs - Laplace_h x) (the operator's
// diagonal is -5/h^2), on interior sites only; halos stay zero. These are the
// same updates, in the same arithmetic, as the one-workgroup small levels and
// the coarsest-level solve use.
constexpr int kDmTile = 16;                // interior sites per side of a smoothing tile
constexpr int kDmTA = kDmTile + 8;         // the input on the tile and a halo of 4
constexpr int kDmTB = kDmTile + 4;         // after one sweep, and rhs: tile and halo 2
constexpr int kDmCT = 8;                   // coarse sites per side of a restriction tile
constexpr int kDmRF = 2 * kDmCT + 2;       // fine residuals it needs per side
constexpr int kDmRP = kDmRF + 4;           // fine psi per side (residuals and a halo of 2)

__host__ __device__ inline int dm_tiles(const DmLevel& L) {
  return ((L.Nx + kDmTile - 1) / kDmTile) * ((L.Ny + kDmTile - 1) / kDmTile);
}

__host__ __device__ inline int dm_rtiles(const DmLevel& C) {
  return ((C.Nx + kDmCT - 1) / kDmCT) * ((C.Ny + kDmCT - 1) / kDmCT);
}

// Two weighted Jacobi sweeps of level L from src into dst, through LDS: the
// first on the tile and a ring of two (zero outside the interior, as the halo of
// a plane is), the second on the tile. With prolong != 0 the input is
// src + P (C.psi), the fine correction of the coarse solve. The loads of a phase
// are unrolled so that a thread has them in flight together.
__global__ void __launch_bounds__(256) dm_jacobi2(DmLevel L, const double* __restrict__ src, double* __restrict__ dst,
                                                  DmLevel C, int prolong, const DevStatus* st) {
  if (dm_skip(st)) return;
  constexpr int NA = kDmTA * kDmTA, NB = kDmTB * kDmTB, NT = kDmTile * kDmTile;
  __shared__ double a[NA];
  __shared__ double b[NB];
  __shared__ double r[NB];
  const double s = kDmOmega * L.h * L.h / 5.0;
  const int ntx = (L.Nx + kDmTile - 1) / kDmTile;
  const int nt = dm_tiles(L);
  auto inside = [&](int j, int i) { return j >= 0 && j < L.Ny && i >= 0 && i < L.Nx; };
  for (int t = blockIdx.x; t < nt; t += gridDim.x) {
    const int y0 = (t / ntx) * kDmTile, x0 = (t % ntx) * kDmTile;
    double va[(NA + 255) / 256], vr[(NB + 255) / 256];
#pragma unroll
    for (int q = 0; q < (NA + 255) / 256; ++q) {
      const int k = threadIdx.x + 256 * q;
      const int ly = k / kDmTA, lx = k - ly * kDmTA;
      const int j = y0 - 4 + ly, i = x0 - 4 + lx;
      va[q] = (k < NA && inside(j, i)) ? src[dm_at(L, j, i)] : 0.0;
      if (prolong && k < NA && inside(j, i)) va[q] += dm_prolong_at(C, C.psi, j, i);
    }
#pragma unroll
    for (int q = 0; q < (NB + 255) / 256; ++q) {
      const int k = threadIdx.x + 256 * q;
      const int ly = k / kDmTB, lx = k - ly * kDmTB;
      const int j = y0 - 2 + ly, i = x0 - 2 + lx;
      vr[q] = (k < NB && inside(j, i)) ? L.rhs[dm_at(L, j, i)] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < (NA + 255) / 256; ++q) {
      const int k = threadIdx.x + 256 * q;
      if (k < NA) a[k] = va[q];
    }
#pragma unroll
    for (int q = 0; q < (NB + 255) / 256; ++q) {
      const int k = threadIdx.x + 256 * q;
      if (k < NB) r[k] = vr[q];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < (NB + 255) / 256; ++q) {
      const int k = threadIdx.x + 256 * q;
      if (k < NB) {
        const int ly = k / kDmTB, lx = k - ly * kDmTB;
        const int j = y0 - 2 + ly, i = x0 - 2 + lx;
        double v = 0.0;
        if (inside(j, i)) v = a[(ly + 2) * kDmTA + (lx + 2)] - s * (r[k] - dm_lap(a, kDmTA, ly, lx, L.h));
        b[k] = v;
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < (NT + 255) / 256; ++q) {
      const int k = threadIdx.x + 256 * q;
      const int ly = k / kDmTile, lx = k - ly * kDmTile;
      const int j = y0 + ly, i = x0 + lx;
      if (k < NT && inside(j, i)) {
        const int o = (ly + 2) * kDmTB + (lx + 2);
        dst[dm_at(L, j, i)] = b[o] - s * (r[o] - dm_lap(b, kDmTB, ly, lx, L.h));
      }
    }
    __syncthreads();
  }
}

// Coarse rhs = P^T (rhs - Laplace_h psi) / 4 on a tile of coarse sites, with the
// fine residuals it needs formed once in LDS (zero outside the fine interior,
// where the restriction gives them no weight); coarse psi = 0.
__global__ void __launch_bounds__(256) dm_restrict_res(DmLevel F, const double* __restrict__ psi, DmLevel C,
                                                       const DevStatus* st) {
  if (dm_skip(st)) return;
  constexpr int NP = kDmRP * kDmRP, NR = kDmRF * kDmRF, NC = kDmCT * kDmCT;
  __shared__ double x[NP];
  __shared__ double res[NR];
  const int ntx = (C.Nx + kDmCT - 1) / kDmCT;
  const int nt = dm_rtiles(C);
  auto inside = [&](int j, int i) { return j >= 0 && j < F.Ny && i >= 0 && i < F.Nx; };
  for (int t = blockIdx.x; t < nt; t += gridDim.x) {
    const int Y0 = (t / ntx) * kDmCT, X0 = (t % ntx) * kDmCT;
    // fine residual rows and columns 2*Y0 - 1 .. 2*Y0 + 2*kDmCT
    const int fy0 = 2 * Y0 - 1, fx0 = 2 * X0 - 1;
    double vx[(NP + 255) / 256], vb[(NR + 255) / 256];
#pragma unroll
    for (int q = 0; q < (NP + 255) / 256; ++q) {
      const int k = threadIdx.x + 256 * q;
      const int ly = k / kDmRP, lx = k - ly * kDmRP;
      const int j = fy0 - 2 + ly, i = fx0 - 2 + lx;
      vx[q] = (k < NP && inside(j, i)) ? psi[dm_at(F, j, i)] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < (NR + 255) / 256; ++q) {
      const int k = threadIdx.x + 256 * q;
      const int ly = k / kDmRF, lx = k - ly * kDmRF;
      const int j = fy0 + ly, i = fx0 + lx;
      vb[q] = (k < NR && inside(j, i)) ? F.rhs[dm_at(F, j, i)] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < (NP + 255) / 256; ++q) {
      const int k = threadIdx.x + 256 * q;
      if (k < NP) x[k] = vx[q];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < (NR + 255) / 256; ++q) {
      const int k = threadIdx.x + 256 * q;
      if (k < NR) {
        const int ly = k / kDmRF, lx = k - ly * kDmRF;
        res[k] = inside(fy0 + ly, fx0 + lx) ? vb[q] - dm_lap(x, kDmRP, ly, lx, F.h) : 0.0;
      }
    }
    __syncthreads();
    if (threadIdx.x < NC) {
      const int cy = threadIdx.x / kDmCT, cx = threadIdx.x - cy * kDmCT;
      const int J = Y0 + cy, I = X0 + cx;
      if (J < C.Ny && I < C.Nx) {
        double acc = 0.0;
        for (int j = max(2 * J - 1, 0); j <= min(2 * J + 2, F.Ny - 1); ++j) {
          double row = 0.0;
          for (int i = max(2 * I - 1, 0); i <= min(2 * I + 2, F.Nx - 1); ++i)
            row += dm_w(i, I) * res[(j - fy0) * kDmRF + (i - fx0)];
          acc += dm_w(j, J) * row;
        }
        const long o = dm_at(C, J, I);
        C.rhs[o] = 0.25 * acc;
        C.psi[o] = 0.0;
      }
    }
    __syncthreads();
  }
}

// Start of a solve for the stage point S (C planes in the flow's layout):
// r = b - A x with b = -(d_x S_1 + d_y S_2) and A = -Laplace_h, then the
// V-cycle's input on level 0: rhs = -r, psi = 0 (it solves Laplace_h z = -r).
template <class T>
__global__ void __launch_bounds__(256) dm_begin(Bufs<T> B, const T* __restrict__ S, DmLevel L0, DmVecs D,
                                                const DevStatus* st) {
  if (dm_skip(st)) return;
  const double c1 = 1.0 / (12.0 * L0.h);
  const long p = B.pitch;
  DM_SITES(L0) {
    const int j = (int)(k_ / L0.Nx), i = (int)(k_ - (long)j * L0.Nx);
    const T* s1 = S + (long)(j + 2) * p + (i + 2);
    const T* s2 = s1 + B.plane;
    const double dx = c1 * (((double)s1[-2] - (double)s1[2]) + 8.0 * ((double)s1[1] - (double)s1[-1]));
    const double dy = c1 * (((double)s2[-2 * p] - (double)s2[2 * p]) + 8.0 * ((double)s2[p] - (double)s2[-p]));
    const long o = dm_at(L0, j, i);
    const double r = -(dx + dy) + dm_lap(D.x, L0.pitch, j, i, L0.h);
    D.r[o] = r;
    L0.rhs[o] = -r;
    L0.psi[o] = 0.0;
  }
}

// Sum of 256 threads' values in a fixed order; valid in thread 0.
__device__ __forceinline__ double dm_block_sum(double v, double* red) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return red[0] + red[1] + red[2] + red[3];
}

// part[block] = sum over the block's sites of a . b (level-0 planes)
__global__ void __launch_bounds__(256) dm_dot(DmLevel L0, const double* __restrict__ a, const double* __restrict__ b,
                                              double* __restrict__ part, const DevStatus* st) {
  if (dm_skip(st)) return;
  __shared__ double red[4];
  double acc = 0.0;
  DM_SITES(L0) {
    const int j = (int)(k_ / L0.Nx), i = (int)(k_ - (long)j * L0.Nx);
    const long o = dm_at(L0, j, i);
    acc += a[o] * b[o];
  }
  const double s = dm_block_sum(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// d = z (first iteration) or z + beta d, with beta = r.z / (r.z of the last
// iteration) (0 on the first iteration or once that is 0). Every workgroup sums
// the r.z partials itself, in the same fixed order, so no launch of its own is
// needed for the scalar.
__global__ void __launch_bounds__(256) dm_dir(DmLevel L0, DmVecs D, int first, const DevStatus* st) {
  if (dm_skip(st)) return;
  __shared__ double red[4];
  const double rz = dm_block_sum(D.part[threadIdx.x], red);  // kDmRedGroups == 256 partials
  const double beta = (first || D.sc[0] == 0.0) ? 0.0 : rz / D.sc[0];
  if (blockIdx.x == 0 && threadIdx.x == 0) D.sc[1] = beta;
  DM_SITES(L0) {
    const int j = (int)(k_ / L0.Nx), i = (int)(k_ - (long)j * L0.Nx);
    const long o = dm_at(L0, j, i);
    D.d[o] = first ? L0.psi[o] : L0.psi[o] + beta * D.d[o];
  }
}

// Ad = -Laplace_h d and pmv[block] = sum of d . Ad over the block's sites
__global__ void __launch_bounds__(256) dm_matvec(DmLevel L0, DmVecs D, const DevStatus* st) {
  if (dm_skip(st)) return;
  __shared__ double red[4];
  double acc = 0.0;
  DM_SITES(L0) {
    const int j = (int)(k_ / L0.Nx), i = (int)(k_ - (long)j * L0.Nx);
    const long o = dm_at(L0, j, i);
    const double ad = -dm_lap(D.d, L0.pitch, j, i, L0.h);
    D.Ad[o] = ad;
    acc += D.d[o] * ad;
  }
  const double s = dm_block_sum(acc, red);
  if (threadIdx.x == 0) D.pmv[blockIdx.x] = s;
}

// alpha = r.z / d.Ad (0 once d.Ad is 0: the residual has vanished), summed by
// every workgroup from the partials in fixed order; then x += alpha d,
// r -= alpha Ad, and the next V-cycle's input (rhs = -r, psi = 0). Workgroup 0
// keeps r.z for the next iteration's beta.
__global__ void __launch_bounds__(256) dm_update(DmLevel L0, DmVecs D, const DevStatus* st) {
  if (dm_skip(st)) return;
  __shared__ double red[4], red2[4];
  const double rz = dm_block_sum(D.part[threadIdx.x], red);
  const double dad = dm_block_sum(D.pmv[threadIdx.x], red2);
  const double alpha = dad > 0.0 ? rz / dad : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    D.sc[0] = rz;
    D.sc[2] = alpha;
    D.sc[3] = dad;
  }
  DM_SITES(L0) {
    const int j = (int)(k_ / L0.Nx), i = (int)(k_ - (long)j * L0.Nx);
    const long o = dm_at(L0, j, i);
    D.x[o] += alpha * D.d[o];
    const double r = D.r[o] - alpha * D.Ad[o];
    D.r[o] = r;
    L0.rhs[o] = -r;
    L0.psi[o] = 0.0;
  }
}

// The stage point a pass evaluates, formed as the pass forms it (phi + cv v + ca a,
// put on the unit sphere at interior sites when the pass moves the field), over
// the whole padded lattice, into `out` (the flow's layout). For an evaluation the
// field is `src` or, when that is null, the current field. Skipped once a flow
// has stopped, as the pass itself is.
template <class T, int PASS>
__global__ void __launch_bounds__(256) dm_stage_point(Bufs<T> B, Coeffs cf, const DevStatus* st,
                                                      const T* __restrict__ src, T* __restrict__ out) {
  if (PASS != kEval && st->done) return;
  constexpr bool ONEPASS = advances_first(PASS);
  constexpr bool STAGED = staged(PASS);
  constexpr bool WITH_V = stage_reads_v(PASS);
  constexpr bool WITH_A = stage_reads_a(PASS);
  constexpr bool AFTER_P1 = (PASS == kP2 || PASS == kP3 || PASS == kP4);
  const long long step = st->step;
  const int cur = AFTER_P1 ? int((step - 1) & 1) : int(step & 1);
  const bool arrest = uses_arrest(PASS) ? (st->arrest != 0) : false;
  const T dt = (T)cf.dt;
  T cv, ca;
  stage_coeffs<T, PASS>(dt, arrest, cv, ca);
  const T* __restrict__ ph = (PASS == kEval && src != nullptr) ? src : (cur ? B.phi[1] : B.phi[0]);
  const T* __restrict__ vv = cur ? B.vel[1] : B.vel[0];
  const T* __restrict__ aa = ONEPASS ? (cur ? B.a2 : B.a1) : (PASS == kP3) ? B.a1 : B.a2;
  const long W = B.Nx + 4, H = B.Ny + 4;
  for (long k = blockIdx.x * 256L + threadIdx.x; k < W * H; k += (long)gridDim.x * 256L) {
    const int jj = (int)(k / W), ii = (int)(k - (long)jj * W);
    const long o = (long)jj * B.pitch + ii;
    T S[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      T x = ph[c * B.plane + o];
      if (STAGED) {
        if (WITH_V) x += cv * vv[c * B.plane + o];
        if (WITH_A) x += ca * aa[c * B.plane + o];
      }
      S[c] = x;
    }
    if (STAGED && ii >= 2 && ii < B.Nx + 2 && jj >= 2 && jj < B.Ny + 2) {
      const T inv = T(1) / sqrt(S[0] * S[0] + S[1] * S[1] + S[2] * S[2]);
#pragma unroll
      for (int c = 0; c < 3; ++c) S[c] *= inv;
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) out[c * B.plane + o] = S[c];
  }
}

// Zero-fill of n doubles (the hierarchy's planes at set-up, and the potential
// when a new field is set).
__global__ void __launch_bounds__(256) dm_fill_zero(double* p, long n) {
  for (long k = blockIdx.x * 256L + threadIdx.x; k < n; k += (long)gridDim.x * 256L) p[k] = 0.0;
}

#undef DM_SITES

}  // namespace ss
