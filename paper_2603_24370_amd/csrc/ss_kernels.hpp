// HIP kernels of the arrested-Newton-flow hot path (gfx950).
//
// One RK4 step (eq. (3), classical RK4 on (phi, phidot), dt = C h) is four
// launches of stage_pass<..., P1..P4> (or P1 and stage_pass_fused, which does
// P2..P4 in one launch). Each launch stages the stage point
// S = phi + c_v v + c_a a of a (TX + 4) x (TY + 4) tile (halo 2, Sec. 3.1) in
// LDS, evaluates the Euler-Lagrange gradient with eq. (1)-(2) from LDS, and
// writes only what the next pass needs:
//   P1: S = phi                                  -> a1 = -G(S), E_h(phi), arrest test
//   P2: S = phi + dt/2 v                         -> a2 = -G(S)
//   P3: S = phi + dt/2 v + dt^2/4 a1             -> q  = a1 + 2 a2 + 2 a3
//   P4: S = phi + dt v + dt^2/2 a2               -> phi' = phi + dt v + dt^2/12 (q + a1)
//                                                   v'   = v + dt/6 (q + a4)
// (v is replaced by 0 once the arrest test of P1 fired, eq. (4)). For the
// chiral magnet every stage point is put back on the unit sphere and G is
// projected on its tangent plane; phi' is renormalised and v' projected.
// P1 also reduces E_h (FP64 from the stored values), max |G| and a non-finite
// count to one partial per workgroup; pass_finalise, launched after it, sums
// the partials in a fixed order, applies the arrest test E > E_prev (strict)
// and the stop rules, and advances the step counter, all on the device.
#pragma once

#include "ss_internal.hpp"
#include "ss_theory.hpp"

namespace ss {

template <int TH>
struct NComp;
template <>
struct NComp<0> { static constexpr int value = 4; };
template <>
struct NComp<1> { static constexpr int value = 3; };
template <>
struct NComp<2> { static constexpr int value = 3; };

// Jets of one component for RY consecutive rows of one LDS column (rows
// ly0 .. ly0 + RY - 1, column lx), by eq. (1) and eq. (2); the mixed derivative
// applies eq. (1) along y to the eq. (1) x-stencil sums of the rows around.
// The y-neighbours are read once per column, the x-stencil of a row is shared
// by D_x, D_xx and the mixed derivative. If E64, the first derivatives are
// also formed in FP64 from the same stored values (for the energy density).
template <class T, int LX, int RY, bool MIXED, bool E64>
__device__ __forceinline__ void column_jets(const T* __restrict__ s, int lx, int ly0, T c1, T c2, double d1,
                                            Jet<T> (&J)[RY], double (&ex)[RY], double (&ey)[RY]) {
  T col[RY + 4];
#pragma unroll
  for (int k = 0; k < RY + 4; ++k) col[k] = s[(ly0 - 2 + k) * LX + lx];
  constexpr int K0 = MIXED ? 0 : 2, K1 = MIXED ? RY + 4 : RY + 2;
  T ddx[RY + 4];
#pragma unroll
  for (int k = K0; k < K1; ++k) {
    const T* r = s + (ly0 - 2 + k) * LX + lx;
    const T xm2 = r[-2], xm1 = r[-1], xp1 = r[1], xp2 = r[2];
    ddx[k] = (xm2 - xp2) + T(8) * (xp1 - xm1);
    if (k >= 2 && k < RY + 2) {
      J[k - 2].xx = c2 * (T(16) * (xp1 + xm1) - (xp2 + xm2) - T(30) * col[k]);
      if (E64) ex[k - 2] = d1 * (((double)xm2 - (double)xp2) + 8.0 * ((double)xp1 - (double)xm1));
    }
  }
#pragma unroll
  for (int r = 0; r < RY; ++r) {
    const int k = r + 2;
    J[r].f = col[k];
    J[r].x = c1 * ddx[k];
    J[r].y = c1 * ((col[k - 2] - col[k + 2]) + T(8) * (col[k + 1] - col[k - 1]));
    J[r].yy = c2 * (T(16) * (col[k + 1] + col[k - 1]) - (col[k + 2] + col[k - 2]) - T(30) * col[k]);
    if (MIXED) J[r].xy = c1 * c1 * ((ddx[k - 2] - ddx[k + 2]) + T(8) * (ddx[k + 1] - ddx[k - 1]));
    else J[r].xy = T(0);
    if (E64)
      ey[r] = d1 * (((double)col[k - 2] - (double)col[k + 2]) + 8.0 * ((double)col[k + 1] - (double)col[k - 1]));
  }
}

template <class T>
struct PassArgs {
  Bufs<T> B;
  Coeffs cf;
  DevStatus* st;
  double* partials;
  const T* src;  // kEval: field to evaluate in the internal layout (nullptr = current field)
  T* out;        // kEval: gradient output in the caller's layout (nullptr = none)
  long out_pitch, out_plane;
  int ntx, nty;  // tiles along x and y
  int seg;       // tiles per work unit: a unit is `seg` tiles stacked along y
};

// Tile traversal of the persistent stage launches. Work units are columns of
// `seg` tiles stacked along y, numbered row-major over (unit row, tile column).
// XCD x (workgroups b with b % 8 == x) owns the contiguous unit range
// [x * per, (x + 1) * per); its m = gridDim.x / 8 workgroups take units
// x*per + q, + m, ... (q = b / 8). Workgroups resident together on an XCD thus
// hold horizontally adjacent units (shared x-halo lines in that XCD's L2), and
// each walks its unit from top to bottom, so a tile's top halo rows are the
// rows its workgroup read for the previous tile.
template <class F>
__device__ __forceinline__ void for_each_tile(int ntx, int nty, int seg, F&& body) {
  const int nseg = (nty + seg - 1) / seg;
  const int nunits = ntx * nseg;
  const int m = gridDim.x >> 3, xcd = blockIdx.x & 7, q = blockIdx.x >> 3;
  const int per = (nunits + 7) >> 3;
  const int uend = min(nunits, (xcd + 1) * per);
  for (int u = xcd * per + q; u < uend; u += m) {
    const int sg = u / ntx, tx = u - sg * ntx;
    const int ty1 = min(nty, (sg + 1) * seg);
    for (int ty = sg * seg; ty < ty1; ++ty) body(tx, ty, ty - sg * seg, ty + 1 < ty1);
  }
}

template <class T>
struct Vec16;
template <>
struct Vec16<float> { typedef float4 type; static constexpr int n = 4; };
template <>
struct Vec16<double> { typedef double2 type; static constexpr int n = 2; };

template <class T>
__device__ __forceinline__ void vload(const T* p, T (&x)[16 / sizeof(T)]) {
  typedef typename Vec16<T>::type V;
  const V v = *reinterpret_cast<const V*>(p);
  if constexpr (sizeof(T) == 4) { x[0] = v.x; x[1] = v.y; x[2] = v.z; x[3] = v.w; }
  else { x[0] = v.x; x[1] = v.y; }
}

template <class T>
__device__ __forceinline__ void vstore_lds(T* p, const T (&x)[16 / sizeof(T)]) {
  typedef typename Vec16<T>::type V;
  V v;
  if constexpr (sizeof(T) == 4) { v.x = x[0]; v.y = x[1]; v.z = x[2]; v.w = x[3]; }
  else { v.x = x[0]; v.y = x[1]; }
  *reinterpret_cast<V*>(p) = v;
}

// eq. (1) gradient of the demagnetising potential at interior site (gi, gj) of a
// padded FP64 plane of row length pp (zero outside the interior); d1 = 1/(12h).
__device__ __forceinline__ void psi_gradient(const double* __restrict__ psi, long pp, int gi, int gj, double d1,
                                             double& gx, double& gy) {
  const double* c = psi + (long)(gj + 2) * pp + (gi + 2);
  gx = d1 * ((c[-2] - c[2]) + 8.0 * (c[1] - c[-1]));
  gy = d1 * ((c[-2 * pp] - c[2 * pp]) + 8.0 * (c[pp] - c[-pp]));
}

// One lattice as the stage passes see it (single context or one batch member).
template <class T>
struct InstView {
  T* phi[2];
  T* vel[2];
  T* a1;
  T* a2;
  T* q;
  long pitch, plane;
  int Nx, Ny;
  double h, dt;
  double p[kNumParams];
  const double* psi;  // demagnetising potential of the stage point (null: none)
  long psi_pitch;
};

template <class T>
__device__ __forceinline__ InstView<T> view_of(const Bufs<T>& B, const Coeffs& cf) {
  InstView<T> V;
  V.phi[0] = B.phi[0]; V.phi[1] = B.phi[1];
  V.vel[0] = B.vel[0]; V.vel[1] = B.vel[1];
  V.a1 = B.a1; V.a2 = B.a2; V.q = B.q;
  V.pitch = B.pitch; V.plane = B.plane;
  V.Nx = B.Nx; V.Ny = B.Ny;
  V.h = cf.h; V.dt = cf.dt;
  for (int k = 0; k < kNumParams; ++k) V.p[k] = cf.p[k];
  V.psi = B.psi;
  V.psi_pitch = B.psi_pitch;
  return V;
}

// Epilogue of the one-pass integrators at one site: the stage point S is the new
// field phi' (normalised for the chiral magnet). Stores phi', its force
// a' = -G(phi') and, for velocity Verlet, v' = v + dt/2 (a + a'), with v = 0
// after an arrest and, for the chiral magnet, v' projected on the tangent plane
// at phi'. a is the current field's force, read by the pass.
// w = v0 + dt/2 a: the part of the stored-force velocity Verlet update known
// before the force at the new field (v0 = 0 after an arrest); formed when the
// inputs are read, so that a thread holds one value per component, not two.
template <class T>
__device__ __forceinline__ T vv_partial(bool arrest, T dt, T v, T a) {
  return (arrest ? T(0) : v) + (T(0.5) * dt) * a;
}

// Epilogue of a one-pass step at one site: S is the new field, G = G(S), and u
// the part of the new velocity known before G: the half-step velocity read by
// the kick-drift-kick step, or w = v0 + dt/2 a of the stored-force step. Both
// velocity Verlet forms take v' = u - dt/2 G (tangent to S for unit fields);
// kick-drift-kick writes the new field and u' = v' - dt/2 G, the stored-force
// form the new field, v' and the force -G, gradient flow the new field and -G.
template <class T, int TH, int PASS>
__device__ __forceinline__ void one_pass_epilogue(T dt, const T (&u)[4], const T (&S)[4], const T (&G)[4],
                                                  T* __restrict__ phn, T* __restrict__ vn, T* __restrict__ an,
                                                  long plane, long off) {
  constexpr int C = NComp<TH>::value;
  if (PASS == kVV || PASS == kVVA) {
    const T hd = T(0.5) * dt;
    T vnew[4];
#pragma unroll
    for (int c = 0; c < C; ++c) vnew[c] = u[c] - hd * G[c];
    if (unit_field(TH)) {
      const T vd = vnew[0] * S[0] + vnew[1] * S[1] + vnew[2] * S[2];
#pragma unroll
      for (int c = 0; c < 3; ++c) vnew[c] -= vd * S[c];
    }
#pragma unroll
    for (int c = 0; c < C; ++c) {
      __builtin_nontemporal_store(S[c], &phn[c * plane + off]);
      if (PASS == kVV) {
        __builtin_nontemporal_store(vnew[c] - hd * G[c], &vn[c * plane + off]);
      } else {
        __builtin_nontemporal_store(vnew[c], &vn[c * plane + off]);
        __builtin_nontemporal_store(-G[c], &an[c * plane + off]);
      }
    }
  } else {
#pragma unroll
    for (int c = 0; c < C; ++c) {
      __builtin_nontemporal_store(S[c], &phn[c * plane + off]);
      __builtin_nontemporal_store(-G[c], &an[c * plane + off]);
    }
  }
}

// Epilogue of a gradient-flow step at one site: phi' = phi - tau G(phi) with
// tau = dt^2/2, put on the unit sphere for unit fields, into the other buffer.
template <class T, int TH>
__device__ __forceinline__ void gd_epilogue(T dt, const T (&phi)[4], const T (&G)[4], T* __restrict__ phn,
                                            long plane, long off) {
  constexpr int C = NComp<TH>::value;
  const T tau = T(0.5) * dt * dt;
  T pn[4];
#pragma unroll
  for (int c = 0; c < C; ++c) pn[c] = phi[c] - tau * G[c];
  if (unit_field(TH)) {
    const T inv = T(1) / sqrt(pn[0] * pn[0] + pn[1] * pn[1] + pn[2] * pn[2]);
#pragma unroll
    for (int c = 0; c < 3; ++c) pn[c] *= inv;
  }
#pragma unroll
  for (int c = 0; c < C; ++c) __builtin_nontemporal_store(pn[c], &phn[c * plane + off]);
}

// Epilogue of the velocity Verlet passes around the steps at one site of the
// current field, whose velocity buffer vc is updated in place (G = G(phi)):
// start u = v - dt/2 G, restart u = -dt/2 G, end v = u + dt/2 G (0 after an
// arrest).
template <class T, int TH, int PASS>
__device__ __forceinline__ void vv_in_place_epilogue(T dt, bool arrest, const T (&G)[4], T* __restrict__ vc,
                                                     long plane, long off) {
  constexpr int C = NComp<TH>::value;
  const T hd = T(0.5) * dt;
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const long k = c * plane + off;
    T x;
    if (PASS == kVVStart) x = vc[k] - hd * G[c];
    else if (PASS == kVVRestart) x = -hd * G[c];
    else x = arrest ? T(0) : vc[k] + hd * G[c];
    vc[k] = x;
  }
}

// LDS of one tile of a stage pass, in elements of T: the stage point on the
// tile and its halo of 2 (C planes of LY x LX). The one-pass integrators (and
// velocity Verlet's passes around the steps) walk a unit's tiles downwards and
// carry the overlap from one tile to the next: the
// last four stage rows (C x 4 x LX), and for velocity Verlet the part of the
// new velocity known before the force (u, or w = v0 + dt/2 a) of the two bottom
// halo rows, which are the next tile's first own rows (2 parities x 2 rows x C x TX).
template <class T, int TH, int PASS, int TX, int TY>
struct TileLds {
  static constexpr int C = NComp<TH>::value;
  static constexpr int LX = TX + 4, LY = TY + 4;
  static constexpr bool CARRY = advances_first(PASS) || vv_in_place(PASS) || PASS == kGD;
  static constexpr int STAGE = C * LY * LX;
  static constexpr int ROWS = CARRY ? C * 4 * LX : 0;
  static constexpr int RAW = (PASS == kVV || PASS == kVVA) ? 2 * 2 * C * TX : 0;
  static constexpr int size = STAGE + ROWS + RAW;
};

// One tile of one pass. Thread (tx, ty) owns column tx and rows ty*RY ..
// ty*RY + RY - 1 of the tile: it loads those sites' raw inputs into registers
// (reused by the epilogue, so no array is read twice) and writes their stage
// point to LDS; the halo ring of the tile is loaded cooperatively. Reduction
// contributions (energy, max |G|, non-finite count) are added to the caller's
// accumulators. Ends with a barrier (LDS is reused by the next tile).
// k is the tile's place in its workgroup's walk down a unit (0 = the unit's top
// tile). For the one-pass passes (TileLds::CARRY) a tile with k > 0 takes the four stage
// rows it shares with the tile above, and the raw inputs of its first two own
// rows, from LDS (see TileLds) instead of reading them again: the values are
// the ones stage_at formed for the tile above, so the result is bitwise the
// same, and each array is read about once plus its x halo. more = another tile
// of the unit follows (only then is the overlap kept).
template <class T, int TH, int PASS, int TX, int TY, int RY>
__device__ __forceinline__ void tile_body(const InstView<T>& V, int cur, bool arrest, const T* __restrict__ src,
                                          T* __restrict__ out, long out_pitch, long out_plane, int x0, int y0, int k,
                                          bool more, T* __restrict__ lds, double& e_acc, double& g_acc, int& nf) {
  constexpr int C = NComp<TH>::value;
  constexpr int LX = TX + 4, LY = TY + 4;
  constexpr int NT = TX * (TY / RY);
  constexpr int NRING = 4 * LX + 4 * TY;
  typedef TileLds<T, TH, PASS, TX, TY> TL;
  constexpr bool CARRY = TL::CARRY;
  static_assert(TY >= 4, "a carried tile takes four rows from the one above");
  constexpr bool REDUCE = reduces(PASS);
  constexpr bool ONEPASS = advances_first(PASS);  // the stage point is the new field
  constexpr bool STAGED = staged(PASS);
  constexpr bool WITH_V = stage_reads_v(PASS);
  constexpr bool WITH_A = stage_reads_a(PASS);
  T* s[C];
#pragma unroll
  for (int c = 0; c < C; ++c) s[c] = lds + c * (LY * LX);

  const int Nx = V.Nx, Ny = V.Ny;
  const long pitch = V.pitch, plane = V.plane;
  // select ping-pong buffers without indexing V's arrays by a runtime value
  // (that would place V in private scratch memory)
  const T* __restrict__ ph = (PASS == kEval && src != nullptr) ? src : (cur ? V.phi[1] : V.phi[0]);
  const T* __restrict__ vv = cur ? V.vel[1] : V.vel[0];
  // force buffers: RK4 stages read a1 (P3) or a2 (P4); gradient flow reads the
  // current field's force from the buffer of the step's parity and writes the
  // new field's force to the other one
  const T* __restrict__ aa = ONEPASS ? (cur ? V.a2 : V.a1) : (PASS == kP3) ? V.a1 : V.a2;
  T* __restrict__ a_store = (PASS == kP1) ? V.a1 : (PASS == kPrime) ? (cur ? V.a2 : V.a1) : (cur ? V.a1 : V.a2);
  const T dt = (T)V.dt;
  T cv, ca;
  stage_coeffs<T, PASS>(dt, arrest, cv, ca);
  const double h = V.h;
  const T c1 = T(1.0 / (12.0 * h)), c2 = T(1.0 / (12.0 * h * h));
  const double d1 = 1.0 / (12.0 * h);
  const int tid = threadIdx.y * TX + threadIdx.x;
  const int lx = threadIdx.x + 2;
  // a 64-wide tile row is one wavefront, so the row index is wave-uniform and
  // can live in a scalar register
  const int wy = (TX == 64) ? __builtin_amdgcn_readfirstlane((int)threadIdx.y) : (int)threadIdx.y;
  const int ly0 = wy * RY + 2;
  const int gi = x0 + threadIdx.x;

  // Stage point of padded element (gi, gj) (interior coordinates) and its raw
  // inputs, in two halves, so that a thread can have the loads of all its own
  // rows in flight together. load_raw: the raw inputs (a row past the padded
  // lattice reads its last row instead; it is discarded below).
  auto load_raw = [&](int gi_, int gj_, T (&raw_p)[4], T (&raw_v)[4], T (&raw_a)[4]) {
    const long off = (long)(min(gj_, Ny + 1) + 2) * pitch + (gi_ + 2);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      raw_p[c] = raw_v[c] = raw_a[c] = T(0);
      if (c < C) {
        raw_p[c] = ph[c * plane + off];
        if (STAGED && WITH_V) raw_v[c] = vv[c * plane + off];
        if (STAGED && WITH_A) raw_a[c] = aa[c * plane + off];
      }
    }
  };
  // stage_of_raw: the stage point (zero past the padded lattice, raw inputs
  // too). Unit fields are normalised with the squared norm in a fixed fma
  // order: a site is formed by its own tile and again in its neighbours' halo
  // rings, and every copy must have the same bits.
  auto stage_of_raw = [&](int gi_, int gj_, T (&raw_p)[4], T (&raw_v)[4], T (&raw_a)[4], T (&S)[4]) {
#pragma unroll
    for (int c = 0; c < 4; ++c) S[c] = T(0);
    if (gj_ > Ny + 1) {
#pragma unroll
      for (int c = 0; c < 4; ++c) raw_p[c] = raw_v[c] = raw_a[c] = T(0);
      return;
    }
#pragma unroll
    for (int c = 0; c < C; ++c) {
      T x = raw_p[c];
      if (STAGED) {
        x = fma(cv, raw_v[c], x);
        if (WITH_A) x = fma(ca, raw_a[c], x);
      }
      S[c] = x;
    }
    if (unit_field(TH) && STAGED && gi_ >= 0 && gi_ < Nx && gj_ >= 0 && gj_ < Ny) {
      const T inv = T(1) / sqrt(fma(S[2], S[2], fma(S[1], S[1], S[0] * S[0])));
      S[0] *= inv;
      S[1] *= inv;
      S[2] *= inv;
    }
  };
  // Both halves at once (halo rings). Columns right of the padded lattice feed
  // only discarded sites. The flow's own rows are long enough to read them; an
  // evaluated field may come in a caller's tight layout (pitch Nx + 4), so
  // there they are not read.
  auto stage_at = [&](int gi_, int gj_, T (&raw_p)[4], T (&raw_v)[4], T (&raw_a)[4], T (&S)[4]) {
    if (gj_ > Ny + 1 || (PASS == kEval && gi_ > Nx + 1)) {
#pragma unroll
      for (int c = 0; c < 4; ++c) raw_p[c] = raw_v[c] = raw_a[c] = S[c] = T(0);
      return;
    }
    load_raw(gi_, gj_, raw_p, raw_v, raw_a);
    stage_of_raw(gi_, gj_, raw_p, raw_v, raw_a, S);
  };

  // ---- carried rows: stage rows 0-3 from the tile above
  T* __restrict__ cs = lds + TL::STAGE;  // C x 4 x LX
  T* __restrict__ cr = cs + TL::ROWS;    // [parity][row][C][TX]
  const bool carried = CARRY && k > 0;
  const int par = k & 1;
  if (carried) {
    for (int idx = tid; idx < C * 4 * LX; idx += NT) {
      const int c = idx / (4 * LX);
      s[c][idx - c * 4 * LX] = cs[idx];
    }
  }

  // ---- own sites: raw inputs kept in registers, stage point to LDS (and, for
  // the one-pass integrators, in registers: it is the new field that is stored)
  T rp[RY][4], rv[RY][4], ra[RY][4], so[RY][4];
  // an evaluated field may lack the columns right of the lattice, so its loads
  // keep stage_at's guard
  constexpr bool SPLIT = PASS != kEval;
  if (SPLIT) {
#pragma unroll
    for (int r = 0; r < RY; ++r)
      if (!(carried && ly0 + r < 4)) load_raw(gi, y0 + ly0 + r - 2, rp[r], rv[r], ra[r]);
  }
  // ---- halo ring of the tile: all of it, or for a carried tile the x halo of
  // rows 4 .. TY+1 and the two bottom rows
  const int nring = carried ? 2 * LX + 4 * (TY - 2) : NRING;
  for (int idx = tid; idx < nring; idx += NT) {
    int ly, lxr;
    if (carried) {
      if (idx < 2 * LX) {
        const int rr = idx / LX;
        ly = LY - 2 + rr;
        lxr = idx - rr * LX;
      } else {
        const int j = idx - 2 * LX;
        ly = 4 + (j >> 2);
        const int cc = j & 3;
        lxr = cc < 2 ? cc : LX - 4 + cc;
      }
    } else if (idx < 4 * LX) {
      const int rr = idx / LX;
      ly = rr < 2 ? rr : LY - 4 + rr;
      lxr = idx - rr * LX;
    } else {
      const int j = idx - 4 * LX;
      ly = 2 + (j >> 2);
      const int cc = j & 3;
      lxr = cc < 2 ? cc : LX - 4 + cc;
    }
    T d0[4], d1v[4], d2[4], S[4];
    stage_at(x0 - 2 + lxr, y0 - 2 + ly, d0, d1v, d2, S);
#pragma unroll
    for (int c = 0; c < C; ++c) s[c][ly * LX + lxr] = S[c];
    if ((PASS == kVV || PASS == kVVA) && more && ly >= LY - 2 && lxr >= 2 && lxr < LX - 2) {
      // the next tile's first own rows: keep their u (or w)
      T* __restrict__ q = cr + (par * 2 + (ly - (LY - 2))) * C * TX + (lxr - 2);
#pragma unroll
      for (int c = 0; c < C; ++c) q[c * TX] = PASS == kVV ? d1v[c] : vv_partial(arrest, dt, d1v[c], d2[c]);
    }
  }
  // ---- own sites' stage points (their loads were issued before the ring's)
#pragma unroll
  for (int r = 0; r < RY; ++r) {
    const int ly = ly0 + r;
    if (carried && ly < 4) {
      const T* __restrict__ q = cr + ((par ^ 1) * 2 + (ly - 2)) * C * TX + threadIdx.x;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        rp[r][c] = rv[r][c] = ra[r][c] = so[r][c] = T(0);
        if (c < C) {
          so[r][c] = cs[(c * 4 + ly) * LX + lx];
          if (PASS == kVV || PASS == kVVA) rv[r][c] = q[c * TX];
        }
      }
    } else {
      if (SPLIT) stage_of_raw(gi, y0 + ly - 2, rp[r], rv[r], ra[r], so[r]);
      else stage_at(gi, y0 + ly - 2, rp[r], rv[r], ra[r], so[r]);
      // the stored-force step keeps w = v0 + dt/2 a in rv (the epilogue's u)
      if (PASS == kVVA) {
#pragma unroll
        for (int c = 0; c < 4; ++c) rv[r][c] = vv_partial(arrest, dt, rv[r][c], ra[r][c]);
      }
#pragma unroll
      for (int c = 0; c < C; ++c) s[c][ly * LX + lx] = so[r][c];
    }
  }
  __syncthreads();
  if (CARRY && more) {
    // stage rows TY .. TY+3 are the next tile's rows 0-3; saved before any
    // in-place change of the stage point below
    for (int idx = tid; idx < C * 4 * LX; idx += NT) {
      const int c = idx / (4 * LX);
      cs[idx] = s[c][(LY - 4) * LX + idx - c * 4 * LX];
    }
  }

  // E_h density in FP64 from the stored (unnormalised) values in LDS, own sites
  auto energy_density = [&]() {
    double ex[C][RY], ey[C][RY];
    Jet<T> Jr[C][RY];
#pragma unroll
    for (int c = 0; c < C; ++c) column_jets<T, LX, RY, false, true>(s[c], lx, ly0, c1, c2, d1, Jr[c], ex[c], ey[c]);
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      const int gj = y0 + ly0 - 2 + r;
      if (gi < Nx && gj < Ny) {
        Jet<double> Jd[4];
#pragma unroll
        for (int c = 0; c < C; ++c) {
          Jd[c].f = (double)Jr[c][r].f;
          Jd[c].x = ex[c][r];
          Jd[c].y = ey[c][r];
          Jd[c].xx = Jd[c].yy = Jd[c].xy = 0.0;
        }
        double e = density<TH>(Jd, V.p);
        if (TH == kCM && V.psi != nullptr) {
          double px, py;
          psi_gradient(V.psi, V.psi_pitch, gi, gj, d1, px, py);
          e += 0.5 * V.p[5] * (px * px + py * py);
        }
        e_acc += e;
        if (!isfinite(e)) ++nf;
      }
    }
  };

  Jet<T> J[C][RY];
  {
    double dx_[C][RY], dy_[C][RY];
#pragma unroll
    for (int c = 0; c < C; ++c)
      column_jets<T, LX, RY, el_mixed(TH), false>(s[c], lx, ly0, c1, c2, d1, J[c], dx_[c], dy_[c]);
  }

  // The chiral magnet needs E_h before the stage point is normalised in LDS;
  // the Abelian Higgs energy is formed after the epilogue, so that the FP64
  // energy and the FP32 gradient do not hold registers at the same time.
  if (REDUCE) {
    if (unit_field(TH)) energy_density();
    if (unit_field(TH)) {
      // the flow evaluates G at the normalised field
      __syncthreads();
      for (int idx = tid; idx < LX * LY; idx += NT) {
        const int ly = idx / LX, lx2 = idx - ly * LX;
        const int gi2 = x0 - 2 + lx2, gj2 = y0 - 2 + ly;
        if (gi2 >= 0 && gi2 < Nx && gj2 >= 0 && gj2 < Ny) {
          const T n0 = s[0][idx], n1 = s[1][idx], n2 = s[2][idx];
          const T inv = T(1) / sqrt(n0 * n0 + n1 * n1 + n2 * n2);
          s[0][idx] = n0 * inv;
          s[1][idx] = n1 * inv;
          s[2][idx] = n2 * inv;
        }
      }
      __syncthreads();
      double dx_[C][RY], dy_[C][RY];
#pragma unroll
      for (int c = 0; c < C; ++c)
        column_jets<T, LX, RY, el_mixed(TH), false>(s[c], lx, ly0, c1, c2, d1, J[c], dx_[c], dy_[c]);
    }
  }

  // ---- gradient and pass epilogue. Outputs are streamed with non-temporal stores,
  // and arrays read only at a thread's own sites with non-temporal loads, so
  // that L2 keeps the staged arrays whose halo rows neighbouring tiles re-read.
  T* __restrict__ phn = cur ? V.phi[0] : V.phi[1];
  T* __restrict__ vn = cur ? V.vel[0] : V.vel[1];
  T* vcur = cur ? V.vel[1] : V.vel[0];  // the velocity Verlet passes around the steps
  // max |G| of the thread's sites in T (exact), folded into the FP64 accumulator once
  T gmx = T(0);
#pragma unroll
  for (int r = 0; r < RY; ++r) {
    const int gj = y0 + ly0 - 2 + r;
    if (gi >= Nx || gj >= Ny) continue;
    Jet<T> Js[4];
#pragma unroll
    for (int c = 0; c < C; ++c) Js[c] = J[c][r];
    T G[4];
    el_gradient<T, TH>(Js, V.p, G);
    if (TH == kCM && V.psi != nullptr) {
      // demagnetising force mu_d grad psi (Euler-Lagrange form)
      double px, py;
      psi_gradient(V.psi, V.psi_pitch, gi, gj, d1, px, py);
      G[0] += (T)(V.p[5] * px);
      G[1] += (T)(V.p[5] * py);
    }
    if (unit_field(TH)) {
      const T gn = G[0] * Js[0].f + G[1] * Js[1].f + G[2] * Js[2].f;
#pragma unroll
      for (int c = 0; c < 3; ++c) G[c] -= gn * Js[c].f;
    }
    const long off = (long)(gj + 2) * pitch + (gi + 2);
    if (REDUCE) {
#pragma unroll
      for (int c = 0; c < C; ++c) {
        gmx = fmax(gmx, fabs(G[c]));
        if (!isfinite(G[c])) ++nf;
      }
    }
    if (PASS == kP1 || PASS == kPrime) {
#pragma unroll
      for (int c = 0; c < C; ++c) __builtin_nontemporal_store(-G[c], &a_store[c * plane + off]);
    } else if (ONEPASS) {
      one_pass_epilogue<T, TH, PASS>(dt, rv[r], so[r], G, phn, vn, a_store, plane, off);
    } else if (vv_in_place(PASS)) {
      vv_in_place_epilogue<T, TH, PASS>(dt, arrest, G, vcur, plane, off);
    } else if (PASS == kGD) {
      gd_epilogue<T, TH>(dt, so[r], G, phn, plane, off);
    } else if (PASS == kEval) {
      if (out != nullptr) {
        const long o = (long)(gj + 2) * out_pitch + (gi + 2);
#pragma unroll
        for (int c = 0; c < C; ++c) out[c * out_plane + o] = G[c];
      }
    } else if (PASS == kP2) {
#pragma unroll
      for (int c = 0; c < C; ++c) __builtin_nontemporal_store(-G[c], &V.a2[c * plane + off]);
    } else if (PASS == kP3) {
      // q = a1 + 2 a2 + 2 a3; a1 (a raw stage input) is in registers
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const long k = c * plane + off;
        __builtin_nontemporal_store(ra[r][c] + T(2) * __builtin_nontemporal_load(&V.a2[k]) - T(2) * G[c], &V.q[k]);
      }
    } else if (PASS == kP4) {
      T pn[4], vnew[4];
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const long k = c * plane + off;
        const T v0 = arrest ? T(0) : rv[r][c];
        const T qq = __builtin_nontemporal_load(&V.q[k]);
        pn[c] = rp[r][c] + dt * v0 + (dt * dt / T(12)) * (qq + __builtin_nontemporal_load(&V.a1[k]));
        vnew[c] = v0 + (dt / T(6)) * (qq - G[c]);
      }
      if (unit_field(TH)) {
        const T inv = T(1) / sqrt(pn[0] * pn[0] + pn[1] * pn[1] + pn[2] * pn[2]);
#pragma unroll
        for (int c = 0; c < 3; ++c) pn[c] *= inv;
        const T vd = vnew[0] * pn[0] + vnew[1] * pn[1] + vnew[2] * pn[2];
#pragma unroll
        for (int c = 0; c < 3; ++c) vnew[c] -= vd * pn[c];
      }
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const long k = c * plane + off;
        __builtin_nontemporal_store(pn[c], &phn[k]);
        __builtin_nontemporal_store(vnew[c], &vn[k]);
      }
    }
  }
  if (REDUCE) g_acc = fmax(g_acc, (double)gmx);
  if (REDUCE && TH == 0) energy_density();
  __syncthreads();
}

// ------------------------------------------------- exact discrete gradient
// G = h^-2 dE_h/dphi for E_h = h^2 sum over interior sites of e(phi, D_x phi, D_y phi)
// with D of eq. (1). By the chain rule, G(k) = de/dphi(k) - sum_i D_i[F_i](k) with
// the fluxes F_i = de/d(D_i phi) set to zero outside the interior (the energy
// has no terms there; eq. (1) is antisymmetric). A tile of 64 x 16 sites stages
// the stage point with halo 4, forms the fluxes on the tile plus a ring of 2
// and then G on the tile. Fluxes (3 per direction):
//   Abelian Higgs  x: (P1, Q1, B)   y: (P2, Q2, B)     with D_k psi = P_k + i Q_k
//   chiral magnet  x: J D_x n + D (0, -n3, n2)   y: J D_y n + Dy (n3, 0, -n1)   (Dy = D bulk, -D Heusler)
constexpr int kExTX = 64, kExTY = 16, kExRY = 4;

template <class T, int LX>
__device__ __forceinline__ void lds_dxdy(const T* __restrict__ p, int ly, int lx, T c1, T& dx, T& dy) {
  const T* r = p + ly * LX + lx;
  dx = c1 * ((r[-2] - r[2]) + T(8) * (r[1] - r[-1]));
  dy = c1 * ((r[-2 * LX] - r[2 * LX]) + T(8) * (r[LX] - r[-LX]));
}

template <class T, int TH, int LX>
__device__ __forceinline__ void site_fluxes(T* const (&s)[4], int ly, int lx, T c1, const InstView<T>& V, bool xdir,
                                            T (&F)[3]) {
  if (TH == 0) {
    T dxp, dyp, dxq, dyq, dxa1, dya1, dxa2, dya2;
    lds_dxdy<T, LX>(s[0], ly, lx, c1, dxp, dyp);
    lds_dxdy<T, LX>(s[1], ly, lx, c1, dxq, dyq);
    lds_dxdy<T, LX>(s[2], ly, lx, c1, dxa1, dya1);
    lds_dxdy<T, LX>(s[3], ly, lx, c1, dxa2, dya2);
    const int o = ly * LX + lx;
    const T p = s[0][o], q = s[1][o], ax = s[2][o], ay = s[3][o];
    if (xdir) { F[0] = dxp + ax * q; F[1] = dxq - ax * p; }
    else { F[0] = dyp + ay * q; F[1] = dyq - ay * p; }
    F[2] = dxa2 - dya1;
  } else if (TH == kBS) {
    // F_x = u + kappa^2 w x (u x w) = u + kappa^2 (u |w|^2 - w (u.w)),
    // F_y = w + kappa^2 (u x w) x u = w + kappa^2 (w |u|^2 - u (u.w))
    const T k2 = (T)(V.p[0] * V.p[0]);
    T u[3], w[3];
    for (int c = 0; c < 3; ++c) lds_dxdy<T, LX>(s[c], ly, lx, c1, u[c], w[c]);
    const T uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2], ww = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
    const T uw = u[0] * w[0] + u[1] * w[1] + u[2] * w[2];
    for (int c = 0; c < 3; ++c)
      F[c] = xdir ? u[c] + k2 * (u[c] * ww - w[c] * uw) : w[c] + k2 * (w[c] * uu - u[c] * uw);
  } else {
    const T J = (T)V.p[0], Dm = (T)V.p[1], Dy = (T)V.p[4];
    const int o = ly * LX + lx;
    T d[3];
    for (int c = 0; c < 3; ++c) {
      T dx, dy;
      lds_dxdy<T, LX>(s[c], ly, lx, c1, dx, dy);
      d[c] = xdir ? dx : dy;
    }
    const T n0 = s[0][o], n1 = s[1][o], n2 = s[2][o];
    if (xdir) { F[0] = J * d[0]; F[1] = J * d[1] - Dm * n2; F[2] = J * d[2] + Dm * n1; }
    else { F[0] = J * d[0] + Dy * n2; F[1] = J * d[1]; F[2] = J * d[2] - Dy * n0; }
  }
}

template <class T, int TH, int PASS>
__device__ __forceinline__ void tile_body_exact(const InstView<T>& V, int cur, bool arrest, const T* __restrict__ src,
                                                T* __restrict__ out, long out_pitch, long out_plane, int x0, int y0,
                                                T* __restrict__ lds, double& e_acc, double& g_acc, int& nf) {
  constexpr int TX = kExTX, TY = kExTY, RY = kExRY, NT = TX * (TY / RY);
  constexpr int C = NComp<TH>::value;
  constexpr int LX = TX + 8, LY = TY + 8;
  constexpr int NRING = 8 * LX + 8 * TY;
  constexpr int FXW = TX + 4, NXF = TY * FXW, NYF = (TY + 4) * TX;
  constexpr int KX = (NXF + NT - 1) / NT, KY = (NYF + NT - 1) / NT;
  constexpr bool REDUCE = reduces(PASS);
  constexpr bool ONEPASS = advances_first(PASS);  // the stage point is the new field
  constexpr bool STAGED = staged(PASS);
  constexpr bool WITH_V = stage_reads_v(PASS);
  constexpr bool WITH_A = stage_reads_a(PASS);
  T* s[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) s[c] = lds + (c < C ? c : 0) * (LY * LX);
  T* fx = lds;             // [3][TY][FXW], written over the stage point after the flux phase
  T* fy = lds + 3 * NXF;   // [3][TY + 4][TX]

  const int Nx = V.Nx, Ny = V.Ny;
  const long pitch = V.pitch, plane = V.plane;
  const T* __restrict__ ph = (PASS == kEval && src != nullptr) ? src : (cur ? V.phi[1] : V.phi[0]);
  const T* __restrict__ vv = cur ? V.vel[1] : V.vel[0];
  // force buffers: RK4 stages read a1 (P3) or a2 (P4); gradient flow reads the
  // current field's force from the buffer of the step's parity and writes the
  // new field's force to the other one
  const T* __restrict__ aa = ONEPASS ? (cur ? V.a2 : V.a1) : (PASS == kP3) ? V.a1 : V.a2;
  T* __restrict__ a_store = (PASS == kP1) ? V.a1 : (PASS == kPrime) ? (cur ? V.a2 : V.a1) : (cur ? V.a1 : V.a2);
  const T dt = (T)V.dt;
  T cv, ca;
  stage_coeffs<T, PASS>(dt, arrest, cv, ca);
  const double h = V.h;
  const T c1 = T(1.0 / (12.0 * h));
  const double d1 = 1.0 / (12.0 * h);
  const int tid = threadIdx.y * TX + threadIdx.x;
  // a 64-wide tile row is one wavefront: its row index is wave-uniform
  const int wy = (TX == 64) ? __builtin_amdgcn_readfirstlane((int)threadIdx.y) : (int)threadIdx.y;
  const int gi = x0 + threadIdx.x;

  auto stage_at = [&](int gi_, int gj_, T (&raw_p)[4], T (&raw_v)[4], T (&raw_a)[4], T (&S)[4]) {
#pragma unroll
    for (int c = 0; c < 4; ++c) raw_p[c] = raw_v[c] = raw_a[c] = S[c] = T(0);
    if (gj_ < -2 || gj_ > Ny + 1 || gi_ < -2 || gi_ > Nx + 1) return;
    const long off = (long)(gj_ + 2) * pitch + (gi_ + 2);
#pragma unroll
    for (int c = 0; c < C; ++c) {
      raw_p[c] = ph[c * plane + off];
      T x = raw_p[c];
      if (STAGED) {
        if (WITH_V) raw_v[c] = vv[c * plane + off];
        x += cv * raw_v[c];
        if (WITH_A) {
          raw_a[c] = aa[c * plane + off];
          x += ca * raw_a[c];
        }
      }
      S[c] = x;
    }
    if (unit_field(TH) && STAGED && gi_ >= 0 && gi_ < Nx && gj_ >= 0 && gj_ < Ny) {
      const T inv = T(1) / sqrt(S[0] * S[0] + S[1] * S[1] + S[2] * S[2]);
      S[0] *= inv;
      S[1] *= inv;
      S[2] *= inv;
    }
  };

  // ---- stage: own sites (raw inputs and stage point kept), then the halo-4 frame
  T rp[RY][4], rv[RY][4], ra[RY][4], so[RY][4];
#pragma unroll
  for (int r = 0; r < RY; ++r) {
    const int ly = 4 + wy * RY + r;
    stage_at(gi, y0 + ly - 4, rp[r], rv[r], ra[r], so[r]);
    // the stored-force step keeps w = v0 + dt/2 a in rv (the epilogue's u)
    if (PASS == kVVA) {
#pragma unroll
      for (int c = 0; c < 4; ++c) rv[r][c] = vv_partial(arrest, dt, rv[r][c], ra[r][c]);
    }
#pragma unroll
    for (int c = 0; c < C; ++c) s[c][ly * LX + 4 + threadIdx.x] = so[r][c];
  }
  for (int idx = tid; idx < NRING; idx += NT) {
    int ly, lx;
    if (idx < 8 * LX) {
      const int rr = idx / LX;
      ly = rr < 4 ? rr : LY - 8 + rr;
      lx = idx - rr * LX;
    } else {
      const int j = idx - 8 * LX;
      ly = 4 + (j >> 3);
      const int cc = j & 7;
      lx = cc < 4 ? cc : LX - 8 + cc;
    }
    T d0[4], d1v[4], d2[4], S[4];
    stage_at(x0 - 4 + lx, y0 - 4 + ly, d0, d1v, d2, S);
#pragma unroll
    for (int c = 0; c < C; ++c) s[c][ly * LX + lx] = S[c];
  }
  __syncthreads();

  // ---- energy density (FP64, stored values) and normalisation for the chiral magnet
  if (REDUCE) {
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      const int ly = 4 + wy * RY + r, lx = 4 + threadIdx.x;
      const int gj = y0 + ly - 4;
      if (gi < Nx && gj < Ny) {
        Jet<double> Jd[4];
#pragma unroll
        for (int c = 0; c < C; ++c) {
          const T* q = s[c] + ly * LX + lx;
          Jd[c].f = (double)q[0];
          Jd[c].x = d1 * (((double)q[-2] - (double)q[2]) + 8.0 * ((double)q[1] - (double)q[-1]));
          Jd[c].y = d1 * (((double)q[-2 * LX] - (double)q[2 * LX]) + 8.0 * ((double)q[LX] - (double)q[-LX]));
          Jd[c].xx = Jd[c].yy = Jd[c].xy = 0.0;
        }
        const double e = density<TH>(Jd, V.p);
        e_acc += e;
        if (!isfinite(e)) ++nf;
      }
    }
    if (unit_field(TH)) {
      __syncthreads();
      for (int idx = tid; idx < LX * LY; idx += NT) {
        const int ly = idx / LX, lx = idx - ly * LX;
        const int gi2 = x0 - 4 + lx, gj2 = y0 - 4 + ly;
        if (gi2 >= 0 && gi2 < Nx && gj2 >= 0 && gj2 < Ny) {
          const T n0 = s[0][idx], n1 = s[1][idx], n2 = s[2][idx];
          const T inv = T(1) / sqrt(n0 * n0 + n1 * n1 + n2 * n2);
          s[0][idx] = n0 * inv;
          s[1][idx] = n1 * inv;
          s[2][idx] = n2 * inv;
        }
      }
      __syncthreads();
    }
  }

  // ---- pointwise terms de/dphi at the own sites (and the stage point there)
  T g[RY][4], cen[RY][4];
#pragma unroll
  for (int r = 0; r < RY; ++r) {
    const int ly = 4 + wy * RY + r, lx = 4 + threadIdx.x;
    const int o = ly * LX + lx;
    T dx[4], dy[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) { cen[r][c] = T(0); dx[c] = dy[c] = T(0); g[r][c] = T(0); }
#pragma unroll
    for (int c = 0; c < C; ++c) {
      cen[r][c] = s[c][o];
      lds_dxdy<T, LX>(s[c], ly, lx, c1, dx[c], dy[c]);
    }
    if (TH == 0) {
      const T p = cen[r][0], q = cen[r][1], ax = cen[r][2], ay = cen[r][3];
      const T P1 = dx[0] + ax * q, Q1 = dx[1] - ax * p, P2 = dy[0] + ay * q, Q2 = dy[1] - ay * p;
      const T Wm = T(1) - (p * p + q * q);
      const T lam = (T)V.p[0];
      g[r][0] = -(ax * Q1 + ay * Q2) - T(0.5) * lam * Wm * p;
      g[r][1] = (ax * P1 + ay * P2) - T(0.5) * lam * Wm * q;
      g[r][2] = P1 * q - Q1 * p;
      g[r][3] = P2 * q - Q2 * p;
    } else if (TH == kBS) {
      g[r][2] = -(T)V.p[1];  // d/dm of mu^2 (1 - m_z); the other terms are fluxes
    } else {
      const T Dm = (T)V.p[1], K = (T)V.p[2], Bz = (T)V.p[3], Dy = (T)V.p[4];
      g[r][0] = -Dy * dy[2];
      g[r][1] = Dm * dx[2];
      g[r][2] = Dy * dy[0] - Dm * dx[1] - (T(2) * K * cen[r][2] + Bz);
    }
  }

  // ---- fluxes on the tile plus a ring of 2 (zero outside the interior), kept in
  // registers until every thread is done with the stage point
  T fxr[KX][3], fyr[KY][3];
#pragma unroll
  for (int k = 0; k < KX; ++k) {
    const int idx = tid + k * NT;
    fxr[k][0] = fxr[k][1] = fxr[k][2] = T(0);
    if (idx < NXF) {
      const int r = idx / FXW, cc = idx - r * FXW - 2;
      const int gi2 = x0 + cc, gj2 = y0 + r;
      if (gi2 >= 0 && gi2 < Nx && gj2 < Ny) site_fluxes<T, TH, LX>(s, r + 4, cc + 4, c1, V, true, fxr[k]);
    }
  }
#pragma unroll
  for (int k = 0; k < KY; ++k) {
    const int idx = tid + k * NT;
    fyr[k][0] = fyr[k][1] = fyr[k][2] = T(0);
    if (idx < NYF) {
      const int r = idx / TX - 2, cc = idx - (idx / TX) * TX;
      const int gi2 = x0 + cc, gj2 = y0 + r;
      if (gi2 < Nx && gj2 >= 0 && gj2 < Ny) site_fluxes<T, TH, LX>(s, r + 4, cc + 4, c1, V, false, fyr[k]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < KX; ++k) {
    const int idx = tid + k * NT;
    if (idx < NXF)
#pragma unroll
      for (int f = 0; f < 3; ++f) fx[f * NXF + idx] = fxr[k][f];
  }
#pragma unroll
  for (int k = 0; k < KY; ++k) {
    const int idx = tid + k * NT;
    if (idx < NYF)
#pragma unroll
      for (int f = 0; f < 3; ++f) fy[f * NYF + idx] = fyr[k][f];
  }
  __syncthreads();

  // ---- G = de/dphi - D_x F_x - D_y F_y, then the pass epilogue
  T* __restrict__ phn = cur ? V.phi[0] : V.phi[1];
  T* __restrict__ vn = cur ? V.vel[0] : V.vel[1];
  T* vcur = cur ? V.vel[1] : V.vel[0];  // the velocity Verlet passes around the steps
  // max |G| of the thread's sites in T (exact), folded into the FP64 accumulator once
  T gmx = T(0);
#pragma unroll
  for (int r = 0; r < RY; ++r) {
    const int tr = wy * RY + r;
    const int gj = y0 + tr;
    if (gi >= Nx || gj >= Ny) continue;
    T dfx[3], dfy[3];
#pragma unroll
    for (int f = 0; f < 3; ++f) {
      const T* px = fx + f * NXF + tr * FXW + threadIdx.x + 2;
      dfx[f] = c1 * ((px[-2] - px[2]) + T(8) * (px[1] - px[-1]));
      const T* py = fy + f * NYF + (tr + 2) * TX + threadIdx.x;
      dfy[f] = c1 * ((py[-2 * TX] - py[2 * TX]) + T(8) * (py[TX] - py[-TX]));
    }
    T G[4];
    if (TH == 0) {
      G[0] = g[r][0] - dfx[0] - dfy[0];
      G[1] = g[r][1] - dfx[1] - dfy[1];
      G[2] = g[r][2] + dfy[2];
      G[3] = g[r][3] - dfx[2];
    } else {
#pragma unroll
      for (int c = 0; c < 3; ++c) G[c] = g[r][c] - dfx[c] - dfy[c];
      const T gn = G[0] * cen[r][0] + G[1] * cen[r][1] + G[2] * cen[r][2];
#pragma unroll
      for (int c = 0; c < 3; ++c) G[c] -= gn * cen[r][c];
      G[3] = T(0);
    }
    const long off = (long)(gj + 2) * pitch + (gi + 2);
    if (REDUCE) {
#pragma unroll
      for (int c = 0; c < C; ++c) {
        gmx = fmax(gmx, fabs(G[c]));
        if (!isfinite(G[c])) ++nf;
      }
    }
    if (PASS == kP1 || PASS == kPrime) {
#pragma unroll
      for (int c = 0; c < C; ++c) __builtin_nontemporal_store(-G[c], &a_store[c * plane + off]);
    } else if (ONEPASS) {
      one_pass_epilogue<T, TH, PASS>(dt, rv[r], so[r], G, phn, vn, a_store, plane, off);
    } else if (vv_in_place(PASS)) {
      vv_in_place_epilogue<T, TH, PASS>(dt, arrest, G, vcur, plane, off);
    } else if (PASS == kGD) {
      gd_epilogue<T, TH>(dt, so[r], G, phn, plane, off);
    } else if (PASS == kEval) {
      if (out != nullptr) {
        const long o = (long)(gj + 2) * out_pitch + (gi + 2);
#pragma unroll
        for (int c = 0; c < C; ++c) out[c * out_plane + o] = G[c];
      }
    } else if (PASS == kP2) {
#pragma unroll
      for (int c = 0; c < C; ++c) __builtin_nontemporal_store(-G[c], &V.a2[c * plane + off]);
    } else if (PASS == kP3) {
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const long k = c * plane + off;
        __builtin_nontemporal_store(ra[r][c] + T(2) * __builtin_nontemporal_load(&V.a2[k]) - T(2) * G[c], &V.q[k]);
      }
    } else if (PASS == kP4) {
      T pn[4], vnew[4];
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const long k = c * plane + off;
        const T v0 = arrest ? T(0) : rv[r][c];
        const T qq = __builtin_nontemporal_load(&V.q[k]);
        pn[c] = rp[r][c] + dt * v0 + (dt * dt / T(12)) * (qq + __builtin_nontemporal_load(&V.a1[k]));
        vnew[c] = v0 + (dt / T(6)) * (qq - G[c]);
      }
      if (unit_field(TH)) {
        const T inv = T(1) / sqrt(pn[0] * pn[0] + pn[1] * pn[1] + pn[2] * pn[2]);
#pragma unroll
        for (int c = 0; c < 3; ++c) pn[c] *= inv;
        const T vd = vnew[0] * pn[0] + vnew[1] * pn[1] + vnew[2] * pn[2];
#pragma unroll
        for (int c = 0; c < 3; ++c) vnew[c] -= vd * pn[c];
      }
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const long k = c * plane + off;
        __builtin_nontemporal_store(pn[c], &phn[k]);
        __builtin_nontemporal_store(vnew[c], &vn[k]);
      }
    }
  }
  if (REDUCE) g_acc = fmax(g_acc, (double)gmx);
  __syncthreads();
}

// Status update after a reduction of one field (thread 0 of the finalising
// workgroup): arrest test E > E_prev (strict, eq. (4)), the stop rules when
// minimising, and the step counter (P1 only). E is already multiplied by h^2.
template <int PASS>
__device__ __forceinline__ void finalise_status(DevStatus* st, double E, double gmax, int nfin) {
  st->counter = 0u;
  if (PASS == kEval) {
    st->eval_E = E;
    st->eval_gmax = gmax;
    st->nonfinite = nfin;
    return;
  }
  // a one-pass step has written the new field: it becomes the current one, and
  // the tests below are those of the new field
  long long s0 = st->step;
  if (advances_first(PASS)) st->step = ++s0;
  // The first test of a run is of the field the last run ended on, whose arrest
  // that run decided (and applied), or of a fresh field (E_prev infinite): it
  // takes no new arrest decision and keeps the energy the next test compares
  // with, so a run split in two decides its arrests as one run does. (Its own
  // sum of the same field may differ in the last bits: another launch shape.)
  const bool retest = st->fresh != 0;
  st->fresh = 0;
  // gradient flow has no velocity, hence no arrest
  const int arr = (!no_arrest(PASS) && !retest && E > st->E_prev) ? 1 : 0;
  if (!retest) st->arrest = arr;
  if (arr) st->n_arrests += 1;
  if (!retest || !isfinite(st->E_prev)) st->E_prev = E;
  st->E = E;
  st->gmax = gmax;
  st->nonfinite = nfin;
  st->hist[s0 % kHistLen] = E;
  int done = 0;
  if (nfin > 0) {
    done = 4;
  } else if (st->minimise) {
    const int W = st->window;
    if (gmax < st->grad_tol) done = 1;
    else if (W > 0 && s0 >= W && fabs(E - st->hist[(s0 - W) % kHistLen]) <= st->rel_e_tol * fabs(E)) done = 2;
    else if (E <= st->e_target) done = 5;
    else if (s0 >= st->max_steps) done = 3;
  }
  if (done) st->done = done;
  else if (PASS == kP1 || PASS == kGD) st->step = s0 + 1;
}

// Launch: gridDim.x is a multiple of 8; tiles are assigned by for_each_tile.
// Each workgroup accumulates its tiles' reductions into one partial;
// pass_finalise sums the partials in a fixed order and updates the status.
// Waves per SIMD a stage pass is compiled for. The Abelian-Higgs one-pass
// integrators in FP32 on two-row tiles are held to 128 VGPRs (four waves; 160
// uncapped), so that two 512-thread workgroups share a CU, without spills; the
// chiral magnet and four-row tiles would spill under that cap, and the other
// passes fit it uncapped.
template <class T, int TH, int PASS, int RY>
struct StageWaves {
  static constexpr int value = (sizeof(T) == 4 && TH == 0 && RY == 2 && (advances_first(PASS) || PASS == kGD)) ? 4 : 1;
};

template <class T, int TH, int PASS, int TX, int TY, int RY>
__global__ void __launch_bounds__(TX*(TY / RY))
__attribute__((amdgpu_waves_per_eu(StageWaves<T, TH, PASS, RY>::value))) stage_pass(PassArgs<T> a) {
  constexpr int C = NComp<TH>::value;
  constexpr int LX = TX + 4, LY = TY + 4;
  constexpr int NT = TX * (TY / RY);
  constexpr bool REDUCE = reduces(PASS);
  // stages 2-4 of RK4 run after P1 advanced the step counter; the one-pass
  // integrators read the current field and advance it in their finalise
  constexpr bool AFTER_P1 = (PASS == kP2 || PASS == kP3 || PASS == kP4);
  __shared__ __align__(16) T lds[TileLds<T, TH, PASS, TX, TY>::size];
  __shared__ double red[3 * (NT / 64)];

  DevStatus* __restrict__ st = a.st;
  // a finished flow skips its remaining passes; velocity Verlet's end of run
  // converts the velocity whatever the status, and its restart runs only after
  // an arrest
  if (PASS != kEval && PASS != kVVEnd && st->done) return;
  if (PASS == kVVRestart && !st->arrest) return;
  const long long step = st->step;
  const int cur = AFTER_P1 ? int((step - 1) & 1) : int(step & 1);
  const bool arrest = uses_arrest(PASS) ? (st->arrest != 0) : false;
  const InstView<T> V = view_of<T>(a.B, a.cf);

  double e_acc = 0.0, g_acc = 0.0;
  int nf = 0;
  for_each_tile(a.ntx, a.nty, a.seg, [&](int tx, int ty, int k, bool more) {
    tile_body<T, TH, PASS, TX, TY, RY>(V, cur, arrest, a.src, a.out, a.out_pitch, a.out_plane, tx * TX, ty * TY, k,
                                       more, lds, e_acc, g_acc, nf);
  });
  if (!REDUCE) return;

  // ---- first level of the FP64 reduction: one partial per workgroup (the
  // second level is pass_finalise, launched after the pass)
  block_reduce3<NT>(e_acc, g_acc, nf, red);
  if (threadIdx.y * TX + threadIdx.x == 0) {
    double* p = a.partials + 4 * (long)blockIdx.x;
    p[0] = e_acc;
    p[1] = g_acc;
    p[2] = (double)nf;
  }
}

// Second level of a reducing pass (one workgroup of 256 threads): the nparts
// workgroup partials summed in workgroup order, then the status update. Being a
// launch of its own, it needs no fence or atomic inside the pass.
template <int PASS>
__global__ void __launch_bounds__(256) pass_finalise(DevStatus* st, const double* __restrict__ partials, int nparts,
                                                     double h) {
  if (PASS != kEval && st->done) return;
  double se = 0.0, sg = 0.0;
  int sn = 0;
  for (int k = threadIdx.x; k < nparts; k += 256) {
    const double* p = partials + 4 * (long)k;
    se += p[0];
    sg = fmax(sg, p[1]);
    sn += (int)p[2];
  }
  __shared__ double red[3 * 4];
  block_reduce3<256>(se, sg, sn, red);
  if (threadIdx.x == 0) finalise_status<PASS>(st, h * h * se, sg, sn);
}

// ------------------------------------------------- fused stages 2-4 (EL gradient)
// One pass computes stages 2, 3 and 4 of the step and the update, reading phi, v
// and a1 (written by P1) and writing phi', v':
//   S2 = phi + dt/2 v            a2 = -G(S2)     on the tile plus a ring of 2
//   S3 = S2 + dt^2/4 a1          a3 = -G(S3)     on the tile
//   S4 = phi + dt v + dt^2/2 a2  a4 = -G(S4)     on the tile
//   q = a1 + 2 a2 + 2 a3, phi' = phi + dt v + dt^2 (q + a1) / 12, v' = v + dt (q + a4) / 6
// (v -> 0 after an arrest; chiral magnet: stage points normalised, forces
// projected, phi' normalised and v' projected, as in the separate passes).
// a2 is needed at the halo of S4's stencil, so it is recomputed on a ring of 2
// around the tile from S2 staged with halo 4. Per site the pass reads 3 field
// sets and writes 2, against 10 and 4 for P2, P3 and P4 run separately.

// Jets of one site from an LDS plane with row length LX, arithmetic as column_jets.
template <class T, int LX, bool MIXED>
__device__ __forceinline__ void site_jet(const T* __restrict__ s, int ly, int lx, T c1, T c2, Jet<T>& J) {
  const T* r0 = s + ly * LX + lx;
  const T xm2 = r0[-2], xm1 = r0[-1], xp1 = r0[1], xp2 = r0[2], f = r0[0];
  const T ym2 = r0[-2 * LX], ym1 = r0[-LX], yp1 = r0[LX], yp2 = r0[2 * LX];
  J.f = f;
  J.x = c1 * ((xm2 - xp2) + T(8) * (xp1 - xm1));
  J.xx = c2 * (T(16) * (xp1 + xm1) - (xp2 + xm2) - T(30) * f);
  J.y = c1 * ((ym2 - yp2) + T(8) * (yp1 - ym1));
  J.yy = c2 * (T(16) * (yp1 + ym1) - (yp2 + ym2) - T(30) * f);
  if (MIXED) {
    T ddx[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      const T* r = s + (ly - 2 + k) * LX + lx;
      ddx[k] = (r[-2] - r[2]) + T(8) * (r[1] - r[-1]);
    }
    J.xy = c1 * c1 * ((ddx[0] - ddx[4]) + T(8) * (ddx[3] - ddx[1]));
  } else {
    J.xy = T(0);
  }
}

// G at one site from its jets (the chiral magnet's G is projected at the site).
template <class T, int TH>
__device__ __forceinline__ void site_gradient(const Jet<T> (&Js)[4], const InstView<T>& V, T (&G)[4]) {
  el_gradient<T, TH>(Js, V.p, G);
  if (unit_field(TH)) {
    const T gn = G[0] * Js[0].f + G[1] * Js[1].f + G[2] * Js[2].f;
#pragma unroll
    for (int c = 0; c < 3; ++c) G[c] -= gn * Js[c].f;
  }
}

template <class T>
__device__ __forceinline__ void unit3(T (&x)[4]) {
  const T inv = T(1) / sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
  x[0] *= inv;
  x[1] *= inv;
  x[2] *= inv;
}

template <class T, int TH, int TX, int TY, int RY>
__device__ __forceinline__ void tile_body_fused(const InstView<T>& V, int cur, bool arrest, int x0, int y0,
                                                T* __restrict__ lds) {
  constexpr int C = NComp<TH>::value;
  constexpr int AX = TX + 8, AY = TY + 8;   // A: S2 with halo 4, then S3 / S4 with halo 2
  constexpr int BX = TX + 4, BY = TY + 4;   // B-shaped planes (tile plus halo 2)
  constexpr int NA = AX * AY, NB = BX * BY;
  constexpr int NT = TX * (TY / RY);
  constexpr int NRB = NB - TX * TY;         // ring of B around the tile
  constexpr int KRB = (NRB + NT - 1) / NT;
  constexpr bool MIXED = el_mixed(TH);
  // LDS: A [C][AY][AX] | a2 [C][BY][BX] | phi [C][BY][BX] | v [C][BY][BX] | a1 [C][BY][BX]
  T* sa[4];
  T* s2[4];
  T* sp[4];
  T* sv[4];
  T* s1[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int cc = c < C ? c : 0;
    sa[c] = lds + cc * NA;
    s2[c] = lds + C * NA + cc * NB;
    sp[c] = lds + C * NA + C * NB + cc * NB;
    sv[c] = lds + C * NA + 2 * C * NB + cc * NB;
    s1[c] = lds + C * NA + 3 * C * NB + cc * NB;
  }
  const int Nx = V.Nx, Ny = V.Ny;
  const long pitch = V.pitch, plane = V.plane;
  const T* __restrict__ ph = cur ? V.phi[1] : V.phi[0];
  const T* __restrict__ vv = cur ? V.vel[1] : V.vel[0];
  const T* __restrict__ a1p = V.a1;
  const T dt = (T)V.dt;
  const T cv2 = arrest ? T(0) : T(0.5) * dt;
  const T cv4 = arrest ? T(0) : dt;
  const T ca3 = T(0.25) * dt * dt, ca4 = T(0.5) * dt * dt;
  const double h = V.h;
  const T c1 = T(1.0 / (12.0 * h)), c2 = T(1.0 / (12.0 * h * h));
  const int tid = threadIdx.y * TX + threadIdx.x;
  const int gi = x0 + threadIdx.x;
  // a 64-wide tile row is one wavefront: its row index is wave-uniform
  const int wy = (TX == 64) ? __builtin_amdgcn_readfirstlane((int)threadIdx.y) : (int)threadIdx.y;
  auto inside = [&](int x, int y) { return x >= 0 && x < Nx && y >= 0 && y < Ny; };
  // site (x, y) of the padded lattice (x, y in [-2, N + 1]) as an element offset
  auto offs = [&](int x, int y) { return (long)(y + 2) * pitch + (x + 2); };
  auto in_pad = [&](int x, int y) { return x >= -2 && x <= Nx + 1 && y >= -2 && y <= Ny + 1; };

  // ---- phase 1 (all global reads of the tile): phi, v on the tile plus halo 4,
  // S2 = phi + dt/2 v -> A; raw phi, v and a1 on the tile plus halo 2 -> LDS
  auto load_entry = [&](int idx) {
    const int ly = idx / AX, lx = idx - ly * AX;
    const int x = x0 - 4 + lx, y = y0 - 4 + ly;
    const bool inb = ly >= 2 && ly < AY - 2 && lx >= 2 && lx < AX - 2;
    const int ib = (ly - 2) * BX + (lx - 2);
    T P[4] = {T(0), T(0), T(0), T(0)}, W[4] = {T(0), T(0), T(0), T(0)}, S[4] = {T(0), T(0), T(0), T(0)};
    T A1[4] = {T(0), T(0), T(0), T(0)};
    if (in_pad(x, y)) {
      const long o = offs(x, y);
#pragma unroll
      for (int c = 0; c < C; ++c) {
        P[c] = ph[c * plane + o];
        W[c] = vv[c * plane + o];
        if (inb) A1[c] = a1p[c * plane + o];
        S[c] = P[c] + cv2 * W[c];
      }
      if (unit_field(TH) && inside(x, y)) unit3(S);
    }
#pragma unroll
    for (int c = 0; c < C; ++c) sa[c][idx] = S[c];
    if (inb) {
#pragma unroll
      for (int c = 0; c < C; ++c) {
        sp[c][ib] = P[c];
        sv[c][ib] = W[c];
        s1[c][ib] = A1[c];
      }
    }
  };
  // Tall tiles take one fully unrolled sweep (every load of the tile in flight
  // at once); 64 x 8 tiles schedule better with two sweeps in flight (measured).
  if constexpr (TY >= 16) {
    constexpr int KA = (NA + NT - 1) / NT;
#pragma unroll
    for (int k = 0; k < KA; ++k)
      if (tid + k * NT < NA) load_entry(tid + k * NT);
  } else {
#pragma unroll 2
    for (int idx = tid; idx < NA; idx += NT) load_entry(idx);
  }
  __syncthreads();

  // ---- phase 2: a2 = -G(S2) on the tile (column jets) and its ring (site jets); 0 off the interior
  {
    Jet<T> J[C][RY];
    double dx_[C][RY], dy_[C][RY];
#pragma unroll
    for (int c = 0; c < C; ++c)
      column_jets<T, AX, RY, MIXED, false>(sa[c], 4 + threadIdx.x, 4 + wy * RY, c1, c2, 0.0, J[c], dx_[c],
                                           dy_[c]);
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      Jet<T> Js[4];
#pragma unroll
      for (int c = 0; c < C; ++c) Js[c] = J[c][r];
      T G[4] = {T(0), T(0), T(0), T(0)};
      site_gradient<T, TH>(Js, V, G);
      const bool in = inside(gi, y0 + wy * RY + r);
      const int ib = (2 + wy * RY + r) * BX + 2 + threadIdx.x;
#pragma unroll
      for (int c = 0; c < C; ++c) s2[c][ib] = in ? -G[c] : T(0);
    }
  }
#pragma unroll
  for (int k = 0; k < KRB; ++k) {
    const int idx = tid + k * NT;
    if (idx < NRB) {
      int by, bx;
      if (idx < 4 * BX) {
        const int rr = idx / BX;
        by = rr < 2 ? rr : BY - 4 + rr;
        bx = idx - rr * BX;
      } else {
        const int j = idx - 4 * BX;
        by = 2 + (j >> 2);
        const int cc = j & 3;
        bx = cc < 2 ? cc : BX - 4 + cc;
      }
      T a[4] = {T(0), T(0), T(0), T(0)};
      if (inside(x0 - 2 + bx, y0 - 2 + by)) {
        Jet<T> Js[4];
#pragma unroll
        for (int c = 0; c < C; ++c) site_jet<T, AX, MIXED>(sa[c], by + 2, bx + 2, c1, c2, Js[c]);
        T G[4] = {T(0), T(0), T(0), T(0)};
        site_gradient<T, TH>(Js, V, G);
#pragma unroll
        for (int c = 0; c < C; ++c) a[c] = -G[c];
      }
#pragma unroll
      for (int c = 0; c < C; ++c) s2[c][by * BX + bx] = a[c];
    }
  }
  __syncthreads();

  // stage point on the tile plus halo 2 -> A (offset 2): phi + cv v + ca acc
  auto stage_b = [&](T cv, T ca, T* const (&acc)[4]) {
#pragma unroll 1
    for (int ib = tid; ib < NB; ib += NT) {
      const int by = ib / BX, bx = ib - by * BX;
      T S[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
      for (int c = 0; c < C; ++c) S[c] = sp[c][ib] + cv * sv[c][ib] + ca * acc[c][ib];
      if (unit_field(TH) && inside(x0 - 2 + bx, y0 - 2 + by)) unit3(S);
#pragma unroll
      for (int c = 0; c < C; ++c) sa[c][(by + 2) * AX + bx + 2] = S[c];
    }
  };

  // ---- phase 3: S3 = phi + dt/2 v + dt^2/4 a1
  stage_b(cv2, ca3, s1);
  __syncthreads();

  // ---- phase 4: q = a1 + 2 a2 - 2 G(S3) at the own sites
  T qo[RY][4];
  {
    Jet<T> J[C][RY];
    double dx_[C][RY], dy_[C][RY];
#pragma unroll
    for (int c = 0; c < C; ++c)
      column_jets<T, AX, RY, MIXED, false>(sa[c], 4 + threadIdx.x, 4 + wy * RY, c1, c2, 0.0, J[c], dx_[c],
                                           dy_[c]);
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      Jet<T> Js[4];
#pragma unroll
      for (int c = 0; c < C; ++c) Js[c] = J[c][r];
      T G[4] = {T(0), T(0), T(0), T(0)};
      site_gradient<T, TH>(Js, V, G);
      const int ib = (2 + wy * RY + r) * BX + 2 + threadIdx.x;
#pragma unroll
      for (int c = 0; c < 4; ++c) qo[r][c] = T(0);
#pragma unroll
      for (int c = 0; c < C; ++c) qo[r][c] = s1[c][ib] + T(2) * s2[c][ib] - T(2) * G[c];
    }
  }
  __syncthreads();

  // ---- phase 5: S4 = phi + dt v + dt^2/2 a2
  stage_b(cv4, ca4, s2);
  __syncthreads();

  // ---- phase 6: a4 = -G(S4); phi', v' at the own sites
  T* __restrict__ phn = cur ? V.phi[0] : V.phi[1];
  T* __restrict__ vn = cur ? V.vel[0] : V.vel[1];
  {
    Jet<T> J[C][RY];
    double dx_[C][RY], dy_[C][RY];
#pragma unroll
    for (int c = 0; c < C; ++c)
      column_jets<T, AX, RY, MIXED, false>(sa[c], 4 + threadIdx.x, 4 + wy * RY, c1, c2, 0.0, J[c], dx_[c],
                                           dy_[c]);
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      const int gj = y0 + wy * RY + r;
      if (gi >= Nx || gj >= Ny) continue;
      Jet<T> Js[4];
#pragma unroll
      for (int c = 0; c < C; ++c) Js[c] = J[c][r];
      T G[4] = {T(0), T(0), T(0), T(0)};
      site_gradient<T, TH>(Js, V, G);
      const int ib = (2 + wy * RY + r) * BX + 2 + threadIdx.x;
      T pn[4], vnew[4];
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const T v0 = arrest ? T(0) : sv[c][ib];
        pn[c] = sp[c][ib] + dt * v0 + (dt * dt / T(12)) * (qo[r][c] + s1[c][ib]);
        vnew[c] = v0 + (dt / T(6)) * (qo[r][c] - G[c]);
      }
      if (unit_field(TH)) {
        unit3(pn);
        const T vd = vnew[0] * pn[0] + vnew[1] * pn[1] + vnew[2] * pn[2];
#pragma unroll
        for (int c = 0; c < 3; ++c) vnew[c] -= vd * pn[c];
      }
      const long o = offs(gi, gj);
#pragma unroll
      for (int c = 0; c < C; ++c) {
        __builtin_nontemporal_store(pn[c], &phn[c * plane + o]);
        __builtin_nontemporal_store(vnew[c], &vn[c * plane + o]);
      }
    }
  }
  __syncthreads();
}

// Waves per SIMD the fused pass is compiled for. With FP32 fields two
// workgroups share a CU (LDS), so registers are capped at 256 per lane; with
// FP64 fields the LDS of one workgroup fills the CU and no cap applies.
template <class T>
struct FusedWaves {
  static constexpr int value = sizeof(T) == 4 ? 2 : 1;
};

// LDS elements of the fused pass for a tile shape
template <class T, int TH, int TX, int TY>
struct FusedLds {
  static constexpr int C = NComp<TH>::value;
  static constexpr int value = C * ((TX + 8) * (TY + 8) + 4 * (TX + 4) * (TY + 4));
};

template <class T, int TH, int TX, int TY, int RY>
__global__ void __launch_bounds__(TX*(TY / RY)) __attribute__((amdgpu_waves_per_eu(FusedWaves<T>::value)))
stage_pass_fused(PassArgs<T> a) {
  __shared__ __align__(16) T lds[FusedLds<T, TH, TX, TY>::value];
  DevStatus* __restrict__ st = a.st;
  if (st->done) return;
  const int cur = int((st->step - 1) & 1);
  const bool arrest = st->arrest != 0;
  const InstView<T> V = view_of<T>(a.B, a.cf);
  for_each_tile(a.ntx, a.nty, a.seg, [&](int tx, int ty, int, bool) {
    tile_body_fused<T, TH, TX, TY, RY>(V, cur, arrest, tx * TX, ty * TY, lds);
  });
}

// The single-lattice launch of the exact-gradient passes (tile 64 x 16, 256 threads).
template <class T, int TH, int PASS>
__global__ void __launch_bounds__(256) stage_pass_exact(PassArgs<T> a) {
  constexpr int C = NComp<TH>::value;
  constexpr int LX = kExTX + 8, LY = kExTY + 8;
  constexpr int NFL = 3 * (kExTY * (kExTX + 4) + (kExTY + 4) * kExTX);
  constexpr int NLDS = C * LY * LX > NFL ? C * LY * LX : NFL;
  constexpr int NT = 256;
  constexpr bool REDUCE = reduces(PASS);
  constexpr bool AFTER_P1 = (PASS == kP2 || PASS == kP3 || PASS == kP4);
  __shared__ __align__(16) T lds[NLDS];
  __shared__ double red[3 * (NT / 64)];

  DevStatus* __restrict__ st = a.st;
  if (PASS != kEval && PASS != kVVEnd && st->done) return;
  if (PASS == kVVRestart && !st->arrest) return;
  const long long step = st->step;
  const int cur = AFTER_P1 ? int((step - 1) & 1) : int(step & 1);
  const bool arrest = uses_arrest(PASS) ? (st->arrest != 0) : false;
  const InstView<T> V = view_of<T>(a.B, a.cf);
  double e_acc = 0.0, g_acc = 0.0;
  int nf = 0;
  for_each_tile(a.ntx, a.nty, a.seg, [&](int tx, int ty, int, bool) {
    tile_body_exact<T, TH, PASS>(V, cur, arrest, a.src, a.out, a.out_pitch, a.out_plane, tx * kExTX, ty * kExTY,
                                 lds, e_acc, g_acc, nf);
  });
  if (!REDUCE) return;
  block_reduce3<NT>(e_acc, g_acc, nf, red);
  if (threadIdx.y * kExTX + threadIdx.x == 0) {
    double* p = a.partials + 4 * (long)blockIdx.x;
    p[0] = e_acc;
    p[1] = g_acc;
    p[2] = (double)nf;
  }
}

// ------------------------------------------------------------------ batching
// Many independent lattices (uneven sizes and couplings) stepped by one launch
// per pass. The unit of work is a column segment of one member: n tiles stacked
// along y from tile row ty0 in tile column tx, walked top to bottom by one
// workgroup (so a tile's top halo rows are the rows that workgroup just read).
// The launch walks the work list work[0 .. *nwork) (the units of the members
// still running, rebuilt by the host between graph replays) as for_each_tile
// walks one lattice. Reductions are per member: each unit writes its own
// partial, and batch_finalise (one workgroup per member, launched after the
// pass) sums that member's partials in unit order and updates its status.
template <class T>
struct BatchInst {
  InstView<T> V;
  DevStatus* st;
  int unit0, nunits;  // the member's units (and partial slots): unit0 .. unit0 + nunits - 1
};

struct BatchUnit {
  int inst, tx, ty0, n;
};

template <class T>
struct BatchArgs {
  const BatchInst<T>* inst;
  const BatchUnit* units;
  const int* work;   // indices into units
  const int* nwork;
  double* partials;  // 4 doubles per unit
};

// XCD x owns the contiguous item range [x * per, (x + 1) * per) of the work
// list; its m = gridDim.x / 8 workgroups take items x*per + q, + m, ...
// (q = blockIdx.x / 8), so workgroups resident together on an XCD hold
// neighbouring units of the same members.
template <class F>
__device__ __forceinline__ void for_each_item(int nwork, F&& body) {
  const int m = gridDim.x >> 3, xcd = blockIdx.x & 7, q = blockIdx.x >> 3;
  const int per = (nwork + 7) >> 3;
  const int wend = min(nwork, (xcd + 1) * per);
  for (int w = xcd * per + q; w < wend; w += m) body(w);
}

template <class T, int TH, int PASS, int TX, int TY, int RY>
__global__ void __launch_bounds__(TX*(TY / RY))
__attribute__((amdgpu_waves_per_eu(StageWaves<T, TH, PASS, RY>::value))) batch_pass(BatchArgs<T> a) {
  constexpr int C = NComp<TH>::value;
  constexpr int LX = TX + 4, LY = TY + 4;
  constexpr int NT = TX * (TY / RY);
  constexpr bool REDUCE = reduces(PASS);
  // stages 2-4 of RK4 run after P1 advanced the member's step counter; the
  // one-pass integrators read the current field
  constexpr bool STAGED = (PASS == kP2 || PASS == kP3 || PASS == kP4);
  __shared__ __align__(16) T lds[TileLds<T, TH, PASS, TX, TY>::size];
  __shared__ double red[3 * (NT / 64)];
  const int tid = threadIdx.y * TX + threadIdx.x;
  for_each_item(*a.nwork, [&](int w) {
    const int u = a.work[w];
    const BatchUnit U = a.units[u];
    const BatchInst<T>& I = a.inst[U.inst];
    DevStatus* __restrict__ st = I.st;
    if (PASS != kVVEnd && st->done) return;
    if (PASS == kVVRestart && !st->arrest) return;
    const long long step = st->step;
    const int cur = STAGED ? int((step - 1) & 1) : int(step & 1);
    const bool arrest = uses_arrest(PASS) ? (st->arrest != 0) : false;
    double e_acc = 0.0, g_acc = 0.0;
    int nf = 0;
    for (int k = 0; k < U.n; ++k)
      tile_body<T, TH, PASS, TX, TY, RY>(I.V, cur, arrest, nullptr, nullptr, 0, 0, U.tx * TX, (U.ty0 + k) * TY, k,
                                         k + 1 < U.n, lds, e_acc, g_acc, nf);
    if (!REDUCE) return;
    block_reduce3<NT>(e_acc, g_acc, nf, red);
    if (tid == 0) {
      double* p = a.partials + 4 * (long)u;
      p[0] = e_acc;
      p[1] = g_acc;
      p[2] = (double)nf;
    }
    __syncthreads();
  });
}

// End of a batch reducing pass, one workgroup (256 threads) per member: the
// member's unit partials summed in unit order, then its status update. Being
// a launch of its own, it needs no fence or atomic inside the pass.
template <class T, int PASS>
__global__ void __launch_bounds__(256) batch_finalise(const BatchInst<T>* inst, const double* __restrict__ partials) {
  const BatchInst<T>& I = inst[blockIdx.x];
  DevStatus* __restrict__ st = I.st;
  if (st->done) return;
  double se = 0.0, sg = 0.0;
  int sn = 0;
  for (int k = threadIdx.x; k < I.nunits; k += 256) {
    const double* p = partials + 4 * (long)(I.unit0 + k);
    se += p[0];
    sg = fmax(sg, p[1]);
    sn += (int)p[2];
  }
  __shared__ double red[3 * 4];
  block_reduce3<256>(se, sg, sn, red);
  if (threadIdx.x == 0) finalise_status<PASS>(st, I.V.h * I.V.h * se, sg, sn);
}

// Fused stages 2-4 for the batch: the work list's units, each with its member's
// arrest flag and step parity (members that stopped are skipped).
template <class T, int TH, int TX, int TY, int RY>
__global__ void __launch_bounds__(TX*(TY / RY)) __attribute__((amdgpu_waves_per_eu(FusedWaves<T>::value)))
batch_pass_fused(BatchArgs<T> a) {
  __shared__ __align__(16) T lds[FusedLds<T, TH, TX, TY>::value];
  for_each_item(*a.nwork, [&](int w) {
    const BatchUnit U = a.units[a.work[w]];
    const BatchInst<T>& I = a.inst[U.inst];
    const DevStatus* __restrict__ st = I.st;
    if (st->done) return;
    const int cur = int((st->step - 1) & 1);
    const bool arrest = st->arrest != 0;
    for (int k = 0; k < U.n; ++k)
      tile_body_fused<T, TH, TX, TY, RY>(I.V, cur, arrest, U.tx * TX, (U.ty0 + k) * TY, lds);
  });
}

// Zero the velocity of every batch member whose last arrest test fired.
template <class T>
__global__ void __launch_bounds__(256) batch_apply_arrest(const BatchInst<T>* inst, int C) {
  const BatchInst<T>& I = inst[blockIdx.x];
  if (!I.st->arrest) return;
  T* v = I.V.vel[int(I.st->step & 1)];
  const long n = (long)C * I.V.plane;
  for (long k = threadIdx.x; k < n; k += 256) v[k] = T(0);
}

// Arm every batch member for a run (same rule for all).
__global__ void batch_arm(DevStatus* const* st, int n, int minimise, double grad_tol, double rel_e_tol, int window,
                          long long max_steps) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    DevStatus* s = st[i];
    s->done = 0;
    s->fresh = 1;
    s->minimise = minimise;
    s->grad_tol = grad_tol;
    s->rel_e_tol = rel_e_tol;
    s->window = window;
    s->max_steps = max_steps;
  }
}

// Collect the stop flags of all batch members (host reads n ints, not n status blocks).
__global__ void batch_done_flags(DevStatus* const* st, int n, int* flags) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) flags[i] = st[i]->done;
}

// Zero the velocity of the current field if the last arrest test fired.
template <class T>
__global__ void apply_arrest(Bufs<T> B, const DevStatus* __restrict__ st, int C) {
  if (!st->arrest) return;
  const int cur = int(st->step & 1);
  const long n = (long)C * B.plane;
  for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x)
    B.vel[cur][k] = T(0);
}

// Reset the stop flag and load the stop rules before a run of steps.
__global__ void arm_status(DevStatus* st, int minimise, double grad_tol, double rel_e_tol, int window,
                           long long max_steps) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    st->done = 0;
    st->fresh = 1;
    st->minimise = minimise;
    st->grad_tol = grad_tol;
    st->rel_e_tol = rel_e_tol;
    st->window = window;
    st->max_steps = max_steps;
  }
}

// ---------------------------------------------------------------- observables
// Sums over interior sites (FP64 from the stored values, first derivatives by
// eq. (1)), two-level reduction into st->obs[0..4]:
//   AH: E density, B, rho = [B W + 2 (P1 Q2 - Q1 P2)]/(2 pi), |r1|^2, r2^2
//   CM: E density, n.(d_x n x d_y n)
template <int N, int NT>
__device__ __forceinline__ void reduce_n_to(double (&v)[N], double* partials, unsigned* counter,
                                            int nlaunch, double* dst) {
  constexpr int NW = NT / 64;
  __shared__ double red[N * NW];
  __shared__ int last;
  const int tid = threadIdx.y * blockDim.x + threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
#pragma unroll
  for (int k = 0; k < N; ++k) {
    const double x = wave_sum(v[k]);
    if (lane == 0) red[k * NW + w] = x;
  }
  __syncthreads();
  if (tid == 0) {
    for (int k = 0; k < N; ++k) {
      double s = 0.0;
      for (int j = 0; j < NW; ++j) s += red[k * NW + j];
      partials[(long)blockIdx.x * N + k] = s;
    }
    __threadfence();
    last = (atomicAdd(counter, 1u) == (unsigned)(nlaunch - 1));
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  double acc[N];
#pragma unroll
  for (int k = 0; k < N; ++k) acc[k] = 0.0;
  for (int b = tid; b < nlaunch; b += NT)
#pragma unroll
    for (int k = 0; k < N; ++k) acc[k] += __builtin_nontemporal_load(partials + (long)b * N + k);
  __syncthreads();
#pragma unroll
  for (int k = 0; k < N; ++k) {
    const double x = wave_sum(acc[k]);
    if (lane == 0) red[k * NW + w] = x;
  }
  __syncthreads();
  if (tid == 0) {
    for (int k = 0; k < N; ++k) {
      double s = 0.0;
      for (int j = 0; j < NW; ++j) s += red[k * NW + j];
      dst[k] = s;
    }
    *counter = 0u;
  }
}

template <class T, int TH>
__global__ void __launch_bounds__(256) obs_sites(Bufs<T> B, Coeffs cf, DevStatus* st, double* partials,
                                                 int nlaunch) {
  const int cur = int(st->step & 1);
  const T* __restrict__ ph = B.phi[cur];
  const long nsite = (long)B.Nx * B.Ny;
  const double c1 = 1.0 / (12.0 * cf.h);
  double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  const double inv2pi = 0.15915494309189533577;
  for (long k = blockIdx.x * 256L + threadIdx.x; k < nsite; k += (long)gridDim.x * 256L) {
    const int j = (int)(k / B.Nx), i = (int)(k - (long)j * B.Nx);
    const long off = (long)(j + 2) * B.pitch + (i + 2);
    double f[4], dx[4], dy[4];
    for (int c = 0; c < (TH == 0 ? 4 : 3); ++c) {
      const T* p = ph + c * B.plane + off;
      f[c] = p[0];
      dx[c] = c1 * (((double)p[-2] - (double)p[2]) + 8.0 * ((double)p[1] - (double)p[-1]));
      dy[c] = c1 * (((double)p[-2 * B.pitch] - (double)p[2 * B.pitch]) +
                    8.0 * ((double)p[B.pitch] - (double)p[-B.pitch]));
    }
    if (TH == 0) {
      const double p = f[0], q = f[1], ax = f[2], ay = f[3];
      const double P1 = dx[0] + ax * q, Q1 = dx[1] - ax * p, P2 = dy[0] + ay * q, Q2 = dy[1] - ay * p;
      const double Bf = dx[3] - dy[2], W = 1.0 - (p * p + q * q);
      v[0] += 0.5 * (P1 * P1 + Q1 * Q1 + P2 * P2 + Q2 * Q2) + 0.5 * Bf * Bf + 0.125 * cf.p[0] * W * W;
      v[1] += Bf;
      v[2] += (Bf * W + 2.0 * (P1 * Q2 - Q1 * P2)) * inv2pi;
      const double r1r = P1 - Q2, r1i = Q1 + P2, r2 = Bf - 0.5 * W;
      v[3] += r1r * r1r + r1i * r1i;
      v[4] += r2 * r2;
    } else {
      // unit-vector theories: energy density and n . (d_x n x d_y n)
      Jet<double> Jd[4];
      for (int c = 0; c < 4; ++c) {
        Jd[c].f = c < 3 ? f[c] : 0.0;
        Jd[c].x = c < 3 ? dx[c] : 0.0;
        Jd[c].y = c < 3 ? dy[c] : 0.0;
        Jd[c].xx = Jd[c].yy = Jd[c].xy = 0.0;
      }
      v[0] += density<TH>(Jd, cf.p);
      if (TH == kCM && B.psi != nullptr) {
        double px, py;
        psi_gradient(B.psi, B.psi_pitch, i, j, c1, px, py);
        v[0] += 0.5 * cf.p[5] * (px * px + py * py);
      }
      const double tx = dx[1] * dy[2] - dx[2] * dy[1], ty = dx[2] * dy[0] - dx[0] * dy[2],
                   tz = dx[0] * dy[1] - dx[1] * dy[0];
      v[1] += f[0] * tx + f[1] * ty + f[2] * tz;
    }
  }
  reduce_n_to<5, 256>(v, partials, &st->counter_obs, nlaunch, st->obs);
}

// Berg-Luescher charge: every plaquette (i, j) .. (i+1, j+1) of the padded
// lattice, split into triangles (a, b, c) and (a, c, d), each contributing its
// signed solid angle 2 atan2(a.(b x c), 1 + a.b + b.c + c.a). Sum into st->obs[5].
template <class T>
__global__ void __launch_bounds__(256) obs_berg_luscher(Bufs<T> B, DevStatus* st, double* partials, int nlaunch) {
  const int cur = int(st->step & 1);
  const T* __restrict__ ph = B.phi[cur];
  const int PW = B.Nx + 3, PH = B.Ny + 3;  // plaquettes per row / column
  double v[1] = {0.0};
  for (long k = blockIdx.x * 256L + threadIdx.x; k < (long)PW * PH; k += (long)gridDim.x * 256L) {
    const int j = (int)(k / PW), i = (int)(k - (long)j * PW);  // padded indices of corner a
    double n[4][3];
    const int cj[4] = {j, j, j + 1, j + 1}, ci[4] = {i, i + 1, i + 1, i};
    for (int q = 0; q < 4; ++q)
      for (int c = 0; c < 3; ++c) n[q][c] = (double)ph[c * B.plane + (long)cj[q] * B.pitch + ci[q]];
    const int tri[2][3] = {{0, 1, 2}, {0, 2, 3}};
    for (int t = 0; t < 2; ++t) {
      const double* A = n[tri[t][0]];
      const double* Bv = n[tri[t][1]];
      const double* Cv = n[tri[t][2]];
      const double bx = Bv[1] * Cv[2] - Bv[2] * Cv[1], by = Bv[2] * Cv[0] - Bv[0] * Cv[2],
                   bz = Bv[0] * Cv[1] - Bv[1] * Cv[0];
      const double num = A[0] * bx + A[1] * by + A[2] * bz;
      const double den = 1.0 + (A[0] * Bv[0] + A[1] * Bv[1] + A[2] * Bv[2]) +
                         (Bv[0] * Cv[0] + Bv[1] * Cv[1] + Bv[2] * Cv[2]) + (Cv[0] * A[0] + Cv[1] * A[1] + Cv[2] * A[2]);
      v[0] += 2.0 * atan2(num, den);
    }
  }
  reduce_n_to<1, 256>(v, partials, &st->counter_obs, nlaunch, st->obs + 5);
}

// Phase winding of psi along the ring of outermost interior sites (one
// workgroup, fixed order), into st->obs[6] (in units of 2 pi).
template <class T>
__global__ void __launch_bounds__(256) obs_winding(Bufs<T> B, DevStatus* st) {
  const int cur = int(st->step & 1);
  const T* __restrict__ ph = B.phi[cur];
  const int Nx = B.Nx, Ny = B.Ny;
  const long L = 2L * (Nx - 1) + 2L * (Ny - 1);
  auto site = [&](long k, int& j, int& i) {
    if (k < Nx - 1) { j = 0; i = (int)k; return; }
    k -= Nx - 1;
    if (k < Ny - 1) { j = (int)k; i = Nx - 1; return; }
    k -= Ny - 1;
    if (k < Nx - 1) { j = Ny - 1; i = Nx - 1 - (int)k; return; }
    k -= Nx - 1;
    j = Ny - 1 - (int)k; i = 0;
  };
  double acc[1] = {0.0};
  const double pi = 3.14159265358979323846;
  for (long k = threadIdx.x; k < L; k += 256) {
    int ja, ia, jb, ib;
    site(k, ja, ia);
    site((k + 1) % L, jb, ib);
    const long oa = (long)(ja + 2) * B.pitch + ia + 2, ob = (long)(jb + 2) * B.pitch + ib + 2;
    double d = atan2((double)ph[B.plane + ob], (double)ph[ob]) - atan2((double)ph[B.plane + oa], (double)ph[oa]);
    if (d > pi) d -= 2.0 * pi;
    if (d <= -pi) d += 2.0 * pi;
    acc[0] += d;
  }
  __shared__ double red[4];
  const double x = wave_sum(acc[0]);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
  __syncthreads();
  if (threadIdx.x == 0) st->obs[6] = (red[0] + red[1] + red[2] + red[3]) / (2.0 * pi);
}

// --------------------------------------------------------------- state init
// SplitMix64 (Steele, Lea and Flood 2014): output function, and the counter
// draw u(seed, stream, n) = mix(key + (n + 1) * golden) with
// key = mix(seed * golden + stream), as double in [0, 1).
__device__ __forceinline__ unsigned long long splitmix_mix(unsigned long long z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

__device__ __forceinline__ double splitmix_u01(unsigned long long key, unsigned long long n) {
  const unsigned long long z = splitmix_mix(key + (n + 1ULL) * 0x9E3779B97F4A7C15ULL);
  return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

struct InitArgs {
  int kind, n;
  const double* xy;  // device copy of the centres
  const double* w;   // device copy of the windings
  double R, gamma;  // skyrmion: radius and helicity; BEC: cloud radius and vortex core width
  unsigned long long key;  // noise stream key (0 = no noise)
  double amp;
};

// One thread per padded site; writes phi[0] and phi[1].
template <class T>
__global__ void __launch_bounds__(256) init_ansatz(Bufs<T> B, Coeffs cf, InitArgs ia) {
  const long W = B.Nx + 4, H = B.Ny + 4;
  const long k = blockIdx.x * 256L + threadIdx.x;
  if (k >= W * H) return;
  const int jj = (int)(k / W), ii = (int)(k - (long)jj * W);  // padded indices
  const int i = ii - 2, j = jj - 2;
  const bool inner = i >= 0 && i < B.Nx && j >= 0 && j < B.Ny;
  const double x = (i - 0.5 * (B.Nx - 1)) * cf.h, y = (j - 0.5 * (B.Ny - 1)) * cf.h;
  double out[4] = {0.0, 0.0, 0.0, 0.0};
  int C = 3;
  if (ia.kind == 2) {
    // BEC: Gaussian cloud of radius R with vortices of core width xi; psi = 0 on the halo
    C = 2;
    if (inner) {
      double amp = exp(-(x * x + y * y) / (2.0 * ia.R * ia.R)) / (sqrt(M_PI) * ia.R), ph = 0.0;
      for (int v = 0; v < ia.n; ++v) {
        const double dx = x - ia.xy[2 * v], dy = y - ia.xy[2 * v + 1];
        amp *= tanh(sqrt(dx * dx + dy * dy) / ia.gamma);
        ph += ia.w[v] * atan2(dy, dx);
      }
      out[0] = amp * cos(ph);
      out[1] = amp * sin(ph);
    }
  } else if (ia.kind == 0) {
    C = 4;
    double mod = 1.0, ph = 0.0, ax = 0.0, ay = 0.0;
    for (int v = 0; v < ia.n; ++v) {
      const double dx = x - ia.xy[2 * v], dy = y - ia.xy[2 * v + 1], wv = ia.w[v];
      const double r2 = dx * dx + dy * dy;
      ph += wv * atan2(dy, dx);
      double prof;
      if (inner) {
        mod *= tanh(sqrt(r2));
        prof = r2 > 1e-300 ? -expm1(-r2) / r2 : 1.0;
      } else {
        prof = r2 > 1e-300 ? 1.0 / r2 : 0.0;
      }
      ax += wv * prof * (-dy);
      ay += wv * prof * dx;
    }
    out[0] = mod * cos(ph);
    out[1] = mod * sin(ph);
    out[2] = ax;
    out[3] = ay;
  } else {
    if (inner) {
      const double dx = x - ia.xy[0], dy = y - ia.xy[1];
      const double r = sqrt(dx * dx + dy * dy), th = atan2(dy, dx);
      const double Th = 2.0 * atan2(ia.R, r);
      const double az = ia.w[0] * th + ia.gamma;  // vorticity w[0] (-1: antiskyrmion)
      out[0] = sin(Th) * cos(az);
      out[1] = sin(Th) * sin(az);
      out[2] = cos(Th);
    } else {
      out[2] = 1.0;
    }
  }
  if (inner && ia.key != 0ULL) {
    for (int c = 0; c < C; ++c) {
      const unsigned long long n = ((unsigned long long)c * B.Ny + j) * B.Nx + i;
      out[c] += ia.amp * (2.0 * splitmix_u01(ia.key, n) - 1.0);
    }
    if (ia.kind == 1) {  // unit vectors are renormalised after the noise
      const double r = sqrt(out[0] * out[0] + out[1] * out[1] + out[2] * out[2]);
      for (int c = 0; c < 3; ++c) out[c] /= r;
    }
  }
  const long off = (long)jj * B.pitch + ii;
  for (int c = 0; c < C; ++c) {
    B.phi[0][c * B.plane + off] = (T)out[c];
    B.phi[1][c * B.plane + off] = (T)out[c];
  }
}

// ------------------------------------------------------- learned initialiser
// Network input on the interior grid (Ny x Nx x 2, fp32, row-major):
// channel 0 = sum_k exp(-r_k^2 / 2) (unit Gaussians at the vortex centres),
// channel 1 = kappa.
__global__ void __launch_bounds__(256) learned_input(int Nx, int Ny, double h, const double* xy, int n, double kappa,
                                                     float* out) {
  const long k = blockIdx.x * 256L + threadIdx.x;
  if (k >= (long)Nx * Ny) return;
  const int j = (int)(k / Nx), i = (int)(k - (long)j * Nx);
  const double x = (i - 0.5 * (Nx - 1)) * h, y = (j - 0.5 * (Ny - 1)) * h;
  double b = 0.0;
  for (int v = 0; v < n; ++v) {
    const double dx = x - xy[2 * v], dy = y - xy[2 * v + 1];
    b += exp(-0.5 * (dx * dx + dy * dy));
  }
  out[2 * k] = (float)b;
  out[2 * k + 1] = (float)kappa;
}

// Ansatz modulus, phase and gauge field at one point (product ansatz of the
// Abelian-Higgs vortices, as in init_ansatz).
__device__ __forceinline__ void ah_ansatz_parts(double x, double y, const double* xy, const double* w, int n,
                                                double& mod, double& ph, double& ax, double& ay) {
  mod = 1.0; ph = 0.0; ax = 0.0; ay = 0.0;
  for (int v = 0; v < n; ++v) {
    const double dx = x - xy[2 * v], dy = y - xy[2 * v + 1], wv = w[v];
    const double r2 = dx * dx + dy * dy;
    ph += wv * atan2(dy, dx);
    mod *= tanh(sqrt(r2));
    const double prof = r2 > 1e-300 ? -expm1(-r2) / r2 : 1.0;
    ax += wv * prof * (-dy);
    ay += wv * prof * dx;
  }
}

// Training target of a relaxed field in the co-rotating frame of the ansatz:
// (Re, Im) of psi e^{-i Theta} - f_ans, then A_x - A_ans_x, A_y - A_ans_y, at every
// interior site (Ny x Nx x 4, fp32). Theta = sum_k w_k theta_k. The first pair is
// smooth through the vortex cores (no phase cut, no 0/0 where |psi| vanishes).
template <class T>
__global__ void __launch_bounds__(256) learned_targets(Bufs<T> B, Coeffs cf, const DevStatus* st, const double* xy,
                                                       const double* w, int n, float* out) {
  const long k = blockIdx.x * 256L + threadIdx.x;
  if (k >= (long)B.Nx * B.Ny) return;
  const int j = (int)(k / B.Nx), i = (int)(k - (long)j * B.Nx);
  const double x = (i - 0.5 * (B.Nx - 1)) * cf.h, y = (j - 0.5 * (B.Ny - 1)) * cf.h;
  double mod, ph, ax, ay;
  ah_ansatz_parts(x, y, xy, w, n, mod, ph, ax, ay);
  const T* f = st->step & 1 ? B.phi[1] : B.phi[0];
  const long off = (long)(j + 2) * B.pitch + (i + 2);
  const double p = f[off], q = f[B.plane + off];
  const double cs = cos(ph), sn = sin(ph);
  out[4 * k] = (float)(p * cs + q * sn - mod);
  out[4 * k + 1] = (float)(q * cs - p * sn);
  out[4 * k + 2] = (float)((double)f[2 * B.plane + off] - ax);
  out[4 * k + 3] = (float)((double)f[3 * B.plane + off] - ay);
}

// Field from the ansatz plus predicted corrections c, weighted by an envelope
// that is 1 at the vortex centres and decays away from them,
//   env = 1 - prod_k (1 - exp(-r_k^2 / (2 sigma^2)))   (sigma <= 0: env = 1),
// so that a network's small errors far from the vortices (where the ansatz is
// already the vacuum) do not seed slow, lattice-wide modes, and (pin > 0) a
// factor on the psi correction that vanishes at every centre,
//   pinf = prod_k (1 - exp(-r_k^2 / (2 pin^2)))        (pin <= 0: pinf = 1),
// which keeps the zeros of psi at the given centres:
//   psi = (f_ans + env pinf (c0 + i c1)) e^{i Theta},   A = A_ans + env (c2, c3)
// on the interior, plus (key != 0) the seeded uniform noise of init_ansatz
// (same stream and amplitude, so zero corrections without envelope or pin
// reproduce the noisy ansatz); the halo gets the pure-gauge vacuum.
template <class T>
__global__ void __launch_bounds__(256) init_learned(Bufs<T> B, Coeffs cf, const double* xy, const double* w, int n,
                                                    const float* corr, double sigma, double pin,
                                                    unsigned long long key, double amp) {
  const long W = B.Nx + 4, H = B.Ny + 4;
  const long k = blockIdx.x * 256L + threadIdx.x;
  if (k >= W * H) return;
  const int jj = (int)(k / W), ii = (int)(k - (long)jj * W);
  const int i = ii - 2, j = jj - 2;
  const bool inner = i >= 0 && i < B.Nx && j >= 0 && j < B.Ny;
  const double x = (i - 0.5 * (B.Nx - 1)) * cf.h, y = (j - 0.5 * (B.Ny - 1)) * cf.h;
  double out[4];
  if (inner) {
    double mod, ph, ax, ay;
    ah_ansatz_parts(x, y, xy, w, n, mod, ph, ax, ay);
    double env = 1.0;
    if (sigma > 0.0) {
      double far = 1.0;
      const double s2 = 0.5 / (sigma * sigma);
      for (int v = 0; v < n; ++v) {
        const double dx = x - xy[2 * v], dy = y - xy[2 * v + 1];
        far *= -expm1(-(dx * dx + dy * dy) * s2);
      }
      env = 1.0 - far;
    }
    double pinf = 1.0;
    if (pin > 0.0) {
      const double s2 = 0.5 / (pin * pin);
      for (int v = 0; v < n; ++v) {
        const double dx = x - xy[2 * v], dy = y - xy[2 * v + 1];
        pinf *= -expm1(-(dx * dx + dy * dy) * s2);
      }
    }
    const float* c = corr + 4 * ((long)j * B.Nx + i);
    const double re = mod + env * pinf * c[0], im = env * pinf * c[1];
    const double cs = cos(ph), sn = sin(ph);
    out[0] = re * cs - im * sn;
    out[1] = re * sn + im * cs;
    out[2] = ax + env * c[2];
    out[3] = ay + env * c[3];
    if (key != 0ULL)
      for (int cc = 0; cc < 4; ++cc) {
        const unsigned long long q = ((unsigned long long)cc * B.Ny + j) * B.Nx + i;
        out[cc] += amp * (2.0 * splitmix_u01(key, q) - 1.0);
      }
  } else {
    double ph = 0.0, ax = 0.0, ay = 0.0;
    for (int v = 0; v < n; ++v) {
      const double dx = x - xy[2 * v], dy = y - xy[2 * v + 1], wv = w[v];
      const double r2 = dx * dx + dy * dy;
      ph += wv * atan2(dy, dx);
      const double prof = r2 > 1e-300 ? 1.0 / r2 : 0.0;
      ax += wv * prof * (-dy);
      ay += wv * prof * dx;
    }
    out[0] = cos(ph);
    out[1] = sin(ph);
    out[2] = ax;
    out[3] = ay;
  }
  const long off = (long)jj * B.pitch + ii;
  for (int c = 0; c < 4; ++c) {
    B.phi[0][c * B.plane + off] = (T)out[c];
    B.phi[1][c * B.plane + off] = (T)out[c];
  }
}

}  // namespace ss
