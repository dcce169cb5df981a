// Rotating trapped Bose-Einstein condensate (Sec. 4.3) on the device.
//
// Trap units (hbar = m = omega = 1), psi = u + i w, two components:
//   e = 1/2 |grad psi|^2 + 1/2 r^2 |psi|^2 + g/2 |psi|^4 - Omega Re(psi* L_z psi),
//   L_z = -i (x d_y - y d_x), Re(psi* L_z psi) = u (x w_y - y w_x) - w (x u_y - y u_x),
// with eq. (1) first derivatives in the energy and the Euler-Lagrange gradient
//   G_u = -lap u + r^2 u + 2 g |psi|^2 u - 2 Omega (x w_y - y w_x),
//   G_w = -lap w + r^2 w + 2 g |psi|^2 w + 2 Omega (x u_y - y u_x)
// (eq. (2) second derivatives). Sites are cell-centred: x_i = (i - (Nx-1)/2) h.
//
// The flow holds the atom number N = h^2 sum |psi|^2 fixed: every stage point is
// scaled to N before its force is taken, the force is -(G - mu psi) with
// mu = <psi, G> / <psi, psi> (its projection on the tangent space of that
// sphere), and after each step the field is scaled to N and the velocity
// projected on the tangent space. Both need sums over the whole lattice, so a
// stage is three launches: the stage point and the partials of its norm; the
// scale and G with the partials of psi.G and psi.psi; mu and the pass's own
// update. All sums are FP64 per-workgroup partials added in workgroup order, by
// every workgroup of the launch that needs the total.
#pragma once

#include "ss_internal.hpp"

namespace ss {

constexpr int kBecGroups = 512;  // workgroups of every BEC launch (grid-stride over sites)

// Work buffers: the stage point S and the gradient G (two planes each, the flow's
// layout), three sets of FP64 workgroup partials (the stage point's norm,
// kBecGroups; the gradient's sums and the update's, kBecGroups * 4 each), and the
// scalars of a stage {c (scale to N), mu, E h^2, non-finite count, c' (end of
// step), m (velocity projection)}. The scale c and mu are summed from their
// partials by every workgroup of the launch that uses them (in the same fixed
// order), workgroup 0 keeping them in sc for the launches after.
template <class T>
struct BecBufs {
  T* S;
  T* G;
  double* part;  // partials of the update (bec_apply)
  double* sc;
  double* ps;    // partials of the stage point's norm (bec_stage)
  double* pg;    // partials of the gradient's sums (bec_grad)
};

#define BEC_SITES(n) for (long k_ = blockIdx.x * 256L + threadIdx.x; k_ < (n); k_ += (long)gridDim.x * 256L)

// Sum of 256 threads' value in a fixed order (valid in thread 0).
__device__ __forceinline__ double bec_block_sum(double v, double* red) {
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return red[0] + red[1] + red[2] + red[3];
}

// Sum over the kBecGroups partials part[k * stride + off] by one workgroup of 256
// threads in a fixed order (strided per thread, then in wave order); valid in
// thread 0.
__device__ __forceinline__ double bec_partials_sum(const double* __restrict__ part, int stride, int off,
                                                   double* red) {
  double acc = 0.0;
  for (int k = threadIdx.x; k < kBecGroups; k += 256) acc += part[(long)k * stride + off];
  return bec_block_sum(acc, red);
}

__device__ __forceinline__ double bec_block_max(double v, double* red) {
  v = wave_max(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

// Stage point of a pass over the padded lattice (as the stage passes form it) and
// the partial sums of its squares over the interior.
template <class T, int PASS>
__global__ void __launch_bounds__(256) bec_stage(Bufs<T> B, Coeffs cf, const DevStatus* __restrict__ st,
                                                 const T* __restrict__ src, BecBufs<T> W) {
  if (PASS != kEval && st->done) return;
  __shared__ double red[4];
  constexpr bool AFTER_P1 = (PASS == kP2 || PASS == kP3 || PASS == kP4);
  constexpr bool ONEPASS = advances_first(PASS);
  constexpr bool STAGED = AFTER_P1 || ONEPASS;
  const long long step = st->step;
  const int cur = AFTER_P1 ? int((step - 1) & 1) : int(step & 1);
  const bool arrest = (AFTER_P1 || PASS == kVVA) ? (st->arrest != 0) : false;
  const T dt = (T)cf.dt;
  T cv = T(0), ca = T(0);
  if (PASS == kP2) cv = T(0.5) * dt;
  if (PASS == kP3) { cv = T(0.5) * dt; ca = T(0.25) * dt * dt; }
  if (PASS == kP4 || PASS == kVVA) { cv = dt; ca = T(0.5) * dt * dt; }
  if (PASS == kGF) ca = T(0.5) * dt * dt;
  if (arrest) cv = T(0);
  const T* __restrict__ ph = (PASS == kEval && src != nullptr) ? src : (cur ? B.phi[1] : B.phi[0]);
  const T* __restrict__ vv = cur ? B.vel[1] : B.vel[0];
  // one-pass integrators: the current field's force in the buffer of the step's parity
  const T* __restrict__ aa = ONEPASS ? (cur ? B.a2 : B.a1) : (PASS == kP3) ? B.a1 : B.a2;
  const long Wd = B.Nx + 4, H = B.Ny + 4;
  double acc = 0.0;
  BEC_SITES(Wd * H) {
    const int jj = (int)(k_ / Wd), ii = (int)(k_ - (long)jj * Wd);
    const long o = (long)jj * B.pitch + ii;
    const bool inner = ii >= 2 && ii < B.Nx + 2 && jj >= 2 && jj < B.Ny + 2;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      T x = ph[c * B.plane + o];
      if (STAGED) {
        if (PASS != kGF) x += cv * vv[c * B.plane + o];
        if (PASS != kP2) x += ca * aa[c * B.plane + o];
      }
      W.S[c * B.plane + o] = x;
      if (inner) acc += (double)x * (double)x;
    }
  }
  const double s = bec_block_sum(acc, red);
  if (threadIdx.x == 0) W.ps[blockIdx.x] = s;
}

// c = sqrt(N / (h^2 sum S^2)): the scale of the stage point onto the sphere of
// atom number N, from the stage partials (every thread of the workgroup).
__device__ __forceinline__ double bec_scale_of(const double* __restrict__ ps, const Coeffs& cf, double* red) {
  const double s = bec_partials_sum(ps, 1, 0, red);
  return sqrt(cf.p[2] / (cf.h * cf.h * s));
}

// Value of the scaled stage point at padded (jj, ii): c S inside the interior, S on the halo.
template <class T>
__device__ __forceinline__ T bec_at(const T* __restrict__ S, long pitch, int Nx, int Ny, T c, int jj, int ii) {
  const T v = S[(long)jj * pitch + ii];
  return (ii >= 2 && ii < Nx + 2 && jj >= 2 && jj < Ny + 2) ? c * v : v;
}

// G at the scaled stage point; partials {psi.G, psi.psi, energy density sum,
// non-finite count}. The energy is that of the field the pass tests, in FP64: the
// stage point as stored (unscaled) for an evaluation, a check or the first stage of
// RK4; the scaled stage point, which becomes the new field, for a one-pass step.
template <class T, int PASS>
__global__ void __launch_bounds__(256) bec_grad(Bufs<T> B, Coeffs cf, const DevStatus* __restrict__ st,
                                                BecBufs<T> W) {
  if (PASS != kEval && st->done) return;
  __shared__ double red[4];
  constexpr bool REDUCE = reduces(PASS);
  const double cd = bec_scale_of(W.ps, cf, red);
  if (blockIdx.x == 0 && threadIdx.x == 0) W.sc[0] = cd;
  const T c = (T)cd;
  const T g = (T)cf.p[0], Om = (T)cf.p[1];
  const double h = cf.h;
  const T c1 = T(1.0 / (12.0 * h)), c2 = T(1.0 / (12.0 * h * h));
  const double d1 = 1.0 / (12.0 * h);
  const long n = (long)B.Nx * B.Ny;
  double sG = 0.0, ss = 0.0, se = 0.0, nf = 0.0;
  BEC_SITES(n) {
    const int j = (int)(k_ / B.Nx), i = (int)(k_ - (long)j * B.Nx);
    const int jj = j + 2, ii = i + 2;
    T f[2], dx[2], dy[2], lap[2];
    double fd[2], dxd[2], dyd[2];
#pragma unroll
    for (int comp = 0; comp < 2; ++comp) {
      const T* Sc = W.S + comp * B.plane;
      auto at = [&](int dj, int di) { return bec_at(Sc, B.pitch, B.Nx, B.Ny, c, jj + dj, ii + di); };
      const T xm2 = at(0, -2), xm1 = at(0, -1), x0 = at(0, 0), xp1 = at(0, 1), xp2 = at(0, 2);
      const T ym2 = at(-2, 0), ym1 = at(-1, 0), yp1 = at(1, 0), yp2 = at(2, 0);
      f[comp] = x0;
      dx[comp] = c1 * ((xm2 - xp2) + T(8) * (xp1 - xm1));
      dy[comp] = c1 * ((ym2 - yp2) + T(8) * (yp1 - ym1));
      lap[comp] = c2 * ((-(xm2 + xp2) + T(16) * (xm1 + xp1)) + (-(ym2 + yp2) + T(16) * (ym1 + yp1)) - T(60) * x0);
      if (REDUCE) {
        auto raw = [&](int dj, int di) {
          return advances_first(PASS) ? (double)at(dj, di) : (double)Sc[(long)(jj + dj) * B.pitch + (ii + di)];
        };
        fd[comp] = raw(0, 0);
        dxd[comp] = d1 * ((raw(0, -2) - raw(0, 2)) + 8.0 * (raw(0, 1) - raw(0, -1)));
        dyd[comp] = d1 * ((raw(-2, 0) - raw(2, 0)) + 8.0 * (raw(1, 0) - raw(-1, 0)));
      }
    }
    const double xd = (i - 0.5 * (B.Nx - 1)) * h, yd = (j - 0.5 * (B.Ny - 1)) * h;
    const T x = (T)xd, y = (T)yd, r2 = (T)(xd * xd + yd * yd);
    const T u = f[0], w = f[1], rho = u * u + w * w;
    const T G0 = -lap[0] + r2 * u + T(2) * g * rho * u - T(2) * Om * (x * dy[1] - y * dx[1]);
    const T G1 = -lap[1] + r2 * w + T(2) * g * rho * w + T(2) * Om * (x * dy[0] - y * dx[0]);
    const long o = (long)jj * B.pitch + ii;
    W.G[o] = G0;
    W.G[B.plane + o] = G1;
    sG += (double)u * (double)G0 + (double)w * (double)G1;
    ss += (double)u * (double)u + (double)w * (double)w;
    if (!isfinite(G0) || !isfinite(G1)) nf += 1.0;
    if (REDUCE) {
      const double ud = fd[0], wd = fd[1];
      const double rhod = ud * ud + wd * wd;
      const double lz = ud * (xd * dyd[1] - yd * dxd[1]) - wd * (xd * dyd[0] - yd * dxd[0]);
      const double e = 0.5 * (dxd[0] * dxd[0] + dyd[0] * dyd[0] + dxd[1] * dxd[1] + dyd[1] * dyd[1]) +
                       0.5 * (xd * xd + yd * yd) * rhod + 0.5 * cf.p[0] * rhod * rhod - cf.p[1] * lz;
      se += e;
      if (!isfinite(e)) nf += 1.0;
    }
  }
  const double a0 = bec_block_sum(sG, red);
  const double a1 = bec_block_sum(ss, red);
  const double a2 = bec_block_sum(se, red);
  const double a3 = bec_block_sum(nf, red);
  if (threadIdx.x == 0) {
    double* p = W.pg + 4 * (long)blockIdx.x;
    p[0] = a0;
    p[1] = a1;
    p[2] = a2;
    p[3] = a3;
  }
}

// mu = <psi, G> / <psi, psi> from the gradient partials (every thread of the
// workgroup); workgroup 0 also keeps mu, E h^2 and the non-finite count of the
// stage in sc[1..3].
__device__ __forceinline__ double bec_mu_of(const double* __restrict__ pg, double* sc, const Coeffs& cf,
                                            double* red) {
  const double sG = bec_partials_sum(pg, 4, 0, red);
  const double ss = bec_partials_sum(pg, 4, 1, red);
  const double se = bec_partials_sum(pg, 4, 2, red);
  const double nf = bec_partials_sum(pg, 4, 3, red);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc[1] = sG / ss;
    sc[2] = cf.h * cf.h * se;
    sc[3] = nf;
  }
  return sG / ss;
}

// The force a = -(G - mu psi) at the scaled stage point and the pass's update; a
// reducing pass also writes the partial max |G - mu psi|. P4 writes the new field
// and velocity before the end-of-step constraint (bec_fix) and the partial sums
// {phi'.phi', phi'.v'}.
template <class T, int PASS>
__global__ void __launch_bounds__(256) bec_apply(Bufs<T> B, Coeffs cf, const DevStatus* __restrict__ st,
                                                 BecBufs<T> W, const double* __restrict__ sc, T* __restrict__ out,
                                                 long out_pitch, long out_plane) {
  if (PASS != kEval && st->done) return;
  __shared__ double red[4];
  constexpr bool STAGED = (PASS == kP2 || PASS == kP3 || PASS == kP4);
  const long long step = st->step;
  const int cur = STAGED ? int((step - 1) & 1) : int(step & 1);
  const bool arrest = (STAGED || PASS == kVVA) ? (st->arrest != 0) : false;
  const T mu = (T)bec_mu_of(W.pg, W.sc, cf, red);
  const T c = (T)sc[0];
  // one-pass integrators: current force (read) and new force (written) by parity
  const T* __restrict__ a_cur = cur ? B.a2 : B.a1;
  T* __restrict__ a_new = cur ? B.a1 : B.a2;
  const T dt = (T)cf.dt;
  const T* __restrict__ ph = cur ? B.phi[1] : B.phi[0];
  const T* __restrict__ vv = cur ? B.vel[1] : B.vel[0];
  T* __restrict__ phn = cur ? B.phi[0] : B.phi[1];
  T* __restrict__ vn = cur ? B.vel[0] : B.vel[1];
  const long n = (long)B.Nx * B.Ny;
  double gm = 0.0, spp = 0.0, spv = 0.0;
  BEC_SITES(n) {
    const int j = (int)(k_ / B.Nx), i = (int)(k_ - (long)j * B.Nx);
    const long o = (long)(j + 2) * B.pitch + (i + 2);
    T a[2];
#pragma unroll
    for (int comp = 0; comp < 2; ++comp) {
      const long k = comp * B.plane + o;
      const T Gp = W.G[k] - mu * (c * W.S[k]);
      a[comp] = -Gp;
      gm = fmax(gm, fabs((double)Gp));
    }
    if (PASS == kEval) {
      if (out != nullptr) {
        const long oo = (long)(j + 2) * out_pitch + (i + 2);
        out[oo] = -a[0];
        out[out_plane + oo] = -a[1];
      }
    } else if (PASS == kP1) {
      B.a1[o] = a[0];
      B.a1[B.plane + o] = a[1];
    } else if (PASS == kPrime) {
      // the current field's force, in the buffer of the step's parity
      T* __restrict__ as = cur ? B.a2 : B.a1;
      as[o] = a[0];
      as[B.plane + o] = a[1];
    } else if (PASS == kVVA || PASS == kGF) {
      // the scaled stage point is the new field; velocity Verlet also forms
      // v' = v + dt/2 (a + a'), projected by bec_vproj after the sums below
#pragma unroll
      for (int comp = 0; comp < 2; ++comp) {
        const long k = comp * B.plane + o;
        const T pn = c * W.S[k];
        phn[k] = pn;
        a_new[k] = a[comp];
        spp += (double)pn * (double)pn;
        if (PASS == kVVA) {
          const T vnew = (arrest ? T(0) : vv[k]) + (T(0.5) * dt) * (a_cur[k] + a[comp]);
          vn[k] = vnew;
          spv += (double)pn * (double)vnew;
        }
      }
    } else if (PASS == kP2) {
      B.a2[o] = a[0];
      B.a2[B.plane + o] = a[1];
    } else if (PASS == kP3) {
#pragma unroll
      for (int comp = 0; comp < 2; ++comp) {
        const long k = comp * B.plane + o;
        B.q[k] = B.a1[k] + T(2) * B.a2[k] + T(2) * a[comp];
      }
    } else if (PASS == kP4) {
#pragma unroll
      for (int comp = 0; comp < 2; ++comp) {
        const long k = comp * B.plane + o;
        const T v0 = arrest ? T(0) : vv[k];
        const T qq = B.q[k];
        const T pn = ph[k] + dt * v0 + (dt * dt / T(12)) * (qq + B.a1[k]);
        const T vnew = v0 + (dt / T(6)) * (qq + a[comp]);
        phn[k] = pn;
        vn[k] = vnew;
        spp += (double)pn * (double)pn;
        spv += (double)pn * (double)vnew;
      }
    }
  }
  // partials, four per workgroup: {max |G - mu psi|, phi'.phi', phi'.v', unused}
  const double m = reduces(PASS) ? bec_block_max(gm, red) : 0.0;
  const double a1 = (PASS == kP4 || PASS == kVVA) ? bec_block_sum(spp, red) : 0.0;
  const double a2 = (PASS == kP4 || PASS == kVVA) ? bec_block_sum(spv, red) : 0.0;
  if (threadIdx.x == 0) {
    double* p = W.part + 4 * (long)blockIdx.x;
    p[0] = m;
    p[1] = a1;
    p[2] = a2;
  }
}

// Status update of a reducing BEC pass: the stage's energy and non-finite count
// (bec_mu) and the max of the constrained force, through the common finalise.
template <int PASS>
__global__ void __launch_bounds__(256) bec_finalise(DevStatus* st, const double* __restrict__ part,
                                                    const double* __restrict__ sc) {
  if (PASS != kEval && st->done) return;
  __shared__ double red[4];
  double gm = 0.0;
  for (int k = threadIdx.x; k < kBecGroups; k += 256) gm = fmax(gm, part[4 * (long)k]);
  gm = bec_block_max(gm, red);
  if (threadIdx.x == 0) finalise_status<PASS>(st, sc[2], gm, (int)sc[3]);
}

// End of a step: phi' scaled to N, v' projected on the tangent space at phi'
// (the projection uses the unscaled phi'; the coefficient is scale-free).
__global__ void __launch_bounds__(256) bec_fix_scalars(const double* __restrict__ part, double* sc, Coeffs cf,
                                                       const DevStatus* __restrict__ st) {
  if (st->done) return;
  __shared__ double red[4];
  const double pp = bec_partials_sum(part, 4, 1, red);
  const double pv = bec_partials_sum(part, 4, 2, red);
  if (threadIdx.x == 0) {
    sc[4] = sqrt(cf.p[2] / (cf.h * cf.h * pp));
    sc[5] = pv / pp;
  }
}

template <class T>
__global__ void __launch_bounds__(256) bec_fix(Bufs<T> B, const DevStatus* __restrict__ st, const double* __restrict__ sc) {
  if (st->done) return;
  // P4 ran after P1 advanced the step: the new field is in the buffer of parity step & 1
  const int nxt = int(st->step & 1);
  T* __restrict__ ph = nxt ? B.phi[1] : B.phi[0];
  T* __restrict__ v = nxt ? B.vel[1] : B.vel[0];
  const T cs = (T)sc[4], m = (T)sc[5];
  const long n = (long)B.Nx * B.Ny;
  BEC_SITES(n) {
    const int j = (int)(k_ / B.Nx), i = (int)(k_ - (long)j * B.Nx);
    const long o = (long)(j + 2) * B.pitch + (i + 2);
#pragma unroll
    for (int comp = 0; comp < 2; ++comp) {
      const long k = comp * B.plane + o;
      const T p = ph[k];
      v[k] = v[k] - m * p;
      ph[k] = cs * p;
    }
  }
}

// Velocity Verlet: v' projected on the tangent space at the new field (which the
// pass wrote into the buffer of the other parity; the step counter advances after).
template <class T>
__global__ void __launch_bounds__(256) bec_vproj(Bufs<T> B, const DevStatus* __restrict__ st,
                                                 const double* __restrict__ sc) {
  if (st->done) return;
  const int nxt = 1 - int(st->step & 1);
  const T* __restrict__ ph = nxt ? B.phi[1] : B.phi[0];
  T* __restrict__ v = nxt ? B.vel[1] : B.vel[0];
  const T m = (T)sc[5];
  const long n = (long)B.Nx * B.Ny;
  BEC_SITES(n) {
    const int j = (int)(k_ / B.Nx), i = (int)(k_ - (long)j * B.Nx);
    const long o = (long)(j + 2) * B.pitch + (i + 2);
#pragma unroll
    for (int comp = 0; comp < 2; ++comp) {
      const long k = comp * B.plane + o;
      v[k] = v[k] - m * ph[k];
    }
  }
}

// Observables of the current field: {E density, |psi|^2, Re(psi* L_z psi)} summed.
template <class T>
__global__ void __launch_bounds__(256) bec_obs(Bufs<T> B, Coeffs cf, DevStatus* st, double* partials, int nlaunch) {
  const int cur = int(st->step & 1);
  const T* __restrict__ ph = cur ? B.phi[1] : B.phi[0];
  const double h = cf.h, d1 = 1.0 / (12.0 * h);
  double v[3] = {0.0, 0.0, 0.0};
  const long n = (long)B.Nx * B.Ny;
  BEC_SITES(n) {
    const int j = (int)(k_ / B.Nx), i = (int)(k_ - (long)j * B.Nx);
    const long o = (long)(j + 2) * B.pitch + (i + 2);
    double f[2], dx[2], dy[2];
    for (int comp = 0; comp < 2; ++comp) {
      const T* p = ph + comp * B.plane + o;
      f[comp] = p[0];
      dx[comp] = d1 * (((double)p[-2] - (double)p[2]) + 8.0 * ((double)p[1] - (double)p[-1]));
      dy[comp] = d1 * (((double)p[-2 * B.pitch] - (double)p[2 * B.pitch]) +
                       8.0 * ((double)p[B.pitch] - (double)p[-B.pitch]));
    }
    const double x = (i - 0.5 * (B.Nx - 1)) * h, y = (j - 0.5 * (B.Ny - 1)) * h;
    const double rho = f[0] * f[0] + f[1] * f[1];
    const double lz = f[0] * (x * dy[1] - y * dx[1]) - f[1] * (x * dy[0] - y * dx[0]);
    v[0] += 0.5 * (dx[0] * dx[0] + dy[0] * dy[0] + dx[1] * dx[1] + dy[1] * dy[1]) + 0.5 * (x * x + y * y) * rho +
            0.5 * cf.p[0] * rho * rho - cf.p[1] * lz;
    v[1] += rho;
    v[2] += lz;
  }
  reduce_n_to<3, 256>(v, partials, &st->counter_obs, nlaunch, st->obs);
}

#undef BEC_SITES

}  // namespace ss
