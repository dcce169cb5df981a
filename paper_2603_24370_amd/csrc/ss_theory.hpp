// Per-site physics of the two theories on the device: energy density and the
// Euler-Lagrange gradient, written in complex / vector form.
#pragma once

#include "ss_internal.hpp"

namespace ss {

// Local jet of one component at one site: value and derivatives by eq. (1)-(2).
template <class T>
struct Jet {
  T f, x, y, xx, yy, xy;
};

// Abelian Higgs with u = e = 1, D_k = d_k - i A_k, psi = p + i q (Tab. 1).
//   e = 1/2 sum_k |D_k psi|^2 + 1/2 B^2 + lambda/8 (1 - |psi|^2)^2,   B = d_x A_y - d_y A_x.
// Euler-Lagrange gradient:
//   G_psi = -sum_k D_k D_k psi - lambda/2 (1 - |psi|^2) psi,
//     D_k D_k psi = d_kk psi - i (d_k A_k) psi - 2 i A_k d_k psi - A_k^2 psi;
//   G_Ax = (q d_x p - p d_x q) + A_x |psi|^2 + d_y B,
//   G_Ay = (q d_y p - p d_y q) + A_y |psi|^2 - d_x B.
template <class T>
__device__ __forceinline__ void ah_el_gradient(const Jet<T> (&J)[4], T lambda, T (&G)[4]) {
  const T p = J[0].f, q = J[1].f, ax = J[2].f, ay = J[3].f;
  const T m2 = p * p + q * q;
  const T a2 = ax * ax + ay * ay;
  const T divA = J[2].x + J[3].y;
  const T lap_p = J[0].xx + J[0].yy, lap_q = J[1].xx + J[1].yy;
  const T agp = ax * J[0].x + ay * J[0].y;  // A . grad p
  const T agq = ax * J[1].x + ay * J[1].y;  // A . grad q
  const T pot = T(0.5) * lambda * (T(1) - m2);
  // real and imaginary parts of -(D.D psi) - pot psi
  G[0] = -lap_p - divA * q - T(2) * agq + a2 * p - pot * p;
  G[1] = -lap_q + divA * p + T(2) * agp + a2 * q - pot * q;
  const T dxB = J[3].xx - J[2].xy;  // d_x (d_x A_y - d_y A_x)
  const T dyB = J[3].xy - J[2].yy;  // d_y (d_x A_y - d_y A_x)
  G[2] = (q * J[0].x - p * J[1].x) + ax * m2 + dyB;
  G[3] = (q * J[0].y - p * J[1].y) + ay * m2 - dxB;
}

template <class T>
__device__ __forceinline__ double ah_density(const Jet<T> (&J)[4], double lambda) {
  const double p = J[0].f, q = J[1].f, ax = J[2].f, ay = J[3].f;
  const double rx = (double)J[0].x + ax * q, ix = (double)J[1].x - ax * p;
  const double ry = (double)J[0].y + ay * q, iy = (double)J[1].y - ay * p;
  const double B = (double)J[3].x - (double)J[2].y;
  const double W = 1.0 - (p * p + q * q);
  return 0.5 * (rx * rx + ix * ix + ry * ry + iy * iy) + 0.5 * B * B + 0.125 * lambda * W * W;
}

// Chiral magnet (eq. (5), local terms), unit field n, DMI vectors d_1 = e_1 and
// d_2 = e_2 (bulk, Dy = D) or d_2 = -e_2 (Heusler, Dy = -D):
//   e = J/2 |grad n|^2 + D e_1.(n x d_x n) + Dy e_2.(n x d_y n) + K (1 - n_z^2) + B (1 - n_z),
//   G = -J lap n + 2 D (d_x n x e_1) + 2 Dy (d_y n x e_2) - (2 K n_z + B) e_z   (before projection),
// with d_x n x e_1 = (0, d_x n_z, -d_x n_y) and d_y n x e_2 = (-d_y n_z, 0, d_y n_x). For the
// bulk case the DMI force is -2 D curl n.
template <class T>
__device__ __forceinline__ void cm_el_gradient(const Jet<T> (&J)[4], T Jx, T Dm, T K, T Bz, T Dy, T (&G)[4]) {
  G[0] = -Jx * (J[0].xx + J[0].yy) - T(2) * Dy * J[2].y;
  G[1] = -Jx * (J[1].xx + J[1].yy) + T(2) * Dm * J[2].x;
  G[2] = -Jx * (J[2].xx + J[2].yy) + T(2) * (Dy * J[0].y - Dm * J[1].x) - (T(2) * K * J[2].f + Bz);
  G[3] = T(0);
}

template <class T>
__device__ __forceinline__ double cm_density(const Jet<T> (&J)[4], double Jx, double Dm, double K, double Bz,
                                             double Dy) {
  double ex = 0.0;
#pragma unroll
  for (int c = 0; c < 3; ++c) ex += (double)J[c].x * J[c].x + (double)J[c].y * J[c].y;
  const double nx = J[0].f, ny = J[1].f, nz = J[2].f;
  const double dmi = Dm * (ny * (double)J[2].x - nz * (double)J[1].x) + Dy * (nz * (double)J[0].y - nx * (double)J[2].y);
  return 0.5 * Jx * ex + dmi + K * (1.0 - nz * nz) + Bz * (1.0 - nz);
}

// Baby Skyrme model (Tab. 1) with the standard potential, unit field m:
//   e = 1/2 (|u|^2 + |w|^2) + kappa^2/2 |u x w|^2 + mu^2 (1 - m_z),   u = d_x m, w = d_y m
// (kappa^2/4 sum_ij |d_i m x d_j m|^2 = kappa^2/2 |u x w|^2). The Euler-Lagrange
// derivative, with the Skyrme term's cross products expanded into dot products:
//   G = -lap m - mu^2 e_z - kappa^2 [ m_xx |w|^2 + m_yy |u|^2 - 2 m_xy (u.w)
//         - w (w.m_xx) - u (u.m_yy) + u (w.m_xy) + w (u.m_xy) ]   (before projection).
template <class T>
__device__ __forceinline__ void bs_el_gradient(const Jet<T> (&J)[4], T kappa2, T mu2, T (&G)[4]) {
  T u[3], w[3], mxx[3], myy[3], mxy[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    u[c] = J[c].x; w[c] = J[c].y; mxx[c] = J[c].xx; myy[c] = J[c].yy; mxy[c] = J[c].xy;
  }
  auto dot = [](const T (&a)[3], const T (&b)[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; };
  const T uu = dot(u, u), ww = dot(w, w), uw = dot(u, w);
  const T w_xx = dot(w, mxx), u_yy = dot(u, myy), w_xy = dot(w, mxy), u_xy = dot(u, mxy);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const T sk = mxx[c] * ww + myy[c] * uu - T(2) * mxy[c] * uw - w[c] * w_xx - u[c] * u_yy + u[c] * w_xy + w[c] * u_xy;
    G[c] = -(mxx[c] + myy[c]) - kappa2 * sk;
  }
  G[2] -= mu2;
  G[3] = T(0);
}

template <class T>
__device__ __forceinline__ double bs_density(const Jet<T> (&J)[4], double kappa2, double mu2) {
  double uu = 0.0, ww = 0.0, uw = 0.0;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    uu += (double)J[c].x * J[c].x;
    ww += (double)J[c].y * J[c].y;
    uw += (double)J[c].x * J[c].y;
  }
  return 0.5 * (uu + ww) + 0.5 * kappa2 * (uu * ww - uw * uw) + mu2 * (1.0 - (double)J[2].f);
}

// Theory ids of the kernels' template argument, and what each needs.
constexpr int kAH = 0, kCM = 1, kBS = 2;
constexpr bool unit_field(int TH) { return TH != kAH; }     // |m| = 1, projected forces
constexpr bool el_mixed(int TH) { return TH != kCM; }       // the EL form uses d_x d_y

// Euler-Lagrange gradient and FP64 energy density of theory TH (p: theory parameters).
template <class T, int TH>
__device__ __forceinline__ void el_gradient(const Jet<T> (&J)[4], const double (&p)[kNumParams], T (&G)[4]) {
  if (TH == kAH) ah_el_gradient<T>(J, (T)p[0], G);
  else if (TH == kCM) cm_el_gradient<T>(J, (T)p[0], (T)p[1], (T)p[2], (T)p[3], (T)p[4], G);
  else bs_el_gradient<T>(J, (T)(p[0] * p[0]), (T)p[1], G);
}

template <int TH>
__device__ __forceinline__ double density(const Jet<double> (&J)[4], const double (&p)[kNumParams]) {
  if (TH == kAH) return ah_density<double>(J, p[0]);
  if (TH == kCM) return cm_density<double>(J, p[0], p[1], p[2], p[3], p[4]);
  return bs_density<double>(J, p[0] * p[0], p[1]);
}

}  // namespace ss
