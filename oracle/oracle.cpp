// FP64 CPU oracle for the soliton energy-minimisation flow.
//
// TEST INFRASTRUCTURE ONLY. Nothing in the product library links, includes or
// calls this file; only the test-suite, the smoke check and the CPU-baseline
// leg of the benchmark load it. It is built with g++ (never hipcc), runs on one
// thread, and is written for clarity, not speed.
//
// What it computes (paper: "soliton_solver", arXiv 2603.24370):
//   * Lattice: rectangular Nx x Ny interior with a fixed halo of width 2
//     (Sec. 3.1). Field arrays are planar (C, Ny+4, Nx+4), x fastest.
//   * First derivative: the 4th-order central stencil of eq. (1), along x
//     and, "analogously", along y.
//   * Discrete energy E_h = h^2 * sum over interior sites of the continuum
//     density with partial derivatives replaced by eq. (1) (Sec. 3.2). The
//     densities are Tab. 1 (Abelian Higgs) and eq. (5) without the
//     demagnetising term (chiral magnet).
//   * Gradient G = h^-2 dE_h/dphi at interior sites, the force of eq. (3),
//     formed by differentiating E_h site by site and scattering each site's
//     contribution onto the stencil points it read (chain rule).
//   * Arrested Newton flow, eq. (3)-(4): classical fourth-order Runge-Kutta on
//     the first-order system (phi, phidot) with step dt = C*h, C = 0.5
//     (Sec. 3.1); after each step, if E_h rose the velocity is set to zero and
//     the flow continues from the new configuration.
//   * Unit-length constraint of the chiral magnet enforced in every Runge-Kutta
//     stage (Sec. 3.2, constraint projections).
//   * Observables (Sec. 3.3 names energy, topological charge, flux): energy,
//     magnetic flux, topological charge density integral, phase winding,
//     Bogomolny residuals (Abelian Higgs); lattice charge by finite
//     differences and by the Berg-Luescher solid-angle sum (chiral magnet).
//
// Readings where the paper is silent are listed in the project design notes;
// in short: two forms of the gradient (the exact dE_h/dphi, and the continuum
// Euler-Lagrange expression evaluated with eq. (1)-(2)), Dirichlet halo held at its initial values, u = e = 1 and D = grad - iA for
// the Abelian Higgs model, strict ">" in the arrest test, energies compared in
// FP64.
//
// Parity pins: see the test-suite (stencil exactness, complex-step and
// finite-difference gradient checks, the discrete Bogomolny identity, the
// Bogomolny bound E = pi|N|, integer charges, RK4 amplification on a harmonic
// toy theory, symmetry invariants).

#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <limits>
#include <vector>

namespace {

enum Theory { TH_AH = 0, TH_CM = 1, TH_TOY = 2, TH_TOY_OFFSET = 3, TH_BS = 4, TH_CMX = 5, TH_BEC = 6 };

int n_components(int theory) {
  switch (theory) {
    case TH_AH: return 4;   // psi_1, psi_2, A_1, A_2
    case TH_CM: return 3;   // n_1, n_2, n_3
    case TH_TOY: return 1;  // one real scalar per site
    case TH_TOY_OFFSET: return 1;
    case TH_BS: return 3;   // m_1, m_2, m_3
    case TH_CMX: return 3;  // chiral magnet with a general DMI and demagnetisation
    case TH_BEC: return 2;  // Re psi, Im psi
  }
  return -1;
}

struct Lat {
  int Nx, Ny;
  double h;
  long W, H;  // padded width and height
  Lat(int nx, int ny, double hh) : Nx(nx), Ny(ny), h(hh), W(nx + 4), H(ny + 4) {}
  long at(int c, int j, int i) const { return ((long)c * H + (j + 2)) * W + (i + 2); }
  long plane() const { return W * H; }
  bool interior(int j, int i) const { return i >= 0 && i < Nx && j >= 0 && j < Ny; }
};

// eq. (1): weight of f(s + m e_axis) in D f(s), for m = -2..2 (times 1/h).
const double kW[5] = {1.0 / 12.0, -8.0 / 12.0, 0.0, 8.0 / 12.0, -1.0 / 12.0};

template <class T>
T deriv(const T* f, const Lat& L, int c, int j, int i, int axis) {
  int di = axis == 0 ? 1 : 0, dj = axis == 1 ? 1 : 0;
  T acc = T(0);
  for (int m = -2; m <= 2; ++m) {
    if (m == 0) continue;
    acc += kW[m + 2] * f[L.at(c, j + m * dj, i + m * di)];
  }
  return acc / L.h;
}

// eq. (2): 4th-order central second derivative along one axis.
const double kW2[5] = {-1.0 / 12.0, 16.0 / 12.0, -30.0 / 12.0, 16.0 / 12.0, -1.0 / 12.0};

template <class T>
T deriv2(const T* f, const Lat& L, int c, int j, int i, int axis) {
  int di = axis == 0 ? 1 : 0, dj = axis == 1 ? 1 : 0;
  T acc = T(0);
  for (int m = -2; m <= 2; ++m) acc += kW2[m + 2] * f[L.at(c, j + m * dj, i + m * di)];
  return acc / (L.h * L.h);
}

// Mixed derivative d_x d_y: eq. (1) along x applied to eq. (1) along y.
template <class T>
T deriv_xy(const T* f, const Lat& L, int c, int j, int i) {
  T acc = T(0);
  for (int m = -2; m <= 2; ++m)
    for (int n = -2; n <= 2; ++n) {
      if (m == 0 || n == 0) continue;
      acc += kW[m + 2] * kW[n + 2] * f[L.at(c, j + n, i + m)];
    }
  return acc / (L.h * L.h);
}

// Values and first derivatives of all components at one site.
template <class T>
struct Jet {
  T f[4];
  T d[2][4];  // d[axis][component]
  double x, y;  // position of the site (for the BEC's trap and rotation)
};

// Site coordinates: cell-centred, the origin at the lattice centre.
double site_x(const Lat& L, int i) { return (i - 0.5 * (L.Nx - 1)) * L.h; }
double site_y(const Lat& L, int j) { return (j - 0.5 * (L.Ny - 1)) * L.h; }

template <class T>
Jet<T> jet_at(const T* phi, const Lat& L, int C, int j, int i) {
  Jet<T> J;
  J.x = site_x(L, i);
  J.y = site_y(L, j);
  for (int c = 0; c < C; ++c) {
    J.f[c] = phi[L.at(c, j, i)];
    J.d[0][c] = deriv(phi, L, c, j, i, 0);
    J.d[1][c] = deriv(phi, L, c, j, i, 1);
  }
  return J;
}

// --- Abelian Higgs (Tab. 1, u = e = 1, D = grad - i A) ---------------------
// With psi = psi_1 + i psi_2:  D_k psi = (d_k psi_1 + A_k psi_2) + i (d_k psi_2 - A_k psi_1).
// e = 1/2 |D psi|^2 + 1/2 B^2 + lambda/8 (1 - |psi|^2)^2,  B = d_1 A_2 - d_2 A_1.
template <class T>
T ah_density(const Jet<T>& J, double lambda) {
  T p1 = J.f[0], p2 = J.f[1], a1 = J.f[2], a2 = J.f[3];
  T Re1 = J.d[0][0] + a1 * p2, Im1 = J.d[0][1] - a1 * p1;
  T Re2 = J.d[1][0] + a2 * p2, Im2 = J.d[1][1] - a2 * p1;
  T B = J.d[0][3] - J.d[1][2];
  T W = 1.0 - (p1 * p1 + p2 * p2);
  return 0.5 * (Re1 * Re1 + Im1 * Im1 + Re2 * Re2 + Im2 * Im2) + 0.5 * B * B +
         (lambda / 8.0) * W * W;
}

// Partial derivatives of the density: g[c] = de/dphi_c, F[axis][c] = de/d(D_axis phi_c).
void ah_partials(const Jet<double>& J, double lambda, double g[4], double F[2][4]) {
  double p1 = J.f[0], p2 = J.f[1], a1 = J.f[2], a2 = J.f[3];
  double Re1 = J.d[0][0] + a1 * p2, Im1 = J.d[0][1] - a1 * p1;
  double Re2 = J.d[1][0] + a2 * p2, Im2 = J.d[1][1] - a2 * p1;
  double B = J.d[0][3] - J.d[1][2];
  double W = 1.0 - (p1 * p1 + p2 * p2);
  // d/dpsi_1: Im_k depends on -A_k psi_1; potential gives lambda/4 W (-2 psi_1).
  g[0] = -a1 * Im1 - a2 * Im2 - 0.5 * lambda * W * p1;
  g[1] = a1 * Re1 + a2 * Re2 - 0.5 * lambda * W * p2;
  g[2] = Re1 * p2 - Im1 * p1;
  g[3] = Re2 * p2 - Im2 * p1;
  F[0][0] = Re1; F[0][1] = Im1; F[0][2] = 0.0; F[0][3] = B;
  F[1][0] = Re2; F[1][1] = Im2; F[1][2] = -B;  F[1][3] = 0.0;
}

// --- Chiral magnet (eq. (5); the demagnetising term is added below) --------
// e = J/2 sum_k |D_k n|^2 + D sum_k d_k . (n x D_k n) + K (1 - n_3^2) + B (1 - n_3),
// DMI vectors for k = 1, 2 (there is no z-derivative in 2-D): bulk d_k = e_k, or the
// Heusler (D_2d) pair d_1 = e_1, d_2 = -e_2; Dy is D times the sign of d_2 . e_2.
template <class T>
T cm_density(const Jet<T>& Jt, double J, double D, double K, double Bz, double Dy) {
  const T* n = Jt.f;
  T ex = 0.0;
  for (int k = 0; k < 2; ++k)
    for (int c = 0; c < 3; ++c) ex += Jt.d[k][c] * Jt.d[k][c];
  // e_1 . (n x d_1 n) = n_2 d_1 n_3 - n_3 d_1 n_2;  e_2 . (n x d_2 n) = n_3 d_2 n_1 - n_1 d_2 n_3
  T dmi = D * (n[1] * Jt.d[0][2] - n[2] * Jt.d[0][1]) + Dy * (n[2] * Jt.d[1][0] - n[0] * Jt.d[1][2]);
  return 0.5 * J * ex + dmi + K * (1.0 - n[2] * n[2]) + Bz * (1.0 - n[2]);
}

void cm_partials(const Jet<double>& Jt, double J, double D, double K, double Bz, double Dy, double g[4],
                 double F[2][4]) {
  const double* n = Jt.f;
  g[0] = -Dy * Jt.d[1][2];
  g[1] = D * Jt.d[0][2];
  g[2] = -D * Jt.d[0][1] + Dy * Jt.d[1][0] - 2.0 * K * n[2] - Bz;
  g[3] = 0.0;
  F[0][0] = J * Jt.d[0][0];
  F[0][1] = J * Jt.d[0][1] - D * n[2];
  F[0][2] = J * Jt.d[0][2] + D * n[1];
  F[1][0] = J * Jt.d[1][0] + Dy * n[2];
  F[1][1] = J * Jt.d[1][1];
  F[1][2] = J * Jt.d[1][2] - Dy * n[0];
  F[0][3] = F[1][3] = 0.0;
}

// --- Baby Skyrme (Tab. 1, standard potential) --------------------------------
// e = 1/2 sum_k |D_k m|^2 + kappa^2/4 sum_{i,j} |D_i m x D_j m|^2 + mu2 (1 - m_3);
// the double sum has the two equal terms (i, j) = (1, 2), (2, 1), so the Skyrme term
// is kappa^2/2 |D_1 m x D_2 m|^2.
template <class T>
void cross(const T* a, const T* b, T* out) {
  out[0] = a[1] * b[2] - a[2] * b[1];
  out[1] = a[2] * b[0] - a[0] * b[2];
  out[2] = a[0] * b[1] - a[1] * b[0];
}

template <class T>
T bs_density(const Jet<T>& Jt, double kappa, double mu2) {
  T s[3];
  cross(Jt.d[0], Jt.d[1], s);
  T grad2 = 0.0, skyrme = 0.0;
  for (int c = 0; c < 3; ++c) {
    grad2 += Jt.d[0][c] * Jt.d[0][c] + Jt.d[1][c] * Jt.d[1][c];
    skyrme += s[c] * s[c];
  }
  return 0.5 * grad2 + 0.5 * kappa * kappa * skyrme + mu2 * (1.0 - Jt.f[2]);
}

// de/dm = -mu2 e_3;  de/d(D_1 m) = D_1 m + kappa^2 D_2 m x s;  de/d(D_2 m) = D_2 m + kappa^2 s x D_1 m,
// with s = D_1 m x D_2 m (d|s|^2/2 = s . (dD_1 m x D_2 m) = dD_1 m . (D_2 m x s), likewise for D_2 m).
void bs_partials(const Jet<double>& Jt, double kappa, double mu2, double g[4], double F[2][4]) {
  double s[3], ws[3], su[3];
  cross(Jt.d[0], Jt.d[1], s);
  cross(Jt.d[1], s, ws);
  cross(s, Jt.d[0], su);
  const double k2 = kappa * kappa;
  for (int c = 0; c < 3; ++c) {
    g[c] = 0.0;
    F[0][c] = Jt.d[0][c] + k2 * ws[c];
    F[1][c] = Jt.d[1][c] + k2 * su[c];
  }
  g[2] = -mu2;
  g[3] = F[0][3] = F[1][3] = 0.0;
}

// --- Rotating trapped Bose-Einstein condensate (Sec. 4.3) --------------------
// Trap units (hbar = m = omega = 1), psi = u + i w:
//   e = 1/2 |grad psi|^2 + 1/2 r^2 |psi|^2 + g/2 |psi|^4 - Omega Re(psi* L_z psi),
//   L_z = -i (x d_y - y d_x), so Re(psi* L_z psi) = u (x w_y - y w_x) - w (x u_y - y u_x)
//   (the imaginary part is a total derivative). p = {g, Omega, N}; N = h^2 sum |psi|^2
// is held fixed by the flow.
template <class T>
T bec_density(const Jet<T>& J, double g, double Om) {
  const T u = J.f[0], w = J.f[1];
  const T ux = J.d[0][0], uy = J.d[1][0], wx = J.d[0][1], wy = J.d[1][1];
  const T rho = u * u + w * w;
  const double r2 = J.x * J.x + J.y * J.y;
  const T lz = u * (J.x * wy - J.y * wx) - w * (J.x * uy - J.y * ux);
  return 0.5 * (ux * ux + uy * uy + wx * wx + wy * wy) + 0.5 * r2 * rho + 0.5 * g * rho * rho - Om * lz;
}

void bec_partials(const Jet<double>& J, double g, double Om, double gg[4], double F[2][4]) {
  const double u = J.f[0], w = J.f[1];
  const double ux = J.d[0][0], uy = J.d[1][0], wx = J.d[0][1], wy = J.d[1][1];
  const double rho = u * u + w * w, r2 = J.x * J.x + J.y * J.y, x = J.x, y = J.y;
  gg[0] = r2 * u + 2.0 * g * rho * u - Om * (x * wy - y * wx);
  gg[1] = r2 * w + 2.0 * g * rho * w + Om * (x * uy - y * ux);
  F[0][0] = ux - Om * y * w;
  F[1][0] = uy + Om * x * w;
  F[0][1] = wx + Om * y * u;
  F[1][1] = wy - Om * x * u;
}

// --- Harmonic toy theories (tests of the integrator and stop rules only) ------
// e = m2/2 phi^2, and e = m2/2 phi^2 + e0 (a floor under the energy, so that its
// relative change over a window tends to zero and the stall rule can fire).
template <class T>
T toy_density(const Jet<T>& Jt, double m2) { return 0.5 * m2 * Jt.f[0] * Jt.f[0]; }

template <class T>
T density(int theory, const Jet<T>& Jt, const double* p) {
  switch (theory) {
    case TH_AH: return ah_density(Jt, p[0]);
    case TH_CM: return cm_density(Jt, p[0], p[1], p[2], p[3], p[1]);
    case TH_CMX: return cm_density(Jt, p[0], p[1], p[2], p[3], p[4]);
    case TH_TOY_OFFSET: return toy_density(Jt, p[0]) + p[1];
    case TH_BS: return bs_density(Jt, p[0], p[1]);
    case TH_BEC: return bec_density(Jt, p[0], p[1]);
    default: return toy_density(Jt, p[0]);
  }
}

void partials(int theory, const Jet<double>& Jt, const double* p, double g[4], double F[2][4]) {
  for (int c = 0; c < 4; ++c) g[c] = F[0][c] = F[1][c] = 0.0;
  switch (theory) {
    case TH_AH: ah_partials(Jt, p[0], g, F); break;
    case TH_CM: cm_partials(Jt, p[0], p[1], p[2], p[3], p[1], g, F); break;
    case TH_CMX: cm_partials(Jt, p[0], p[1], p[2], p[3], p[4], g, F); break;
    case TH_BS: bs_partials(Jt, p[0], p[1], g, F); break;
    case TH_BEC: bec_partials(Jt, p[0], p[1], g, F); break;
    default: g[0] = p[0] * Jt.f[0]; break;
  }
}

// --- Euler-Lagrange form of the gradient ------------------------------------
// G = de/dphi - sum_k d_k [de/d(d_k phi)] with the outer derivative expanded by the
// product rule, first derivatives from eq. (1), pure second derivatives from
// eq. (2) and the mixed derivative d_x d_y from eq. (1) applied twice. This is the
// continuum functional derivative evaluated pointwise with the paper's stencils.
struct ELJet {
  double f[4];
  double d[2][4];   // first derivatives d[axis][c]
  double dd[2][4];  // pure second derivatives dd[axis][c]
  double dxy[4];    // mixed derivative
  double x, y;      // site position
};

ELJet el_jet_at(const double* phi, const Lat& L, int C, int j, int i) {
  ELJet J;
  J.x = site_x(L, i);
  J.y = site_y(L, j);
  for (int c = 0; c < 4; ++c) {
    J.f[c] = J.d[0][c] = J.d[1][c] = J.dd[0][c] = J.dd[1][c] = J.dxy[c] = 0.0;
  }
  for (int c = 0; c < C; ++c) {
    J.f[c] = phi[L.at(c, j, i)];
    for (int a = 0; a < 2; ++a) {
      J.d[a][c] = deriv(phi, L, c, j, i, a);
      J.dd[a][c] = deriv2(phi, L, c, j, i, a);
    }
    J.dxy[c] = deriv_xy(phi, L, c, j, i);
  }
  return J;
}

// Abelian Higgs:
//   G_psi1 = -A.Q - lambda/2 W psi1 - lap psi1 - (div A) psi2 - A.grad psi2
//   G_psi2 = +A.P - lambda/2 W psi2 - lap psi2 + (div A) psi1 + A.grad psi1
//   G_A1   = P1 psi2 - Q1 psi1 + d_2 B,   d_2 B = d_x d_y A2 - d_yy A1
//   G_A2   = P2 psi2 - Q2 psi1 - d_1 B,   d_1 B = d_xx A2 - d_x d_y A1
void ah_el(const ELJet& J, double lambda, double G[4]) {
  double p1 = J.f[0], p2 = J.f[1], a1 = J.f[2], a2 = J.f[3];
  double P1 = J.d[0][0] + a1 * p2, Q1 = J.d[0][1] - a1 * p1;
  double P2 = J.d[1][0] + a2 * p2, Q2 = J.d[1][1] - a2 * p1;
  double W = 1.0 - (p1 * p1 + p2 * p2);
  double lap1 = J.dd[0][0] + J.dd[1][0], lap2 = J.dd[0][1] + J.dd[1][1];
  double divA = J.d[0][2] + J.d[1][3];
  double Agp1 = a1 * J.d[0][0] + a2 * J.d[1][0], Agp2 = a1 * J.d[0][1] + a2 * J.d[1][1];
  G[0] = -(a1 * Q1 + a2 * Q2) - 0.5 * lambda * W * p1 - lap1 - divA * p2 - Agp2;
  G[1] = (a1 * P1 + a2 * P2) - 0.5 * lambda * W * p2 - lap2 + divA * p1 + Agp1;
  G[2] = P1 * p2 - Q1 * p1 + (J.dxy[3] - J.dd[1][2]);
  G[3] = P2 * p2 - Q2 * p1 - (J.dd[0][3] - J.dxy[2]);
}

// Chiral magnet: G = -J lap n + 2 sum_k D_k (d_k n x e_k) - (2 K n3 + B) e3, D_1 = D, D_2 = Dy.
void cm_el(const ELJet& Jt, double J, double D, double K, double Bz, double Dy, double G[4]) {
  double lap[3];
  for (int c = 0; c < 3; ++c) lap[c] = Jt.dd[0][c] + Jt.dd[1][c];
  // d_1 n x e_1 = (0, d1n3, -d1n2);  d_2 n x e_2 = (-d2n3, 0, d2n1)
  G[0] = -J * lap[0] + 2.0 * Dy * (-Jt.d[1][2]);
  G[1] = -J * lap[1] + 2.0 * D * (Jt.d[0][2]);
  G[2] = -J * lap[2] + 2.0 * (-D * Jt.d[0][1] + Dy * Jt.d[1][0]) - 2.0 * K * Jt.f[2] - Bz;
  G[3] = 0.0;
}

// Baby Skyrme: G = de/dm - d_1 [de/d(d_1 m)] - d_2 [de/d(d_2 m)] with
//   d_1 [d_1 m + k^2 d_2 m x s] = m_xx + k^2 (m_xy x s + d_2 m x s_x),  s_x = m_xx x d_2 m + d_1 m x m_xy,
//   d_2 [d_2 m + k^2 s x d_1 m] = m_yy + k^2 (s_y x d_1 m + s x m_xy),  s_y = m_xy x d_2 m + d_1 m x m_yy.
void bs_el(const ELJet& J, double kappa, double mu2, double G[4]) {
  const double* u = J.d[0];
  const double* w = J.d[1];
  const double* mxx = J.dd[0];
  const double* myy = J.dd[1];
  const double* mxy = J.dxy;
  double s[3], sx[3], sy[3], t1[3], t2[3];
  cross(u, w, s);
  cross(mxx, w, t1);
  cross(u, mxy, t2);
  for (int c = 0; c < 3; ++c) sx[c] = t1[c] + t2[c];
  cross(mxy, w, t1);
  cross(u, myy, t2);
  for (int c = 0; c < 3; ++c) sy[c] = t1[c] + t2[c];
  double a1[3], a2[3], b1[3], b2[3];
  cross(mxy, s, a1);
  cross(w, sx, a2);
  cross(sy, u, b1);
  cross(s, mxy, b2);
  const double k2 = kappa * kappa;
  for (int c = 0; c < 3; ++c) {
    const double d1F1 = mxx[c] + k2 * (a1[c] + a2[c]);
    const double d2F2 = myy[c] + k2 * (b1[c] + b2[c]);
    G[c] = -d1F1 - d2F2;
  }
  G[2] -= mu2;
  G[3] = 0.0;
}

// BEC: G_u = -lap u + r^2 u + 2 g |psi|^2 u - 2 Omega (x d_y - y d_x) w,
//      G_w = -lap w + r^2 w + 2 g |psi|^2 w + 2 Omega (x d_y - y d_x) u
// (the rotation term's two parts, from the density and from its flux, are equal).
void bec_el(const ELJet& J, double g, double Om, double G[4]) {
  const double u = J.f[0], w = J.f[1], x = J.x, y = J.y;
  const double rho = u * u + w * w, r2 = x * x + y * y;
  const double Dw = x * J.d[1][1] - y * J.d[0][1], Du = x * J.d[1][0] - y * J.d[0][0];
  G[0] = -(J.dd[0][0] + J.dd[1][0]) + r2 * u + 2.0 * g * rho * u - 2.0 * Om * Dw;
  G[1] = -(J.dd[0][1] + J.dd[1][1]) + r2 * w + 2.0 * g * rho * w + 2.0 * Om * Du;
  G[2] = G[3] = 0.0;
}

// Neumaier-compensated sum.
struct KSum {
  double s = 0.0, c = 0.0;
  void add(double x) {
    double t = s + x;
    if (std::fabs(s) >= std::fabs(x)) c += (s - t) + x; else c += (x - t) + s;
    s = t;
  }
  double value() const { return s + c; }
};

// --- Demagnetisation (eq. (5)-(6)) ------------------------------------------
// In units where mu_0 M_s^2 is the coefficient mu_d, the magnetostatic potential psi
// solves Laplace(psi) = div n (the in-plane divergence; no z-dependence in 2-D) with
// psi = 0 outside the interior, and the energy gains mu_d/2 |grad psi|^2 per site.
// Discretely: div and grad by eq. (1), the Laplacian by eq. (2) along each axis.

// One plane of scalars on the padded lattice (component 0 of a 1-component layout).
struct Plane {
  Lat L;
  std::vector<double> v;
  explicit Plane(const Lat& l) : L(l), v(l.plane(), 0.0) {}
  double& at(int j, int i) { return v[L.at(0, j, i)]; }
  double at(int j, int i) const { return v[L.at(0, j, i)]; }
};

// eq. (1) derivative of a plane along an axis at an interior site (the plane is zero outside).
double plane_deriv(const Plane& P, int j, int i, int axis) { return deriv(P.v.data(), P.L, 0, j, i, axis); }

// y = -Laplace_h(x) on the interior (x zero outside), eq. (2) along both axes.
void neg_laplacian(const Plane& x, Plane& y) {
  for (int j = 0; j < x.L.Ny; ++j)
    for (int i = 0; i < x.L.Nx; ++i)
      y.at(j, i) = -(deriv2(x.v.data(), x.L, 0, j, i, 0) + deriv2(x.v.data(), x.L, 0, j, i, 1));
}

double dot_interior(const Plane& a, const Plane& b) {
  KSum s;
  for (int j = 0; j < a.L.Ny; ++j)
    for (int i = 0; i < a.L.Nx; ++i) s.add(a.at(j, i) * b.at(j, i));
  return s.value();
}

// Solve Laplace_h(psi) = rhs by conjugate gradients on the symmetric positive
// definite -Laplace_h (zero outside the interior), to a relative residual of 1e-14.
void poisson_solve(const Plane& rhs, Plane& psi) {
  const Lat& L = rhs.L;
  Plane r(L), d(L), Ad(L);
  std::fill(psi.v.begin(), psi.v.end(), 0.0);
  for (int j = 0; j < L.Ny; ++j)
    for (int i = 0; i < L.Nx; ++i) r.at(j, i) = -rhs.at(j, i);  // b of  (-Laplace) psi = -rhs
  d = r;
  double rr = dot_interior(r, r);
  const double stop = 1e-28 * rr;
  for (long it = 0; it < 20L * (L.Nx + L.Ny) + 1000 && rr > stop && rr > 0.0; ++it) {
    neg_laplacian(d, Ad);
    const double alpha = rr / dot_interior(d, Ad);
    for (int j = 0; j < L.Ny; ++j)
      for (int i = 0; i < L.Nx; ++i) {
        psi.at(j, i) += alpha * d.at(j, i);
        r.at(j, i) -= alpha * Ad.at(j, i);
      }
    const double rr1 = dot_interior(r, r);
    for (int j = 0; j < L.Ny; ++j)
      for (int i = 0; i < L.Nx; ++i) d.at(j, i) = r.at(j, i) + (rr1 / rr) * d.at(j, i);
    rr = rr1;
  }
}

// psi of a field n: Laplace_h psi = d_x n_1 + d_y n_2 (the halo of n holds the boundary values).
void demag_potential(const Lat& L, const double* n, Plane& psi) {
  Plane rhs(L);
  for (int j = 0; j < L.Ny; ++j)
    for (int i = 0; i < L.Nx; ++i) rhs.at(j, i) = deriv(n, L, 0, j, i, 0) + deriv(n, L, 1, j, i, 1);
  poisson_solve(rhs, psi);
}

// mu_d / 2 h^2 sum |grad psi|^2
double demag_energy(const Lat& L, double mu_d, const double* n) {
  Plane psi(L);
  demag_potential(L, n, psi);
  KSum s;
  for (int j = 0; j < L.Ny; ++j)
    for (int i = 0; i < L.Nx; ++i) {
      const double gx = plane_deriv(psi, j, i, 0), gy = plane_deriv(psi, j, i, 1);
      s.add(gx * gx + gy * gy);
    }
  return 0.5 * mu_d * L.h * L.h * s.value();
}

bool has_demag(int theory, const double* p) { return theory == TH_CMX && p[5] != 0.0; }

// Euler-Lagrange demagnetising force: mu_d (d_x psi, d_y psi, 0) added to G.
void add_demag_el(const Lat& L, double mu_d, const double* n, double* G) {
  Plane psi(L);
  demag_potential(L, n, psi);
  for (int j = 0; j < L.Ny; ++j)
    for (int i = 0; i < L.Nx; ++i) {
      G[L.at(0, j, i)] += mu_d * plane_deriv(psi, j, i, 0);
      G[L.at(1, j, i)] += mu_d * plane_deriv(psi, j, i, 1);
    }
}

// Exact derivative of the discrete demagnetising energy: with B_c the eq. (1)
// derivatives restricted to the interior (antisymmetric), L the eq. (2) Laplacian and
// M = B_x^T B_x + B_y^T B_y, E_d = mu_d/2 h^2 psi^T M psi and psi = L^-1 (B_x n_1 + B_y n_2),
// so h^-2 dE_d/dn_c = mu_d B_c^T L^-1 M psi = -mu_d B_c chi with L chi = M psi.
void add_demag_exact(const Lat& L, double mu_d, const double* n, double* G) {
  Plane psi(L), gx(L), gy(L), Mpsi(L), chi(L);
  demag_potential(L, n, psi);
  for (int j = 0; j < L.Ny; ++j)
    for (int i = 0; i < L.Nx; ++i) {
      gx.at(j, i) = plane_deriv(psi, j, i, 0);
      gy.at(j, i) = plane_deriv(psi, j, i, 1);
    }
  for (int j = 0; j < L.Ny; ++j)
    for (int i = 0; i < L.Nx; ++i) Mpsi.at(j, i) = -(plane_deriv(gx, j, i, 0) + plane_deriv(gy, j, i, 1));
  poisson_solve(Mpsi, chi);
  for (int j = 0; j < L.Ny; ++j)
    for (int i = 0; i < L.Nx; ++i) {
      G[L.at(0, j, i)] += -mu_d * plane_deriv(chi, j, i, 0);
      G[L.at(1, j, i)] += -mu_d * plane_deriv(chi, j, i, 1);
    }
}

void gradient_el(int theory, const Lat& L, const double* p, const double* phi, double* G) {
  int C = n_components(theory);
  std::memset(G, 0, sizeof(double) * C * L.plane());
  for (int j = 0; j < L.Ny; ++j)
    for (int i = 0; i < L.Nx; ++i) {
      ELJet J = el_jet_at(phi, L, C, j, i);
      double g[4] = {0.0, 0.0, 0.0, 0.0};
      if (theory == TH_AH) ah_el(J, p[0], g);
      else if (theory == TH_CM) cm_el(J, p[0], p[1], p[2], p[3], p[1], g);
      else if (theory == TH_CMX) cm_el(J, p[0], p[1], p[2], p[3], p[4], g);
      else if (theory == TH_BS) bs_el(J, p[0], p[1], g);
      else if (theory == TH_BEC) bec_el(J, p[0], p[1], g);
      else g[0] = p[0] * J.f[0];
      for (int c = 0; c < C; ++c) G[L.at(c, j, i)] = g[c];
    }
  if (has_demag(theory, p)) add_demag_el(L, p[5], phi, G);
}

double energy(int theory, const Lat& L, const double* p, const double* phi) {
  int C = n_components(theory);
  KSum s;
  for (int j = 0; j < L.Ny; ++j)
    for (int i = 0; i < L.Nx; ++i) s.add(density(theory, jet_at(phi, L, C, j, i), p));
  const double e_demag = has_demag(theory, p) ? demag_energy(L, p[5], phi) : 0.0;
  return L.h * L.h * s.value() + e_demag;
}

// G = h^-2 dE_h/dphi on interior sites (halo entries set to 0). Scatter form:
// site s contributes de/dphi_c(s) to G_c(s), and de/d(D_k phi_c)(s) * w_m / h to
// G_c(s + m e_k) for every stencil point s + m e_k that is an interior site.
void gradient(int theory, const Lat& L, const double* p, const double* phi, double* G) {
  int C = n_components(theory);
  std::memset(G, 0, sizeof(double) * C * L.plane());
  for (int j = 0; j < L.Ny; ++j)
    for (int i = 0; i < L.Nx; ++i) {
      double g[4], F[2][4];
      partials(theory, jet_at(phi, L, C, j, i), p, g, F);
      for (int c = 0; c < C; ++c) {
        G[L.at(c, j, i)] += g[c];
        for (int m = -2; m <= 2; ++m) {
          if (m == 0) continue;
          double w = kW[m + 2] / L.h;
          if (L.interior(j, i + m)) G[L.at(c, j, i + m)] += F[0][c] * w;
          if (L.interior(j + m, i)) G[L.at(c, j + m, i)] += F[1][c] * w;
        }
      }
    }
  if (has_demag(theory, p)) add_demag_exact(L, p[5], phi, G);
}

void normalise_interior(const Lat& L, double* n) {
  for (int j = 0; j < L.Ny; ++j)
    for (int i = 0; i < L.Nx; ++i) {
      double a = n[L.at(0, j, i)], b = n[L.at(1, j, i)], c = n[L.at(2, j, i)];
      double r = std::sqrt(a * a + b * b + c * c);
      n[L.at(0, j, i)] = a / r; n[L.at(1, j, i)] = b / r; n[L.at(2, j, i)] = c / r;
    }
}

// Remove the component of X along the unit field n at every interior site.
void tangent_project(const Lat& L, const double* n, double* X) {
  for (int j = 0; j < L.Ny; ++j)
    for (int i = 0; i < L.Nx; ++i) {
      double dot = 0.0;
      for (int c = 0; c < 3; ++c) dot += X[L.at(c, j, i)] * n[L.at(c, j, i)];
      for (int c = 0; c < 3; ++c) X[L.at(c, j, i)] -= dot * n[L.at(c, j, i)];
    }
}

// Theories of a unit-vector field (chiral magnet, Baby Skyrme).
bool unit_theory(int theory) { return theory == TH_CM || theory == TH_BS || theory == TH_CMX; }

// Theories whose flow holds a global norm fixed: the BEC's atom number
// N = h^2 sum |psi|^2 (Sec. 4.3), p[2] = N.
bool norm_theory(int theory) { return theory == TH_BEC; }

// Interior sum of a . b over all components.
double interior_dot(const Lat& L, int C, const double* a, const double* b) {
  KSum s;
  for (int c = 0; c < C; ++c)
    for (int j = 0; j < L.Ny; ++j)
      for (int i = 0; i < L.Nx; ++i) s.add(a[L.at(c, j, i)] * b[L.at(c, j, i)]);
  return s.value();
}

// Scale the interior so that h^2 sum |phi|^2 = N (the halo keeps its values).
void normalise_global(const Lat& L, int C, double N, double* phi) {
  const double c = std::sqrt(N / (L.h * L.h * interior_dot(L, C, phi, phi)));
  for (int cc = 0; cc < C; ++cc)
    for (int j = 0; j < L.Ny; ++j)
      for (int i = 0; i < L.Nx; ++i) phi[L.at(cc, j, i)] *= c;
}

// Remove from X its component along phi in the interior inner product (the
// tangent space of the sphere h^2 sum |phi|^2 = N).
void project_global(const Lat& L, int C, const double* phi, double* X) {
  const double m = interior_dot(L, C, phi, X) / interior_dot(L, C, phi, phi);
  for (int c = 0; c < C; ++c)
    for (int j = 0; j < L.Ny; ++j)
      for (int i = 0; i < L.Nx; ++i) X[L.at(c, j, i)] -= m * phi[L.at(c, j, i)];
}

// The force used by the flow: -G at the stage point; for the chiral magnet the
// stage point is first put back on the unit sphere and -G is projected onto its
// tangent plane; for the BEC the stage point is scaled to the atom number N and
// -G is projected onto the tangent space of that sphere (the chemical potential
// mu = <phi, G> / <phi, phi> is the multiplier of the constraint).
void acceleration(int theory, int mode, const Lat& L, const double* p, const double* stage, double* a) {
  int C = n_components(theory);
  long n = (long)C * L.plane();
  std::vector<double> s(stage, stage + n);
  if (unit_theory(theory)) normalise_interior(L, s.data());
  if (norm_theory(theory)) normalise_global(L, C, p[2], s.data());
  if (mode == 0) gradient(theory, L, p, s.data(), a);
  else gradient_el(theory, L, p, s.data(), a);
  if (unit_theory(theory)) tangent_project(L, s.data(), a);
  if (norm_theory(theory)) project_global(L, C, s.data(), a);
  for (long k = 0; k < n; ++k) a[k] = -a[k];
}

double max_abs_interior(const Lat& L, int C, const double* X) {
  double m = 0.0;
  for (int c = 0; c < C; ++c)
    for (int j = 0; j < L.Ny; ++j)
      for (int i = 0; i < L.Nx; ++i) m = std::fmax(m, std::fabs(X[L.at(c, j, i)]));
  return m;
}

// One classical RK4 step of  phi' = v,  v' = a(phi)  with step dt (interior sites;
// the halo of phi is never changed and the halo of v stays zero).
void rk4_step(int theory, int mode, const Lat& L, const double* p, double dt, double* phi, double* v) {
  int C = n_components(theory);
  long n = (long)C * L.plane();
  std::vector<double> k1p(n), k1v(n), k2p(n), k2v(n), k3p(n), k3v(n), k4p(n), k4v(n), y(n);
  // stage 1
  for (long k = 0; k < n; ++k) k1p[k] = v[k];
  acceleration(theory, mode, L, p, phi, k1v.data());
  // stage 2
  for (long k = 0; k < n; ++k) { k2p[k] = v[k] + 0.5 * dt * k1v[k]; y[k] = phi[k] + 0.5 * dt * k1p[k]; }
  acceleration(theory, mode, L, p, y.data(), k2v.data());
  // stage 3
  for (long k = 0; k < n; ++k) { k3p[k] = v[k] + 0.5 * dt * k2v[k]; y[k] = phi[k] + 0.5 * dt * k2p[k]; }
  acceleration(theory, mode, L, p, y.data(), k3v.data());
  // stage 4
  for (long k = 0; k < n; ++k) { k4p[k] = v[k] + dt * k3v[k]; y[k] = phi[k] + dt * k3p[k]; }
  acceleration(theory, mode, L, p, y.data(), k4v.data());
  for (int c = 0; c < C; ++c)
    for (int j = 0; j < L.Ny; ++j)
      for (int i = 0; i < L.Nx; ++i) {
        long k = L.at(c, j, i);
        phi[k] += dt / 6.0 * (k1p[k] + 2.0 * k2p[k] + 2.0 * k3p[k] + k4p[k]);
        v[k] += dt / 6.0 * (k1v[k] + 2.0 * k2v[k] + 2.0 * k3v[k] + k4v[k]);
      }
  if (unit_theory(theory)) {
    normalise_interior(L, phi);
    tangent_project(L, phi, v);
  }
  if (norm_theory(theory)) {
    normalise_global(L, C, p[2], phi);
    project_global(L, C, phi, v);
  }
}

// The other integrators of the flow (Sec. 3.2 names RK4 as one choice of explicit
// integrator and contrasts the method with first-order descent):
//   scheme 1, velocity Verlet (Stoermer-Verlet) of phi'' = a(phi):
//       phi' = phi + dt v + dt^2/2 a(phi),   v' = v + dt/2 (a(phi) + a(phi'));
//   scheme 2, gradient flow phi' = -G(phi) by explicit Euler with step tau = dt^2/2,
//       the step velocity Verlet takes from rest (after an arrest):
//       phi' = phi + tau a(phi)   (the velocity stays zero).
// For the chiral magnet the force is the projected one of acceleration(); phi' is
// renormalised before a(phi') is taken, and v' is projected on the tangent plane
// at phi', as after an RK4 step.
enum Scheme { SCHEME_RK4 = 0, SCHEME_VV = 1, SCHEME_GF = 2 };

void one_pass_step(int theory, int mode, int scheme, const Lat& L, const double* p, double dt, double* phi,
                   double* v) {
  int C = n_components(theory);
  long n = (long)C * L.plane();
  std::vector<double> a0(n), a1(n);
  acceleration(theory, mode, L, p, phi, a0.data());
  for (int c = 0; c < C; ++c)
    for (int j = 0; j < L.Ny; ++j)
      for (int i = 0; i < L.Nx; ++i) {
        long k = L.at(c, j, i);
        if (scheme == SCHEME_VV) phi[k] += dt * v[k] + 0.5 * dt * dt * a0[k];
        else phi[k] += 0.5 * dt * dt * a0[k];
      }
  if (unit_theory(theory)) normalise_interior(L, phi);
  if (norm_theory(theory)) normalise_global(L, C, p[2], phi);
  if (scheme != SCHEME_VV) return;
  acceleration(theory, mode, L, p, phi, a1.data());
  for (int c = 0; c < C; ++c)
    for (int j = 0; j < L.Ny; ++j)
      for (int i = 0; i < L.Nx; ++i) {
        long k = L.at(c, j, i);
        v[k] += 0.5 * dt * (a0[k] + a1[k]);
      }
  if (unit_theory(theory)) tangent_project(L, phi, v);
  if (norm_theory(theory)) project_global(L, C, phi, v);
}

void step_scheme(int theory, int mode, int scheme, const Lat& L, const double* p, double dt, double* phi, double* v) {
  if (scheme == SCHEME_RK4) rk4_step(theory, mode, L, p, dt, phi, v);
  else one_pass_step(theory, mode, scheme, L, p, dt, phi, v);
}

double wrap_angle(double a) {
  const double pi = 3.14159265358979323846;
  while (a > pi) a -= 2.0 * pi;
  while (a <= -pi) a += 2.0 * pi;
  return a;
}

}  // namespace

extern "C" {

int or_components(int theory) { return n_components(theory); }

double or_deriv_at(const double* phi, int Nx, int Ny, double h, int C, int c, int j, int i, int axis) {
  (void)C;
  Lat L(Nx, Ny, h);
  return deriv(phi, L, c, j, i, axis);
}

double or_energy(int theory, int Nx, int Ny, double h, const double* p, const double* phi) {
  return energy(theory, Lat(Nx, Ny, h), p, phi);
}

// Solve Laplace_h psi = rhs (eq. (2) along each axis, psi = 0 outside the interior);
// rhs and psi are (Ny, Nx) arrays of the interior.
void or_poisson(int Nx, int Ny, double h, const double* rhs, double* psi) {
  Lat L(Nx, Ny, h);
  Plane r(L), x(L);
  for (int j = 0; j < Ny; ++j)
    for (int i = 0; i < Nx; ++i) r.at(j, i) = rhs[(long)j * Nx + i];
  poisson_solve(r, x);
  for (int j = 0; j < Ny; ++j)
    for (int i = 0; i < Nx; ++i) psi[(long)j * Nx + i] = x.at(j, i);
}

// Energy density e at every interior site, written to dens[(Ny, Nx)].
void or_energy_density(int theory, int Nx, int Ny, double h, const double* p, const double* phi,
                       double* dens) {
  Lat L(Nx, Ny, h);
  int C = n_components(theory);
  for (int j = 0; j < Ny; ++j)
    for (int i = 0; i < Nx; ++i) dens[(long)j * Nx + i] = density(theory, jet_at(phi, L, C, j, i), p);
}

// Complex-step energy: returns E_h(re + i im) as (out[0], out[1]).
void or_energy_complex(int theory, int Nx, int Ny, double h, const double* p, const double* re,
                       const double* im, double* out) {
  typedef std::complex<double> Z;
  Lat L(Nx, Ny, h);
  int C = n_components(theory);
  long n = (long)C * L.plane();
  std::vector<Z> z(n);
  for (long k = 0; k < n; ++k) z[k] = Z(re[k], im[k]);
  Z s(0.0, 0.0);
  for (int j = 0; j < Ny; ++j)
    for (int i = 0; i < Nx; ++i) s += density(theory, jet_at(z.data(), L, C, j, i), p);
  s *= h * h;
  out[0] = s.real();
  out[1] = s.imag();
}

// mode 0: G = h^-2 dE_h/dphi (exact, scatter form); mode 1: Euler-Lagrange form.
void or_gradient(int theory, int mode, int Nx, int Ny, double h, const double* p, const double* phi,
                 double* G) {
  if (mode == 0) gradient(theory, Lat(Nx, Ny, h), p, phi, G);
  else gradient_el(theory, Lat(Nx, Ny, h), p, phi, G);
}

// The flow's force a(phi) (normalised + projected for the chiral magnet).
void or_acceleration(int theory, int mode, int Nx, int Ny, double h, const double* p,
                     const double* phi, double* a) {
  acceleration(theory, mode, Lat(Nx, Ny, h), p, phi, a);
}

// n_steps of the flow with the given integrator (0 = RK4, 1 = velocity Verlet,
// 2 = gradient flow). On entry *E_cur = E_h(phi). After every step: E' = E_h(phi');
// for the second-order schemes, if E' > *E_cur the velocity is zeroed (*n_arrests
// incremented; eq. (4)); then *E_cur = E'. Gradient flow has no velocity to arrest.
void or_flow_scheme(int theory, int mode, int scheme, int Nx, int Ny, double h, const double* p, double courant,
                    double* phi, double* v, double* E_cur, int n_steps, long* n_arrests) {
  Lat L(Nx, Ny, h);
  int C = n_components(theory);
  long n = (long)C * L.plane();
  double dt = courant * h;
  for (int s = 0; s < n_steps; ++s) {
    step_scheme(theory, mode, scheme, L, p, dt, phi, v);
    double E = energy(theory, L, p, phi);
    if (scheme != SCHEME_GF && E > *E_cur) {
      for (long k = 0; k < n; ++k) v[k] = 0.0;
      ++*n_arrests;
    }
    *E_cur = E;
  }
}

// n_steps of arrested Newton flow, eq. (3)-(4), integrated by RK4.
void or_flow(int theory, int mode, int Nx, int Ny, double h, const double* p, double courant, double* phi,
             double* v, double* E_cur, int n_steps, long* n_arrests) {
  or_flow_scheme(theory, mode, SCHEME_RK4, Nx, Ny, h, p, courant, phi, v, E_cur, n_steps, n_arrests);
}

// Minimise from (phi, v) with the given integrator (as or_flow_scheme). Stops at the first state whose
// (projected) gradient satisfies max|G| < grad_tol, or whose energy changed by at
// most rel_e_tol * |E| over the last `window` steps (window > 0), or after
// max_steps steps. info = {E, gmax, steps, arrests, converged(1/0), reason}
// with reason 1 = gradient, 2 = energy stall, 0 = max steps.
void or_minimise_scheme(int theory, int mode, int scheme, int Nx, int Ny, double h, const double* p,
                        double courant, double* phi, double* v, double grad_tol, double rel_e_tol, int window,
                        long max_steps, double* info) {
  Lat L(Nx, Ny, h);
  int C = n_components(theory);
  long n = (long)C * L.plane();
  double dt = courant * h;
  std::vector<double> a(n);
  std::vector<double> hist;
  double E = energy(theory, L, p, phi);
  long arrests = 0, step = 0;
  int reason = 0;
  for (;; ++step) {
    acceleration(theory, mode, L, p, phi, a.data());
    double gmax = max_abs_interior(L, C, a.data());
    hist.push_back(E);
    info[0] = E; info[1] = gmax;
    if (gmax < grad_tol) { reason = 1; break; }
    if (window > 0 && step >= window &&
        std::fabs(E - hist[step - window]) <= rel_e_tol * std::fabs(E)) { reason = 2; break; }
    if (step >= max_steps) break;
    step_scheme(theory, mode, scheme, L, p, dt, phi, v);
    double En = energy(theory, L, p, phi);
    if (scheme != SCHEME_GF && En > E) { for (long k = 0; k < n; ++k) v[k] = 0.0; ++arrests; }
    E = En;
  }
  info[2] = (double)step;
  info[3] = (double)arrests;
  info[4] = reason != 0 ? 1.0 : 0.0;
  info[5] = (double)reason;
}

// Minimise by arrested Newton flow integrated by RK4.
void or_minimise(int theory, int mode, int Nx, int Ny, double h, const double* p, double courant, double* phi,
                 double* v, double grad_tol, double rel_e_tol, int window, long max_steps, double* info) {
  or_minimise_scheme(theory, mode, SCHEME_RK4, Nx, Ny, h, p, courant, phi, v, grad_tol, rel_e_tol, window,
                     max_steps, info);
}

// Observables of the Abelian Higgs field.
// out = {E, flux, N_rho, N_wind, R1, R2}:
//   flux   = h^2 sum B,
//   N_rho  = h^2 sum rho, rho = [B W + 2 (P1 Q2 - Q1 P2)] / (2 pi), where D_k psi = P_k + i Q_k,
//   N_wind = phase winding of psi along the ring of outermost interior sites,
//            counter-clockwise, with each step wrapped to (-pi, pi],
//   R1     = h^2 sum |(P1 - Q2) + i (Q1 + P2)|^2,  R2 = h^2 sum (B - W/2)^2.
// At lambda = 1:  E = pi N_rho + (R1 + R2)/2  for every field (Bogomolny identity).
void or_observables_ah(int Nx, int Ny, double h, const double* p, const double* phi, double* out) {
  Lat L(Nx, Ny, h);
  const double pi = 3.14159265358979323846;
  KSum sE, sB, sR, sR1, sR2;
  for (int j = 0; j < Ny; ++j)
    for (int i = 0; i < Nx; ++i) {
      Jet<double> J = jet_at(phi, L, 4, j, i);
      double p1 = J.f[0], p2 = J.f[1], a1 = J.f[2], a2 = J.f[3];
      double P1 = J.d[0][0] + a1 * p2, Q1 = J.d[0][1] - a1 * p1;
      double P2 = J.d[1][0] + a2 * p2, Q2 = J.d[1][1] - a2 * p1;
      double B = J.d[0][3] - J.d[1][2];
      double W = 1.0 - (p1 * p1 + p2 * p2);
      sE.add(ah_density(J, p[0]));
      sB.add(B);
      sR.add((B * W + 2.0 * (P1 * Q2 - Q1 * P2)) / (2.0 * pi));
      double r1re = P1 - Q2, r1im = Q1 + P2, r2 = B - 0.5 * W;
      sR1.add(r1re * r1re + r1im * r1im);
      sR2.add(r2 * r2);
    }
  double h2 = h * h;
  // ring of outermost interior sites, counter-clockwise starting at (0, 0)
  std::vector<std::pair<int, int>> ring;
  for (int i = 0; i < Nx - 1; ++i) ring.push_back({0, i});
  for (int j = 0; j < Ny - 1; ++j) ring.push_back({j, Nx - 1});
  for (int i = Nx - 1; i > 0; --i) ring.push_back({Ny - 1, i});
  for (int j = Ny - 1; j > 0; --j) ring.push_back({j, 0});
  KSum sw;
  for (size_t k = 0; k < ring.size(); ++k) {
    auto a = ring[k], b = ring[(k + 1) % ring.size()];
    double tha = std::atan2(phi[L.at(1, a.first, a.second)], phi[L.at(0, a.first, a.second)]);
    double thb = std::atan2(phi[L.at(1, b.first, b.second)], phi[L.at(0, b.first, b.second)]);
    sw.add(wrap_angle(thb - tha));
  }
  out[0] = h2 * sE.value();
  out[1] = h2 * sB.value();
  out[2] = h2 * sR.value();
  out[3] = sw.value() / (2.0 * pi);
  out[4] = h2 * sR1.value();
  out[5] = h2 * sR2.value();
}

// Observables of the chiral magnet.
// out = {E, Q_fd, Q_bl}:
//   Q_fd = h^2 / (4 pi) sum n . (D_1 n x D_2 n) over interior sites,
//   Q_bl = Berg-Luescher: over every plaquette of the padded lattice (corners
//          a=(i,j), b=(i+1,j), c=(i+1,j+1), d=(i,j+1)) the signed solid angles of the
//          triangles (a,b,c) and (a,c,d), each 2 atan2(a.(b x c), 1 + a.b + b.c + c.a),
//          summed and divided by 4 pi.
void or_observables_unit(int theory, int Nx, int Ny, double h, const double* p, const double* phi, double* out);

void or_observables_cm(int Nx, int Ny, double h, const double* p, const double* phi, double* out) {
  or_observables_unit(TH_CM, Nx, Ny, h, p, phi, out);
}

// Observables of a unit-vector field of either theory (as for the chiral magnet).
void or_observables_unit(int theory, int Nx, int Ny, double h, const double* p, const double* phi, double* out) {
  Lat L(Nx, Ny, h);
  const double pi = 3.14159265358979323846;
  KSum sE, sQ, sBL;
  for (int j = 0; j < Ny; ++j)
    for (int i = 0; i < Nx; ++i) {
      Jet<double> J = jet_at(phi, L, 3, j, i);
      sE.add(density(theory, J, p));
      const double* n = J.f;
      const double* u = J.d[0];
      const double* w = J.d[1];
      double cx = u[1] * w[2] - u[2] * w[1], cy = u[2] * w[0] - u[0] * w[2], cz = u[0] * w[1] - u[1] * w[0];
      sQ.add(n[0] * cx + n[1] * cy + n[2] * cz);
    }
  auto vec = [&](int j, int i, double* o) {
    for (int c = 0; c < 3; ++c) o[c] = phi[L.at(c, j, i)];
  };
  auto tri = [&](const double* a, const double* b, const double* c) {
    double bxc[3] = {b[1] * c[2] - b[2] * c[1], b[2] * c[0] - b[0] * c[2], b[0] * c[1] - b[1] * c[0]};
    double num = a[0] * bxc[0] + a[1] * bxc[1] + a[2] * bxc[2];
    double den = 1.0 + (a[0] * b[0] + a[1] * b[1] + a[2] * b[2]) + (b[0] * c[0] + b[1] * c[1] + b[2] * c[2]) +
                 (c[0] * a[0] + c[1] * a[1] + c[2] * a[2]);
    return 2.0 * std::atan2(num, den);
  };
  for (int j = -2; j < Ny + 1; ++j)
    for (int i = -2; i < Nx + 1; ++i) {
      double a[3], b[3], c[3], d[3];
      vec(j, i, a); vec(j, i + 1, b); vec(j + 1, i + 1, c); vec(j + 1, i, d);
      sBL.add(tri(a, b, c));
      sBL.add(tri(a, c, d));
    }
  // the energy is that of eq. (5), demagnetising term included
  out[0] = h * h * sE.value() + (has_demag(theory, p) ? demag_energy(L, p[5], phi) : 0.0);
  out[1] = h * h * sQ.value() / (4.0 * pi);
  out[2] = sBL.value() / (4.0 * pi);
}

// BEC observables (Sec. 4.3): out = {E_h, N = h^2 sum |psi|^2, L = h^2 sum Re(psi* L_z psi)}
// with L_z = -i (x d_y - y d_x) and eq. (1) derivatives.
void or_observables_bec(int Nx, int Ny, double h, const double* p, const double* phi, double* out) {
  Lat L(Nx, Ny, h);
  KSum sE, sN, sL;
  for (int j = 0; j < Ny; ++j)
    for (int i = 0; i < Nx; ++i) {
      Jet<double> J = jet_at(phi, L, 2, j, i);
      sE.add(bec_density(J, p[0], p[1]));
      const double u = J.f[0], w = J.f[1];
      sN.add(u * u + w * w);
      sL.add(u * (J.x * J.d[1][1] - J.y * J.d[0][1]) - w * (J.x * J.d[1][0] - J.y * J.d[0][0]));
    }
  out[0] = h * h * sE.value();
  out[1] = h * h * sN.value();
  out[2] = h * h * sL.value();
}

}  // extern "C"
