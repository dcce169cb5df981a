// Address- and undefined-behaviour-sanitizer run of the FP64 oracle.
//
// TEST INFRASTRUCTURE ONLY: built by the test-suite with g++ together with
// oracle.cpp and the sanitizers, then run. It calls every exported oracle
// function on small lattices of each theory (the sanitizers then check every
// array access and arithmetic operation the oracle makes) and prints "ok".
#include <cmath>
#include <cstdio>
#include <vector>

extern "C" {
int or_components(int theory);
double or_deriv_at(const double* phi, int Nx, int Ny, double h, int C, int c, int j, int i, int axis);
double or_energy(int theory, int Nx, int Ny, double h, const double* p, const double* phi);
void or_energy_density(int theory, int Nx, int Ny, double h, const double* p, const double* phi, double* dens);
void or_energy_complex(int theory, int Nx, int Ny, double h, const double* p, const double* re, const double* im,
                       double* out);
void or_gradient(int theory, int mode, int Nx, int Ny, double h, const double* p, const double* phi, double* G);
void or_acceleration(int theory, int mode, int Nx, int Ny, double h, const double* p, const double* phi,
                     double* a);
void or_flow(int theory, int mode, int Nx, int Ny, double h, const double* p, double courant, double* phi,
             double* v, double* E_cur, int n_steps, long* n_arrests);
void or_minimise(int theory, int mode, int Nx, int Ny, double h, const double* p, double courant, double* phi,
                 double* v, double grad_tol, double rel_e_tol, int window, long max_steps, double* info);
void or_flow_scheme(int theory, int mode, int scheme, int Nx, int Ny, double h, const double* p, double courant,
                    double* phi, double* v, double* E_cur, int n_steps, long* n_arrests);
void or_minimise_scheme(int theory, int mode, int scheme, int Nx, int Ny, double h, const double* p,
                        double courant, double* phi, double* v, double grad_tol, double rel_e_tol, int window,
                        long max_steps, double* info);
void or_observables_ah(int Nx, int Ny, double h, const double* p, const double* phi, double* out);
void or_observables_cm(int Nx, int Ny, double h, const double* p, const double* phi, double* out);
void or_observables_unit(int theory, int Nx, int Ny, double h, const double* p, const double* phi, double* out);
void or_observables_bec(int Nx, int Ny, double h, const double* p, const double* phi, double* out);
void or_poisson(int Nx, int Ny, double h, const double* rhs, double* psi);
}

namespace {

// a smooth, deterministic field with a unit-length option (no random generator needed)
std::vector<double> field(int C, int Nx, int Ny, bool unit) {
  std::vector<double> f((size_t)C * (Ny + 4) * (Nx + 4));
  for (int c = 0; c < C; ++c)
    for (int j = 0; j < Ny + 4; ++j)
      for (int i = 0; i < Nx + 4; ++i)
        f[((size_t)c * (Ny + 4) + j) * (Nx + 4) + i] = std::sin(0.37 * i + 0.91 * j + 1.3 * c) + 0.2 * c;
  if (unit)
    for (int j = 0; j < Ny + 4; ++j)
      for (int i = 0; i < Nx + 4; ++i) {
        double r = 0.0;
        for (int c = 0; c < C; ++c) r += f[((size_t)c * (Ny + 4) + j) * (Nx + 4) + i] * f[((size_t)c * (Ny + 4) + j) * (Nx + 4) + i];
        r = std::sqrt(r);
        for (int c = 0; c < C; ++c) f[((size_t)c * (Ny + 4) + j) * (Nx + 4) + i] /= r;
      }
  return f;
}

int check_theory(int theory, const double* p, int Nx, int Ny) {
  const int C = or_components(theory);
  const double h = 0.3;
  const bool unit = theory == 1 || theory == 4 || theory == 5;
  std::vector<double> phi = field(C, Nx, Ny, unit), zero(phi.size(), 0.0), G(phi.size()), a(phi.size());
  std::vector<double> dens((size_t)Nx * Ny), out(8), info(6);
  double acc = or_energy(theory, Nx, Ny, h, p, phi.data());
  or_energy_density(theory, Nx, Ny, h, p, phi.data(), dens.data());
  or_energy_complex(theory, Nx, Ny, h, p, phi.data(), zero.data(), out.data());
  acc += out[0] + or_deriv_at(phi.data(), Nx, Ny, h, C, C - 1, Ny - 1, Nx - 1, 1);
  for (int mode = 0; mode < 2; ++mode) {
    or_gradient(theory, mode, Nx, Ny, h, p, phi.data(), G.data());
    or_acceleration(theory, mode, Nx, Ny, h, p, phi.data(), a.data());
    std::vector<double> f2 = phi, v(phi.size(), 0.0);
    double E = or_energy(theory, Nx, Ny, h, p, f2.data());
    long na = 0;
    or_flow(theory, mode, Nx, Ny, h, p, 0.5, f2.data(), v.data(), &E, 3, &na);
    std::vector<double> f3 = phi, v3(phi.size(), 0.0);
    or_minimise(theory, mode, Nx, Ny, h, p, 0.5, f3.data(), v3.data(), 0.0, 1e-3, 2, 6, info.data());
    acc += G[G.size() / 2] + a[a.size() / 3] + E + info[0];
    for (int scheme = 1; scheme < 3; ++scheme) {
      std::vector<double> f4 = phi, v4(phi.size(), 0.0), f5 = phi, v5(phi.size(), 0.0);
      double E4 = or_energy(theory, Nx, Ny, h, p, f4.data());
      or_flow_scheme(theory, mode, scheme, Nx, Ny, h, p, 0.5, f4.data(), v4.data(), &E4, 3, &na);
      or_minimise_scheme(theory, mode, scheme, Nx, Ny, h, p, 0.5, f5.data(), v5.data(), 0.0, 1e-3, 2, 6,
                         info.data());
      acc += E4 + info[0];
    }
  }
  if (theory == 0) or_observables_ah(Nx, Ny, h, p, phi.data(), out.data());
  if (theory == 1) or_observables_cm(Nx, Ny, h, p, phi.data(), out.data());
  if (theory == 4 || theory == 5) or_observables_unit(theory, Nx, Ny, h, p, phi.data(), out.data());
  if (theory == 6) or_observables_bec(Nx, Ny, h, p, phi.data(), out.data());
  acc += out[0];
  return std::isfinite(acc) ? 0 : 1;
}

}  // namespace

int main() {
  const double p_ah[1] = {0.8}, p_cm[4] = {1.1, 0.9, 0.2, 0.5}, p_toy[2] = {1.3, 0.1}, p_bs[2] = {0.9, 0.2};
  int bad = 0;
  bad += check_theory(0, p_ah, 9, 7);
  bad += check_theory(1, p_cm, 8, 10);
  bad += check_theory(2, p_toy, 5, 6);
  bad += check_theory(3, p_toy, 6, 5);
  bad += check_theory(4, p_bs, 7, 8);
  const double p_cmx[6] = {1.0, 0.9, 0.3, 0.1, -0.9, 0.7}, p_bec[3] = {1.2, 0.6, 2.0};
  bad += check_theory(5, p_cmx, 9, 8);
  bad += check_theory(6, p_bec, 8, 9);
  std::vector<double> rhs(7 * 6, 0.3), psi(7 * 6, 0.0);
  or_poisson(7, 6, 0.3, rhs.data(), psi.data());
  if (!std::isfinite(psi[20])) ++bad;
  if (bad) {
    std::printf("non-finite result\n");
    return 1;
  }
  std::printf("ok\n");
  return 0;
}
