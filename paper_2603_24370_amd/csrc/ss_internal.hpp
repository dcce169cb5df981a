// Internal definitions shared by the host API and the HIP kernels of libss.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ss {

constexpr int kHalo = 2;          // Sec. 3.1: default halo width two
constexpr int kMaxWindow = 128;   // largest stall-rule window accepted by the API
// Ring of energies for the stall rule. It is longer than the largest window, so
// the entry of step s - W is never the slot that step s overwrites.
constexpr int kHistLen = 2 * kMaxWindow;
constexpr int kMaxComp = 4;
constexpr int kNumParams = 6;  // theory parameters packed for the kernels

// Device-resident state of one flow (written only by kernels, read by the host
// through a stream-ordered copy).
struct DevStatus {
  double E;          // E_h of the field at the last arrest test
  double E_prev;     // energy the next arrest test compares with
  double gmax;       // max |G| at the last arrest test
  double eval_E;     // result slots of ss_energy_grad
  double eval_gmax;
  double grad_tol;   // stop rules (used when minimise != 0)
  double rel_e_tol;
  long long max_steps;
  long long step;        // RK4 steps started since set_field
  long long n_arrests;
  int arrest;            // 1 if the last arrest test fired
  int done;              // stop reason once a stop rule held (SS_STOP_*), else 0
  int nonfinite;         // non-finite count of the last test
  int window;
  int minimise;          // 1: the arrest pass applies the stop rules
  unsigned counter;      // last-block counter of the arrest pass
  unsigned counter_obs;  // last-block counter of the observable passes
  int fresh;             // set when a run is armed: its first test is of the field
                         // the last run ended on (or a fresh one), whose arrest is decided
  double e_target;       // minimise stops once E <= e_target (-inf: never)
  double hist[kHistLen]; // E at step s is kept at hist[s % kHistLen]
  double obs[16];        // observable sums (see ss_api)
};

// Field buffers of one context, in the device layout: component planes of
// (Ny + 4) rows of `pitch` elements; element (c, j, i) at c*plane + (j+2)*pitch + (i+2).
template <class T>
struct Bufs {
  T* phi[2];   // ping-pong field
  T* vel[2];   // ping-pong fictitious velocity
  T* a1;       // stage-1 acceleration
  T* a2;       // stage-2 acceleration
  T* q;        // a1 + 2 a2 + 2 a3
  long pitch;
  long plane;
  int Nx, Ny;
  // demagnetising potential of the stage point a pass evaluates (FP64, padded
  // plane of row length psi_pitch = Nx + 4, zero outside the interior); null
  // when the theory has no demagnetising term
  const double* psi;
  long psi_pitch;
};

// Theory constants packed for the kernels.
struct Coeffs {
  double h, dt;
  double p[kNumParams];  // AH: {lambda}; CM: {J, D, K, B, Dy, mu_d}; BS: {kappa, mu^2}
};

// Passes of one RK4 step and the single-evaluation variants.
enum Pass : int {
  kP1 = 0,     // stage 1: a1 = -G(phi), energy, arrest test and stop rules
  kP2 = 1,     // stage 2: a2 = -G(phi + dt/2 v)
  kP3 = 2,     // stage 3: q  = a1 + 2 a2 + 2 a3, a3 = -G(phi + dt/2 v + dt^2/4 a1)
  kP4 = 3,     // stage 4: a4 = -G(phi + dt v + dt^2/2 a2); phi', v'
  kEval = 4,   // G and E of a given field; flow state untouched
  kCheck = 5,  // arrest test of the current field only (after a run of steps)
  // Gradient flow, and velocity Verlet in its stored-force form, keep the force
  // a = -G of the current field in one of two force buffers (a1, a2 by step parity):
  kPrime = 6,  // arrest test of the current field, as kCheck, and its force stored
  kGF = 8,     // gradient flow: phi' = phi + dt^2/2 a, a' = -G(phi'), E_h(phi')
  kVVA = 12,   // velocity Verlet: phi' = phi + dt v + dt^2/2 a, a' = -G(phi'),
               //   v' = v + dt/2 (a + a'), E_h(phi'); then the arrest test of phi'
  // Velocity Verlet in kick-drift-kick form (large lattices and batches): within
  // a run the velocity buffer holds u = v + dt/2 a of the current field (the
  // next half-step velocity), so a step reads and writes the field and u only.
  kVV = 7,          // phi' = phi + dt u, G' = G(phi'), v' = u - dt/2 G' (tangent
                    //   to phi' for unit fields), u' = v' - dt/2 G', E_h(phi');
                    //   then the arrest test of phi'
  kVVStart = 9,     // start of a run: u = v - dt/2 G(phi), and the arrest test
                    //   of the current field as kCheck
  kVVRestart = 10,  // before a step that follows an arrest (v = 0): u = -dt/2 G(phi)
  kVVEnd = 11,      // end of a run: v = u + dt/2 G(phi), or 0 after an arrest
  // Gradient flow on the lattice theories keeps only the field: a step tests the
  // field it reads and writes the next one.
  kGD = 13,       // E_h(phi), G(phi) and the stop rules of phi (no arrest); writes
                  //   phi' = phi - tau G(phi) (tau = dt^2/2; on the unit sphere for
                  //   unit fields); the step advances unless a rule fired
  kGDCheck = 14,  // end of a run: E_h and G of the current field, tested without arrest
};

// The pass writes a new field and tests it (its finalise advances the step first).
constexpr bool advances_first(int pass) { return pass == kVV || pass == kVVA || pass == kGF; }
// The pass reduces energy, max |G| and a non-finite count.
constexpr bool reduces(int pass) {
  return pass == kP1 || pass == kEval || pass == kCheck || pass == kPrime || advances_first(pass) ||
         pass == kVVStart || pass == kGD || pass == kGDCheck;
}
// The pass's status update takes no arrest decision (gradient flow has no velocity).
constexpr bool no_arrest(int pass) { return pass == kGF || pass == kGD || pass == kGDCheck; }
// The pass evaluates G at a stage point phi + cv v + ca a (stage_coeffs) rather
// than at the current field.
constexpr bool staged(int pass) { return pass == kP2 || pass == kP3 || pass == kP4 || advances_first(pass); }
constexpr bool stage_reads_v(int pass) { return staged(pass) && pass != kGF; }
constexpr bool stage_reads_a(int pass) { return pass == kP3 || pass == kP4 || pass == kGF || pass == kVVA; }
// The pass reads the arrest flag: RK4 stages 2-4 and the stored-force velocity
// Verlet step start from rest after an arrest, and the kick-drift-kick end of
// run sets v = 0.
constexpr bool uses_arrest(int pass) {
  return pass == kP2 || pass == kP3 || pass == kP4 || pass == kVVA || pass == kVVEnd;
}
// The pass writes the velocity buffer of the current field in place (each site
// by the thread that reads it): the velocity Verlet passes around the steps.
constexpr bool vv_in_place(int pass) { return pass == kVVStart || pass == kVVRestart || pass == kVVEnd; }
// Passes launched once per run (or after an arrest) on one tile shape, whatever
// the context's tile.
constexpr bool fixed_tile(int pass) { return vv_in_place(pass) || pass == kGDCheck; }

// Coefficients of the stage point phi + cv v + ca a of a pass. After an arrest
// the RK4 stages 2-4 and the stored-force velocity Verlet step start from rest
// (cv = 0); the kick-drift-kick u already carries the arrest (kVVRestart).
template <class T, int PASS>
__device__ __forceinline__ void stage_coeffs(T dt, bool arrest, T& cv, T& ca) {
  cv = T(0);
  ca = T(0);
  if (PASS == kP2) cv = T(0.5) * dt;
  if (PASS == kP3) { cv = T(0.5) * dt; ca = T(0.25) * dt * dt; }
  if (PASS == kP4 || PASS == kVVA) { cv = dt; ca = T(0.5) * dt * dt; }
  if (PASS == kVV) cv = dt;
  if (PASS == kGF) ca = T(0.5) * dt * dt;
  if (arrest) cv = T(0);
}

// Map a launched workgroup id to a tile so that the workgroups one XCD receives
// (ids congruent mod 8 go to the same XCD) cover a contiguous range of tiles
// and share their halos in that XCD's L2.
__device__ __forceinline__ int xcd_tile(int b, int nlaunch) {
  const int per = nlaunch >> 3;
  return (b & 7) * per + (b >> 3);
}

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

__device__ __forceinline__ double wave_max(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o, 64));
  return x;
}

__device__ __forceinline__ int wave_isum(int x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// Workgroup reduction of (sum, max, count) in a fixed order; the result is valid
// in thread 0. `red` needs 3 * (blockDim/64) doubles of LDS.
template <int NT>
__device__ __forceinline__ void block_reduce3(double& s, double& m, int& n, double* red) {
  constexpr int NW = NT / 64;
  const int lane = threadIdx.x & 63;
  const int w = (threadIdx.y * blockDim.x + threadIdx.x) >> 6;
  s = wave_sum(s);
  m = wave_max(m);
  n = wave_isum(n);
  if (lane == 0) {
    red[w] = s;
    red[NW + w] = m;
    red[2 * NW + w] = (double)n;
  }
  __syncthreads();
  if (w == 0 && lane == 0) {
    double ss = 0.0, mm = 0.0, nn = 0.0;
    for (int k = 0; k < NW; ++k) {
      ss += red[k];
      mm = fmax(mm, red[NW + k]);
      nn += red[2 * NW + k];
    }
    s = ss;
    m = mm;
    n = (int)nn;
  }
}

}  // namespace ss
