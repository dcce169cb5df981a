/*
 * ss.h -- C ABI of the MI355X (gfx950) soliton energy-minimisation library.
 *
 * The library minimises a discretised energy E_h[phi] of a multi-component
 * field on a 2-D lattice by arrested Newton flow, as set out in
 * "soliton_solver" (arXiv 2603.24370):
 *   - lattice: Nx x Ny interior sites, spacing h, fixed halo of width 2
 *     (Sec. 3.1);
 *   - derivatives: the 4th-order central stencils of eq. (1) and eq. (2);
 *   - flow: eq. (3), phi'' = -grad E_h, integrated as a first-order system in
 *     (phi, phidot) by classical 4th-order Runge-Kutta with dt = C h, C = 0.5
 *     by default (Sec. 3.1-3.2); the flow starts from rest;
 *   - arrest: eq. (4), after a step that raised E_h the velocity is set to zero
 *     and the flow continues from the new configuration;
 *   - constraint: the chiral magnet's unit length is enforced in every
 *     Runge-Kutta stage (Sec. 3.2);
 *   - reductions: energy, convergence norm and observables are reduced on the
 *     GPU (Sec. 3.3), here entirely on the device in FP64.
 *
 * Theories (Tab. 1; eq. (5)-(6)):
 *   "abelian_higgs" (aliases "Abelian Higgs", "Ginzburg-Landau", "GL", "AH"):
 *       C = 4 components (psi_1, psi_2, A_1, A_2), u = e = 1, D = grad - iA,
 *       e = 1/2 |D psi|^2 + 1/2 (d_1 A_2 - d_2 A_1)^2 + lambda/8 (1 - |psi|^2)^2.
 *       params.f = {lambda [, courant]}.
 *   "chiral_magnet" (aliases "Chiral magnet", "CM"):
 *       C = 3 components (n_1, n_2, n_3), |n| = 1, DMI vectors d_1 = e_1 and
 *       d_2 = e_2 (SS_DMI_BULK) or d_2 = -e_2 (SS_DMI_HEUSLER, Sec. 4.2),
 *       e = J/2 |grad n|^2 + D sum_k d_k.(n x d_k n) + K (1 - n_3^2) + B (1 - n_3)
 *           [+ mu_d/2 |grad psi|^2 with demagnetisation].
 *       params.f = {J, D, K, B [, courant]}, or {J, D, K, B, mu_d [, courant]}
 *       with demagnetisation. The demagnetising potential psi of a field n
 *       (eq. (6), in units where mu_0 M_s^2 is mu_d) solves
 *       Laplace_h psi = d_x n_1 + d_y n_2 with psi = 0 outside the interior
 *       (eq. (1) divergence, eq. (2) Laplacian); it is solved on the device by
 *       multigrid-preconditioned conjugate gradients for every field the flow
 *       evaluates (see ss_set_demag_iters). Demagnetisation needs the
 *       Euler-Lagrange gradient and the SS_PLAN_STAGES launch plan, single
 *       contexts (no batches), and the workspace of ss_workspace_bytes_for.
 *   "baby_skyrme" (aliases "Baby Skyrme", "BS"):
 *       C = 3 components (m_1, m_2, m_3), |m| = 1, the standard potential,
 *       e = 1/2 |grad m|^2 + kappa^2/4 sum_ij |d_i m x d_j m|^2 + mu^2 (1 - m_3).
 *       params.f = {kappa, mu^2 [, courant]}. Single contexts only (no batches).
 *   "bec" (aliases "bose_einstein", "Bose-Einstein condensate", "BEC"):
 *       the rotating trapped condensate of Sec. 4.3 in trap units (hbar = m = omega = 1),
 *       C = 2 components (Re psi, Im psi), sites at x_i = (i - (Nx-1)/2) h,
 *       e = 1/2 |grad psi|^2 + 1/2 r^2 |psi|^2 + g/2 |psi|^4 - Omega Re(psi* L_z psi),
 *       L_z = -i (x d_y - y d_x). params.f = {g, Omega, N [, courant]}: the flow
 *       holds the atom number N = h^2 sum |psi|^2 fixed (every stage point is
 *       scaled to N and the force projected on the tangent space of that sphere,
 *       with the chemical potential as multiplier; after each step the field is
 *       scaled and the velocity projected). Euler-Lagrange gradient,
 *       SS_PLAN_STAGES and single contexts only (every integrator); ss_energy_grad returns the
 *       projected gradient at the field scaled to N and the energy of the field as
 *       given.
 *   params.i (optional, ni <= 3) = {grad_mode, dmi_kind, demag}:
 *   grad_mode SS_GRAD_EL (default) evaluates the continuum Euler-Lagrange
 *   derivative with eq. (1)-(2); SS_GRAD_EXACT uses h^-2 dE_h/dphi, the exact
 *   derivative of the discrete energy. dmi_kind SS_DMI_BULK (default) or
 *   SS_DMI_HEUSLER, and demag 0 (default) or 1, apply to the chiral magnet only.
 *
 * Memory layout of every field array passed in or out: planar, component
 * major, rows of x fastest, shape (C, Ny + 4, Nx + 4) including the halo,
 * contiguous; element (c, j, i) of interior site (i, j) is at
 * c * (Ny + 4) * (Nx + 4) + (j + 2) * (Nx + 4) + (i + 2). Element type is
 * float (SS_F32) or double (SS_F64), the context's dtype.
 *
 * Ownership: every device buffer (fields, gradients, the workspace) belongs
 * to the caller; the library never calls hipMalloc. The library owns the
 * host-side context and the HIP graph and stream objects it creates;
 * ss_destroy releases them. The workspace must stay valid and untouched by
 * the caller between ss_create and ss_destroy.
 *
 * Streams: work is queued on the stream given to ss_create (NULL = the
 * default stream). Calls that return host values synchronise that stream.
 *
 * Errors: functions return SS_OK (0), a positive warning, or a negative
 * error code; ss_last_error() gives a thread-local message for the last
 * failure. No exception crosses this boundary. A context is not thread-safe:
 * use one context per host thread.
 */
#ifndef SS_H
#define SS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define SS_OK 0
#define SS_NOT_CONVERGED 1
#define SS_EINVAL (-1)
#define SS_ETHEORY (-2)
#define SS_ESHAPE (-3)
#define SS_EHIP (-4)
#define SS_ENONFINITE (-5)
#define SS_ESTATE (-6)

/* element types */
#define SS_F32 0
#define SS_F64 1

/* theories */
#define SS_THEORY_AH 0
#define SS_THEORY_CM 1
#define SS_THEORY_BS 2
#define SS_THEORY_BEC 3

/* gradient forms */
#define SS_GRAD_EL 0
#define SS_GRAD_EXACT 1

/* DMI vectors of the chiral magnet (params.i[1]) */
#define SS_DMI_BULK 0
#define SS_DMI_HEUSLER 1

/* stop reasons reported by ss_minimise */
#define SS_STOP_NONE 0
#define SS_STOP_GRAD 1
#define SS_STOP_STALL 2
#define SS_STOP_MAXSTEPS 3
#define SS_STOP_NONFINITE 4
#define SS_STOP_TARGET 5

typedef struct ss_ctx ss_ctx;

/* Theory parameters packed as float and int arrays (Sec. 3.1: theory-specific
 * parameters are packed into integer and floating-point arrays). Pointers are
 * host memory, read during the call only. */
typedef struct {
  const double* f;
  int nf;
  const int* i;
  int ni;
} ss_params;

/* Result of a run of flow steps; all values refer to the field at the end. */
typedef struct {
  double energy;      /* E_h of the current field (FP64 reduction) */
  double energy_prev; /* E_h compared against by the next arrest test */
  double gnorm_inf;   /* max |G| over interior sites and components */
  int64_t step;       /* flow steps completed since ss_set_field */
  int64_t n_arrests;  /* arrests since ss_set_field */
  int32_t arrested;   /* 1 if the last arrest test fired */
  int32_t nonfinite;  /* number of non-finite values seen by the last test */
} ss_step_info;

/* Stop rule for ss_minimise. The first rule met ends the run:
 *   gnorm_inf < grad_tol                                    (SS_STOP_GRAD)
 *   window > 0, step >= window and
 *   |E(step) - E(step - window)| <= rel_e_tol |E(step)|     (SS_STOP_STALL)
 *   E(step) <= the context's energy target (ss_set_energy_target)  (SS_STOP_TARGET)
 *   step >= max_steps                                        (SS_STOP_MAXSTEPS)
 * graph_steps: flow steps per replayed HIP graph (0 = library default; an even
 * number). window <= 128. */
typedef struct {
  double grad_tol;
  double rel_e_tol;
  int32_t window;
  int32_t graph_steps;
  int64_t max_steps;
} ss_stop;

typedef struct {
  ss_step_info last; /* state at the stop */
  int32_t reason;    /* SS_STOP_* */
  int32_t converged; /* 1 for SS_STOP_GRAD or SS_STOP_STALL */
} ss_min_info;

/* Observables (FP64). Abelian Higgs: flux = h^2 sum B; n_rho = h^2 sum rho with
 * rho = [B W + 2 (P1 Q2 - Q1 P2)] / (2 pi), D_k psi = P_k + i Q_k, W = 1 - |psi|^2;
 * n_wind = phase winding of psi along the ring of outermost interior sites,
 * counter-clockwise; bogo_r1 = h^2 sum |(P1 - Q2) + i (Q1 + P2)|^2,
 * bogo_r2 = h^2 sum (B - W/2)^2. Chiral magnet: q_fd = h^2/(4 pi) sum
 * n.(D1 n x D2 n); q_bl = Berg-Luescher solid-angle charge over all plaquettes
 * of the padded lattice (also the Baby Skyrme model). BEC (Sec. 4.3): atoms and
 * lz below. energy includes every term of the theory (with the chiral magnet's
 * demagnetising term, from a fresh solve of the current field). Fields that do
 * not apply are 0. */
typedef struct {
  double energy;
  double flux;
  double n_rho;
  double n_wind;
  double bogo_r1;
  double bogo_r2;
  double q_fd;
  double q_bl;
  double gnorm_inf;
  double atoms; /* BEC: N = h^2 sum |psi|^2 */
  double lz;    /* BEC: h^2 sum Re(psi* L_z psi), eq. (1) derivatives */
} ss_obs;

/* Canonical theory id of a name or alias (Sec. 2.3 registry), or SS_ETHEORY. */
int ss_theory_id(const char* name);

/* Number of field components of a theory, or SS_ETHEORY. */
int ss_components(const char* theory);

/* Workspace bytes ss_create needs for this theory, grid and dtype, without
 * demagnetisation. */
int ss_workspace_bytes(const char* theory, int Nx, int Ny, int dtype, size_t* bytes);

/* Workspace bytes ss_create needs for these parameters: ss_workspace_bytes
 * plus, with demagnetisation, the solver's stage point (C planes of the
 * dtype) and its FP64 planes (seven on the lattice, three per coarser level;
 * about 75 bytes per site in all for FP32). Validates params as ss_create
 * does. */
int ss_workspace_bytes_for(const char* theory, int Nx, int Ny, const ss_params* params, int dtype, size_t* bytes);

/* Create a context. Parameters are validated and resolved before any device
 * work (Sec. 3.1). workspace: device memory of at least ss_workspace_bytes_for
 * (= ss_workspace_bytes without demagnetisation), 256-byte aligned. stream: a
 * hipStream_t or NULL. Requires 8 <= Nx, Ny <= 65536 and h > 0. */
int ss_create(const char* theory, int Nx, int Ny, double h, const ss_params* params, int dtype,
              void* workspace, size_t ws_bytes, void* stream, ss_ctx** out);

/* Release a context: wait for its stream, destroy the HIP graph and the
 * capture stream it created (Sec. 3.1: the simulation object owns its
 * buffers; here the caller keeps the device memory and the library the host
 * objects). The workspace may be freed by the caller afterwards. */
void ss_destroy(ss_ctx* ctx);

/* Copy the initial field (device array of the context's dtype and the layout
 * above; its halo holds the fixed boundary values) into the context, start
 * from rest (phidot = 0, Sec. 3.2) and reset step and arrest counters. The
 * array is tightly packed (row pitch Nx + 4 elements); there is no pitch
 * argument. */
int ss_set_field(ss_ctx* ctx, const void* field);

/* Initial field from an analytic ansatz, computed on the device (the paper's
 * "model-specific ansatz", Sec. 4.1), then the same reset as ss_set_field.
 *   Abelian Higgs, kind SS_ANSATZ_VORTICES: n vortices at xy[2k], xy[2k+1]
 *     (host array, lattice coordinates x_i = (i - (Nx-1)/2) h) with windings
 *     w[k] (host array or NULL = all +1):
 *       psi = prod_k tanh(r_k) exp(i w_k theta_k),
 *       A   = sum_k w_k (1 - exp(-r_k^2)) / r_k^2 (-(y - y_k), x - x_k);
 *     the halo holds the pure-gauge vacuum psi = exp(i sum w_k theta_k),
 *     A = sum_k w_k grad theta_k.
 *   BEC, kind SS_ANSATZ_BEC: shape = {R, xi}, n >= 0 vortices at xy with windings
 *     w (NULL = all +1): psi = exp(-r^2 / (2 R^2)) / (sqrt(pi) R) prod_k tanh(r_k / xi)
 *     exp(i w_k theta_k) in the interior, psi = 0 on the halo (the flow scales it to N).
 *   Chiral magnet and Baby Skyrme, kind SS_ANSATZ_SKYRMION: n = 1, xy = centre, shape = {R, gamma},
 *     w = {m} (vorticity, a nonzero integer; NULL = 1; m = -1 is the
 *     antiskyrmion of Sec. 4.2):
 *       n = (sin T cos(m theta + gamma), sin T sin(m theta + gamma), cos T),
 *       T = 2 atan(R / r) (Belavin-Polyakov); halo n = e_3.
 * Noise: if noise_amp > 0, every interior component gets noise_amp * (2u - 1),
 * u the SplitMix64 counter draw of (seed, c, j, i) (same generator as the
 * project's input module); the chiral magnet is renormalised afterwards.
 * Synchronises. */
#define SS_ANSATZ_VORTICES 0
#define SS_ANSATZ_SKYRMION 1
#define SS_ANSATZ_BEC 2
int ss_init_ansatz(ss_ctx* ctx, int kind, int n, const double* xy, const double* w, const double* shape,
                   uint64_t seed, double noise_amp);

/* Mean device time per launch of each of the passes, measured with HIP events
 * on the context's stream over n_steps flow steps (the steps are real flow
 * steps). RK4: ms[0..3] = stage passes P1..P4 (P1 including the one-workgroup
 * launch that finalises its reduction), ms[4] = whole step; under a fused plan
 * ms[1] is the pass of stages 2-4 and ms[2] = ms[3] = 0. One-pass integrators:
 * ms[0] = the step's pass with its finalise, ms[1] = velocity Verlet's restart
 * pass (the force of an arrested field; a launch that returns at once on the
 * other steps), ms[2] = ms[3] = 0. Synchronises. */
int ss_time_passes(ss_ctx* ctx, int n_steps, double* ms);

/* Copy the current field and (if velocity != NULL) the fictitious velocity
 * (Sec. 3.1 buffers, Sec. 3.2 first-order system) to device arrays of the
 * layout above, halo included. Synchronises. */
int ss_get_field(ss_ctx* ctx, void* field, void* velocity);

/* Checkpoint and resume. ss_get_state copies the current field and velocity
 * into device buffers of the ss_get_field layout (both required) and the flow
 * status into state, a host buffer of ss_state_bytes() bytes: step counter,
 * the energies the arrest test compares, arrest flag and count, the energy
 * history of the stall rule and the stop settings. ss_set_state on a context
 * of the same theory, dtype, gradient form and lattice restores all of it, so
 * that the flow continues exactly (bitwise) as it would have without the
 * interruption. A blob from another problem returns SS_ESHAPE, a corrupt one
 * SS_EINVAL. Both synchronise. */
size_t ss_state_bytes(void);
int ss_get_state(ss_ctx* ctx, void* field, void* velocity, void* state);
int ss_set_state(ss_ctx* ctx, const void* field, const void* velocity, const void* state);

/* E_h and gradient of a field (the force of eq. (3), Sec. 3.2; energy density of
 * Tab. 1 / eq. (5) with the eq. (1) stencil): `field` (device, NULL = the
 * current field).
 * If grad != NULL it receives G (device array, layout above, zero halo): the
 * gradient of the selected form; for the chiral magnet, at the normalised
 * field and projected on the tangent plane. Does not change the flow state.
 * Synchronises; energy and gnorm_inf (may be NULL) are host outputs. */
int ss_energy_grad(ss_ctx* ctx, const void* field, void* grad, double* energy, double* gnorm_inf);

/* Allocation-free ss_energy_grad, for callers that cannot allocate device
 * memory (code under stream capture, serving loops, harnesses that forbid
 * hipMalloc). Same result as ss_energy_grad on a context created with the same
 * theory, lattice, h, params and dtype, from the same kernels, but without a
 * context or workspace: field and grad (grad may be NULL) are device arrays of
 * the tight layout above (pitch Nx + 4); energy and gnorm_inf are host outputs
 * (may be NULL). The status block and the workgroup partials live in a
 * file-scope device array of the library, one per GPU, of fixed size (a status
 * block plus 2048 partials of 32 bytes, about 67 KB), kept until the process
 * ends; every lattice the API accepts (8 <= Nx, Ny <= 65536) fits it, and a
 * launch that would need more partials returns SS_ESHAPE. The call uses the
 * calling thread's current device, which must be the device of field, grad
 * and stream. It calls no hipMalloc or hipFree. Calls that overlap on one GPU
 * (concurrent streams or threads) share the array and race; serialise them.
 * The array keeps the last call's contents; nothing in it needs clearing,
 * since every slot read is written first by the same call. Synchronises. */
int ss_energy_grad_noalloc(const char* theory, int Nx, int Ny, double h, const ss_params* params, int dtype,
                           const void* field, void* grad, double* energy, double* gnorm_inf, void* stream);

/* n_steps arrested-Newton-flow steps, then the arrest test of the final field
 * (so the state afterwards is that of eq. (4) applied after every step).
 * If info != NULL the stream is synchronised and info filled. */
int ss_flow_step(ss_ctx* ctx, int n_steps, ss_step_info* info);

/* Arrested Newton flow (Sec. 3.2, eq. (3)-(4)) until a stop rule holds, replaying a captured HIP graph of
 * stop->graph_steps steps; each kernel skips its work once the device-side
 * stop flag is set, so the field stops exactly at the first state meeting a
 * rule. Returns SS_OK if converged, SS_NOT_CONVERGED at max_steps,
 * SS_ENONFINITE if a non-finite value appeared. */
int ss_minimise(ss_ctx* ctx, const ss_stop* stop, ss_min_info* info);

/* Observables of the current field (ss_obs; the global quantities of Sec. 3.3:
 * energy, topological charge, flux), reduced on the device in FP64.
 * Synchronises. */
int ss_observables(ss_ctx* ctx, ss_obs* out);

/* Energy target of the minimise stop rule SS_STOP_TARGET (E <= e_target);
 * -infinity (the value after ss_set_field / ss_init_*) disables it. Used to
 * time the flow to a reference energy. Synchronises. */
int ss_set_energy_target(ss_ctx* ctx, double e_target);

/* ------------------------------------------- learned initialiser (Abelian Higgs)
 * The network (include/ssn.h) maps an input image to smooth corrections of the
 * vortex ansatz. Images are fp32 device arrays over the interior grid, row-major
 * (Ny, Nx, channels):
 *   ss_learned_input:   (Ny, Nx, 2): sum_k exp(-r_k^2 / 2) at the n centres xy
 *                       (host, lattice coordinates), and the constant kappa;
 *   ss_learned_targets: (Ny, Nx, 4) from the context's current field psi, A in
 *                       the co-rotating frame of the ansatz: Re and Im of
 *                       psi exp(-i Theta) - f_ans, then A_x - A_ans_x, A_y - A_ans_y,
 *                       with Theta = sum_k w_k theta_k and f_ans, A_ans the ansatz
 *                       of ss_init_ansatz for the same centres and windings;
 *   ss_init_learned:    sets psi = (f_ans + env (c0 + i c1)) exp(i Theta),
 *                       A = A_ans + env (c2, c3) on the interior from corrections
 *                       corr (Ny, Nx, 4), the vacuum on the halo, and starts the
 *                       flow from rest (as ss_set_field). The envelope
 *                       env = 1 - prod_k (1 - exp(-r_k^2 / (2 sigma^2))) keeps the
 *                       corrections near the vortices (sigma <= 0: env = 1); with
 *                       pin > 0 the psi correction is also multiplied by
 *                       prod_k (1 - exp(-r_k^2 / (2 pin^2))), which keeps the zeros
 *                       of psi at the centres (pin <= 0: factor 1). If noise_amp > 0
 *                       every interior component then gets the seeded noise of
 *                       ss_init_ansatz (same seed, generator and amplitude), so
 *                       zero corrections with sigma <= 0 and pin <= 0 give
 *                       ss_init_ansatz's field; without noise, sigma <= 0 and
 *                       pin <= 0 ss_init_learned inverts ss_learned_targets.
 *                       Negative or non-finite noise_amp returns SS_EINVAL.
 * The first two synchronise. */
int ss_learned_input(ss_ctx* ctx, int n, const double* xy, double kappa, float* out);
int ss_learned_targets(ss_ctx* ctx, int n, const double* xy, const double* w, float* out);
int ss_init_learned(ss_ctx* ctx, int n, const double* xy, const double* w, const float* corr, double sigma,
                    double pin, uint64_t seed, double noise_amp);

/* Plans: how the four stages of an RK4 step (Sec. 3.2, eq. (3)) are launched.
 *   SS_PLAN_STAGES      one pass per stage, P1..P4 (17 field sets of HBM
 *                       traffic per site and step);
 *   SS_PLAN_FUSED       P1, then one pass that evaluates stages 2, 3 and 4 and
 *                       the update on a tile, recomputing stage 2 on a ring
 *                       of 2 around it (7 field sets per site and step).
 * All plans give the same step up to rounding order. The fused plans exist for
 * the Euler-Lagrange gradient only (SS_EINVAL otherwise). New FP32 contexts
 * with the Euler-Lagrange gradient start with SS_PLAN_FUSED, others with
 * SS_PLAN_STAGES. ss_set_plan synchronises the stream. */
#define SS_PLAN_STAGES 0
#define SS_PLAN_FUSED 1
#define SS_NUM_PLANS 2
int ss_set_plan(ss_ctx* ctx, int plan);
int ss_get_plan(ss_ctx* ctx);

/* Integrators of the flow (Sec. 3.2: the second-order flow is integrated by an
 * explicit scheme, RK4 for example, and contrasted with first-order descent).
 *   SS_INTEG_RK4  classical RK4 on (phi, phidot), launched by the plan above
 *                 (default);
 *   SS_INTEG_VV   velocity Verlet, phi' = phi + dt v + dt^2/2 a, a' = -G(phi'),
 *                 v' = v + dt/2 (a + a'), with E_h(phi') reduced in the pass that
 *                 forms phi', so the arrest test of eq. (4) for the next step is
 *                 ready when that step starts. One pass per step reads phi, v
 *                 and the stored force a and writes phi', v', a' (6 field sets
 *                 of HBM traffic per site and step), or, in kick-drift-kick
 *                 form (ss_set_vv_form), keeps u = v + dt/2 a in the velocity
 *                 buffer within a run and reads phi and u and writes
 *                 phi' = phi + dt u and u' = v' + dt/2 a' (4 sets); there a
 *                 step after an arrest (v = 0) is preceded by a pass that sets
 *                 u = dt/2 a from the field;
 *   SS_INTEG_GF   gradient flow phi' = phi + tau a with tau = dt^2/2 (the step
 *                 velocity Verlet takes from rest); no velocity, no arrest. On
 *                 the lattice theories one pass per step reads phi, tests it
 *                 (E_h, max |G|, stop rules) and writes phi' (2 field sets), the
 *                 step counter advancing after the test as after RK4's first
 *                 stage; the BEC's pass reads phi and the stored force a and
 *                 writes phi' and a' (4 sets).
 * dt = C h as for RK4. Every run of velocity Verlet (ss_flow_step, ss_minimise)
 * begins with one pass that tests the current field and stores its force
 * (kick-drift-kick: forms u) and ends with the velocity of the last field (0
 * after an arrest; kick-drift-kick: v = u - dt/2 a), so between runs the
 * velocity buffer holds v; an ss_flow_step run of gradient flow ends, as RK4's
 * does, with a pass that tests the last field. Chiral magnet: phi' is normalised
 * before its force is taken and v' is projected on its tangent plane.
 * Batches: ss_batch_set_integrator. Synchronises. */
#define SS_INTEG_RK4 0
#define SS_INTEG_VV 1
#define SS_INTEG_GF 2
int ss_set_integrator(ss_ctx* ctx, int integ);
int ss_get_integrator(ss_ctx* ctx);

/* How velocity Verlet (SS_INTEG_VV, Sec. 3.2) keeps its state between steps;
 * both forms take the same steps up to rounding, and between runs the velocity
 * buffer holds v either way.
 *   SS_VV_STORED_FORCE  v and a = -G(phi) (6 field sets per step, no extra launch);
 *   SS_VV_HALF_STEP     kick-drift-kick: u = v + dt/2 a (4 field sets per step,
 *                       plus a restart pass launched every step that works only
 *                       after an arrest);
 *   SS_VV_AUTO          (default) the half-step form on lattices of at least
 *                       2^20 interior sites, where bytes outweigh the extra
 *                       launch, the stored force below. The BEC always keeps the
 *                       stored force (SS_EINVAL for SS_VV_HALF_STEP).
 * ss_get_vv_form returns the form the context's runs use (never SS_VV_AUTO).
 * Batches always use the half-step form (one restart launch serves every
 * member). Synchronises. */
#define SS_VV_AUTO 0
#define SS_VV_STORED_FORCE 1
#define SS_VV_HALF_STEP 2
int ss_set_vv_form(ss_ctx* ctx, int form);
int ss_get_vv_form(ss_ctx* ctx);

/* Conjugate-gradient iterations per solve of the demagnetising potential
 * (Sec. 4.2, eq. (6)): iters_flow for every field a flow step evaluates (the
 * solve starts from the last potential, so a few iterations track the slowly
 * moving field; default 2), iters_eval for ss_energy_grad and ss_observables
 * (default 40; each iteration lowers the residual about five-fold). Each
 * iteration is one multigrid V-cycle and one operator application. Only for
 * contexts with demagnetisation (else SS_EINVAL); values in [1, 1000]. */
int ss_set_demag_iters(ss_ctx* ctx, int iters_flow, int iters_eval);

/* Tile shapes of the stage kernels. The library carries ss_tile_count()
 * compiled shapes (a workgroup covers TX x TY sites, each thread RY rows of
 * one column); under a fused plan the shape applies to P1. ss_set_tile selects
 * one for a context. ss_autotune times every plan with every shape over
 * n_steps flow steps of a uniform vacuum on the context's lattice, keeps the
 * fastest pair, writes the mean step times in ms_out (may be NULL, else
 * SS_NUM_PLANS * ss_tile_count() doubles, index plan * ss_tile_count() + tile;
 * -1 where a pair does not apply) and returns the chosen tile index (>= 0; the
 * plan is read with ss_get_plan). It overwrites the field: call ss_set_field
 * or ss_init_ansatz afterwards. If the environment variable SS_AUTOTUNE_CACHE
 * names a file, ss_autotune first looks the problem (theory, dtype, gradient
 * form, Nx, Ny, compiled shapes, integrator, demagnetisation) up there and, if found, applies the stored
 * plan and tile without timing (ms_out all -1, the field untouched); otherwise
 * it times as above and appends its choice to the file. The environment
 * variable SS_TILE selects the initial shape of new contexts. */
int ss_tile_count(void);
int ss_tile_shape(int tile, int* tx, int* ty, int* ry);
int ss_set_tile(ss_ctx* ctx, int tile);
int ss_get_tile(ss_ctx* ctx);
int ss_autotune(ss_ctx* ctx, int n_steps, double* ms_out);

/* ------------------------------------------------------------ batching
 * Many independent minimisations (uneven lattices and couplings, one theory
 * and dtype) advanced together: each flow pass is one launch over a flat list
 * of work units (column segments of tiles) of all members still running,
 * followed, for the reducing passes, by one launch that takes every member's
 * reduction, arrest test and stop rules on the device. ss_batch_minimise
 * replays a captured HIP graph of stop->graph_steps steps and drops stopped
 * members' units from the list between replays. Each member is an ss_ctx carved from
 * the batch workspace (ss_batch_member): set its field with ss_set_field or
 * ss_init_ansatz and read results with the single-context calls; do not
 * destroy it separately. */
typedef struct {
  int Nx, Ny;
  double h;
  const double* f; /* theory float parameters as in ss_params.f (host) */
  int nf;
} ss_instance;

typedef struct ss_batch ss_batch;

int ss_batch_workspace_bytes(const char* theory, int n, const ss_instance* inst, int dtype, size_t* bytes);
int ss_batch_create(const char* theory, int n, const ss_instance* inst, int dtype, void* workspace, size_t ws_bytes,
                    void* stream, ss_batch** out);
void ss_batch_destroy(ss_batch* batch);
ss_ctx* ss_batch_member(ss_batch* batch, int i);
int ss_batch_size(ss_batch* batch);
/* n_steps for every member, then the arrest test; infos (n entries, may be NULL). */
int ss_batch_flow_step(ss_batch* batch, int n_steps, ss_step_info* infos);
/* Same stop rule for every member; infos (n entries, may be NULL). Returns
 * SS_OK if all converged, SS_NOT_CONVERGED if any hit max_steps. */
int ss_batch_minimise(ss_batch* batch, const ss_stop* stop, ss_min_info* infos);
int ss_batch_set_tile(ss_batch* batch, int tile);
/* Plan of the batch's steps (SS_PLAN_*, default SS_PLAN_FUSED). The fused pass
 * runs on one tile shape, 64 x 16 (FP32) or 64 x 8 (FP64), i.e. tile 0 or 1;
 * with any other shape the batch runs separate stage passes. */
int ss_batch_set_plan(ss_batch* batch, int plan);
int ss_batch_get_plan(ss_batch* batch);
/* Integrator of the batch's steps (SS_INTEG_*, default SS_INTEG_RK4; Sec. 3.2),
 * as ss_set_integrator for one context: with velocity Verlet or gradient flow
 * every step is one batched pass (the plan does not apply), and each run starts
 * with one pass that tests every member's field and stores its force.
 * Synchronises. */
int ss_batch_set_integrator(ss_batch* batch, int integ);
int ss_batch_get_integrator(ss_batch* batch);
/* Observables of every member (out: n entries, host), each as ss_observables
 * gives it for one context. All members' observable passes are enqueued on the
 * batch stream before the first read-back, which synchronises. SS_EINVAL if
 * batch or out is NULL; after an error part of out may be filled. */
int ss_batch_observables(ss_batch* batch, ss_obs* out);
/* Times every plan with every tile shape it runs on over n_steps batch steps
 * (overwrites all fields with the vacuum), keeps the fastest pair, writes the
 * step times in ms_out (may be NULL, else SS_NUM_PLANS * ss_tile_count()
 * doubles, index plan * ss_tile_count() + tile, -1 where a pair does not
 * apply) and returns the chosen tile (the plan: ss_batch_get_plan). */
int ss_batch_autotune(ss_batch* batch, int n_steps, double* ms_out);

/* Read the device status into info (synchronises). */
int ss_get_info(ss_ctx* ctx, ss_step_info* info);

/* Text of a status code, and the calling thread's last error message. */
const char* ss_status_string(int code);
const char* ss_last_error(void);

/* GL helper: lambda = 2 kappa^2 in units u = e = 1 (textbook relation). */
double ss_gl_lambda_from_kappa(double kappa);

#ifdef __cplusplus
}
#endif
#endif /* SS_H */
