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
#include <cstdio>
#include <cstring>
#include <limits>
#include <new>
#include <string>
#include <vector>
#include <algorithm>

#include "../../include/ss.h"
#include "ss_kernels.hpp"

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

// Tile of one workgroup: TX x TY sites, RY rows per thread (256 threads).
constexpr int kTX = 64, kTY = 16, kRY = 4;
constexpr int kDefaultGraphSteps = 16;

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
  size_t set_bytes;         // bytes of one C-plane field set (256-B aligned)
  size_t status_off, partial_off, init_off, total;
  int ntx, nty, nlaunch;
};

Layout make_layout(int C, int Nx, int Ny, int esize) {
  Layout L;
  L.pitch = round_up(Nx + 4, 32);
  L.plane = round_up(L.pitch * (Ny + 4), 64);
  L.set_bytes = (size_t)round_up((long)C * L.plane * esize, 256);
  L.ntx = (Nx + kTX - 1) / kTX;
  L.nty = (Ny + kTY - 1) / kTY;
  L.nlaunch = (int)round_up((long)L.ntx * L.nty, 8);
  L.status_off = 7 * L.set_bytes;
  L.partial_off = L.status_off + (size_t)round_up(sizeof(DevStatus), 256);
  // partials: 4 doubles per stage-pass workgroup, 5 per observable workgroup
  const long nobs = 1024;
  const long nparts = std::max<long>(4L * L.nlaunch, 5L * nobs);
  L.init_off = L.partial_off + (size_t)round_up(nparts * 8, 256);
  // staging of ansatz centres and windings for ss_init_ansatz
  L.total = L.init_off + (size_t)round_up(3L * kMaxVortices * 8, 256);
  return L;
}

}  // namespace

struct ss_ctx {
  int theory, dtype, grad_mode, C, Nx, Ny;
  double h, courant;
  double p[4];
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
  return B;
}

Coeffs coeffs_of(const ss_ctx* c) {
  Coeffs cf;
  cf.h = c->h;
  cf.dt = c->courant * c->h;
  for (int k = 0; k < 4; ++k) cf.p[k] = c->p[k];
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
  a.src_pitch = a.src_plane = 0;
  a.out = nullptr;
  a.out_pitch = a.out_plane = 0;
  a.nlaunch = c->L.nlaunch;
  a.ntx = c->L.ntx;
  a.nty = c->L.nty;
  return a;
}

template <class T, int TH, int PASS>
void launch_pass_t(const PassArgs<T>& a, hipStream_t s) {
  hipLaunchKernelGGL((stage_pass<T, TH, PASS, kTX, kTY, kRY>), dim3(a.nlaunch), dim3(kTX, kTY / kRY), 0, s, a);
}

template <class T, int PASS>
void launch_pass(const ss_ctx* c, const PassArgs<T>& a, hipStream_t s) {
  if (c->theory == SS_THEORY_AH) launch_pass_t<T, 0, PASS>(a, s);
  else launch_pass_t<T, 1, PASS>(a, s);
}

template <class T>
void enqueue_steps(const ss_ctx* c, int n, hipStream_t s) {
  PassArgs<T> a = pass_args<T>(c);
  for (int k = 0; k < n; ++k) {
    launch_pass<T, kP1>(c, a, s);
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

template <class T>
void enqueue_apply_arrest(const ss_ctx* c, hipStream_t s) {
  hipLaunchKernelGGL((apply_arrest<T>), dim3(1024), dim3(256), 0, s, bufs_of<T>(c), c->st, c->C);
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
  SS_HIP(hipMemsetAsync(c->vel[0], 0, 5 * c->L.set_bytes, c->stream));
  DevStatus s;
  std::memset(&s, 0, sizeof(s));
  s.E = s.E_prev = std::numeric_limits<double>::infinity();
  s.gmax = std::numeric_limits<double>::infinity();
  SS_HIP(hipMemcpyAsync(c->st, &s, sizeof(s), hipMemcpyHostToDevice, c->stream));
  SS_HIP(hipStreamSynchronize(c->stream));
  return SS_OK;
}

}  // namespace

extern "C" {

int ss_theory_id(const char* name) {
  if (!name) return SS_ETHEORY;
  static const char* ah[] = {"abelian_higgs", "abelian higgs", "ginzburg-landau", "gl", "ah", "ginzburg landau"};
  static const char* cm[] = {"chiral_magnet", "chiral magnet", "cm"};
  for (const char* a : ah)
    if (lower_eq(name, a)) return SS_THEORY_AH;
  for (const char* a : cm)
    if (lower_eq(name, a)) return SS_THEORY_CM;
  return SS_ETHEORY;
}

int ss_components(const char* theory) {
  const int t = ss_theory_id(theory);
  if (t < 0) return t;
  return t == SS_THEORY_AH ? 4 : 3;
}

int ss_workspace_bytes(const char* theory, int Nx, int Ny, int dtype, size_t* bytes) {
  const int C = ss_components(theory);
  if (C < 0) return fail(SS_ETHEORY, std::string("unknown theory '") + (theory ? theory : "(null)") + "'");
  if (dtype != SS_F32 && dtype != SS_F64) return fail(SS_EINVAL, "dtype must be SS_F32 or SS_F64");
  if (Nx < 8 || Ny < 8 || Nx > 65536 || Ny > 65536) return fail(SS_ESHAPE, "Nx, Ny must lie in [8, 65536]");
  if (!bytes) return fail(SS_EINVAL, "bytes is NULL");
  *bytes = make_layout(C, Nx, Ny, (int)esize_of(dtype)).total;
  return SS_OK;
}

int ss_create(const char* theory, int Nx, int Ny, double h, const ss_params* params, int dtype, void* workspace,
              size_t ws_bytes, void* stream, ss_ctx** out) {
  if (!out) return fail(SS_EINVAL, "out is NULL");
  *out = nullptr;
  const int th = ss_theory_id(theory);
  if (th < 0) return fail(SS_ETHEORY, std::string("unknown theory '") + (theory ? theory : "(null)") + "'");
  size_t need = 0;
  int rc = ss_workspace_bytes(theory, Nx, Ny, dtype, &need);
  if (rc) return rc;
  if (!(h > 0.0) || !std::isfinite(h)) return fail(SS_EINVAL, "lattice spacing h must be positive and finite");
  if (!workspace || ws_bytes < need) return fail(SS_EINVAL, "workspace missing or smaller than ss_workspace_bytes");
  if (((uintptr_t)workspace) % 256 != 0) return fail(SS_EINVAL, "workspace must be 256-byte aligned");
  const int nf_need = th == SS_THEORY_AH ? 1 : 4;
  if (!params || !params->f || params->nf < nf_need || params->nf > nf_need + 1)
    return fail(SS_EINVAL, th == SS_THEORY_AH ? "abelian_higgs needs params.f = {lambda [, courant]}"
                                              : "chiral_magnet needs params.f = {J, D, K, B [, courant]}");
  for (int k = 0; k < params->nf; ++k)
    if (!std::isfinite(params->f[k])) return fail(SS_EINVAL, "non-finite parameter");
  double courant = params->nf > nf_need ? params->f[nf_need] : 0.5;
  if (!(courant > 0.0 && courant < 1.0)) return fail(SS_EINVAL, "courant number C must lie in (0, 1)");
  int grad_mode = SS_GRAD_EL;
  if (params->ni > 0) {
    if (!params->i) return fail(SS_EINVAL, "params.i is NULL with ni > 0");
    grad_mode = params->i[0];
    if (grad_mode != SS_GRAD_EL && grad_mode != SS_GRAD_EXACT) return fail(SS_EINVAL, "unknown grad_mode");
    if (grad_mode == SS_GRAD_EXACT) return fail(SS_EINVAL, "grad_mode SS_GRAD_EXACT is not built in this library");
  }

  ss_ctx* c = new (std::nothrow) ss_ctx();
  if (!c) return fail(SS_EINVAL, "out of host memory");
  c->theory = th;
  c->dtype = dtype;
  c->grad_mode = grad_mode;
  c->C = th == SS_THEORY_AH ? 4 : 3;
  c->Nx = Nx;
  c->Ny = Ny;
  c->h = h;
  c->courant = courant;
  for (int k = 0; k < 4; ++k) c->p[k] = k < nf_need ? params->f[k] : 0.0;
  c->stream = (hipStream_t)stream;
  c->ws = (char*)workspace;
  c->L = make_layout(c->C, Nx, Ny, (int)esize_of(dtype));
  void** sets[7] = {&c->phi[0], &c->phi[1], &c->vel[0], &c->vel[1], &c->a1, &c->a2, &c->q};
  for (int k = 0; k < 7; ++k) *sets[k] = c->ws + k * c->L.set_bytes;
  c->st = (DevStatus*)(c->ws + c->L.status_off);
  c->partials = (double*)(c->ws + c->L.partial_off);
  c->graph = nullptr;
  c->graph_steps = 0;
  hipError_t e = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    delete c;
    return fail(SS_EHIP, std::string("hipStreamCreateWithFlags: ") + hipGetErrorString(e));
  }
  // zero the whole workspace once: halos of velocity and stage arrays stay 0
  e = hipMemsetAsync(c->ws, 0, c->L.total, c->stream);
  if (e != hipSuccess) {
    (void)hipStreamDestroy(c->cap_stream);
    delete c;
    return fail(SS_EHIP, std::string("hipMemsetAsync: ") + hipGetErrorString(e));
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
  if ((kind == SS_ANSATZ_VORTICES) != (c->theory == SS_THEORY_AH) ||
      (kind != SS_ANSATZ_VORTICES && kind != SS_ANSATZ_SKYRMION))
    return fail(SS_EINVAL, "ansatz kind does not match the theory");
  if (n < 0 || n > kMaxVortices || (n > 0 && !xy)) return fail(SS_EINVAL, "bad vortex list");
  if (kind == SS_ANSATZ_SKYRMION && (n != 1 || !shape)) return fail(SS_EINVAL, "skyrmion needs n = 1 and shape");
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
  ia.kind = kind == SS_ANSATZ_VORTICES ? 0 : 1;
  ia.n = n;
  ia.xy = dev;
  ia.w = dev + 2 * (size_t)n;
  ia.R = shape ? shape[0] : 0.0;
  ia.gamma = shape ? shape[1] : 0.0;
  ia.amp = noise_amp;
  ia.key = 0ULL;
  if (noise_amp > 0.0) {
    // key = mix(seed * golden + stream), stream 1 = interior noise
    unsigned long long z = (unsigned long long)seed * 0x9E3779B97F4A7C15ULL + 1ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    ia.key = z ^ (z >> 31);
    if (ia.key == 0ULL) ia.key = 1ULL;  // 0 marks "no noise"
  }
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
  for (int s = 0; s < n_steps; ++s) {
    SS_HIP(hipEventRecord(ev[0], c->stream));
    if (c->dtype == SS_F32) {
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
      acc[k] += t;
    }
    float t = 0.f;
    SS_HIP(hipEventElapsedTime(&t, ev[0], ev[4]));
    acc[4] += t;
  }
  enqueue_check_any(c, c->stream);
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

int ss_energy_grad(ss_ctx* c, const void* field, void* grad, double* energy, double* gnorm_inf) {
  if (!c) return fail(SS_EINVAL, "ctx is NULL");
  const size_t es = esize_of(c->dtype);
  const long upitch = c->Nx + 4, uplane = upitch * (c->Ny + 4);
  if (grad) SS_HIP(hipMemsetAsync(grad, 0, (size_t)c->C * uplane * es, c->stream));
  if (c->dtype == SS_F32) {
    PassArgs<float> a = pass_args<float>(c);
    a.src = (const float*)field;
    a.src_pitch = upitch;
    a.src_plane = uplane;
    a.out = (float*)grad;
    a.out_pitch = upitch;
    a.out_plane = uplane;
    launch_pass<float, kEval>(c, a, c->stream);
  } else {
    PassArgs<double> a = pass_args<double>(c);
    a.src = (const double*)field;
    a.src_pitch = upitch;
    a.src_plane = uplane;
    a.out = (double*)grad;
    a.out_pitch = upitch;
    a.out_plane = uplane;
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

int ss_flow_step(ss_ctx* c, int n_steps, ss_step_info* info) {
  if (!c) return fail(SS_EINVAL, "ctx is NULL");
  if (n_steps < 0) return fail(SS_EINVAL, "n_steps < 0");
  hipLaunchKernelGGL(arm_status, dim3(1), dim3(64), 0, c->stream, c->st, 0, 0.0, 0.0, 0, 0LL);
  enqueue_steps_any(c, n_steps, c->stream);
  enqueue_check_any(c, c->stream);
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
  if (stop->window < 0 || stop->window > kHistLen) return fail(SS_EINVAL, "window must lie in [0, 128]");
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
  SS_HIP(hipGetLastError());
  DevStatus d;
  for (;;) {
    // a few replays between status reads keep the queue busy
    for (int r = 0; r < 4; ++r) SS_HIP(hipGraphLaunch(c->graph, c->stream));
    int rc = read_status(c, &d);
    if (rc) return rc;
    if (d.done) break;
  }
  if (c->dtype == SS_F32) enqueue_apply_arrest<float>(c, c->stream);
  else enqueue_apply_arrest<double>(c, c->stream);
  int rc = read_status(c, &d);
  if (rc) return rc;
  if (info) {
    fill_info(d, &info->last);
    info->reason = d.done;
    info->converged = (d.done == SS_STOP_GRAD || d.done == SS_STOP_STALL) ? 1 : 0;
  }
  if (d.done == SS_STOP_NONFINITE) return fail(SS_ENONFINITE, "non-finite value in the flow");
  if (d.done == SS_STOP_MAXSTEPS) return SS_NOT_CONVERGED;
  return SS_OK;
}

int ss_observables(ss_ctx* c, ss_obs* out) {
  if (!c || !out) return fail(SS_EINVAL, "ctx or out is NULL");
  const int nobs = 1024;
  if (c->dtype == SS_F32) {
    Bufs<float> B = bufs_of<float>(c);
    if (c->theory == SS_THEORY_AH) {
      hipLaunchKernelGGL((obs_sites<float, 0>), dim3(nobs), dim3(256), 0, c->stream, B, coeffs_of(c), c->st, c->partials, nobs);
      hipLaunchKernelGGL((obs_winding<float>), dim3(1), dim3(256), 0, c->stream, B, c->st);
    } else {
      hipLaunchKernelGGL((obs_sites<float, 1>), dim3(nobs), dim3(256), 0, c->stream, B, coeffs_of(c), c->st, c->partials, nobs);
      hipLaunchKernelGGL((obs_berg_luscher<float>), dim3(nobs), dim3(256), 0, c->stream, B, c->st, c->partials, nobs);
    }
  } else {
    Bufs<double> B = bufs_of<double>(c);
    if (c->theory == SS_THEORY_AH) {
      hipLaunchKernelGGL((obs_sites<double, 0>), dim3(nobs), dim3(256), 0, c->stream, B, coeffs_of(c), c->st, c->partials, nobs);
      hipLaunchKernelGGL((obs_winding<double>), dim3(1), dim3(256), 0, c->stream, B, c->st);
    } else {
      hipLaunchKernelGGL((obs_sites<double, 1>), dim3(nobs), dim3(256), 0, c->stream, B, coeffs_of(c), c->st, c->partials, nobs);
      hipLaunchKernelGGL((obs_berg_luscher<double>), dim3(nobs), dim3(256), 0, c->stream, B, c->st, c->partials, nobs);
    }
  }
  SS_HIP(hipGetLastError());
  DevStatus d;
  int rc = read_status(c, &d);
  if (rc) return rc;
  const double h2 = c->h * c->h;
  std::memset(out, 0, sizeof(*out));
  out->energy = h2 * d.obs[0];
  out->gnorm_inf = d.gmax;
  if (c->theory == SS_THEORY_AH) {
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
