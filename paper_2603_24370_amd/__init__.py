"""Python binding of libss, the MI355X soliton energy-minimisation library.

Thin ctypes marshalling over the C ABI of ``include/ss.h``: the functions
below carry the C names and arguments; PyTorch supplies device memory and the
stream. All computation happens in the library's HIP kernels. There is no CPU
fallback: if ``libss.so`` is missing or no GPU is present, calls raise.

``Solver`` is a convenience holder of one context and its workspace tensor.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libss.so")

SS_OK, SS_NOT_CONVERGED = 0, 1
SS_EINVAL, SS_ETHEORY, SS_ESHAPE, SS_EHIP, SS_ENONFINITE, SS_ESTATE = -1, -2, -3, -4, -5, -6
SS_F32, SS_F64 = 0, 1
SS_GRAD_EL, SS_GRAD_EXACT = 0, 1
SS_DMI_BULK, SS_DMI_HEUSLER = 0, 1
DMI_KINDS = {"bulk": SS_DMI_BULK, "heusler": SS_DMI_HEUSLER}
SS_PLAN_STAGES, SS_PLAN_FUSED = 0, 1
SS_INTEG_RK4, SS_INTEG_VV, SS_INTEG_GF = 0, 1, 2
INTEGRATORS = {"rk4": SS_INTEG_RK4, "vv": SS_INTEG_VV, "gf": SS_INTEG_GF}
SS_VV_AUTO, SS_VV_STORED_FORCE, SS_VV_HALF_STEP = 0, 1, 2
VV_FORMS = {"auto": SS_VV_AUTO, "stored_force": SS_VV_STORED_FORCE, "half_step": SS_VV_HALF_STEP}
SS_NUM_PLANS = 2
SS_THEORY_AH, SS_THEORY_CM, SS_THEORY_BS, SS_THEORY_BEC = 0, 1, 2, 3
SS_ANSATZ_VORTICES, SS_ANSATZ_SKYRMION, SS_ANSATZ_BEC = 0, 1, 2
STOP_REASONS = {0: "none", 1: "grad", 2: "stall", 3: "max_steps", 4: "nonfinite", 5: "target"}


class ss_params(ctypes.Structure):
    _fields_ = [("f", ctypes.POINTER(ctypes.c_double)), ("nf", ctypes.c_int),
                ("i", ctypes.POINTER(ctypes.c_int)), ("ni", ctypes.c_int)]


class ss_step_info(ctypes.Structure):
    _fields_ = [("energy", ctypes.c_double), ("energy_prev", ctypes.c_double), ("gnorm_inf", ctypes.c_double),
                ("step", ctypes.c_int64), ("n_arrests", ctypes.c_int64), ("arrested", ctypes.c_int32),
                ("nonfinite", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ss_stop(ctypes.Structure):
    _fields_ = [("grad_tol", ctypes.c_double), ("rel_e_tol", ctypes.c_double), ("window", ctypes.c_int32),
                ("graph_steps", ctypes.c_int32), ("max_steps", ctypes.c_int64)]


class ss_min_info(ctypes.Structure):
    _fields_ = [("last", ss_step_info), ("reason", ctypes.c_int32), ("converged", ctypes.c_int32)]


class ss_obs(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in
                ("energy", "flux", "n_rho", "n_wind", "bogo_r1", "bogo_r2", "q_fd", "q_bl", "gnorm_inf", "atoms",
                 "lz")]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ss_instance(ctypes.Structure):
    _fields_ = [("Nx", ctypes.c_int), ("Ny", ctypes.c_int), ("h", ctypes.c_double),
                ("f", ctypes.POINTER(ctypes.c_double)), ("nf", ctypes.c_int)]


class SSError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libss error {code}: {msg}")
        self.code = code


EXPORTS = ["ss_theory_id", "ss_components", "ss_workspace_bytes", "ss_create", "ss_destroy", "ss_set_field",
           "ss_init_ansatz", "ss_time_passes",
           "ss_get_field", "ss_energy_grad", "ss_flow_step", "ss_minimise", "ss_observables", "ss_get_info",
           "ss_status_string", "ss_last_error", "ss_gl_lambda_from_kappa", "ss_tile_count", "ss_tile_shape",
           "ss_set_tile", "ss_get_tile", "ss_autotune", "ss_set_plan", "ss_get_plan", "ss_batch_workspace_bytes",
           "ss_batch_create",
           "ss_batch_destroy", "ss_batch_member", "ss_batch_size", "ss_batch_flow_step", "ss_batch_minimise",
           "ss_batch_set_tile", "ss_batch_autotune", "ss_batch_set_plan", "ss_batch_get_plan", "ss_batch_observables", "ss_set_energy_target", "ss_learned_input",
           "ss_learned_targets", "ss_init_learned", "ss_state_bytes", "ss_get_state", "ss_set_state",
           "ss_energy_grad_noalloc", "ss_set_integrator", "ss_get_integrator", "ss_workspace_bytes_for",
           "ss_set_demag_iters", "ss_batch_set_integrator", "ss_batch_get_integrator", "ss_set_vv_form",
           "ss_get_vv_form"]
SSN_EXPORTS = ["ssn_param_count", "ssn_workspace_bytes", "ssn_create", "ssn_destroy", "ssn_num_params",
               "ssn_set_weights", "ssn_get_weights", "ssn_get_grads", "ssn_forward", "ssn_forward_graph", "ssn_backward",
               "ssn_adam_step", "ssn_set_grad_clip",
               "ssn_train_step", "ssn_flops", "ssn_init_field_workspace_bytes", "ssn_init_field", "ssn_last_error",
               "ssn_tensor_shape", "ssn_read_tensor"]
SSN_T_INPUT, SSN_T_PREACT, SSN_T_OUTPUT, SSN_T_GRAD_PREACT, SSN_T_GRAD_DATA = 0, 1, 2, 3, 4

_lib = None


def lib():
    """Load libss.so (built by ``paper_2603_24370_amd.build``); raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2603_24370_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i, d, cp = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_char_p
    L.ss_theory_id.argtypes = [cp]
    L.ss_components.argtypes = [cp]
    L.ss_workspace_bytes.argtypes = [cp, i, i, i, ctypes.POINTER(ctypes.c_size_t)]
    L.ss_workspace_bytes_for.argtypes = [cp, i, i, ctypes.POINTER(ss_params), i, ctypes.POINTER(ctypes.c_size_t)]
    L.ss_set_demag_iters.argtypes = [vp, i, i]
    L.ss_create.argtypes = [cp, i, i, d, ctypes.POINTER(ss_params), i, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    L.ss_destroy.argtypes = [vp]
    L.ss_destroy.restype = None
    L.ss_set_field.argtypes = [vp, vp]
    L.ss_get_field.argtypes = [vp, vp, vp]
    L.ss_state_bytes.argtypes = []
    L.ss_state_bytes.restype = ctypes.c_size_t
    L.ss_get_state.argtypes = [vp, vp, vp, vp]
    L.ss_set_state.argtypes = [vp, vp, vp, vp]
    dp = ctypes.POINTER(d)
    L.ss_init_ansatz.argtypes = [vp, i, i, dp, dp, dp, ctypes.c_uint64, d]
    L.ss_time_passes.argtypes = [vp, i, dp]
    L.ss_energy_grad.argtypes = [vp, vp, vp, ctypes.POINTER(d), ctypes.POINTER(d)]
    L.ss_energy_grad_noalloc.argtypes = [cp, i, i, d, ctypes.POINTER(ss_params), i, vp, vp, ctypes.POINTER(d),
                                         ctypes.POINTER(d), vp]
    L.ss_flow_step.argtypes = [vp, i, ctypes.POINTER(ss_step_info)]
    L.ss_minimise.argtypes = [vp, ctypes.POINTER(ss_stop), ctypes.POINTER(ss_min_info)]
    L.ss_observables.argtypes = [vp, ctypes.POINTER(ss_obs)]
    L.ss_get_info.argtypes = [vp, ctypes.POINTER(ss_step_info)]
    L.ss_status_string.argtypes = [i]
    L.ss_status_string.restype = cp
    L.ss_last_error.argtypes = []
    L.ss_last_error.restype = cp
    L.ss_gl_lambda_from_kappa.argtypes = [d]
    L.ss_gl_lambda_from_kappa.restype = d
    ip = ctypes.POINTER(i)
    L.ss_tile_count.argtypes = []
    L.ss_tile_shape.argtypes = [i, ip, ip, ip]
    L.ss_set_tile.argtypes = [vp, i]
    L.ss_get_tile.argtypes = [vp]
    L.ss_autotune.argtypes = [vp, i, dp]
    L.ss_set_plan.argtypes = [vp, i]
    L.ss_set_integrator.argtypes = [vp, i]
    L.ss_get_integrator.argtypes = [vp]
    L.ss_set_vv_form.argtypes = [vp, i]
    L.ss_get_vv_form.argtypes = [vp]
    L.ss_get_plan.argtypes = [vp]
    ins = ctypes.POINTER(ss_instance)
    L.ss_batch_workspace_bytes.argtypes = [cp, i, ins, i, ctypes.POINTER(ctypes.c_size_t)]
    L.ss_batch_create.argtypes = [cp, i, ins, i, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    L.ss_batch_destroy.argtypes = [vp]
    L.ss_batch_destroy.restype = None
    L.ss_batch_member.argtypes = [vp, i]
    L.ss_batch_member.restype = vp
    L.ss_batch_size.argtypes = [vp]
    L.ss_batch_flow_step.argtypes = [vp, i, ctypes.POINTER(ss_step_info)]
    L.ss_batch_minimise.argtypes = [vp, ctypes.POINTER(ss_stop), ctypes.POINTER(ss_min_info)]
    L.ss_batch_set_tile.argtypes = [vp, i]
    L.ss_batch_autotune.argtypes = [vp, i, dp]
    L.ss_batch_set_plan.argtypes = [vp, i]
    L.ss_batch_get_plan.argtypes = [vp]
    L.ss_batch_set_integrator.argtypes = [vp, i]
    L.ss_batch_get_integrator.argtypes = [vp]
    L.ss_batch_observables.argtypes = [vp, ctypes.POINTER(ss_obs)]
    _lib = L
    return L


def _check(rc, allow=(SS_OK,)):
    if rc in allow:
        return rc
    if rc < 0 or rc not in (SS_OK, SS_NOT_CONVERGED):
        raise SSError(rc, lib().ss_last_error().decode())
    return rc


def _b(s: str) -> bytes:
    return s.encode() if isinstance(s, str) else s


# ----------------------------------------------------------- C-ABI mirrors

def ss_theory_id(name: str) -> int:
    return lib().ss_theory_id(_b(name))


def ss_components(theory: str) -> int:
    return _check_nonneg(lib().ss_components(_b(theory)))


def _check_nonneg(rc):
    if rc < 0:
        raise SSError(rc, lib().ss_last_error().decode() or "error")
    return rc


def ss_workspace_bytes(theory: str, Nx: int, Ny: int, dtype: int) -> int:
    n = ctypes.c_size_t(0)
    _check(lib().ss_workspace_bytes(_b(theory), Nx, Ny, dtype, ctypes.byref(n)))
    return n.value


def ss_workspace_bytes_for(theory: str, Nx: int, Ny: int, f_params, i_params, dtype: int) -> int:
    fa = (ctypes.c_double * max(1, len(f_params)))(*f_params)
    ia = (ctypes.c_int * max(1, len(i_params)))(*i_params)
    p = ss_params(fa, len(f_params), ia, len(i_params))
    n = ctypes.c_size_t(0)
    _check(lib().ss_workspace_bytes_for(_b(theory), Nx, Ny, ctypes.byref(p), dtype, ctypes.byref(n)))
    return n.value


def ss_set_demag_iters(ctx, iters_flow, iters_eval):
    _check(lib().ss_set_demag_iters(ctx, int(iters_flow), int(iters_eval)))


def ss_create(theory, Nx, Ny, h, f_params, i_params, dtype, workspace_ptr, ws_bytes, stream_ptr):
    fa = (ctypes.c_double * max(1, len(f_params)))(*f_params)
    ia = (ctypes.c_int * max(1, len(i_params)))(*i_params)
    p = ss_params(fa, len(f_params), ia, len(i_params))
    out = ctypes.c_void_p(0)
    _check(lib().ss_create(_b(theory), Nx, Ny, h, ctypes.byref(p), dtype, ctypes.c_void_p(workspace_ptr), ws_bytes,
                           ctypes.c_void_p(stream_ptr), ctypes.byref(out)))
    return out


def ss_destroy(ctx):
    lib().ss_destroy(ctx)


def ss_set_field(ctx, field_ptr):
    _check(lib().ss_set_field(ctx, ctypes.c_void_p(field_ptr)))


def _darr(x):
    if x is None:
        return None
    vals = [float(v) for v in x]
    return (ctypes.c_double * max(1, len(vals)))(*vals)


def ss_init_ansatz(ctx, kind, centres, windings=None, shape=None, seed=0, noise_amp=0.0):
    flat = [float(v) for p in centres for v in p]
    n = len(flat) // 2
    _check(lib().ss_init_ansatz(ctx, kind, n, _darr(flat), _darr(windings), _darr(shape), int(seed),
                                float(noise_amp)))


def ss_time_passes(ctx, n_steps):
    ms = (ctypes.c_double * 5)()
    _check(lib().ss_time_passes(ctx, int(n_steps), ms))
    return list(ms)


def ss_get_field(ctx, field_ptr, vel_ptr=None):
    _check(lib().ss_get_field(ctx, ctypes.c_void_p(field_ptr), ctypes.c_void_p(vel_ptr or 0)))


def ss_state_bytes() -> int:
    return int(lib().ss_state_bytes())


def ss_get_state(ctx, field_ptr, vel_ptr) -> bytes:
    buf = ctypes.create_string_buffer(ss_state_bytes())
    _check(lib().ss_get_state(ctx, ctypes.c_void_p(field_ptr), ctypes.c_void_p(vel_ptr), buf))
    return buf.raw


def ss_set_state(ctx, field_ptr, vel_ptr, state: bytes):
    state = bytes(state)
    if len(state) != ss_state_bytes():
        raise ValueError(f"a state blob has {ss_state_bytes()} bytes, not {len(state)}")
    buf = ctypes.create_string_buffer(state, len(state))
    _check(lib().ss_set_state(ctx, ctypes.c_void_p(field_ptr), ctypes.c_void_p(vel_ptr), buf))


def ss_energy_grad(ctx, field_ptr=None, grad_ptr=None):
    e, g = ctypes.c_double(0), ctypes.c_double(0)
    _check(lib().ss_energy_grad(ctx, ctypes.c_void_p(field_ptr or 0), ctypes.c_void_p(grad_ptr or 0),
                                ctypes.byref(e), ctypes.byref(g)))
    return e.value, g.value


def ss_energy_grad_noalloc(theory, Nx, Ny, h, f_params, i_params, dtype, field_ptr, grad_ptr, stream_ptr):
    """Allocation-free evaluation (no context, no workspace). Returns (E, max |G|)."""
    fa = (ctypes.c_double * max(1, len(f_params)))(*f_params)
    ia = (ctypes.c_int * max(1, len(i_params)))(*i_params)
    p = ss_params(fa, len(f_params), ia, len(i_params))
    e, g = ctypes.c_double(0), ctypes.c_double(0)
    _check(lib().ss_energy_grad_noalloc(_b(theory), int(Nx), int(Ny), float(h), ctypes.byref(p), int(dtype),
                                        ctypes.c_void_p(field_ptr), ctypes.c_void_p(grad_ptr or 0), ctypes.byref(e),
                                        ctypes.byref(g), ctypes.c_void_p(stream_ptr or 0)))
    return e.value, g.value


def ss_flow_step(ctx, n_steps, want_info=True):
    info = ss_step_info()
    _check(lib().ss_flow_step(ctx, int(n_steps), ctypes.byref(info) if want_info else None))
    return info.as_dict() if want_info else None


def ss_minimise(ctx, grad_tol=0.0, rel_e_tol=0.0, window=0, max_steps=100000, graph_steps=0):
    s = ss_stop(grad_tol, rel_e_tol, window, graph_steps, max_steps)
    info = ss_min_info()
    rc = _check(lib().ss_minimise(ctx, ctypes.byref(s), ctypes.byref(info)), allow=(SS_OK, SS_NOT_CONVERGED))
    d = info.last.as_dict()
    d.update(reason=STOP_REASONS.get(info.reason, str(info.reason)), converged=bool(info.converged), rc=rc)
    return d


def ss_observables(ctx):
    o = ss_obs()
    _check(lib().ss_observables(ctx, ctypes.byref(o)))
    return o.as_dict()


def ss_get_info(ctx):
    info = ss_step_info()
    _check(lib().ss_get_info(ctx, ctypes.byref(info)))
    return info.as_dict()


def ss_tile_count() -> int:
    return lib().ss_tile_count()


def ss_tile_shape(tile: int):
    tx, ty, ry = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(lib().ss_tile_shape(tile, ctypes.byref(tx), ctypes.byref(ty), ctypes.byref(ry)))
    return tx.value, ty.value, ry.value


def ss_set_tile(ctx, tile: int):
    _check(lib().ss_set_tile(ctx, tile))


def ss_get_tile(ctx) -> int:
    return _check_nonneg(lib().ss_get_tile(ctx))


def ss_set_plan(ctx, plan: int):
    _check(lib().ss_set_plan(ctx, plan))


def ss_get_plan(ctx) -> int:
    return _check_nonneg(lib().ss_get_plan(ctx))


def ss_set_integrator(ctx, integ):
    _check(lib().ss_set_integrator(ctx, INTEGRATORS.get(integ, integ)))


def ss_get_integrator(ctx) -> int:
    return _check_nonneg(lib().ss_get_integrator(ctx))


def ss_set_vv_form(ctx, form):
    _check(lib().ss_set_vv_form(ctx, VV_FORMS.get(form, form)))


def ss_get_vv_form(ctx) -> int:
    return _check_nonneg(lib().ss_get_vv_form(ctx))


def ss_autotune(ctx, n_steps=10):
    """Returns (tile, plan, ms) with ms[plan][tile] the mean step time (-1: not timed)."""
    nt = ss_tile_count()
    ms = (ctypes.c_double * (SS_NUM_PLANS * nt))()
    best = _check_nonneg(lib().ss_autotune(ctx, int(n_steps), ms))
    grid = [list(ms[p * nt:(p + 1) * nt]) for p in range(SS_NUM_PLANS)]
    return best, ss_get_plan(ctx), grid


def ss_gl_lambda_from_kappa(kappa: float) -> float:
    return lib().ss_gl_lambda_from_kappa(kappa)


def _instances(instances):
    arr = (ss_instance * len(instances))()
    keep = []
    for k, (Nx, Ny, h, params) in enumerate(instances):
        fa = (ctypes.c_double * len(params))(*[float(x) for x in params])
        keep.append(fa)
        arr[k] = ss_instance(int(Nx), int(Ny), float(h), fa, len(params))
    return arr, keep


def ss_batch_workspace_bytes(theory, instances, dtype) -> int:
    arr, keep = _instances(instances)
    n = ctypes.c_size_t(0)
    _check(lib().ss_batch_workspace_bytes(_b(theory), len(instances), arr, dtype, ctypes.byref(n)))
    return n.value


def ss_batch_create(theory, instances, dtype, workspace_ptr, ws_bytes, stream_ptr):
    arr, keep = _instances(instances)
    out = ctypes.c_void_p(0)
    _check(lib().ss_batch_create(_b(theory), len(instances), arr, dtype, ctypes.c_void_p(workspace_ptr), ws_bytes,
                                 ctypes.c_void_p(stream_ptr), ctypes.byref(out)))
    return out


def ss_batch_destroy(batch):
    lib().ss_batch_destroy(batch)


def ss_batch_member(batch, i):
    p = lib().ss_batch_member(batch, i)
    if not p:
        raise SSError(-1, lib().ss_last_error().decode())
    return ctypes.c_void_p(p)


def ss_batch_size(batch) -> int:
    return _check_nonneg(lib().ss_batch_size(batch))


def ss_batch_observables(batch, n_members):
    out = (ss_obs * n_members)()
    _check(lib().ss_batch_observables(batch, out))
    return [x.as_dict() for x in out]


def ss_batch_flow_step(batch, n_steps, n_members=None):
    infos = (ss_step_info * n_members)() if n_members else None
    _check(lib().ss_batch_flow_step(batch, int(n_steps), infos))
    return [x.as_dict() for x in infos] if infos is not None else None


def ss_batch_minimise(batch, n_members, grad_tol=0.0, rel_e_tol=0.0, window=0, max_steps=100000, graph_steps=0):
    s = ss_stop(grad_tol, rel_e_tol, window, graph_steps, max_steps)
    infos = (ss_min_info * n_members)()
    rc = _check(lib().ss_batch_minimise(batch, ctypes.byref(s), infos), allow=(SS_OK, SS_NOT_CONVERGED))
    out = []
    for x in infos:
        d = x.last.as_dict()
        d.update(reason=STOP_REASONS.get(x.reason, str(x.reason)), converged=bool(x.converged))
        out.append(d)
    return rc, out


def ss_batch_set_tile(batch, tile):
    _check(lib().ss_batch_set_tile(batch, tile))


def ss_batch_set_plan(batch, plan: int):
    _check(lib().ss_batch_set_plan(batch, plan))


def ss_batch_set_integrator(batch, integ):
    _check(lib().ss_batch_set_integrator(batch, INTEGRATORS.get(integ, integ)))


def ss_batch_get_integrator(batch) -> int:
    return _check_nonneg(lib().ss_batch_get_integrator(batch))


def ss_batch_get_plan(batch) -> int:
    return _check_nonneg(lib().ss_batch_get_plan(batch))


def ss_batch_autotune(batch, n_steps=5):
    """Returns (tile, plan, ms) with ms[plan][tile] the mean step time (-1: not timed)."""
    nt = ss_tile_count()
    ms = (ctypes.c_double * (SS_NUM_PLANS * nt))()
    best = _check_nonneg(lib().ss_batch_autotune(batch, int(n_steps), ms))
    grid = [list(ms[p * nt:(p + 1) * nt]) for p in range(SS_NUM_PLANS)]
    return best, ss_batch_get_plan(batch), grid


# ------------------------------------------------------------ convenience

class Solver:
    """One library context plus its torch-allocated workspace on a CUDA/HIP device."""

    def __init__(self, theory, Nx, Ny, h, params, dtype="f32", grad_mode=SS_GRAD_EL, courant=None,
                 device="cuda:0", stream=None, _ctx=None, dmi="bulk", demag=False):
        """Chiral magnet options: dmi "bulk" or "heusler" (d_2 = -e_2); demag=True
        adds the demagnetising term, with params = (J, D, K, B, mu_d)."""
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("libss needs a HIP GPU; none is available")
        self.torch = torch
        if _ctx is not None:
            # a member of a Batch: the batch owns the context and the workspace
            self.theory, self.Nx, self.Ny, self.h = theory, int(Nx), int(Ny), float(h)
            self.dtype_code = SS_F32 if dtype in ("f32", torch.float32) else SS_F64
            self.tdtype = torch.float32 if self.dtype_code == SS_F32 else torch.float64
            self.C = ss_components(theory)
            self.device = torch.device(device)
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            self.ctx = _ctx
            self._owned = False
            return
        self._owned = True
        self.theory, self.Nx, self.Ny, self.h = theory, int(Nx), int(Ny), float(h)
        self.dtype_code = SS_F32 if dtype in ("f32", torch.float32) else SS_F64
        self.tdtype = torch.float32 if self.dtype_code == SS_F32 else torch.float64
        self.C = ss_components(theory)
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        f = list(params) + ([courant] if courant is not None else [])
        ip = [grad_mode]
        if dmi != "bulk" or demag:
            ip += [DMI_KINDS[dmi], int(bool(demag))]
        nbytes = ss_workspace_bytes_for(theory, self.Nx, self.Ny, f, ip, self.dtype_code)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        self.ctx = ss_create(theory, self.Nx, self.Ny, self.h, f, ip, self.dtype_code, self._ws_ptr,
                             nbytes, self.stream.cuda_stream)

    @property
    def shape(self):
        return (self.C, self.Ny + 4, self.Nx + 4)

    def _dev(self, x):
        t = self.torch.as_tensor(x)
        return t.to(device=self.device, dtype=self.tdtype).contiguous()

    def init_vortices(self, centres, windings=None, seed=0, noise_amp=0.0):
        ss_init_ansatz(self.ctx, SS_ANSATZ_VORTICES, centres, windings, None, seed, noise_amp)

    def init_skyrmion(self, R=2.0, gamma=-1.5707963267948966, centre=(0.0, 0.0), seed=0, noise_amp=0.0,
                      vorticity=1):
        """Belavin-Polyakov ansatz; vorticity -1 gives the antiskyrmion."""
        ss_init_ansatz(self.ctx, SS_ANSATZ_SKYRMION, [centre], [float(vorticity)], [R, gamma], seed, noise_amp)

    def init_bec(self, R=1.0, xi=1.0, centres=(), windings=None, seed=0, noise_amp=0.0):
        """Gaussian cloud of radius R with vortices (core width xi) at the centres."""
        ss_init_ansatz(self.ctx, SS_ANSATZ_BEC, list(centres), windings, [R, xi], seed, noise_amp)

    def set_demag_iters(self, iters_flow, iters_eval):
        ss_set_demag_iters(self.ctx, iters_flow, iters_eval)

    def autotune(self, n_steps=10):
        return ss_autotune(self.ctx, n_steps)

    def set_tile(self, tile):
        ss_set_tile(self.ctx, tile)

    def set_plan(self, plan):
        ss_set_plan(self.ctx, plan)

    @property
    def plan(self):
        return ss_get_plan(self.ctx)

    def set_integrator(self, integ):
        """"rk4" (default), "vv" (velocity Verlet, one pass) or "gf" (gradient flow, one pass)."""
        ss_set_integrator(self.ctx, integ)

    @property
    def integrator(self):
        return ss_get_integrator(self.ctx)

    def set_vv_form(self, form):
        """Velocity Verlet's state between steps: "auto" (default), "stored_force" or "half_step"."""
        ss_set_vv_form(self.ctx, form)

    @property
    def vv_form(self):
        """The form this context's velocity Verlet runs use (SS_VV_STORED_FORCE or SS_VV_HALF_STEP)."""
        return ss_get_vv_form(self.ctx)

    def set_energy_target(self, e_target):
        ss_set_energy_target(self.ctx, e_target)

    def time_passes(self, n_steps):
        return ss_time_passes(self.ctx, n_steps)

    def set_field(self, field):
        t = self._dev(field)
        if tuple(t.shape) != self.shape:
            raise ValueError(f"field shape {tuple(t.shape)} != {self.shape}")
        ss_set_field(self.ctx, t.data_ptr())
        self.stream.synchronize()

    def get_field(self, velocity=False):
        f = self.torch.empty(self.shape, dtype=self.tdtype, device=self.device)
        v = self.torch.empty(self.shape, dtype=self.tdtype, device=self.device) if velocity else None
        ss_get_field(self.ctx, f.data_ptr(), v.data_ptr() if velocity else None)
        return (f, v) if velocity else f

    def get_state(self):
        """Checkpoint: (field, velocity, status bytes) of the flow."""
        f = self.torch.empty(self.shape, dtype=self.tdtype, device=self.device)
        v = self.torch.empty(self.shape, dtype=self.tdtype, device=self.device)
        blob = ss_get_state(self.ctx, f.data_ptr(), v.data_ptr())
        return f, v, blob

    def set_state(self, state):
        """Resume from a checkpoint of get_state (same theory, dtype and lattice)."""
        f, v, blob = state
        f, v = self._dev(f), self._dev(v)
        if tuple(f.shape) != self.shape or tuple(v.shape) != self.shape:
            raise ValueError(f"state shapes {tuple(f.shape)}, {tuple(v.shape)} != {self.shape}")
        ss_set_state(self.ctx, f.data_ptr(), v.data_ptr(), blob)

    def energy_grad(self, field=None, want_grad=True):
        src = None if field is None else self._dev(field)
        g = self.torch.empty(self.shape, dtype=self.tdtype, device=self.device) if want_grad else None
        E, gmax = ss_energy_grad(self.ctx, src.data_ptr() if src is not None else None,
                                 g.data_ptr() if g is not None else None)
        return E, gmax, g

    def flow_step(self, n=1, want_info=True):
        return ss_flow_step(self.ctx, n, want_info)

    def minimise(self, **kw):
        return ss_minimise(self.ctx, **kw)

    def observables(self):
        return ss_observables(self.ctx)

    def info(self):
        return ss_get_info(self.ctx)

    def close(self):
        if getattr(self, "ctx", None) is not None and getattr(self, "_owned", True):
            ss_destroy(self.ctx)
        self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many independent lattices of one theory advanced by batched launches.

    instances: list of (Nx, Ny, h, params). Members are Solver views (members[i])."""

    def __init__(self, theory, instances, dtype="f32", device="cuda:0", stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("libss needs a HIP GPU; none is available")
        self.torch = torch
        self.theory = theory
        self.instances = [tuple(x) for x in instances]
        self.n = len(self.instances)
        self.dtype_code = SS_F32 if dtype in ("f32", torch.float32) else SS_F64
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        nbytes = ss_batch_workspace_bytes(theory, self.instances, self.dtype_code)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        ptr = (self.workspace.data_ptr() + 255) // 256 * 256
        self.batch = ss_batch_create(theory, self.instances, self.dtype_code, ptr, nbytes, self.stream.cuda_stream)
        self.members = [Solver(theory, Nx, Ny, h, p, dtype=dtype, device=device, stream=self.stream,
                               _ctx=ss_batch_member(self.batch, i))
                        for i, (Nx, Ny, h, p) in enumerate(self.instances)]

    def flow_step(self, n=1, want_info=True):
        return ss_batch_flow_step(self.batch, n, self.n if want_info else None)

    def minimise(self, **kw):
        return ss_batch_minimise(self.batch, self.n, **kw)

    def observables(self):
        return ss_batch_observables(self.batch, self.n)

    def set_tile(self, tile):
        ss_batch_set_tile(self.batch, tile)

    def autotune(self, n_steps=5):
        return ss_batch_autotune(self.batch, n_steps)

    def set_plan(self, plan):
        ss_batch_set_plan(self.batch, plan)

    @property
    def plan(self):
        return ss_batch_get_plan(self.batch)

    def set_integrator(self, integ):
        """"rk4" (default), "vv" or "gf", as Solver.set_integrator."""
        ss_batch_set_integrator(self.batch, integ)

    @property
    def integrator(self):
        return ss_batch_get_integrator(self.batch)

    def close(self):
        if getattr(self, "batch", None) is not None:
            for m in self.members:
                m.ctx = None
            ss_batch_destroy(self.batch)
            self.batch = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------ learned initialiser (C ABI)

def _ssn_lib():
    L = lib()
    if getattr(L, "_ssn_ready", False):
        return L
    vp, i, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    fp = ctypes.POINTER(ctypes.c_float)
    dp = ctypes.POINTER(d)
    L.ss_set_energy_target.argtypes = [vp, d]
    L.ss_learned_input.argtypes = [vp, i, dp, d, vp]
    L.ss_learned_targets.argtypes = [vp, i, dp, dp, vp]
    L.ss_init_learned.argtypes = [vp, i, dp, dp, vp, d, d, ctypes.c_uint64, d]
    L.ssn_param_count.argtypes = [i, i, i, i]
    L.ssn_param_count.restype = ctypes.c_long
    L.ssn_workspace_bytes.argtypes = [i, i, i, i, i, i, i, ctypes.POINTER(ctypes.c_size_t)]
    L.ssn_create.argtypes = [i, i, i, i, i, i, i, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    L.ssn_destroy.argtypes = [vp]
    L.ssn_destroy.restype = None
    L.ssn_num_params.argtypes = [vp]
    L.ssn_num_params.restype = ctypes.c_long
    L.ssn_set_weights.argtypes = [vp, fp, ctypes.c_long]
    L.ssn_get_weights.argtypes = [vp, fp, ctypes.c_long]
    L.ssn_get_grads.argtypes = [vp, fp, ctypes.c_long]
    L.ssn_forward.argtypes = [vp, vp, i, vp]
    L.ssn_forward_graph.argtypes = [vp, vp, i, vp]
    L.ssn_backward.argtypes = [vp, vp, i, dp]
    L.ssn_adam_step.argtypes = [vp, ctypes.c_float]
    L.ssn_set_grad_clip.argtypes = [vp, ctypes.c_float]
    L.ssn_train_step.argtypes = [vp, vp, vp, i, ctypes.c_float, dp]
    L.ssn_flops.argtypes = [vp, dp, dp]
    L.ssn_init_field_workspace_bytes.argtypes = [vp]
    L.ssn_init_field_workspace_bytes.restype = ctypes.c_size_t
    L.ssn_init_field.argtypes = [vp, vp, i, dp, dp, d, d, d, ctypes.c_uint64, d, vp, ctypes.c_size_t]
    L.ssn_last_error.argtypes = []
    L.ssn_last_error.restype = ctypes.c_char_p
    ip = ctypes.POINTER(i)
    L.ssn_tensor_shape.argtypes = [vp, i, i, ip, ip, ip]
    L.ssn_read_tensor.argtypes = [vp, i, i, i, fp, ctypes.c_long]
    L._ssn_ready = True
    return L


def _ncheck(rc):
    if rc < 0:
        raise SSError(rc, _ssn_lib().ssn_last_error().decode() or lib().ss_last_error().decode())
    return rc


def ss_set_energy_target(ctx, e_target):
    _check(_ssn_lib().ss_set_energy_target(ctx, float(e_target)))


def ss_learned_input(ctx, centres, kappa, out_ptr):
    flat = [float(v) for p in centres for v in p]
    _check(_ssn_lib().ss_learned_input(ctx, len(flat) // 2, _darr(flat), float(kappa), ctypes.c_void_p(out_ptr)))


def ss_learned_targets(ctx, centres, windings, out_ptr):
    flat = [float(v) for p in centres for v in p]
    _check(_ssn_lib().ss_learned_targets(ctx, len(flat) // 2, _darr(flat), _darr(windings), ctypes.c_void_p(out_ptr)))


def ss_init_learned(ctx, centres, windings, corr_ptr, sigma=0.0, pin=0.0, seed=0, noise_amp=0.0):
    flat = [float(v) for p in centres for v in p]
    _check(_ssn_lib().ss_init_learned(ctx, len(flat) // 2, _darr(flat), _darr(windings), ctypes.c_void_p(corr_ptr),
                                      float(sigma), float(pin), int(seed), float(noise_amp)))


def ssn_param_count(levels, base, cin, cout):
    return _ssn_lib().ssn_param_count(levels, base, cin, cout)


class Net:
    """The learned initialiser's U-Net (ssn_* C ABI); torch supplies memory and the stream."""

    def __init__(self, levels=4, base=32, cin=2, cout=4, N=8, H=256, W=256, device="cuda:0", stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the network needs a HIP GPU; none is available")
        self.torch = torch
        self.levels, self.base, self.cin, self.cout, self.N, self.H, self.W = levels, base, cin, cout, N, H, W
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        L = _ssn_lib()
        nb = ctypes.c_size_t(0)
        _ncheck(L.ssn_workspace_bytes(levels, base, cin, cout, N, H, W, ctypes.byref(nb)))
        self.workspace = torch.empty(nb.value + 256, dtype=torch.uint8, device=self.device)
        ptr = (self.workspace.data_ptr() + 255) // 256 * 256
        out = ctypes.c_void_p(0)
        _ncheck(L.ssn_create(levels, base, cin, cout, N, H, W, ctypes.c_void_p(ptr), nb.value,
                             ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(out)))
        self.net = out
        self.n_params = L.ssn_num_params(self.net)

    def _fp(self, a):
        return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))

    def set_weights(self, flat):
        import numpy as np
        a = np.ascontiguousarray(flat, dtype=np.float32)
        _ncheck(_ssn_lib().ssn_set_weights(self.net, self._fp(a), a.size))

    def get_weights(self):
        import numpy as np
        a = np.zeros(self.n_params, dtype=np.float32)
        _ncheck(_ssn_lib().ssn_get_weights(self.net, self._fp(a), a.size))
        return a

    def get_grads(self):
        import numpy as np
        a = np.zeros(self.n_params, dtype=np.float32)
        _ncheck(_ssn_lib().ssn_get_grads(self.net, self._fp(a), a.size))
        return a

    def _dev(self, x):
        return self.torch.as_tensor(x).to(device=self.device, dtype=self.torch.float32).contiguous()

    def forward(self, x, out=None, graph=False):
        """Forward pass; with graph=True (x and out kept by the caller between calls)
        it replays a captured HIP graph."""
        x = self._dev(x)
        n = x.shape[0]
        if out is None:
            if graph:
                raise ValueError("graph=True needs a persistent out buffer")
            out = self.torch.empty((n, self.H, self.W, self.cout), dtype=self.torch.float32, device=self.device)
        fn = _ssn_lib().ssn_forward_graph if graph else _ssn_lib().ssn_forward
        _ncheck(fn(self.net, ctypes.c_void_p(x.data_ptr()), n, ctypes.c_void_p(out.data_ptr())))
        return out

    def read_tensor(self, kind, layer, n=None):
        """An internal BF16 tensor (SSN_T_*) of 3x3 layer `layer` as float32 (n, H, W, C)."""
        import numpy as np
        H, W, C = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _ncheck(_ssn_lib().ssn_tensor_shape(self.net, kind, layer, ctypes.byref(H), ctypes.byref(W),
                                            ctypes.byref(C)))
        n = self.N if n is None else n
        out = np.empty((n, H.value, W.value, C.value), dtype=np.float32)
        _ncheck(_ssn_lib().ssn_read_tensor(self.net, kind, layer, n, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                           out.size))
        return out

    def backward(self, target):
        t = self._dev(target)
        loss = ctypes.c_double(0)
        _ncheck(_ssn_lib().ssn_backward(self.net, ctypes.c_void_p(t.data_ptr()), t.shape[0], ctypes.byref(loss)))
        return loss.value

    def adam_step(self, lr):
        _ncheck(_ssn_lib().ssn_adam_step(self.net, float(lr)))

    def set_grad_clip(self, max_norm):
        """Global L2-norm gradient clipping of later Adam steps (0 turns it off)."""
        _ncheck(_ssn_lib().ssn_set_grad_clip(self.net, float(max_norm)))

    def train_step(self, x, target, lr, want_loss=True):
        x, t = self._dev(x), self._dev(target)
        loss = ctypes.c_double(0)
        _ncheck(_ssn_lib().ssn_train_step(self.net, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(t.data_ptr()),
                                          x.shape[0], float(lr), ctypes.byref(loss) if want_loss else None))
        return loss.value if want_loss else None

    def flops(self):
        f, b = ctypes.c_double(0), ctypes.c_double(0)
        _ncheck(_ssn_lib().ssn_flops(self.net, ctypes.byref(f), ctypes.byref(b)))
        return f.value, b.value

    def init_field(self, solver, centres, kappa, windings=None, sigma=0.0, pin=0.0, seed=0, noise_amp=0.0):
        """Learned start of solver's lattice in one call (input image, forward, corrected ansatz)."""
        L = _ssn_lib()
        nbytes = L.ssn_init_field_workspace_bytes(self.net)
        work = self.torch.empty(nbytes + 256, dtype=self.torch.uint8, device=self.device)
        ptr = (work.data_ptr() + 255) // 256 * 256
        flat = [float(v) for p in centres for v in p]
        _ncheck(L.ssn_init_field(self.net, solver.ctx, len(flat) // 2, _darr(flat), _darr(windings), float(kappa),
                                 float(sigma), float(pin), int(seed), float(noise_amp), ctypes.c_void_p(ptr), nbytes))

    def close(self):
        if getattr(self, "net", None) is not None:
            _ssn_lib().ssn_destroy(self.net)
            self.net = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
