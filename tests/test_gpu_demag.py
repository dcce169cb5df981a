"""Heusler DMI, the antiskyrmion ansatz and the demagnetising term of the chiral
magnet (Sec. 4.2, eq. (5)-(6)) on the device, through the C ABI, against the FP64
oracle's chiral_magnet_ext theory {J, D, K, B, Dy, mu_d}.

Parameters are those of Fig. 2 made dimensionless with the length J/D and the
energy density D^2/J: J = D = 1, K = 0.8 MJ/m^3 / (D^2/J) = 2, B = 0 and
mu_d = mu_0 M_s^2 / (D^2/J) = 1.057 (J = 40 pJ/m, D = 4 mJ/m^2, M_s = 580 kA/m).

Tolerances. Without demagnetisation, as for the bulk chiral magnet: FP64 gradients
1e-10 of max|G|, energies 1e-12; FP32 gradients within the stencil rounding bound
32 * 2^-24 * 13 * max|n| / h^2. The device solves the potential by preconditioned
conjugate gradients in FP64 (40 iterations for an evaluation, each lowering the
residual about five-fold), the oracle by unpreconditioned conjugate gradients to a
relative residual of 1e-14: both are converged to rounding, so FP64 energies agree
to 1e-11 and gradients to 1e-9 of max|G|; the FP32 bound gains 4 * 2^-24 max|G| for
the demagnetising force's rounding to FP32.
"""
import math

import numpy as np
import pytest

from paper_2603_24370_amd import inputs as I

pytestmark = pytest.mark.gpu

CM, CMX = "chiral_magnet", "chiral_magnet_ext"
EPS32 = 2.0 ** -24
J, D, K, B, MU = 1.0, 1.0, 2.0, 0.0, 1.057


@pytest.fixture(scope="module")
def ss():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2603_24370_amd as m
    m.lib()
    return m


def _np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def _anti(Nx, Ny, h, seed, R=None, amp=1e-2):
    R = R if R is not None else min(Nx, Ny) * h / 6
    f = I.cm_skyrmion_ansatz(Nx, Ny, h, R=R, gamma=-math.pi / 2, vorticity=-1)
    return I.renormalise_interior(f + I.noise(seed, 3, Nx, Ny, amp))


def _oracle_params(dmi, demag):
    return [J, D, K, B, -D if dmi == "heusler" else D, MU if demag else 0.0]


def _solver(ss, Nx, Ny, h, dtype, dmi, demag, mode=0):
    p = [J, D, K, B] + ([MU] if demag else [])
    return ss.Solver(CM, Nx, Ny, h, p, dtype=dtype, grad_mode=mode, dmi=dmi, demag=demag)


def _f32_tol(f, h):
    return 32 * EPS32 * 13 * np.abs(f).max() / h ** 2


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("shape", [(150, 37), (64, 16), (77, 61)])
def test_heusler_energy_and_gradient(ss, orc, dtype, mode, shape):
    Nx, Ny = shape
    h = 0.17
    print(f"[case] heusler energy_grad {dtype} mode={mode} {shape}", flush=True)
    f = _anti(Nx, Ny, h, seed=Nx + 3 * Ny)
    if dtype == "f32":
        f = f.astype(np.float32).astype(np.float64)
    s = _solver(ss, Nx, Ny, h, dtype, "heusler", False, mode)
    s.set_field(f)
    E, gmax, G = s.energy_grad()
    p = _oracle_params("heusler", False)
    G_ref = -orc.acceleration(CMX, f, h, p, mode=orc.GRAD_EL if mode == 0 else orc.GRAD_EXACT)
    assert E == pytest.approx(orc.energy(CMX, f, h, p), rel=1e-12, abs=1e-12)
    scale = np.abs(G_ref).max()
    tol = 1e-10 * scale if dtype == "f64" else _f32_tol(f, h)
    assert np.abs(_np(G) - G_ref).max() <= tol
    s.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("dmi", ["bulk", "heusler"])
@pytest.mark.parametrize("shape", [(64, 48), (77, 61), (150, 37), (8, 8)])
def test_demag_energy_and_gradient(ss, orc, dtype, dmi, shape):
    Nx, Ny = shape
    h = 0.15
    print(f"[case] demag energy_grad {dtype} {dmi} {shape}", flush=True)
    f = _anti(Nx, Ny, h, seed=2 * Nx + Ny)
    if dtype == "f32":
        f = f.astype(np.float32).astype(np.float64)
    s = _solver(ss, Nx, Ny, h, dtype, dmi, True)
    s.set_field(f)
    E, gmax, G = s.energy_grad()
    p = _oracle_params(dmi, True)
    E_ref = orc.energy(CMX, f, h, p)
    E_loc = orc.energy(CMX, f, h, p[:5] + [0.0])
    assert E_ref - E_loc > 1e-6 * abs(E_ref)  # the term is present
    assert E == pytest.approx(E_ref, rel=1e-11, abs=1e-12)
    G_ref = -orc.acceleration(CMX, f, h, p)
    scale = np.abs(G_ref).max()
    tol = 1e-9 * scale if dtype == "f64" else _f32_tol(f, h) + 4 * EPS32 * scale
    assert np.abs(_np(G) - G_ref).max() <= tol
    # observables take the same potential (a fresh solve of the current field)
    o = s.observables()
    assert o["energy"] == pytest.approx(orc.observables(CMX, f, h, p)["E"], rel=1e-11, abs=1e-12)
    s.close()


def test_demag_solver_converges_geometrically(ss, orc):
    """The energy of a fresh context's first evaluation with k iterations (from a
    zero potential) approaches the oracle's: the error falls by at least 10^3 from
    3 to 12 iterations and is at rounding level by 40."""
    Nx, Ny, h = 96, 80, 0.15
    f = _anti(Nx, Ny, h, seed=5)
    p = _oracle_params("heusler", True)
    E_ref = orc.energy(CMX, f, h, p)
    errs = {}
    for k in (3, 6, 12, 40):
        s = _solver(ss, Nx, Ny, h, "f64", "heusler", True)
        s.set_demag_iters(2, k)
        s.set_field(f)
        E, _, _ = s.energy_grad(want_grad=False)
        errs[k] = abs(E - E_ref)
        s.close()
    print(f"[demag] energy error by iterations {errs}", flush=True)
    assert errs[12] <= 1e-3 * errs[3]
    assert errs[40] <= 1e-11 * abs(E_ref)


@pytest.mark.parametrize("how", ["rk4", "vv", "vv_half", "gf"])
def test_demag_flow_tracks_the_oracle(ss, orc, how):
    """With converged solves (30 iterations per stage point) the FP64 flow is the
    oracle's to 1e-9; the stage points of RK4 and of the one-pass integrators get
    their own potentials (velocity Verlet in both of its forms: the half-step
    form's restart and end passes reuse the potential of the field they read)."""
    Nx, Ny, h = 64, 40, 0.15
    print(f"[case] demag flow {how}", flush=True)
    f = _anti(Nx, Ny, h, seed=9)
    s = _solver(ss, Nx, Ny, h, "f64", "heusler", True)
    s.set_demag_iters(30, 40)
    if how != "rk4":
        s.set_integrator("vv" if how == "vv_half" else how)
    if how == "vv_half":
        s.set_vv_form("half_step")
    s.set_field(f)
    n = 6
    info = s.flow_step(n)
    phi, vel = (_np(x) for x in s.get_field(velocity=True))
    p = _oracle_params("heusler", True)
    phi_r, v_r, E_r, na_r = orc.flow(CMX, f, np.zeros_like(f), h, p, n, scheme="vv" if how == "vv_half" else how)
    assert np.abs(phi - phi_r).max() <= 1e-9
    assert np.abs(vel - v_r).max() <= 1e-9
    assert info["step"] == n and info["n_arrests"] == na_r
    assert info["energy"] == pytest.approx(E_r, rel=1e-11)
    s.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_warm_started_solves_track_the_converged_flow(ss, orc, dtype):
    """With the default two iterations per stage point (warm-started from the last
    potential) 20 RK4 steps stay within 1e-4 of the oracle's trajectory, whose
    potentials are exact: the warm start tracks the slowly moving field."""
    Nx, Ny, h = 64, 40, 0.15
    f = _anti(Nx, Ny, h, seed=10)
    if dtype == "f32":
        f = f.astype(np.float32).astype(np.float64)
    s = _solver(ss, Nx, Ny, h, dtype, "heusler", True)
    s.set_field(f)
    n = 20
    s.flow_step(n)
    phi = _np(s.get_field())
    p = _oracle_params("heusler", True)
    phi_r, _, _, _ = orc.flow(CMX, f, np.zeros_like(f), h, p, n)
    err = np.abs(phi - phi_r).max()
    print(f"[demag] {dtype} 2-iteration trajectory error after {n} steps: {err:.3e}", flush=True)
    assert err <= 1e-4
    s.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_antiskyrmion_relaxes_under_demagnetisation(ss, orc, dtype):
    """The Heusler antiskyrmion of Fig. 2 (vorticity -1) relaxed with demagnetisation
    under velocity Verlet (graph replays, two iterations per stage point): the device
    field is a stationary point of the oracle's energy (its projected gradient there
    is below twice the device's stop tolerance), its energy (observables, a fresh
    converged solve) equals the oracle's, its Berg-Luescher charge is +1, and its
    energy lies above the minimum without demagnetisation (the term is >= 0). In
    FP32 the stored field is unit to about 2^-24, so the charge is +1 to 1e-6."""
    N, h = 64, 0.15
    tol = 1e-5 if dtype == "f64" else 2e-3
    print(f"[case] antiskyrmion relax {dtype}", flush=True)
    s = _solver(ss, N, N, h, dtype, "heusler", True)
    s.set_integrator("vv")
    s.init_skyrmion(R=0.6, gamma=-math.pi / 2, vorticity=-1)
    res = s.minimise(grad_tol=tol, max_steps=60000, graph_steps=32)
    assert res["reason"] == "grad", res
    phi = _np(s.get_field())
    p = _oracle_params("heusler", True)
    G = orc.acceleration(CMX, phi, h, p)
    print(f"[demag] {dtype} stop step {res['step']}, E {res['energy']:.10f}, oracle |G| {np.abs(G).max():.3e}",
          flush=True)
    assert np.abs(G).max() <= 2 * tol
    o = s.observables()
    ref = orc.observables(CMX, phi, h, p)
    assert o["energy"] == pytest.approx(ref["E"], rel=1e-11)
    # the charge of the stored field: an integer up to the unit length's rounding
    assert o["q_bl"] == pytest.approx(ref["Q_bl"], abs=1e-9)
    assert abs(o["q_bl"] - 1.0) < (1e-9 if dtype == "f64" else 1e-6)
    s0 = _solver(ss, N, N, h, dtype, "heusler", False)
    s0.set_integrator("vv")
    s0.init_skyrmion(R=0.6, gamma=-math.pi / 2, vorticity=-1)
    r0 = s0.minimise(grad_tol=tol, max_steps=60000, graph_steps=32)
    assert r0["reason"] == "grad"
    assert o["energy"] > s0.observables()["energy"]
    s.close()
    s0.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_device_antiskyrmion_ansatz_matches_input_module(ss, dtype):
    Nx, Ny, h = 70, 45, 0.2
    s = _solver(ss, Nx, Ny, h, dtype, "heusler", False)
    s.init_skyrmion(R=1.1, gamma=0.4, centre=(0.3, -0.2), vorticity=-1)
    want = I.cm_skyrmion_ansatz(Nx, Ny, h, R=1.1, gamma=0.4, centre=(0.3, -0.2), vorticity=-1)
    tol = 1e-13 if dtype == "f64" else 2e-7
    assert np.abs(_np(s.get_field()) - want).max() <= tol
    s.close()


def test_demag_context_refuses_what_it_cannot_run(ss):
    s = _solver(ss, 32, 32, 0.2, "f32", "heusler", True)
    assert s.plan == ss.SS_PLAN_STAGES
    with pytest.raises(ss.SSError):
        s.set_plan(ss.SS_PLAN_FUSED)
    with pytest.raises(ss.SSError):
        s.set_demag_iters(0, 10)
    with pytest.raises(ss.SSError):
        s.init_skyrmion(vorticity=0)
    s.close()
    t = _solver(ss, 32, 32, 0.2, "f32", "heusler", False)
    with pytest.raises(ss.SSError):
        t.set_demag_iters(2, 10)  # no demagnetising term
    t.close()
