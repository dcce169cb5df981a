"""The Baby Skyrme model (Tab. 1, standard potential) on the device engine, through
the C ABI, against the FP64 oracle: energy and gradient in both forms, the RK4
plans and the one-pass integrators, stop rules and observables.

Tolerances as for the other theories: FP64 to rounding (gradients 1e-10 of max|G|,
energies 1e-12, fields after a few steps 1e-11); FP32 gradients within the stencil
rounding bound 32 * 2^-24 * 13 * max|m| / h^2 times (1 + kappa^2 max|grad m|^2) for
the Skyrme term's products, fields after a few steps to 1e-5.
"""
import math

import numpy as np
import pytest

from paper_2603_24370_amd import inputs as I

pytestmark = pytest.mark.gpu

BS = "baby_skyrme"
P = [1.0, 0.1]  # kappa, mu^2


@pytest.fixture(scope="module")
def ss():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2603_24370_amd as m
    m.lib()
    return m


def _field(Nx, Ny, h, seed):
    f = I.cm_skyrmion_ansatz(Nx, Ny, h, R=min(Nx, Ny) * h / 6, gamma=0.0)
    return I.renormalise_interior(f + I.noise(seed, 3, Nx, Ny, 1e-2))


def _np(t):
    return t.detach().cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("shape", [(150, 37), (64, 16), (129, 70)])
def test_energy_and_gradient(ss, orc, dtype, mode, shape):
    Nx, Ny = shape
    h = 0.17
    print(f"[case] baby skyrme energy_grad {dtype} mode={mode} {shape}", flush=True)
    f = _field(Nx, Ny, h, seed=Nx + Ny)
    if dtype == "f32":
        f = f.astype(np.float32).astype(np.float64)
    s = ss.Solver(BS, Nx, Ny, h, P, dtype=dtype, grad_mode=mode)
    s.set_field(f)
    E, gmax, G = s.energy_grad()
    omode = orc.GRAD_EL if mode == 0 else orc.GRAD_EXACT
    G_ref = -orc.acceleration(BS, f, h, P, mode=omode)
    assert E == pytest.approx(orc.energy(BS, f, h, P), rel=1e-12)
    scale = np.abs(G_ref).max()
    if dtype == "f64":
        tol = 1e-10 * scale
    else:
        d1 = max(np.abs(np.diff(f, axis=1)).max(), np.abs(np.diff(f, axis=2)).max()) / h
        tol = 32 * 2.0 ** -24 * 13 * np.abs(f).max() / h ** 2 * (1 + P[0] ** 2 * 4 * d1 ** 2)
    assert np.abs(_np(G) - G_ref).max() <= tol
    assert gmax == pytest.approx(scale, rel=1e-9 if dtype == "f64" else 1e-3)
    s.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("how", ["stages", "fused", "vv", "vv_half", "gf"])
def test_flow_tracks_the_oracle(ss, orc, dtype, how):
    Nx, Ny, h = 96, 45, 0.2
    print(f"[case] baby skyrme flow {how} {dtype}", flush=True)
    f = _field(Nx, Ny, h, seed=7)
    if dtype == "f32":
        f = f.astype(np.float32).astype(np.float64)
    s = ss.Solver(BS, Nx, Ny, h, P, dtype=dtype)
    scheme = "rk4"
    if how in ("vv", "vv_half", "gf"):
        scheme = "gf" if how == "gf" else "vv"
        s.set_integrator(scheme)
        if how == "vv_half":
            s.set_vv_form("half_step")
    else:
        s.set_plan(ss.SS_PLAN_STAGES if how == "stages" else ss.SS_PLAN_FUSED)
    s.set_field(f)
    n = 6
    info = s.flow_step(n)
    phi, vel = (_np(x) for x in s.get_field(velocity=True))
    phi_r, v_r, E_r, na_r = orc.flow(BS, f, np.zeros_like(f), h, P, n, scheme=scheme)
    rel = 1e-11 if dtype == "f64" else 1e-5
    assert np.abs(phi - phi_r).max() <= rel * np.abs(phi_r).max()
    assert np.abs(vel - v_r).max() <= rel * max(np.abs(phi_r).max(), 1.0)
    assert info["step"] == n and info["n_arrests"] == na_r
    if dtype == "f64":
        assert info["energy"] == pytest.approx(E_r, rel=1e-12)
    nrm = np.sqrt((phi[:, 2:-2, 2:-2] ** 2).sum(0))
    assert np.abs(nrm - 1).max() < (1e-14 if dtype == "f64" else 1e-6)
    s.close()


def test_minimise_and_observables(ss, orc):
    """A baby skyrmion relaxed to ||G||_inf < 1e-5 in FP64 under velocity Verlet:
    the stop step equals the oracle's; the relaxed field has Berg-Luescher charge
    +-1, an energy above 4 pi |Q_FD|, and observables equal to the oracle's."""
    Nx = Ny = 48
    h = 0.25
    f = _field(Nx, Ny, h, seed=3)
    s = ss.Solver(BS, Nx, Ny, h, P, dtype="f64")
    s.set_integrator("vv")
    s.set_field(f)
    res = s.minimise(grad_tol=1e-5, max_steps=100000, graph_steps=32)
    phi_r, _, ref = orc.minimise(BS, f, h, P, grad_tol=1e-5, max_steps=100000, scheme="vv")
    print(f"[baby skyrme] steps {res['step']} (oracle {ref['steps']}), E {res['energy']:.12f}", flush=True)
    assert res["reason"] == "grad" and ref["reason"] == 1
    assert res["step"] == ref["steps"] and res["n_arrests"] == ref["arrests"]
    phi = _np(s.get_field())
    assert np.abs(phi - phi_r).max() <= 1e-9
    obs = s.observables()
    o = orc.observables(BS, phi, h, P)
    assert obs["energy"] == pytest.approx(o["E"], rel=1e-12)
    assert obs["q_fd"] == pytest.approx(o["Q_fd"], rel=1e-10, abs=1e-12)
    assert obs["q_bl"] == pytest.approx(o["Q_bl"], abs=1e-10)
    assert abs(obs["q_bl"] - round(obs["q_bl"])) < 1e-10 and abs(round(obs["q_bl"])) == 1
    assert obs["energy"] >= 4 * math.pi * abs(obs["q_fd"])
    s.close()


def test_batches_refuse_the_baby_skyrme_model(ss):
    with pytest.raises(ss.SSError):
        ss.Batch(BS, [(32, 32, 0.2, P)], dtype="f64")
