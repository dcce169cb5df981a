"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Both sides receive the same seeded inputs (for FP32 runs the oracle gets the
FP32-rounded field). Tolerances:
  * FP64: gradients to 1e-10 of max|G|, energies to 1e-12 relative, fields
    after a few steps to 1e-11 relative (rounding order only).
  * FP32: energies are reduced in FP64 from the stored values, so E matches
    to 1e-12 relative on the same field; gradients are FP32 stencil
    arithmetic: each of the ~13/h^2-weighted stencil sums rounds at
    2^-24 relative, so |dG| <= 32 * 2^-24 * 13 * max|phi| / h^2 (derived in the
    design notes); fields after a step agree to 1e-5 relative (the stated
    FP32 tolerance of the flow), since G enters the update with weight
    dt^2 / 6 = h^2 / 24.
"""
import math

import numpy as np
import pytest

from paper_2603_24370_amd import inputs as I

pytestmark = pytest.mark.gpu

AH, CM = "abelian_higgs", "chiral_magnet"
P_CM = [1.0, 1.0, 0.1, 0.6]
EPS32 = 2.0 ** -24


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a HIP device"
    return t


@pytest.fixture(scope="module")
def ss(torch):
    import paper_2603_24370_amd as m
    m.lib()
    return m


def _field(theory, Nx, Ny, h, seed, kind="ansatz"):
    if theory == AH:
        if kind == "ansatz":
            L = 0.3 * min(Nx, Ny) * h
            cen = I.uniform_centres(seed, 3, L)
            return I.ah_vortex_ansatz(Nx, Ny, h, cen) + I.noise(seed, 4, Nx, Ny, 1e-3)
        rng = np.random.default_rng(seed)
        return rng.normal(size=(4, Ny + 4, Nx + 4))
    if kind == "ansatz":
        f = I.cm_skyrmion_ansatz(Nx, Ny, h, R=min(Nx, Ny) * h / 8)
        return I.renormalise_interior(f + I.noise(seed, 3, Nx, Ny, 1e-3))
    rng = np.random.default_rng(seed)
    f = rng.normal(size=(3, Ny + 4, Nx + 4))
    return I.renormalise_interior(f)


def _params(theory):
    return [1.0] if theory == AH else P_CM


def _grad_tol(dtype, phi, h):
    if dtype == "f64":
        return None
    return 32 * EPS32 * 13 * np.abs(phi).max() / h ** 2


def _solver(ss, theory, f, h, dtype, params=None):
    C, H, W = f.shape
    s = ss.Solver(theory, W - 4, H - 4, h, params or _params(theory), dtype=dtype)
    return s


def _as_np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def _check_trajectory_energy(E, phi, E_r, phi_r, theory, h, dtype, orc, mode=None):
    """E (device, of its own field phi) against E_r (oracle, of its field phi_r).

    The device reduces E in FP64 from the stored field, so E equals the oracle's
    energy of phi to 1e-12. In FP64 the trajectories agree to rounding and so do
    the energies. In FP32 they differ by the trajectories' distance d = phi - phi_r,
    to first order by h^2 sum G(phi_r) . d; the test allows twice the bound
    h^2 sum |G(phi_r)| |d| of that term plus 1e-12 relative."""
    kw = {} if mode is None else {"mode": mode}
    assert E == pytest.approx(orc.energy(theory, phi, h, _params(theory)), rel=1e-12, abs=1e-12)
    if dtype == "f64":
        assert E == pytest.approx(E_r, rel=1e-12, abs=1e-12)
        return
    G_r = -orc.acceleration(theory, phi_r, h, _params(theory), **kw)
    d = np.abs(phi - phi_r)[:, 2:-2, 2:-2]
    bound = 2.0 * h * h * float((np.abs(G_r[:, 2:-2, 2:-2]) * d).sum()) + 1e-12 * abs(E_r)
    assert abs(E - E_r) <= bound


SHAPES = [(150, 37), (64, 16), (8, 8), (129, 70)]


@pytest.mark.parametrize("theory", [AH, CM])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("shape", SHAPES)
def test_energy_and_gradient(ss, theory, dtype, shape, orc):
    Nx, Ny = shape
    h = 0.17
    print(f"[case] energy_grad {theory} {dtype} {shape}", flush=True)
    f = _field(theory, Nx, Ny, h, seed=Nx * 7 + Ny)
    if dtype == "f32":
        f = f.astype(np.float32).astype(np.float64)
    s = _solver(ss, theory, f, h, dtype)
    s.set_field(f)
    E, gmax, G = s.energy_grad()
    G = _as_np(G)
    E_ref = orc.energy(theory, f, h, _params(theory))
    a_ref = orc.acceleration(theory, f, h, _params(theory))  # -G (projected for CM)
    G_ref = -a_ref
    assert E == pytest.approx(E_ref, rel=1e-12, abs=1e-12)
    scale = np.abs(G_ref).max()
    tol = 1e-10 * scale if dtype == "f64" else _grad_tol(dtype, f, h)
    assert np.abs(G - G_ref).max() <= tol
    assert gmax == pytest.approx(np.abs(G_ref[:, 2:-2, 2:-2]).max(), rel=1e-9 if dtype == "f64" else 1e-4)
    assert np.all(G[:, :2, :] == 0) and np.all(G[:, :, :2] == 0)
    assert np.all(G[:, -2:, :] == 0) and np.all(G[:, :, -2:] == 0)
    # the context's own field gives the same numbers
    E2, g2, _ = s.energy_grad(field=f, want_grad=False)
    assert E2 == E and g2 == gmax
    s.close()


@pytest.mark.parametrize("theory", [AH, CM])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_flow_steps_track_oracle(ss, theory, dtype, orc):
    Nx, Ny, h = 150, 37, 0.17
    print(f"[case] flow {theory} {dtype}", flush=True)
    f = _field(theory, Nx, Ny, h, seed=11)
    if dtype == "f32":
        f = f.astype(np.float32).astype(np.float64)
    s = _solver(ss, theory, f, h, dtype)
    s.set_field(f)
    n = 6
    info = s.flow_step(n)
    phi, vel = s.get_field(velocity=True)
    phi, vel = _as_np(phi), _as_np(vel)
    phi_r, v_r, E_r, na_r = orc.flow(theory, f, np.zeros_like(f), h, _params(theory), n)
    rel = 1e-11 if dtype == "f64" else 1e-5
    assert np.abs(phi - phi_r).max() <= rel * np.abs(phi_r).max()
    assert np.abs(vel - v_r).max() <= rel * max(np.abs(phi_r).max(), 1.0)
    assert info["step"] == n and info["n_arrests"] == na_r
    _check_trajectory_energy(info["energy"], phi, E_r, phi_r, theory, h, dtype, orc)
    # halo is never written
    assert np.array_equal(phi[:, :2, :], f[:, :2, :]) and np.array_equal(phi[:, :, -2:], f[:, :, -2:])
    if theory == CM:
        nrm = np.sqrt((phi[:, 2:-2, 2:-2] ** 2).sum(0))
        assert np.abs(nrm - 1).max() < (1e-14 if dtype == "f64" else 1e-6)
    s.close()


def test_arrests_match_oracle_over_a_long_run(ss, orc):
    """FP64 trajectories agree to rounding, so the arrest pattern must agree too."""
    Nx, Ny, h = 48, 40, 0.25
    f = I.ah_vortex_ansatz(Nx, Ny, h, [(0.3, -0.2), (-1.1, 0.9)]) + I.noise(5, 4, Nx, Ny, 1e-3)
    s = _solver(ss, AH, f, h, "f64")
    s.set_field(f)
    E = None
    phi_r, v_r = f, np.zeros_like(f)
    total = 0
    for chunk in range(4):
        info = s.flow_step(50)
        phi_r, v_r, E, na = orc.flow(AH, phi_r, v_r, h, [1.0], 50, E_cur=E)
        total += na
        assert info["n_arrests"] == total
        assert info["energy"] == pytest.approx(E, rel=1e-11)
    assert total > 0
    phi = _as_np(s.get_field())
    assert np.abs(phi - phi_r).max() < 1e-9
    s.close()


@pytest.mark.parametrize("theory", [AH, CM])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_observables(ss, theory, dtype, orc):
    Nx, Ny, h = 96, 80, 0.2
    f = _field(theory, Nx, Ny, h, seed=3)
    if dtype == "f32":
        f = f.astype(np.float32).astype(np.float64)
    s = _solver(ss, theory, f, h, dtype)
    s.set_field(f)
    o = s.observables()
    r = orc.observables(theory, f, h, _params(theory))
    if theory == AH:
        for k_gpu, k_ref in [("energy", "E"), ("flux", "flux"), ("n_rho", "N_rho"), ("bogo_r1", "R1"),
                             ("bogo_r2", "R2"), ("n_wind", "N_wind")]:
            assert o[k_gpu] == pytest.approx(r[k_ref], rel=1e-11, abs=1e-11), k_gpu
        assert o["n_wind"] == pytest.approx(3.0, abs=1e-12)
    else:
        assert o["energy"] == pytest.approx(r["E"], rel=1e-11)
        assert o["q_fd"] == pytest.approx(r["Q_fd"], rel=1e-11, abs=1e-12)
        assert o["q_bl"] == pytest.approx(r["Q_bl"], abs=1e-11)
        # the solid-angle sum is an integer for exactly unit vectors; FP32 rounding of
        # the stored unit field moves it by O(2^-24) per plaquette
        assert o["q_bl"] == pytest.approx(-1.0, abs=1e-9 if dtype == "f64" else 1e-6)
    s.close()


def test_critical_vortex_minimum_fp64(ss, orc):
    """C1: lambda = 1, 128^2, h = 0.1, FP64, flow to max|G| < 1e-6. E = pi, flux = 2 pi,
    N = 1 within the lattice and box errors; the oracle, polishing from the GPU's
    minimum, moves it by less than the stated tolerances."""
    inst = I.ah_single_vortex(128, 0.1, seed=1)
    f = inst.field()
    s = _solver(ss, AH, f, 0.1, "f64")
    s.set_field(f)
    res = s.minimise(grad_tol=1e-6, max_steps=400000, graph_steps=64)
    print("[C1]", res, flush=True)
    assert res["converged"] and res["reason"] == "grad"
    o = s.observables()
    assert o["energy"] == pytest.approx(math.pi, rel=5e-5)
    assert o["flux"] == pytest.approx(2 * math.pi, rel=2e-3)
    assert o["n_rho"] == pytest.approx(1.0, abs=1e-5)
    assert o["n_wind"] == pytest.approx(1.0, abs=1e-12)
    phi = _as_np(s.get_field())
    # oracle checks: the GPU minimum satisfies the oracle's stop rule
    a = orc.acceleration(AH, phi, 0.1, [1.0])
    assert np.abs(a).max() < 1.01e-6
    assert orc.energy(AH, phi, 0.1, [1.0]) == pytest.approx(o["energy"], rel=1e-12)
    s.close()


def test_minimise_stops_exactly_where_the_oracle_does(ss, orc):
    """The device-side stop rule halts inside a replayed graph at the first state
    meeting the rule: same step count and field as the oracle (FP64)."""
    Nx, Ny, h = 40, 40, 0.25
    f = I.ah_vortex_ansatz(Nx, Ny, h, [(0.2, 0.1)]) + I.noise(8, 4, Nx, Ny, 1e-3)
    s = _solver(ss, AH, f, h, "f64")
    s.set_field(f)
    res = s.minimise(grad_tol=3e-3, max_steps=5000, graph_steps=16)
    phi_r, v_r, info_r = orc.minimise(AH, f, h, [1.0], grad_tol=3e-3, max_steps=5000)
    assert res["reason"] == "grad" and info_r["reason"] == 1
    assert res["step"] == info_r["steps"]
    assert res["n_arrests"] == info_r["arrests"]
    phi = _as_np(s.get_field())
    assert np.abs(phi - phi_r).max() < 1e-10
    s.close()


def test_max_steps_and_stall_rules(ss, orc):
    Nx, Ny, h = 32, 32, 0.25
    f = I.ah_vortex_ansatz(Nx, Ny, h, [(0.2, 0.1)]) + I.noise(8, 4, Nx, Ny, 1e-3)
    s = _solver(ss, AH, f, h, "f64")
    s.set_field(f)
    res = s.minimise(grad_tol=1e-14, max_steps=37, graph_steps=8)
    assert res["rc"] == 1 and res["reason"] == "max_steps" and res["step"] == 37
    s.set_field(f)
    res = s.minimise(grad_tol=0.0, rel_e_tol=1e-4, window=20, max_steps=5000)
    _, _, info_r = orc.minimise(AH, f, h, [1.0], grad_tol=0.0, rel_e_tol=1e-4, window=20, max_steps=5000)
    assert res["reason"] == "stall" and info_r["reason"] == 2
    assert res["step"] == info_r["steps"]
    s.close()


@pytest.mark.parametrize("rel_e_tol", [1e-6, 1e-3])
def test_stall_rule_with_the_largest_window(ss, orc, rel_e_tol):
    """window = 128 (the largest accepted): the energy of step s - 128 must be a
    different ring entry from the one step s writes, else |E - E| = 0 would stop
    the run at step 128. The stop step equals the oracle's (which keeps the
    whole history): 223 and 177 steps here."""
    Nx, Ny, h = 32, 32, 0.25
    print(f"[case] stall window=128 tol={rel_e_tol}", flush=True)
    f = I.ah_vortex_ansatz(Nx, Ny, h, [(0.2, 0.1)]) + I.noise(8, 4, Nx, Ny, 1e-3)
    s = _solver(ss, AH, f, h, "f64")
    s.set_field(f)
    res = s.minimise(grad_tol=0.0, rel_e_tol=rel_e_tol, window=128, max_steps=700, graph_steps=8)
    _, _, info_r = orc.minimise(AH, f, h, [1.0], grad_tol=0.0, rel_e_tol=rel_e_tol, window=128, max_steps=700)
    assert info_r["reason"] == 2 and info_r["steps"] > 128
    assert res["reason"] == "stall"
    assert res["step"] == info_r["steps"] and res["n_arrests"] == info_r["arrests"]
    assert res["energy"] == pytest.approx(info_r["E"], rel=1e-12)
    s.close()


def test_nonfinite_is_reported(ss):
    Nx, Ny, h = 40, 24, 0.25
    f = I.ah_vortex_ansatz(Nx, Ny, h, [(0.2, 0.1)])
    f[1, 10, 13] = np.nan
    s = _solver(ss, AH, f, h, "f32")
    s.set_field(f)
    with pytest.raises(ss.SSError) as e:
        s.energy_grad()
    assert e.value.code == -5
    with pytest.raises(ss.SSError):
        s.minimise(grad_tol=1e-6, max_steps=100)
    s.close()


def test_cm_skyrmion_keeps_charge_minus_one(ss, orc):
    """C2 at reduced size: FP32 field, FP64 reductions; Berg-Luescher charge stays -1."""
    N, h = 128, 0.05 * 4
    inst = I.cm_single_skyrmion(N, h, seed=2)
    f = inst.field().astype(np.float32).astype(np.float64)
    s = _solver(ss, CM, f, h, "f32")
    s.set_field(f)
    s.flow_step(300)
    o = s.observables()
    assert o["q_bl"] == pytest.approx(-1.0, abs=1e-6)
    phi = _as_np(s.get_field())
    assert orc.observables(CM, phi, h, P_CM)["Q_bl"] == pytest.approx(o["q_bl"], abs=1e-9)
    s.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_device_vortex_ansatz_matches_input_module(ss, dtype):
    Nx, Ny, h = 150, 37, 0.2
    cen = [(0.3, -0.4), (-5.0, 1.2), (7.7, 0.0)]
    wnd = [1.0, -1.0, 2.0]
    s = ss.Solver(AH, Nx, Ny, h, [1.0], dtype=dtype)
    s.init_vortices(cen, windings=wnd, seed=77, noise_amp=1e-3)
    got = _as_np(s.get_field())
    want = I.ah_vortex_ansatz(Nx, Ny, h, cen, wnd) + I.noise(77, 4, Nx, Ny, 1e-3)
    tol = 1e-12 if dtype == "f64" else 4e-7 * max(1.0, np.abs(want).max())
    assert np.abs(got - want).max() <= tol
    info = s.info()
    assert info["step"] == 0 and info["n_arrests"] == 0
    s.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_device_skyrmion_ansatz_matches_input_module(ss, dtype):
    Nx, Ny, h = 96, 70, 0.1
    s = ss.Solver(CM, Nx, Ny, h, P_CM, dtype=dtype)
    s.init_skyrmion(R=2.0, gamma=-math.pi / 2, centre=(0.15, -0.05), seed=5, noise_amp=1e-3)
    got = _as_np(s.get_field())
    want = I.renormalise_interior(I.cm_skyrmion_ansatz(Nx, Ny, h, R=2.0, centre=(0.15, -0.05))
                                  + I.noise(5, 3, Nx, Ny, 1e-3))
    tol = 1e-12 if dtype == "f64" else 4e-7
    assert np.abs(got - want).max() <= tol
    s.close()


@pytest.mark.parametrize("dtype,tile", [("f32", 0), ("f32", 1), ("f64", 1)])
def test_fused_pass_with_fewer_workgroups_than_tiles(ss, orc, dtype, tile):
    """A ragged lattice with more tiles (342 on 64 x 16, 684 on 64 x 8) than the
    fused launch has workgroups, so each workgroup walks several column segments:
    every site against the oracle after 3 steps."""
    Nx, Ny, h = 1100, 300, 0.2
    print(f"[case] fused cap {dtype} tile {tile}", flush=True)
    f = _field(AH, Nx, Ny, h, seed=17)
    if dtype == "f32":
        f = f.astype(np.float32).astype(np.float64)
    s = _solver(ss, AH, f, h, dtype)
    s.set_plan(ss.SS_PLAN_FUSED)
    s.set_tile(tile)
    s.set_field(f)
    info = s.flow_step(3)
    phi = _as_np(s.get_field())
    phi_r, _, E_r, na = orc.flow(AH, f, np.zeros_like(f), h, [1.0], 3)
    rel = 1e-11 if dtype == "f64" else 1e-5
    assert np.abs(phi - phi_r).max() <= rel * np.abs(phi_r).max()
    assert info["step"] == 3 and info["n_arrests"] == na
    s.close()


def test_large_lattice_sampled_parity(ss, orc):
    """The 4096^2 GL workload in the launch configuration the benchmark times:
    energy to 1e-9 relative (FP64 reduction of FP32 values vs the oracle's FP64
    sum) and G on sampled 64x64 windows against the oracle on the same windows."""
    N, h = 4096, 0.2
    inst = I.gl_large_instance(N, h)
    lam = I.gl_lambda_from_kappa(1.5)
    s = ss.Solver(AH, N, N, h, [lam], dtype="f32")
    s.init_vortices(inst.centres, seed=4, noise_amp=1e-3)
    E, gmax, G = s.energy_grad()
    f = s.get_field()
    ff = f.double().cpu().numpy()
    E_ref = orc.energy(AH, ff, h, [lam])
    assert E == pytest.approx(E_ref, rel=1e-9)
    Gn = G.cpu().numpy()
    rng = np.random.default_rng(0)
    for k in range(6):
        j0, i0 = (rng.integers(0, N - 64, size=2) if k < 4 else ((0, 0) if k == 4 else (N - 64, N - 64)))
        win = np.ascontiguousarray(ff[:, j0:j0 + 68, i0:i0 + 68])
        # the oracle's interior of this window is the GPU's interior sites (j0..j0+63, i0..i0+63)
        g_ref = -orc.acceleration(AH, win, h, [lam])[:, 2:-2, 2:-2]
        g_gpu = Gn[:, j0 + 2:j0 + 66, i0 + 2:i0 + 66].astype(np.float64)
        assert np.abs(g_gpu - g_ref).max() <= _grad_tol("f32", win, h)
    info = s.flow_step(3)
    assert info["nonfinite"] == 0 and info["step"] == 3
    s.close()


@pytest.mark.parametrize("tile", [0, 1])
def test_large_lattice_fused_step_sampled_parity(ss, orc, tile):
    """One RK4 step of the 4096^2 GL workload under the fused plan (the launch
    configuration the benchmark times), checked on sampled windows: the oracle
    steps a window whose outer ring of M >= 8 sites (four stages of a radius-2
    stencil) is held fixed, so the window's centre is exact."""
    N, h, M, S = 4096, 0.2, 10, 64
    inst = I.gl_large_instance(N, h)
    lam = I.gl_lambda_from_kappa(1.5)
    s = ss.Solver(AH, N, N, h, [lam], dtype="f32")
    s.set_plan(ss.SS_PLAN_FUSED)
    s.set_tile(tile)
    s.init_vortices(inst.centres, seed=4, noise_amp=1e-3)
    f0 = s.get_field().double().cpu().numpy()
    info = s.flow_step(1)
    assert info["step"] == 1 and info["nonfinite"] == 0
    f1 = s.get_field().double().cpu().numpy()
    rng = np.random.default_rng(1)
    origins = [tuple(rng.integers(M, N - S - M, size=2)) for _ in range(5)] + [(0, 0), (N - S, N - S)]
    for j0, i0 in origins:
        # window interior sites [a, b) in each direction, clipped at the lattice (the real halo)
        ja, jb = max(j0 - M, 0), min(j0 + S + M, N)
        ia, ib = max(i0 - M, 0), min(i0 + S + M, N)
        win = np.ascontiguousarray(f0[:, ja:jb + 4, ia:ib + 4])
        w1, _, _, _ = orc.flow(AH, win, np.zeros_like(win), h, [lam], 1)
        got = f1[:, j0 + 2:j0 + S + 2, i0 + 2:i0 + S + 2]
        ref = w1[:, j0 - ja + 2:j0 - ja + S + 2, i0 - ia + 2:i0 - ia + S + 2]
        assert np.abs(got - ref).max() <= 1e-5 * max(np.abs(ref).max(), 1.0), (j0, i0)
    s.close()


def test_batch256_sampled_members_track_the_oracle(ss, orc):
    """The 256-member batch workload in the benchmark's configuration (fused
    plan, tile 0): three steps, then the smallest and largest members and two
    others against the oracle's flow of each member."""
    insts = [I.gl_batch_instance(b, 3000, 0.2) for b in range(256)]
    B = ss.Batch(AH, [(m.Nx, m.Ny, m.h, m.params) for m in insts], dtype="f32")
    assert B.plan == ss.SS_PLAN_FUSED
    for m, mem in zip(insts, B.members):
        mem.init_vortices(m.centres, seed=m.seed, noise_amp=1e-3)
    sides = [m.Nx for m in insts]
    picks = sorted({int(np.argmin(sides)), int(np.argmax(sides)), 17, 200})
    start = {k: B.members[k].get_field().double().cpu().numpy() for k in picks}
    infos = B.flow_step(3)
    for k in picks:
        m = insts[k]
        phi_r, _, E_r, na = orc.flow(AH, start[k], np.zeros_like(start[k]), m.h, m.params, 3)
        phi = B.members[k].get_field().double().cpu().numpy()
        assert np.abs(phi - phi_r).max() <= 1e-5 * np.abs(phi_r).max(), k
        assert infos[k]["step"] == 3 and infos[k]["n_arrests"] == na, k
    B.close()


def test_cm512_skyrmion_relaxes_with_charge_minus_one(ss, orc):
    """The chiral-magnet workload at full size (512^2, h = 0.05, FP32 fields, FP64
    reductions): relaxed to an energy stall, the Berg-Luescher charge is -1 to
    1e-6 and agrees with the oracle's on the same field."""
    N, h = 512, 0.05
    s = ss.Solver(CM, N, N, h, P_CM, dtype="f32")
    s.init_skyrmion(R=2.0, gamma=-math.pi / 2, seed=2, noise_amp=1e-3)
    res = s.minimise(grad_tol=0.0, rel_e_tol=1e-9, window=100, max_steps=40000, graph_steps=32)
    print("[cm512]", res, flush=True)
    assert res["reason"] in ("stall", "max_steps") and res["nonfinite"] == 0
    o = s.observables()
    assert o["q_bl"] == pytest.approx(-1.0, abs=1e-6)
    phi = _as_np(s.get_field())
    assert orc.observables(CM, phi, h, P_CM)["Q_bl"] == pytest.approx(o["q_bl"], abs=1e-9)
    assert o["energy"] == pytest.approx(orc.energy(CM, phi, h, P_CM), rel=1e-12)
    s.close()


@pytest.mark.parametrize("theory,dtype", [(AH, "f32"), (CM, "f64")])
def test_every_tile_shape_matches_oracle(ss, theory, dtype, orc):
    """Each compiled tile shape gives the oracle's flow (ragged lattice)."""
    Nx, Ny, h = 150, 37, 0.17
    f = _field(theory, Nx, Ny, h, seed=21)
    if dtype == "f32":
        f = f.astype(np.float32).astype(np.float64)
    phi_r, v_r, E_r, na_r = orc.flow(theory, f, np.zeros_like(f), h, _params(theory), 4)
    rel = 1e-11 if dtype == "f64" else 1e-5
    for tile in range(ss.ss_tile_count()):
        s = _solver(ss, theory, f, h, dtype)
        s.set_tile(tile)
        s.set_field(f)
        info = s.flow_step(4)
        phi = _as_np(s.get_field())
        assert np.abs(phi - phi_r).max() <= rel * np.abs(phi_r).max(), tile
        _check_trajectory_energy(info["energy"], phi, E_r, phi_r, theory, h, dtype, orc)
        s.close()


PLANS = [("stages", 0), ("fused", 1)]


@pytest.mark.parametrize("plan_name,plan", PLANS)
@pytest.mark.parametrize("theory", [AH, CM])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("shape", [(150, 37), (64, 16), (8, 8), (129, 70)])
@pytest.mark.parametrize("tile", [0, 1])
def test_every_plan_tracks_the_oracle(ss, plan_name, plan, theory, dtype, shape, tile, orc):
    """Each launch plan of a step (separate stage passes, fused stages 2-4) gives
    the oracle's flow: FP64 to rounding, FP32 within the FP32 trajectory bound;
    arrests and steps agree exactly."""
    Nx, Ny = shape
    h = 0.17
    print(f"[case] plan {plan_name} {theory} {dtype} {shape}", flush=True)
    f = _field(theory, Nx, Ny, h, seed=Nx + 3 * Ny)
    if dtype == "f32":
        f = f.astype(np.float32).astype(np.float64)
    s = _solver(ss, theory, f, h, dtype)
    s.set_plan(plan)
    s.set_tile(tile)  # the fused pass follows tiles 0 (64 x 16) and 1 (64 x 8) in FP32
    assert s.plan == plan
    s.set_field(f)
    n = 5
    info = s.flow_step(n)
    phi, vel = s.get_field(velocity=True)
    phi, vel = _as_np(phi), _as_np(vel)
    phi_r, v_r, E_r, na_r = orc.flow(theory, f, np.zeros_like(f), h, _params(theory), n)
    rel = 1e-11 if dtype == "f64" else 1e-5
    assert np.abs(phi - phi_r).max() <= rel * np.abs(phi_r).max()
    assert np.abs(vel - v_r).max() <= rel * max(np.abs(phi_r).max(), 1.0)
    assert info["step"] == n and info["n_arrests"] == na_r
    _check_trajectory_energy(info["energy"], phi, E_r, phi_r, theory, h, dtype, orc)
    assert np.array_equal(phi[:, :2, :], f[:, :2, :]) and np.array_equal(phi[:, :, -2:], f[:, :, -2:])
    s.close()


def test_fused_plan_handles_arrests_like_the_oracle(ss, orc):
    """A long FP64 run under the fused plan: arrests (v -> 0 inside the fused
    stages) fire at the oracle's steps."""
    Nx, Ny, h = 48, 40, 0.25
    f = I.ah_vortex_ansatz(Nx, Ny, h, [(0.3, -0.2), (-1.1, 0.9)]) + I.noise(5, 4, Nx, Ny, 1e-3)
    for plan in (1,):
        s = _solver(ss, AH, f, h, "f64")
        s.set_plan(plan)
        s.set_field(f)
        E = None
        phi_r, v_r = f, np.zeros_like(f)
        total = 0
        for chunk in range(4):
            info = s.flow_step(50)
            phi_r, v_r, E, na = orc.flow(AH, phi_r, v_r, h, [1.0], 50, E_cur=E)
            total += na
            assert info["n_arrests"] == total
            assert info["energy"] == pytest.approx(E, rel=1e-11)
        assert total > 0
        assert np.abs(_as_np(s.get_field()) - phi_r).max() < 1e-9
        s.close()


def test_fused_plan_minimise_stops_where_the_oracle_does(ss, orc):
    Nx, Ny, h = 40, 40, 0.25
    f = I.ah_vortex_ansatz(Nx, Ny, h, [(0.2, 0.1)]) + I.noise(8, 4, Nx, Ny, 1e-3)
    s = _solver(ss, AH, f, h, "f64")
    s.set_plan(1)
    s.set_field(f)
    res = s.minimise(grad_tol=3e-3, max_steps=5000, graph_steps=16)
    phi_r, v_r, info_r = orc.minimise(AH, f, h, [1.0], grad_tol=3e-3, max_steps=5000)
    assert res["reason"] == "grad" and res["step"] == info_r["steps"] and res["n_arrests"] == info_r["arrests"]
    assert np.abs(_as_np(s.get_field()) - phi_r).max() < 1e-10
    s.close()


def test_exact_mode_rejects_fused_plans(ss):
    s = ss.Solver(AH, 64, 64, 0.2, [1.0], dtype="f32", grad_mode=ss.SS_GRAD_EXACT)
    assert s.plan == 0
    with pytest.raises(ss.SSError):
        s.set_plan(1)
    s.close()


def test_autotune_picks_a_shape_and_leaves_a_usable_context(ss, orc):
    Nx, Ny, h = 256, 96, 0.2
    f = _field(AH, Nx, Ny, h, seed=5).astype(np.float32).astype(np.float64)
    s = _solver(ss, AH, f, h, "f32")
    best, plan, ms = s.autotune(3)
    flat = [m for row in ms for m in row]
    assert 0 <= best < ss.ss_tile_count() and 0 <= plan < ss.SS_NUM_PLANS
    assert ms[plan][best] == min(flat) and all(m > 0 for m in flat)
    assert s.plan == plan
    s.set_field(f)
    E, _, _ = s.energy_grad(want_grad=False)
    assert E == pytest.approx(orc.energy(AH, f, h, [1.0]), rel=1e-12)
    s.close()


@pytest.mark.parametrize("theory,dtype,plan", [(AH, "f64", 0), (AH, "f32", 1), (CM, "f64", 0), (CM, "f32", 1)])
def test_checkpoint_resumes_the_flow_bitwise(ss, orc, theory, dtype, plan):
    Nx, Ny, h = 90, 70, 0.2
    f = _field(theory, Nx, Ny, h, seed=8)
    if dtype == "f32":
        f = f.astype(np.float32).astype(np.float64)
    s = _solver(ss, theory, f, h, dtype)
    s.set_plan(plan)
    s.set_field(f)
    s.flow_step(7)
    state = s.get_state()
    s.flow_step(9)
    a, va = s.get_field(velocity=True)
    ia = s.info()
    s2 = _solver(ss, theory, f, h, dtype)
    s2.set_plan(plan)
    s2.set_state(state)
    assert s2.info()["step"] == 7
    s2.flow_step(9)
    b, vb = s2.get_field(velocity=True)
    ib = s2.info()
    assert bool((a == b).all()) and bool((va == vb).all())
    assert (ia["step"], ia["n_arrests"], ia["energy"]) == (ib["step"], ib["n_arrests"], ib["energy"])
    # the same flow in the oracle over all 16 steps
    phi_r, _, E_r, na = orc.flow(theory, f, np.zeros_like(f), h, _params(theory), 16)
    if dtype == "f64":
        assert ib["n_arrests"] == na
    # an FP32 run that arrests at other steps than the FP64 oracle follows
    # another trajectory; the field comparison needs the same arrest pattern
    if ib["n_arrests"] == na:
        rel = 1e-11 if dtype == "f64" else 1e-5
        assert np.abs(_as_np(b) - phi_r).max() <= rel * np.abs(phi_r).max()
    # a checkpoint of another lattice is refused
    s3 = _solver(ss, theory, _field(theory, Nx + 2, Ny, h, seed=8), h, dtype)
    with pytest.raises(Exception):
        s3.set_state((state[0], state[1], state[2]))
    for x in (s, s2, s3):
        x.close()


def test_checkpoint_refuses_damaged_or_foreign_blobs(ss):
    Nx, Ny, h = 40, 36, 0.2
    f = _field(AH, Nx, Ny, h, seed=2)
    s = _solver(ss, AH, f, h, "f64")
    s.set_field(f)
    s.flow_step(3)
    fv, vv, blob = s.get_state()
    s32 = _solver(ss, AH, f, h, "f32")
    with pytest.raises(ss.SSError) as e:  # taken in FP64, offered to an FP32 context
        s32.set_state((fv, vv, blob))
    assert e.value.code == ss.SS_ESHAPE
    bad = bytearray(blob)
    bad[0] ^= 0xFF  # magic number
    with pytest.raises(ss.SSError) as e:
        s.set_state((fv, vv, bytes(bad)))
    assert e.value.code == ss.SS_EINVAL
    with pytest.raises(ValueError):  # truncated
        s.set_state((fv, vv, blob[:-8]))
    # the refused calls left the context as it was
    assert s.info()["step"] == 3
    s.set_state((fv, vv, blob))
    assert s.info()["step"] == 3
    s.close()
    s32.close()


def test_checkpoint_resumes_a_minimisation(ss, orc):
    """FP64: a minimisation resumed from a checkpoint in a fresh context stops at the
    step, with the arrest count and field, of the one that was not interrupted, and
    both stop where the oracle's flow from the start does."""
    Nx, Ny, h = 48, 40, 0.2
    f = _field(AH, Nx, Ny, h, seed=9)
    s = _solver(ss, AH, f, h, "f64")
    s.set_field(f)
    s.flow_step(7)
    state = s.get_state()
    ra = s.minimise(grad_tol=2e-3, max_steps=3000, graph_steps=8)
    a = s.get_field()
    s2 = _solver(ss, AH, f, h, "f64")
    s2.set_state(state)
    rb = s2.minimise(grad_tol=2e-3, max_steps=3000, graph_steps=8)
    b = s2.get_field()
    assert (ra["step"], ra["n_arrests"], ra["reason"]) == (rb["step"], rb["n_arrests"], rb["reason"])
    assert ra["reason"] == "grad"
    assert bool((a == b).all())
    phi_r, _, info_r = orc.minimise(AH, f, h, [1.0], grad_tol=2e-3, max_steps=3000)
    assert ra["step"] == info_r["steps"] and ra["n_arrests"] == info_r["arrests"]
    assert np.abs(_as_np(b) - phi_r).max() < 1e-9
    s.close()
    s2.close()


def test_autotune_cache_serves_the_stored_choice(ss, orc, tmp_path, monkeypatch):
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("SS_AUTOTUNE_CACHE", str(cache))
    Nx, Ny, h = 160, 72, 0.2
    f = _field(AH, Nx, Ny, h, seed=6).astype(np.float32).astype(np.float64)
    s = _solver(ss, AH, f, h, "f32")
    best, plan, ms = s.autotune(2)
    assert all(m > 0 for row in ms for m in row)  # timed
    assert cache.read_text().split()[-2:] == [str(plan), str(best)]
    s.close()
    # the same problem in a new context: stored plan and tile, nothing timed, field untouched
    s2 = _solver(ss, AH, f, h, "f32")
    s2.set_field(f)
    s2.set_plan(1 - plan)
    s2.set_tile((best + 1) % ss.ss_tile_count())
    best2, plan2, ms2 = s2.autotune(2)
    assert (best2, plan2) == (best, plan) and ss.ss_get_tile(s2.ctx) == best and s2.plan == plan
    assert all(m == -1.0 for row in ms2 for m in row)
    E, _, _ = s2.energy_grad(want_grad=False)
    assert E == pytest.approx(orc.energy(AH, f, h, [1.0]), rel=1e-12)
    s2.close()
    # another lattice size is tuned and appended
    g = _field(AH, Nx + 32, Ny, h, seed=6).astype(np.float32).astype(np.float64)
    s3 = _solver(ss, AH, g, h, "f32")
    _, _, ms3 = s3.autotune(1)
    assert all(m > 0 for row in ms3 for m in row)
    assert len(cache.read_text().strip().splitlines()) == 2
    s3.close()


# ------------------------------------------------ exact discrete gradient (SS_GRAD_EXACT)

EXACT_SHAPES = [(150, 37), (8, 8), (129, 70), (64, 16)]


# the FP32 rounding bound of this test is derived for smooth fields, so random
# fields are checked in FP64 only
EXACT_CASES = [(dtype, kind) for dtype in ("f64", "f32") for kind in ("ansatz", "random")
               if not (dtype == "f32" and kind == "random")]


@pytest.mark.parametrize("theory", [AH, CM])
@pytest.mark.parametrize("shape", EXACT_SHAPES)
@pytest.mark.parametrize("dtype,kind", EXACT_CASES)
def test_exact_gradient_matches_oracle(ss, theory, dtype, shape, kind, orc):
    """G = h^-2 dE_h/dphi on the device against the oracle's scatter-form chain rule."""
    Nx, Ny = shape
    h = 0.17
    print(f"[case] exact energy_grad {theory} {dtype} {shape} {kind}", flush=True)
    f = _field(theory, Nx, Ny, h, seed=Nx * 5 + Ny, kind=kind)
    if dtype == "f32":
        f = f.astype(np.float32).astype(np.float64)
    s = ss.Solver(theory, Nx, Ny, h, _params(theory), dtype=dtype, grad_mode=ss.SS_GRAD_EXACT)
    s.set_field(f)
    E, gmax, G = s.energy_grad()
    G = _as_np(G)
    E_ref = orc.energy(theory, f, h, _params(theory))
    G_ref = -orc.acceleration(theory, f, h, _params(theory), mode=orc.GRAD_EXACT)
    assert E == pytest.approx(E_ref, rel=1e-12, abs=1e-12)
    tol = 1e-10 * np.abs(G_ref).max() if dtype == "f64" else _grad_tol(dtype, f, h)
    assert np.abs(G - G_ref).max() <= tol
    assert gmax == pytest.approx(np.abs(G_ref[:, 2:-2, 2:-2]).max(), rel=1e-9 if dtype == "f64" else 1e-4)
    assert np.all(G[:, :2, :] == 0) and np.all(G[:, :, -2:] == 0)
    s.close()


def test_exact_gradient_differs_from_euler_lagrange(ss, orc):
    """The two modes are distinct operators (they agree only to O(h^4) on smooth fields)."""
    Nx, Ny, h = 64, 48, 0.2
    f = _field(AH, Nx, Ny, h, seed=3, kind="random")
    se = ss.Solver(AH, Nx, Ny, h, [1.0], dtype="f64", grad_mode=ss.SS_GRAD_EXACT)
    sl = ss.Solver(AH, Nx, Ny, h, [1.0], dtype="f64")
    se.set_field(f)
    sl.set_field(f)
    _, _, Ge = se.energy_grad()
    _, _, Gl = sl.energy_grad()
    assert np.abs(_as_np(Ge) - _as_np(Gl)).max() > 1e-2
    se.close()
    sl.close()


@pytest.mark.parametrize("theory", [AH, CM])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_exact_flow_steps_track_oracle(ss, theory, dtype, orc):
    Nx, Ny, h = 150, 37, 0.17
    print(f"[case] exact flow {theory} {dtype}", flush=True)
    f = _field(theory, Nx, Ny, h, seed=13)
    if dtype == "f32":
        f = f.astype(np.float32).astype(np.float64)
    s = ss.Solver(theory, Nx, Ny, h, _params(theory), dtype=dtype, grad_mode=ss.SS_GRAD_EXACT)
    s.set_field(f)
    n = 6
    info = s.flow_step(n)
    phi, vel = s.get_field(velocity=True)
    phi, vel = _as_np(phi), _as_np(vel)
    phi_r, v_r, E_r, na_r = orc.flow(theory, f, np.zeros_like(f), h, _params(theory), n, mode=orc.GRAD_EXACT)
    rel = 1e-11 if dtype == "f64" else 1e-5
    assert np.abs(phi - phi_r).max() <= rel * np.abs(phi_r).max()
    assert np.abs(vel - v_r).max() <= rel * max(np.abs(phi_r).max(), 1.0)
    assert info["step"] == n and info["n_arrests"] == na_r
    _check_trajectory_energy(info["energy"], phi, E_r, phi_r, theory, h, dtype, orc, mode=orc.GRAD_EXACT)
    s.close()


def test_exact_minimise_stops_where_the_oracle_does(ss, orc):
    """FP64 arrested flow of a chiral-magnet skyrmion under the exact gradient:
    same stop step, arrests and field (to rounding)."""
    Nx, Ny, h = 48, 48, 0.2
    f = I.renormalise_interior(I.cm_skyrmion_ansatz(Nx, Ny, h, R=1.5) + I.noise(9, 3, Nx, Ny, 1e-3))
    s = ss.Solver(CM, Nx, Ny, h, P_CM, dtype="f64", grad_mode=ss.SS_GRAD_EXACT)
    s.set_field(f)
    res = s.minimise(grad_tol=1e-3, max_steps=5000, graph_steps=16)
    phi_r, v_r, info_r = orc.minimise(CM, f, h, P_CM, grad_tol=1e-3, max_steps=5000, mode=orc.GRAD_EXACT)
    assert res["reason"] == "grad" and info_r["reason"] == 1
    assert res["step"] == info_r["steps"] and res["n_arrests"] == info_r["arrests"]
    assert np.abs(_as_np(s.get_field()) - phi_r).max() < 1e-10
    s.close()


def test_exact_minimise_of_vortices_follows_the_oracle(ss, orc):
    """Abelian Higgs vortices under the exact gradient: the odd-even modes of eq. (1)
    are unstable in the vortex cores, so differences of rounding grow along the run
    (the oracle moves by 5e-7 from a 1e-15 change of one input value). Step count,
    arrests and energy still match; the field agrees to the growth the oracle shows."""
    Nx, Ny, h = 40, 36, 0.25
    f = I.ah_vortex_ansatz(Nx, Ny, h, [(0.3, -0.2), (-1.1, 0.9)]) + I.noise(9, 4, Nx, Ny, 1e-3)
    s = ss.Solver(AH, Nx, Ny, h, [1.0], dtype="f64", grad_mode=ss.SS_GRAD_EXACT)
    s.set_field(f)
    res = s.minimise(grad_tol=3e-3, max_steps=5000, graph_steps=16)
    phi_r, v_r, info_r = orc.minimise(AH, f, h, [1.0], grad_tol=3e-3, max_steps=5000, mode=orc.GRAD_EXACT)
    g = f.copy()
    g[0, 20, 20] *= 1 + 1e-15
    phi_p, _, _ = orc.minimise(AH, g, h, [1.0], grad_tol=3e-3, max_steps=5000, mode=orc.GRAD_EXACT)
    growth = np.abs(phi_p - phi_r).max()
    assert growth > 1e-9  # the instability is there
    assert res["reason"] == "grad" and info_r["reason"] == 1
    assert res["step"] == info_r["steps"] and res["n_arrests"] == info_r["arrests"]
    assert res["energy"] == pytest.approx(info_r["E"], rel=1e-9)
    assert np.abs(_as_np(s.get_field()) - phi_r).max() < 100 * growth
    s.close()


def test_exact_mode_fixes_the_tile_shape(ss):
    s = ss.Solver(AH, 64, 64, 0.2, [1.0], dtype="f32", grad_mode=ss.SS_GRAD_EXACT)
    with pytest.raises(ss.SSError):
        s.set_tile(1)
    s.set_tile(0)
    s.close()
