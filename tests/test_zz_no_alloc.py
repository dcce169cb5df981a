"""ss_energy_grad_noalloc (no context, no workspace, library-held scratch) against
ss_energy_grad on a context of the same problem, through the C ABI.

Both calls run the same evaluation kernels with the same tile shape and
workgroup count, so the energy reduction has the same order and the result is
expected bit for bit; the test holds it to the parity bar of the evaluation
tests (energy 1e-12 relative, gradient 1e-12 of max|G|) and reports whether it
was bitwise. Two calls in a row, the second on a smaller lattice, so the second
reads a scratch array that still holds the first call's partials.
"""
import numpy as np
import pytest

from paper_2603_24370_amd import inputs as I

pytestmark = pytest.mark.gpu

AH, CM = "abelian_higgs", "chiral_magnet"


def _field(theory, Nx, Ny, h, seed):
    if theory == AH:
        cen = I.uniform_centres(seed, 3, 0.3 * min(Nx, Ny) * h)
        return I.ah_vortex_ansatz(Nx, Ny, h, cen) + I.noise(seed, 4, Nx, Ny, 1e-3)
    f = I.cm_skyrmion_ansatz(Nx, Ny, h, R=min(Nx, Ny) * h / 8)
    return I.renormalise_interior(f + I.noise(seed, 3, Nx, Ny, 1e-3))


CASES = [
    (AH, "f64", 0, [1.0]),
    (AH, "f32", 0, [0.7]),
    (CM, "f32", 0, [1.0, 1.0, 0.1, 0.6]),
    (CM, "f64", 1, [1.0, 1.0, 0.1, 0.6]),
    (AH, "f64", 1, [1.0]),
]


@pytest.mark.parametrize("theory,dtype,mode,params", CASES)
def test_noalloc_matches_context_call_twice(theory, dtype, mode, params):
    import torch
    import paper_2603_24370_amd as ss
    assert torch.cuda.is_available()
    h = 0.2
    tdt = torch.float32 if dtype == "f32" else torch.float64
    code = ss.SS_F32 if dtype == "f32" else ss.SS_F64
    stream = torch.cuda.current_stream()
    for (Nx, Ny) in [(300, 170), (77, 45)]:  # second call smaller
        print(f"[case] noalloc {theory} {dtype} mode={mode} {Nx}x{Ny}", flush=True)
        f = _field(theory, Nx, Ny, h, seed=Nx + Ny)
        ft = torch.as_tensor(f).to(device="cuda:0", dtype=tdt).contiguous()
        g0 = torch.full_like(ft, 7.0)  # the entry point must clear the halo itself
        E0, m0 = ss.ss_energy_grad_noalloc(theory, Nx, Ny, h, params, [mode], code, ft.data_ptr(), g0.data_ptr(),
                                           stream.cuda_stream)
        s = ss.Solver(theory, Nx, Ny, h, params, dtype=dtype, grad_mode=mode)
        E1, m1, g1 = s.energy_grad(field=ft)
        s.close()
        a, b = g0.cpu().numpy().astype(np.float64), g1.cpu().numpy().astype(np.float64)
        bitwise = (E0 == E1) and (m0 == m1) and np.array_equal(a, b)
        print(f"   E {E0!r} vs {E1!r}, max|G| {m0!r} vs {m1!r}, bitwise={bitwise}", flush=True)
        assert E0 == pytest.approx(E1, rel=1e-12, abs=1e-300)
        assert m0 == pytest.approx(m1, rel=1e-12, abs=1e-300)
        assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max()
        # the halo is zero and the interior carries the gradient
        assert not a[:, :2, :].any() and not a[:, -2:, :].any() and not a[:, :, :2].any() and not a[:, :, -2:].any()


def test_noalloc_rejects_bad_arguments():
    import torch
    import paper_2603_24370_amd as ss
    ft = torch.zeros((4, 20, 20), dtype=torch.float64, device="cuda:0")
    with pytest.raises(ss.SSError):
        ss.ss_energy_grad_noalloc(AH, 16, 16, 0.2, [1.0], [], ss.SS_F64, 0, 0, 0)  # no field
    with pytest.raises(ss.SSError):
        ss.ss_energy_grad_noalloc(AH, 4, 16, 0.2, [1.0], [], ss.SS_F64, ft.data_ptr(), 0, 0)  # lattice too small
    with pytest.raises(ss.SSError):
        ss.ss_energy_grad_noalloc("no_such_theory", 16, 16, 0.2, [1.0], [], ss.SS_F64, ft.data_ptr(), 0, 0)
