"""The C-ABI library loads, exports every function declared in include/ss.h, and
validates its arguments on the host (no GPU work is queued by these calls)."""
import ctypes
import os
import re

import pytest

import paper_2603_24370_amd as ss

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions(header="ss.h", prefix="ss_"):
    src = open(os.path.join(ROOT, "include", header)).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = set(re.findall(r"^\s*(?:const\s+)?(?:int|void|double|long|char|size_t|ss_ctx)\s*\**\s*(" + prefix + r"\w+)\s*\(",
                           src, flags=re.M))
    return names


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(ss.LIB_PATH):
        from paper_2603_24370_amd import build
        build.build()
    return ss.lib()


def test_every_declared_symbol_is_exported(L):
    names = _declared_functions()
    assert {"ss_create", "ss_energy_grad", "ss_flow_step", "ss_minimise", "ss_observables", "ss_destroy"} <= names
    for n in names:
        assert hasattr(L, n), n
    assert set(ss.EXPORTS) == names
    nn = _declared_functions("ssn.h", "ssn_")
    assert {"ssn_create", "ssn_forward", "ssn_backward", "ssn_adam_step"} <= nn
    for n in nn:
        assert hasattr(L, n), n
    assert set(ss.SSN_EXPORTS) == nn


def test_network_parameter_count_matches_oracle(L):
    from oracle import unet as U
    import numpy as np
    for lv, base in [(3, 16), (4, 32)]:
        want = sum(int(np.prod(s)) for _, s in U.layer_shapes(lv, base, 2, 4))
        assert ss.ssn_param_count(lv, base, 2, 4) == want


def test_network_validates_shapes(L):
    import ctypes as ct
    n = ct.c_size_t(0)
    assert ss._ssn_lib().ssn_workspace_bytes(4, 32, 2, 4, 8, 100, 256, ct.byref(n)) == -3  # H not a multiple of 128
    assert ss._ssn_lib().ssn_workspace_bytes(4, 24, 2, 4, 8, 256, 256, ct.byref(n)) == -1  # base not a multiple of 16
    assert ss._ssn_lib().ssn_workspace_bytes(4, 32, 2, 4, 8, 256, 256, ct.byref(n)) == 0 and n.value > 0


def test_theory_registry_names_and_aliases(L):
    for name in ["abelian_higgs", "Abelian Higgs", "Ginzburg-Landau", "GL", "ah"]:
        assert ss.ss_theory_id(name) == ss.SS_THEORY_AH
    for name in ["chiral_magnet", "Chiral magnet", "CM"]:
        assert ss.ss_theory_id(name) == ss.SS_THEORY_CM
    for name in ["baby_skyrme", "Baby Skyrme", "BS"]:
        assert ss.ss_theory_id(name) == ss.SS_THEORY_BS
    for name in ["bec", "Bose-Einstein condensate", "bose_einstein"]:
        assert ss.ss_theory_id(name) == ss.SS_THEORY_BEC
    assert ss.ss_theory_id("liquid_crystal") < 0
    assert ss.ss_components("GL") == 4 and ss.ss_components("CM") == 3 and ss.ss_components("BS") == 3
    assert ss.ss_components("BEC") == 2


def test_workspace_bytes_grow_with_size_and_dtype(L):
    a = ss.ss_workspace_bytes("AH", 256, 64, ss.SS_F32)
    b = ss.ss_workspace_bytes("AH", 512, 64, ss.SS_F32)
    c = ss.ss_workspace_bytes("AH", 256, 64, ss.SS_F64)
    assert a < b and a < c
    # seven C-plane field sets (phi x2, v x2, a1, a2, q) dominate
    assert b >= 7 * 4 * (512 + 4) * (64 + 4) * 4


@pytest.mark.parametrize("args,code", [
    (("nope", 64, 64, ss.SS_F32), -2),
    (("AH", 4, 64, ss.SS_F32), -3),
    (("AH", 64, 64, 7), -1),
])
def test_workspace_bytes_rejects_bad_arguments(L, args, code):
    n = ctypes.c_size_t(0)
    assert L.ss_workspace_bytes(args[0].encode(), args[1], args[2], args[3], ctypes.byref(n)) == code
    assert L.ss_last_error().decode()


def test_create_validates_before_any_device_work(L):
    out = ctypes.c_void_p(0)
    f = (ctypes.c_double * 1)(1.0)
    p = ss.ss_params(f, 1, None, 0)
    # no workspace
    assert L.ss_create(b"AH", 64, 64, 0.1, ctypes.byref(p), ss.SS_F32, None, 0, None, ctypes.byref(out)) == -1
    # bad h
    assert L.ss_create(b"AH", 64, 64, -0.1, ctypes.byref(p), ss.SS_F32, ctypes.c_void_p(256), 1 << 40, None,
                       ctypes.byref(out)) == -1
    # wrong parameter count for the chiral magnet
    assert L.ss_create(b"CM", 64, 64, 0.1, ctypes.byref(p), ss.SS_F32, ctypes.c_void_p(256), 1 << 40, None,
                       ctypes.byref(out)) == -1
    # misaligned workspace
    assert L.ss_create(b"AH", 64, 64, 0.1, ctypes.byref(p), ss.SS_F32, ctypes.c_void_p(8), 1 << 40, None,
                       ctypes.byref(out)) == -1
    # courant number outside (0, 1)
    f2 = (ctypes.c_double * 2)(1.0, 1.5)
    p2 = ss.ss_params(f2, 2, None, 0)
    assert L.ss_create(b"AH", 64, 64, 0.1, ctypes.byref(p2), ss.SS_F32, ctypes.c_void_p(256), 1 << 40, None,
                       ctypes.byref(out)) == -1
    assert out.value is None


def test_status_strings_and_kappa_helper(L):
    assert ss.lib().ss_status_string(0) == b"ok"
    assert ss.lib().ss_status_string(-5) == b"non-finite value"
    assert ss.ss_gl_lambda_from_kappa(1 / 2 ** 0.5) == pytest.approx(1.0)


def test_checkpoint_calls_validate_their_arguments(L):
    assert ss.ss_state_bytes() > 0
    buf = ctypes.create_string_buffer(ss.ss_state_bytes())
    assert L.ss_get_state(None, None, None, buf) == -1
    assert L.ss_set_state(None, None, None, buf) == -1


def test_batch_observables_rejects_null_arguments(L):
    out = (ss.ss_obs * 2)()
    assert L.ss_batch_observables(None, out) == -1
    assert L.ss_batch_observables(None, None) == -1


def test_one_call_learned_start_rejects_null_arguments(L):
    N = ss._ssn_lib()
    assert N.ssn_init_field_workspace_bytes(None) == 0
    assert N.ssn_init_field(None, None, 0, None, None, 1.0, 0.0, 0.0, 0, 0.0, None, 0) == -1


def _wsf(theory, f, i, Nx=64, Ny=48, dtype=None):
    fa = (ctypes.c_double * max(1, len(f)))(*f)
    ia = (ctypes.c_int * max(1, len(i)))(*i)
    p = ss.ss_params(fa, len(f), ia, len(i))
    n = ctypes.c_size_t(0)
    rc = ss.lib().ss_workspace_bytes_for(theory.encode(), Nx, Ny, ctypes.byref(p),
                                         ss.SS_F32 if dtype is None else dtype, ctypes.byref(n))
    return rc, n.value


def test_workspace_for_demagnetisation_and_dmi_options(L):
    base = ss.ss_workspace_bytes("CM", 64, 48, ss.SS_F32)
    assert _wsf("CM", [1, 1, 0.1, 0.6], []) == (0, base)
    assert _wsf("CM", [1, 1, 0.1, 0.6], [0, ss.SS_DMI_HEUSLER]) == (0, base)  # Heusler DMI is local
    rc, n = _wsf("CM", [1, 1, 2.0, 0.0, 1.057], [0, ss.SS_DMI_HEUSLER, 1])
    # stage point (3 FP32 planes) + 7 FP64 planes on the lattice + 3 per coarser level
    site = (64 + 4) * (48 + 4)
    assert rc == 0 and n - base >= 10 * 8 * site and n - base < 3 * base
    assert _wsf("AH", [1.0], [0, 0, 1])[0] == -1          # demagnetisation is the chiral magnet's
    assert _wsf("AH", [1.0], [0, ss.SS_DMI_HEUSLER])[0] == -1
    assert _wsf("CM", [1, 1, 2, 0, 1.0], [1, 0, 1])[0] == -1  # exact gradient with demagnetisation
    assert _wsf("CM", [1, 1, 2, 0, 0.0], [0, 0, 1])[0] == -1  # mu_d must be positive
    assert _wsf("CM", [1, 1, 2, 0], [0, 0, 1])[0] == -1       # mu_d missing
    assert _wsf("CM", [1, 1, 2, 0, 1.0], [0, 0, 1, 0])[0] == -1  # ni > 3
    assert _wsf("CM", [1, 1, 2, 0], [0, 2])[0] == -1          # unknown dmi_kind
    assert L.ss_set_demag_iters(None, 2, 40) == -1


def test_integrator_and_form_calls_validate_their_arguments(L):
    """The integrator and velocity Verlet form calls refuse a null context on the
    host, before any device work."""
    assert L.ss_set_integrator(None, ss.SS_INTEG_VV) == -1
    assert L.ss_get_integrator(None) == -1
    assert L.ss_set_vv_form(None, ss.SS_VV_HALF_STEP) == -1
    assert L.ss_get_vv_form(None) == -1
    assert (ss.SS_VV_AUTO, ss.SS_VV_STORED_FORCE, ss.SS_VV_HALF_STEP) == (0, 1, 2)
    assert set(ss.VV_FORMS) == {"auto", "stored_force", "half_step"}
