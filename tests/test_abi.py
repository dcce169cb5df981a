"""The C-ABI library loads, exports every function declared in include/ss.h, and
validates its arguments on the host (no GPU work is queued by these calls)."""
import ctypes
import os
import re

import pytest

import paper_2603_24370_amd as ss

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "ss.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = set(re.findall(r"^\s*(?:const\s+)?(?:int|void|double|char|ss_ctx)\s*\**\s*(ss_\w+)\s*\(",
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


def test_theory_registry_names_and_aliases(L):
    for name in ["abelian_higgs", "Abelian Higgs", "Ginzburg-Landau", "GL", "ah"]:
        assert ss.ss_theory_id(name) == ss.SS_THEORY_AH
    for name in ["chiral_magnet", "Chiral magnet", "CM"]:
        assert ss.ss_theory_id(name) == ss.SS_THEORY_CM
    assert ss.ss_theory_id("baby_skyrme") < 0
    assert ss.ss_components("GL") == 4 and ss.ss_components("CM") == 3


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
