"""Host helpers of bench.py (no GPU): the kernel-code fingerprint that decides
whether committed traffic counters still describe the built kernels."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_code_only_strips_comments_but_keeps_literals():
    src = ('int a = 1; // note\n/* block\n comment */ const char* s = "x // y \\" z";\n'
           "char q = '\"'; /* tail */\n\n  f();\n")
    out = bench._code_only(src)
    assert "note" not in out and "block" not in out and "tail" not in out
    assert '"x // y \\" z"' in out and "'\"'" in out and "f();" in out
    assert "\n\n" not in out


def test_comment_edits_leave_the_fingerprint_unchanged():
    code = "__global__ void k(float* p) {\n  p[threadIdx.x] = 1.0f;\n}\n"
    assert bench._code_only(code) == bench._code_only("// what k does\n" + code.replace("{\n", "{  /* x */\n"))
    assert bench._code_only(code) != bench._code_only(code.replace("1.0f", "2.0f"))


def test_traffic_record_is_keyed_by_tile_and_source():
    rec = bench.traffic_record("P234", "gl4096", 0)
    # either the committed counters match the current kernel code, or nothing is reported
    assert rec is None or (rec["total_GB"] > 0 and "kernel" in rec)
    assert bench.traffic_record("P234", "gl4096", 99) is None


def test_cpu_baseline_runs_the_oracle_on_every_usable_core(monkeypatch):
    """The CPU leg times the unchanged oracle on one core and on every usable
    core (one window per thread); on a small field both figures are positive
    and the reported core count is the usable count."""
    import numpy as np
    import torch
    from paper_2603_24370_amd import inputs as I
    monkeypatch.setenv("OMP_NUM_THREADS", "3")
    f = I.ah_vortex_ansatz(64, 64, 0.2, [(0.5, -0.3)])

    class FakeSolver:
        def get_field(self):
            return torch.as_tensor(f, dtype=torch.float32)

    wl = dict(theory="abelian_higgs", N=64, h=0.2)
    r = bench.cpu_baseline(FakeSolver(), wl, [1.0], window=32, steps=1)
    assert r["cores"] == min(3, bench.host_cores()) and r["kind"] == "oracle"
    assert r["value"] > 0 and r["value_1core"] > 0 and "32x32" in r["sample"]
