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


def test_unet_step_bytes_and_roofline_bound():
    """The U-Net step model counts (4 C_in + 5 C_out) BF16 values per pixel and conv
    layer; with one level and base 16 (enc... none, mid.a 2->16, mid.b 16->16 at full
    resolution) that is 2 * N * H * W * ((4*2 + 5*16) + (4*16 + 5*16)) bytes. The
    roofline names HBM below the BF16 ridge (312.5 flop/B) and MFMA above it."""
    import bench
    wl = dict(levels=1, base=16, cin=2, cout=4, N=2, H=8, W=8)
    want = 2 * 2 * 8 * 8 * ((4 * 2 + 5 * 16) + (4 * 16 + 5 * 16))
    assert bench.unet_step_bytes(wl) == want
    r = bench.unet_roofline(100.0, 1e9, 1e11, 1e-3, 50.0)  # 100 flop/B
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["achieved"] == 1000.0 and r["peak"] == 8000.0
    r = bench.unet_roofline(100.0, 1e9, 1e12, 1e-3, 50.0)  # 1000 flop/B
    assert r["bound"] == "mfma" and r["unit"] == "TFLOP/s" and r["achieved"] == 100.0


def test_other_theory_step_models():
    import bench
    assert bench.other_theory_bytes("bs512", {}) == 72
    assert bench.other_theory_bytes("bs512", {}, half_step=True) == 48
    assert bench.other_theory_bytes("bec256", {}) == 352
    assert bench.other_theory_bytes("heusler_demag512", {}, demag_iters=2) == 72 + 48 + 40 + 2 * 210
    assert bench.other_theory_bytes("heusler_demag512", {}, demag_iters=2, half_step=True) == 48 + 36 + 40 + 2 * 210
