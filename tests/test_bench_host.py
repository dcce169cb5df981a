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
