"""The stage-kernel report turns rocprofv3 CSVs into per-launch traffic (CPU only)."""
import csv
import json
import os

import pytest

import profile_report as R

CTR_FIELDS = ["Kernel_Name", "Counter_Name", "Counter_Value"]


def _ctr_dir(tmp, name, rows):
    d = tmp / name
    d.mkdir()
    with open(d / "run_counter_collection.csv", "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=CTR_FIELDS)
        w.writeheader()
        for k, c, v in rows:
            w.writerow({"Kernel_Name": f"void {k}(int)", "Counter_Name": c, "Counter_Value": v})
    return str(d)


def test_traffic_is_scaled_by_the_copy_and_matches_the_algorithmic_bytes(tmp_path):
    k1, kf = R.kernel_name("P1", 0), R.kernel_name("P234", 0)
    fused_alg = R.SITES * R.C * R.ELEM * 5  # 3 field sets read, 2 written
    # a 1024 MiB copy: FETCH_SIZE shows half the bytes, WRITE_SIZE all of them
    cf = _ctr_dir(tmp_path, "cf", [(R.COPY_KERNEL, "FETCH_SIZE", 524288.0)])
    cw = _ctr_dir(tmp_path, "cw", [(R.COPY_KERNEL, "WRITE_SIZE", 1048576.0)])
    # the fused pass reads 10% more than its 3 sets (two dispatches, median taken)
    rd = R.SITES * R.C * R.ELEM * 3 * 1.1
    wr = R.SITES * R.C * R.ELEM * 2
    f = _ctr_dir(tmp_path, "f", [(kf, "FETCH_SIZE", rd / 2 / 1024), (kf, "FETCH_SIZE", rd / 2 / 1024),
                                 (k1, "FETCH_SIZE", 1.0)])
    w = _ctr_dir(tmp_path, "w", [(kf, "WRITE_SIZE", wr / 1024), (k1, "WRITE_SIZE", 1.0)])
    sq = [(k, c, 1.0) for k in (k1, kf) for c in ("SQ_INSTS_VALU", "SQ_WAIT_INST_ANY", "SQ_WAVE_CYCLES")]
    lds = [(k, c, 1.0) for k in (k1, kf) for c in ("SQ_INSTS_LDS", "SQ_LDS_BANK_CONFLICT", "SQ_INSTS_SALU")]
    v, l = _ctr_dir(tmp_path, "v", sq), _ctr_dir(tmp_path, "l", lds)
    st = tmp_path / "st"
    st.mkdir()
    with open(st / "run_kernel_stats.csv", "w", newline="") as fh:
        wr_ = csv.DictWriter(fh, fieldnames=["Name", "Calls", "AverageNs"])
        wr_.writeheader()
        wr_.writerow({"Name": f"void {kf}(int)", "Calls": 10, "AverageNs": 600000.0})
        wr_.writerow({"Name": f"void {k1}(int)", "Calls": 10, "AverageNs": 180000.0})
    bl = tmp_path / "bench.log"
    bl.write_text("warm-up\n" + json.dumps({"tile": {"chosen": list(R.TILES[0])}}) + "\n")
    md, js = tmp_path / "o.md", tmp_path / "o.json"
    R.main(["--stats", str(st), "--fetch", f, "--write", w, "--valu", v, "--lds", l, "--bench", str(bl),
            "--copy-fetch", cf, "--copy-write", cw, "--out-md", str(md), "--out-json", str(js)])
    rec = json.loads(js.read_text())
    assert rec["scale"] == {"FETCH_SIZE": 2.0, "WRITE_SIZE": 1.0}
    t = rec["gl4096"]["tile0"]["P234"]
    assert t["algorithmic_GB"] == pytest.approx(fused_alg / 1e9, abs=1e-4)
    assert t["total_GB"] == pytest.approx((rd + wr) / 1e9, abs=1e-4)
    assert t["ratio"] == pytest.approx((rd + wr) / fused_alg, abs=1e-3)
    text = md.read_text()
    assert "P234 (tile 64x16, 2 rows/thread; chosen)" in text and "600.0" in text
