"""Host-side bookkeeping of the learned-start A/B comparison (no GPU)."""
import pytest

from paper_2603_24370_amd import learned as L


def _rec(ta, sa, ra, tl, sl, rl, coarse=None):
    r = {"ansatz_s": ta, "ansatz_steps": sa, "ansatz_reached": ra,
         "learned_s@3.0": tl, "learned_steps@3.0": sl, "learned_reached@3.0": rl}
    if coarse:
        (cta, csa, cra, ctl, csl, crl) = coarse
        r.update({"ansatz_s~0.001": cta, "ansatz_steps~0.001": csa, "ansatz_reached~0.001": cra,
                  "learned_s@3.0~0.001": ctl, "learned_steps@3.0~0.001": csl, "learned_reached@3.0~0.001": crl})
    return r


def test_summarise_ratios_misses_and_coarse_tolerances():
    recs = [
        _rec(1.0, 100, True, 0.5, 40, True, coarse=(0.4, 40, True, 0.1, 4, True)),
        _rec(2.0, 200, True, 3.0, 300, True, coarse=(0.5, 50, True, 0.2, 10, True)),
        _rec(1.0, 100, True, 9.0, 900, False, coarse=(0.3, 30, True, 0.6, 60, True)),
        _rec(4.0, 400, False, 1.0, 100, True, coarse=(0.2, 20, True, 0.1, 5, True)),
    ]
    s = L.summarise(recs, 3.0, tol=1e-6)
    assert s["tol"] == 1e-6 and s["instances"] == 4
    # only the first two instances count for the ratios
    assert s["both_reached"] == 2 and s["learned_missed"] == 1 and s["ansatz_missed"] == 1
    assert s["median_time_ratio"] == pytest.approx((0.5 + 1.5) / 2)
    assert s["median_step_ratio"] == pytest.approx((0.4 + 1.5) / 2)
    assert s["learned_win_fraction"] == pytest.approx(0.5)
    assert s["total_ansatz_s"] == pytest.approx(8.0) and s["total_learned_s"] == pytest.approx(13.5)
    c = L.summarise(recs, 3.0, coarse=1e-3)
    assert c["tol"] == 1e-3 and c["both_reached"] == 4 and c["learned_missed"] == 0
    # step ratios 0.1, 0.2, 2.0, 0.25: median 0.225
    assert c["median_step_ratio"] == pytest.approx(0.225)
    assert c["learned_win_fraction"] == pytest.approx(0.75)
