"""Heuristic-weight calibration arithmetic (Sec. 3.3's two-run procedure)."""
import pytest

from paper_2104_11385_amd.calibrate import heuristic_weights


def test_recovers_linear_model():
    # a machine where a particle costs 3 ns and a cell 1 ns
    n_p, n_c = 27 * 4096, 4096
    t_full = 3e-9 * n_p + 1e-9 * n_c
    t_empty = 1e-9 * n_c
    wp, wc, tp, tc = heuristic_weights(t_full, t_empty, n_p, n_c)
    assert tp == pytest.approx(3e-9, rel=1e-12) and tc == pytest.approx(1e-9, rel=1e-12)
    assert wp == pytest.approx(0.75, rel=1e-12) and wc == pytest.approx(0.25, rel=1e-12)
    assert wp + wc == pytest.approx(1.0, rel=1e-15)


def test_rejects_inconsistent_runs():
    with pytest.raises(ValueError):
        heuristic_weights(1.0, 2.0, 10, 10)
    with pytest.raises(ValueError):
        heuristic_weights(1.0, 0.5, 0, 10)
