"""Host logic of the warm-start driver (no GPU)."""
import math

import pytest


def test_snap_eps_onto_schedule():
    from paper_1501_03105_amd.warmstart import snap_eps
    assert snap_eps(math.log(0.1), 0.1, 0.5, 1e-4) == 0.1
    assert snap_eps(math.log(10.0), 0.1, 0.5, 1e-4) == 0.1             # clamped to eps0
    assert snap_eps(math.log(1e-9), 0.1, 0.5, 1e-4) == pytest.approx(0.1 * 0.5 ** 10)   # 1e-4 -> k = 10
    assert snap_eps(math.log(0.026), 0.1, 0.5, 1e-4) == pytest.approx(0.025)
    assert snap_eps(math.log(1e-3), 0.1, 0.5, 1e-4) == pytest.approx(0.1 * 0.5 ** 7)
