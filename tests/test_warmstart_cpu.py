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


def test_schedule_rounds_end_at_the_plain_last_eps():
    """A start at eps_1 runs down to the plain schedule's last eps: the plain
    start (eps0) runs all T rounds; a start k halvings in runs T - k."""
    from paper_1501_03105_amd.warmstart import schedule_rounds
    eps0, f, T = 0.1, 0.5, 40
    last = eps0 * f ** (T - 1)
    assert schedule_rounds(eps0, last, f) == T
    for k in range(0, 12):
        assert schedule_rounds(eps0 * f ** k, last, f) == T - k
    assert schedule_rounds(last, last, f) == 1
    assert schedule_rounds(last * 0.1, last, f) == 1          # never fewer than one round
