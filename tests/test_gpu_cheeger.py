"""Cheeger-type bracket of the minimum cut (irls_mincut_cheeger_bracket):
the round-0 energy E01 against the oracle's round-0 flow value, the bracket
E01 <= mu* <= 2 sqrt(C E01) against exhaustive and exact minimum cuts, and
when the bracket is (in)valid."""
import numpy as np
import pytest

import gen
from tests.gpu_util import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available()
    import paper_1501_03105_amd as P
    P.lib()
    return P


def test_bracket_small_graphs(P, oracle_mod):
    for seed in range(1, 51):
        g = gen.gnp(16, 0.3, seed=seed)
        with P.MinCut.from_graph(g, rounds=3, cg_rtol=1e-13) as mc:
            mc.solve()
            lo, hi = mc.cheeger_bracket()
        _, R, _ = oracle_mod.irls(g, rounds=0, cg_rtol=1e-14)
        _, mu, _ = oracle_mod.bruteforce(g)
        e0 = R[0]["flow"]
        assert lo == pytest.approx(e0, rel=1e-10)
        assert hi == pytest.approx(2 * np.sqrt(2 * g.cap.sum() * e0), rel=1e-10)
        assert lo <= mu * (1 + 1e-12) and mu <= hi * (1 + 1e-12)


@pytest.mark.parametrize("make", [lambda: gen.grid2d(64, 64, seed=0), lambda: gen.grid3d_seg(24, seed=2)])
def test_bracket_grids(P, oracle_mod, make):
    g = make()
    with P.MinCut.from_graph(g, rounds=2, cg_rtol=1e-12) as mc:
        mc.solve()
        lo, hi = mc.cheeger_bracket()
    _, R, _ = oracle_mod.irls(g, rounds=0, cg_rtol=1e-12)
    _, mu = oracle_mod.maxflow(g)
    say(f"n={g.n}: E01 {lo:.6g} <= mu* {mu:.6g} <= {hi:.6g}")
    assert lo == pytest.approx(R[0]["flow"], rel=1e-9)
    assert lo <= mu * (1 + 1e-9) and mu <= hi


def test_bracket_validity(P):
    g = gen.grid2d(16, 16, seed=1)
    with P.MinCut.from_graph(g, solver=1, rounds=2) as mc:
        with pytest.raises(P.IrlsError) as e:
            mc.cheeger_bracket()
        assert e.value.code == P.ERR_NOT_SOLVED
        mc.solve()
        b0 = mc.cheeger_bracket()
        mc.solve_range(1, 2, eps_first=1e-3)           # later rounds leave round 0 alone
        assert mc.cheeger_bracket() == b0
        mc.update_capacities(g.eu, g.ev, 2.0 * g.cap)
        with pytest.raises(P.IrlsError) as e:
            mc.cheeger_bracket()
        assert e.value.code == P.ERR_NOT_SOLVED
        mc.solve()
        lo, hi = mc.cheeger_bracket()
        assert lo == pytest.approx(2 * b0[0], rel=1e-9) and hi == pytest.approx(2 * b0[1], rel=1e-9)
    with P.MinCut.from_graph(g, solver=1, rounds=2, init=1) as mc:   # no round-0 solve at W = C
        mc.solve()
        with pytest.raises(P.IrlsError):
            mc.cheeger_bracket()
