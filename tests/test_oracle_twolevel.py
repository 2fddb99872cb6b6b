"""Pins of the oracle's two-level rounding (the paper's two-level rounding
procedure and its proposition): K-means by hand, the coarse edge weights of
the four cases by hand, the proposition against exhaustive minimum cuts, and
the lifted cut against the exact minimum cut and the sweep cut."""
import numpy as np
import pytest

import gen
from gen.graphs import Graph


@pytest.fixture(scope="module")
def T(oracle_mod):
    from oracle import twolevel
    return twolevel


def test_kmeans_by_hand(T):
    # 0.55 starts in the upper cluster (above 0.5), then the midpoint of
    # (0.345, 0.775) = 0.56 moves it down; the next assignment repeats.
    c0, c1, n = T.kmeans2([0.0, 0.45, 0.46, 0.47, 0.55, 1.0])
    assert n == 2
    assert c0 == pytest.approx(1.93 / 5, abs=1e-15) and c1 == 1.0
    # a well separated set stops after one update at the two means
    c0, c1, n = T.kmeans2([0.0, 0.1, 0.9, 1.0, 1.0])
    assert (c0, n) == (0.05, 1) and c1 == pytest.approx(2.9 / 3, abs=1e-15)
    # an empty upper cluster keeps its starting centre
    c0, c1, n = T.kmeans2([0.0, 0.2, 0.3])
    assert c1 == 0.9 and c0 == pytest.approx(0.5 / 3, abs=1e-15) and n == 1


def test_coarse_edges_by_hand(T):
    # nodes 0..3 interior, s = 4, t = 5; 0 in S1, 1 and 2 in Sc, 3 in S0
    eu = np.array([4, 0, 1, 2, 3, 0, 4, 1, 4])
    ev = np.array([0, 1, 2, 3, 5, 2, 5, 5, 3])
    cap = np.array([1.0, 2.0, 3.0, 0.5, 1.5, 0.25, 0.1, 0.7, 0.2])
    g = Graph(6, 4, 5, eu, ev, cap)
    x = np.array([0.97, 0.6, 0.4, 0.02, 1.0, 0.0])
    cls = T.classify(x, 0.05, 0.95)
    assert list(cls) == [1, 2, 2, 0, 1, 0]
    cg, sc = T.coarse_graph(g, cls)
    assert list(sc) == [1, 2] and (cg.n, cg.s, cg.t) == (4, 2, 3)
    got = {(int(a), int(b)): c for a, b, c in zip(cg.eu, cg.ev, cg.cap)}
    # inside Sc; Sc-S1 -> s_c; Sc-S0 -> t_c; S1-S0 (incl. s-t and s-S0) -> s_c-t_c
    want = {(0, 1): 3.0, (0, 2): 2.0, (0, 3): 0.7, (1, 2): 0.25, (1, 3): 0.5, (2, 3): 0.1 + 0.2}
    assert got.keys() == want.keys()
    for k in want:
        assert got[k] == pytest.approx(want[k], abs=1e-15)


def test_proposition_on_small_graphs(T, oracle_mod):
    """If the exhaustive minimum cut keeps S1 on the source side and S0 on the
    sink side, the lifted coarse minimum cut is a minimum cut; and the lifted
    cut is never below the minimum and equals the coarse cut's value."""
    respected = 0
    for seed in range(1, 51):
        g = gen.gnp(16, 0.3, seed=seed)
        x, _, _ = oracle_mod.irls(g, rounds=20, cg_rtol=1e-12)
        S, val, info = T.two_level(g, x)
        Sb, mu, _ = oracle_mod.bruteforce(g)
        assert S[g.s] and not S[g.t]
        assert val >= mu
        assert val == pytest.approx(info["coarse_value"], rel=1e-12)
        cls = T.classify(x, info["gamma0"], info["gamma1"])
        if Sb[cls == 1].all() and not Sb[cls == 0].any():
            respected += 1
            assert val == mu
    assert respected >= 40


@pytest.mark.parametrize("maker,polarized", [(lambda: gen.grid2d(40, 30, seed=5), False),
                                             (lambda: gen.grid3d_seg(12, seed=2), True)])
def test_grids_against_exact_and_sweep(T, oracle_mod, maker, polarized):
    """On grids the two-level cut reaches the exact minimum (the paper's
    grids show delta 0), and it is never worse than the sweep cut whenever the
    sweep set respects the split.  On the segmentation grid the potentials
    polarise, so the coarse graph is a small fraction of the graph; on the
    2-D grid with terminals only on two sides they do not."""
    g = maker()
    x, _, _ = oracle_mod.irls(g, rounds=25, cg_rtol=1e-10)
    S, val, info = T.two_level(g, x)
    _, mu = oracle_mod.maxflow(g)
    Ssw, vsw, _, _ = oracle_mod.sweep(g, x)
    assert val >= mu * (1 - 1e-12)
    assert (val - mu) / mu <= 1e-9
    cls = T.classify(x, info["gamma0"], info["gamma1"])
    if Ssw[cls == 1].all() and not Ssw[cls == 0].any():
        assert val <= vsw
    if polarized:
        assert info["n_sc"] < g.n // 10
