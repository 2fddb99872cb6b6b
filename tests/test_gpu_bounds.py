"""Per-round lower bound on the minimum cut (irls_round_stats.lower_bound:
the round's electrical flow scaled to respect every capacity) and the
stopping rule built on it (irls_options.stop_gap): the bound against the
oracle's round by round on every solver, below the exact minimum cut, and a
stopped solve equal to the full solve up to the stop round, with the rounds
after it not run and the certified bracket holding."""
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


# (name, graph, solver options); the flows at s and t, hence the bound, carry
# terminal conductances up to c / sqrt(eps), so they are compared at 1e-5
CASES = [("grid2d 64x64, CSR", lambda: gen.grid2d(64, 64, seed=0), dict(solver=1, format=1)),
         ("grid2d 64x64, diagonal", lambda: gen.grid2d(64, 64, seed=0), dict(solver=1, format=2)),
         ("seg 24^3, scaled marching", lambda: gen.grid3d_seg(24, seed=2), dict(solver=1)),
         ("grid2d 64x64, resident", lambda: gen.grid2d(64, 64, seed=0), dict(solver=2))]
OPTS = dict(rounds=30, cg_rtol=1e-10)


def exact_min_cut(oracle_mod, g):
    return oracle_mod.maxflow(g)[1]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_lower_bound_matches_oracle(P, oracle_mod, case):
    name, make, kw = CASES[case]
    g = make()
    with P.MinCut.from_graph(g, **OPTS, **kw) as mc:
        _, st = mc.solve()
    _, so, _ = oracle_mod.irls(g, **OPTS)
    mu = exact_min_cut(oracle_mod, g)
    worst = 0.0
    for l, (a, b) in enumerate(zip(st, so)):
        err = abs(a["lower_bound"] - b["lower_bound"]) / b["lower_bound"]
        worst = max(worst, err)
        assert err <= 1e-5, (l, a["lower_bound"], b["lower_bound"])
        assert a["lower_bound"] <= mu * (1 + 1e-9), l
    assert st[0]["lower_bound"] == pytest.approx(st[0]["flow"], rel=1e-6)
    say(f"{name}: lower bound within {worst:.1e} of the oracle's; last round "
        f"{st[-1]['lower_bound'] / mu:.5f} mu*, l1 {st[-1]['l1'] / mu:.5f} mu*")


def test_lower_bound_batch(P, oracle_mod):
    gs = [gen.gnp(16, 0.3, seed=s) for s in range(1, 21)] + [gen.grid2d(20, 20, seed=3)]
    with P.MinCutBatch(gs, **OPTS) as mb:
        _, sts = mb.solve()
    for g, st in zip(gs, sts):
        _, so, _ = oracle_mod.irls(g, **OPTS)
        mu = exact_min_cut(oracle_mod, g)
        for a, b in zip(st, so):
            assert a["lower_bound"] == pytest.approx(b["lower_bound"], rel=1e-5)
            assert a["lower_bound"] <= mu * (1 + 1e-9)


def first_round_within(st, gap):
    for l, r in enumerate(st):
        if r["l1"] - r["lower_bound"] <= gap * r["l1"]:
            return l
    return None


STOP_CASES = [("G(16,0.3) seed 3, multi-workgroup", lambda: gen.gnp(16, 0.3, seed=3), dict(solver=1), 1e-3),
              ("G(16,0.3) seed 3, resident", lambda: gen.gnp(16, 0.3, seed=3), dict(solver=2), 1e-3),
              ("seg 24^3, scaled marching", lambda: gen.grid3d_seg(24, seed=2), dict(solver=1), 0.06),
              ("grid2d 64x64, CSR", lambda: gen.grid2d(64, 64, seed=0), dict(solver=1, format=1), 0.15)]


@pytest.mark.parametrize("case", range(len(STOP_CASES)))
def test_stop_gap(P, oracle_mod, case):
    """The stopped solve runs exactly the rounds of the full solve up to the
    first round whose certified gap is within stop_gap (records and
    potentials bit-identical), leaves later records empty, and its sweep cut
    lies in [mu*, lower_bound / (1 - stop_gap)]."""
    name, make, kw, gap = STOP_CASES[case]
    g = make()
    with P.MinCut.from_graph(g, **OPTS, **kw) as full:
        _, sf = full.solve()
    L = first_round_within(sf, gap)
    assert L is not None and 0 < L < OPTS["rounds"], L
    with P.MinCut.from_graph(g, **OPTS, **kw) as ref:          # the first L rounds, no stop rule
        ref.solve_range(0, L)
        x_ref = ref.potentials()
    with P.MinCut.from_graph(g, stop_gap=gap, **OPTS, **kw) as mc:
        _, st = mc.solve()
        x = mc.potentials()
        _, val, _ = mc.cut()
    for l in range(L + 1):
        assert st[l] == sf[l], l
    for r in st[L + 1:]:
        assert r["eps"] == 0.0 and r["cg_iters"] == 0
    assert np.array_equal(x, x_ref)
    _, so, _ = oracle_mod.irls(g, **OPTS)
    Lo = first_round_within(so, gap)
    assert Lo is not None and abs(L - Lo) <= 1
    mu = exact_min_cut(oracle_mod, g)
    assert mu * (1 - 1e-12) <= val <= st[L]["lower_bound"] / (1 - gap) * (1 + 1e-9)
    say(f"{name}: stop_gap {gap} stops after round {L} of {OPTS['rounds']} (oracle: {Lo}); "
        f"cut {val:.8g}, mu* {mu:.8g}, certified <= {st[L]['lower_bound'] / (1 - gap):.8g}")


def test_stop_gap_batch(P):
    """Each graph of a batch stops on its own: its records up to its stop
    round equal those of the batch solved without the rule."""
    gs = [gen.gnp(16, 0.3, seed=s) for s in range(1, 11)]
    gap = 1e-3
    with P.MinCutBatch(gs, **OPTS) as mb:
        _, sf = mb.solve()
    with P.MinCutBatch(gs, stop_gap=gap, **OPTS) as mb:
        _, st = mb.solve()
    stopped = 0
    for a, b in zip(st, sf):
        L = first_round_within(b, gap)
        if L is None:                                   # never within the gap: every round runs
            assert a == b
            continue
        stopped += 1
        assert a[:L + 1] == b[:L + 1]
        assert all(r["eps"] == 0.0 and r["cg_iters"] == 0 for r in a[L + 1:])
    assert stopped >= 5


def test_stop_gap_options(P):
    g = gen.grid2d(16, 16, seed=1)
    for bad in (-0.1, 1.0, float("nan")):
        with pytest.raises(P.IrlsError) as e:
            P.MinCut.from_graph(g, stop_gap=bad)
        assert e.value.code == P.ERR_OPTIONS


def test_stop_gap_precision_form_and_continuation(P):
    """The rule on the FP32 form, and on a continuation (solve_range from the
    kept potentials): in both the stopped run equals the run without the rule
    up to its first round within the gap, and later records are empty."""
    g = gen.grid3d_seg(24, seed=2)
    gap = 0.06
    for kw in (dict(precision=1), dict()):
        with P.MinCut.from_graph(g, **OPTS, **kw) as full:
            _, sf = full.solve()
        L = first_round_within(sf, gap)
        assert L is not None and 0 < L < OPTS["rounds"]
        with P.MinCut.from_graph(g, stop_gap=gap, **OPTS, **kw) as mc:
            _, st = mc.solve()
        assert st[:L + 1] == sf[:L + 1]
        assert all(r["eps"] == 0.0 and r["cg_iters"] == 0 for r in st[L + 1:])
    # continuation: rounds 1..12 from the potentials of a 6-round solve
    with P.MinCut.from_graph(g, **OPTS) as a, P.MinCut.from_graph(g, stop_gap=gap, **OPTS) as b:
        a.solve_range(0, 6)
        x6 = a.potentials()
        _, cf = a.solve_range(1, 12, eps_first=1e-2)
        b.set_potentials(x6)
        _, cs = b.solve_range(1, 12, eps_first=1e-2)
    L = first_round_within(cf, gap)
    assert L is not None and L < 12
    assert cs[:L + 1] == cf[:L + 1]
    assert all(r["eps"] == 0.0 and r["cg_iters"] == 0 for r in cs[L + 1:])
    say(f"stop_gap {gap}: precision form and continuation stop where the unstopped runs first reach it")
