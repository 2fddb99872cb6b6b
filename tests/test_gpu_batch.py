"""Batched form: many independent graphs in one persistent launch, replayed
from a captured HIP graph.  Each graph is compared with the oracle run on it
alone."""
import numpy as np
import pytest

import gen
from tests.gpu_util import max_pot_err, mk, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available()
    import paper_1501_03105_amd as P
    P.lib()
    return P


def mixed_batch():
    gs = [gen.gnp(16, 0.3, seed=s) for s in range(1, 31)]
    gs += [gen.grid2d(20, 20, seed=3), gen.grid2d(33, 17, seed=4)]
    gs += [gen.rmat_flowimprove(2000 + s, log2_lo=8.0, log2_hi=10.5) for s in range(6)]
    gs += [mk(2, 0, 1, [(0, 1, 0.75)]),                                   # only s and t
           mk(4, 0, 1, [(0, 1, 1.0), (2, 1, 1.0), (3, 2, 1.0)]),          # no source edges
           mk(5, 4, 0, [(4, 2, 1.0), (2, 0, 2.0), (3, 0, 0.5), (4, 0, 0.1), (2, 1, 0.3),
                        (1, 2, 0.2), (1, 1, 7.0), (1, 0, 0.05)])]          # s > t, parallel edges, loop
    return gs


OPTS = dict(rounds=30, cg_rtol=1e-10)


def test_batch_matches_oracle(P, oracle_mod):
    gs = mixed_batch()
    with P.MinCutBatch(gs, **OPTS) as mb:
        rc, st = mb.solve()
        xs = mb.potentials()
        masks, vals = mb.cut()
    assert rc == P.OK
    worst = 0.0
    for g, x, S, v, sg in zip(gs, xs, masks, vals, st):
        xo, so, _ = oracle_mod.irls(g, **OPTS)
        So, vo, _, _ = oracle_mod.sweep(g, xo)
        err = max_pot_err(x, xo)
        worst = max(worst, err)
        # two CG runs to the same rtol 1e-10 may stop a few iterations apart
        # (summation order differs); on these grids that moves potentials by
        # up to ~1e-8 (the oracle alone moves 1.3e-7 between rtol 1e-10 and
        # 1e-13 on the 64x64 grid).  The cuts must agree exactly.
        assert err <= 1e-7
        assert v == vo and np.array_equal(S, So)
        assert all(abs(a["cg_iters"] - b["cg_iters"]) <= max(3, 0.02 * b["cg_iters"])
                   for a, b in zip(sg, so))
    say(f"batch of {len(gs)}: worst potential error {worst:.2e}")


def test_batch_graph_replays(P):
    """The captured solve replayed several times, with other GPU work and
    synchronisations in between, gives the same bits every time."""
    import torch
    gs = mixed_batch()[:20] + [gen.rmat_flowimprove(2100, log2_lo=9.0, log2_hi=11.0)]
    with P.MinCutBatch(gs, rounds=12, cg_rtol=1e-10) as mb:
        ref = None
        for rep in range(4):
            mb.solve()
            xs = mb.potentials()
            masks, vals = mb.cut()
            a = torch.randn(1 << 20, device="cuda")
            (a * 2).sum().item()
            torch.cuda.synchronize()
            cur = (np.concatenate(xs), vals.copy())
            if ref is None:
                ref = cur
            else:
                assert np.array_equal(cur[0], ref[0]) and np.array_equal(cur[1], ref[1]), rep


@pytest.fixture(scope="module")
def rmat512():
    return gen.rmat_batch(512, first_seed=1000)


def test_batch_rmat512_fullsize(P, oracle_mod, rmat512):
    """The 512-instance R-MAT batch (30 rounds, CG to 1e-8): every graph's cut is
    the oracle's exact sweep of the GPU potentials; the smallest graphs are run
    through the oracle's IRLS too; cuts never fall below the exact minimum."""
    gs = rmat512
    opts = dict(rounds=30, cg_rtol=1e-8)
    with P.MinCutBatch(gs, **opts) as mb:
        rc, st = mb.solve()
        xs = mb.potentials()
        masks, vals = mb.cut()
    assert rc == P.OK
    for i, (g, x, S, v) in enumerate(zip(gs, xs, masks, vals)):
        So, vo, _, _ = oracle_mod.sweep(g, x)
        assert v == vo and np.array_equal(S, So), i
    small = np.argsort([g.n for g in gs])[:6]
    errs = []
    for i in small:
        xo, _, _ = oracle_mod.irls(gs[i], **opts)
        _, vo, _, _ = oracle_mod.sweep(gs[i], xo)
        errs.append(max_pot_err(xs[i], xo))
        assert abs(vals[i] - vo) <= 1e-9 * vo, i
        _, mu = oracle_mod.maxflow(gs[i])
        assert vals[i] >= mu
    say(f"rmat512: potential error on the 6 smallest graphs {max(errs):.2e}; "
        f"total CG iterations {sum(r['cg_iters'] for s in st for r in s)}")
    assert max(errs) <= 1e-6


def lane_bounds():
    return [min(2 << b, 64) for b in range(6)]


def check_against_oracle(P, oracle_mod, gs, mb):
    rc, st = mb.solve()
    xs = mb.potentials()
    masks, vals = mb.cut()
    assert rc == P.OK
    for g, x, S, v, sg in zip(gs, xs, masks, vals, st):
        xo, so, _ = oracle_mod.irls(g, **OPTS)
        So, vo, _, _ = oracle_mod.sweep(g, xo)
        assert max_pot_err(x, xo) <= 1e-7
        assert v == vo and np.array_equal(S, So)
        assert all(abs(a["cg_iters"] - b["cg_iters"]) <= max(3, 0.02 * b["cg_iters"])
                   for a, b in zip(sg, so))
    return np.concatenate(xs), vals


@pytest.mark.parametrize("table", ["one lane per row", "half the default"])
def test_batch_row_lanes_match_oracle(P, oracle_mod, table):
    """Fewer lanes per row (each lane then takes several entries of a row)
    only reorders each row's sums: the oracle bars hold, reruns are
    bit-identical, and the captured graph is re-captured with the new table."""
    gs = mixed_batch()
    lanes = [1] * 6 if table == "one lane per row" else [max(1, L // 2) for L in lane_bounds()]
    say(f"row lanes {lanes}")
    with P.MinCutBatch(gs, **OPTS) as mb:
        mb.solve()                                       # captured with the default table
        x_def = np.concatenate(mb.potentials())
        mb.set_row_lanes(lanes)
        x1, v1 = check_against_oracle(P, oracle_mod, gs, mb)
        x2, v2 = check_against_oracle(P, oracle_mod, gs, mb)
        assert np.array_equal(x1, x2) and np.array_equal(v1, v2)
        assert np.max(np.abs(x1 - x_def)) <= 1e-7
        mb.set_row_lanes(lane_bounds())                  # back to the default: the same bits as before
        mb.solve()
        assert np.array_equal(np.concatenate(mb.potentials()), x_def)


def test_batch_autotune(P, oracle_mod):
    """The autotuner returns a valid table, leaves the potentials and the
    solved state in place, and the next solve with its table meets the
    oracle bars."""
    gs = mixed_batch()
    with P.MinCutBatch(gs, **OPTS) as mb:
        mb.solve()
        x0 = np.concatenate(mb.potentials())
        _, v0 = mb.cut()
        lanes = mb.autotune(rounds=2, reps=1)
        say(f"autotuned row lanes {lanes}")
        for L, hi in zip(lanes, lane_bounds()):
            assert 1 <= L <= hi and L & (L - 1) == 0
        assert np.array_equal(np.concatenate(mb.potentials()), x0)
        _, v1 = mb.cut()
        assert np.array_equal(v0, v1)
        check_against_oracle(P, oracle_mod, gs, mb)


def test_single_graph_resident_autotune(P, oracle_mod):
    g = gen.rmat_flowimprove(2003, log2_lo=10.0, log2_hi=10.5)
    with P.MinCut.from_graph(g, solver=2, **OPTS) as mc:
        lanes = mc.autotune(rounds=1, reps=1)
        for L, hi in zip(lanes, lane_bounds()):
            assert 1 <= L <= hi and L & (L - 1) == 0
        mc.set_row_lanes([1] * 6)
        mc.solve()
        x = mc.potentials()
        _, v, _ = mc.cut()
    xo, _, _ = oracle_mod.irls(g, **OPTS)
    _, vo, _, _ = oracle_mod.sweep(g, xo)
    assert max_pot_err(x, xo) <= 1e-7 and v == vo


def test_row_lanes_errors(P):
    g = gen.gnp(16, 0.3, seed=2)
    with P.MinCutBatch([g]) as mb:
        for bad in ([3, 4, 8, 16, 32, 64], [0, 4, 8, 16, 32, 64], [4, 4, 8, 16, 32, 64],
                    [2, 4, 8, 16, 32, 128]):
            with pytest.raises(P.IrlsError) as e:
                mb.set_row_lanes(bad)
            assert e.value.code == P.ERR_OPTIONS
        for rounds, reps in ((-1, 1), (31, 1), (1, 0), (1, 101)):
            with pytest.raises(P.IrlsError) as e:
                mb.autotune(rounds, reps)
            assert e.value.code == P.ERR_OPTIONS
    with P.MinCut.from_graph(gen.grid2d(16, 16, seed=1), solver=1) as mc:   # diagonal format
        mc.solve()
        with pytest.raises(P.IrlsError) as e:
            mc.autotune()                                 # nothing to tune
        assert e.value.code == P.ERR_OPTIONS


def test_csr_rows_per_wave_autotune(P, oracle_mod):
    """The multi-workgroup CSR path: autotuning times its SpMV at each rows
    per wavefront and keeps one; solves with it still meet the oracle bars."""
    for g in (gen.grid2d(64, 64, seed=0), gen.rmat_flowimprove(2003, log2_lo=10.0, log2_hi=10.5)):
        with P.MinCut.from_graph(g, solver=1, format=1, **OPTS) as mc:
            with pytest.raises(P.IrlsError) as e:
                mc.autotune()                             # needs a solved system to time
            assert e.value.code == P.ERR_NOT_SOLVED
            mc.solve()
            lanes = mc.autotune(reps=1)
            assert lanes[0] in (1, 2, 4, 8, 16, 32, 64) and lanes[1:] == [0] * 5
            say(f"CSR n={g.n}: autotuned lanes per row {lanes[0]}")
            mc.solve()
            x = mc.potentials()
            _, v, _ = mc.cut()
        xo, _, _ = oracle_mod.irls(g, **OPTS)
        _, vo, _, _ = oracle_mod.sweep(g, xo)
        assert max_pot_err(x, xo) <= 1e-7 and v == vo
