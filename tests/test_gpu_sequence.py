"""Sequences of related min-cut problems (irls_mincut_update_capacities):
new capacities on a kept handle give the same results as a new handle with
those capacities, for a fresh solve and for a continuation from the
previous potentials, on the multi-workgroup (scaled marching, CSR) and the
resident solvers; a continuation equals the oracle's continuation from the
same potentials; structure changes are refused."""
import numpy as np
import pytest

import gen
from gen.graphs import Graph
from tests.gpu_util import cmp_stats, max_pot_err, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available()
    import paper_1501_03105_amd as P
    P.lib()
    return P


def perturbed(g, seed, spread=0.2):
    """The same edges with capacities scaled by seeded factors in [1-spread, 1+spread]."""
    f = 1.0 + spread * (2.0 * np.random.default_rng(seed).random(g.cap.shape[0]) - 1.0)
    return Graph(g.n, g.s, g.t, g.eu, g.ev, g.cap * f, meta=dict(g.meta))


CASES = [("seg 24^3 (scaled marching SpMV)", lambda: gen.grid3d_seg(24, seed=2), dict(solver=1)),
         ("grid2d 64x64 as CSR", lambda: gen.grid2d(64, 64, seed=0), dict(solver=1, format=1)),
         ("G(16,0.3) (resident)", lambda: gen.gnp(16, 0.3, seed=5), dict(solver=2))]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_update_equals_new_handle(P, case):
    name, make, kw = CASES[case]
    g1 = make()
    g2 = perturbed(g1, seed=17)
    opts = dict(rounds=20, cg_rtol=1e-10, **kw)
    say(f"capacity update: {name}")
    with P.MinCut.from_graph(g1, **opts) as a, P.MinCut.from_graph(g2, **opts) as b:
        a.solve()
        x1 = a.potentials()
        a.update_capacities(g2.eu, g2.ev, g2.cap)
        # a fresh solve after the update
        _, sa = a.solve()
        _, sb = b.solve()
        xa, xb = a.potentials(), b.potentials()
        assert np.array_equal(xa, xb)
        assert [r["cg_iters"] for r in sa] == [r["cg_iters"] for r in sb]
        Sa, va, ka = a.cut()
        Sb, vb, kb = b.cut()
        assert va == vb and ka == kb and np.array_equal(Sa, Sb)
        # a continuation from the potentials of the old capacities
        a.set_potentials(x1)
        b.set_potentials(x1)
        _, ca = a.solve_range(1, 8, eps_first=1e-3)
        _, cb = b.solve_range(1, 8, eps_first=1e-3)
        assert np.array_equal(a.potentials(), b.potentials())
        assert [r["cg_iters"] for r in ca] == [r["cg_iters"] for r in cb]
        assert a.cut()[1] == b.cut()[1]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_continuation_equals_oracle(P, oracle_mod, case):
    """A continuation after new capacities against the oracle's continuation:
    the oracle solves the old capacities, then runs 12 rounds on the new ones
    from its own potentials (init 2, eps from 1e-3 halved).  The handle solves
    the old capacities, takes the new ones, and continues from the oracle's
    old potentials (potentials within 1e-8, cut set, k* and value equal) and,
    as a sequence really runs, from the potentials it kept."""
    name, make, kw = CASES[case]
    g1 = make()
    g2 = perturbed(g1, seed=17)
    opts = dict(rounds=20, cg_rtol=1e-10)
    x_old, _, _ = oracle_mod.irls(g1, **opts)
    xo, so, _ = oracle_mod.irls(g2, init=2, x0=x_old, eps0=1e-3, rounds=12, cg_rtol=1e-10)
    So, vo, ko, _ = oracle_mod.sweep(g2, xo)
    with P.MinCut.from_graph(g1, **opts, **kw) as mc:
        mc.solve()
        mc.update_capacities(g2.eu, g2.ev, g2.cap)
        _, ck = mc.solve_range(1, 12, eps_first=1e-3)          # from the kept potentials
        xk = mc.potentials()
        Sk, vk, kk = mc.cut()
        mc.set_potentials(x_old)
        _, cs = mc.solve_range(1, 12, eps_first=1e-3)          # from the oracle's
        x = mc.potentials()
        S, v, k = mc.cut()
    err, errk = max_pot_err(x, xo), max_pot_err(xk, xo)
    it_o = [r["cg_iters"] for r in so[1:]]
    say(f"continuation {name}: potentials within {err:.2e} (kept: {errk:.2e}); cut {v!r} / kept {vk!r} / "
        f"oracle {vo!r}; CG per round {[r['cg_iters'] for r in cs[1:]]} vs oracle {it_o}")
    assert err <= 1e-8
    assert v == vo and k == ko and np.array_equal(S, So)
    assert max(abs(a["cg_iters"] - b) for a, b in zip(cs[1:], it_o)) <= 1
    for l in range(1, 13):
        assert cs[l]["eps"] == so[l]["eps"], l
        assert not cmp_stats(cs[l], so[l], rtol=1e-7), (l, cmp_stats(cs[l], so[l], rtol=1e-7))
    assert errk <= 1e-7
    assert vk == vo and kk == ko and np.array_equal(Sk, So)


def test_update_refuses_structure_changes(P):
    g = gen.grid2d(16, 16, seed=1)
    with P.MinCut.from_graph(g, solver=1) as mc:
        # an interior edge less changes the structure (a terminal edge less
        # would not: its node just loses its capacity to s or t)
        for eu, ev, cap, code in [(g.eu[1:], g.ev[1:], g.cap[1:], P.ERR_OPTIONS),
                                  (g.eu, g.ev, np.where(np.arange(g.m) == 3, 0.0, g.cap), P.ERR_CAPACITY)]:
            with pytest.raises(P.IrlsError) as e:
                mc.update_capacities(eu, ev, cap)
            assert e.value.code == code
        # parallel copies and reordering merge to the same structure: accepted
        order = np.random.default_rng(3).permutation(g.m)
        eu = np.concatenate([g.eu[order], g.eu[:5]])
        ev = np.concatenate([g.ev[order], g.ev[:5]])
        cap = np.concatenate([g.cap[order], 0.5 * g.cap[:5]])
        mc.update_capacities(eu, ev, cap)
    b = P.MinCutBatch([gen.gnp(16, 0.3, seed=2)])
    import ctypes as C
    assert P.lib().irls_mincut_update_capacities(b.h, 0, None, None, None) == P.ERR_OPTIONS
    b.close()


def test_sequence_warm_continuation(P, oracle_mod):
    """Measured: after a 20 % capacity change on a 32^3 segmentation grid, the
    kept handle continues from the old potentials; the continuation's cut is
    a valid cut (at least the exact minimum), and both CG counts are shown."""
    g1 = gen.grid3d_seg(32, seed=4)
    g2 = perturbed(g1, seed=23)
    opts = dict(rounds=30, cg_rtol=1e-8, solver=1)
    with P.MinCut.from_graph(g1, **opts) as mc:
        mc.solve()
        mc.update_capacities(g2.eu, g2.ev, g2.cap)
        _, sw = mc.solve_range(1, 12, eps_first=1e-3)
        _, vw, _ = mc.cut()
        _, vw2, _ = mc.cut_two_level()
        _, sf = mc.solve()
        _, vf, _ = mc.cut()
        _, vf2, _ = mc.cut_two_level()
    _, mu = oracle_mod.maxflow(g2)
    itw = sum(r["cg_iters"] for r in sw)
    itf = sum(r["cg_iters"] for r in sf)
    say(f"32^3 after a 20% capacity change: continuation {itw} CG iterations, sweep {(vw - mu) / mu:.2e} / "
        f"two-level {(vw2 - mu) / mu:.2e} above the minimum; full solve {itf} CG iterations, "
        f"{(vf - mu) / mu:.2e} / {(vf2 - mu) / mu:.2e}")
    for v in (vw, vw2, vf, vf2):
        assert v >= mu * (1 - 1e-12)


def test_update_and_potentials_from_either_memory(P):
    """The binding moves arrays to where the handle reads its inputs: torch
    CUDA tensors on a handle created from host arrays, and host arrays on a
    handle created from device tensors, give the host-only results."""
    import torch
    g1 = gen.grid2d(32, 32, seed=3)
    g2 = perturbed(g1, seed=5)
    opts = dict(rounds=12, cg_rtol=1e-10, solver=1)
    cuda = lambda a: torch.as_tensor(np.asarray(a)).cuda()
    with P.MinCut.from_graph(g1, **opts) as ref:
        ref.update_capacities(g2.eu, g2.ev, g2.cap)
        ref.solve()
        x_ref = ref.potentials()
        ref.set_potentials(x_ref)
        _, c_ref = ref.solve_range(1, 4, eps_first=1e-3)
        y_ref = ref.potentials()
    with P.MinCut.from_graph(g1, **opts) as a:                    # host handle, device arrays
        a.update_capacities(cuda(g2.eu), cuda(g2.ev), cuda(g2.cap))
        a.solve()
        assert np.array_equal(a.potentials(), x_ref)
        a.set_potentials(cuda(x_ref))
        _, ca = a.solve_range(1, 4, eps_first=1e-3)
        assert ca == c_ref and np.array_equal(a.potentials(), y_ref)
    with P.MinCut(g1.n, cuda(g1.eu), cuda(g1.ev), cuda(g1.cap), g1.s, g1.t, **opts) as b:   # device handle
        b.update_capacities(g2.eu, g2.ev, g2.cap)
        b.solve()
        assert np.array_equal(b.potentials(), x_ref)
        b.set_potentials(x_ref)
        _, cb = b.solve_range(1, 4, eps_first=1e-3)
        assert cb == c_ref and np.array_equal(b.potentials(), y_ref)
