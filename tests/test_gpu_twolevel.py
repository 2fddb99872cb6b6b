"""Two-level rounding on the GPU (irls_mincut_cut_two_level) against the
oracle's two-level rounding: on the GPU's own potentials the centres,
thresholds and class sizes agree to rounding, and the lifted cut set and its
exact value are identical; end to end (each side on its own potentials) the
values agree; on the small graphs the result is a minimum cut wherever the
proposition's premise holds."""
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


@pytest.fixture(scope="module")
def T(oracle_mod):
    from oracle import twolevel
    return twolevel


def compare(T, g, x, S, val, info):
    So, vo, io = T.two_level(g, x)
    assert info["c0"] == pytest.approx(io["c0"], abs=1e-12)
    assert info["c1"] == pytest.approx(io["c1"], abs=1e-12)
    assert info["kmeans_updates"] == io["updates"]
    for k in ("n_s0", "n_s1", "n_sc", "coarse_edges"):
        assert info[k] == io[k], k
    assert np.array_equal(S, So)
    assert val == vo
    return vo, io


CASES = [("grid2d 64x64", lambda: gen.grid2d(64, 64, seed=0), dict(rounds=30, cg_rtol=1e-10)),
         ("seg 24^3", lambda: gen.grid3d_seg(24, seed=2), dict(rounds=30, cg_rtol=1e-10)),
         ("box 32x32, 10 planes + 500", lambda: gen.grid3d_box(32, 32, 32 * 32 * 10 + 500, seed=3),
          dict(rounds=20, cg_rtol=1e-10)),
         ("rmat", lambda: gen.rmat_flowimprove(1003), dict(rounds=20, cg_rtol=1e-10))]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_two_level_matches_oracle(P, oracle_mod, T, case):
    name, make, opts = CASES[case]
    g = make()
    say(f"two-level: {name}")
    with P.MinCut.from_graph(g, **opts) as mc:
        mc.solve()
        x = mc.potentials()
        S, val, info = mc.cut_two_level()
        _, vsw, _ = mc.cut()
    assert S[g.s] and not S[g.t]
    assert val == oracle_mod.cut_value(g, S)
    vo, io = compare(T, g, x, S, val, info)
    # end to end: the oracle's own potentials
    xo, _, _ = oracle_mod.irls(g, **opts)
    _, ve, _ = T.two_level(g, xo)
    assert val == pytest.approx(ve, rel=1e-12)
    _, mu = oracle_mod.maxflow(g)
    say(f"  S0 {info['n_s0']} S1 {info['n_s1']} Sc {info['n_sc']} coarse edges {info['coarse_edges']}; "
        f"delta two-level {(val - mu) / mu:.2e}, sweep {(vsw - mu) / mu:.2e}")
    assert val >= mu * (1 - 1e-12)


def test_two_level_small_graphs(P, oracle_mod, T):
    """50 G(16, 0.3) graphs (resident solver): identical to the oracle on the
    same potentials, and a minimum cut whenever the exhaustive minimum cut
    respects the split."""
    respected = 0
    for seed in range(1, 51):
        g = gen.gnp(16, 0.3, seed=seed)
        with P.MinCut.from_graph(g, rounds=20, cg_rtol=1e-12) as mc:
            mc.solve()
            x = mc.potentials()
            S, val, info = mc.cut_two_level()
        compare(T, g, x, S, val, info)
        Sb, mu, _ = oracle_mod.bruteforce(g)
        cls = T.classify(x, info["gamma0"], info["gamma1"])
        if Sb[cls == 1].all() and not Sb[cls == 0].any():
            respected += 1
            assert val == mu
        assert val >= mu
    assert respected >= 40


def test_two_level_errors(P):
    g = gen.grid2d(16, 16, seed=1)
    with P.MinCut.from_graph(g) as mc:
        with pytest.raises(P.IrlsError) as e:
            mc.cut_two_level()
        assert e.value.code == P.ERR_NOT_SOLVED
    b = P.MinCutBatch([gen.gnp(16, 0.3, seed=2), gen.gnp(16, 0.3, seed=3)])
    b.solve()
    mask = np.zeros(64, np.uint8)
    import ctypes as C
    rc = P.lib().irls_mincut_cut_two_level(b.h, mask.ctypes.data_as(C.POINTER(C.c_uint8)), None, None)
    assert rc == P.ERR_OPTIONS
    b.close()
