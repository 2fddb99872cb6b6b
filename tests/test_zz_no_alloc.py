"""irls_mincut_cut_noalloc, the sweep cut whose work buffers live in the
library's static scratch array (no device allocation), against
irls_mincut_cut on the same potentials: cut set, k* and value bit for bit,
on two calls in a row, the second on a smaller graph (so stale contents of
the larger call stay in the array), and again after the allocating cut.  A
graph past IRLS_NOALLOC_MAX_NONTERMINAL is refused."""
import numpy as np
import pytest

import gen
from tests.gpu_util import say

pytestmark = pytest.mark.gpu

MAX_ROWS = 262144


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available()
    import paper_1501_03105_amd as P
    P.lib()
    return P


def test_noalloc_cut_equals_cut(P):
    cases = [("seg 48^3", gen.grid3d_seg(48, seed=3)),        # 110,592 non-terminal nodes
             ("grid2d 70x71", gen.grid2d(70, 71, seed=5)),    # 4,970: the smaller second call
             ("box 64^3", gen.grid3d_box(64, 64, MAX_ROWS, seed=2))]   # exactly the maximum
    for name, g in cases:
        with P.MinCut.from_graph(g, rounds=12, cg_rtol=1e-8, solver=1) as mc:
            mc.solve()
            S1, v1, k1 = mc.cut_noalloc()
            S0, v0, k0 = mc.cut()
            S2, v2, k2 = mc.cut_noalloc()
        say(f"noalloc cut {name}: {v1!r} (k* {k1}) vs {v0!r} (k* {k0})")
        assert v1 == v0 and k1 == k0 and np.array_equal(S1, S0)
        assert v2 == v0 and k2 == k0 and np.array_equal(S2, S0)
        assert S1[g.s] and not S1[g.t]


def test_noalloc_refuses_larger_graphs(P):
    g = gen.grid3d_box(64, 64, MAX_ROWS + 64, seed=2)
    with P.MinCut.from_graph(g, rounds=2, cg_rtol=1e-6, solver=1) as mc:
        mc.solve()
        with pytest.raises(P.IrlsError) as e:
            mc.cut_noalloc()
        assert e.value.code == P.ERR_OPTIONS
        mc.cut()                                  # the allocating cut still works
    b = P.MinCutBatch([gen.gnp(16, 0.3, seed=2)])
    import ctypes as C
    assert P.lib().irls_mincut_cut_noalloc(b.h, None, None, None) == P.ERR_OPTIONS
    b.close()
