"""The multi-workgroup CSR path on power-law graphs (Section 3.1's PCG on a
general graph), whose hub rows the SpMV cuts into chunks of a wavefront
each: against the oracle's run of the same graph.  The graphs are R-MAT
FlowImprove instances with rows far longer than the chunking threshold (256
entries), checked at several lanes-per-row settings of the light rows and in
the precision form.

Bars: potentials within 1e-8 of the oracle (FP64), the cut set and value
equal; CG iterations per round within max(3, 2 %); precision form: cut within
1e-4 of the FP64 oracle's."""
import numpy as np
import pytest

import gen
from tests.gpu_util import max_pot_err, say

pytestmark = pytest.mark.gpu

OPTS = dict(rounds=30, cg_rtol=1e-8, solver=1, format=1)
CASES = [(9, 12.0, 12.5), (8, 14.0, 14.5), (11, 15.5, 16.0)]


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available()
    import paper_1501_03105_amd as P
    P.lib()
    return P


def longest_row(g):
    keep = np.ones(g.n, bool)
    keep[[g.s, g.t]] = False
    m = keep[g.eu] & keep[g.ev] & (g.eu != g.ev)
    return int(np.bincount(np.concatenate([g.eu[m], g.ev[m]]), minlength=g.n).max())


@pytest.mark.parametrize("case", range(len(CASES)))
def test_hub_rows_match_oracle(P, oracle_mod, case):
    seed, lo, hi = CASES[case]
    g = gen.rmat_flowimprove(seed, log2_lo=lo, log2_hi=hi)
    longest = longest_row(g)
    assert longest > 256                         # the chunked path runs
    xo, so, _ = oracle_mod.irls(g, rounds=30, cg_rtol=1e-8)
    So, vo, _, _ = oracle_mod.sweep(g, xo)
    it_o = [r["cg_iters"] for r in so]
    for rpw in (0, 1, 32):                       # 0: the default lanes per row
        with P.MinCut.from_graph(g, rows_per_wave=rpw, **OPTS) as mc:
            assert mc.info()["format"] == 1
            rc, st = mc.solve()
            x = mc.potentials()
            S, v, _ = mc.cut()
        err = max_pot_err(x, xo)
        it_g = [r["cg_iters"] for r in st]
        say(f"R-MAT n={g.n} (longest row {longest}), rows per wave {rpw}: potential error {err:.2e}, "
            f"CG {sum(it_g)} (oracle {sum(it_o)})")
        assert rc == P.OK
        assert err <= 1e-8
        assert v == vo and np.array_equal(S, So)
        assert all(abs(a - b) <= max(3, 0.02 * b) for a, b in zip(it_g, it_o))
    with P.MinCut.from_graph(g, precision=1, refine_every=20, **OPTS) as mc:
        rc, st = mc.solve()
        _, vp, _ = mc.cut()
    rel = abs(vp - vo) / vo
    say(f"  precision form: cut relative error vs the FP64 oracle {rel:.2e}")
    assert rc == P.OK and rel <= 1e-4
