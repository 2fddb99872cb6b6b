"""Reduced-precision form: FP32 conductances, SpMV and CG vectors; FP64
potentials, dot products and residual replacement every 20 CG steps; FP64
conductances once eps < 1e-4.  Bar: cut value within 1e-4 relative of the FP64
oracle; the potential error is measured and printed."""
import numpy as np
import pytest

import gen
from tests.gpu_util import max_pot_err, say

pytestmark = pytest.mark.gpu

MIXED = dict(precision=1, refine_every=20, solver=1)


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available()
    import paper_1501_03105_amd as P
    P.lib()
    return P


def _gpu(P, g, **opts):
    with P.MinCut.from_graph(g, **opts) as mc:
        rc, st = mc.solve()
        x = mc.potentials()
        inS, val, k = mc.cut()
    return rc, st, x, inS, val


@pytest.mark.parametrize("which", ["grid64", "seg48", "seg48-csr"])
def test_mixed_vs_oracle(P, oracle_mod, which):
    if which == "grid64":
        g, opts = gen.grid2d(64, 64, seed=0), dict(rounds=30, cg_rtol=1e-8)
    else:
        g, opts = gen.grid3d_seg(48, seed=3), dict(rounds=40, cg_rtol=1e-8)
    extra = dict(format=1) if which.endswith("csr") else {}
    say(f"mixed {which}")
    xo, so, _ = oracle_mod.irls(g, **opts)
    _, vo, _, _ = oracle_mod.sweep(g, xo)
    rc, st, x, inS, val = _gpu(P, g, **MIXED, **extra, **opts)
    err = max_pot_err(x, xo)
    rel = abs(val - vo) / vo
    say(f"  status {rc}  cut {val:.12g} vs {vo:.12g} rel {rel:.2e}  potential err {err:.2e}  "
        f"CG iters {sum(r['cg_iters'] for r in st)} vs {sum(r['cg_iters'] for r in so)}")
    assert rc == P.OK
    assert rel <= 1e-4
    # every round met the stopping rule on the FP64 true residual
    assert all(r["true_rel_res"] <= 2 * opts["cg_rtol"] for r in st[1:])
    # the sweep of the GPU potentials is an exact cut of G: the oracle agrees
    assert oracle_mod.cut_value(g, inS) == val


def test_mixed_vs_plain_gpu_128(P, oracle_mod):
    """Full-size 128^3 instance: mixed vs the plain FP64 GPU path (which the
    FP64 tests pin to the oracle), and the oracle's exact value of the cut."""
    g = gen.grid3d_seg(128, seed=1)
    opts = dict(rounds=40, cg_rtol=1e-8)
    rc64, st64, x64, S64, v64 = _gpu(P, g, solver=1, **opts)
    rc32, st32, x32, S32, v32 = _gpu(P, g, **MIXED, **opts)
    rel = abs(v32 - v64) / v64
    say(f"128^3 mixed vs fp64: cut rel {rel:.2e}, potential diff {np.max(np.abs(x32 - x64)):.2e}, "
        f"iters {sum(r['cg_iters'] for r in st32)} vs {sum(r['cg_iters'] for r in st64)}")
    assert rc64 == P.OK and rc32 == P.OK
    assert rel <= 1e-4
    assert oracle_mod.cut_value(g, S32) == v32
    assert oracle_mod.cut_value(g, S64) == v64
