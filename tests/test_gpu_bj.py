"""Block-Jacobi preconditioning (Section 3.1, eq. block-jacobi-subsystem) on
the GPU against the oracle's block-Jacobi PCG, with the paper's two block
solvers: exact solves of blocks of consecutive rows inside one line of
offset-1 edges (tridiagonal), applied by wavefront scans; and ILU(0) of
cubic tiles of 3-D grids (precond 2, tile edges 2, 4 and 8), against the oracle's
ILU(0) of the same tiles given as block ids."""
import numpy as np
import pytest

import gen
from tests.gpu_util import max_pot_err, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available()
    import paper_1501_03105_amd as P
    P.lib()
    return P


OPTS = dict(rounds=20, cg_rtol=1e-10)


def cases():
    return [("grid2d 64x64, lines of 64", gen.grid2d(64, 64, seed=0), 0, 64),
            ("grid2d 64x64, blocks of 2", gen.grid2d(64, 64, seed=0), 2, 2),
            ("grid2d 64x64, blocks of 48 (not dividing a line)", gen.grid2d(64, 64, seed=0), 48, 48),
            ("seg 24^3, lines of 24", gen.grid3d_seg(24, seed=6), 0, 24),
            ("box 32x32 + partial plane (marching SpMV)", gen.grid3d_box(32, 32, 32 * 32 * 10 + 500, seed=3), 32, 32)]


@pytest.mark.parametrize("case", range(5))
def test_block_jacobi_matches_oracle(P, oracle_mod, case):
    name, g, bs, bs_oracle = cases()[case]
    say(f"block-Jacobi: {name}")
    xo, so, _ = oracle_mod.irls(g, precond=1, block_size=bs_oracle, **OPTS)
    So, vo, _, _ = oracle_mod.sweep(g, xo)
    _, sj, _ = oracle_mod.irls(g, **OPTS)
    with P.MinCut.from_graph(g, precond=1, block_size=bs, **OPTS) as mc:
        assert mc.info()["solver"] == 1 and mc.info()["format"] == 2
        rc, st = mc.solve()
        x = mc.potentials()
        S, v, _ = mc.cut()
    err = max_pot_err(x, xo)
    it_g = [r["cg_iters"] for r in st]
    it_o = [r["cg_iters"] for r in so]
    say(f"  potential error {err:.2e}; CG iterations {sum(it_g)} (oracle {sum(it_o)}, Jacobi {sum(r['cg_iters'] for r in sj)})")
    assert rc == P.OK
    assert err <= 1e-8
    assert v == vo and np.array_equal(S, So)
    assert all(abs(a - b) <= max(3, 0.02 * b) for a, b in zip(it_g, it_o))
    assert all(r["true_rel_res"] <= 1e-9 for r in st)


def test_block_jacobi_option_errors(P):
    g = gen.grid2d(16, 16, seed=1)
    for kw in (dict(precision=1), dict(format=1), dict(solver=2), dict(block_size=3),
               dict(block_size=18), dict(block_size=130)):
        assert P.create_error(g.n, g.eu, g.ev, g.cap, g.s, g.t, precond=1, **kw) == P.ERR_OPTIONS, kw
    h = gen.gnp(16, 0.3, seed=2)                       # no diagonal layout
    assert P.create_error(h.n, h.eu, h.ev, h.cap, h.s, h.t, precond=1) == P.ERR_OPTIONS


def tile_ids(nx, ny, nn, B):
    """Block id of every node of gen.grid3d_box(nx, ny, nn) (s, t last): cubic
    tiles of B rows on a side, x fastest (the oracle's blocks)."""
    ids = np.arange(nn + 2, dtype=np.int64)
    x, y, z = ids % nx, (ids // nx) % ny, ids // (nx * ny)
    return (x // B) + (nx // B) * ((y // B) + (ny // B) * (z // B))


ILU_CASES = [("box 16x12x10, tiles of 4 (a short top tile)", 16, 12, 10, 4),
             ("box 16x12x9, tiles of 2 (a short top tile)", 16, 12, 9, 2),
             ("box 32x32x24, tiles of 4 (the marching SpMV)", 32, 32, 24, 4),
             ("box 32x24x20, tiles of 8 (a short top tile)", 32, 24, 20, 8),
             ("box 48x32x24, tiles of 8 (six tiles a plane)", 48, 32, 24, 8)]


@pytest.mark.parametrize("case", range(len(ILU_CASES)))
def test_ilu0_tiles_match_oracle(P, oracle_mod, case):
    name, nx, ny, nz, B = ILU_CASES[case]
    g = gen.grid3d_box(nx, ny, nx * ny * nz, seed=5 + case)
    blk = tile_ids(nx, ny, nx * ny * nz, B)
    say(f"ILU(0) block-Jacobi: {name}")
    xo, so, _ = oracle_mod.irls(g, precond=2, block_of=blk, **OPTS)
    So, vo, _, _ = oracle_mod.sweep(g, xo)
    _, sj, _ = oracle_mod.irls(g, **OPTS)
    with P.MinCut.from_graph(g, precond=2, block_size=B, **OPTS) as mc:
        assert mc.info()["solver"] == 1 and mc.info()["format"] == 2
        rc, st = mc.solve()
        x = mc.potentials()
        S, v, _ = mc.cut()
    err = max_pot_err(x, xo)
    it_g = [r["cg_iters"] for r in st]
    it_o = [r["cg_iters"] for r in so]
    say(f"  potential error {err:.2e}; CG iterations {sum(it_g)} (oracle {sum(it_o)}, Jacobi "
        f"{sum(r['cg_iters'] for r in sj)})")
    assert rc == P.OK
    assert err <= 1e-8
    assert v == vo and np.array_equal(S, So)
    assert all(abs(a - b) <= max(3, 0.02 * b) for a, b in zip(it_g, it_o))
    assert all(r["true_rel_res"] <= 1e-9 for r in st)


# The precision form with ILU(0) of 4x4x4 tiles: FP32 conductances, pivots,
# residual, direction and SpMV, the substitutions in FP32; FP64 potentials,
# dot products and an FP64 residual replacement (followed by the application)
# every 20 iterations.  Against the oracle's FP64 run with the same tiles.
# Where the tiles along x come in pairs each lane applies two of them; with an
# odd number of tiles a line (the 20-row lines) one.
# Bars: cut within 1e-4 relative (the precision form's bar), the GPU cut's
# value exact for its set, every round's true residual within 2x the
# tolerance, and CG iterations within 10 % + 5 of the FP64 run's, which a
# wrong preconditioner (still symmetric positive definite) would break.
PREC_CASES = [("box 16x12x10 (a short top tile)", lambda: gen.grid3d_box(16, 12, 16 * 12 * 10, seed=5), 16, 12, 20),
              ("box 32x32x24 (the marching SpMV)", lambda: gen.grid3d_box(32, 32, 32 * 32 * 24, seed=7), 32, 32, 20),
              ("box 20x12x9 (five tiles a line: one tile per lane)",
               lambda: gen.grid3d_box(20, 12, 20 * 12 * 9, seed=8), 20, 12, 20),
              ("segmentation grid 48^3", lambda: gen.grid3d_seg(48, seed=3), 48, 48, 40)]


@pytest.mark.parametrize("case", range(len(PREC_CASES)))
def test_ilu0_tiles_precision_form(P, oracle_mod, case):
    name, make, nx, ny, rounds = PREC_CASES[case]
    g = make()
    opts = dict(rounds=rounds, cg_rtol=1e-8)
    say(f"ILU(0) tiles, precision form: {name}")
    with P.MinCut.from_graph(g, precond=2, precision=1, refine_every=20, **opts) as mc:
        info = mc.info()
        assert info["solver"] == 1 and info["format"] == 2
        rc, st = mc.solve()
        x = mc.potentials()
        S, v, _ = mc.cut()
    blk = tile_ids(nx, ny, g.n - 2, 4)
    xo, so, _ = oracle_mod.irls(g, precond=2, block_of=blk, **opts)
    _, vo, _, _ = oracle_mod.sweep(g, xo)
    err = max_pot_err(x, xo)
    rel = abs(v - vo) / vo
    it_g = sum(r["cg_iters"] for r in st)
    it_o = sum(r["cg_iters"] for r in so)
    say(f"  cut rel {rel:.2e}, potential error {err:.2e}, CG {it_g} (oracle FP64 {it_o})")
    assert rc == P.OK
    assert rel <= 1e-4
    assert oracle_mod.cut_value(g, S) == v
    assert all(r["true_rel_res"] <= 2e-8 for r in st[1:])
    assert abs(it_g - it_o) <= 0.1 * it_o + 5


def test_ilu0_tiles_precision_form_driver_paths(P, oracle_mod):
    """The precision form over 4x4x4 ILU(0) tiles through the round driver's
    other paths, where its potentials (moved every second iteration, a
    pending step flushed after CG) must come out whole: a continuation after
    new capacities from the oracle's old potentials against the oracle's FP64
    continuation with the same tiles (cut within 1e-4, value exact for its
    set); the certified-gap stop (the cut at or above the exact minimum cut,
    the last round's gap within the stated fraction); in-solve timing of the
    update (one launch per CG iteration) and of the replacement."""
    from gen import Graph
    g1 = gen.grid3d_box(32, 32, 32 * 32 * 24, seed=7)
    f = 1.0 + 0.2 * (2.0 * np.random.default_rng(17).random(g1.cap.shape[0]) - 1.0)
    g2 = Graph(g1.n, g1.s, g1.t, g1.eu, g1.ev, g1.cap * f, meta=dict(g1.meta))
    blk = tile_ids(32, 32, 32 * 32 * 24, 4)
    opts = dict(rounds=20, cg_rtol=1e-8)
    x_old, _, _ = oracle_mod.irls(g1, precond=2, block_of=blk, **opts)
    xo, so, _ = oracle_mod.irls(g2, init=2, x0=x_old, eps0=1e-3, rounds=12, cg_rtol=1e-8, precond=2, block_of=blk)
    _, vo, _, _ = oracle_mod.sweep(g2, xo)
    prec = dict(precond=2, precision=1, refine_every=20)
    with P.MinCut.from_graph(g1, **prec, **opts) as mc:
        mc.solve()
        mc.update_capacities(g2.eu, g2.ev, g2.cap)
        mc.set_potentials(x_old)
        rc, cs = mc.solve_range(1, 12, eps_first=1e-3)
        x = mc.potentials()
        S, v, _ = mc.cut()
    rel = abs(v - vo) / vo
    say(f"ILU(0) tiles, precision form, continuation: cut rel {rel:.2e}, potential error "
        f"{max_pot_err(x, xo):.2e}, CG {sum(r['cg_iters'] for r in cs[1:])} (oracle FP64 "
        f"{sum(r['cg_iters'] for r in so[1:])})")
    assert rc == P.OK and rel <= 1e-4
    assert oracle_mod.cut_value(g2, S) == v
    assert all(cs[l]["true_rel_res"] <= 2e-8 for l in range(1, 13))
    _, mu = oracle_mod.maxflow(g1)
    with P.MinCut.from_graph(g1, **prec, rounds=40, cg_rtol=1e-8, stop_gap=0.01) as mc:
        rc, st = mc.solve()
        S, v, _ = mc.cut()
        last = st[-1]
    say(f"  stop_gap 0.01: {len(st)} rounds, cut {v!r}, exact minimum {mu!r}")
    assert rc == P.OK and len(st) <= 41
    assert v >= mu * (1 - 1e-12) and oracle_mod.cut_value(g1, S) == v
    if len(st) < 41:                                       # stopped on the gap
        assert last["l1"] - last["lower_bound"] <= 0.01 * last["l1"]
    with P.MinCut.from_graph(g1, **prec, rounds=4, cg_rtol=1e-8) as mc:
        mc.set_kernel_timing(1, 1)
        rc, st = mc.solve()
        assert rc == P.OK and mc.kernel_timing()["n_working"] == sum(r["cg_iters"] for r in st)
        mc.set_kernel_timing(2, 1)
        rc2, st2 = mc.solve()
        assert rc2 == P.OK and [r["cg_iters"] for r in st2] == [r["cg_iters"] for r in st]


def test_ilu0_tile_option_errors(P):
    ok = gen.grid3d_box(16, 12, 16 * 12 * 4, seed=1)
    assert P.create_error(ok.n, ok.eu, ok.ev, ok.cap, ok.s, ok.t, precond=2) == P.OK
    # the precision form takes 4x4x4 tiles (only)
    assert P.create_error(ok.n, ok.eu, ok.ev, ok.cap, ok.s, ok.t, precond=2, precision=1) == P.OK
    # format 1 on the same grid is allowed: CSR blocks instead of tiles
    assert P.create_error(ok.n, ok.eu, ok.ev, ok.cap, ok.s, ok.t, precond=2, format=1, solver=1) == P.OK
    g16 = gen.grid3d_box(16, 16, 16 * 16 * 3, seed=1)
    assert P.create_error(g16.n, g16.eu, g16.ev, g16.cap, g16.s, g16.t, precond=2, block_size=8) == P.OK
    for g, kw in ((ok, dict(block_size=8)),                                  # lines of 12: not a multiple of 8
                  (ok, dict(block_size=6)), (g16, dict(block_size=16)),
                  (ok, dict(precision=1, block_size=2)), (g16, dict(precision=1, block_size=8)),
                  (ok, dict(precision=1, format=1)), (ok, dict(solver=2)),
                  (gen.grid3d_box(18, 12, 18 * 12 * 4, seed=1), {}),        # lines not a multiple of 4
                  (gen.grid3d_box(16, 12, 16 * 12 * 4 + 5, seed=1), {}),    # a partial plane
                  (gen.grid2d(64, 64, seed=0), {})):                       # not a 3-D grid
        assert P.create_error(g.n, g.eu, g.ev, g.cap, g.s, g.t, precond=2, **kw) == P.ERR_OPTIONS, kw


def bfs_blocks(g, B):
    """Block ids of the CSR ILU(0) blocks by their stated rule, written out
    here on its own: the non-terminal nodes in ascending id are the rows; a
    breadth-first ordering of the rows over the interior edges, from the
    smallest unvisited row with neighbours in ascending order; block q is
    positions q*B .. q*B + B - 1 of that ordering."""
    n, s, t = g.n, g.s, g.t
    row = np.full(n, -1, np.int64)
    nts = [u for u in range(n) if u != s and u != t]
    row[nts] = np.arange(len(nts))
    nbrs = [set() for _ in nts]
    for a, b in zip(g.eu.tolist(), g.ev.tolist()):
        if a != b and row[a] >= 0 and row[b] >= 0:
            nbrs[row[a]].add(int(row[b]))
            nbrs[row[b]].add(int(row[a]))
    seen = [False] * len(nts)
    order = []
    for r in range(len(nts)):
        if seen[r]:
            continue
        seen[r] = True
        q = [r]
        head = 0
        while head < len(q):
            u = q[head]
            head += 1
            for v in sorted(nbrs[u]):
                if not seen[v]:
                    seen[v] = True
                    q.append(v)
        order += q
    blk = np.zeros(n, np.int64)
    for pos, r in enumerate(order):
        blk[nts[r]] = pos // B
    return blk


CSR_CASES = [("R-MAT (FlowImprove), blocks of 32", lambda: gen.rmat_flowimprove(2003, log2_lo=9.0, log2_hi=10.0), 32),
             ("G(60, 0.1), blocks of 8", lambda: gen.gnp(60, 0.1, seed=4), 8),
             ("grid2d 40x30 as CSR, blocks of 16", lambda: gen.grid2d(40, 30, seed=2), 16)]


@pytest.mark.parametrize("case", range(len(CSR_CASES)))
def test_ilu0_csr_blocks_match_oracle(P, oracle_mod, case):
    name, make, B = CSR_CASES[case]
    g = make()
    blk = bfs_blocks(g, B)
    say(f"ILU(0) CSR blocks: {name} (n = {g.n})")
    xo, so, _ = oracle_mod.irls(g, precond=2, block_of=blk, **OPTS)
    So, vo, _, _ = oracle_mod.sweep(g, xo)
    _, sj, _ = oracle_mod.irls(g, **OPTS)
    with P.MinCut.from_graph(g, precond=2, block_size=B, format=1, solver=1, **OPTS) as mc:
        assert mc.info()["format"] == 1
        rc, st = mc.solve()
        x = mc.potentials()
        S, v, _ = mc.cut()
    err = max_pot_err(x, xo)
    it_g = [r["cg_iters"] for r in st]
    it_o = [r["cg_iters"] for r in so]
    say(f"  potential error {err:.2e}; CG iterations {sum(it_g)} (oracle {sum(it_o)}, Jacobi "
        f"{sum(r['cg_iters'] for r in sj)})")
    assert rc == P.OK
    assert err <= 1e-8
    assert v == vo and np.array_equal(S, So)
    assert all(abs(a - b) <= max(3, 0.02 * b) for a, b in zip(it_g, it_o))
    assert all(r["true_rel_res"] <= 1e-9 for r in st)


def test_ilu0_csr_option_errors(P):
    g = gen.gnp(40, 0.15, seed=3)
    assert P.create_error(g.n, g.eu, g.ev, g.cap, g.s, g.t, precond=2, solver=1) == P.OK
    for kw in (dict(block_size=3), dict(block_size=130), dict(precision=1), dict(solver=2)):
        assert P.create_error(g.n, g.eu, g.ev, g.cap, g.s, g.t, precond=2, **kw) == P.ERR_OPTIONS, kw


def test_ilu0_fused_update_timing(P):
    """With 4x4x4 tiles the vector update and the ILU(0) application are one
    kernel: in-solve timing of the update (which = 1) sees one launch per CG
    iteration, and the separate application (which = 3) is refused; with
    2x2x2 tiles it is a kernel of its own and can be timed."""
    g = gen.grid3d_box(16, 16, 16 * 16 * 8, seed=2)
    with P.MinCut.from_graph(g, precond=2, rounds=4, cg_rtol=1e-8) as mc:
        with pytest.raises(P.IrlsError):
            mc.set_kernel_timing(3)
        mc.set_kernel_timing(1, 1)
        rc, st = mc.solve()
        t = mc.kernel_timing()
        assert rc == P.OK and t["n_working"] == sum(r["cg_iters"] for r in st)
    with P.MinCut.from_graph(g, precond=2, block_size=2, rounds=4, cg_rtol=1e-8) as mc:
        mc.set_kernel_timing(3, 1)
        rc, st = mc.solve()
        assert rc == P.OK and mc.kernel_timing()["n_working"] == sum(r["cg_iters"] for r in st)
