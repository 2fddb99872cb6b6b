"""The diagonal SpMV that marches along the plane offset, against the CPU
oracle.  Layouts chosen to hit its edge cases: a 2-D grid whose rows (the
planes of two offsets) fill one and a fraction of a tile, and a 3-D box whose
last plane is partial, in FP64 and in the FP32 form, each on the
symmetrically scaled system (the default) and in the z = D^-1 r form."""
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
    # grid2d 1200 x 20: planes (x-rows) of 1200 rows = 600 FP64 / 300 FP32
    #   groups, so the last tile of each plane is partial; 20 planes
    # box 32 x 32, 10 planes + 500 rows: full tiles, a partial last plane
    # box 48 x 24, 7 planes + 36 rows: partial tiles and a partial plane
    return [("grid2d 1200x20", gen.grid2d(1200, 20, seed=2)),
            ("box 32x32, 10 planes + 500", gen.grid3d_box(32, 32, 32 * 32 * 10 + 500, seed=3)),
            ("box 48x24, 7 planes + 36", gen.grid3d_box(48, 24, 48 * 24 * 7 + 36, seed=4))]


FORMS = {"fp64": (dict(precision=0), 4),                       # scaled system (default)
         "fp64-unscaled": (dict(precision=0, unscaled_cg=1), 3),  # z = D^-1 r form
         "fp32": (dict(precision=1), 4),
         "fp32-unscaled": (dict(precision=1, unscaled_cg=1), 3)}


@pytest.mark.parametrize("case", range(3))
@pytest.mark.parametrize("form", list(FORMS))
def test_march_matches_oracle(P, oracle_mod, case, form):
    name, g = cases()[case]
    kw, variant = FORMS[form]
    say(f"march: {name}, {form}")
    xo, so, _ = oracle_mod.irls(g, **OPTS)
    So, vo, _, _ = oracle_mod.sweep(g, xo)
    with P.MinCut.from_graph(g, solver=1, **kw, **OPTS) as mc:
        info = mc.info()
        assert mc.spmv_variant()[0] == variant
        assert mc.spmv_kernel()[0] == "k_spmv_dia_march"
        rc, st = mc.solve()
        x = mc.potentials()
        S, v, _ = mc.cut()
    assert info["format"] == 2 and info["n_diagonals"] == (2 if case == 0 else 3)
    err = max_pot_err(x, xo)
    it_g = [r["cg_iters"] for r in st]
    it_o = [r["cg_iters"] for r in so]
    say(f"  potential error {err:.2e}; cut {v!r} vs {vo!r}; CG iterations {sum(it_g)} (oracle {sum(it_o)})")
    if kw["precision"] == 0:
        assert err <= 1e-8
        assert v == vo and np.array_equal(S, So)
        assert all(abs(a - b) <= 3 for a, b in zip(it_g, it_o))
        assert all(r["true_rel_res"] <= 1e-9 for r in st)
    else:
        assert err <= 1e-4
        assert abs(v - vo) <= 1e-4 * vo


def test_small_planes_use_the_vector_kernel(P):
    """64 x 64: a plane (x-row) of 32 FP64 groups is less than a tile, so the
    row-slab vector kernel runs instead."""
    with P.MinCut.from_graph(gen.grid2d(64, 64, seed=0), solver=1) as mc:
        assert mc.spmv_kernel()[0] == "k_spmv_dia_vec"
    with P.MinCut.from_graph(gen.grid2d(64, 64, seed=0), solver=1, format=1) as mc:
        assert mc.spmv_kernel()[0] == "k_spmv_csr"


@pytest.mark.parametrize("maxit", [1, 2, 3, 4])
@pytest.mark.parametrize("precision", [0, 1])
def test_scaled_form_at_fixed_iteration_counts(P, oracle_mod, maxit, precision):
    """CG stopped after a fixed number of iterations in every round: the
    scaled form moves the potentials every second iteration, so an odd count
    leaves a step pending that must be added after CG (and, in the FP32 form,
    seen by the residual replacement).  The potentials after 1..4 iterations
    per round match the oracle's Jacobi PCG run with the same cap."""
    name, g = cases()[1]
    say(f"scaled form, cg_maxit {maxit}, precision {precision}: {name}")
    kw = dict(rounds=3, cg_rtol=1e-12, cg_maxit=maxit)
    xo, so, rco = oracle_mod.irls(g, allow_maxit=True, **kw)
    extra = dict(refine_every=1) if precision == 1 else {}   # a replacement after every update
    with P.MinCut.from_graph(g, solver=1, precision=precision, **extra, **kw) as mc:
        assert mc.spmv_variant()[0] == 4
        rc, st = mc.solve(allow_maxit=True)
        x = mc.potentials()
        if precision == 0:
            t_odd, t_even = mc.time_kernel(1, 3), mc.time_kernel(2, 3)
            assert t_odd > 0 and t_even > 0
            with pytest.raises(P.IrlsError):
                mc.time_kernel(3, 3)
    assert rc == P.WARN_CG_MAXIT and rco == 100
    assert [r["cg_iters"] for r in st] == [r["cg_iters"] for r in so] == [maxit] * 4
    err = max_pot_err(x, xo)
    say(f"  potential error {err:.2e}")
    assert err <= (1e-10 if precision == 0 else 1e-5)


def tile_shapes(R, N, lines, P):
    """The tile shapes irls_mincut_set_march_tile accepts (its documented rule)."""
    out = []
    for bs in (256, 512):
        for ty in (0, 1, 2, 4, 8, 16, 32, 64):
            if ty == 0:
                ok = P // R >= bs
            else:
                ok = bs % ty == 0 and ty <= lines and bs // ty <= N // R
            if ok:
                out.append((bs, ty))
    return out


@pytest.mark.parametrize("precision", [0, 1])
def test_march_tile_shapes_match_oracle(P, oracle_mod, precision):
    """Every tile shape the marching SpMV accepts (256 or 512 threads; 0 or
    1..64 lines) on a box whose lines (96 rows) and planes (80 lines) leave
    partial tiles in x and in y and whose last plane is partial: the
    potentials and the cut against the oracle's, for each shape in turn on one
    handle.  Shapes outside the rule are refused and leave the shape as it was."""
    nx, ny = 96, 80
    g = gen.grid3d_box(nx, ny, nx * ny * 6 + 1000, seed=6)
    R = 2 if precision == 0 else 4
    want = tile_shapes(R, nx, ny, nx * ny)
    xo, so, _ = oracle_mod.irls(g, **OPTS)
    So, vo, _, _ = oracle_mod.sweep(g, xo)
    seen = []
    with P.MinCut.from_graph(g, solver=1, precision=precision, **OPTS) as mc:
        assert mc.march_tile()[:2] == (256, 0)
        for bs in (256, 512, 128):
            for ty in (0, 1, 2, 3, 4, 8, 16, 32, 64, 128):
                before = mc.march_tile()
                try:
                    mc.set_march_tile(bs, ty)
                except P.IrlsError as e:
                    assert e.code == P.ERR_OPTIONS and mc.march_tile() == before
                    continue
                assert mc.march_tile()[:2] == (bs, ty)
                rc, st = mc.solve()
                x = mc.potentials()
                S, v, _ = mc.cut()
                err = max_pot_err(x, xo)
                say(f"  tile {bs} threads x {ty} lines ({mc.march_tile()[2]} planes per workgroup): "
                    f"potential error {err:.2e}, cut {v!r} vs {vo!r}")
                assert rc == P.OK
                if precision == 0:
                    assert err <= 1e-8
                    assert v == vo and np.array_equal(S, So)
                else:
                    assert err <= 1e-4 and abs(v - vo) <= 1e-4 * vo
                seen.append((bs, ty))
        mc.set_march_tile(0, 0)
        assert mc.march_tile()[:2] == (256, 0)
    assert seen == want


def test_in_solve_kernel_timing(P):
    """irls_mincut_set_kernel_timing: with every launch timed, the launches that
    did work are one per CG iteration of every round; with a stride of 4,
    iterations 0, 4, 8, ... of each round; results are unchanged by it."""
    g = gen.grid3d_box(64, 64, 64 * 64 * 8, seed=7)
    with P.MinCut.from_graph(g, solver=1, **OPTS) as mc:
        _, st0 = mc.solve()
        x0 = mc.potentials()
        for which in (0, 1):
            for every in (1, 4):
                mc.set_kernel_timing(which, every)
                _, st = mc.solve()
                assert np.array_equal(mc.potentials(), x0)
                t = mc.kernel_timing()
                iters = [r["cg_iters"] for r in st]
                assert iters == [r["cg_iters"] for r in st0]
                assert t["n_working"] == sum((i + every - 1) // every for i in iters if i > 0)
                assert t["n_all"] >= t["n_working"] and t["ms_working"] > 0
                assert t["ms_all"] >= t["ms_working"]
                say(f"  kernel {which}, every {every}: {t['n_working']} working launches, "
                    f"mean {1e3 * t['ms_working'] / t['n_working']:.1f} us")
        mc.set_kernel_timing(-1)
        mc.solve()
        assert mc.kernel_timing()["n_all"] == 0
        with pytest.raises(P.IrlsError):
            mc.set_kernel_timing(2)              # the replacement kernel: precision form only
        with pytest.raises(P.IrlsError):
            mc.set_kernel_timing(0, 0)


def test_stream_probe(P):
    """irls_stream_probe: a positive launch time for the SpMV's mix of streams
    and for a copy; arguments outside its range are refused."""
    rows = 1 << 22
    for nr, nw in ((5, 2), (1, 1)):
        ms = P.stream_probe(rows, nr, nw, 256, 5)
        gbs = (nr + nw) * rows * 8 / (ms * 1e-3) / 1e9
        say(f"  {nr} reads + {nw} writes of {rows} doubles: {ms * 1e3:.1f} us, {gbs:.0f} GB/s")
        assert ms > 0 and gbs < 20000
    for bad in ((rows + 1, 5, 2, 256), (rows, 7, 2, 256), (rows, 5, 3, 256), (rows, 5, 2, 100)):
        with pytest.raises(P.IrlsError) as e:
            P.stream_probe(*bad, reps=1)
        assert e.value.code == P.ERR_OPTIONS
