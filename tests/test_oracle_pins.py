"""Pins of the CPU oracle to facts that do not come from the oracle itself.

Each test names the passage of the paper (or the piece of mathematics) it
relies on.  Together they are chosen so that a plausible slip in the oracle
(a dropped term, a wrong sign, a swapped index or operand, a wrong
conductance form) breaks at least one of them.
"""
from fractions import Fraction

import numpy as np
import pytest

import gen
from gen import rng
from gen.graphs import Graph


def mk(n, s, t, edges):
    e = np.asarray(edges, dtype=np.float64).reshape(-1, 3)
    return Graph(n, s, t, e[:, 0].astype(np.int64), e[:, 1].astype(np.int64), e[:, 2].copy())


def path_graph(caps):
    """s - u1 - ... - uk - t with capacities caps[0..k]; ids: u_i = i-1, s = k, t = k+1."""
    k = len(caps) - 1
    s, t = k, k + 1
    chain = [s] + list(range(k)) + [t]
    return mk(k + 2, s, t, [(chain[j], chain[j + 1], caps[j]) for j in range(k + 1)])


def series_potentials(cond):
    """Series conductances g_0..g_k from s (potential 1) to t (0): potentials of the
    k inner nodes.  The current is 1/sum(1/g); each conductor drops current/g."""
    F = 1.0 / sum(1.0 / g for g in cond)
    out, v = [], 1.0
    for g in cond[:-1]:
        v -= F / g
        out.append(v)
    return np.array(out)


def exact_cut(g, in_S):
    """Exact cut value with rational arithmetic (parallel edges summed)."""
    tot = Fraction(0)
    for a, b, c in zip(g.eu.tolist(), g.ev.tolist(), g.cap.tolist()):
        if a != b and bool(in_S[a]) != bool(in_S[b]):
            tot += Fraction(c)
    return tot


# ---------------------------------------------------------------------------
# closed forms
# ---------------------------------------------------------------------------
def test_single_node_round0_and_limit(oracle_mod):
    """One non-terminal u with capacities a (to s) and b (to t).

    Round 0 (Section 2.1, W0 = C): u is a voltage divider, v = a/(a+b).
    Every later round solves a 1x1 system, v' = g_s/(g_s+g_t).  With a
    vanishing smoothing eps the conductances are c/|d| (Step 1 with the
    reweighted Laplacian), so the odds v/(1-v) are multiplied by a/b each
    round, and the sweep picks the cheaper edge: cut = min(a, b)."""
    a, b = 0.7, 0.3
    g = mk(3, 1, 2, [(1, 0, a), (0, 2, b)])
    x, R, _ = oracle_mod.irls(g, rounds=0)
    assert x[0] == pytest.approx(a / (a + b), rel=1e-15)
    odds0 = x[0] / (1 - x[0])
    for T in range(1, 6):
        xT, _, _ = oracle_mod.irls(g, rounds=T, eps0=1e-30, eps_factor=1.0)
        odds = xT[0] / (1 - xT[0])
        assert odds == pytest.approx(odds0 * (a / b) ** T, rel=1e-12)
    inS, val, k, _ = oracle_mod.sweep(g, xT)
    assert val == b and inS[0]          # the t-edge (b < a) is cut: u stays with s


def test_single_node_paper_form_scale(oracle_mod):
    """Paper form (eq. define-reweight-vector + eq. reweighted-laplacian):
    conductance c^2/sqrt((c d)^2 + eps).  Scaling every capacity by k leaves
    the potentials unchanged when eps is scaled by k^2: the conductances all
    scale by k.  The other form c/sqrt(d^2+eps) has the same invariance with
    eps fixed.  A wrong power of c in either form breaks one of these."""
    base = [(1, 0, 0.9), (0, 2, 0.4), (0, 3, 0.5), (3, 2, 1.3), (1, 3, 0.2)]
    k = 3.0
    g1 = mk(4, 1, 2, base)
    g2 = mk(4, 1, 2, [(u, v, c * k) for u, v, c in base])
    xa, _, _ = oracle_mod.irls(g1, rounds=4, weight_form=1, eps0=1e-2, eps_factor=0.5)
    xb, _, _ = oracle_mod.irls(g2, rounds=4, weight_form=1, eps0=1e-2 * k * k, eps_factor=0.5)
    np.testing.assert_allclose(xa, xb, rtol=1e-11, atol=1e-13)
    ya, _, _ = oracle_mod.irls(g1, rounds=4, weight_form=0, eps0=1e-2, eps_factor=0.5)
    yb, _, _ = oracle_mod.irls(g2, rounds=4, weight_form=0, eps0=1e-2, eps_factor=0.5)
    np.testing.assert_allclose(ya, yb, rtol=1e-11, atol=1e-13)
    # and the two forms really differ once capacities differ from 1
    assert np.max(np.abs(xa - ya)) > 1e-4


def test_path_every_round_matches_series_circuit(oracle_mod):
    """Path s-u1-...-uk-t: each round is a series circuit (Proposition 3, the
    WLS is an electrical flow), solved in closed form from the conductances.
    Round 0 conductances are the capacities; later ones c/sqrt(d^2+eps_l)
    with d taken from the oracle's previous round.  The min cut of a path is
    its smallest capacity."""
    caps = [0.9, 0.35, 0.8, 0.6, 0.25, 1.1, 0.7]
    g = path_graph(caps)
    k = len(caps) - 1
    x0, _, _ = oracle_mod.irls(g, rounds=0, cg_rtol=1e-14)
    np.testing.assert_allclose(x0[:k], series_potentials(caps), rtol=1e-12, atol=1e-14)
    prev = x0
    eps = 0.1
    for T in range(1, 12):
        xT, _, _ = oracle_mod.irls(g, rounds=T, cg_rtol=1e-14)
        pot = [1.0] + list(prev[:k]) + [0.0]
        cond = [c / np.sqrt((pot[j] - pot[j + 1]) ** 2 + eps) for j, c in enumerate(caps)]
        np.testing.assert_allclose(xT[:k], series_potentials(cond), rtol=1e-9, atol=1e-12)
        prev = xT
        eps *= 0.5
    _, val, _, _ = oracle_mod.sweep(g, prev)
    assert val == min(caps)


def by_hand_bound(F, caps):
    """A series circuit carries one flow F on every edge: rho = F / min(c),
    the overload is sum(max(0, F - c_j))."""
    return max(min(F, min(caps)), F - sum(max(0.0, F - c) for c in caps))


def test_path_lower_bound_by_hand(oracle_mod):
    """The per-round lower bound on a path, by hand: a series circuit carries
    one flow F = 1 / sum(1/g_j) on every edge, so the scaled bound
    F / max(1, rho) is min(F, min c) and the overload bound is
    F - sum(max(0, F - c_j)); the record holds the larger (the path's minimum
    cut is min c).  Round 0 (g = c) gives F < min c: the bound is the flow."""
    caps = [0.9, 0.35, 0.8, 0.6, 0.25, 1.1, 0.7]
    g = path_graph(caps)
    k = len(caps) - 1
    x, R, _ = oracle_mod.irls(g, rounds=0, cg_rtol=1e-14)
    F0 = 1.0 / sum(1.0 / c for c in caps)
    assert F0 < min(caps)
    assert R[0]["lower_bound"] == pytest.approx(F0, rel=1e-12)         # the residual is ~1e-16
    prev = x
    eps = 0.1
    for T in range(1, 12):
        xT, R, _ = oracle_mod.irls(g, rounds=T, cg_rtol=1e-14)
        pot = [1.0] + list(prev[:k]) + [0.0]
        cond = [c / np.sqrt((pot[j] - pot[j + 1]) ** 2 + eps) for j, c in enumerate(caps)]
        F = 1.0 / sum(1.0 / w for w in cond)
        assert R[T]["lower_bound"] == pytest.approx(by_hand_bound(F, caps), rel=1e-9), T
        assert R[T]["lower_bound"] <= min(caps) * (1 + 1e-12)
        prev = xT
        eps *= 0.5


def test_record_l1_and_s_eps_by_hand(oracle_mod):
    """||CBx||_1 and the smoothed objective S_eps of every round record, by
    hand (eq. l1-min and the smoothed objective of Section 2.1): on a path
    the potentials of every round follow from the series circuit alone, so
    both sums are written out from closed-form potentials, never from the
    oracle's.  S_eps of round l is taken at the next round's eps (eps0 for
    round 0).  Both conductance forms, and a triangle with an s-t edge (it
    is cut by every s-t cut, so it adds c to ||CBx||_1 and c*sqrt(1+eps) to
    S_eps)."""
    caps = [0.9, 0.35, 0.8, 0.6, 0.25, 1.1, 0.7]
    g = path_graph(caps)
    k = len(caps) - 1
    for form in (0, 1):
        def cond(c, d, eps):
            return c / np.sqrt(d * d + eps) if form == 0 else c * c / np.sqrt((c * d) ** 2 + eps)

        def smooth(c, d, eps):
            return c * np.sqrt(d * d + eps) if form == 0 else np.sqrt((c * d) ** 2 + eps)

        pot = [1.0] + list(series_potentials(caps)) + [0.0]        # round 0: W = C
        eps = 0.1
        for T in range(0, 10):
            _, R, _ = oracle_mod.irls(g, rounds=T, cg_rtol=1e-14, weight_form=form)
            d = [pot[j] - pot[j + 1] for j in range(k + 1)]
            eps_next = 0.1 if T == 0 else eps * 0.5
            l1 = sum(c * abs(dj) for c, dj in zip(caps, d))
            se = sum(smooth(c, dj, eps_next) for c, dj in zip(caps, d))
            assert R[T]["l1"] == pytest.approx(l1, rel=1e-10), (form, T)
            assert R[T]["s_eps"] == pytest.approx(se, rel=1e-10), (form, T)
            eps = eps_next if T > 0 else 0.1
            pot = [1.0] + list(series_potentials([cond(c, dj, eps) for c, dj in zip(caps, d)])) + [0.0]
    # one non-terminal u between s and t, plus the s-t edge itself
    a, b, c = 0.7, 0.3, 0.45
    g = mk(3, 1, 2, [(1, 0, a), (0, 2, b), (1, 2, c)])
    v, eps = a / (a + b), 0.1
    for T in range(0, 8):
        _, R, _ = oracle_mod.irls(g, rounds=T, cg_rtol=1e-14)
        eps_next = 0.1 if T == 0 else eps * 0.5
        assert R[T]["l1"] == pytest.approx(a * (1 - v) + b * v + c, rel=1e-12), T
        assert R[T]["s_eps"] == pytest.approx(a * np.sqrt((1 - v) ** 2 + eps_next) + b * np.sqrt(v * v + eps_next)
                                              + c * np.sqrt(1 + eps_next), rel=1e-12), T
        eps = eps_next if T > 0 else 0.1
        gs, gt = a / np.sqrt((1 - v) ** 2 + eps), b / np.sqrt(v * v + eps)
        v = gs / (gs + gt)


def test_lower_bound_below_min_cut(oracle_mod):
    """Every round's lower bound lies below the exact minimum cut, round 0's
    is its flow value E0 less the residual (there |x_u - x_v| <= 1, so
    rho <= 1), ||CBx||_1 lies above the minimum cut, and the bound closes in
    on it."""
    for seed in range(1, 51):
        g = gen.gnp(16, 0.3, seed=seed)
        _, R, _ = oracle_mod.irls(g, rounds=20, cg_rtol=1e-12)
        _, mu, _ = oracle_mod.bruteforce(g)
        assert R[0]["lower_bound"] == pytest.approx(R[0]["flow"], rel=1e-9)
        for r in R:
            assert r["lower_bound"] <= mu * (1 + 1e-12)
            assert mu <= r["l1"] * (1 + 1e-12)
        assert R[-1]["lower_bound"] >= 0.99 * mu
    # where the potentials polarise (the segmentation grid) few edges carry
    # more than their capacity and the overload bound is tight
    for g, tight in ((gen.grid2d(40, 30, seed=5), 0.95), (gen.grid3d_seg(12, seed=2), 0.999)):
        _, R, _ = oracle_mod.irls(g, rounds=30, cg_rtol=1e-10)
        _, mu = oracle_mod.maxflow(g)
        assert all(r["lower_bound"] <= mu * (1 + 1e-12) for r in R)
        assert R[-1]["lower_bound"] >= tight * mu


def test_uniform_grid_reduces_to_path(oracle_mod):
    """Uniform interior capacity 1 on an nx-by-ny grid with equal terminal
    capacity q on the left and right columns: by symmetry the round-0
    potentials depend on the column only, giving a path whose column-to-column
    conductance is ny and whose terminal conductances are ny*q."""
    nx, ny, q = 12, 5, 0.8
    g = gen.grid2d(nx, ny, seed=0)
    g.cap[:] = 1.0
    g.cap[g.meta["interior"]:] = q
    x, _, _ = oracle_mod.irls(g, rounds=0, cg_rtol=1e-14)
    cols = [ny * q] + [float(ny)] * (nx - 1) + [ny * q]
    want = series_potentials(cols)
    got = x[:nx * ny].reshape(ny, nx)
    for r in range(ny):
        np.testing.assert_allclose(got[r], want, rtol=1e-11, atol=1e-13)


# ---------------------------------------------------------------------------
# solver against a direct solve
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("which", ["grid", "gnp"])
def test_pcg_matches_dense_solve(oracle_mod, which):
    """Section 3.1: L~ v = b is symmetric positive definite; PCG must reach
    the direct solution.  Also: L~ is symmetric, has a positive diagonal,
    non-positive off-diagonals, and L~ e >= b (proof of Proposition 2)."""
    g = gen.grid2d(20, 20, seed=5) if which == "grid" else gen.gnp(16, 0.3, seed=9)
    nt = g.n - 2
    for T in (0, 3):
        x, _, _ = oracle_mod.irls(g, rounds=T, cg_rtol=1e-14)
        xprev = None
        if T > 0:
            xprev, _, _ = oracle_mod.irls(g, rounds=T - 1, cg_rtol=1e-14)
        eps = 0.0 if T == 0 else 0.1 * 0.5 ** (T - 1)
        rp, col, val, b = oracle_mod.reduced_system(g, xprev, eps)
        A = np.zeros((nt, nt))
        for i in range(nt):
            A[i, col[rp[i]:rp[i + 1]]] = val[rp[i]:rp[i + 1]]
        assert np.array_equal(A, A.T)
        assert np.all(np.diag(A) > 0)
        off = A - np.diag(np.diag(A))
        assert np.all(off <= 0)
        assert np.all(A.sum(axis=1) >= b - 1e-12 * np.diag(A))
        ids = [u for u in range(g.n) if u not in (g.s, g.t)]
        v = np.linalg.solve(A, b)
        np.testing.assert_allclose(x[ids], v, rtol=1e-9, atol=1e-11)


# ---------------------------------------------------------------------------
# invariants from the paper
# ---------------------------------------------------------------------------
def test_prop2_prop3_descent_on_grid(oracle_mod):
    """Proposition 2: 0 <= v <= 1.  Proposition 3: the WLS solution is an
    electrical flow whose value x^T L x equals the flow leaving s and the flow
    entering t.  Section 2.2 (majorisation-minimisation of S_eps, Beck's
    theorems): S at this round's x with the next round's eps never increases,
    because eps decreases and each round minimises a majoriser."""
    g = gen.grid2d(32, 32, seed=3)
    _, R, _ = oracle_mod.irls(g, rounds=25, cg_rtol=1e-12)
    tol = 1e-8
    prev = np.inf
    for r in R:
        assert r["vmin"] >= -tol and r["vmax"] <= 1 + tol
        assert r["flow_s"] == pytest.approx(r["flow"], rel=1e-7)
        assert r["flow_t"] == pytest.approx(r["flow"], rel=1e-7)
        assert r["s_eps"] <= prev * (1 + 1e-10)
        prev = r["s_eps"]


def test_cheeger_bounds_round0(oracle_mod):
    """Section 2.3 and the appendix: with C = 2 sum c and E0 the round-0 flow
    value, lambda_2 = 2 E0 / C and phi = mu*/C, so phi^2/2 <= lambda_2 <= 2 phi
    reads mu*^2/(4C) <= E0 <= mu*."""
    for seed in range(1, 21):
        g = gen.gnp(16, 0.3, seed=seed)
        _, R, _ = oracle_mod.irls(g, rounds=0, cg_rtol=1e-14)
        _, mu, _ = oracle_mod.bruteforce(g)
        Ctot = 2 * g.cap.sum()
        E0 = R[0]["flow"]
        assert mu * mu / (4 * Ctot) <= E0 * (1 + 1e-12)
        assert E0 <= mu * (1 + 1e-12)


def test_chain_invariant_random_potentials(oracle_mod):
    """eq. l1-min: for any x in [0,1] with x_s=1, x_t=0 the threshold (coarea)
    argument gives mu* <= sweep(x) <= ||CBx||_1 <= S_eps(x)."""
    for seed in range(1, 11):
        g = gen.gnp(16, 0.3, seed=seed)
        _, mu, _ = oracle_mod.bruteforce(g)
        x = rng.uniform(seed, 99, np.arange(g.n, dtype=np.uint64))
        x[g.s], x[g.t] = 1.0, 0.0
        _, sw, _, _ = oracle_mod.sweep(g, x)
        l1 = sum(c * abs(x[a] - x[b]) for a, b, c in zip(g.eu, g.ev, g.cap))
        seps = sum(c * np.sqrt((x[a] - x[b]) ** 2 + 1e-3) for a, b, c in zip(g.eu, g.ev, g.cap))
        assert mu <= sw * (1 + 1e-15)
        assert sw <= l1 * (1 + 1e-12)
        assert l1 <= seps


# ---------------------------------------------------------------------------
# the sweep and exact cut values
# ---------------------------------------------------------------------------
def _sweep_by_definition(g, x):
    nt_ids = [u for u in range(g.n) if u not in (g.s, g.t)]
    order = sorted(nt_ids, key=lambda u: (-x[u], u))
    best, bk = None, None
    inS = np.zeros(g.n, bool)
    inS[g.s] = True
    for k in range(len(order) + 1):
        if k > 0:
            inS[order[k - 1]] = True
        v = exact_cut(g, inS)
        if best is None or v < best:
            best, bk = v, k
    return best, bk


@pytest.mark.parametrize("seed", [1, 2, 3, 4, 5])
def test_sweep_equals_prefix_definition(oracle_mod, seed):
    """The sweep recomputed from scratch for every prefix set with exact
    rational sums must pick the same k and value (ties included: potentials
    are rounded to a few levels so many nodes tie)."""
    g = gen.gnp(16, 0.3, seed=seed)
    x = np.round(rng.uniform(seed, 5, np.arange(g.n, dtype=np.uint64)) * 4) / 4
    _, val, k, _ = oracle_mod.sweep(g, x)
    best, bk = _sweep_by_definition(g, x)
    assert k == bk
    assert val == float(best)


def test_cut_value_exact_with_parallel_edges(oracle_mod):
    """Parallel edges add up, self loops never count (problem statement)."""
    g = mk(5, 0, 4, [(0, 1, 0.1), (1, 0, 0.2), (1, 2, 0.3), (2, 2, 9.0), (2, 3, 1e-3),
                     (3, 4, 0.7), (1, 4, 0.05), (0, 3, 0.4), (2, 4, 0.6)])
    for mask in range(8):
        inS = np.array([1, mask & 1, (mask >> 1) & 1, (mask >> 2) & 1, 0], dtype=bool)
        assert oracle_mod.cut_value(g, inS) == float(exact_cut(g, inS))


def test_fixed_point_extreme_scales(oracle_mod):
    """Capacities 16 decimal orders apart are summed exactly: 1 + 1e-16 + 1e-16
    is 1 in left-to-right double arithmetic but 1 + 2^-52 when rounded once
    from the exact sum (the 128-bit scale keeps every capacity exact)."""
    caps = [1.0, 1e-16, 2.5, 1e-16, 0.3, 3.0]
    g = path_graph(caps)
    x = np.array([0.9, 0.8, 0.7, 0.6, 0.5, 1.0, 0.0])
    inS, val, k, _ = oracle_mod.sweep(g, x)
    assert val == 1e-16 and k == 1     # S_1 = {s, u0}; the tie at k = 3 loses to the smaller k
    inS2 = np.zeros(g.n, bool)
    inS2[[g.s, 1, 2]] = True          # cuts s-u0 (1), u0-u1 (1e-16) and u2-u3 (1e-16)
    exact = float(exact_cut(g, inS2))
    assert exact == 1.0 + 2.0 ** -52 and (1.0 + 1e-16) + 1e-16 == 1.0
    assert oracle_mod.cut_value(g, inS2) == exact


# ---------------------------------------------------------------------------
# exact solvers
# ---------------------------------------------------------------------------
def test_bruteforce_hand_graphs(oracle_mod):
    # two disjoint s-t paths: min cut = sum of each path's bottleneck
    g = mk(6, 0, 5, [(0, 1, 3.0), (1, 5, 1.0), (0, 2, 0.5), (2, 3, 2.0), (3, 4, 4.0), (4, 5, 1.5)])
    _, v, sec = oracle_mod.bruteforce(g)
    assert v == 1.5
    # path 1 (caps 3, 1) and path 2 (caps 0.5, 2, 4, 1.5): the best cut takes the
    # bottleneck of each, 1 + 0.5; the next distinct value is 1 + 1.5
    assert sec == 2.5


def test_maxflow_equals_bruteforce(oracle_mod):
    """FIFO push-relabel (Section 4 names the family) against enumeration of
    all 2^14 source sides on the 50 G(16,0.3) graphs."""
    for seed in range(1, 51):
        g = gen.gnp(16, 0.3, seed=seed)
        S1, v1 = oracle_mod.maxflow(g)
        S2, v2, sec = oracle_mod.bruteforce(g)
        assert v1 == v2
        assert oracle_mod.cut_value(g, S1) == v1
        if sec > v2:
            assert np.array_equal(S1, S2)


def test_maxflow_random_small_graphs(oracle_mod):
    for seed in range(100, 130):
        n = 6 + seed % 14
        g = gen.gnp(n, 0.35, seed=seed)
        _, v1 = oracle_mod.maxflow(g)
        _, v2, _ = oracle_mod.bruteforce(g)
        assert v1 == v2


# ---------------------------------------------------------------------------
# quality and determinism of the whole oracle
# ---------------------------------------------------------------------------
def test_irls_sweep_bounded_by_exact(oracle_mod):
    """IRLS with sweep rounding is an approximation (Section 1, delta-accurate):
    its cut can never be below mu*.  On these well-separated small graphs it
    finds the exact minimum in the large majority of cases."""
    exact = 0
    for seed in range(1, 51):
        g = gen.gnp(16, 0.3, seed=seed)
        x, _, _ = oracle_mod.irls(g, rounds=30, cg_rtol=1e-12)
        _, val, _, _ = oracle_mod.sweep(g, x)
        _, mu, _ = oracle_mod.bruteforce(g)
        assert val >= mu
        exact += val == mu
    assert exact >= 45


def test_grid64_exact(oracle_mod):
    g = gen.grid2d(64, 64, seed=0)
    x, R, rc = oracle_mod.irls(g, rounds=30, cg_rtol=1e-10)
    assert rc == 0
    _, val, _, _ = oracle_mod.sweep(g, x)
    _, mu = oracle_mod.maxflow(g)
    assert val == mu


def test_thread_count_does_not_change_bits(oracle_mod):
    g = gen.grid2d(40, 30, seed=2)
    x1, R1, _ = oracle_mod.irls(g, rounds=8, threads=1)
    x4, R4, _ = oracle_mod.irls(g, rounds=8, threads=4)
    assert np.array_equal(x1, x4)
    assert [r["cg_iters"] for r in R1] == [r["cg_iters"] for r in R4]


def test_parallel_edges_and_self_loops_merge(oracle_mod):
    g = gen.gnp(12, 0.4, seed=3)
    # split every edge into two halves, reverse one, add self loops
    half = g.cap / 2
    g2 = Graph(g.n, g.s, g.t, np.concatenate([g.eu, g.ev, np.arange(g.n)]),
               np.concatenate([g.ev, g.eu, np.arange(g.n)]),
               np.concatenate([half, g.cap - half, np.ones(g.n)]))
    x1, _, _ = oracle_mod.irls(g, rounds=5)
    x2, _, _ = oracle_mod.irls(g2, rounds=5)
    np.testing.assert_allclose(x1, x2, rtol=1e-12, atol=1e-14)
    assert oracle_mod.sweep(g, x1)[1] == oracle_mod.sweep(g2, x1)[1]


def test_error_codes(oracle_mod):
    o = oracle_mod
    g = gen.gnp(8, 0.5, seed=1)
    assert o.error_code(o.irls, Graph(g.n, 0, 0, g.eu, g.ev, g.cap)) == 2
    assert o.error_code(o.irls, Graph(g.n, 0, 99, g.eu, g.ev, g.cap)) == 2
    bad = g.cap.copy()
    bad[0] = -1
    assert o.error_code(o.irls, Graph(g.n, g.s, g.t, g.eu, g.ev, bad)) == 3
    bad[0] = np.nan
    assert o.error_code(o.irls, Graph(g.n, g.s, g.t, g.eu, g.ev, bad)) == 3
    dis = mk(5, 0, 4, [(0, 1, 1.0), (1, 4, 1.0), (2, 3, 1.0)])
    assert o.error_code(o.irls, dis) == 4
    assert o.error_code(o.irls, g, rounds=-1) == 5
    assert o.error_code(o.irls, g, cg_rtol=0.0) == 5
    assert o.error_code(o.irls, g, weight_form=3) == 5


def test_degenerate_graphs(oracle_mod):
    # only s and t: the cut is the s-t edge
    g = mk(2, 0, 1, [(0, 1, 0.75), (1, 0, 0.25)])
    x, R, _ = oracle_mod.irls(g, rounds=3)
    inS, val, k, _ = oracle_mod.sweep(g, x)
    assert val == 1.0 and k == 0 and list(inS) == [True, False]
    # a node hanging off t only: its potential is 0, it never joins S
    g = mk(4, 0, 1, [(0, 2, 1.0), (2, 1, 2.0), (3, 1, 0.5), (0, 1, 0.1)])
    x, _, _ = oracle_mod.irls(g, rounds=5)
    assert x[3] == 0.0
    inS, val, _, _ = oracle_mod.sweep(g, x)
    assert val == pytest.approx(1.1) and not inS[3]


# ---------------------------------------------------------------------------
# block-Jacobi preconditioner (Section 3.1: blocks of the reduced Laplacian)
# ---------------------------------------------------------------------------
def test_block_jacobi_single_block_is_the_exact_solve(oracle_mod):
    """One block covering every row makes M = L~: PCG then ends after one
    iteration of every round, and the rounds still match the series circuit
    (same check as the Jacobi run above)."""
    caps = [0.9, 0.35, 0.8, 0.6, 0.25, 1.1, 0.7]
    g = path_graph(caps)
    k = len(caps) - 1
    x, st, _ = oracle_mod.irls(g, rounds=6, cg_rtol=1e-14, precond=1, block_size=k)
    assert all(r["cg_iters"] <= 1 for r in st)
    xj, _, _ = oracle_mod.irls(g, rounds=6, cg_rtol=1e-14)
    np.testing.assert_allclose(x, xj, rtol=0, atol=1e-12)
    g2 = gen.gnp(16, 0.3, seed=7)
    _, st2, _ = oracle_mod.irls(g2, rounds=5, cg_rtol=1e-12, precond=1, block_size=14)
    assert all(r["cg_iters"] <= 1 for r in st2)


def test_block_jacobi_size_one_is_jacobi(oracle_mod):
    """Blocks of one row are the diagonal: same iteration counts, potentials
    equal up to the rounding of sqrt(D)^2 against D."""
    g = gen.grid2d(20, 16, seed=2)
    xj, sj, _ = oracle_mod.irls(g, rounds=12, cg_rtol=1e-10)
    xb, sb, _ = oracle_mod.irls(g, rounds=12, cg_rtol=1e-10, precond=1, block_size=1)
    assert [r["cg_iters"] for r in sj] == [r["cg_iters"] for r in sb]
    np.testing.assert_allclose(xb, xj, rtol=0, atol=1e-11)


def test_block_jacobi_same_solution_fewer_iterations(oracle_mod):
    """Line blocks of a grid: the rounds converge to the same potentials (the
    preconditioner changes the path, not the system) in fewer CG iterations;
    block sizes that do not divide the row count leave a short last block."""
    g = gen.grid3d_seg(10, seed=4)
    xj, sj, _ = oracle_mod.irls(g, rounds=15, cg_rtol=1e-12)
    for bs in (10, 7, 100):
        xb, sb, _ = oracle_mod.irls(g, rounds=15, cg_rtol=1e-12, precond=1, block_size=bs)
        np.testing.assert_allclose(xb, xj, rtol=0, atol=1e-8)
        assert sum(r["cg_iters"] for r in sb) < sum(r["cg_iters"] for r in sj)
    assert oracle_mod.error_code(oracle_mod.irls, g, rounds=1, precond=1, block_size=0) != 0
    assert oracle_mod.error_code(oracle_mod.irls, g, rounds=1, precond=3) != 0


def tile_blocks(nx, ny, nn, tx, ty, tz):
    """Block id of every node of gen.grid3d_box(nx, ny, nn) (s and t last):
    tiles of tx * ty * tz nodes in x, y and z."""
    ids = np.arange(nn + 2, dtype=np.int64)
    x, y, z = ids % nx, (ids // nx) % ny, ids // (nx * ny)
    bx, by = (nx + tx - 1) // tx, (ny + ty - 1) // ty
    return (x // tx) + bx * ((y // ty) + by * (z // tz))


def test_block_solvers_by_definition(oracle_mod):
    """Section 3.1, eq. block-jacobi-subsystem, with the paper's two block
    solvers, checked against their definitions on a reweighted round of a
    6x6x4 grid cut into 3x3x2 tiles: applying M^-1 to every unit vector
    gives M, which is block diagonal over the tiles; the exact solve has
    M = L~ on every block; ILU(0) has M = L~ exactly on the block's pattern
    (the defining property (LU)_ij = A_ij there) and fill elsewhere in the
    block, so the two strategies really differ."""
    nx, ny, nn = 6, 6, 6 * 6 * 4
    g = gen.grid3d_box(nx, ny, nn, seed=3)
    blk = tile_blocks(nx, ny, nn, 3, 3, 2)
    xs = np.concatenate([rng.uniform(3, 5, np.arange(nn, dtype=np.uint64)), [1.0, 0.0]])
    eps = 1e-2
    rp, col, val, _ = oracle_mod.reduced_system(g, xs, eps)
    nt = g.n - 2
    A = np.zeros((nt, nt))
    pat = np.zeros((nt, nt), bool)
    for i in range(nt):
        A[i, col[rp[i]:rp[i + 1]]] = val[rp[i]:rp[i + 1]]
        pat[i, col[rp[i]:rp[i + 1]]] = True
    same = blk[:nt, None] == blk[None, :nt]
    scale = np.max(np.abs(A))
    for kind in (1, 2):
        Minv = np.stack([oracle_mod.block_apply(g, np.eye(nt)[j], kind, block_of=blk, x=xs, eps=eps)
                         for j in range(nt)], axis=1)
        M = np.linalg.inv(Minv)
        assert np.max(np.abs(M[~same])) <= 1e-10 * scale            # block diagonal
        if kind == 1:
            assert np.max(np.abs(M - A)[same]) <= 1e-10 * scale
        else:
            on = same & pat
            assert np.max(np.abs(M - A)[on]) <= 1e-10 * scale
            fill = same & ~pat
            assert np.max(np.abs(M[fill])) >= 1e-4 * scale           # not the exact block
    # a tridiagonal block (one x-line of a grid) has no fill: ILU(0) is exact
    r = rng.uniform(9, 1, np.arange(nt, dtype=np.uint64))
    z1 = oracle_mod.block_apply(g, r, 1, block_size=nx, x=xs, eps=eps)
    z2 = oracle_mod.block_apply(g, r, 2, block_size=nx, x=xs, eps=eps)
    np.testing.assert_allclose(z2, z1, rtol=1e-12, atol=1e-14 * np.max(np.abs(z1)))
    with pytest.raises(oracle_mod.OracleError):
        oracle_mod.block_apply(g, r, 3, block_size=nx)


def test_tile_blocks_same_solution_fewer_iterations(oracle_mod):
    """Tile blocks (rows not consecutive in the numbering) for both block
    solvers: every round converges to the potentials of Jacobi-PCG (the
    preconditioner changes the path, not the system) in fewer CG iterations;
    the exact blocks take no more iterations than their ILU(0)."""
    nx, ny, nn = 12, 12, 12 * 12 * 8
    g = gen.grid3d_box(nx, ny, nn, seed=4)
    blk = tile_blocks(nx, ny, nn, 4, 4, 4)
    xj, sj, _ = oracle_mod.irls(g, rounds=12, cg_rtol=1e-12)
    its = {}
    for kind in (1, 2):
        xb, sb, _ = oracle_mod.irls(g, rounds=12, cg_rtol=1e-12, precond=kind, block_of=blk)
        np.testing.assert_allclose(xb, xj, rtol=0, atol=1e-8)
        its[kind] = sum(r["cg_iters"] for r in sb)
    jac = sum(r["cg_iters"] for r in sj)
    assert its[1] <= its[2] < jac
    bad = blk.copy()
    bad[5] = -1
    assert oracle_mod.error_code(oracle_mod.irls, g, rounds=1, precond=2, block_of=bad) != 0
