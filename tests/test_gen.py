"""Seeded input generators: sizes, determinism, value ranges."""
import numpy as np

import gen
from gen import rng


def test_rng_is_counter_based():
    a = rng.uniform(7, 3, np.arange(100, dtype=np.uint64))
    b = rng.uniform(7, 3, np.arange(50, 100, dtype=np.uint64))
    assert np.array_equal(a[50:], b)
    assert np.all((a >= 0) & (a < 1))
    assert not np.array_equal(a, rng.uniform(7, 4, np.arange(100, dtype=np.uint64)))
    z = rng.normal(1, 0, 200000)
    assert abs(z.mean()) < 0.01 and abs(z.std() - 1) < 0.01


def test_grid2d_sizes():
    g = gen.grid2d(64, 64, seed=0)
    assert g.n == 4098 and g.meta["interior"] == 8064 and g.m == 8064 + 128
    ci = g.cap[:8064]
    ct = g.cap[8064:]
    assert ci.min() >= 0.1 and ci.max() < 1.0
    assert ct.min() >= 0.5 and ct.max() < 2.0
    g2 = gen.grid2d(64, 64, seed=0)
    assert np.array_equal(g.cap, g2.cap) and np.array_equal(g.eu, g2.eu)
    # s links column 0, t links column 63
    assert set(g.ev[8064:8128] % 64) == {0} and set(g.eu[8128:] % 64) == {63}


def test_gnp_connected_and_deterministic():
    gs = [gen.gnp(16, 0.3, seed=i) for i in range(1, 51)]
    for g in gs:
        assert g.n == 16 and g.s == 0 and g.t == 15
        assert gen.graphs._connected(16, g.eu, g.ev)
    assert np.array_equal(gs[3].cap, gen.gnp(16, 0.3, seed=4).cap)


def test_grid3d_sizes_small():
    g = gen.grid3d_seg(16, seed=3, with_intensity=True)
    N = 16
    assert g.n == N ** 3 + 2
    assert g.meta["interior"] == 3 * N * N * (N - 1)
    assert g.m == 3 * N * N * (N - 1) + 2 * N ** 3
    I = g.meta["I"]
    assert I.min() >= 0 and I.max() <= 1
    ci = g.cap[:g.meta["interior"]]
    assert ci.max() <= 1.0 and ci.min() > 0


def test_grid3d_128_counts():
    N = 128
    assert 3 * N * N * (N - 1) == 6242304


def test_rmat_instance():
    g = gen.rmat_flowimprove(1000)
    mi = g.meta["interior"]
    assert np.all(g.eu[:mi] != g.ev[:mi])
    keys = np.minimum(g.eu[:mi], g.ev[:mi]) * g.n + np.maximum(g.eu[:mi], g.ev[:mi])
    assert np.unique(keys).shape[0] == mi
    c = g.cap[:mi]
    assert c.min() >= 0.5 and c.max() <= 1.0
    assert np.array_equal(c.astype(np.float32).astype(np.float64), c)
    nt = g.n - 2
    # every non-terminal has exactly one terminal edge
    term = np.concatenate([g.ev[g.eu == g.s], g.eu[g.ev == g.t]])
    assert np.array_equal(np.sort(term), np.arange(nt))
    nball = int(np.sum(g.eu == g.s))
    assert nball == int(np.ceil(0.05 * nt))


def test_seg_slab_is_the_first_planes():
    """The slab is the full grid restricted to its first planes: the same
    interior edges and capacities among them, and both terminal edges of
    every kept node with the full grid's capacities."""
    import numpy as np
    full = gen.grid3d_seg(24, seed=2)
    g = gen.grid3d_seg_slab(24, 5, seed=2)
    keep = 24 * 24 * 5
    assert (g.n, g.s, g.t) == (keep + 2, keep, keep + 1)
    m = (full.eu < keep) & (full.ev < keep)
    k = int(m.sum())
    assert g.meta["interior"] == k
    assert np.array_equal(g.eu[:k], full.eu[m]) and np.array_equal(g.ev[:k], full.ev[m])
    assert np.array_equal(g.cap[:k], full.cap[m])
    src = g.eu == g.s
    snk = g.ev == g.t
    assert np.array_equal(np.sort(g.ev[src]), np.arange(keep)) and np.array_equal(np.sort(g.eu[snk]), np.arange(keep))
    fsrc = (full.eu == full.s) & (full.ev < keep)
    assert np.array_equal(g.cap[src], full.cap[fsrc])
