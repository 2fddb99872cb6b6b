"""Seeded synthetic s-t min-cut instances.

The paper evaluates on road networks (FlowImprove instances) and on 3-D
segmentation volumes (Section 5, Table 1).  Those files are not available,
so these generators produce inputs of the same kinds and sizes:

* ``grid2d``     -- a 4-connected 2-D grid, source on the left column, sink
                    on the right column (small parity case).
* ``gnp``        -- small G(n, p) graphs for exhaustive checking.
* ``grid3d_seg`` -- a 6-connected 3-D grid whose capacities come from a
                    smooth Gaussian random field, as in graph-cut image
                    segmentation (stand-in for the paper's MRI volumes).
* ``rmat_flowimprove`` -- an R-MAT power-law graph with a FlowImprove-like
                    terminal attachment (stand-in for the road networks).

Node ids: non-terminal nodes first (x fastest for grids), then s, then t.
Edge order: interior edges first (per node in id order, +x, +y, +z), then
source edges, then sink edges.  Every graph is returned as plain arrays;
nothing here computes any part of the min-cut method.
"""
import os
from dataclasses import dataclass, field

import numpy as np

from . import rng


@dataclass
class Graph:
    n: int                 # number of nodes including s and t
    s: int
    t: int
    eu: np.ndarray         # int64 [m]
    ev: np.ndarray         # int64 [m]
    cap: np.ndarray        # float64 [m], all > 0
    meta: dict = field(default_factory=dict)

    @property
    def m(self):
        return int(self.eu.shape[0])


# ----------------------------------------------------------------------------
# small 2-D grid (4096 nodes at 64 x 64)
# ----------------------------------------------------------------------------
def grid2d(nx=64, ny=64, seed=0, cap_lo=0.1, cap_hi=1.0, term_lo=0.5, term_hi=2.0):
    """4-connected nx*ny grid; s links column x=0, t links column x=nx-1.

    Streams: 0 interior capacities (by interior edge index), 1 source
    capacities (by row y), 2 sink capacities (by row y).
    """
    nn = nx * ny
    ids = np.arange(nn, dtype=np.int64)
    x = ids % nx
    y = ids // nx
    has = np.stack([x < nx - 1, y < ny - 1], axis=1)
    nbr = np.stack([ids + 1, ids + nx], axis=1)
    src = np.broadcast_to(ids[:, None], has.shape)[has]
    dst = nbr[has]
    mi = src.shape[0]
    c_int = rng.uniform_range(seed, 0, mi, cap_lo, cap_hi)
    s, t = nn, nn + 1
    left = np.arange(ny, dtype=np.int64) * nx
    right = left + (nx - 1)
    c_s = rng.uniform_range(seed, 1, ny, term_lo, term_hi)
    c_t = rng.uniform_range(seed, 2, ny, term_lo, term_hi)
    eu = np.concatenate([src, np.full(ny, s, np.int64), right])
    ev = np.concatenate([dst, left, np.full(ny, t, np.int64)])
    cap = np.concatenate([c_int, c_s, c_t])
    return Graph(nn + 2, s, t, eu, ev, cap,
                 meta=dict(kind="grid2d", shape=(nx, ny), seed=seed, interior=mi))


def grid3d_box(nx, ny, nn, seed=0, cap_lo=0.1, cap_hi=1.0, term_lo=0.5, term_hi=2.0):
    """nn nodes numbered x + nx*y + nx*ny*z, 6-connected where both ends
    exist: whole nx*ny planes and, if nx*ny does not divide nn, a partial
    last plane.  s links the nodes of plane 0, t those of the last (partial)
    plane.  Streams: 0 interior capacities, 1 source, 2 sink capacities."""
    P = nx * ny
    ids = np.arange(nn, dtype=np.int64)
    x = ids % nx
    y = (ids // nx) % ny
    has = np.stack([(x < nx - 1) & (ids + 1 < nn), (y < ny - 1) & (ids + nx < nn), ids + P < nn], axis=1)
    nbr = np.stack([ids + 1, ids + nx, ids + P], axis=1)
    src = np.broadcast_to(ids[:, None], has.shape)[has]
    dst = nbr[has]
    mi = src.shape[0]
    c_int = rng.uniform_range(seed, 0, mi, cap_lo, cap_hi)
    s, t = nn, nn + 1
    first = np.arange(min(P, nn), dtype=np.int64)
    last = np.arange((nn - 1) // P * P, nn, dtype=np.int64)
    c_s = rng.uniform_range(seed, 1, first.shape[0], term_lo, term_hi)
    c_t = rng.uniform_range(seed, 2, last.shape[0], term_lo, term_hi)
    eu = np.concatenate([src, np.full(first.shape[0], s, np.int64), last])
    ev = np.concatenate([dst, first, np.full(last.shape[0], t, np.int64)])
    cap = np.concatenate([c_int, c_s, c_t])
    return Graph(nn + 2, s, t, eu, ev, cap,
                 meta=dict(kind="grid3d_box", shape=(nx, ny), nodes=nn, seed=seed, interior=mi))


# ----------------------------------------------------------------------------
# G(n, p) for exhaustive checks
# ----------------------------------------------------------------------------
def _connected(n, eu, ev):
    adj = [[] for _ in range(n)]
    for a, b in zip(eu.tolist(), ev.tolist()):
        adj[a].append(b)
        adj[b].append(a)
    seen = [False] * n
    seen[0] = True
    stack = [0]
    while stack:
        u = stack.pop()
        for v in adj[u]:
            if not seen[v]:
                seen[v] = True
                stack.append(v)
    return all(seen)


def gnp(n=16, p=0.3, seed=1, cap_lo=0.1, cap_hi=1.0, max_attempts=10000):
    """G(n,p) with s=0, t=n-1, resampled until connected.

    Attempt a uses streams 2a (edge coins, by pair index in lexicographic
    order) and 2a+1 (capacities, by kept-edge index).
    """
    iu, jv = np.triu_indices(n, k=1)
    for attempt in range(max_attempts):
        coin = rng.uniform(seed, 2 * attempt, np.arange(iu.shape[0], dtype=np.uint64))
        keep = coin < p
        eu = iu[keep].astype(np.int64)
        ev = jv[keep].astype(np.int64)
        if eu.shape[0] == 0 or not _connected(n, eu, ev):
            continue
        cap = rng.uniform_range(seed, 2 * attempt + 1, eu.shape[0], cap_lo, cap_hi)
        return Graph(n, 0, n - 1, eu, ev, cap,
                     meta=dict(kind="gnp", n=n, p=p, seed=seed, attempt=attempt))
    raise RuntimeError("gnp: no connected sample")


# ----------------------------------------------------------------------------
# 3-D segmentation-like grid
# ----------------------------------------------------------------------------
def smooth_field(N, seed, corr_len=8.0, trunc=17):
    """Standardised periodic Gaussian random field on an N^3 grid.

    White N(0,1) noise (stream 0, index = node id) is filtered along each
    axis by a periodic Gaussian of std corr_len/sqrt(2), truncated at
    +-trunc voxels, so that the field's autocorrelation has std corr_len.
    Returns an array indexed [z, y, x].
    """
    sig = corr_len / np.sqrt(2.0)
    w = rng.normal(seed, 0, N * N * N).reshape(N, N, N)
    d = np.arange(N)
    d = np.minimum(d, N - d)
    h = np.where(d <= trunc, np.exp(-(d.astype(np.float64) ** 2) / (2.0 * sig * sig)), 0.0)
    H = np.fft.rfft(h)
    for axis in range(3):
        F = np.fft.rfft(w, axis=axis)
        shape = [1, 1, 1]
        shape[axis] = H.shape[0]
        F *= H.reshape(shape)
        w = np.fft.irfft(F, n=N, axis=axis)
        del F
    w -= w.mean()
    w /= w.std()
    return w


def grid3d_seg(N=128, seed=1, corr_len=8.0, beta=0.05, mu_fg=0.3, mu_bg=0.7, sd=0.15,
               floor=1e-3, with_intensity=False):
    """6-connected N^3 grid with intensity-driven capacities.

    I = clip(0.5 + 0.2 z, 0, 1) for a standardised smooth field z.
    Interior capacity exp(-(I_i - I_j)^2 / beta).  Terminal capacities are
    negative log-likelihoods (Gaussian normaliser dropped, + floor): the
    source edge carries the background cost, the sink edge the foreground
    cost, so foreground (mean mu_fg) ends on the source side.
    """
    nn = N * N * N
    I = np.clip(0.5 + 0.2 * smooth_field(N, seed, corr_len), 0.0, 1.0).reshape(-1)
    ids = np.arange(nn, dtype=np.int64)
    x = ids % N
    y = (ids // N) % N
    z = ids // (N * N)
    has = np.stack([x < N - 1, y < N - 1, z < N - 1], axis=1)
    del x, y, z
    nbr = np.stack([ids + 1, ids + N, ids + N * N], axis=1)
    src = np.broadcast_to(ids[:, None], has.shape)[has]
    dst = nbr[has]
    del nbr, has
    dI = I[src] - I[dst]
    c_int = np.exp(-(dI * dI) / beta)
    del dI
    c_s = (I - mu_bg) ** 2 / (2.0 * sd * sd) + floor
    c_t = (I - mu_fg) ** 2 / (2.0 * sd * sd) + floor
    s, t = nn, nn + 1
    eu = np.concatenate([src, np.full(nn, s, np.int64), ids])
    ev = np.concatenate([dst, ids, np.full(nn, t, np.int64)])
    cap = np.concatenate([c_int, c_s, c_t])
    meta = dict(kind="grid3d_seg", N=N, seed=seed, interior=int(src.shape[0]))
    if with_intensity:
        meta["I"] = I
    return Graph(nn + 2, s, t, eu, ev, cap, meta=meta)


def grid3d_seg_slab(N=256, planes=32, seed=2):
    """The first `planes` z-planes of grid3d_seg(N, seed): the share of one
    GPU when the N^3 instance is split into z-slabs (N^2 * planes nodes,
    numbered as in the full grid; edges to the next slab dropped)."""
    g = grid3d_seg(N, seed=seed)
    keep_n = N * N * planes
    s, t = keep_n, keep_n + 1
    term_u, term_v = (g.eu == g.s) | (g.eu == g.t), (g.ev == g.s) | (g.ev == g.t)
    inside = (term_u | (g.eu < keep_n)) & (term_v | (g.ev < keep_n))
    eu = np.where(g.eu == g.s, s, np.where(g.eu == g.t, t, g.eu))[inside]
    ev = np.where(g.ev == g.s, s, np.where(g.ev == g.t, t, g.ev))[inside]
    cap = g.cap[inside]
    interior = int(np.sum((eu < keep_n) & (ev < keep_n)))
    meta = dict(kind="grid3d_seg_slab", N=N, planes=planes, seed=seed, interior=interior)
    return Graph(keep_n + 2, s, t, eu, ev, cap, meta=meta)


# ----------------------------------------------------------------------------
# R-MAT FlowImprove-style instances
# ----------------------------------------------------------------------------
_RMAT_Q = (0.57, 0.19, 0.19)          # (a, b, c); d = 1 - a - b - c = 0.05


def _rmat_candidates(seed, scale, start, count):
    """`count` R-MAT candidate pairs; candidate j uses stream 1 words.

    Each 64-bit word supplies four 16-bit uniforms, one per recursion
    level (most significant bit first).
    """
    a, b, c = _RMAT_Q
    ta = int(round(a * 65536))
    tb = int(round((a + b) * 65536))
    tc = int(round((a + b + c) * 65536))
    words = (scale + 3) // 4
    j = np.arange(start, start + count, dtype=np.uint64)
    src = np.zeros(count, np.int64)
    dst = np.zeros(count, np.int64)
    level = 0
    for wi in range(words):
        w = rng.bits64(seed, 1, j * np.uint64(words) + np.uint64(wi))
        for q in range(4):
            if level >= scale:
                break
            u = ((w >> np.uint64(16 * q)) & np.uint64(0xFFFF)).astype(np.int64)
            bit = scale - 1 - level
            right = (u >= ta) & ((u < tb) | (u >= tc))       # quadrants b and d
            down = u >= tb                                   # quadrants c and d
            src |= down.astype(np.int64) << bit
            dst |= right.astype(np.int64) << bit
            level += 1
    return src, dst


def rmat_flowimprove(seed, log2_lo=10.0, log2_hi=17.0, avg_degree=8, ball_frac=0.05,
                     cap_lo=0.5, cap_hi=1.0, t_scale=0.05):
    """One R-MAT instance with a seeded BFS ball attached to s.

    n = floor(2^U(log2_lo, log2_hi)) (stream 0, index 0); candidates from
    stream 1; endpoints >= n and self loops rejected; duplicates dropped
    keeping the first occurrence, until avg_degree*n/2 unique edges.
    Capacities U[cap_lo, cap_hi) rounded to float32 (stream 2).  Isolated
    nodes are removed.  The ball is the first ceil(ball_frac n') nodes of a
    BFS (neighbours in ascending id) from a node of the largest component
    chosen by stream 3; ball nodes link to s with their weighted degree,
    all others link to t with t_scale times their weighted degree.
    """
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components

    u0 = rng.uniform(seed, 0, [0])[0]
    n = int(np.floor(2.0 ** (log2_lo + (log2_hi - log2_lo) * u0)))
    scale = max(1, int(np.ceil(np.log2(n))))
    want = avg_degree * n // 2
    keys = np.empty(0, np.int64)
    start = 0
    while True:
        cnt = max(2 * want, 1024)
        a, b = _rmat_candidates(seed, scale, start, cnt)
        start += cnt
        ok = (a < n) & (b < n) & (a != b)
        lo = np.minimum(a[ok], b[ok])
        hi = np.maximum(a[ok], b[ok])
        keys = np.concatenate([keys, lo * n + hi])
        _, first = np.unique(keys, return_index=True)
        if first.shape[0] >= want:
            keys = keys[np.sort(first)][:want]
            break
        keys = keys[np.sort(first)]
    eu = keys // n
    ev = keys % n
    cap = rng.uniform_range(seed, 2, want, cap_lo, cap_hi).astype(np.float32).astype(np.float64)
    deg = np.bincount(eu, minlength=n) + np.bincount(ev, minlength=n)
    alive = deg > 0
    relabel = np.cumsum(alive) - 1
    n2 = int(alive.sum())
    eu = relabel[eu].astype(np.int64)
    ev = relabel[ev].astype(np.int64)
    wdeg = np.bincount(eu, weights=cap, minlength=n2) + np.bincount(ev, weights=cap, minlength=n2)
    A = coo_matrix((np.ones(2 * want), (np.concatenate([eu, ev]), np.concatenate([ev, eu]))),
                   shape=(n2, n2)).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    ncomp, lab = connected_components(A, directed=False)
    big = np.argmax(np.bincount(lab))
    members = np.nonzero(lab == big)[0]
    start_node = int(members[int(rng.uniform(seed, 3, [0])[0] * members.shape[0])])
    ball_size = int(np.ceil(ball_frac * n2))
    if ball_size >= members.shape[0]:
        raise RuntimeError("rmat: ball would cover the whole component")
    indptr, indices = A.indptr, A.indices
    order = [start_node]
    seen = np.zeros(n2, bool)
    seen[start_node] = True
    head = 0
    while len(order) < ball_size:
        u = order[head]
        head += 1
        for v in indices[indptr[u]:indptr[u + 1]]:
            if not seen[v]:
                seen[v] = True
                order.append(int(v))
    in_ball = np.zeros(n2, bool)
    in_ball[np.asarray(order[:ball_size])] = True
    s, t = n2, n2 + 1
    bnodes = np.nonzero(in_ball)[0].astype(np.int64)
    onodes = np.nonzero(~in_ball)[0].astype(np.int64)
    eu_all = np.concatenate([eu, np.full(bnodes.shape[0], s, np.int64), onodes])
    ev_all = np.concatenate([ev, bnodes, np.full(onodes.shape[0], t, np.int64)])
    cap_all = np.concatenate([cap, wdeg[bnodes], t_scale * wdeg[onodes]])
    return Graph(n2 + 2, s, t, eu_all, ev_all, cap_all,
                 meta=dict(kind="rmat", seed=seed, n_raw=n, interior=int(want),
                           components=int(ncomp)))


def _rmat_one(args):
    seed, kw = args
    return rmat_flowimprove(seed, **kw)


def rmat_batch(count=512, first_seed=1000, workers=None, **kw):
    """Instances first_seed .. first_seed+count-1 (each a pure function of its
    seed), generated by a pool of threads in this process (numpy releases the
    interpreter lock in the heavy steps).  No child process is started, so a
    GPU or profiled process that calls this stays a single process."""
    seeds = [(first_seed + i, kw) for i in range(count)]
    if workers is None:
        workers = min(16, os.cpu_count() or 1)
    if workers <= 1 or count < 4:
        return [_rmat_one(a) for a in seeds]
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(workers) as pool:
        return list(pool.map(_rmat_one, seeds))


# ----------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------
def workload(name, **kw):
    """Named workloads: 'grid64' (64x64 2-D), 'seg128', 'seg256', 'seg192',
    'seg64' (3-D segmentation grids), 'gnp16' (one G(16,0.3) graph)."""
    if name == "grid64":
        return grid2d(64, 64, seed=kw.get("seed", 0))
    if name.startswith("seg"):
        N = int(name[3:])
        return grid3d_seg(N, seed=kw.get("seed", {128: 1, 256: 2}.get(N, 20000)))
    if name == "gnp16":
        return gnp(16, 0.3, seed=kw.get("seed", 1))
    raise KeyError(name)
