"""Two-level rounding of the final potentials (the paper's two-level rounding
procedure, Section 3.4, with the proposition on its correctness).

TEST INFRASTRUCTURE ONLY: imported by tests/ and nothing on the product path.

Steps, in the paper's order and notation:

1. K-means with two centres on the components of x^(T), started at 0.1 and
   0.9, gives centres c0 < c1; gamma0 = c0 + 0.05 and gamma1 = c1 - 0.05.
2. Nodes split into S0 (x_u <= gamma0, coalesced with the sink), S1
   (x_u >= gamma1, coalesced with the source) and Sc (the rest).
3. The coarse graph G_c has nodes {s_c, t_c} and Sc; its edges are the
   edges inside Sc, {s_c, u} with the summed capacity from u to S1, {t_c, u}
   with the summed capacity from u to S0, and {s_c, t_c} with the summed
   capacity between S1 and S0.
4. An exact minimum s_c-t_c cut of G_c (the oracle's push-relabel) induces
   the cut S = S1 united with the source side's part of Sc.

Readings where the paper is silent: K-means runs on all n components of x
(x_s = 1 and x_t = 0 included); it is Lloyd's iteration in one dimension, a
value joins the upper cluster when it lies strictly above the midpoint of
the two centres, a centre is its cluster's mean (unchanged if the cluster is
empty), and it stops when an assignment repeats (at most 100 updates).  The
coarse nodes are Sc in ascending id, then s_c, then t_c.
"""
import numpy as np

from . import cut_value, maxflow


def kmeans2(x, c0=0.1, c1=0.9, max_updates=100):
    """Two-centre K-means on the values x.  Returns (c0, c1, updates)."""
    x = np.asarray(x, dtype=np.float64)
    prev = None
    updates = 0
    while updates < max_updates:
        hi = x > 0.5 * (c0 + c1)
        if prev is not None and np.array_equal(hi, prev):
            break
        lo = ~hi
        if lo.any():
            c0 = float(np.sum(x[lo]) / lo.sum())
        if hi.any():
            c1 = float(np.sum(x[hi]) / hi.sum())
        prev = hi
        updates += 1
    return c0, c1, updates


class Coarse:
    """The coarse graph of step 3: node count, s_c, t_c, merged edges."""

    def __init__(self, n, s, t, eu, ev, cap):
        self.n, self.s, self.t = n, s, t
        self.eu, self.ev, self.cap = eu, ev, cap


def classify(x, gamma0, gamma1):
    """0 for S0, 1 for S1, 2 for Sc."""
    x = np.asarray(x, dtype=np.float64)
    return np.where(x <= gamma0, 0, np.where(x >= gamma1, 1, 2)).astype(np.int8)


def coarse_graph(g, cls):
    """Step 3: contract S1 to s_c and S0 to t_c; merge parallel edges by
    summing their capacities in input order; drop edges inside S0 or S1."""
    sc_nodes = np.flatnonzero(cls == 2)
    nc = sc_nodes.size
    cid = np.empty(g.n, dtype=np.int64)
    cid[sc_nodes] = np.arange(nc)
    cid[cls == 1] = nc          # s_c
    cid[cls == 0] = nc + 1      # t_c
    merged = {}
    for a, b, c in zip(cid[g.eu], cid[g.ev], g.cap):
        if a == b:
            continue
        key = (min(a, b), max(a, b))
        merged[key] = merged.get(key, 0.0) + float(c)
    keys = sorted(merged)
    eu = np.array([k[0] for k in keys], dtype=np.int64)
    ev = np.array([k[1] for k in keys], dtype=np.int64)
    cap = np.array([merged[k] for k in keys], dtype=np.float64)
    return Coarse(nc + 2, nc, nc + 1, eu, ev, cap), sc_nodes


def two_level(g, x):
    """Steps 1-4 on graph g with potentials x (all n nodes).  Returns
    (in_S bool [n], exact cut value, info dict)."""
    c0, c1, updates = kmeans2(x)
    gamma0, gamma1 = c0 + 0.05, c1 - 0.05
    cls = classify(x, gamma0, gamma1)
    cg, sc_nodes = coarse_graph(g, cls)
    in_c, value_c = maxflow(cg)
    in_S = cls == 1
    in_S[sc_nodes] = in_c[:sc_nodes.size]
    value = cut_value(g, in_S)
    info = dict(c0=c0, c1=c1, updates=updates, gamma0=gamma0, gamma1=gamma1,
                n_s0=int((cls == 0).sum()), n_s1=int((cls == 1).sum()), n_sc=int(sc_nodes.size),
                coarse_edges=int(cg.eu.size), coarse_value=value_c)
    return in_S, value, info
