"""Helpers shared by the GPU tests (graph builders and comparison helpers)."""
import sys

import numpy as np

from gen.graphs import Graph


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def mk(n, s, t, edges):
    e = np.asarray(edges, dtype=np.float64).reshape(-1, 3)
    return Graph(n, s, t, e[:, 0].astype(np.int64), e[:, 1].astype(np.int64), e[:, 2].copy())


def max_pot_err(x_gpu, x_orc):
    """Relative potential error: max |dx| / max |x| (x_s = 1 so this is absolute)."""
    return float(np.max(np.abs(x_gpu - x_orc)) / max(np.max(np.abs(x_orc)), 1e-300))


def cmp_stats(sg, so, fields=("s_eps", "l1", "flow", "flow_s", "flow_t", "vmin", "vmax"), rtol=1e-7):
    bad = []
    for f in fields:
        a, b = sg[f], so[f]
        if abs(a - b) > rtol * max(abs(b), 1e-12):
            bad.append((f, a, b))
    return bad
