"""Writes tests/golden/grid64_oracle.json: the oracle's run on the 64x64
grid configuration (seed 0; 30 rounds, eps 0.1 halved per round, Jacobi-PCG
to 1e-10).  It calls only oracle/ and gen/; the file lets a CPU test catch
any later change of the oracle's arithmetic.  Rerun only for a change whose
commit names the passage of the paper that justifies it:

    python tests/golden/make_golden.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import gen  # noqa: E402
import oracle  # noqa: E402

FIELDS = ("eps", "cg_iters", "l1", "flow", "flow_s", "flow_t", "s_eps", "vmin", "vmax", "lower_bound")
OPTS = dict(rounds=30, cg_rtol=1e-10)


def run():
    g = gen.grid2d(64, 64, seed=0)
    x, recs, rc = oracle.irls(g, **OPTS)
    inS, val, k, _ = oracle.sweep(g, x)
    return {
        "config": "grid2d 64x64 seed 0, rounds 30, eps0 0.1 halved, cg_rtol 1e-10 (oracle, FP64)",
        "status": int(rc),
        "rounds": [{f: (int(r[f]) if f == "cg_iters" else float(r[f])) for f in FIELDS} for r in recs],
        "potentials_sum": float(np.sum(x)),
        "potentials_norm2": float(np.sqrt(np.sum(x * x))),
        "sweep": {"value": float(val), "k_star": int(k), "source_side_size": int(np.sum(inS))},
    }


if __name__ == "__main__":
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "grid64_oracle.json"), "w") as f:
        json.dump(run(), f, indent=1)
