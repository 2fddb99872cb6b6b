"""Writes the oracle's full runs of the two segmentation-grid workloads:

* ``seg128_oracle.json``: 128^3 grid, seed 1, 40 rounds, eps 0.1 halved per
  round, Jacobi-PCG to 1e-8;
* ``seg256_oracle.json``: 256^3 grid, seed 2, the same options;
* ``seg128-ilu_oracle.json``: the 128^3 instance with block-Jacobi PCG whose
  blocks are 4x4x4 tiles, each by ILU(0) (Section 3.1's second block
  strategy), the same rounds and tolerance.

Each file holds every round's record, the sweep cut (value, k*, size of the
source side, SHA-256 of the packed source-side mask), the potentials at a
seeded sample of nodes, the wall time of the run and the host it ran on.  It
calls only oracle/ and gen/.  A full 256^3 run takes about 11 minutes on 8
host threads.  Rerun only for a change of the oracle whose commit names the
passage of the paper that justifies it:

    python tests/golden/make_golden_fullsize.py [seg128|seg256 ...]
"""
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import gen  # noqa: E402
from gen import rng  # noqa: E402
import oracle  # noqa: E402

FIELDS = ("eps", "cg_iters", "rel_res", "true_rel_res", "s_eps", "l1", "flow", "flow_s", "flow_t",
          "vmin", "vmax", "lower_bound")
OPTS = dict(rounds=40, cg_rtol=1e-8)
# name: (grid edge, seed, ILU(0) tile edge or None for Jacobi)
WORKLOADS = {"seg128": (128, 1, None), "seg256": (256, 2, None), "seg128-ilu": (128, 1, 4)}
SAMPLES = 65536
SAMPLE_STREAM = 77          # the sample's own random stream, distinct from the generator's


def sample_nodes(n_nonterminal, seed):
    """Seeded sample of non-terminal node ids (sorted, distinct), always
    including the first and the last row."""
    u = rng.uniform(seed, SAMPLE_STREAM, np.arange(SAMPLES, dtype=np.uint64))
    ids = np.unique(np.minimum((u * n_nonterminal).astype(np.int64), n_nonterminal - 1))
    return np.unique(np.concatenate([ids, [0, n_nonterminal - 1]]))


def mask_digest(in_S):
    return hashlib.sha256(np.packbits(np.asarray(in_S, dtype=np.uint8)).tobytes()).hexdigest()


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def tile_blocks(N, B):
    """Block id of every node of an N^3 grid numbered x + N y + N^2 z (s and t
    last, given ids of their own past the grid): cubic tiles of B rows on a
    side, numbered x fastest."""
    ids = np.arange(N ** 3 + 2, dtype=np.int64)
    x, y, z = ids % N, (ids // N) % N, ids // (N * N)
    return (x // B) + (N // B) * ((y // B) + (N // B) * (z // B))


def run(name):
    N, seed, tile = WORKLOADS[name]
    g = gen.grid3d_seg(N, seed=seed)
    pre = dict(precond=2, block_of=tile_blocks(N, tile)) if tile else {}
    t0 = time.perf_counter()
    x, recs, rc = oracle.irls(g, **OPTS, **pre)
    inS, val, k, scale = oracle.sweep(g, x)
    secs = time.perf_counter() - t0
    nt = g.n - 2
    ids = sample_nodes(nt, seed)
    return {
        "config": f"grid3d_seg {N}^3 seed {seed}, rounds 40, eps0 0.1 halved, cg_rtol 1e-8 (oracle, FP64)"
                  + (f", block-Jacobi PCG over {tile}x{tile}x{tile} tiles by ILU(0)" if tile else ", Jacobi PCG"),
        "status": int(rc),
        "rounds": [{f: (int(r[f]) if f == "cg_iters" else float(r[f])) for f in FIELDS} for r in recs],
        "cg_iters_total": int(sum(r["cg_iters"] for r in recs)),
        "sweep": {"value": float(val), "k_star": int(k), "source_side_size": int(np.sum(inS)),
                  "mask_sha256": mask_digest(inS), "scale_exponent": int(scale)},
        "sample_ids": [int(i) for i in ids],
        "sample_potentials": [float(x[i]) for i in ids],
        "potentials_sum": float(np.sum(x[:nt])),
        "timing": {"seconds": secs, "threads": int(oracle.max_threads()), "cpu_model": cpu_model(),
                   "span": "irls (all rounds) + sweep, graph in host memory"},
    }


if __name__ == "__main__":
    names = sys.argv[1:] or list(WORKLOADS)
    here = os.path.dirname(os.path.abspath(__file__))
    for name in names:
        out = run(name)
        with open(os.path.join(here, f"{name}_oracle.json"), "w") as f:
            json.dump(out, f, indent=0)
        print(name, out["sweep"], out["cg_iters_total"], f"{out['timing']['seconds']:.1f} s", flush=True)
