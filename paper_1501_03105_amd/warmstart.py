"""Learned warm start: training examples, the training loop and the
round-by-round solves used to measure what the network saves.

Every computation runs in the library (irls_gnn_* for the network,
irls_mincut_* for IRLS); this module only sequences the calls.
"""
import time
from dataclasses import dataclass, field

import numpy as np

from . import Gnn, MinCut


def eps_target(stats, tol=0.01):
    """Log of the eps of the first round whose ||CBx||_1 is within `tol` of
    the last round's: how far the plain trajectory has to run before its
    potentials settle (the network learns to start about there)."""
    final = stats[-1]["l1"]
    for r in stats[1:]:
        if abs(r["l1"] - final) <= tol * final:
            return float(np.log(r["eps"]))
    return float(np.log(stats[-1]["eps"]))


@dataclass
class Example:
    mc: MinCut
    intensity: np.ndarray
    y: np.ndarray
    t: float
    stats: list = field(default_factory=list)


def make_example(g, intensity, opts, stream=None):
    """Solve g with the plain start; its converged potentials are the target."""
    mc = MinCut.from_graph(g, stream=stream, solver=1, **opts)
    _, st = mc.solve()
    return Example(mc=mc, intensity=intensity, y=mc.potentials(), t=eps_target(st), stats=st)


def train(gnn, examples, epochs, lr=2e-3, lam=0.1, seed=0, log=None):
    """Adam over the examples, one graph per step, in a seeded order."""
    order_rng = np.random.default_rng(seed)
    history = []
    for ep in range(epochs):
        tot = 0.0
        for i in order_rng.permutation(len(examples)):
            e = examples[i]
            loss, _ = gnn.loss_grad(e.mc, e.y, e.t, lam=lam, intensity=e.intensity)
            gnn.adam_step(lr)
            tot += loss
        history.append(tot / len(examples))
        if log:
            log(f"epoch {ep}: mean loss {history[-1]:.5f}")
    return history


def snap_eps(log_eps, eps0, factor, eps_last):
    """Predicted eps snapped onto the schedule eps0 * factor^k, k >= 0."""
    eps = float(np.exp(log_eps))
    eps = min(max(eps, eps_last), eps0)
    k = int(round(np.log(eps / eps0) / np.log(factor)))
    return eps0 * factor ** max(k, 0)


def rounds_to_cut(mc, ref_cut, tol, eps_first, factor, max_rounds, x0=None, sync=None):
    """IRLS one round at a time until the sweep cut is within tol (relative)
    of ref_cut.  x0 None: the plain start (round 0 with W = C, then rounds
    from eps_first); else start from x0 at eps_first.  Time counts the solves
    and one final sweep (the per-round sweeps only decide when to stop)."""
    sync = sync or (lambda: None)
    solve_s = 0.0
    iters = 0
    t0 = time.perf_counter()
    if x0 is None:
        _, st = mc.solve_range(0, 0)
        iters += st[0]["cg_iters"]
    else:
        mc.solve_range(2, 0, x0=x0)
    sync()
    solve_s += time.perf_counter() - t0
    eps = eps_first
    rounds = 0
    _, val, _ = mc.cut()
    while abs(val - ref_cut) > tol * ref_cut and rounds < max_rounds:
        t0 = time.perf_counter()
        _, st = mc.solve_range(1, 1, eps_first=eps)
        sync()
        solve_s += time.perf_counter() - t0
        iters += st[1]["cg_iters"]
        rounds += 1
        eps *= factor
        _, val, _ = mc.cut()
    t0 = time.perf_counter()
    mc.cut()
    sync()
    sweep_s = time.perf_counter() - t0
    return dict(rounds=rounds, cg_iters=iters, seconds=solve_s + sweep_s, cut=val,
                reached=abs(val - ref_cut) <= tol * ref_cut)
