"""Learned warm start: training examples, training, the choice of how the
prediction enters the start, and the round-by-round solves that measure what
the network saves.

Every computation runs in the library (irls_gnn_* for the network,
irls_mincut_* for IRLS); this module only sequences the calls.

The rounds start from
    x0 = x_r0 + gamma (xhat - x_r0)     at eps_1 = the predicted eps,
where x_r0 is the round-0 solution (W = C) and xhat the network's prediction
of the converged potentials.  gamma is chosen on the training graphs from
GAMMAS; gamma = 0 keeps round 0's potentials and uses the predicted eps only.
A confidently wrong xhat is harmful at small eps (its node gets tiny
conductances to its neighbours and the rounds are slow to move it back),
which is why the prediction enters as a bounded blend.
"""
import time
from dataclasses import dataclass

import numpy as np

from . import Gnn, MinCut

GAMMAS = (0.0, 0.1, 0.25)
EPS_GRID = (1e-2, 3e-3, 1e-3, 3e-4, 1e-4)


@dataclass
class Example:
    mc: MinCut
    intensity: np.ndarray
    x_r0: np.ndarray          # round-0 potentials (network input)
    y: np.ndarray             # converged potentials (x target)
    ref_cut: float
    t: float = 0.0            # log of the best starting eps (eps target)


def _sync(stream):
    if stream is not None:
        stream.synchronize()


def run_rounds(mc, ref_cut, tol, eps_first, factor, max_rounds, stream=None):
    """Reweighted rounds from the potentials mc holds, one at a time, until the
    sweep cut is within tol (relative) of ref_cut or max_rounds are done.
    Returns (rounds, CG iterations, seconds in the solves, last cut)."""
    rounds, iters, sec = 0, 0, 0.0
    _, val, _ = mc.cut()
    eps = eps_first
    while val > ref_cut * (1.0 + tol) and rounds < max_rounds:
        t0 = time.perf_counter()
        _, st = mc.solve_range(1, 1, eps_first=eps)
        _sync(stream)
        sec += time.perf_counter() - t0
        iters += st[1]["cg_iters"]
        rounds += 1
        eps *= factor
        _, val, _ = mc.cut()
    return rounds, iters, sec, val


def make_example(g, intensity, opts, stream=None):
    """Solve g with the plain start; keep round 0's potentials (input), the
    converged potentials (target) and the cut (reference)."""
    mc = MinCut.from_graph(g, stream=stream, solver=1, **opts)
    o = mc.opt
    mc.solve_range(0, 0)
    x_r0 = mc.potentials()
    mc.solve_range(1, o.rounds, eps_first=o.eps0)
    y = mc.potentials()
    _, ref, _ = mc.cut()
    return Example(mc=mc, intensity=intensity, x_r0=x_r0, y=y, ref_cut=ref, t=float(np.log(o.eps0)))


def train(gnn, examples, epochs, lr=1e-3, lam=0.01, seed=0, log=None):
    """Adam over the examples, one graph per step, in a seeded order.
    Returns the mean loss of every epoch."""
    order_rng = np.random.default_rng(seed)
    history = []
    for ep in range(epochs):
        tot = 0.0
        for i in order_rng.permutation(len(examples)):
            e = examples[i]
            loss, _ = gnn.loss_grad(e.mc, e.y, e.t, lam=lam, intensity=e.intensity, x_start=e.x_r0)
            gnn.adam_step(lr)
            tot += loss
        history.append(tot / len(examples))
        if log:
            log(f"epoch {ep}: mean loss {history[-1]:.5f}")
    return history


def start_costs(gnn, e, gammas=GAMMAS, eps_grid=EPS_GRID, tol=1e-6, stream=None):
    """CG iterations to reach the example's cut from every (gamma, eps_1)
    start (inf where max rounds do not reach it)."""
    o = e.mc.opt
    xh, _ = gnn.predict(e.mc, e.intensity, x_start=e.x_r0)
    out = np.full((len(gammas), len(eps_grid)), np.inf)
    for i, gam in enumerate(gammas):
        x0 = e.x_r0 + gam * (xh - e.x_r0)
        for j, eps in enumerate(eps_grid):
            e.mc.solve_range(2, 0, x0=x0)
            _, it, _, val = run_rounds(e.mc, e.ref_cut, tol, eps, o.eps_factor, o.rounds, stream)
            if val <= e.ref_cut * (1.0 + tol):
                out[i, j] = it
    return out


def fit(examples, epochs_x, epochs_eps, lr=1e-3, seed=0, gammas=GAMMAS, eps_grid=EPS_GRID, stream=None,
        log=None):
    """Two stages.  (1) Train on the converged potentials.  (2) With that x
    head, measure every (gamma, eps_1) start on the training graphs; gamma is
    the one with the least total CG work, each graph's eps target is its best
    eps_1 under that gamma; train on, now with the eps term weighted in.
    Returns (network, gamma, cost table [graphs, gammas, eps])."""
    net = Gnn(seed=seed)
    h1 = train(net, examples, epochs_x, lr=lr, lam=0.0, seed=seed)
    costs = np.stack([start_costs(net, e, gammas, eps_grid, stream=stream) for e in examples])
    best_per = costs.min(axis=2)                           # [graphs, gammas]
    total = np.where(np.isfinite(best_per), best_per, 1e30).sum(axis=0)
    gi = int(np.argmin(total))
    for e, c in zip(examples, costs[:, gi, :]):
        e.t = float(np.log(eps_grid[int(np.argmin(c))] if np.isfinite(c).any() else e.mc.opt.eps0))
    h2 = train(net, examples, epochs_eps, lr=lr, lam=1.0, seed=seed + 1)
    if log:
        log(f"x stage loss {h1[0]:.4f} -> {h1[-1]:.4f}; gamma {gammas[gi]}; "
            f"eps stage loss {h2[0]:.4f} -> {h2[-1]:.4f}")
    return net, gammas[gi], costs


def snap_eps(log_eps, eps0, factor, lo):
    """Predicted eps snapped onto the schedule eps0 * factor^k, clamped to [lo, eps0]."""
    eps = float(np.exp(log_eps))
    eps = min(max(eps, lo), eps0)
    k = int(round(np.log(eps / eps0) / np.log(factor)))
    return eps0 * factor ** max(k, 0)


def time_to_cut(mc, ref_cut, tol, max_rounds, net=None, gamma=0.0, intensity=None, eps_first=None,
                stream=None):
    """Round 0, then (with a network) the warm start, then rounds until the
    sweep cut is within tol of ref_cut.  The per-round sweeps only decide when
    to stop and are not timed; one final sweep is.  eps_first: the first
    round's eps (default: the options' eps0, or the network's prediction)."""
    o = mc.opt
    t0 = time.perf_counter()
    _, st = mc.solve_range(0, 0)
    le = None
    if net is not None:
        le = net.warm_start(mc, gamma, intensity)
    _sync(stream)
    sec = time.perf_counter() - t0
    if eps_first is None:
        eps_first = o.eps0 if le is None else snap_eps(le, o.eps0, o.eps_factor, min(EPS_GRID))
    r, it, s2, val = run_rounds(mc, ref_cut, tol, eps_first, o.eps_factor, max_rounds, stream)
    t0 = time.perf_counter()
    mc.cut()
    _sync(stream)
    sec += s2 + time.perf_counter() - t0
    return dict(rounds=r, cg_iters=it + st[0]["cg_iters"], seconds=sec, cut=val, eps_first=eps_first,
                log_eps=le, reached=val <= ref_cut * (1.0 + tol))
