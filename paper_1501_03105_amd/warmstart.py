"""Learned warm start: training examples, training, the choice of how the
prediction enters the start, the no-network baseline (the best constant first
eps, chosen on the training graphs), and the solves that measure what the
network saves.

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


def schedule_rounds(eps_first, eps_last, factor):
    """Rounds from eps_first down to eps_last (inclusive) at the given factor."""
    return max(1, int(np.floor(np.log(eps_last / eps_first) / np.log(factor) + 1e-9)) + 1)


def time_to_final(mc, eps_first=None, net=None, gamma=0.0, intensity=None, stream=None):
    """Round 0, then (with a network) the warm start, then the reweighted
    rounds from the first round's eps down to the plain schedule's last eps
    (eps0 * factor^(T-1)) in one solve, then the sweep cut: a start that skips
    the early rounds ends at the same smoothing as the plain start, and
    nothing here knows the answer.  eps_first: the first round's eps (default:
    the options' eps0, or the network's prediction snapped to the schedule).
    Returns rounds, CG iterations, seconds (all of it timed) and the cut."""
    o = mc.opt
    eps_last = o.eps0 * o.eps_factor ** (o.rounds - 1)
    _sync(stream)
    t0 = time.perf_counter()
    _, st0 = mc.solve_range(0, 0)
    le = None
    if net is not None:
        le = net.warm_start(mc, gamma, intensity)
    if eps_first is None:
        eps_first = o.eps0 if le is None else snap_eps(le, o.eps0, o.eps_factor, min(EPS_GRID))
    k = schedule_rounds(eps_first, eps_last, o.eps_factor)
    _, st = mc.solve_range(1, k, eps_first=eps_first)
    _, val, _ = mc.cut()
    _sync(stream)
    sec = time.perf_counter() - t0
    return dict(rounds=k, cg_iters=int(st0[0]["cg_iters"] + sum(r["cg_iters"] for r in st[1:])),
                seconds=sec, cut=val, eps_first=eps_first, log_eps=le)


def best_constant_eps(examples, eps_grid=EPS_GRID, tol=1e-6, stream=None, log=None):
    """The no-network baseline: the first eps (from eps_grid and the options'
    eps0) with the least total CG work over the training graphs, among those
    whose cut is within tol of every graph's reference under time_to_final.
    Returns (eps, {eps: (total CG iterations, all reached)})."""
    table = {}
    cands = sorted(set(eps_grid) | {examples[0].mc.opt.eps0}, reverse=True)
    for eps in cands:
        tot, ok = 0, True
        for e in examples:
            r = time_to_final(e.mc, eps_first=eps, stream=stream)
            tot += r["cg_iters"]
            ok &= r["cut"] <= e.ref_cut * (1.0 + tol)
        table[eps] = (tot, ok)
        if log:
            log(f"constant first eps {eps:.3g}: {tot} CG iterations, all cuts reached: {ok}")
    feasible = [eps for eps in cands if table[eps][1]]
    best = min(feasible, key=lambda eps: table[eps][0]) if feasible else examples[0].mc.opt.eps0
    return best, table


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
    """CG iterations of the rounds from every (gamma, eps_1) start down to the
    plain schedule's last eps (inf where the cut is not within tol of the
    example's).  The blend x_r0 + gamma (xhat - x_r0) is formed on the device
    by irls_gnn_warm_start."""
    o = e.mc.opt
    eps_last = o.eps0 * o.eps_factor ** (o.rounds - 1)
    out = np.full((len(gammas), len(eps_grid)), np.inf)
    for i, gam in enumerate(gammas):
        for j, eps in enumerate(eps_grid):
            e.mc.set_potentials(e.x_r0)
            gnn.warm_start(e.mc, gam, e.intensity)
            _, st = e.mc.solve_range(1, schedule_rounds(eps, eps_last, o.eps_factor), eps_first=eps)
            _, val, _ = e.mc.cut()
            if val <= e.ref_cut * (1.0 + tol):
                out[i, j] = sum(r["cg_iters"] for r in st[1:])
    _sync(stream)
    return out


def fit(examples, epochs_x, epochs_eps, lr=1e-3, seed=0, gammas=GAMMAS, eps_grid=EPS_GRID, stream=None,
        log=None, max_cost_graphs=None):
    """Two stages.  (1) Train on the converged potentials of every example.
    (2) With that x head, measure every (gamma, eps_1) start on the training
    graphs (at most max_cost_graphs of them, evenly spaced); gamma is the one
    with the least total CG work, each measured graph's eps target is its best
    eps_1 under that gamma; train on those graphs, now with the eps term
    weighted in.  Returns (network, gamma, cost table [graphs, gammas, eps])."""
    net = Gnn(seed=seed)
    h1 = train(net, examples, epochs_x, lr=lr, lam=0.0, seed=seed, log=log)
    sub = examples
    if max_cost_graphs and len(examples) > max_cost_graphs:
        sub = [examples[int(i)] for i in np.linspace(0, len(examples) - 1, max_cost_graphs)]
    rows = []
    for j, e in enumerate(sub):
        rows.append(start_costs(net, e, gammas, eps_grid, stream=stream))
        if log and (j + 1) % 8 == 0:
            log(f"start costs measured on {j + 1} of {len(sub)} graphs")
    costs = np.stack(rows)
    best_per = costs.min(axis=2)                           # [graphs, gammas]
    total = np.where(np.isfinite(best_per), best_per, 1e30).sum(axis=0)
    gi = int(np.argmin(total))
    for e, c in zip(sub, costs[:, gi, :]):
        e.t = float(np.log(eps_grid[int(np.argmin(c))] if np.isfinite(c).any() else e.mc.opt.eps0))
    h2 = train(net, sub, epochs_eps, lr=lr, lam=1.0, seed=seed + 1, log=log)
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
