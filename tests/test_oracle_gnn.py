"""Pins of the learned warm-start oracle (oracle/gnn.py) to facts that do not
come from the oracle itself: the bfloat16 format, hand-computed features and
message passing on a small graph, closed forms of the loss, central finite
differences of the smooth model, and invariance under relabelling."""
import math

import numpy as np
import pytest
import torch

import gen
from tests.gpu_util import mk


@pytest.fixture
def G():
    import oracle.gnn as G
    saved = G.ROUND_BF16
    yield G
    G.ROUND_BF16 = saved


def five_node():
    # s = 0, t = 1, interior a = 2, b = 3, c = 4; a parallel edge and a loop
    return mk(5, 0, 1, [(0, 2, 1.0), (2, 3, 1.5), (3, 2, 0.5), (2, 4, 6.0), (3, 1, 3.0),
                        (4, 1, 1.0), (3, 4, 4.0), (4, 4, 9.0), (0, 1, 2.0)])


def test_bf16_rounding_is_nearest_even(G):
    # bfloat16 keeps 7 fraction bits: the spacing at 1 is 2^-7
    G.ROUND_BF16 = True
    u = 2.0 ** -7
    x = torch.tensor([1 + u / 2, 1 + 1.5 * u, 1 + u / 2 + 2.0 ** -20, -(1 + u / 2), 3.0, 1 + u / 4],
                     dtype=torch.float64)
    want = [1.0, 1 + 2 * u, 1 + u, -1.0, 3.0, 1.0]
    assert G.bf16(x).tolist() == want


def test_features_and_row_normalisation_by_hand(G):
    feats, A, ids = G.graph_inputs(five_node(), intensity=np.array([0, 0, 0.25, 0.5, 0.75]),
                                   x_start=np.array([1, 0, 0.9, 0.4, 0.1]))
    assert ids.tolist() == [2, 3, 4]
    # capacities at a: s 1, b 1.5 + 0.5, c 6; at b: a 2, t 3, c 4; at c: a 6, t 1, b 4
    want = [[math.log(2), 0, math.log(10), 0.25, 0.9],
            [0, math.log(4), math.log(10), 0.5, 0.4],
            [0, math.log(2), math.log(12), 0.75, 0.1]]
    assert np.allclose(feats.numpy(), want, rtol=0, atol=1e-15)
    dense = A.to_dense().numpy()
    assert np.allclose(dense, [[0, 2 / 8, 6 / 8], [2 / 6, 0, 4 / 6], [6 / 10, 4 / 10, 0]], rtol=0, atol=1e-15)


def test_one_layer_width_one_by_hand(G):
    """hidden = 1, one layer: every step written out with the numbers of the
    five-node graph; catches a transposed A, a swapped [h | A h] order, a
    missing bias or a wrong pooling."""
    G.ROUND_BF16 = False
    feats, A, _ = G.graph_inputs(five_node(), x_start=np.array([1, 0, 0.9, 0.4, 0.1]))
    p = {"W_in": torch.tensor([[1.0], [2.0], [0.0], [0.0], [1.0]], dtype=torch.float64),
         "b_in": torch.tensor([-0.1], dtype=torch.float64),
         "W0": torch.tensor([[1.0], [10.0]], dtype=torch.float64),
         "b0": torch.tensor([-5.0], dtype=torch.float64),
         "w_x": torch.tensor([0.5], dtype=torch.float64), "b_x": torch.tensor([-1.0], dtype=torch.float64),
         "w_e": torch.tensor([2.0], dtype=torch.float64), "b_e": torch.tensor([-3.0], dtype=torch.float64)}
    z, s, _ = G.forward(p, feats, A, hidden=1, layers=1)
    h0 = {"a": math.log(2) + 0.9 - 0.1, "b": 2 * math.log(4) + 0.4 - 0.1, "c": 2 * math.log(2) + 0.1 - 0.1}
    agg = {"a": 0.25 * h0["b"] + 0.75 * h0["c"],
           "b": h0["a"] / 3 + 2 * h0["c"] / 3,
           "c": 0.6 * h0["a"] + 0.4 * h0["b"]}
    h1 = {k: max(h0[k] + 10 * agg[k] - 5.0, 0.0) for k in "abc"}
    assert h1["a"] > 0 and h1["b"] > 0 and h1["c"] > 0
    assert np.allclose(z.numpy(), [0.5 * h1[k] - 1.0 for k in "abc"], rtol=0, atol=1e-13)
    assert abs(float(s) - (2.0 * sum(h1.values()) / 3 - 3.0)) < 1e-13


def test_zero_network_closed_form(G):
    """All weights zero: z = 0 everywhere, so the loss is log 2 plus the eps
    term, dL/db_x = mean(1/2 - y) and dL/db_e = 2 lam (b_e - t)."""
    G.ROUND_BF16 = True
    g = gen.grid2d(6, 5, seed=1)
    feats, A, ids = G.graph_inputs(g)
    y = np.zeros(g.n)
    y[ids[::3]] = 1.0
    flat = np.zeros(G.n_params())
    flat[-1] = -2.0
    lam, t = 0.3, -5.0
    L, grad = G.loss_and_grad(flat, feats, A, y[ids], t, lam)
    assert abs(L - (math.log(2) + lam * 9.0)) < 1e-14
    P = G.unflatten(np.arange(G.n_params()))
    assert abs(grad[int(P["b_x"][0])] - np.mean(0.5 - y[ids])) < 1e-15
    assert abs(grad[int(P["b_e"][0])] - 2 * lam * 3.0) < 1e-14


@pytest.mark.parametrize("seed", [1, 2])
def test_gradient_matches_central_differences(G, seed):
    G.ROUND_BF16 = False
    g = gen.gnp(14, 0.35, seed=seed)
    r = np.random.default_rng(seed)
    feats, A, ids = G.graph_inputs(g, intensity=r.uniform(0, 1, g.n), x_start=r.uniform(0, 1, g.n))
    y = (r.uniform(size=ids.shape[0]) < 0.5).astype(np.float64)
    flat = r.normal(0, 0.3, G.n_params())
    L, grad = G.loss_and_grad(flat, feats, A, y, -4.0, 0.2)
    h = 1e-6
    idx = r.choice(G.n_params(), 60, replace=False)
    P = G.unflatten(np.arange(G.n_params()))
    idx = np.concatenate([idx, [int(P["b_e"][0]), int(P["b_x"][0]), int(P["W_in"][0, 0]), int(P["b0"][3])]])
    for i in idx:
        fp, fm = flat.copy(), flat.copy()
        fp[i] += h
        fm[i] -= h
        fd = (G.loss_and_grad(fp, feats, A, y, -4.0, 0.2)[0] - G.loss_and_grad(fm, feats, A, y, -4.0, 0.2)[0]) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-6 * max(1.0, abs(grad[i])), (i, fd, grad[i])


def test_relabelling_permutes_predictions(G):
    """Renumbering the nodes permutes xhat and leaves the eps head alone."""
    G.ROUND_BF16 = False
    g = gen.grid2d(7, 6, seed=5)
    r = np.random.default_rng(0)
    perm = r.permutation(g.n)                  # old id -> new id
    g2 = mk(g.n, perm[g.s], perm[g.t], np.stack([perm[g.eu], perm[g.ev], g.cap], axis=1))
    flat = r.normal(0, 0.3, G.n_params())
    xs1 = r.uniform(0, 1, g.n)
    xs2 = np.empty(g.n)
    xs2[perm] = xs1
    f1, A1, ids1 = G.graph_inputs(g, x_start=xs1)
    f2, A2, ids2 = G.graph_inputs(g2, x_start=xs2)
    x1, s1 = G.predict(flat, f1, A1)
    x2, s2 = G.predict(flat, f2, A2)
    by_new = dict(zip(ids2.tolist(), x2.tolist()))
    assert np.allclose(x1, [by_new[int(perm[u])] for u in ids1], rtol=0, atol=1e-12)
    assert abs(s1 - s2) < 1e-12
