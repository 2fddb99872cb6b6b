"""CPU oracle of the learned warm start (test infrastructure only).

Not part of the paper: the paper warm-starts each CG solve from the previous
round (Section 3.1).  The learned warm start predicts a starting potential
vector and a starting smoothing eps for the IRLS rounds from per-node inputs,
with a small message-passing network.  This module states that network in
plain PyTorch CPU operations in float64, rounding to bfloat16 exactly where
the GPU kernels round (the inputs of every matrix product: weights, the
concatenated [h | A h] rows, and the gradient rows dZ), so the two can be
compared element by element.  Gradients come from torch.autograd, with the
bfloat16 roundings passed straight through.

Model (hidden width H = 64, three message-passing layers):
  f_u   = [log1p(c_us), log1p(c_ut), log1p(w_u), I_u, x0_u]
          w_u: all capacities at u; x0: the potentials the rounds start from
  h0    = relu(f W_in + b_in)
  a_l   = A h_{l-1},  A_uv = c_uv / sum_v' c_uv'           (interior neighbours)
  h_l   = relu(bf16([h_{l-1} | a_l]) bf16(W_l) + b_l)        l = 1, 2, 3
  z     = h3 w_x + b_x,  xhat = sigmoid(z)
  s     = mean_u(h3) w_e + b_e                               (log of the starting eps)
  loss  = mean_u BCE(sigmoid(z_u), y_u) + lam (s - t)^2
"""
import numpy as np
import torch

H = 64
F = 5
LAYERS = 3
ROUND_BF16 = True       # tests of the smooth model switch the roundings off


def param_shapes(hidden=H, layers=LAYERS):
    shapes = [("W_in", (F, hidden)), ("b_in", (hidden,))]
    for l in range(layers):
        shapes += [(f"W{l}", (2 * hidden, hidden)), (f"b{l}", (hidden,))]
    shapes += [("w_x", (hidden,)), ("b_x", (1,)), ("w_e", (hidden,)), ("b_e", (1,))]
    return shapes


def n_params(hidden=H, layers=LAYERS):
    return int(sum(np.prod(s) for _, s in param_shapes(hidden, layers)))


def unflatten(flat, hidden=H, layers=LAYERS):
    out, o = {}, 0
    for name, shp in param_shapes(hidden, layers):
        k = int(np.prod(shp))
        out[name] = flat[o:o + k].reshape(shp)
        o += k
    return out


class _RoundBF16(torch.autograd.Function):
    """bfloat16 round-to-nearest-even in the forward pass, identity backward."""

    @staticmethod
    def forward(ctx, x):
        return x.to(torch.bfloat16).to(x.dtype) if ROUND_BF16 else x.clone()

    @staticmethod
    def backward(ctx, g):
        return g


class _RoundGradBF16(torch.autograd.Function):
    """identity forward; the gradient flowing back is rounded to bfloat16."""

    @staticmethod
    def forward(ctx, x):
        return x.view_as(x)

    @staticmethod
    def backward(ctx, g):
        return g.to(torch.bfloat16).to(g.dtype) if ROUND_BF16 else g


def bf16(x):
    return _RoundBF16.apply(x)


def graph_inputs(g, intensity=None, x_start=None):
    """Non-terminal rows in ascending id: features, the row-normalised
    capacity matrix A (sparse) and the node ids.  intensity and x_start are
    indexed by node id; absent, they are 0 and 1/2."""
    ids = np.array([u for u in range(g.n) if u not in (g.s, g.t)], dtype=np.int64)
    pos = -np.ones(g.n, np.int64)
    pos[ids] = np.arange(ids.shape[0])
    nt = ids.shape[0]
    cs = np.zeros(nt)
    ct = np.zeros(nt)
    wdeg = np.zeros(nt)
    rows, cols, vals = [], [], []
    for a, b, c in zip(g.eu.tolist(), g.ev.tolist(), g.cap.tolist()):
        if a == b:
            continue
        for u, v in ((a, b), (b, a)):
            if u in (g.s, g.t):
                continue
            wdeg[pos[u]] += c
            if v == g.s:
                cs[pos[u]] += c
            elif v == g.t:
                ct[pos[u]] += c
            else:
                rows.append(pos[u]); cols.append(pos[v]); vals.append(c)
    I = np.zeros(nt) if intensity is None else np.asarray(intensity, np.float64)[ids]
    X0 = np.full(nt, 0.5) if x_start is None else np.asarray(x_start, np.float64)[ids]
    feats = np.stack([np.log1p(cs), np.log1p(ct), np.log1p(wdeg), I, X0], axis=1)
    rows = np.asarray(rows, np.int64)
    cols = np.asarray(cols, np.int64)
    vals = np.asarray(vals, np.float64)
    rowsum = np.bincount(rows, weights=vals, minlength=nt)
    A = torch.sparse_coo_tensor(np.stack([rows, cols]), vals / rowsum[rows], (nt, nt)).coalesce()
    return torch.from_numpy(feats), A, ids


def forward(params, feats, A, hidden=H, layers=LAYERS):
    """Returns (logits z [nt], s, h3).  params: dict of float64 tensors."""
    h = torch.relu(feats @ params["W_in"] + params["b_in"])
    h = bf16(h)                                      # stored activations are bfloat16
    for l in range(layers):
        a = torch.sparse.mm(A, h)
        X = bf16(torch.cat([h, a], dim=1))
        Z = _RoundGradBF16.apply(X @ bf16(params[f"W{l}"]) + params[f"b{l}"])
        h = bf16(torch.relu(Z))
    z = h @ params["w_x"] + params["b_x"]
    s = h.mean(dim=0) @ params["w_e"] + params["b_e"]
    return z, s[0] if s.dim() else s, h


def loss_fn(z, s, y, t, lam):
    bce = torch.nn.functional.binary_cross_entropy_with_logits(z, y, reduction="mean")
    return bce + lam * (s - t) ** 2


def loss_and_grad(flat_params, feats, A, y, t, lam=0.1):
    """Loss and its gradient w.r.t. the flat parameter vector (float64)."""
    p = torch.tensor(np.asarray(flat_params, np.float64), requires_grad=True)
    params = unflatten(p)
    z, s, _ = forward(params, feats, A)
    L = loss_fn(z, s, torch.as_tensor(y, dtype=torch.float64), float(t), lam)
    L.backward()
    return float(L.detach()), p.grad.detach().numpy().copy()


def predict(flat_params, feats, A):
    with torch.no_grad():
        params = unflatten(torch.tensor(np.asarray(flat_params, np.float64)))
        z, s, _ = forward(params, feats, A)
    return torch.sigmoid(z).numpy(), float(s)
