"""FP64 CPU twin of the deep-sets EMD surrogate -- test infrastructure only.

Only the test-suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module; the GPU library never does.

The surrogate is not part of the paper (which treats NNS-EMD as a
non-differentiable procedure); it is a learned pre-filter for retrieval whose
candidates NNS-EMD then re-ranks.  Its definition:

  phi(x)   = relu(W2 relu(W1 x + b1) + b2)                 (per point, 3 -> H -> H)
  E(X, a)  = sum_i a_i phi(x_i)                             (mass-weighted pooling)
  z        = [E_q, E_c, |E_q - E_c|]                        (3H)
  pred     = softplus(w4 . relu(W3 z + b3) + b4)            (3H -> H -> 1)
  loss     = mean_b (log pred_b - log y_b)^2                (y = NNS-EMD label)

Precision of the GPU path (mirrored here when ``rounding=True``): every
weight matrix and w4 is used rounded to BF16 (FP32 master copies are what the
optimiser updates, with the gradient of the rounded weight applied to the
master one); the operands of the matrix-core products -- the layer-1
activations H1, the pair features Z, and the back-propagated dPRE2 and dG --
are rounded to BF16; everything else is FP32 on the GPU and FP64 here.  With
``rounding=False`` the function is smooth and the finite-difference pins of
the tests apply to it.

Flat parameter layout (float index order): W1 (H x 3), b1 (H), W2 (H x H),
b2 (H), W3 (H x 3H), b3 (H), w4 (H), b4 (1); matrices row-major [out][in].
Training batches: pair b compares set 2b (query side) with set 2b+1.
"""
from __future__ import annotations

import numpy as np

D_IN = 3


def layout(hidden: int = 256):
    H = hidden
    shapes = [("W1", (H, D_IN)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)),
              ("W3", (H, 3 * H)), ("b3", (H,)), ("w4", (H,)), ("b4", (1,))]
    out, o = {}, 0
    for name, shp in shapes:
        n = int(np.prod(shp))
        out[name] = (o, shp)
        o += n
    return out, o


def num_params(hidden: int = 256) -> int:
    return layout(hidden)[1]


def unpack(theta, hidden: int = 256) -> dict:
    lay, total = layout(hidden)
    theta = np.asarray(theta, np.float64)
    assert theta.shape == (total,)
    return {k: theta[o:o + int(np.prod(s))].reshape(s) for k, (o, s) in lay.items()}


def bf16(x):
    """Round to the nearest BF16 value (ties to even), returned as float64.
    The value is first rounded to FP32, as the GPU holds it."""
    f = np.ascontiguousarray(np.asarray(x, np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def _q(x, rounding):
    return bf16(x) if rounding else np.asarray(x, np.float64)


def softplus(t):
    t = np.asarray(t, np.float64)
    return np.where(t > 20.0, t, np.log1p(np.exp(np.minimum(t, 20.0))))


def sigmoid(t):
    t = np.asarray(t, np.float64)
    return 1.0 / (1.0 + np.exp(-t))


def embed(theta, X, a, set_off, hidden: int = 256, rounding: bool = True, keep: bool = False):
    """Pooled embeddings E (num_sets x H) of concatenated point sets."""
    P = unpack(theta, hidden)
    X = np.asarray(X, np.float64).reshape(-1, D_IN)
    a = np.asarray(a, np.float64)
    W1, W2 = _q(P["W1"], rounding), _q(P["W2"], rounding)
    pre1 = X @ W1.T + P["b1"]
    h1 = _q(np.maximum(pre1, 0.0), rounding)
    pre2 = h1 @ W2.T + P["b2"]
    h2 = np.maximum(pre2, 0.0)
    S = len(set_off) - 1
    E = np.zeros((S, hidden))
    for s in range(S):
        lo, hi = set_off[s], set_off[s + 1]
        E[s] = a[lo:hi] @ h2[lo:hi]
    if keep:
        return E, {"X": X, "a": a, "pre1": pre1, "h1": h1, "pre2": pre2, "W1": W1, "W2": W2}
    return E


def head(theta, Eq, Ec, hidden: int = 256, rounding: bool = True, keep: bool = False):
    """pred for pairs of embeddings (rows of Eq, Ec)."""
    P = unpack(theta, hidden)
    Eq, Ec = np.atleast_2d(Eq), np.atleast_2d(Ec)
    Z = _q(np.concatenate([Eq, Ec, np.abs(Eq - Ec)], axis=1), rounding)
    W3, w4 = _q(P["W3"], rounding), _q(P["w4"], rounding)
    pre3 = Z @ W3.T + P["b3"]
    g = np.maximum(pre3, 0.0)
    t = g @ w4 + P["b4"][0]
    pred = softplus(t)
    if keep:
        return pred, {"Z": Z, "pre3": pre3, "g": g, "t": t, "W3": W3, "w4": w4}
    return pred


def predict(theta, X, a, set_off, hidden: int = 256, rounding: bool = True):
    """pred of each training pair (set 2b vs set 2b+1)."""
    E = embed(theta, X, a, set_off, hidden, rounding)
    return head(theta, E[0::2], E[1::2], hidden, rounding)


def loss_and_grad(theta, X, a, set_off, labels, hidden: int = 256, rounding: bool = True):
    """Loss of one training batch and its gradient (flat, master layout)."""
    lay, total = layout(hidden)
    P = unpack(theta, hidden)
    E, ce = embed(theta, X, a, set_off, hidden, rounding, keep=True)
    Eq, Ec = E[0::2], E[1::2]
    pred, ch = head(theta, Eq, Ec, hidden, rounding, keep=True)
    y = np.asarray(labels, np.float64)
    B = len(y)
    r = np.log(pred) - np.log(y)
    loss = float(np.mean(r * r))
    dpred = 2.0 * r / (B * pred)
    dt = dpred * sigmoid(ch["t"])
    grad = {}
    grad["b4"] = np.array([dt.sum()])
    grad["w4"] = dt @ ch["g"]
    dg = np.outer(dt, ch["w4"]) * (ch["pre3"] > 0)
    grad["b3"] = dg.sum(axis=0)
    dgq = _q(dg, rounding)
    grad["W3"] = dgq.T @ ch["Z"]
    dZ = dgq @ ch["W3"]
    H = hidden
    sgn = np.sign(Eq - Ec)
    dE = np.zeros_like(E)
    dE[0::2] = dZ[:, :H] + dZ[:, 2 * H:] * sgn
    dE[1::2] = dZ[:, H:2 * H] - dZ[:, 2 * H:] * sgn
    S = len(set_off) - 1
    setid = np.repeat(np.arange(S), np.diff(set_off))
    dpre2 = ce["a"][:, None] * dE[setid] * (ce["pre2"] > 0)
    grad["b2"] = dpre2.sum(axis=0)
    dp2q = _q(dpre2, rounding)
    grad["W2"] = dp2q.T @ ce["h1"]
    dh1 = dp2q @ ce["W2"]
    dpre1 = dh1 * (ce["pre1"] > 0)
    grad["b1"] = dpre1.sum(axis=0)
    grad["W1"] = dpre1.T @ ce["X"]
    flat = np.zeros(total)
    for k, (o, s) in lay.items():
        flat[o:o + int(np.prod(s))] = np.asarray(grad[k]).reshape(-1)
    return loss, flat


def adam(theta, m, v, grad, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
         eps: float = 1e-8):
    """One Adam update (bias-corrected, step >= 1); returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def topk_smallest(values, k: int) -> np.ndarray:
    """Indices of the k smallest values, ascending by (value, index)."""
    v = np.asarray(values)
    order = np.lexsort((np.arange(len(v)), v))
    return order[:k]
