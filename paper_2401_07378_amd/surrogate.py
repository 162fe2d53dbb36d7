"""Deep-sets EMD surrogate on the library's kernels: parameter initialisation,
NNS-EMD training labels, the training loop, the candidate index and
surrogate-pruned retrieval.

Every numerical step runs in libnnsemd (binding.sg_*, emd_approx_batched);
this module only draws the initial weights, slices batches and sequences the
calls.  The network and its precision are described in include/nnsemd.h.
"""
from __future__ import annotations

import math

import numpy as np

from . import binding

HIDDEN = binding.SG_HIDDEN


def param_layout(hidden: int = HIDDEN):
    """(name, offset, shape) of the flat FP32 parameter vector."""
    H = hidden
    shapes = [("W1", (H, 3)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)),
              ("W3", (H, 3 * H)), ("b3", (H,)), ("w4", (H,)), ("b4", (1,))]
    out, o = [], 0
    for name, shp in shapes:
        out.append((name, o, shp))
        o += int(np.prod(shp))
    return out, o


def init_params(seed: int, hidden: int = HIDDEN, b4: float = -1.0) -> np.ndarray:
    """He-uniform weights (bound sqrt(6 / fan_in)), zero biases, b4 such that
    softplus(b4) is near a typical EMD of the retrieval clouds."""
    lay, total = param_layout(hidden)
    r = np.random.default_rng(seed)
    th = np.zeros(total, np.float64)
    for name, o, shp in lay:
        n = int(np.prod(shp))
        if name.startswith("W") or name == "w4":
            fan_in = shp[-1] if len(shp) == 2 else shp[0]
            lim = math.sqrt(6.0 / fan_in)
            th[o:o + n] = r.uniform(-lim, lim, n)
    th[[o for name, o, _ in lay if name == "b4"][0]] = b4
    return th.astype(np.float32)


def nnsemd_labels(X, a, set_off, num_pairs: int, max_points: int):
    """NNS-EMD (greedy, L2) of training pairs (set 2b -> set 2b+1), on the
    GPU: returns (labels float32 device tensor, stats numpy records)."""
    import torch
    dev = X.device
    px = torch.arange(num_pairs, dtype=torch.int32, device=dev) * 2
    r = binding.emd_approx_batched(X, a, set_off, X, a, set_off, pair_x=px, pair_y=px + 1, num_pairs=num_pairs,
                                   max_m=max_points, max_n=max_points, metric="l2")
    torch.cuda.synchronize()
    return r["costs"][:num_pairs].to(torch.float32), binding.stats_numpy(r["stats"])[:num_pairs]


class Trainer:
    """Adam on the FP32 master parameters, minibatches of consecutive pairs."""

    def __init__(self, theta_np, device):
        import torch
        self.theta = torch.from_numpy(np.ascontiguousarray(theta_np, np.float32)).to(device)
        self.m = torch.zeros_like(self.theta)
        self.v = torch.zeros_like(self.theta)
        self.grad = torch.empty_like(self.theta)
        self.loss = torch.empty(1, dtype=torch.float32, device=device)
        self.step = 0

    def fit(self, X, a, set_off_np, labels, batch: int, epochs: int, lr: float, lr_end: float | None = None,
            log_every: int = 0, log=None):
        """Train on pairs (2b, 2b+1).  set_off_np: host offsets (2P + 1).
        Cosine learning-rate decay from lr to lr_end over all steps.
        Returns the mean loss of each epoch."""
        import torch
        dev = X.device
        P = len(labels)
        nb = (P + batch - 1) // batch
        offs = []
        for k in range(nb):
            p0, p1 = k * batch, min(P, (k + 1) * batch)
            o = set_off_np[2 * p0:2 * p1 + 1]
            offs.append((int(o[0]), int(o[-1]), torch.from_numpy(o - o[0]).to(dev), p0, p1))
        total = nb * epochs
        lr_end = lr * 0.01 if lr_end is None else lr_end
        hist = []
        for ep in range(epochs):
            acc = torch.zeros(1, dtype=torch.float32, device=dev)
            for k, (x0, x1, off, p0, p1) in enumerate(offs):
                self.step += 1
                frac = (self.step - 1) / max(1, total - 1)
                cur = lr_end + 0.5 * (lr - lr_end) * (1 + math.cos(math.pi * min(1.0, frac)))
                binding.sg_train_step(self.theta, self.m, self.v, self.step, cur, X[x0:x1], a[x0:x1], off,
                                      labels[p0:p1], loss=self.loss, grad=self.grad)
                acc += self.loss
            torch.cuda.synchronize()
            hist.append(float(acc.item()) / nb)
            if log is not None and log_every and (ep + 1) % log_every == 0:
                log(f"epoch {ep + 1}/{epochs}: loss {hist[-1]:.5f}")
        return hist


def build_index(theta, Y, b, y_off):
    """Embeddings (N x 256) of the candidate sets."""
    return binding.sg_embed(theta, Y, b, y_off)


def retrieve(theta, index_E, Xq, aq, Y, b, y_off, max_n: int, keep: int = 1000, top: int = 10, out=None):
    """Surrogate keeps `keep` candidates, NNS-EMD re-ranks them, the best
    `top` are returned (device tensors idx, cost, kept, kept_stats)."""
    return binding.sg_retrieve(theta, index_E, Xq, aq, Y, b, y_off, max_n, keep, top, out=out)
