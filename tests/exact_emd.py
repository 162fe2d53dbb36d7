"""Exact EMD references used to pin the oracle (test helpers).

These solve the transport LP of the paper's Eqs. (1)-(3) with library
solvers; they share nothing with the oracle.
"""
import numpy as np
from scipy.optimize import linear_sum_assignment, linprog
from scipy.stats import wasserstein_distance


def ground(X, Y, metric):
    X = np.asarray(X, np.float64)
    Y = np.asarray(Y, np.float64)
    diff = X[:, None, :] - Y[None, :, :]
    if metric == "l1":
        return np.abs(diff).sum(-1)
    sq = (diff ** 2).sum(-1)
    return np.sqrt(sq) if metric == "l2" else sq


def exact_lp(X, a, Y, b, metric="l2"):
    """min sum F_ij D_ij  s.t. row sums a, column sums b, F >= 0 (HiGHS).
    Masses are rescaled to a common total first (FP32 rounding)."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    b = b * (a.sum() / b.sum())
    D = ground(X, Y, metric)
    m, n = D.shape
    A_eq = np.zeros((m + n, m * n))
    for i in range(m):
        A_eq[i, i * n:(i + 1) * n] = 1.0
    for j in range(n):
        A_eq[m + j, j::n] = 1.0
    res = linprog(D.ravel(), A_eq=A_eq, b_eq=np.concatenate([a, b]), bounds=(0, None),
                  method="highs")
    assert res.status == 0, res.message
    return float(res.fun), res.x.reshape(m, n)


def exact_assignment(X, Y, metric="l2"):
    """Uniform masses 1/n on both sides with n = m: the optimum is a permutation."""
    D = ground(X, Y, metric)
    r, c = linear_sum_assignment(D)
    return float(D[r, c].sum() / D.shape[0])


def exact_1d(x, a, y, b):
    """W1 on the line (CDF formula) for |x - y| ground cost."""
    return float(wasserstein_distance(np.ravel(x), np.ravel(y), a, b))
