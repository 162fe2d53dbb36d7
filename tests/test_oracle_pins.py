"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these re-types the oracle's own loop: they check hand-derived runs of
Algorithm 1 (tests/golden), exact transport optima from library LP /
assignment / 1-D solvers (Theorem 1: R >= EMD), the Theorem 1 upper bound,
the exact special cases of Theorem 2, the feasibility of Lemma 1 and
structural invariants, and the published SplitMix64 vectors behind the random
protocol.
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2401_07378_amd import workloads as W
from tests.exact_emd import exact_1d, exact_assignment, exact_lp, ground

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_examples.json")


def _golden():
    with open(GOLDEN) as f:
        return json.load(f)


def _plan(r):
    return [[int(i), int(j), float(f)] for i, j, f in zip(r["src"], r["dst"], r["flow"])]


def check_invariants(r, X, a, Y, b, metric):
    """Lemma 1 feasibility, positivity, sparsity and cost bookkeeping."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    m, n = len(a), len(b)
    assert r["status"] == 0
    src, dst, flow = r["src"], r["dst"], r["flow"]
    assert np.all(flow > 0)
    assert np.all((src >= 0) & (src < m)) and np.all((dst >= 0) & (dst < n))
    assert r["nnz"] <= max(m + n - 1, 0)
    assert r["rounds"] <= max(m + n - 1, 0)
    rows = np.bincount(src, weights=flow, minlength=m)
    cols = np.bincount(dst, weights=flow, minlength=n)
    assert np.all(rows <= a + 1e-12) and np.all(cols <= b + 1e-12)
    # Mass left over sits on one side only, and equals what was not shipped.
    assert min(r["residual_src"], r["residual_dst"]) <= 1e-15
    assert abs((a.sum() - rows.sum()) - r["residual_src"]) <= 1e-12
    assert abs((b.sum() - cols.sum()) - r["residual_dst"]) <= 1e-12
    if r["residual_src"] == 0.0:
        np.testing.assert_allclose(rows, a, rtol=0, atol=1e-12)
    if r["residual_dst"] == 0.0:
        np.testing.assert_allclose(cols, b, rtol=0, atol=1e-12)
    D = ground(X, Y, metric)
    cost = float((flow * D[src, dst]).sum()) if len(flow) else 0.0
    assert abs(cost - r["cost"]) <= 1e-12 * max(1.0, abs(cost))


# ---------------------------------------------------------------- golden runs
@pytest.mark.parametrize("ex", _golden()["examples"], ids=lambda e: e["name"])
def test_hand_examples(ex):
    r = oracle.solve(ex["X"], ex["a"], ex["Y"], ex["b"], metric=ex["metric"])
    e = ex["expected"]
    assert r["status"] == 0
    assert r["cost"] == pytest.approx(e["cost"], rel=0, abs=1e-15)
    assert r["rounds"] == e["rounds"]
    assert r["nnz"] == e["nnz"]
    assert r["work"] == e["work"]
    assert _plan(r) == e["plan"]
    check_invariants(r, ex["X"], ex["a"], ex["Y"], ex["b"], ex["metric"])


@pytest.mark.parametrize("ex", _golden()["examples"], ids=lambda e: e["name"])
def test_hand_examples_exact_emd(ex):
    opt, _ = exact_lp(ex["X"], ex["a"], ex["Y"], ex["b"], ex["metric"])
    assert opt == pytest.approx(ex["exact_emd"], abs=1e-9)
    assert ex["expected"]["cost"] >= opt - 1e-12


def test_roles_are_asymmetric():
    ex = {e["name"]: e for e in _golden()["examples"]}["E5_roles_not_symmetric"]
    r = oracle.solve(ex["Y"], ex["b"], ex["X"], ex["a"])
    assert r["cost"] == pytest.approx(ex["swapped_cost"], abs=1e-15)


def test_near_ties_are_counted():
    ex = {e["name"]: e for e in _golden()["examples"]}["E3_tie_rules"]
    r = oracle.solve(ex["X"], ex["a"], ex["Y"], ex["b"])
    assert r["near_ties_nn"] >= 1 and r["near_ties_order"] >= 1


def test_splitmix_published_vectors():
    want = [int(h, 16) for h in _golden()["splitmix64_state0_outputs"]["hex"]]
    assert [oracle.rp_key(0, 0, j) for j in range(4)] == want


# ------------------------------------------------------ Theorem 1 lower bound
CASES = [(s, m, n, d, mass, metric)
         for s, (m, n, d, mass, metric) in enumerate(
             [(m, n, d, mass, metric)
              for (m, n) in [(1, 4), (4, 1), (3, 5), (7, 7), (9, 6), (12, 10)]
              for d in (1, 2, 3)
              for mass in ("dirichlet", "integer", "uniform")
              for metric in ("l2", "sqeuclidean", "l1")])]


@pytest.mark.parametrize("case", CASES[::3], ids=lambda c: "-".join(map(str, c)))
def test_lower_bound_and_invariants_lp(case):
    seed, m, n, d, mass, metric = case
    X, a, Y, b = W.random_pair(seed, m, n, d, masses=mass)
    r = oracle.solve(X, a, Y, b, metric=metric)
    check_invariants(r, X, a, Y, b, metric)
    opt, Fopt = exact_lp(X, a, Y, b, metric)
    slack = mass_slack(X, a, Y, b, metric)
    assert r["cost"] >= opt - slack
    # Theorem 1 upper bound with the optimal plan.
    assert r["cost"] - opt <= theorem1_bound(r, X, Y, b, Fopt, metric) + slack


def mass_slack(X, a, Y, b, metric):
    """The LP ships the same total on both sides; the oracle ships the smaller
    FP32-rounded total.  Costs may differ by at most Dmax * |sum a - sum b|."""
    gap = abs(np.asarray(a, np.float64).sum() - np.asarray(b, np.float64).sum())
    return 2.0 * float(ground(X, Y, metric).max(initial=0.0)) * gap + 1e-12


def theorem1_bound(r, X, Y, b, F, metric):
    """sum_i D_{i,j*_i} sum_{j in J_i} (c_j - F_ij), J_i = consumers served by
    supplier i in the NNS-EMD plan, j*_i the farthest of them."""
    D = ground(X, Y, metric)
    b = np.asarray(b, np.float64)
    total = 0.0
    for i in np.unique(r["src"]):
        J = np.unique(r["dst"][r["src"] == i])
        jstar = J[np.argmax(D[i, J])]
        total += D[i, jstar] * float((b[J] - F[i, J]).sum())
    return total


@pytest.mark.parametrize("seed", range(4))
def test_theorem1_upper_bound_product_coupling(seed):
    """The per-supplier bound holds for any feasible F; use F = a b^T."""
    X, a, Y, b = W.random_pair(100 + seed, 150, 220, 3)
    r = oracle.solve(X, a, Y, b)
    a64, b64 = a.astype(np.float64), b.astype(np.float64)
    F = np.outer(a64, b64) / a64.sum()
    D = ground(X, Y, "l2")
    assert r["cost"] - float((F * D).sum()) <= theorem1_bound(r, X, Y, b, F, "l2") + 1e-12


def test_lower_bound_assignment_full_size_single_pair():
    """The 256 x 256 uniform 2-D pair: exact EMD is an assignment problem."""
    ps = W.single_pair_2d()
    r = oracle.solve(ps.X, ps.a, ps.Y, ps.b)
    check_invariants(r, ps.X, ps.a, ps.Y, ps.b, "l2")
    opt = exact_assignment(ps.X, ps.Y)
    assert opt <= r["cost"] <= 1.5 * opt
    # uniform dyadic masses => every serve empties both ends: a permutation
    assert r["nnz"] == 256
    assert sorted(r["src"]) == list(range(256)) and sorted(r["dst"]) == list(range(256))
    assert np.all(r["flow"] == 2.0 ** -8)


@pytest.mark.parametrize("seed", range(6))
def test_lower_bound_1d_cdf(seed):
    rng = np.random.default_rng(seed)
    m, n = int(rng.integers(20, 200)), int(rng.integers(20, 200))
    X, a, Y, b = W.random_pair(200 + seed, m, n, 1)
    r = oracle.solve(X, a, Y, b, metric="l2")
    check_invariants(r, X, a, Y, b, "l2")
    b_scaled = b.astype(np.float64) * (a.astype(np.float64).sum() / b.astype(np.float64).sum())
    assert r["cost"] >= exact_1d(X, a.astype(np.float64), Y, b_scaled) - mass_slack(X, a, Y, b, "l2")


# ------------------------------------------------- Theorem 2 exact special cases
@pytest.mark.parametrize("metric", ["l2", "sqeuclidean", "l1"])
def test_single_supplier_is_exact(metric):
    _, _, Y, b = W.random_pair(7, 1, 40, 3)
    X = np.array([[0.3, 0.6, 0.2]], np.float32)
    a = np.array([b.astype(np.float64).sum()])
    r = oracle.solve(X, a, Y, b, metric=metric)
    want = float((b.astype(np.float64) * ground(X, Y, metric)[0]).sum())
    assert r["rounds"] == 1
    assert r["cost"] == pytest.approx(want, rel=1e-13)


@pytest.mark.parametrize("metric", ["l2", "sqeuclidean", "l1"])
def test_single_consumer_takes_m_rounds_and_is_exact(metric):
    X, a, _, _ = W.random_pair(8, 30, 1, 2)
    Y = np.array([[0.5, 0.5]], np.float32)
    b = np.array([a.astype(np.float64).sum()])
    r = oracle.solve(X, a, Y, b, metric=metric)
    D = ground(X, Y, metric)[:, 0]
    assert r["rounds"] == 30
    # nearest supplier first, one per round
    assert list(r["src"]) == list(np.argsort(D, kind="stable"))
    assert r["cost"] == pytest.approx(float((a.astype(np.float64) * D).sum()), rel=1e-13)


@pytest.mark.parametrize("metric", ["l2", "sqeuclidean"])
def test_translated_copy_is_exact(metric):
    """Y = X + delta with b = a and |delta| under half the minimum spacing:
    each y_i's nearest supplier is x_i, one round, and the identity coupling
    is optimal (W1 of a translate is |delta|)."""
    g = np.arange(12, dtype=np.float64)
    X = np.stack(np.meshgrid(g, g), -1).reshape(-1, 2).astype(np.float32)  # spacing 1
    rng = np.random.default_rng(3)
    w = rng.random(len(X)) + 0.1
    a = (w / w.sum()).astype(np.float32)
    delta = np.array([0.125, -0.25])  # exact in FP32, |delta| < 0.5
    Y = (X.astype(np.float64) + delta).astype(np.float32)
    r = oracle.solve(X, a, Y, a, metric=metric)
    assert r["rounds"] == 1
    assert list(r["src"]) == list(range(len(X))) and list(r["dst"]) == list(range(len(X)))
    norm = float(np.sqrt((delta ** 2).sum()))
    want = norm if metric == "l2" else norm ** 2
    assert r["cost"] == pytest.approx(want * a.astype(np.float64).sum(), rel=1e-12)


def test_identical_sets_cost_zero():
    X, a, _, _ = W.random_pair(9, 64, 1, 3)
    r = oracle.solve(X, a, X, a)
    assert r["cost"] == 0.0 and r["rounds"] == 1
    assert list(r["src"]) == list(range(64)) and list(r["dst"]) == list(range(64))


# ------------------------------------------------------------ invariants
@pytest.mark.parametrize("seed", range(8))
@pytest.mark.parametrize("metric", ["l2", "sqeuclidean", "l1"])
def test_invariants_random(seed, metric):
    rng = np.random.default_rng(1000 + seed)
    m, n, d = int(rng.integers(1, 300)), int(rng.integers(1, 300)), int(rng.integers(1, 5))
    X, a, Y, b = W.random_pair(300 + seed, m, n, d, masses=["dirichlet", "integer"][seed % 2])
    r = oracle.solve(X, a, Y, b, metric=metric)
    check_invariants(r, X, a, Y, b, metric)


@pytest.mark.parametrize("seed", range(4))
def test_lattice_ties_lower_bound(seed):
    X, a, Y, b = W.random_pair(400 + seed, 10, 12, 2, masses="integer", lattice=4)
    r = oracle.solve(X, a, Y, b)
    check_invariants(r, X, a, Y, b, "l2")
    assert r["cost"] >= exact_lp(X, a, Y, b)[0] - mass_slack(X, a, Y, b, "l2")


def test_zero_mass_points_start_inactive():
    X, a, Y, b = W.random_pair(11, 20, 25, 2)
    a = a.copy()
    b = b.copy()
    a[[0, 5]] = 0
    b[[3]] = 0
    a = (a / a.astype(np.float64).sum()).astype(np.float32)
    b = (b / b.astype(np.float64).sum()).astype(np.float32)
    r = oracle.solve(X, a, Y, b)
    check_invariants(r, X, a, Y, b, "l2")
    assert 0 not in r["src"] and 5 not in r["src"] and 3 not in r["dst"]


def test_determinism():
    X, a, Y, b = W.random_pair(12, 200, 180, 3)
    r1 = oracle.solve(X, a, Y, b)
    r2 = oracle.solve(X, a, Y, b)
    assert r1["cost"] == r2["cost"] and _plan(r1) == _plan(r2)


def test_empty_sides():
    r = oracle.solve(np.zeros((0, 2)), np.zeros(0), np.zeros((0, 2)), np.zeros(0))
    assert r["status"] == 0 and r["cost"] == 0 and r["rounds"] == 0 and r["nnz"] == 0


def test_status_codes():
    X, a, Y, b = W.random_pair(13, 5, 6, 2)
    Xn = X.copy()
    Xn[1, 0] = np.nan
    assert oracle.solve(Xn, a, Y, b)["status_name"] == "INVALID_ARG"
    an = a.copy()
    an[0] = -an[0]
    assert oracle.solve(X, an, Y, b)["status_name"] == "INVALID_ARG"
    assert oracle.solve(X, a * 2, Y, b)["status_name"] == "MASS_MISMATCH"
    assert oracle.solve(X, a, Y, b, plan_capacity=9)["status_name"] == "CAPACITY"
    assert oracle.solve(X, a, Y, b, max_rounds=1)["status_name"] == "NOT_CONVERGED"


# ------------------------------------------------------------ random protocol
def test_random_protocol_hand_run():
    """s0 = (0,0) holds .5, s1 = (10,0) holds .5; four consumers of .25 at
    x = 1..4 all pick s0 in round 0.  With seed 0 their order keys are
    SplitMix64 outputs 1..4 (see the golden vectors): ascending order is
    j2, j1, j0, j3, so s0 serves j2 (d 3) and j1 (d 2); round 1 sends j0
    (d 9) and j3 (d 6) to s1.  R = .75 + .5 + 2.25 + 1.5 = 5.0 (the greedy
    protocol gives 4.0)."""
    X = [[0, 0], [10, 0]]
    Y = [[1, 0], [2, 0], [3, 0], [4, 0]]
    a, b = [0.5, 0.5], [0.25] * 4
    r = oracle.solve(X, a, Y, b, protocol="random", seed=0)
    assert r["cost"] == 5.0 and r["rounds"] == 2
    assert _plan(r)[:2] == [[0, 2, 0.25], [0, 1, 0.25]]
    assert oracle.solve(X, a, Y, b)["cost"] == 4.0


@pytest.mark.parametrize("seed", range(3))
def test_random_protocol_invariants(seed):
    X, a, Y, b = W.random_pair(500 + seed, 9, 11, 2)
    r = oracle.solve(X, a, Y, b, protocol="random", seed=seed)
    check_invariants(r, X, a, Y, b, "l2")
    assert r["cost"] >= exact_lp(X, a, Y, b)[0] - mass_slack(X, a, Y, b, "l2")


# ------------------------------------------------------------ barycentric map
def test_barycentric_map():
    X, a, Y, b = W.random_pair(14, 40, 60, 3)
    r = oracle.solve(X, a, Y, b)
    T = oracle.barycentric(r["src"], r["dst"], r["flow"], Y, 40)
    rows = np.bincount(r["src"], weights=r["flow"], minlength=40)
    cols = np.bincount(r["dst"], weights=r["flow"], minlength=60)
    # mass-weighted mean is preserved: sum_i w_i T_i = sum_j w_j y_j
    np.testing.assert_allclose((rows[:, None] * T).sum(0), (cols[:, None] * Y).sum(0), atol=1e-12)
    # each T_i lies in the bounding box of the consumers it serves
    for i in range(40):
        ys = Y[r["dst"][r["src"] == i]].astype(np.float64)
        assert np.all(T[i] >= ys.min(0) - 1e-12) and np.all(T[i] <= ys.max(0) + 1e-12)
    # a permutation plan maps x_i to its partner exactly
    ps = W.single_pair_2d(64)
    r = oracle.solve(ps.X, ps.a, ps.Y, ps.b)
    T = oracle.barycentric(r["src"], r["dst"], r["flow"], ps.Y, 64)
    np.testing.assert_array_equal(T[r["src"]], ps.Y[r["dst"]].astype(np.float64))
