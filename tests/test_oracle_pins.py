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


# ------------------------------------------------------------ near-tie counters
# A near tie is a gap of at most 1e-6 relative between two distances (second
# - first <= 1e-6 * first), or at most 1e-12 when the first is 0.  Inputs are
# dyadic, so every distance below is exact in FP32 and FP64 and the expected
# counts follow by hand.
def test_near_ties_exact_counts_on_tie_rules_example():
    """E3: c0 is equidistant from s0 and s1 (one NNS near tie); c0 and c1
    both claim s0 at distance 1 (one neighbour near tie in the greedy order);
    round 2 has a single supplier, which counts nothing."""
    ex = {e["name"]: e for e in _golden()["examples"]}["E3_tie_rules"]
    r = oracle.solve(ex["X"], ex["a"], ex["Y"], ex["b"])
    assert r["near_ties_nn"] == 1 and r["near_ties_order"] == 1


@pytest.mark.parametrize("metric,far,want", [
    # L2: distances 1 and 1 + 2^-21 (gap 4.8e-7 <= 1e-6) / 1 + 2^-19 (1.9e-6)
    ("l2", 2 + 2.0 ** -21, 1), ("l2", 2 + 2.0 ** -19, 0),
    # 1 + 2^-20: a distance gap of 9.5e-7 (near) is a squared-key gap of 1.9e-6
    ("l2", 2 + 2.0 ** -20, 1), ("sqeuclidean", 2 + 2.0 ** -20, 0),
    # squared: 1 and (1 + 2^-21)^2 (gap 9.5e-7) / (1 + 2^-19)^2 (gap 3.8e-6)
    ("sqeuclidean", 2 + 2.0 ** -21, 1), ("sqeuclidean", 2 + 2.0 ** -19, 0),
    ("l1", 2 + 2.0 ** -21, 1), ("l1", 2 + 2.0 ** -19, 0),
])
def test_near_tie_nn_relative_rule(metric, far, want):
    """One consumer at 1 between suppliers at 0 and `far` (1-D): it picks
    s0 in round 1 (counted when the second distance is within 1e-6); round 2
    has one supplier left and counts nothing."""
    r = oracle.solve([[0.0], [far]], [0.5, 0.5], [[1.0]], [1.0], metric=metric)
    assert r["status"] == 0 and r["rounds"] == 2
    assert r["near_ties_nn"] == want and r["near_ties_order"] == 0


@pytest.mark.parametrize("metric,far,want", [
    # the consumer sits on s0 (distance 0): absolute rule, gap <= 1e-12
    ("l2", 2.0 ** -41, 1),           # 4.5e-13
    ("l2", 2.0 ** -39, 0),           # 1.8e-12
    ("sqeuclidean", 2.0 ** -39, 1),  # squared: 3.3e-24
    ("l1", 2.0 ** -39, 0),
])
def test_near_tie_nn_absolute_rule_at_zero(metric, far, want):
    r = oracle.solve([[0.0], [far]], [0.5, 0.5], [[0.0]], [1.0], metric=metric)
    assert r["near_ties_nn"] == want


def test_near_tie_order_neighbours_only():
    """Three claimants of one supplier at distances 1, 1 + 2^-21, 1 + 2^-19:
    the first two neighbours are a near tie, the second two are not
    (gap 2^-19 - 2^-21 = 1.4e-6), and the first and last are not neighbours."""
    r = oracle.solve([[0.0]], [1.0], [[1.0], [-(1 + 2.0 ** -21)], [1 + 2.0 ** -19]], [0.25, 0.25, 0.5])
    assert r["rounds"] == 1 and r["near_ties_order"] == 1 and r["near_ties_nn"] == 0
    rr = oracle.solve([[0.0]], [1.0], [[1.0], [-(1 + 2.0 ** -21)], [1 + 2.0 ** -19]], [0.25, 0.25, 0.5],
                      protocol="random", seed=3)
    assert rr["near_ties_order"] == 0  # counted for the greedy order only


# ------------------------------------------------------------ batched driver
@pytest.mark.parametrize("metric,protocol", [("l2", "greedy"), ("sqeuclidean", "random"), ("l1", "greedy")])
def test_solve_batched_matches_per_pair_solve(metric, protocol):
    """Pair tables that reuse sets (one supplier set against many consumer
    sets, repeated pairs, swapped indices): every pair's stats and cost equal
    the single-pair solve of the same two sets."""
    ps = W.batched_hist_3d(12, lo=3, hi=40, seed=2024)
    pair_x = np.array([0, 3, 3, 7, 11, 2, 5, 0, 9, 9], np.int32)
    pair_y = np.array([1, 3, 4, 7, 0, 11, 5, 1, 2, 10], np.int32)
    stats, threads = oracle.solve_batched(ps.X, ps.a, ps.x_off, ps.Y, ps.b, ps.y_off, pair_x=pair_x,
                                          pair_y=pair_y, metric=metric, protocol=protocol, seed=77)
    assert threads >= 1 and len(stats) == len(pair_x)
    for p, (px, py) in enumerate(zip(pair_x, pair_y)):
        xs, xe, ys, ye = ps.x_off[px], ps.x_off[px + 1], ps.y_off[py], ps.y_off[py + 1]
        ref = oracle.solve(ps.X[xs:xe], ps.a[xs:xe], ps.Y[ys:ye], ps.b[ys:ye], metric=metric,
                           protocol=protocol, seed=77, with_plan=False)
        for k in ("status", "rounds", "nnz", "work", "near_ties_nn", "near_ties_order"):
            assert stats[p][k] == ref[k], (p, k)
        assert stats[p]["cost"] == ref["cost"]
        assert stats[p]["residual_src"] == ref["residual_src"]


# ------------------------------------------------------------ given D (Alg. 1 input)
def _squared_keys(X, Y):
    """Squared distances summed in dimension order (no fused multiply-add)."""
    X = np.asarray(X, np.float64)
    Y = np.asarray(Y, np.float64)
    acc = np.zeros((len(X), len(Y)))
    for k in range(X.shape[1]):
        t = X[:, None, k] - Y[None, :, k]
        acc = acc + t * t
    return acc


@pytest.mark.parametrize("ex", _golden()["examples"], ids=lambda e: e["name"])
def test_given_D_hand_examples(ex):
    """The hand-worked runs, fed as their ground-distance matrices."""
    D = ground(ex["X"], ex["Y"], ex["metric"])
    r = oracle.solve_cost(D, ex["a"], ex["b"])
    e = ex["expected"]
    assert r["status"] == 0 and r["rounds"] == e["rounds"] and r["work"] == e["work"]
    assert r["cost"] == pytest.approx(e["cost"], rel=0, abs=1e-15)
    assert _plan(r) == e["plan"]


@pytest.mark.parametrize("seed", range(3))
def test_given_D_equals_points_run_on_the_same_keys(seed):
    """Squared Euclidean: key, order and distance are the same number in both
    forms, so the whole run is identical."""
    X, a, Y, b = W.random_pair(600 + seed, 90, 110, 3, masses=["dirichlet", "integer", "uniform"][seed])
    r1 = oracle.solve(X, a, Y, b, metric="sqeuclidean")
    r2 = oracle.solve_cost(_squared_keys(X, Y), a, b)
    for k in ("status", "rounds", "nnz", "work", "near_ties_nn", "near_ties_order", "cost"):
        assert r1[k] == r2[k], k
    assert _plan(r1) == _plan(r2)


@pytest.mark.parametrize("seed", range(4))
def test_given_D_lower_and_upper_bounds(seed):
    """Any non-negative D (not a metric): R >= LP optimum (Theorem 1's lower
    bound needs only feasibility) and the per-supplier upper bound of the
    same theorem with the optimal plan."""
    rng = np.random.default_rng(700 + seed)
    m, n = int(rng.integers(2, 12)), int(rng.integers(2, 12))
    D = rng.random((m, n)) * rng.integers(1, 4, size=(m, n))
    a = rng.random(m) + 0.1
    b = rng.random(n) + 0.1
    a, b = a / a.sum(), b / b.sum()
    r = oracle.solve_cost(D, a, b)
    assert r["status"] == 0 and np.all(r["flow"] > 0) and r["nnz"] <= m + n - 1
    np.testing.assert_allclose(np.bincount(r["src"], weights=r["flow"], minlength=m), a, atol=1e-12)
    np.testing.assert_allclose(np.bincount(r["dst"], weights=r["flow"], minlength=n), b, atol=1e-12)
    assert r["cost"] == pytest.approx(float((r["flow"] * D[r["src"], r["dst"]]).sum()), rel=1e-13)
    A_eq = np.zeros((m + n, m * n))
    for i in range(m):
        A_eq[i, i * n:(i + 1) * n] = 1.0
    for j in range(n):
        A_eq[m + j, j::n] = 1.0
    from scipy.optimize import linprog
    lp = linprog(D.ravel(), A_eq=A_eq, b_eq=np.concatenate([a, b]), bounds=(0, None), method="highs")
    assert r["cost"] >= lp.fun - 1e-12
    F = lp.x.reshape(m, n)
    bound = 0.0
    for i in np.unique(r["src"]):
        J = np.unique(r["dst"][r["src"] == i])
        bound += D[i, J].max() * float((b[J] - F[i, J]).sum())
    assert r["cost"] - lp.fun <= bound + 1e-12


def test_given_D_special_cases():
    rng = np.random.default_rng(9)
    # m = 1: one round, R = sum_j b_j D_0j
    D = rng.random((1, 7))
    b = rng.random(7)
    b = b / b.sum()
    r = oracle.solve_cost(D, [1.0], b)
    assert r["rounds"] == 1 and r["cost"] == pytest.approx(float((b * D[0]).sum()), rel=1e-14)
    # n = 1: suppliers served nearest first, one per round
    D = rng.random((6, 1))
    a = np.full(6, 1 / 6)
    r = oracle.solve_cost(D, a, [1.0])
    assert r["rounds"] == 6 and list(r["src"]) == list(np.argsort(D[:, 0], kind="stable"))
    # zero on a permutation, uniform masses: the permutation, cost 0, 1 round
    perm = rng.permutation(8)
    D = rng.random((8, 8)) + 0.5
    D[np.arange(8), perm] = 0.0
    r = oracle.solve_cost(D, np.full(8, 0.125), np.full(8, 0.125))
    assert r["cost"] == 0.0 and r["rounds"] == 1 and np.array_equal(perm[r["src"]], r["dst"])
    # invalid entries
    D[0, 0] = -1.0
    assert oracle.solve_cost(D, np.full(8, 0.125), np.full(8, 0.125))["status_name"] == "INVALID_ARG"
    D[0, 0] = np.inf
    assert oracle.solve_cost(D, np.full(8, 0.125), np.full(8, 0.125))["status_name"] == "INVALID_ARG"


# ------------------------------------------------------------ per-consumer map
def test_barycentric_dst_hand_values():
    """E1's plan: c1 receives .25 from s0 = (0,0) and .125 from s1 = (1,0),
    so T(c1) = (1/3, 0); c0 <- s0 only, c2 <- s1 only."""
    ex = {e["name"]: e for e in _golden()["examples"]}["E1_partial_serve_carry_over"]
    r = oracle.solve(ex["X"], ex["a"], ex["Y"], ex["b"])
    T = oracle.barycentric_dst(r["src"], r["dst"], r["flow"], ex["X"], 3)
    np.testing.assert_allclose(T, [[0, 0], [1 / 3, 0], [1, 0]], rtol=0, atol=1e-16)


def test_barycentric_dst_permutation_and_empty_rows():
    ps = W.single_pair_2d(64)
    r = oracle.solve(ps.X, ps.a, ps.Y, ps.b)
    T = oracle.barycentric_dst(r["src"], r["dst"], r["flow"], ps.X, 64)
    np.testing.assert_array_equal(T[r["dst"]], ps.X[r["src"]].astype(np.float64))
    X, a, Y, b = W.random_pair(15, 30, 40, 3)
    b = b.copy()
    b[[4, 17]] = 0
    b = (b / b.astype(np.float64).sum()).astype(np.float32)
    r = oracle.solve(X, a, Y, b)
    T = oracle.barycentric_dst(r["src"], r["dst"], r["flow"], X, 40)
    assert np.all(np.isnan(T[[4, 17]])) and not np.any(np.isnan(np.delete(T, [4, 17], axis=0)))


# ------------------------------------------------------------ colour transfer
def _gray(vals):
    return np.repeat(np.asarray(vals, np.uint8)[:, None], 3, axis=1)


def test_kmeans_hand_worked_lloyd():
    """Gray pixels 0, 2, 10, 12 with K = 2: the start takes pixels 0 and 2
    (colours 0 and 10); both iterations assign {0, 2} and {10, 12}, so the
    centroids become 1 and 11 with two pixels each."""
    C, n, asg = oracle.kmeans(_gray([0, 2, 10, 12]), 2, 3)
    np.testing.assert_array_equal(C, [[1, 1, 1], [11, 11, 11]])
    np.testing.assert_array_equal(n, [2, 2])
    np.testing.assert_array_equal(asg, [0, 0, 1, 1])


def test_kmeans_ties_and_empty_clusters():
    """Pixel 5 is equidistant from centroids 0 and 10: it joins cluster 0.
    A start with two equal colours leaves the second cluster empty; it keeps
    its centroid and count 0."""
    C, n, asg = oracle.kmeans(_gray([0, 10, 5]), 2, 0)
    np.testing.assert_array_equal(asg, [0, 1, 0])
    C, n, asg = oracle.kmeans(_gray([7, 7, 7, 7, 9, 9]), 3, 2)
    assert list(n) == [4, 0, 2]
    np.testing.assert_array_equal(C[1], [7, 7, 7])


def test_kmeans_block_image_recovers_colours():
    rng = np.random.default_rng(3)
    cols = rng.integers(0, 256, size=(8, 3)).astype(np.uint8)
    img = np.repeat(cols, 50, axis=0)  # eight blocks of 50 pixels
    C, n, asg = oracle.kmeans(img, 8, 5)
    np.testing.assert_array_equal(C, cols.astype(np.float64))
    np.testing.assert_array_equal(n, np.full(8, 50))
    np.testing.assert_array_equal(asg, np.repeat(np.arange(8), 50))


def test_recolour_rounding_and_nan_rows():
    px = np.array([[10, 20, 30], [40, 50, 60]], np.uint8)
    T = np.array([[0.5, 1.0 / 255.0, np.nan], [2.0, -0.25, 0.0]])
    out = oracle.recolour(px, np.array([0, 1], np.int32), T)
    np.testing.assert_array_equal(out, [[128, 1, 30], [255, 0, 0]])  # 127.5 -> 128 (half to even)


def test_colour_transfer_onto_itself_quantises():
    """Reference = source: the palettes are equal, NNS-EMD is 0 in one round
    (Theorem 2, identical sets) and the map sends every bin to its own colour,
    so each pixel becomes its rounded centroid."""
    img = W.colour_image(5, 48, 40).reshape(-1, 3)
    out = oracle.colour_transfer(img, img, 16, 16, 4)
    assert out["solve"]["cost"] == 0.0 and out["solve"]["rounds"] == 1
    C, _, asg = oracle.kmeans(img, 16, 4)
    want = np.clip(np.rint(255.0 * (C / 255.0).astype(np.float32).astype(np.float64)), 0, 255).astype(np.uint8)[asg]
    np.testing.assert_array_equal(out["image"], want)
