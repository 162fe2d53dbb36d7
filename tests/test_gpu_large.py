"""Parity of the multi-workgroup path (one pair of any size) and of the
barycentric transport map with the FP64 oracle.

Small and medium pairs are forced onto the multi-workgroup path and compared
in full: plan bit-identical, rounds/work/nnz equal, cost to 1e-12, map
bit-identical to the oracle's map of its own plan.  Every case runs twice:
with the single-workgroup finish (pairs whose active sets both fit it start
there; larger ones hand over once they fit) and with every round grid-wide.  The full 65536 x 65536
colour-transfer pair is compared in full with a stored oracle run (hashes of
the plan and map) and checked on properties that hold at any size.
"""
import numpy as np
import pytest

import oracle
from paper_2401_07378_amd import workloads as W
from tests.gpu_helpers import assert_pair_matches, gpu_pair, gpu_pair_map, oracle_pair

pytestmark = pytest.mark.gpu

CASES = [
    (1, 300, 280, 3, "dirichlet", "l2", "greedy"),
    (2, 500, 700, 2, "uniform", "sqeuclidean", "greedy"),
    (3, 700, 500, 1, "integer", "l1", "greedy"),
    (4, 400, 400, 3, "dirichlet", "l2", "random"),
    (5, 129, 1100, 5, "dirichlet", "l2", "greedy"),
    (6, 1, 50, 3, "dirichlet", "l2", "greedy"),
    (7, 50, 1, 3, "dirichlet", "l2", "greedy"),
    # several compaction blocks per round (the last to finish commits the
    # round), then a single one (it counts its own elements)
    (8, 5000, 4500, 3, "dirichlet", "l2", "greedy"),
    (9, 3000, 3000, 3, "uniform", "sqeuclidean", "greedy"),
    (10, 12000, 9000, 3, "dirichlet", "l2", "greedy"),
    # hand-over to the single-workgroup finish under the random order, L1
    # and at d = 7
    (11, 3000, 2800, 3, "dirichlet", "l2", "random"),
    (12, 2600, 3100, 2, "integer", "l1", "greedy"),
    (13, 2500, 2300, 7, "uniform", "l2", "greedy"),
]


@pytest.mark.parametrize("path", ["multi", "multi_no_tail"])
@pytest.mark.parametrize("case", CASES, ids=lambda c: "-".join(map(str, c[1:])))
def test_multi_path_matches_oracle(case, path):
    seed, m, n, d, masses, metric, protocol = case
    X, a, Y, b = W.random_pair(700 + seed, m, n, d, masses=masses)
    kw = dict(protocol=protocol, seed=99)
    g = gpu_pair(X, a, Y, b, metric, path=path, **kw)
    assert_pair_matches(g, oracle_pair(X, a, Y, b, metric, **kw), label=f"{case} {path}")


@pytest.mark.parametrize("path", ["multi", "multi_no_tail"])
def test_multi_path_map_across_the_hand_over(path):
    """A pair that starts grid-wide and finishes in one workgroup: the map
    (per-supplier sums accumulated in serve order on both sides of the
    hand-over) is bit-identical to the oracle's map of its own plan."""
    X, a, Y, b = W.random_pair(760, 2900, 2900, 3)
    g = gpu_pair_map(X, a, Y, b, "sqeuclidean", path=path)
    ref = oracle_pair(X, a, Y, b, "sqeuclidean")
    assert_pair_matches(g, ref, label=f"map {path}")
    want = oracle.barycentric(ref["src"], ref["dst"], ref["flow"], Y, len(a))
    got = g["map"]
    assert np.array_equal(np.isnan(got), np.isnan(want))
    assert np.array_equal(got[~np.isnan(got)], want[~np.isnan(want)])


@pytest.mark.parametrize("seed", range(3))
def test_multi_path_lattice_ties(seed):
    X, a, Y, b = W.random_pair(720 + seed, 400, 450, 2, masses="integer", lattice=7)
    g = gpu_pair(X, a, Y, b, path="multi")
    assert int(g["stats"]["rescored"]) > 0
    assert_pair_matches(g, oracle_pair(X, a, Y, b), label=f"lattice{seed}")


def test_auto_path_routes_a_large_pair():
    """3000 x 2600 does not fit one workgroup: emd_approx takes the
    multi-workgroup path by itself."""
    X, a, Y, b = W.random_pair(730, 3000, 2600, 3)
    assert_pair_matches(gpu_pair(X, a, Y, b), oracle_pair(X, a, Y, b), label="3000x2600")


@pytest.mark.parametrize("metric", ["l2", "sqeuclidean"])
def test_barycentric_map_bit_identical(metric):
    X, a, Y, b = W.random_pair(740, 350, 420, 3)
    g = gpu_pair_map(X, a, Y, b, metric)
    ref = oracle_pair(X, a, Y, b, metric)
    assert_pair_matches(g, ref, label="map")
    want = oracle.barycentric(ref["src"], ref["dst"], ref["flow"], Y, len(a))
    got = g["map"]
    assert np.array_equal(np.isnan(got), np.isnan(want))
    assert np.array_equal(got[~np.isnan(got)], want[~np.isnan(want)])


def test_barycentric_map_zero_mass_rows_are_nan():
    X, a, Y, b = W.random_pair(741, 60, 70, 3)
    a = a.copy()
    a[[3, 9]] = 0
    a = (a / a.astype(np.float64).sum()).astype(np.float32)
    g = gpu_pair_map(X, a, Y, b)
    assert np.all(np.isnan(g["map"][[3, 9]]))
    assert not np.any(np.isnan(np.delete(g["map"], [3, 9], axis=0)))


@pytest.mark.parametrize("path", ["multi", "multi_no_tail"])
def test_multi_path_status_codes(path):
    X, a, Y, b = W.random_pair(750, 40, 50, 3)
    Xn = X.copy()
    Xn[5, 2] = np.nan
    assert int(gpu_pair(Xn, a, Y, b, path=path)["stats"]["status"]) == -1
    assert int(gpu_pair(X, a * 2, Y, b, path=path)["stats"]["status"]) == -2
    g = gpu_pair(X, a, Y, b, path=path, max_rounds=2)
    assert int(g["stats"]["status"]) == -6
    ref = oracle_pair(X, a, Y, b, max_rounds=2)
    assert ref["status"] == -6
    np.testing.assert_array_equal(g["src"], ref["src"])
    np.testing.assert_array_equal(g["flow"], ref["flow"])


def test_round_cap_inside_the_single_workgroup_finish():
    """The round cap reached after the hand-over: status NOT_CONVERGED, the
    plan so far equal to the oracle's capped run."""
    X, a, Y, b = W.random_pair(751, 2700, 2700, 3)
    full = oracle_pair(X, a, Y, b, with_plan=False)
    cap = full["rounds"] - 3
    g = gpu_pair(X, a, Y, b, path="multi", max_rounds=cap)
    ref = oracle_pair(X, a, Y, b, max_rounds=cap)
    assert ref["status"] == -6 and int(g["stats"]["status"]) == -6
    assert int(g["stats"]["rounds"]) == ref["rounds"] == cap
    np.testing.assert_array_equal(g["src"], ref["src"])
    np.testing.assert_array_equal(g["dst"], ref["dst"])
    np.testing.assert_array_equal(g["flow"], ref["flow"])


@pytest.mark.parametrize("path", ["multi", "multi_no_tail"])
def test_multi_path_empty(path):
    g = gpu_pair(np.zeros((0, 3)), np.zeros(0), np.zeros((0, 3)), np.zeros(0), path=path)
    assert int(g["stats"]["status"]) == 0 and g["cost"] == 0.0


def _sha(arr, dtype):
    import hashlib
    return hashlib.sha256(np.ascontiguousarray(arr, dtype=dtype).tobytes()).hexdigest()


def test_colour_transfer_full_size_against_golden():
    """The whole 65536 x 65536 colour-transfer run with its map, against the
    oracle's full run of the same seeded pair (tests/golden, written by a
    script that calls only the oracle): rounds, work, plan size and near-tie
    counts equal, the plan arrays and the map equal bit for bit (SHA-256),
    the cost equal up to summation order."""
    import json
    import os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "colour_transfer_3d.json")))
    ps = W.colour_transfer_3d()
    assert gold["workload"]["n"] == len(ps.a) and gold["workload"]["seed"] == ps.meta["seed"]
    g = gpu_pair_map(ps.X, ps.a, ps.Y, ps.b, "sqeuclidean")
    st = g["stats"]
    assert int(st["status"]) == 0
    for k in ("rounds", "work", "nnz", "near_ties_nn", "near_ties_order"):
        assert int(st[k]) == gold[k], (k, int(st[k]), gold[k])
    assert float(st["residual_src"]) == gold["residual_src"] and float(st["residual_dst"]) == gold["residual_dst"]
    assert abs(g["cost"] - gold["cost"]) <= 1e-12 * gold["cost"]
    assert _sha(g["src"], "<i4") == gold["sha256_src"]
    assert _sha(g["dst"], "<i4") == gold["sha256_dst"]
    assert _sha(g["flow"], "<f8") == gold["sha256_flow"]
    assert _sha(g["map"], "<f8") == gold["sha256_map"]


def test_colour_transfer_full_size_properties():
    """The whole 65536 x 65536 run with its map: uniform dyadic masses make
    the plan a permutation, every point is matched, R is the sum of f * D
    over the plan, and the map sends x_i exactly to its partner y."""
    ps = W.colour_transfer_3d()
    g = gpu_pair_map(ps.X, ps.a, ps.Y, ps.b, "sqeuclidean")
    st = g["stats"]
    n = len(ps.a)
    assert int(st["status"]) == 0
    assert int(st["nnz"]) == n
    assert float(st["residual_src"]) == 0.0 and float(st["residual_dst"]) == 0.0
    assert np.array_equal(np.sort(g["src"]), np.arange(n)) and np.array_equal(np.sort(g["dst"]), np.arange(n))
    assert np.all(g["flow"] == 2.0 ** -16)
    X64, Y64 = ps.X.astype(np.float64), ps.Y.astype(np.float64)
    d2 = ((X64[g["src"]] - Y64[g["dst"]]) ** 2).sum(1)
    assert g["cost"] == pytest.approx(float((g["flow"] * d2).sum()), rel=1e-12)
    np.testing.assert_array_equal(g["map"][g["src"]], Y64[g["dst"]])
    assert int(st["rounds"]) > 100 and int(st["work"]) > 10 * n * n


def test_workspaces_survive_schedule_growth():
    """Growing the batched schedule buffer must leave the multi-workgroup
    workspace alone: large pair, a bigger batch than any before, large pair."""
    from tests.gpu_helpers import gpu_batched
    X, a, Y, b = W.random_pair(760, 300, 280, 3)
    ref = oracle_pair(X, a, Y, b)
    assert_pair_matches(gpu_pair(X, a, Y, b, path="multi"), ref, label="before")
    ps = W.batched_hist_3d(num_pairs=9000, lo=2, hi=6, seed=761)
    g = gpu_batched(ps)
    assert np.all(g["stats"]["status"] == 0)
    assert_pair_matches(gpu_pair(X, a, Y, b, path="multi"), ref, label="after")


@pytest.mark.parametrize("d", [6, 7])
def test_multi_path_high_dims_ties_and_offset(d):
    """The multi-workgroup path at the top of its range of d: lattice ties,
    a large common offset (2^-14 grid collisions), and a box whose centre
    makes x - centre round."""
    X, a, Y, b = W.random_pair(770 + d, 900, 800, d, masses="integer", lattice=3)
    ref = oracle_pair(X, a, Y, b)
    assert ref["near_ties_nn"] > 0
    assert_pair_matches(gpu_pair(X, a, Y, b, path="multi"), ref, label=f"lattice-d{d}")
    X, a, Y, b = W.random_pair(780 + d, 700, 650, d)
    Xo = (X.astype(np.float64) + 1000.0).astype(np.float32)
    Yo = (Y.astype(np.float64) + 1000.0).astype(np.float32)
    for metric in ("l2", "l1"):
        assert_pair_matches(gpu_pair(Xo, a, Yo, b, metric, path="multi"), oracle_pair(Xo, a, Yo, b, metric),
                            label=f"offset-d{d}-{metric}")
    Xc = X.copy()
    Xc[5] = 1000.0
    assert_pair_matches(gpu_pair(Xc, a, Y, b, "sqeuclidean", path="multi"),
                        oracle_pair(Xc, a, Y, b, "sqeuclidean"), label=f"centre-d{d}")
