"""Parity of the given-D path (emd_approx_cost, emd_approx_cost_batched):
Algorithm 1 on a caller's ground-distance matrix (FP32 or FP64) against the
oracle's given-D form.  The entries are compared exactly on both sides, so
plans, rounds, work and near-tie counts must be identical and the cost equal
up to summation order."""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2401_07378_amd import workloads as W
from tests.exact_emd import ground
from tests.gpu_helpers import _collect, assert_pair_matches, to_dev

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_examples.json")


def gpu_cost(D, a, b, plan=True, **kw):
    import torch
    from paper_2401_07378_amd import binding
    r = binding.emd_approx_cost(to_dev(D), to_dev(np.asarray(a, np.float32)), to_dev(np.asarray(b, np.float32)),
                                plan=plan, **kw)
    torch.cuda.synchronize()
    return _collect(r, plan)


def oracle_cost(D, a, b, **kw):
    return oracle.solve_cost(np.asarray(D, np.float64), np.asarray(a, np.float32), np.asarray(b, np.float32), **kw)


@pytest.mark.parametrize("ex", json.load(open(GOLDEN))["examples"], ids=lambda e: e["name"])
def test_hand_examples_as_matrices(ex):
    D = ground(ex["X"], ex["Y"], ex["metric"])
    g = gpu_cost(D, ex["a"], ex["b"])
    e = ex["expected"]
    assert g["cost"] == pytest.approx(e["cost"], rel=1e-15)
    assert int(g["stats"]["rounds"]) == e["rounds"] and int(g["stats"]["work"]) == e["work"]
    assert [[int(i), int(j), float(f)] for i, j, f in zip(g["src"], g["dst"], g["flow"])] == e["plan"]


CASES = [(s, dt, proto) for s in range(5) for dt in ("f32", "f64") for proto in ("greedy", "random")]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "s%d-%s-%s" % c)
def test_random_matrices(case):
    seed, dt, protocol = case
    rng = np.random.default_rng(900 + seed)
    m, n = int(rng.integers(1, 900)), int(rng.integers(1, 900))
    masses = ["dirichlet", "integer", "uniform"][seed % 3]
    X, a, Y, b = W.random_pair(910 + seed, m, n, 3, masses=masses)
    D = ground(X, Y, ["l2", "sqeuclidean", "l1"][seed % 3])
    if seed == 4:
        D = rng.integers(0, 5, size=(m, n)).astype(np.float64)  # a non-metric D full of exact ties
    D = D.astype(np.float32) if dt == "f32" else D
    kw = dict(protocol=protocol, seed=31)
    assert_pair_matches(gpu_cost(D, a, b, **kw), oracle_cost(D, a, b, **kw), label=str(case))


def test_single_pair_2d_full_size_as_matrix():
    """The 256 x 256 single-pair workload, its L2 distances given as D (FP64)."""
    ps = W.single_pair_2d()
    D = ground(ps.X, ps.Y, "l2")
    g = gpu_cost(D, ps.a, ps.b)
    assert_pair_matches(g, oracle_cost(D, ps.a, ps.b), label="256x256")
    assert int(g["stats"]["nnz"]) == 256


def test_maximum_size_matrix():
    """4096 x 4096 FP32 entries (64 MB), the largest pair of the path."""
    rng = np.random.default_rng(920)
    D = W.to_f32(rng.random((4096, 4096)))
    a, b = W.dirichlet_masses(rng, 4096), W.dirichlet_masses(rng, 4096)
    assert_pair_matches(gpu_cost(D, a, b), oracle_cost(D, a, b), label="4096x4096")


def test_batched_matrices_with_plans():
    """64 pairs shaped like the batched histogram workload (sizes 128..1024,
    Dirichlet masses), their L2 distance matrices back to back in FP32; one
    pair carries a negative entry and fails alone."""
    import torch
    from paper_2401_07378_amd import binding
    ps = W.batched_hist_3d(64, seed=930)
    m, n = ps.sizes()
    mats = [W.to_f32(ground(ps.pair(p)[0], ps.pair(p)[2], "l2")).ravel() for p in range(64)]
    mats[17] = mats[17].copy()
    mats[17][5] = -1.0
    d_off = np.zeros(65, np.int64)
    d_off[1:] = np.cumsum([len(x) for x in mats])
    poff = binding.plan_offsets(m, n)
    r = binding.emd_approx_cost_batched(to_dev(np.concatenate(mats)), to_dev(d_off), to_dev(ps.a), to_dev(ps.x_off),
                                        to_dev(ps.b), to_dev(ps.y_off), max_m=int(m.max()), max_n=int(n.max()),
                                        plan_off=to_dev(poff))
    torch.cuda.synchronize()
    st = binding.stats_numpy(r["stats"])[:64]
    costs = r["costs"].cpu().numpy()
    src, dst, flow = (r[k].cpu().numpy() for k in ("plan_src", "plan_dst", "plan_flow"))
    assert int(st[17]["status"]) == -1 and np.isnan(costs[17])
    for p in range(64):
        if p == 17:
            continue
        _, a, _, b = ps.pair(p)
        ref = oracle_cost(mats[p].reshape(m[p], n[p]), a, b)
        k = int(st[p]["nnz"])
        g = {"cost": float(costs[p]), "stats": st[p], "src": src[poff[p]:poff[p] + k],
             "dst": dst[poff[p]:poff[p] + k], "flow": flow[poff[p]:poff[p] + k]}
        assert_pair_matches(g, ref, label=f"pair{p}")


def test_status_codes():
    rng = np.random.default_rng(940)
    D = rng.random((20, 30))
    a, b = W.dirichlet_masses(rng, 20), W.dirichlet_masses(rng, 30)
    Dn = D.copy()
    Dn[3, 4] = np.inf
    assert int(gpu_cost(Dn, a, b)["stats"]["status"]) == -1
    Dn[3, 4] = -0.5
    assert int(gpu_cost(Dn, a, b)["stats"]["status"]) == -1
    assert int(gpu_cost(D, a * 2, b)["stats"]["status"]) == -2
    g = gpu_cost(D, a, b, max_rounds=2)
    ref = oracle_cost(D, a, b, max_rounds=2)
    assert int(g["stats"]["status"]) == -6 and ref["status"] == -6
    np.testing.assert_array_equal(g["src"], ref["src"])
    np.testing.assert_array_equal(g["flow"], ref["flow"])
    e = gpu_cost(np.zeros((0, 0)), np.zeros(0), np.zeros(0))
    assert int(e["stats"]["status"]) == 0 and e["cost"] == 0.0
