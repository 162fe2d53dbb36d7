"""Parity of the high-dimensional path with the FP64 oracle.

BF16 points run the key tile on the matrix cores (FP32 accumulation); FP32
points with d > 7 run it on the vector ALUs.  Both re-score near ties in FP64,
so the plan must be bit-identical to the oracle's on the same values (the
oracle receives the exact FP32 values of the BF16 numbers).  The cost: the
FP32 vector path recomputes every served distance in FP64 (equal to 1e-12
relative); the BF16 split form takes each served distance from its FP32 key
when the key's error bound makes that term accurate to BF16_COST_REL
relative, else recomputes every distance of the pair exactly, so its cost is
within BF16_COST_REL of the definition's (all terms are positive) -- 100
times inside the 1e-3 allowed for BF16 matrix-core mode.  The full
8192-candidate document workload is checked on sampled pairs against the
oracle and, on every pair, against the FP32 vector path: identical plans and
counts, costs within BF16_COST_REL.
"""
import numpy as np
import pytest

import oracle
from paper_2401_07378_amd import workloads as W
from tests.gpu_helpers import assert_pair_matches, gpu_batched, gpu_pair, gpu_pair_bf16, oracle_pair

pytestmark = pytest.mark.gpu

f32 = W.bf16_bits_to_f32

# Per-term relative bound of the split form's key-based distances (the
# library's tau), plus FP64 summation rounding.
BF16_COST_REL = 1e-5 * (1 + 1e-9) + 1e-13

CASES = [
    # seed, m, n, d, masses, metric, protocol
    (1, 40, 60, 300, "zipf", "l2", "greedy"),
    (2, 500, 500, 300, "zipf", "l2", "greedy"),
    (3, 20, 500, 300, "zipf", "l2", "greedy"),
    (4, 500, 20, 300, "zipf", "l2", "greedy"),
    (5, 1, 77, 300, "zipf", "l2", "greedy"),
    (6, 77, 1, 300, "zipf", "l2", "greedy"),
    (7, 130, 170, 33, "dirichlet", "l2", "greedy"),
    (8, 64, 64, 8, "uniform", "sqeuclidean", "greedy"),
    (9, 100, 90, 1, "dirichlet", "l2", "greedy"),
    (10, 257, 129, 300, "dirichlet", "sqeuclidean", "random"),
    (11, 96, 96, 1024, "zipf", "l2", "greedy"),
    (12, 700, 650, 50, "zipf", "l2", "greedy"),
]


def _ids(c):
    return "-".join(map(str, c[1:]))


@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_bf16_matrix_core_pair_matches_oracle(case):
    seed, m, n, d, masses, metric, protocol = case
    Xb, a, Yb, b = W.random_doc_pair(800 + seed, m, n, d, masses=masses)
    kw = dict(protocol=protocol, seed=5)
    g = gpu_pair_bf16(Xb, a, Yb, b, metric, **kw)
    assert_pair_matches(g, oracle_pair(f32(Xb), a, f32(Yb), b, metric, **kw), rel=BF16_COST_REL, label=str(case))


@pytest.mark.parametrize("case", CASES[:8] + CASES[9:], ids=_ids)
def test_fp32_high_dim_pair_matches_oracle(case):
    seed, m, n, d, masses, metric, protocol = case
    d = max(d, 8)  # d <= 7 is the point path
    r = W.rng_for(850 + seed, 0)
    X = W.to_f32(r.standard_normal((m, d)) / np.sqrt(d))
    Y = W.to_f32(r.standard_normal((n, d)) / np.sqrt(d))
    _, a, _, b = W.random_doc_pair(850 + seed, m, n, 1, masses=masses)
    kw = dict(protocol=protocol, seed=5)
    g = gpu_pair(X, a, Y, b, metric, **kw)
    assert_pair_matches(g, oracle_pair(X, a, Y, b, metric, **kw), label=str(case))


@pytest.mark.parametrize("seed", range(3))
def test_bf16_lattice_ties_are_rescored(seed):
    """Integer coordinates make exact key ties: every one must resolve to the
    smallest supplier index, as in the oracle."""
    Xb, a, Yb, b = W.random_doc_pair(870 + seed, 150, 180, 40, masses="uniform", lattice=3)
    g = gpu_pair_bf16(Xb, a, Yb, b)
    assert int(g["stats"]["rescored"]) > 0
    assert_pair_matches(g, oracle_pair(f32(Xb), a, f32(Yb), b), rel=BF16_COST_REL, label=f"lattice{seed}")


def test_bf16_zero_mass_points_and_status_codes():
    Xb, a, Yb, b = W.random_doc_pair(880, 60, 70, 300)
    a = a.copy()
    a[[0, 7]] = 0
    a = (a / a.astype(np.float64).sum()).astype(np.float32)
    assert_pair_matches(gpu_pair_bf16(Xb, a, Yb, b), oracle_pair(f32(Xb), a, f32(Yb), b), rel=BF16_COST_REL,
                        label="zero mass")
    Xn = Xb.copy()
    Xn[3, 100] = 0x7FC0  # NaN
    assert int(gpu_pair_bf16(Xn, a, Yb, b)["stats"]["status"]) == -1
    Xi = Xb.copy()
    Xi[3, 100] = 0x7F80  # +inf
    assert int(gpu_pair_bf16(Xi, a, Yb, b)["stats"]["status"]) == -1
    neg = a.copy()
    neg[2] = -neg[2]
    assert int(gpu_pair_bf16(Xb, neg, Yb, b)["stats"]["status"]) == -1
    assert int(gpu_pair_bf16(Xb, a * 2, Yb, b)["stats"]["status"]) == -2
    g = gpu_pair_bf16(Xb, a, Yb, b, max_rounds=2)
    ref = oracle_pair(f32(Xb), a, f32(Yb), b, max_rounds=2)
    assert int(g["stats"]["status"]) == -6 and ref["status"] == -6
    np.testing.assert_array_equal(g["src"], ref["src"])
    np.testing.assert_array_equal(g["dst"], ref["dst"])
    np.testing.assert_array_equal(g["flow"], ref["flow"])


def test_bf16_key_cost_falls_back_to_exact_distances():
    """Candidates that nearly repeat the query's points: served squared
    distances far below the key bound's reach make the split form recompute
    every distance of the pair in FP64, so the cost is the definition's to
    1e-12; the well-separated pair beside it takes its distances from the
    keys, within BF16_COST_REL."""
    Xb, a, Yb, b = W.random_doc_pair(884, 70, 90, 300)
    Yc = Yb.copy()
    Yc[:70] = Xb
    Yc[:70:3, 5] ^= 1  # one BF16 step in one coordinate of every third copy
    for Y_, rel in ((Yc, 1e-12), (Yb, BF16_COST_REL)):
        g = gpu_pair_bf16(Xb, a, Y_, b)
        assert_pair_matches(g, oracle_pair(f32(Xb), a, f32(Y_), b), rel=rel, label=f"rel {rel}")


def test_bf16_empty_sides():
    z = np.zeros((0, 300), np.uint16)
    Xb, a, Yb, b = W.random_doc_pair(881, 5, 5, 300)
    g = gpu_pair_bf16(z, np.zeros(0, np.float32), z, np.zeros(0, np.float32))
    assert int(g["stats"]["status"]) == 0 and g["cost"] == 0.0
    g = gpu_pair_bf16(Xb, a, z, np.zeros(0, np.float32))
    assert int(g["stats"]["status"]) == -2


def test_unsupported_combinations_raise():
    import torch
    from paper_2401_07378_amd import binding
    from tests.gpu_helpers import to_dev, to_dev_bf16
    Xb, a, Yb, b = W.random_doc_pair(883, 4097, 3, 16)
    with pytest.raises(binding.NNSEMDError) as e:
        binding.emd_approx(to_dev_bf16(Xb), to_dev(a), to_dev_bf16(Yb), to_dev(b), "l1", mode="bf16_mfma_refine")
    assert e.value.status == -7  # L1 keeps sides <= 4096 as well
    with pytest.raises(binding.NNSEMDError) as e:
        binding.emd_approx(to_dev_bf16(Xb), to_dev(a), to_dev_bf16(Yb), to_dev(b), mode="bf16_mfma_refine")
    assert e.value.status == -7
    torch.cuda.synchronize()


def _small_docs(num, seed=890):
    return W.documents_300d(num_candidates=num, seed=seed)


@pytest.mark.parametrize("mode", ["bf16_mfma_refine", "fp32"])
def test_document_batch_matches_oracle(mode):
    """One query against 48 ragged candidates, plans included."""
    ps = _small_docs(48)
    g = gpu_batched(ps, plan=True, mode=mode)
    m_sizes, n_sizes = ps.sizes()
    rel = BF16_COST_REL if mode == "bf16_mfma_refine" else 1e-12
    for p in range(ps.num_pairs):
        X, a, Y, b = ps.pair(p)
        ref = oracle_pair(X, a, Y, b)
        lo = g["plan_off"][p]
        k = int(g["stats"][p]["nnz"])
        gp = {"cost": float(g["costs"][p]), "stats": g["stats"][p], "src": g["src"][lo:lo + k],
              "dst": g["dst"][lo:lo + k], "flow": g["flow"][lo:lo + k]}
        assert_pair_matches(gp, ref, rel=rel, label=f"pair{p}")


def test_document_batch_several_supplier_sets():
    """Three supplier sets of different sizes shared by nine pairs (the
    supplier norms are taken once per set): plans against the oracle; a
    non-finite coordinate in one set fails exactly the pairs that use it."""
    d = 300
    xs = [W.random_doc_pair(960 + s, m, 8, d)[:2] for s, m in enumerate((37, 211, 120))]
    ys = [W.random_doc_pair(970 + c, 8, n, d)[2:] for c, n in enumerate((90, 15, 260, 33, 180, 64, 301, 22, 140))]
    def cat(sets):
        bits = np.concatenate([s[0] for s in sets]).astype(np.uint16)
        mass = np.concatenate([s[1] for s in sets]).astype(np.float32)
        off = np.concatenate([[0], np.cumsum([len(s[1]) for s in sets])]).astype(np.int64)
        return bits, mass, off
    xb, xa, xo = cat(xs)
    yb, ya, yo = cat(ys)
    px = np.array([p % 3 for p in range(9)], np.int32)
    py = np.arange(9, dtype=np.int32)
    def pairset(xbits):
        return W.PairSet("several_sets", d, W.bf16_bits_to_f32(xbits).reshape(-1, d), xa, xo,
                         W.bf16_bits_to_f32(yb).reshape(-1, d), ya, yo, pair_x=px, pair_y=py,
                         metric="l2", dtype="bf16", X_bits=xbits, Y_bits=yb)
    ps = pairset(xb)
    g = gpu_batched(ps, plan=True, mode="bf16_mfma_refine")
    for p in range(ps.num_pairs):
        X, a, Y, b = ps.pair(p)
        ref = oracle_pair(X, a, Y, b)
        lo = g["plan_off"][p]
        k = int(g["stats"][p]["nnz"])
        gp = {"cost": float(g["costs"][p]), "stats": g["stats"][p], "src": g["src"][lo:lo + k],
              "dst": g["dst"][lo:lo + k], "flow": g["flow"][lo:lo + k]}
        assert_pair_matches(gp, ref, rel=BF16_COST_REL, label=f"pair{p}")
    bad = xb.copy()
    bad[xo[1] + 5, 17] = 0x7F80  # +inf in supplier set 1
    gb = gpu_batched(pairset(bad), mode="bf16_mfma_refine")
    for p in range(9):
        want = -1 if px[p] == 1 else 0
        assert int(gb["stats"][p]["status"]) == want, p
        if want == 0:
            assert gb["costs"][p] == g["costs"][p], p


def test_document_autotuner_keeps_results():
    """Both launch forms of the BF16 path (split key-tile kernel, tiles fused
    into the rounds kernel) give the same plans and costs; the autotuner times
    them and records one, and results stay the same."""
    from paper_2401_07378_amd import binding
    ps = _small_docs(40, seed=893)
    m_sizes, n_sizes = ps.sizes()
    side = int(max(m_sizes.max(), n_sizes.max()))
    binding.tuning_reset()
    try:
        split = gpu_batched(ps, plan=True, mode="bf16_mfma_refine")
        binding.tuning_set_docs(300, side, "fused")
        fused = gpu_batched(ps, plan=True, mode="bf16_mfma_refine")
        t = binding.autotune_docs(300, int(m_sizes.max()), int(n_sizes.max()), num_pairs=256)
        assert t["form"] in ("split", "fused") and t["ms_fused"] > 0 and t["ms_split"] > 0
        tuned = gpu_batched(ps, plan=True, mode="bf16_mfma_refine")
        # The forms round their FP32 keys in different orders, so each flags
        # its own near ties for the FP64 re-score; every plan and every other
        # counter is the same.  The fused form recomputes every served
        # distance in FP64, the split form takes them from its keys within
        # BF16_COST_REL.
        for other in (fused, tuned):
            for k in ("src", "dst", "flow"):
                np.testing.assert_array_equal(other[k], split[k])
            np.testing.assert_allclose(other["costs"], split["costs"], rtol=2 * BF16_COST_REL, atol=0)
            for f in split["stats"].dtype.names:
                if f != "rescored":
                    np.testing.assert_array_equal(other["stats"][f], split["stats"][f], err_msg=f)
    finally:
        binding.tuning_reset()


def test_shared_query_tile_pass_same_bits():
    """One query against ragged candidates: the tile pass that stages the
    query once per workgroup and runs stripe by stripe gives the same bits
    as the per-pair tile pass (the same MFMA blocks and FP64 chunk sums), so
    every plan, cost and counter, the re-score count included, is identical;
    both match the oracle.  A non-finite candidate coordinate fails only its
    own pair; one in the query fails every pair."""
    from paper_2401_07378_amd import binding
    ps = _small_docs(300, seed=894)
    m_sizes, n_sizes = ps.sizes()
    side = int(max(m_sizes.max(), n_sizes.max()))
    binding.tuning_reset()
    try:
        shared = gpu_batched(ps, plan=True, mode="bf16_mfma_refine")
        binding.tuning_set_docs(300, side, "split_per_pair")
        per_pair = gpu_batched(ps, plan=True, mode="bf16_mfma_refine")
    finally:
        binding.tuning_reset()
    for k in ("costs", "src", "dst", "flow", "stats"):
        np.testing.assert_array_equal(shared[k], per_pair[k], err_msg=k)
    for p in (0, 1, int(np.argmax(n_sizes)), int(np.argmin(n_sizes)), ps.num_pairs - 1):
        X, a, Y, b = ps.pair(p)
        ref = oracle_pair(X, a, Y, b)
        lo = shared["plan_off"][p]
        k = int(shared["stats"][p]["nnz"])
        gp = {"cost": float(shared["costs"][p]), "stats": shared["stats"][p], "src": shared["src"][lo:lo + k],
              "dst": shared["dst"][lo:lo + k], "flow": shared["flow"][lo:lo + k]}
        assert_pair_matches(gp, ref, rel=BF16_COST_REL, label=f"pair{p}")
    yb = ps.Y_bits.copy()
    yb[ps.y_off[7] + 3, 100] = 0x7FC0  # NaN in candidate 7
    bad_c = W.PairSet("docs_bad", 300, ps.X, ps.a, ps.x_off, W.bf16_bits_to_f32(yb).reshape(-1, 300), ps.b,
                      ps.y_off, pair_x=ps.pair_x, pair_y=ps.pair_y, metric="l2", dtype="bf16",
                      X_bits=ps.X_bits, Y_bits=yb)
    gb = gpu_batched(bad_c, mode="bf16_mfma_refine")
    want = np.zeros(ps.num_pairs, np.int32)
    want[7] = -1
    np.testing.assert_array_equal(gb["stats"]["status"], want)
    keep = want == 0
    np.testing.assert_array_equal(gb["costs"][keep], shared["costs"][keep])
    xb = ps.X_bits.copy()
    xb[5, 0] = 0xFF80  # -inf in the query
    bad_q = W.PairSet("docs_bad_q", 300, W.bf16_bits_to_f32(xb).reshape(-1, 300), ps.a, ps.x_off, ps.Y, ps.b,
                      ps.y_off, pair_x=ps.pair_x, pair_y=ps.pair_y, metric="l2", dtype="bf16",
                      X_bits=xb, Y_bits=ps.Y_bits)
    gq = gpu_batched(bad_q, mode="bf16_mfma_refine")
    assert np.all(gq["stats"]["status"] == -1)


def test_shared_query_two_launches_and_bad_entries():
    """A query of 224 points against 5000 candidates, one of them 1024
    points long, so the key-tile scratch (4 GiB) takes the batch in two
    launches.  Two pair-table entries name a supplier set that does not
    exist and one candidate is empty.  The shared-query tile pass gives the
    same bits as the per-pair one on every pair; sampled pairs from both
    launches, the long one and the empty one match the oracle."""
    from paper_2401_07378_amd import binding
    d = 300
    r = W.rng_for(895, 0)
    qb = W.f32_to_bf16_bits(W.to_f32(r.standard_normal((224, d)) / np.sqrt(d)))
    qa = W.zipf_masses(r, 224)
    sizes = r.integers(20, 41, 5000)
    sizes[2700] = 1024
    sizes[4321] = 0
    yb = W.f32_to_bf16_bits(W.to_f32(r.standard_normal((int(sizes.sum()), d)) / np.sqrt(d)))
    yo = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    ya = np.concatenate([W.zipf_masses(r, int(k)) if k > 0 else np.zeros(0, np.float32) for k in sizes])
    ya = ya.astype(np.float32)
    px = np.zeros(5000, np.int32)
    px[[17, 4800]] = 1  # no supplier set 1
    ps = W.PairSet("two_launches", d, W.bf16_bits_to_f32(qb).reshape(-1, d), qa.astype(np.float32),
                   np.array([0, 224], np.int64), W.bf16_bits_to_f32(yb).reshape(-1, d), ya, yo,
                   pair_x=px, pair_y=np.arange(5000, dtype=np.int32), metric="l2", dtype="bf16",
                   X_bits=qb.reshape(-1, d), Y_bits=yb.reshape(-1, d))
    import torch
    from tests.gpu_helpers import to_dev, to_dev_bf16

    def run():
        r = binding.emd_approx_batched(to_dev_bf16(ps.X_bits), to_dev(ps.a), to_dev(ps.x_off),
                                       to_dev_bf16(ps.Y_bits), to_dev(ps.b), to_dev(ps.y_off),
                                       pair_x=to_dev(px), pair_y=to_dev(ps.pair_y), num_pairs=5000,
                                       max_m=224, max_n=1024, metric="l2", mode="bf16_mfma_refine")
        torch.cuda.synchronize()
        return {"costs": r["costs"][:5000].cpu().numpy(), "stats": binding.stats_numpy(r["stats"])[:5000]}

    binding.tuning_reset()
    try:
        shared = run()
        binding.tuning_set_docs(d, 1024, "split_per_pair")
        per_pair = run()
    finally:
        binding.tuning_reset()
    np.testing.assert_array_equal(shared["costs"], per_pair["costs"])
    np.testing.assert_array_equal(shared["stats"], per_pair["stats"])
    st = shared["stats"]
    assert int(st["status"][17]) == -1 and int(st["status"][4800]) == -1
    assert int(st["status"][4321]) == -2  # empty candidate against a non-empty query: masses differ
    for p in (0, 1, 2699, 2700, 4321, 4680, 4681, 4999):
        X, a = ps.X, ps.a
        Y, b = ps.Y[yo[p]:yo[p + 1]], ps.b[yo[p]:yo[p + 1]]
        ref = oracle_pair(X, a, Y, b)
        gp = {"cost": float(shared["costs"][p]), "stats": st[p]}
        assert_pair_matches(gp, ref, rel=BF16_COST_REL, plan=False, label=f"pair{p}")


def test_shared_query_stripe_edges_and_large_offset():
    """One query against candidates whose sizes sit at the stripe and
    stripe-pair edges (1, 2, 15, 16, 17, 31, 32, 33, 63, 64, 65 consumers),
    with every coordinate offset by 3 (BF16 spacing 2^-6 there): the keys
    ||x||^2 - 2 x.y cancel about 300 times their result, so the FP32 bound
    is about 0.6 % of a squared distance.  Many consumers and serve orders
    then go to FP64 keys, and the cost falls back to exact distances.
    Plans, counts and costs (1e-12) equal the oracle's."""
    d = 64
    r = W.rng_for(896, 0)
    sizes = [1, 2, 15, 16, 17, 31, 32, 33, 63, 64, 65]
    def pts(k):
        return W.f32_to_bf16_bits(W.to_f32(3.0 + r.standard_normal((k, d)) / np.sqrt(d)))
    qb = pts(90)
    qa = W.zipf_masses(r, 90)
    ys = [(pts(k), W.zipf_masses(r, k)) for k in sizes]
    yb = np.concatenate([y[0] for y in ys]).astype(np.uint16)
    ya = np.concatenate([y[1] for y in ys]).astype(np.float32)
    yo = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    P = len(sizes)
    ps = W.PairSet("edges", d, W.bf16_bits_to_f32(qb).reshape(-1, d), qa.astype(np.float32),
                   np.array([0, 90], np.int64), W.bf16_bits_to_f32(yb).reshape(-1, d), ya, yo,
                   pair_x=np.zeros(P, np.int32), pair_y=np.arange(P, dtype=np.int32), metric="l2", dtype="bf16",
                   X_bits=qb.reshape(-1, d), Y_bits=yb.reshape(-1, d))
    g = gpu_batched(ps, plan=True, mode="bf16_mfma_refine")
    assert int(g["stats"]["rescored"].sum()) > 0
    for p in range(P):
        X, a, Y, b = ps.pair(p)
        ref = oracle_pair(X, a, Y, b)
        lo = g["plan_off"][p]
        k = int(g["stats"][p]["nnz"])
        gp = {"cost": float(g["costs"][p]), "stats": g["stats"][p], "src": g["src"][lo:lo + k],
              "dst": g["dst"][lo:lo + k], "flow": g["flow"][lo:lo + k]}
        assert_pair_matches(gp, ref, rel=1e-12, label=f"pair{p} n={sizes[p]}")


@pytest.mark.parametrize("d", [1, 33, 130, 320])
def test_shared_query_tile_pass_dimensions(d):
    """The shared-query tile pass at other dimensions: one K step (d = 1),
    rows that are not a multiple of 8 bytes (d = 33), a partial last K step
    (d = 130) and the largest split-form d (320): the same bits as the
    per-pair pass on every pair, and the oracle's plans on a sample."""
    from paper_2401_07378_amd import binding
    r = W.rng_for(897 + d, 0)
    qb = W.f32_to_bf16_bits(W.to_f32(r.standard_normal((75, d)) / np.sqrt(d)))
    qa = W.zipf_masses(r, 75)
    sizes = r.integers(1, 120, 40)
    yb = W.f32_to_bf16_bits(W.to_f32(r.standard_normal((int(sizes.sum()), d)) / np.sqrt(d)))
    ya = np.concatenate([W.zipf_masses(r, int(k)) for k in sizes]).astype(np.float32)
    yo = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    P = len(sizes)
    ps = W.PairSet("dims", d, W.bf16_bits_to_f32(qb).reshape(-1, d), qa.astype(np.float32),
                   np.array([0, 75], np.int64), W.bf16_bits_to_f32(yb).reshape(-1, d), ya, yo,
                   pair_x=np.zeros(P, np.int32), pair_y=np.arange(P, dtype=np.int32), metric="l2", dtype="bf16",
                   X_bits=qb.reshape(-1, d), Y_bits=yb.reshape(-1, d))
    side = int(max(75, sizes.max()))
    binding.tuning_reset()
    try:
        shared = gpu_batched(ps, plan=True, mode="bf16_mfma_refine")
        binding.tuning_set_docs(d, side, "split_per_pair")
        per_pair = gpu_batched(ps, plan=True, mode="bf16_mfma_refine")
    finally:
        binding.tuning_reset()
    for k in ("costs", "src", "dst", "flow", "stats"):
        np.testing.assert_array_equal(shared[k], per_pair[k], err_msg=k)
    for p in (0, int(np.argmax(sizes)), int(np.argmin(sizes)), P - 1):
        X, a, Y, b = ps.pair(p)
        ref = oracle_pair(X, a, Y, b)
        lo = shared["plan_off"][p]
        k = int(shared["stats"][p]["nnz"])
        gp = {"cost": float(shared["costs"][p]), "stats": shared["stats"][p], "src": shared["src"][lo:lo + k],
              "dst": shared["dst"][lo:lo + k], "flow": shared["flow"][lo:lo + k]}
        assert_pair_matches(gp, ref, rel=BF16_COST_REL, label=f"d{d} pair{p}")


@pytest.mark.parametrize("sizes", [[1], [1024], [32, 33]])
def test_shared_query_smallest_launches(sizes):
    """Shared-query launches at the edges of the record list: one pair of
    one point (one record, one workgroup), one pair of 1024 points (32
    records, the largest stripe-pair number the records hold) and two pairs
    on either side of a record boundary.  Same bits as the per-pair pass,
    and the oracle's plans."""
    from paper_2401_07378_amd import binding
    d = 64
    r = W.rng_for(905 + len(sizes) + sizes[0], 0)
    qb = W.f32_to_bf16_bits(W.to_f32(r.standard_normal((50, d)) / np.sqrt(d)))
    qa = W.zipf_masses(r, 50)
    sizes = np.array(sizes, np.int64)
    yb = W.f32_to_bf16_bits(W.to_f32(r.standard_normal((int(sizes.sum()), d)) / np.sqrt(d)))
    ya = np.concatenate([W.zipf_masses(r, int(k)) for k in sizes]).astype(np.float32)
    yo = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    P = len(sizes)
    ps = W.PairSet("edges", d, W.bf16_bits_to_f32(qb).reshape(-1, d), qa.astype(np.float32),
                   np.array([0, 50], np.int64), W.bf16_bits_to_f32(yb).reshape(-1, d), ya, yo,
                   pair_x=np.zeros(P, np.int32), pair_y=np.arange(P, dtype=np.int32), metric="l2", dtype="bf16",
                   X_bits=qb.reshape(-1, d), Y_bits=yb.reshape(-1, d))
    side = int(max(50, sizes.max()))
    binding.tuning_reset()
    try:
        shared = gpu_batched(ps, plan=True, mode="bf16_mfma_refine")
        binding.tuning_set_docs(d, side, "split_per_pair")
        per_pair = gpu_batched(ps, plan=True, mode="bf16_mfma_refine")
    finally:
        binding.tuning_reset()
    for k in ("costs", "src", "dst", "flow", "stats"):
        np.testing.assert_array_equal(shared[k], per_pair[k], err_msg=k)
    for p in range(P):
        X, a, Y, b = ps.pair(p)
        ref = oracle_pair(X, a, Y, b)
        lo = shared["plan_off"][p]
        k = int(shared["stats"][p]["nnz"])
        gp = {"cost": float(shared["costs"][p]), "stats": shared["stats"][p], "src": shared["src"][lo:lo + k],
              "dst": shared["dst"][lo:lo + k], "flow": shared["flow"][lo:lo + k]}
        assert_pair_matches(gp, ref, rel=BF16_COST_REL, label=f"sizes{list(sizes)} pair{p}")


def test_document_batch_as_given_schedule_same_bits():
    ps = _small_docs(32, seed=891)
    g1 = gpu_batched(ps, mode="bf16_mfma_refine")
    g2 = gpu_batched(ps, mode="bf16_mfma_refine", schedule="as_given")
    np.testing.assert_array_equal(g1["costs"], g2["costs"])
    np.testing.assert_array_equal(g1["stats"], g2["stats"])


def test_documents_full_size_sampled():
    """The 8192-candidate document workload: sampled pairs against the
    oracle; every pair against the FP32 vector path (identical bits)."""
    ps = W.documents_300d()
    g = gpu_batched(ps, mode="bf16_mfma_refine")
    assert np.all(g["stats"]["status"] == 0)
    v = gpu_batched(ps, mode="fp32")
    np.testing.assert_allclose(g["costs"], v["costs"], rtol=2 * BF16_COST_REL, atol=0)
    np.testing.assert_array_equal(g["stats"]["rounds"], v["stats"]["rounds"])
    np.testing.assert_array_equal(g["stats"]["nnz"], v["stats"]["nnz"])
    np.testing.assert_array_equal(g["stats"]["work"], v["stats"]["work"])
    m_sizes, n_sizes = ps.sizes()
    big = int(np.argmax(m_sizes * n_sizes))
    sample = sorted(set(W.rng_for(892, 0).choice(ps.num_pairs, 14, replace=False).tolist()) | {0, big})
    refs, _ = oracle.solve_batched(ps.X, ps.a, ps.x_off, ps.Y, ps.b, ps.y_off,
                                   pair_x=ps.pair_x[sample], pair_y=ps.pair_y[sample])
    for p, ref in zip(sample, refs):
        st = g["stats"][p]
        assert int(st["rounds"]) == ref["rounds"] and int(st["work"]) == ref["work"], p
        assert int(st["nnz"]) == ref["nnz"], p
        assert abs(float(g["costs"][p]) - ref["cost"]) <= BF16_COST_REL * ref["cost"], p
        assert abs(float(v["costs"][p]) - ref["cost"]) <= 1e-12 * ref["cost"], p


# -------------------------------------------------------------- L1 metric
# L1 is not a contraction: each pair's distance matrix is summed exactly in
# FP64 (dimension order, the definition's operations), then Algorithm 1 runs
# on it; plans, counts and cost equal the oracle's.
L1_CASES = [
    (1, 40, 60, 300, "zipf", "greedy"),
    (2, 500, 500, 300, "zipf", "greedy"),
    (3, 1, 77, 300, "zipf", "greedy"),
    (4, 77, 1, 50, "dirichlet", "random"),
    (5, 130, 170, 33, "dirichlet", "greedy"),
    (6, 96, 96, 1024, "uniform", "greedy"),
]


@pytest.mark.parametrize("case", L1_CASES, ids=lambda c: "-".join(map(str, c[1:])))
def test_l1_high_dim_pairs(case):
    seed, m, n, d, masses, protocol = case
    Xb, a, Yb, b = W.random_doc_pair(890 + seed, m, n, d, masses=masses)
    kw = dict(protocol=protocol, seed=9)
    ref = oracle_pair(f32(Xb), a, f32(Yb), b, "l1", **kw)
    assert_pair_matches(gpu_pair_bf16(Xb, a, Yb, b, "l1", **kw), ref, label=f"bf16-{case}")
    assert_pair_matches(gpu_pair(f32(Xb).reshape(m, d), a, f32(Yb).reshape(n, d), b, "l1", **kw), ref,
                        label=f"f32-{case}")


def test_l1_high_dim_lattice_ties():
    Xb, a, Yb, b = W.random_doc_pair(897, 150, 180, 40, masses="uniform", lattice=3)
    ref = oracle_pair(f32(Xb), a, f32(Yb), b, "l1")
    assert ref["near_ties_nn"] > 0
    assert_pair_matches(gpu_pair_bf16(Xb, a, Yb, b, "l1"), ref, label="lattice")


def test_l1_documents_batched_sampled():
    """The document workload's shape (one 300-d query against ragged
    candidates of 20..500 points, Zipf masses) under L1: 256 candidates in
    one call, every pair against the oracle."""
    ps = W.documents_300d(num_candidates=256)
    ps.metric = "l1"
    g = gpu_batched(ps, mode="bf16_mfma_refine", plan=True)
    for p in range(ps.num_pairs):
        X, a, Y, b = ps.pair(p)
        ref = oracle_pair(X, a, Y, b, "l1")
        lo = g["plan_off"][p]
        k = int(g["stats"][p]["nnz"])
        gp = {"cost": float(g["costs"][p]), "stats": g["stats"][p], "src": g["src"][lo:lo + k],
              "dst": g["dst"][lo:lo + k], "flow": g["flow"][lo:lo + k]}
        assert_pair_matches(gp, ref, label=f"cand{p}")
