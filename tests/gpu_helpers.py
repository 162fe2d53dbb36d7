"""Helpers shared by the GPU tests: run the HIP path through the C ABI and
compare with the oracle on the same seeded inputs."""
import numpy as np

import oracle


def dev():
    import torch
    return torch.device("cuda:0")


def to_dev(x, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(dev())


def to_dev_bf16(bits):
    """uint16 BF16 bit patterns -> torch.bfloat16 device tensor (same bits)."""
    import torch
    t = torch.from_numpy(np.ascontiguousarray(bits, dtype=np.uint16).view(np.int16)).view(torch.bfloat16)
    return t.to(dev())


def gpu_pair_bf16(Xbits, a, Ybits, b, metric="l2", plan=True, **kw):
    """emd_approx on BF16 points (matrix-core mode)."""
    import torch
    from paper_2401_07378_amd import binding
    r = binding.emd_approx(to_dev_bf16(Xbits), to_dev(np.asarray(a, np.float32)), to_dev_bf16(Ybits),
                           to_dev(np.asarray(b, np.float32)), metric, plan=plan, mode="bf16_mfma_refine", **kw)
    torch.cuda.synchronize()
    return _collect(r, plan)


def _collect(r, plan):
    from paper_2401_07378_amd import binding
    st = binding.stats_numpy(r["stats"])[0]
    out = {"cost": float(r["cost"].item()), "stats": st}
    if plan and st["status"] in (0, -6):
        k = int(st["nnz"])
        out["src"] = r["plan_src"][:k].cpu().numpy()
        out["dst"] = r["plan_dst"][:k].cpu().numpy()
        out["flow"] = r["plan_flow"][:k].cpu().numpy()
    return out


def gpu_pair(X, a, Y, b, metric="l2", plan=True, **kw):
    """Run emd_approx on one pair; returns (cost, stats record, plan arrays)."""
    import torch
    from paper_2401_07378_amd import binding
    X = np.asarray(X, np.float32)
    Y = np.asarray(Y, np.float32)
    if X.ndim == 1:
        X = X.reshape(-1, 1)
    if Y.ndim == 1:
        Y = Y.reshape(-1, 1)
    r = binding.emd_approx(to_dev(X), to_dev(np.asarray(a, np.float32)), to_dev(Y),
                           to_dev(np.asarray(b, np.float32)), metric, plan=plan, **kw)
    torch.cuda.synchronize()
    return _collect(r, plan)


def gpu_batched(ps, plan=False, **kw):
    """Run emd_approx_batched on a workloads.PairSet."""
    import torch
    from paper_2401_07378_amd import binding
    m_sizes, n_sizes = ps.sizes()
    args = dict(max_m=int(max(m_sizes.max(initial=0), 1)), max_n=int(max(n_sizes.max(initial=0), 1)),
                metric=ps.metric)
    px = to_dev(ps.pair_x) if ps.pair_x is not None else None
    py = to_dev(ps.pair_y) if ps.pair_y is not None else None
    poff = None
    if plan:
        poff_np = binding.plan_offsets(m_sizes, n_sizes)
        poff = to_dev(poff_np)
    if kw.get("mode") == "bf16_mfma_refine":
        Xd, Yd = to_dev_bf16(ps.X_bits), to_dev_bf16(ps.Y_bits)
    else:
        Xd, Yd = to_dev(ps.X), to_dev(ps.Y)
    r = binding.emd_approx_batched(Xd, to_dev(ps.a), to_dev(ps.x_off), Yd,
                                   to_dev(ps.b), to_dev(ps.y_off), pair_x=px, pair_y=py,
                                   num_pairs=ps.num_pairs, plan_off=poff, **args, **kw)
    torch.cuda.synchronize()
    out = {"costs": r["costs"][:ps.num_pairs].cpu().numpy(),
           "stats": binding.stats_numpy(r["stats"])[:ps.num_pairs]}
    if plan:
        out["plan_off"] = poff_np
        out["src"] = r["plan_src"].cpu().numpy()
        out["dst"] = r["plan_dst"].cpu().numpy()
        out["flow"] = r["plan_flow"].cpu().numpy()
    return out


def gpu_pair_map(X, a, Y, b, metric="l2", **kw):
    """emd_approx_map on one pair: (cost, stats, plan arrays, map)."""
    import torch
    from paper_2401_07378_amd import binding
    X = np.asarray(X, np.float32)
    Y = np.asarray(Y, np.float32)
    r = binding.emd_approx_map(to_dev(X), to_dev(np.asarray(a, np.float32)), to_dev(Y),
                               to_dev(np.asarray(b, np.float32)), metric, **kw)
    torch.cuda.synchronize()
    st = binding.stats_numpy(r["stats"])[0]
    out = {"cost": float(r["cost"].item()), "stats": st, "map": r["map"].cpu().numpy()}
    if st["status"] in (0, -6):
        k = int(st["nnz"])
        out["src"] = r["plan_src"][:k].cpu().numpy()
        out["dst"] = r["plan_dst"][:k].cpu().numpy()
        out["flow"] = r["plan_flow"][:k].cpu().numpy()
    return out


def assert_pair_matches(g, ref, rel=1e-12, plan=True, label="", ties=True):
    """GPU result g vs oracle ref: status, rounds, work, nnz and the near-tie
    counters equal; plan bit-identical; cost within rel (summation order
    differs)."""
    st = g["stats"]
    assert int(st["status"]) == ref["status"], (label, int(st["status"]), ref["status"])
    if ref["status"] != 0:
        return
    assert int(st["rounds"]) == ref["rounds"], (label, int(st["rounds"]), ref["rounds"])
    assert int(st["work"]) == ref["work"], (label, int(st["work"]), ref["work"])
    assert int(st["nnz"]) == ref["nnz"], (label, int(st["nnz"]), ref["nnz"])
    c = g["cost"]
    assert abs(c - ref["cost"]) <= rel * max(abs(ref["cost"]), 1e-300), (label, c, ref["cost"])
    assert abs(float(st["residual_src"]) - ref["residual_src"]) <= 1e-12
    assert abs(float(st["residual_dst"]) - ref["residual_dst"]) <= 1e-12
    if ties:
        # near ties (gap <= 1e-6 relative): counted, and equal to the oracle's
        assert int(st["near_ties_nn"]) == ref["near_ties_nn"], (label, int(st["near_ties_nn"]), ref["near_ties_nn"])
        assert int(st["near_ties_order"]) == ref["near_ties_order"], \
            (label, int(st["near_ties_order"]), ref["near_ties_order"])
    if plan:
        np.testing.assert_array_equal(g["src"], ref["src"], err_msg=label)
        np.testing.assert_array_equal(g["dst"], ref["dst"], err_msg=label)
        np.testing.assert_array_equal(g["flow"], ref["flow"], err_msg=label)


def oracle_pair(X, a, Y, b, metric="l2", **kw):
    return oracle.solve(X, a, Y, b, metric=metric, **kw)
