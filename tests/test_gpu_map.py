"""Barycentric transport maps of plans (colour transfer, Sec. IV-D) through
the C ABI: emd_barycentric_map on plans written by each solver path (on-chip,
multi-workgroup, BF16 high-dimensional), per supplier and per consumer, and
emd_approx_map on both of its paths.  Every map must equal the oracle's map
of the oracle's plan bit for bit (rows summed in plan order, NaN where a row
has no flow)."""
import numpy as np
import pytest

import oracle
from paper_2401_07378_amd import workloads as W
from tests.gpu_helpers import assert_pair_matches, gpu_pair, gpu_pair_bf16, oracle_pair, to_dev

pytestmark = pytest.mark.gpu


def _same_map(got, want, label=""):
    assert got.shape == want.shape, label
    assert np.array_equal(np.isnan(got), np.isnan(want)), label
    np.testing.assert_array_equal(got[~np.isnan(got)], want[~np.isnan(want)], err_msg=label)


def _gpu_map(src, dst, flow, P, rows, side, nnz_dev=None, capacity=None):
    import torch
    from paper_2401_07378_amd import binding
    cap = len(src) if capacity is None else capacity
    pad = cap - len(src)
    ps = to_dev(np.concatenate([src, np.zeros(pad, np.int32)]).astype(np.int32))
    pd = to_dev(np.concatenate([dst, np.zeros(pad, np.int32)]).astype(np.int32))
    pf = to_dev(np.concatenate([flow, np.zeros(pad)]).astype(np.float64))
    m = binding.barycentric_map(ps, pd, pf, to_dev(np.asarray(P, np.float32)), rows, side=side, nnz=nnz_dev)
    torch.cuda.synchronize()
    return m.cpu().numpy()


@pytest.mark.parametrize("path", ["on_chip", "multi"])
@pytest.mark.parametrize("metric", ["l2", "sqeuclidean", "l1"])
def test_map_of_point_path_plans(path, metric):
    X, a, Y, b = W.random_pair(800, 300, 340, 3)
    g = gpu_pair(X, a, Y, b, metric, path=path)
    ref = oracle_pair(X, a, Y, b, metric)
    assert_pair_matches(g, ref, label=path)
    _same_map(_gpu_map(g["src"], g["dst"], g["flow"], Y, 300, "suppliers"),
              oracle.barycentric(ref["src"], ref["dst"], ref["flow"], Y, 300), "suppliers")
    _same_map(_gpu_map(g["src"], g["dst"], g["flow"], X, 340, "consumers"),
              oracle.barycentric_dst(ref["src"], ref["dst"], ref["flow"], X, 340), "consumers")


def test_map_of_bf16_path_plan():
    """BF16 points take the high-dimensional (matrix-core) path at any d; its
    plan maps like any other (the points are the BF16 values)."""
    Xb, a, Yb, b = W.random_doc_pair(801, 120, 150, 3, masses="dirichlet")
    X, Y = W.bf16_bits_to_f32(Xb).reshape(-1, 3), W.bf16_bits_to_f32(Yb).reshape(-1, 3)
    g = gpu_pair_bf16(Xb, a, Yb, b)
    ref = oracle_pair(X, a, Y, b)
    assert_pair_matches(g, ref, label="bf16")
    _same_map(_gpu_map(g["src"], g["dst"], g["flow"], Y, 120, "suppliers"),
              oracle.barycentric(ref["src"], ref["dst"], ref["flow"], Y, 120))
    _same_map(_gpu_map(g["src"], g["dst"], g["flow"], X, 150, "consumers"),
              oracle.barycentric_dst(ref["src"], ref["dst"], ref["flow"], X, 150))


def test_map_long_rows_and_device_count():
    """One supplier serving hundreds of consumers (rows far above the
    one-thread row limit, taken by a wavefront), empty rows, and a plan
    buffer longer than the plan whose entry count is read on the device."""
    import torch
    rng = np.random.default_rng(5)
    X = W.to_f32(rng.random((4, 3)))
    a = W.to_f32(np.array([0.7, 0.1, 0.0, 0.2]))
    Y = W.to_f32(rng.random((900, 3)))
    b = W.uniform_masses(900)
    ref = oracle_pair(X, a, Y, b)
    assert ref["status"] == 0
    nnz = len(ref["src"])
    cnt = torch.tensor([nnz], dtype=torch.int64, device="cuda")
    got = _gpu_map(ref["src"], ref["dst"], ref["flow"], Y, 4, "suppliers", nnz_dev=cnt, capacity=nnz + 37)
    want = oracle.barycentric(ref["src"], ref["dst"], ref["flow"], Y, 4)
    _same_map(got, want)
    assert np.all(np.isnan(got[2]))
    got = _gpu_map(ref["src"], ref["dst"], ref["flow"], X, 900, "consumers", nnz_dev=cnt, capacity=nnz + 37)
    _same_map(got, oracle.barycentric_dst(ref["src"], ref["dst"], ref["flow"], X, 900))


@pytest.mark.parametrize("path", ["auto", "multi"])
def test_emd_approx_map_paths(path):
    """emd_approx_map: on chip when the pair fits (asynchronous), or the
    multi-workgroup path; same plan and map either way."""
    from tests.gpu_helpers import gpu_pair_map
    X, a, Y, b = W.random_pair(802, 500, 640, 3)
    for metric in ("l2", "sqeuclidean"):
        g = gpu_pair_map(X, a, Y, b, metric, path=path)
        ref = oracle_pair(X, a, Y, b, metric)
        assert_pair_matches(g, ref, label=f"{path}-{metric}")
        _same_map(g["map"], oracle.barycentric(ref["src"], ref["dst"], ref["flow"], Y, 500))


def test_emd_approx_map_without_plan_or_stats():
    import torch
    from paper_2401_07378_amd import binding
    X, a, Y, b = W.random_pair(803, 200, 180, 3)
    r = binding.emd_approx_map(to_dev(X), to_dev(a), to_dev(Y), to_dev(b), "l2", plan=False)
    torch.cuda.synchronize()
    ref = oracle_pair(X, a, Y, b)
    _same_map(r["map"].cpu().numpy(), oracle.barycentric(ref["src"], ref["dst"], ref["flow"], Y, 200))


def test_map_argument_errors():
    import torch
    from paper_2401_07378_amd import binding
    z = torch.zeros(4, dtype=torch.int32, device="cuda")
    f = torch.zeros(4, dtype=torch.float64, device="cuda")
    P = torch.zeros((5, 9), dtype=torch.float32, device="cuda")
    with pytest.raises(binding.NNSEMDError) as e:
        binding.barycentric_map(z, z, f, P, 3)
    assert e.value.status == -7  # d = 9
