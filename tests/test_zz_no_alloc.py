"""emd_approx_batched_noalloc (the entry point for callers that cannot
allocate) against emd_approx_batched through the C ABI: two calls in a row,
the second with fewer and smaller pairs, each bit for bit equal to the
allocating call on the same inputs (costs, stats, plans)."""
import numpy as np
import pytest

from paper_2401_07378_amd import workloads as W
from tests.gpu_helpers import to_dev

pytestmark = pytest.mark.gpu


def _run(ps, noalloc, out):
    import torch
    from paper_2401_07378_amd import binding
    m, n = ps.sizes()
    poff = to_dev(binding.plan_offsets(m, n))
    r = binding.emd_approx_batched(to_dev(ps.X), to_dev(ps.a), to_dev(ps.x_off), to_dev(ps.Y), to_dev(ps.b),
                                   to_dev(ps.y_off), max_m=int(m.max()), max_n=int(n.max()), plan_off=poff,
                                   noalloc=noalloc, out=out)
    torch.cuda.synchronize()
    k = ps.num_pairs
    return {"costs": r["costs"][:k].cpu().numpy(), "stats": binding.stats_numpy(r["stats"])[:k],
            "src": r["plan_src"].cpu().numpy(), "dst": r["plan_dst"].cpu().numpy(),
            "flow": r["plan_flow"].cpu().numpy()}


def _outputs(ps):
    """Every output preallocated, so the no-allocation call sees none made."""
    import torch
    from paper_2401_07378_amd import binding
    m, n = ps.sizes()
    total = int(binding.plan_offsets(m, n)[-1])
    P = ps.num_pairs
    return {"costs": torch.empty(P, dtype=torch.float64, device="cuda"),
            "stats": torch.empty(P * binding.STATS_BYTES, dtype=torch.uint8, device="cuda"),
            "plan_src": torch.empty(total, dtype=torch.int32, device="cuda"),
            "plan_dst": torch.empty(total, dtype=torch.int32, device="cuda"),
            "plan_flow": torch.empty(total, dtype=torch.float64, device="cuda"), "plan_total": total}


def test_noalloc_matches_allocating_call_twice():
    big = W.batched_hist_3d(700, lo=64, hi=700, seed=4501)
    small = W.batched_hist_3d(90, lo=16, hi=200, seed=4502)
    for ps in (big, small):  # the second call is smaller: the fixed scratch keeps the last contents
        want = _run(ps, False, None)
        got = _run(ps, True, _outputs(ps))
        assert np.all(got["stats"]["status"] == 0)
        np.testing.assert_array_equal(got["costs"], want["costs"])
        np.testing.assert_array_equal(got["stats"], want["stats"])
        for k in ("src", "dst", "flow"):
            np.testing.assert_array_equal(got[k], want[k])


def test_noalloc_limits():
    import torch
    from paper_2401_07378_amd import binding
    ps = W.batched_hist_3d(4, lo=8, hi=16, seed=4503)
    m, n = ps.sizes()
    Xb = torch.zeros((len(ps.X), 3), dtype=torch.bfloat16, device="cuda")
    with pytest.raises(binding.NNSEMDError) as e:
        binding.emd_approx_batched(Xb, to_dev(ps.a), to_dev(ps.x_off), Xb, to_dev(ps.b), to_dev(ps.y_off),
                                   max_m=int(m.max()), max_n=int(n.max()), mode="bf16_mfma_refine", noalloc=True)
    assert e.value.status == -7
    big = 65537
    x_off = to_dev(np.arange(big + 1, dtype=np.int64))
    X1 = torch.zeros((big, 3), dtype=torch.float32, device="cuda")
    a1 = torch.ones(big, dtype=torch.float32, device="cuda")
    with pytest.raises(binding.NNSEMDError) as e:
        binding.emd_approx_batched(X1, a1, x_off, X1, a1, x_off, max_m=1, max_n=1, noalloc=True)
    assert e.value.status == -1
