"""The batched call captured in a HIP graph (through torch.cuda.graph) and
replayed: every replay, with eager work and synchronisations between the
replays, must reproduce the eager result bit for bit."""
import numpy as np
import pytest

from paper_2401_07378_amd import workloads as W
from tests.gpu_helpers import to_dev, to_dev_bf16

pytestmark = pytest.mark.gpu


def _capture_and_check(make_call, read, replays=4):
    import torch
    eager = make_call()  # also sizes the library's workspace before capture
    torch.cuda.synchronize()
    want = read(eager)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        make_call()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        out = make_call()
    for rep in range(replays):
        for v in out.values():
            if v is not None:
                v.fill_(0)  # eager work between replays; the replay must rewrite everything
        junk = torch.randn(1 << 20, device="cuda").sum()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = read(out)
        for k in want:
            np.testing.assert_array_equal(got[k], want[k], err_msg=f"replay {rep}: {k}")
        del junk


def test_batched_point_pairs_graph_replay():
    import torch
    from paper_2401_07378_amd import binding
    ps = W.batched_hist_3d(96, lo=20, hi=300, seed=1402)
    m, n = ps.sizes()
    X, a, xo, Y, b, yo = (to_dev(v) for v in (ps.X, ps.a, ps.x_off, ps.Y, ps.b, ps.y_off))
    po = to_dev(binding.plan_offsets(m, n))
    total = int(binding.plan_offsets(m, n)[-1])
    bufs = {"costs": torch.empty(96, dtype=torch.float64, device="cuda"),
            "stats": torch.empty(96 * binding.STATS_BYTES, dtype=torch.uint8, device="cuda"),
            "plan_src": torch.empty(total, dtype=torch.int32, device="cuda"),
            "plan_dst": torch.empty(total, dtype=torch.int32, device="cuda"),
            "plan_flow": torch.empty(total, dtype=torch.float64, device="cuda"), "plan_total": total}

    def call():
        r = binding.emd_approx_batched(X, a, xo, Y, b, yo, max_m=int(m.max()), max_n=int(n.max()), plan_off=po,
                                       out=bufs)
        return {k: r[k] for k in ("costs", "stats", "plan_src", "plan_dst", "plan_flow")}

    _capture_and_check(call, lambda o: {k: v.cpu().numpy() for k, v in o.items()})


def test_batched_documents_graph_replay():
    import torch
    from paper_2401_07378_amd import binding
    ps = W.documents_300d(num_candidates=40, seed=1403)
    m, n = ps.sizes()
    X, Y = to_dev_bf16(ps.X_bits), to_dev_bf16(ps.Y_bits)
    a, xo, b, yo, px, py = (to_dev(v) for v in (ps.a, ps.x_off, ps.b, ps.y_off, ps.pair_x, ps.pair_y))
    bufs = {"costs": torch.empty(40, dtype=torch.float64, device="cuda"),
            "stats": torch.empty(40 * binding.STATS_BYTES, dtype=torch.uint8, device="cuda")}

    def call():
        r = binding.emd_approx_batched(X, a, xo, Y, b, yo, pair_x=px, pair_y=py, max_m=int(m.max()),
                                       max_n=int(n.max()), mode="bf16_mfma_refine", out=bufs)
        return {k: r[k] for k in ("costs", "stats")}

    _capture_and_check(call, lambda o: {k: v.cpu().numpy() for k, v in o.items()})
