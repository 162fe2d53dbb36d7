"""Benchmark: NNS-EMD pairs/s on the batched histogram workload (one MI355X).

Workload (one step): 4096 independent pairs, each side m, n ~ U{128..1024}
points in 3-D drawn uniform on [0,1]^3 (FP32), Dirichlet(1) masses, L2
ground distance, all pairs in one launch of the per-pair workgroup solver,
cost + plan + stats written for every pair.  Inputs are resident in HBM
before timing; the timed region is exactly --steps launches bracketed by
device synchronisation, measured with events on the launch stream.

Also reported on the same inputs:
  * roofline of the solver kernel (VALU-bound: algorithmic work is
    sum over rounds of |active S| x |active C| pair evaluations, 2d+2 lane
    operations each, against 256 CUs x 64 lanes x 2.4 GHz);
  * the plain single-pair FP32 path (one emd_approx launch per pair);
  * the oracle (FP64, CPU, OpenMP over pairs) on the same pairs, which is
    also the parity check of the timed outputs.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X: 256 CUs x 4 SIMDs x 16 lanes, 2.4 GHz -> 39.3e12 non-packed VALU
# lane-operations per second (half the 157.3 TFLOP/s FP32 figure, which counts
# a packed FMA as four flops; packed FP32 is not used by these kernels).
PEAK_VALU_LANE_OPS = 256 * 64 * 2.4e9
# Dense BF16 matrix-core peak of MI355X (2.5 PFLOP/s, no sparsity) and HBM3E.
PEAK_BF16_MFMA = 2.5e15
PEAK_HBM = 8.0e12
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pair_solver_batched_hist_3d_traffic.json")
SOURCES = [os.path.join(ROOT, "paper_2401_07378_amd", "csrc", f)
           for f in ("pair_solver.hip", "point_search.hpp", "round_common.hpp", "internal.hpp")]


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


# internal.hpp contributes only its point-path part (arguments and LDS
# layout), which ends with this line; the rest of it does not reach the kernel.
PAIR_SECTION_END = b"    L.total = align_up(o, 16);\n    return L;\n}\n"


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in SOURCES:
        with open(p, "rb") as f:
            data = f.read()
        if p.endswith("internal.hpp") and PAIR_SECTION_END in data:
            data = data[:data.index(PAIR_SECTION_END) + len(PAIR_SECTION_END)]
        h.update(data)
    return h.hexdigest()[:16]


DOC_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "doc_pair_kernel_documents_300d_traffic.json")
DOC_SOURCES = [os.path.join(ROOT, "paper_2401_07378_amd", "csrc", f)
               for f in ("doc_solver.hip", "round_common.hpp", "internal.hpp")]


def doc_kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in DOC_SOURCES:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_doc_traffic():
    """HBM bytes per document call (split form, every kernel of the call)
    from the committed rocprofv3 counter summary, or None when a document
    kernel source changed since the counters were taken."""
    if not os.path.exists(DOC_TRAFFIC_FILE):
        return None
    with open(DOC_TRAFFIC_FILE) as f:
        t = json.load(f)
    if t.get("source_hash") != doc_kernel_source_hash():
        return None
    return t.get("bytes_per_call")


def issued_per_eval(d):
    """VALU instructions the point-path search loop issues per evaluation
    (counted in the gfx950 assembly of the unrolled block)."""
    return d + 1.6875


def measured_traffic(per_launch_algorithmic_bytes):
    """HBM bytes per launch from the committed rocprofv3 counter summary,
    or None when the kernel source changed since the counters were taken."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as f:
        t = json.load(f)
    if t.get("source_hash") != kernel_source_hash():
        return None
    return t.get("bytes_per_launch")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--pairs", type=int, default=4096)
    ap.add_argument("--threads", type=int, default=0, help="workgroup size override (256/512)")
    ap.add_argument("--no-plan", action="store_true", help="cost + stats only")
    ap.add_argument("--no-graph", action="store_true",
                    help="batched_hist_3d: launch eagerly instead of replaying a captured graph of one step")
    ap.add_argument("--schedule", default="longest_first", choices=["longest_first", "as_given"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="batched_hist_3d, documents_300d, retrieval_3d: skip the launch autotuner")
    ap.add_argument("--no-single-pair", action="store_true")
    ap.add_argument("--single-pair-sample", type=int, default=512)
    ap.add_argument("--workload", default="batched_hist_3d",
                    choices=["batched_hist_3d", "colour_transfer_3d", "documents_300d", "retrieval_3d",
                             "single_pair_2d", "lattice_sweep", "colour_transfer_app"],
                    help="batched_hist_3d is the headline line; colour_transfer_3d times the 65536 x 65536 "
                         "pair; documents_300d times 8192 BF16 300-d document pairs; retrieval_3d times "
                         "surrogate-pruned retrieval among 100000 candidates")
    ap.add_argument("--train-pairs", type=int, default=200000, help="retrieval_3d: surrogate training labels")
    ap.add_argument("--epochs", type=int, default=16, help="retrieval_3d: training epochs")
    ap.add_argument("--queries", type=int, default=100, help="retrieval_3d: queries for recall@10")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build runs on one GPU only; --gpus N > 1 is not supported "
              "(pairs are independent: N GPUs would each take 1/N of the pairs)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    dev = torch.device("cuda:0")
    if args.calibrate_copy_mib:
        n = args.calibrate_copy_mib * (1 << 20) // 4
        x = torch.ones(n, dtype=torch.float32, device=dev)
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        log(f"copied {args.calibrate_copy_mib} MiB x3")
        return

    from paper_2401_07378_amd import binding
    from paper_2401_07378_amd import workloads as W

    if args.workload == "colour_transfer_3d":
        return bench_colour_transfer(args, dev)
    if args.workload == "documents_300d":
        return bench_documents(args, dev)
    if args.workload == "retrieval_3d":
        return bench_retrieval(args, dev)
    if args.workload == "single_pair_2d":
        return bench_single_pair(args, dev)
    if args.workload == "lattice_sweep":
        return bench_lattice_sweep(args, dev)
    if args.workload == "colour_transfer_app":
        return bench_colour_app(args, dev)

    log(f"generating workload ({args.pairs} pairs)")
    ps = W.batched_hist_3d(args.pairs)
    m_sizes, n_sizes = ps.sizes()
    P = ps.num_pairs
    d = ps.d
    t = lambda v: torch.from_numpy(np.ascontiguousarray(v)).to(dev)
    X, a, xo, Y, b, yo = t(ps.X), t(ps.a), t(ps.x_off), t(ps.Y), t(ps.b), t(ps.y_off)
    plan_off_np = binding.plan_offsets(m_sizes, n_sizes)
    want_plan = not args.no_plan
    out = {
        "costs": torch.empty(P, dtype=torch.float64, device=dev),
        "stats": torch.empty(P * binding.STATS_DTYPE.itemsize, dtype=torch.uint8, device=dev),
    }
    plan_off = None
    if want_plan:
        total = int(plan_off_np[-1])
        plan_off = t(plan_off_np)
        out.update(plan_src=torch.empty(total, dtype=torch.int32, device=dev),
                   plan_dst=torch.empty(total, dtype=torch.int32, device=dev),
                   plan_flow=torch.empty(total, dtype=torch.float64, device=dev),
                   plan_total=total)
    max_m, max_n = int(m_sizes.max()), int(n_sizes.max())
    tuning = None
    if not args.no_autotune and args.threads == 0:
        tuning = binding.autotune(d, "l2", max_m, max_n, num_pairs=1024)
        log(f"autotuned: {tuning}")

    def step(protocol="greedy"):
        binding.emd_approx_batched(X, a, xo, Y, b, yo, max_m=max_m, max_n=max_n, metric="l2",
                                   plan_off=plan_off, threads=args.threads, schedule=args.schedule,
                                   out=out, protocol=protocol, seed=7)

    torch.cuda.synchronize()
    log("warmup")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    use_graph = not args.no_graph
    if use_graph:
        # one step (schedule + solver launch) captured once and replayed: the
        # library allocates nothing and issues no memset once its workspace
        # is sized, so the captured step is the eager one
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            step()
        torch.cuda.synchronize()
        run = graph.replay
    else:
        run = step
    stream = torch.cuda.current_stream(dev)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    log(f"timing {args.steps} steps")
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        run()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    value = P / (ms / 1e3)
    log(f"{ms:.3f} ms/step, {value:.1f} pairs/s")

    st = binding.stats_numpy(out["stats"])[:P]
    costs = out["costs"].cpu().numpy()[:P]
    assert np.all(st["status"] == 0), "some pair failed"
    work = int(st["work"].sum())
    ops = work * (2 * d + 2)
    achieved = ops / (ms / 1e3)
    # the same pairs under the random protocol (Sec. III-A), eager launches
    for _ in range(2):
        step("random")
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        step("random")
    e1.record(stream)
    torch.cuda.synchronize()
    ms_rp = e0.elapsed_time(e1) / args.steps
    st_rp = binding.stats_numpy(out["stats"])[:P]
    random_protocol = {"ms_per_step": ms_rp, "value": P / (ms_rp / 1e3), "unit": "pairs/s",
                       "gp_over_rp_time": ms / ms_rp, "rounds_mean": float(st_rp["rounds"].mean()),
                       "work_evals": int(st_rp["work"].sum())}
    log(f"random protocol {ms_rp:.3f} ms/step (greedy {ms:.3f})")
    # restore the greedy outputs for the parity check below
    run()
    torch.cuda.synchronize()
    alg_bytes = int(ps.X.nbytes + ps.a.nbytes + ps.Y.nbytes + ps.b.nbytes + ps.x_off.nbytes
                    + ps.y_off.nbytes + P * (8 + binding.STATS_BYTES) + (int(st["nnz"].sum()) * 16 if want_plan else 0))
    threads_used = args.threads or (tuning["threads"] if tuning else 256)
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_VALU_LANE_OPS / 1e12,
                "unit": "Tops/s", "frac": achieved / PEAK_VALU_LANE_OPS,
                "traffic": measured_traffic(alg_bytes),
                "kernel": "pair_solver_kernel<3,%d,%d,L2> + order_kernel (one step)" % (
                    threads_used, -(-max(max_m, max_n) // threads_used)),
                "work_evals": work,
                "ops_per_eval": 2 * d + 2, "algorithmic_bytes": alg_bytes,
                "hbm_gbs_algorithmic": alg_bytes / (ms / 1e3) / 1e9,
                # the search loop issues d + 1.6875 VALU instructions per
                # evaluation (per block of 8 records x 4 consumers: 32 d FMAs,
                # 16 med3 and 24 min3 for the best two keys, 14 for the
                # block's slot bookkeeping): the share of the VALU issue
                # slots that went to evaluations
                "issued_ops_per_eval": issued_per_eval(d),
                "issue_frac": work * issued_per_eval(d) / (ms / 1e3) / PEAK_VALU_LANE_OPS}

    single = None
    if not args.no_single_pair:
        S = min(args.single_pair_sample, P)
        log(f"single-pair path on {S} pairs")
        views = []
        for p in range(S):
            xs, xe, ys, ye = ps.x_off[p], ps.x_off[p + 1], ps.y_off[p], ps.y_off[p + 1]
            views.append((X[xs:xe], a[xs:xe], Y[ys:ye], b[ys:ye]))
        outs = [{"cost": torch.empty(1, dtype=torch.float64, device=dev),
                 "stats": torch.empty(binding.STATS_BYTES, dtype=torch.uint8, device=dev)} for _ in range(S)]
        for p in range(min(S, 8)):
            binding.emd_approx(*views[p], "l2", plan=False, out=outs[p])
        torch.cuda.synchronize()
        e0.record(stream)
        for p in range(S):
            binding.emd_approx(*views[p], "l2", plan=False, out=outs[p])
        e1.record(stream)
        torch.cuda.synchronize()
        sms = e0.elapsed_time(e1)
        single = {"value": S / (sms / 1e3), "unit": "pairs/s", "sample": f"first {S} pairs, one launch each",
                  "speedup_batched": value / (S / (sms / 1e3))}
        log(f"single-pair path {single['value']:.1f} pairs/s")

    cpu = None
    parity = None
    if not args.no_cpu_baseline:
        import oracle
        log("oracle on the same pairs (CPU, OpenMP over pairs), repeated for about 10 s")
        t0 = time.perf_counter()
        ref, threads = oracle.solve_batched(ps.X, ps.a, ps.x_off, ps.Y, ps.b, ps.y_off)
        passes = 1
        while time.perf_counter() - t0 < 10.0:
            oracle.solve_batched(ps.X, ps.a, ps.x_off, ps.Y, ps.b, ps.y_off)
            passes += 1
        dt = time.perf_counter() - t0
        cpu = {"value": passes * P / dt, "unit": "pairs/s", "cores": threads, "kind": "oracle",
               "sample": f"all {P} pairs of the workload, {passes} passes, cost only, FP64, "
                         f"{threads} OpenMP threads", "seconds": dt}
        rc = np.array([r["cost"] for r in ref])
        rel = np.abs(costs - rc) / np.abs(rc)
        same = (np.array([r["rounds"] for r in ref]) == st["rounds"]) & \
               (np.array([r["work"] for r in ref]) == st["work"]) & \
               (np.array([r["nnz"] for r in ref]) == st["nnz"])
        near_same = (np.array([r["near_ties_nn"] for r in ref]) == st["near_ties_nn"]) & \
                    (np.array([r["near_ties_order"] for r in ref]) == st["near_ties_order"])
        parity = {"max_rel_err": float(rel.max()), "mean_rel_err": float(rel.mean()),
                  "pairs_checked": P, "stats_identical": int(same.sum()),
                  "rescored_consumers": int(st["rescored"].sum()),
                  "near_ties_nn": int(st["near_ties_nn"].sum()), "near_ties_order": int(st["near_ties_order"].sum()),
                  "near_ties_identical": int(near_same.sum()), "tolerance": 1e-5}
        log(f"oracle {cpu['value']:.1f} pairs/s on {threads} threads; max rel err {rel.max():.3g}")

    line = {
        "metric": "EMD pairs/sec at stated rel. error vs FP64 oracle; batched/MFMA vs plain FP32",
        "value": value, "unit": "pairs/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batched_hist_3d: 4096 pairs, m,n ~ U{128..1024}, 3-D U[0,1]^3 FP32, "
                               "Dirichlet(1) masses, L2, one launch, cost+plan+stats",
                   "num_pairs": P, "plan": want_plan, "graph": use_graph,
                   "threads": args.threads or (tuning["threads"] if tuning else 256),
                   "search_split": tuning["split"] if tuning else 1, "autotuned": tuning is not None,
                   "schedule": args.schedule, "seed": ps.meta["seed"],
                   "rounds_mean": float(st["rounds"].mean())},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "single_pair_fp32": single,
        "random_protocol": random_protocol,
        "parity": parity,
    }
    print(json.dumps(line), flush=True)


def bench_lattice_sweep(args, dev):
    """Pixel-grid histograms (Table 8a's shape): N images of 32 x 32 smooth
    densities, pair p = (image p, image p+1 mod N), N = 1024 .. 16384; each N
    timed as one batched launch and as one emd_approx launch per pair, under
    the greedy and the random protocol.  One 28 x 28 sparse-stroke batch
    beside it.  value = batched greedy pairs/s at the largest N."""
    import numpy as np
    import torch

    from paper_2401_07378_amd import binding
    from paper_2401_07378_amd import workloads as W

    stream = torch.cuda.current_stream(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t = lambda v: torch.from_numpy(np.ascontiguousarray(v)).to(dev)
    sizes = [1024, 2048, 4096, 8192, 16384]
    rows = []
    big = None
    for side, style, Ns in ((32, "smooth", sizes), (28, "strokes", [1024])):
        for N in Ns:
            ps = W.lattice_hist_2d(N, side, style)
            X, a, xo = t(ps.X), t(ps.a), t(ps.x_off)
            px, py = t(ps.pair_x), t(ps.pair_y)
            M = side * side
            out = {"costs": torch.empty(N, dtype=torch.float64, device=dev),
                   "stats": torch.empty(N * binding.STATS_BYTES, dtype=torch.uint8, device=dev)}
            row = {"images": N, "side": side, "style": style}
            for protocol in ("greedy", "random"):
                def step():
                    binding.emd_approx_batched(X, a, xo, X, a, xo, pair_x=px, pair_y=py, max_m=M, max_n=M,
                                               out=out, protocol=protocol, seed=3)
                step()
                torch.cuda.synchronize()
                reps = max(1, min(args.steps, 5))
                e0.record(stream)
                for _ in range(reps):
                    step()
                e1.record(stream)
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1) / reps
                st = binding.stats_numpy(out["stats"])[:N]
                assert np.all(st["status"] == 0)
                # one launch per pair (the unbatched form) on the same inputs
                outs = {"cost": torch.empty(1, dtype=torch.float64, device=dev),
                        "stats": torch.empty(binding.STATS_BYTES, dtype=torch.uint8, device=dev)}
                views = [(X[p * M:(p + 1) * M], a[p * M:(p + 1) * M], X[((p + 1) % N) * M:((p + 1) % N + 1) * M],
                          a[((p + 1) % N) * M:((p + 1) % N + 1) * M]) for p in range(N)]
                binding.emd_approx(*views[0], "l2", plan=False, protocol=protocol, seed=3, out=outs)
                torch.cuda.synchronize()
                e0.record(stream)
                for p in range(N):
                    binding.emd_approx(*views[p], "l2", plan=False, protocol=protocol, seed=3, out=outs)
                e1.record(stream)
                torch.cuda.synchronize()
                ms_single = e0.elapsed_time(e1)
                row[protocol] = {"batched_ms": ms, "batched_pairs_per_s": N / (ms / 1e3),
                                 "per_pair_launch_ms": ms_single, "per_pair_pairs_per_s": N / (ms_single / 1e3),
                                 "batching_speedup": ms_single / ms, "rounds_mean": float(st["rounds"].mean()),
                                 "work_evals": int(st["work"].sum()), "rescored": int(st["rescored"].sum()),
                                 "near_ties_nn": int(st["near_ties_nn"].sum())}
                log(f"{side}x{side} {style} N={N} {protocol}: batched {ms:.3f} ms, one launch per pair "
                    f"{ms_single:.1f} ms")
            row["rp_speedup"] = row["greedy"]["batched_ms"] / row["random"]["batched_ms"]
            rows.append(row)
            if side == 32 and N == sizes[-1]:
                big = (ps, row)
    ps, row = big
    N = ps.num_pairs
    ms = row["greedy"]["batched_ms"]
    work = row["greedy"]["work_evals"]
    roofline = {"bound": "alu", "achieved": work * 6 / (ms / 1e3) / 1e12, "peak": PEAK_VALU_LANE_OPS / 1e12,
                "unit": "Tops/s", "frac": work * 6 / (ms / 1e3) / PEAK_VALU_LANE_OPS, "traffic": None,
                "kernel": "pair_solver_kernel<2,...> (exact-key lattice search) at N = 16384",
                "work_evals": work, "ops_per_eval": 6}
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        S = 512
        t0 = time.perf_counter()
        _, threads = oracle.solve_batched(ps.X, ps.a, ps.x_off, ps.Y, ps.b, ps.y_off, pair_x=ps.pair_x[:S],
                                          pair_y=ps.pair_y[:S])
        dt = time.perf_counter() - t0
        cpu = {"value": S / dt, "unit": "pairs/s", "cores": threads, "kind": "oracle",
               "sample": f"first {S} of the {N} 32 x 32 pairs, greedy, cost only, {threads} OpenMP threads"}
    line = {"metric": "EMD pairs/sec at stated rel. error vs FP64 oracle; batched/MFMA vs plain FP32",
            "value": N / (ms / 1e3), "unit": "pairs/s", "n_gpus": 1, "steps": max(1, min(args.steps, 5)),
            "warmup": 1, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32", "data": "synthetic",
            "config": {"workload": "lattice_sweep: 32 x 32 pixel-grid histograms (smooth 8-bit densities), "
                                   "pairs (p, p+1 mod N), N = 1024..16384, L2; batched vs one launch per pair, "
                                   "greedy vs random protocol; plus 28 x 28 sparse strokes at N = 1024",
                       "seed": ps.meta["seed"]},
            "sweep": rows, "roofline": roofline, "cpu_baseline": cpu}
    print(json.dumps(line), flush=True)


def bench_colour_app(args, dev):
    """The colour-transfer application (Sec. IV-D) on two 1024 x 1024 RGB
    images: k-means palettes of 256 bins (10 update steps), NNS-EMD between
    the palettes, recolouring of the source; one transfer per step."""
    import numpy as np
    import torch

    from paper_2401_07378_amd import binding
    from paper_2401_07378_amd import workloads as W

    ref = W.colour_image(100, 1024, 1024)
    src = W.colour_image(101, 1024, 1024)
    R = torch.from_numpy(ref.reshape(-1, 3)).to(dev)
    Sd = torch.from_numpy(src.reshape(-1, 3)).to(dev)
    r = binding.colour_transfer(R, Sd, 256, 256, 10)
    for _ in range(max(args.warmup, 1)):
        r = binding.colour_transfer(R, Sd, 256, 256, 10, out=r)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    steps = max(1, min(args.steps, 20))
    e0.record(stream)
    for _ in range(steps):
        r = binding.colour_transfer(R, Sd, 256, 256, 10, out=r)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    st = binding.stats_numpy(r["stats"])[0]
    # dominant work: the palette reduction, 2 images x 11 assignment passes x
    # 1M pixels x 256 centroids, each distance 3 FP64 subtracts, 3 multiplies,
    # 3 adds (no fused multiply-add)
    flops = 2 * 11 * (1024 * 1024) * 256 * 9.0
    roofline = {"bound": "alu", "achieved": flops / (ms / 1e3) / 1e12, "peak": 78.6 / 2,
                "unit": "FP64 TFLOP/s (non-fused)", "frac": flops / (ms / 1e3) / 39.3e12, "traffic": None,
                "kernel": "km_assign (k-means assignment, FP64, one thread per pixel)", "flops_per_step": flops}
    cpu = parity = None
    if not args.no_cpu_baseline:
        import oracle
        t0 = time.perf_counter()
        want = oracle.colour_transfer(ref.reshape(-1, 3), src.reshape(-1, 3), 256, 256, 10)
        dt = time.perf_counter() - t0
        cpu = {"value": 1.0 / dt, "unit": "transfers/s", "cores": 1, "kind": "oracle",
               "sample": f"one whole transfer of the same images, one thread ({dt:.1f} s)"}
        got = r["image"].cpu().numpy().reshape(-1, 3)
        parity = {"image_identical": bool(np.array_equal(got, want["image"])),
                  "cost_rel_err": abs(float(r["cost"].item()) - want["solve"]["cost"]) / want["solve"]["cost"],
                  "rounds_gpu": int(st["rounds"]), "rounds_oracle": int(want["solve"]["rounds"])}
    line = {"metric": "EMD pairs/sec at stated rel. error vs FP64 oracle; batched/MFMA vs plain FP32",
            "value": 1e3 / ms, "unit": "transfers/s", "n_gpus": 1, "steps": steps, "warmup": max(args.warmup, 1),
            "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f64+f32", "data": "synthetic",
            "config": {"workload": "colour_transfer_app: 1024 x 1024 RGB reference and source, k-means palettes "
                                   "of 256 bins (10 update steps), NNS-EMD reference -> source palette (L2), "
                                   "per-consumer barycentric recolouring",
                       "rounds": int(st["rounds"]), "cost": float(r["cost"].item())},
            "paper_context": "4.572 s per 1024 x 1024 transfer on an RTX 3080 Ti (palette size not stated)",
            "roofline": roofline, "cpu_baseline": cpu, "parity": parity}
    print(json.dumps(line), flush=True)


def bench_single_pair(args, dev):
    """One 256 x 256 pair in 2-D (uniform on [0,1]^2, masses 1/256, L2) with
    its plan, one emd_approx call per step: the latency of a single pair on
    one workgroup (one compute unit), which no whole-GPU roofline describes."""
    import numpy as np
    import torch

    from paper_2401_07378_amd import binding
    from paper_2401_07378_amd import workloads as W

    ps = W.single_pair_2d()
    t = lambda v: torch.from_numpy(np.ascontiguousarray(v)).to(dev)
    X, a, Y, b = t(ps.X), t(ps.a), t(ps.Y), t(ps.b)
    r = binding.emd_approx(X, a, Y, b, "l2", plan=True)  # allocates the outputs once
    for _ in range(max(args.warmup, 1)):
        r = binding.emd_approx(X, a, Y, b, "l2", plan=True, out=r)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    steps = max(args.steps, 1) * 5
    e0.record(stream)
    for _ in range(steps):
        r = binding.emd_approx(X, a, Y, b, "l2", plan=True, out=r)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    st = binding.stats_numpy(r["stats"])[0]
    assert int(st["status"]) == 0
    work = int(st["work"])
    achieved = work * (2 * ps.d + 2) / (ms / 1e3)
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_VALU_LANE_OPS / 1e12, "unit": "Tops/s",
                "frac": achieved / PEAK_VALU_LANE_OPS, "traffic": None,
                "kernel": "pair_solver_kernel (one workgroup): latency-bound, "
                          "rounds x barrier-separated phases; the whole-GPU fraction does not describe it",
                "work_evals": work, "ops_per_eval": 2 * ps.d + 2}
    cpu, parity = None, None
    if not args.no_cpu_baseline:
        import oracle
        ref = oracle.solve(ps.X, ps.a, ps.Y, ps.b, metric="l2")
        nnz = int(st["nnz"])
        same = (np.array_equal(r["plan_src"][:nnz].cpu().numpy(), ref["src"])
                and np.array_equal(r["plan_dst"][:nnz].cpu().numpy(), ref["dst"])
                and np.array_equal(r["plan_flow"][:nnz].cpu().numpy(), ref["flow"]))
        parity = {"rel_err": abs(float(r["cost"].item()) - ref["cost"]) / ref["cost"], "plan_identical": bool(same),
                  "rounds_gpu": int(st["rounds"]), "rounds_oracle": ref["rounds"], "tolerance": 1e-5}
        times = []
        for _ in range(100):
            t0 = time.perf_counter()
            oracle.solve(ps.X, ps.a, ps.Y, ps.b, metric="l2")
            times.append(time.perf_counter() - t0)
        med = float(np.median(times))
        cpu = {"value": 1.0 / med, "unit": "pairs/s", "cores": 1, "kind": "oracle",
               "sample": f"the same pair, plan included, median of 100 runs ({med * 1e3:.2f} ms), one thread"}
    line = {"metric": "EMD pairs/sec at stated rel. error vs FP64 oracle; batched/MFMA vs plain FP32",
            "value": 1e3 / ms, "unit": "pairs/s", "n_gpus": 1, "steps": steps, "warmup": max(args.warmup, 1),
            "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32", "data": "synthetic",
            "config": {"workload": "single_pair_2d: one 256 x 256 pair, U[0,1]^2 FP32, masses 1/256, L2, "
                                   "cost + plan, one call per step",
                       "us_per_pair": ms * 1e3, "rounds": int(st["rounds"])},
            "roofline": roofline, "cpu_baseline": cpu, "parity": parity}
    print(json.dumps(line), flush=True)


def bench_colour_transfer(args, dev):
    """One 65536 x 65536 pair (two clipped Gaussian mixtures in 3-D, uniform
    masses, squared Euclidean) through the multi-workgroup path, with the
    barycentric map.  The host waits for the device inside the call, so one
    step is timed with events around the whole call."""
    import numpy as np
    import torch

    from paper_2401_07378_amd import binding
    from paper_2401_07378_amd import workloads as W

    ps = W.colour_transfer_3d()
    t = lambda v: torch.from_numpy(np.ascontiguousarray(v)).to(dev)
    X, a, Y, b = t(ps.X), t(ps.a), t(ps.Y), t(ps.b)
    for _ in range(args.warmup):
        binding.emd_approx_map(X, a, Y, b, "sqeuclidean")
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    steps = max(1, min(args.steps, 5))
    e0.record(stream)
    for _ in range(steps):
        r = binding.emd_approx_map(X, a, Y, b, "sqeuclidean")
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    st = binding.stats_numpy(r["stats"])[0]
    assert int(st["status"]) == 0
    work = int(st["work"])
    d = ps.d
    achieved = work * (2 * d + 2) / (ms / 1e3)
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_VALU_LANE_OPS / 1e12, "unit": "Tops/s",
                "frac": achieved / PEAK_VALU_LANE_OPS, "traffic": None, "kernel": "lp_search + round kernels",
                "work_evals": work, "ops_per_eval": 2 * d + 2}
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        log("oracle, first round of the same pair (bounded sample)")
        t0 = time.perf_counter()
        ref = oracle.solve(ps.X, ps.a, ps.Y, ps.b, metric="sqeuclidean", with_plan=False, max_rounds=1)
        dt = time.perf_counter() - t0
        rate = ref["work"] / dt
        cpu = {"value": rate / work, "unit": "pairs/s", "cores": 1, "kind": "oracle",
               "sample": f"first round of the pair ({ref['work']} pair evaluations in {dt:.1f} s, one thread); "
                         f"scaled by the pair's total {work} evaluations"}
    line = {"metric": "EMD pairs/sec at stated rel. error vs FP64 oracle; batched/MFMA vs plain FP32",
            "value": 1e3 / ms, "unit": "pairs/s", "n_gpus": 1, "steps": steps, "warmup": args.warmup,
            "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32", "data": "synthetic",
            "config": {"workload": "colour_transfer_3d: one 65536 x 65536 pair, 2-component Gaussian mixtures "
                                   "clipped to [0,1]^3, uniform masses, squared Euclidean, cost + barycentric map",
                       "rounds": int(st["rounds"]), "rescored": int(st["rescored"]),
                       "near_ties_nn": int(st["near_ties_nn"]), "near_ties_order": int(st["near_ties_order"])},
            "roofline": roofline, "cpu_baseline": cpu}
    print(json.dumps(line), flush=True)


def bench_documents(args, dev):
    """One 300-d BF16 query against 8192 ragged candidates (20..500 points,
    Zipf(1.1) masses, L2) through the high-dimensional path: key tiles on the
    matrix cores.  Compared on the same values with the batched FP32 vector
    path and the plain single-pair FP32 path (one emd_approx per pair)."""
    import numpy as np
    import torch

    from paper_2401_07378_amd import binding
    from paper_2401_07378_amd import workloads as W

    log("generating documents_300d (8192 candidates)")
    ps = W.documents_300d()
    P, d = ps.num_pairs, ps.d
    m_sizes, n_sizes = ps.sizes()
    t = lambda v: torch.from_numpy(np.ascontiguousarray(v)).to(dev)
    bf = lambda bits: torch.from_numpy(np.ascontiguousarray(bits).view(np.int16)).view(torch.bfloat16).to(dev)
    Xb, Yb = bf(ps.X_bits), bf(ps.Y_bits)
    Xf, Yf = t(ps.X), t(ps.Y)
    a, b, xo, yo, px, py = t(ps.a), t(ps.b), t(ps.x_off), t(ps.y_off), t(ps.pair_x), t(ps.pair_y)
    plan_off_np = binding.plan_offsets(m_sizes, n_sizes)
    want_plan = not args.no_plan
    max_m, max_n = int(m_sizes.max()), int(n_sizes.max())

    def buffers():
        o = {"costs": torch.empty(P, dtype=torch.float64, device=dev),
             "stats": torch.empty(P * binding.STATS_DTYPE.itemsize, dtype=torch.uint8, device=dev)}
        if want_plan:
            total = int(plan_off_np[-1])
            o.update(plan_src=torch.empty(total, dtype=torch.int32, device=dev),
                     plan_dst=torch.empty(total, dtype=torch.int32, device=dev),
                     plan_flow=torch.empty(total, dtype=torch.float64, device=dev), plan_total=total)
        return o

    plan_off = t(plan_off_np) if want_plan else None
    stream = torch.cuda.current_stream(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(X, Y, mode, out, steps):
        def step():
            binding.emd_approx_batched(X, a, xo, Y, b, yo, pair_x=px, pair_y=py, max_m=max_m, max_n=max_n,
                                       metric="l2", plan_off=plan_off, mode=mode, schedule=args.schedule,
                                       out=out)
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(steps):
            step()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    doc_tuning = None
    if not args.no_autotune:
        doc_tuning = binding.autotune_docs(d, max_m, max_n, num_pairs=1024)
        log(f"autotuned launch form: {doc_tuning}")
    out = buffers()
    log(f"timing {args.steps} steps (BF16 matrix-core path)")
    ms = timed(Xb, Yb, "bf16_mfma_refine", out, args.steps)
    value = P / (ms / 1e3)
    log(f"{ms:.3f} ms/step, {value:.1f} pairs/s")
    st = binding.stats_numpy(out["stats"])[:P]
    costs = out["costs"].cpu().numpy()[:P]
    assert np.all(st["status"] == 0), "some pair failed"

    out_v = buffers()
    vsteps = max(1, min(args.steps, 5))
    ms_v = timed(Xf, Yf, "fp32", out_v, vsteps)
    # The FP32 vector path recomputes every served distance in FP64; the BF16
    # split form takes them from its keys within 1e-5 (plans identical).
    vcosts = out_v["costs"].cpu().numpy()[:P]
    v_rel = float(np.max(np.abs(vcosts - costs) / np.maximum(np.abs(vcosts), 1e-300)))
    log(f"batched FP32 vector path {ms_v:.3f} ms/step; max rel cost difference {v_rel:.3g}")

    single = None
    if not args.no_single_pair:
        S = min(args.single_pair_sample, P)
        views = []
        for p in range(S):
            xs, xe = ps.x_off[ps.pair_x[p]], ps.x_off[ps.pair_x[p] + 1]
            ys, ye = ps.y_off[ps.pair_y[p]], ps.y_off[ps.pair_y[p] + 1]
            views.append((Xf[xs:xe], a[xs:xe], Yf[ys:ye], b[ys:ye]))
        outs = [{"cost": torch.empty(1, dtype=torch.float64, device=dev),
                 "stats": torch.empty(binding.STATS_BYTES, dtype=torch.uint8, device=dev)} for _ in range(S)]
        for p in range(min(S, 8)):
            binding.emd_approx(*views[p], "l2", plan=False, out=outs[p])
        torch.cuda.synchronize()
        e0.record(stream)
        for p in range(S):
            binding.emd_approx(*views[p], "l2", plan=False, out=outs[p])
        e1.record(stream)
        torch.cuda.synchronize()
        sms = e0.elapsed_time(e1)
        single = {"value": S / (sms / 1e3), "unit": "pairs/s",
                  "sample": f"first {S} pairs, FP32 values of the same BF16 points, one launch each",
                  "speedup_batched": value / (S / (sms / 1e3))}
        log(f"single-pair FP32 path {single['value']:.1f} pairs/s")

    flops = float(2.0 * (m_sizes * n_sizes).sum() * d)
    work = int(st["work"].sum())
    alg_bytes = int(ps.X_bits.nbytes + ps.a.nbytes + ps.Y_bits.nbytes + ps.b.nbytes + ps.x_off.nbytes
                    + ps.y_off.nbytes + 8 * P + P * (8 + binding.STATS_BYTES)
                    + (int(st["nnz"].sum()) * 16 if want_plan else 0))
    # One query of m points against the candidates: about m flops per byte
    # of candidate rows, below the BF16 ridge (2.5e15 / 8e12 = 312), so the
    # call is bound by HBM; the matrix-core rate is reported beside it.
    fused = doc_tuning is not None and doc_tuning["form"] == "fused"
    roofline = {"bound": "hbm", "achieved": alg_bytes / (ms / 1e3) / 1e9, "peak": PEAK_HBM / 1e9,
                "unit": "GB/s", "frac": alg_bytes / (ms / 1e3) / PEAK_HBM,
                "traffic": None if fused else measured_doc_traffic(),
                "kernel": ("doc_pair_kernel<bf16, mfma, 256, 4, fused> (one call)"
                           if fused else
                           "doc_tile_shared_kernel + doc_pair_kernel<bf16, mfma, 256, 4, split> (one call)"),
                "algorithmic_bytes": alg_bytes, "mfma_flops_per_launch": flops,
                "mfma_tflops": flops / (ms / 1e3) / 1e12, "mfma_frac": flops / (ms / 1e3) / PEAK_BF16_MFMA,
                "work_evals": work}

    cpu = parity = None
    if not args.no_cpu_baseline:
        import oracle
        S = P  # about 7 s of FP64 work on 16 host threads
        log(f"oracle on the first {S} pairs (CPU, OpenMP over pairs)")
        t0 = time.perf_counter()
        ref, threads = oracle.solve_batched(ps.X, ps.a, ps.x_off, ps.Y, ps.b, ps.y_off,
                                            pair_x=ps.pair_x[:S], pair_y=ps.pair_y[:S])
        dt = time.perf_counter() - t0
        cpu = {"value": S / dt, "unit": "pairs/s", "cores": threads, "kind": "oracle",
               "sample": (f"all {P} pairs" if S == P else f"first {S} of the {P} pairs")
                         + f", cost only, FP64, {threads} OpenMP threads", "seconds": dt}
        rc = np.array([r["cost"] for r in ref])
        rel = np.abs(costs[:S] - rc) / np.abs(rc)
        same = (np.array([r["rounds"] for r in ref]) == st["rounds"][:S]) & \
               (np.array([r["work"] for r in ref]) == st["work"][:S]) & \
               (np.array([r["nnz"] for r in ref]) == st["nnz"][:S])
        ref_nn = np.array([r["near_ties_nn"] for r in ref])
        ref_ord = np.array([r["near_ties_order"] for r in ref])
        near_same = (ref_nn == st["near_ties_nn"][:S]) & (ref_ord == st["near_ties_order"][:S])
        bad = np.nonzero(~near_same)[0][:8]
        mismatch = [[int(p), int(st["near_ties_nn"][p]), int(st["near_ties_order"][p]), int(ref_nn[p]),
                     int(ref_ord[p])] for p in bad]
        parity = {"max_rel_err": float(rel.max()), "pairs_checked": S, "stats_identical": int(same.sum()),
                  "oracle_near_ties_nn": int(ref_nn.sum()), "oracle_near_ties_order": int(ref_ord.sum()),
                  "near_tie_mismatch_first": mismatch,
                  "rescored_consumers": int(st["rescored"].sum()),
                  "near_ties_nn": int(st["near_ties_nn"].sum()), "near_ties_order": int(st["near_ties_order"].sum()),
                  "near_ties_identical": int(near_same.sum()), "tolerance": 1e-3,
                  "fp32_vector_path_max_rel_cost_diff": v_rel}
        log(f"oracle {cpu['value']:.1f} pairs/s; max rel err {rel.max():.3g}")

    line = {"metric": "EMD pairs/sec at stated rel. error vs FP64 oracle; batched/MFMA vs plain FP32",
            "value": value, "unit": "pairs/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "bf16", "data": "synthetic",
            "config": {"workload": "documents_300d: 1 query vs 8192 candidates, sizes U{20..500}, 300-d "
                                   "N(0,1)/sqrt(300) stored BF16, Zipf(1.1) masses, L2, cost+plan+stats",
                       "num_pairs": P, "plan": want_plan, "seed": ps.meta["seed"],
                       "rounds_mean": float(st["rounds"].mean()),
                       "launch_form": doc_tuning if doc_tuning is not None else {"form": "split", "autotuned": False}},
            "roofline": roofline, "cpu_baseline": cpu, "single_pair_fp32": single,
            "batched_fp32_vector": {"value": P / (ms_v / 1e3), "unit": "pairs/s", "ms_per_step": ms_v,
                                   "max_rel_cost_diff": v_rel},
            "parity": parity}
    print(json.dumps(line), flush=True)


def bench_retrieval(args, dev):
    """Surrogate-pruned retrieval (one query against 100000 candidate clouds
    of 256 3-D points, uniform masses, L2): the surrogate keeps 1000, NNS-EMD
    re-ranks them, top 10.  Trained first on NNS-EMD labels of independent
    cloud pairs; the index of candidate embeddings is built once.  value =
    candidates ranked per second per query; the exhaustive NNS-EMD scan of
    the same candidates is timed beside it, and recall@10 against it."""
    import numpy as np
    import torch

    from paper_2401_07378_amd import binding
    from paper_2401_07378_amd import surrogate as SG
    from paper_2401_07378_amd import workloads as W

    t = lambda v: torch.from_numpy(np.ascontiguousarray(v)).to(dev)
    log(f"generating {args.train_pairs} training pairs")
    X, a, off = W.surrogate_training_pairs(args.train_pairs)
    Xd, ad, offd = t(X), t(a), t(off)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    labels, st = SG.nnsemd_labels(Xd, ad, offd, args.train_pairs, 256)
    t_labels = time.perf_counter() - t0
    assert np.all(st["status"] == 0)
    log(f"labels in {t_labels:.2f} s; training {args.epochs} epochs")
    tr = SG.Trainer(SG.init_params(11), dev)
    t0 = time.perf_counter()
    hist = tr.fit(Xd, ad, off, labels, batch=512, epochs=args.epochs, lr=2e-3, log_every=4, log=log)
    t_train = time.perf_counter() - t0
    del Xd, ad, offd, labels
    log(f"trained in {t_train:.1f} s, loss {hist[0]:.4f} -> {hist[-1]:.4f}")
    ps = W.retrieval_3d(100000)
    N = ps.meta["num_candidates"]
    Y, b, yo = t(ps.Y), t(ps.b), t(ps.y_off)
    stream = torch.cuda.current_stream(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    E = SG.build_index(tr.theta, Y, b, yo)
    torch.cuda.synchronize()
    e0.record(stream)
    E = SG.build_index(tr.theta, Y, b, yo)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_index = e0.elapsed_time(e1)
    log(f"index of {N} candidates in {ms_index:.2f} ms")
    aq = t(W.uniform_masses(256))
    xo = t(np.array([0, 256], np.int64))
    zeros = torch.zeros(N, dtype=torch.int32, device=dev)
    cand = torch.arange(N, dtype=torch.int32, device=dev)
    Q = args.queries
    queries = [t(W.retrieval_query(q)) for q in range(Q)]
    ex_out = {"costs": torch.empty(N, dtype=torch.float64, device=dev),
              "stats": torch.empty(N * binding.STATS_BYTES, dtype=torch.uint8, device=dev)}
    pr_out = {}
    truth, got = [], []
    tuning = None
    if not args.no_autotune and args.threads == 0:
        tuning = binding.autotune(3, "l2", 256, 256, num_pairs=1024)  # the re-rank's and the scan's pair size
        log(f"autotuned: {tuning}")
    for q in range(min(2, Q)):  # warm-up
        SG.retrieve(tr.theta, E, queries[q], aq, Y, b, yo, 256, out=pr_out)
        binding.emd_approx_batched(queries[q], aq, xo, Y, b, yo, pair_x=zeros, pair_y=cand, max_m=256, max_n=256,
                                   out=ex_out)
    torch.cuda.synchronize()
    e0.record(stream)
    for q in range(Q):
        r = SG.retrieve(tr.theta, E, queries[q], aq, Y, b, yo, 256)
        got.append(r["idx"])
    e1.record(stream)
    torch.cuda.synchronize()
    ms_pruned = e0.elapsed_time(e1) / Q
    e0.record(stream)
    for q in range(Q):
        ex = binding.emd_approx_batched(queries[q], aq, xo, Y, b, yo, pair_x=zeros, pair_y=cand, max_m=256,
                                        max_n=256)
        truth.append(binding.topk_smallest(ex["costs"][:N], 10))
    e1.record(stream)
    torch.cuda.synchronize()
    ms_exh = e0.elapsed_time(e1) / Q
    rec = [len(set(g.cpu().numpy()) & set(tt.cpu().numpy())) / 10 for g, tt in zip(got, truth)]
    recall = float(np.mean(rec))
    log(f"pruned {ms_pruned:.3f} ms/query, exhaustive {ms_exh:.3f} ms/query, recall@10 {recall:.4f}")
    # dominant kernel of a pruned query: the rho GEMM over all candidates (timed alone)
    Eq = binding.sg_embed(tr.theta, queries[0], aq, xo)
    pred = torch.empty(N, dtype=torch.float32, device=dev)
    binding.sg_predict(tr.theta, Eq, E, out=pred)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(10):
        binding.sg_predict(tr.theta, Eq, E, out=pred)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_pred = e0.elapsed_time(e1) / 10
    flops = 2.0 * N * 768 * 256
    roofline = {"bound": "mfma", "achieved": flops / (ms_pred / 1e3) / 1e12, "peak": PEAK_BF16_MFMA / 1e12,
                "unit": "TFLOP/s", "frac": flops / (ms_pred / 1e3) / PEAK_BF16_MFMA, "traffic": None,
                "kernel": "sg_predict (pair features + gemm_nt_kernel + head) over 100000 candidates",
                "ms": ms_pred, "flops_per_launch": flops}
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        S = N  # the whole exhaustive scan of query 0: about 8 s of FP64 work on 16 host threads
        log(f"oracle on {S} of the exhaustive pairs of query 0 (CPU, OpenMP)")
        Xq0 = W.retrieval_query(0)
        t0 = time.perf_counter()
        _, threads = oracle.solve_batched(Xq0, W.uniform_masses(256), np.array([0, 256]), ps.Y, ps.b, ps.y_off,
                                          pair_x=np.zeros(S, np.int32), pair_y=np.arange(S, dtype=np.int32))
        dt = time.perf_counter() - t0
        cpu = {"value": S / dt, "unit": "candidates/s (exhaustive scan)", "cores": threads, "kind": "oracle",
               "sample": f"{S} of the 100000 query-candidate pairs, FP64, {threads} OpenMP threads "
                         f"(an exhaustive scan on the host), seconds {dt:.2f}"}
    line = {"metric": "EMD pairs/sec at stated rel. error vs FP64 oracle; batched/MFMA vs plain FP32",
            "value": N / (ms_pruned / 1e3), "unit": "candidates/s (pruned retrieval)", "n_gpus": 1,
            "steps": Q, "warmup": 2, "ms_per_step": ms_pruned, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "bf16+f32", "data": "synthetic",
            "config": {"workload": "retrieval_3d: 1 query vs 100000 Gaussian-mixture clouds of 256 3-D points, "
                                   "uniform masses, L2; surrogate keeps 1000, NNS-EMD re-ranks, top 10",
                       "train_pairs": args.train_pairs, "epochs": args.epochs, "loss_first": hist[0],
                       "loss_last": hist[-1], "train_s": t_train, "labels_s": t_labels, "index_ms": ms_index,
                       "queries": Q, "recall_at_10": recall,
                       "pair_launch": ({"threads": tuning["threads"], "search_split": tuning["split"], "autotuned": True}
                                       if tuning else {"autotuned": False})},
            "exhaustive_nnsemd": {"value": N / (ms_exh / 1e3), "unit": "pairs/s", "ms_per_query": ms_exh,
                                  "speedup_pruned": ms_exh / ms_pruned},
            "roofline": roofline, "cpu_baseline": cpu}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
