"""Write tests/golden/colour_transfer_3d.json: the FP64 oracle's full run of
the 65536 x 65536 colour-transfer pair (two clipped 3-D Gaussian mixtures,
uniform masses, squared Euclidean ground distance).

The stored record (cost, rounds, work, nnz, near-tie counters, residuals,
SHA-256 of the plan arrays and of the per-supplier barycentric map of that
plan) comes from the oracle alone: this script imports only the seeded input
generator and ``oracle``.  One single-threaded oracle solve takes several
minutes.

Usage: python tests/golden/make_colour_transfer_golden.py
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2401_07378_amd import workloads as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "colour_transfer_3d.json")


def sha(arr, dtype) -> str:
    return hashlib.sha256(np.ascontiguousarray(arr, dtype=dtype).tobytes()).hexdigest()


def main():
    ps = W.colour_transfer_3d()
    t0 = time.perf_counter()
    ref = oracle.solve(ps.X, ps.a, ps.Y, ps.b, metric="sqeuclidean")
    dt = time.perf_counter() - t0
    assert ref["status"] == 0, ref
    bary = oracle.barycentric(ref["src"], ref["dst"], ref["flow"], ps.Y, len(ps.a))
    rec = {
        "_about": "FP64 oracle (Algorithm 1, greedy protocol, Sec. III-A) on the seeded "
                  "colour_transfer_3d pair: 65536 x 65536 points, two clipped Gaussian mixtures in "
                  "[0,1]^3, uniform masses 2^-16, squared Euclidean. Written by "
                  "tests/golden/make_colour_transfer_golden.py, which calls only the oracle. Plan "
                  "hashes are over little-endian int32 src, int32 dst, float64 flow in (round, "
                  "supplier, claimant) order; the map hash is over the float64 per-supplier "
                  "barycentric map (Sec. IV-D) of that plan, m x 3 row-major.",
        "workload": {"name": ps.name, "n": int(ps.meta["n"]), "seed": int(ps.meta["seed"]),
                     "metric": "sqeuclidean"},
        "cost": float(ref["cost"]), "cost_hex": float(ref["cost"]).hex(),
        "rounds": int(ref["rounds"]), "work": int(ref["work"]), "nnz": int(ref["nnz"]),
        "near_ties_nn": int(ref["near_ties_nn"]), "near_ties_order": int(ref["near_ties_order"]),
        "residual_src": float(ref["residual_src"]), "residual_dst": float(ref["residual_dst"]),
        "sha256_src": sha(ref["src"], "<i4"), "sha256_dst": sha(ref["dst"], "<i4"),
        "sha256_flow": sha(ref["flow"], "<f8"), "sha256_map": sha(bary, "<f8"),
        "oracle_seconds": round(dt, 1),
    }
    with open(OUT, "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")
    print(json.dumps(rec, indent=1))


if __name__ == "__main__":
    main()
