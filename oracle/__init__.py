"""Plain FP64 CPU oracle for NNS-EMD -- test infrastructure only.

Only the test-suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never does, and this
package never imports the GPU library: the two share no code.

The arithmetic lives in ``nnsemd_oracle.c`` (Algorithm 1 of the paper, FP64,
no fused multiply-add); this module only compiles it with gcc and marshals
numpy arrays through ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nnsemd_oracle.c")
_LIB = os.path.join(_HERE, "libnnsemd_oracle.so")
# A prebuilt variant may be substituted (used only by the mutation tests,
# which compile deliberately broken copies to show the pins catch them).
_LIB_OVERRIDE = os.environ.get("NNSEMD_ORACLE_LIB")
_lock = threading.Lock()
_lib = None

METRICS = {"l2": 0, "sqeuclidean": 1, "l1": 2}
PROTOCOLS = {"greedy": 0, "random": 1}

STATUS = {
    0: "OK",
    -1: "INVALID_ARG",
    -2: "MASS_MISMATCH",
    -3: "CAPACITY",
    -4: "OUT_OF_MEMORY",
    -6: "NOT_CONVERGED",
}


class OracleStats(ctypes.Structure):
    _fields_ = [
        ("cost", ctypes.c_double),
        ("rounds", ctypes.c_int64),
        ("nnz", ctypes.c_int64),
        ("work", ctypes.c_int64),
        ("near_ties_nn", ctypes.c_int64),
        ("near_ties_order", ctypes.c_int64),
        ("residual_src", ctypes.c_double),
        ("residual_dst", ctypes.c_double),
        ("status", ctypes.c_int32),
        ("pad", ctypes.c_int32),
    ]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad"}


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, no fused multiply-add, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if _LIB_OVERRIDE:
                lib = ctypes.CDLL(_LIB_OVERRIDE)
            else:
                build()
                lib = ctypes.CDLL(_LIB)
            P = ctypes.c_void_p
            lib.nnsemd_oracle_solve.restype = ctypes.c_int
            lib.nnsemd_oracle_solve.argtypes = [
                P, P, ctypes.c_int64, P, P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                ctypes.c_int32, ctypes.c_uint64, ctypes.c_int64, P, P, P, ctypes.c_int64,
                ctypes.POINTER(OracleStats)]
            lib.nnsemd_oracle_solve_batched.restype = ctypes.c_int
            lib.nnsemd_oracle_solve_batched.argtypes = [
                ctypes.c_int64, P, P, P, P, P, P, P, P, ctypes.c_int32, ctypes.c_int32,
                ctypes.c_int32, ctypes.c_uint64, P]
            lib.nnsemd_oracle_solve_cost.restype = ctypes.c_int
            lib.nnsemd_oracle_solve_cost.argtypes = [
                P, P, ctypes.c_int64, P, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64,
                ctypes.c_int64, P, P, P, ctypes.c_int64, ctypes.POINTER(OracleStats)]
            lib.nnsemd_oracle_barycentric_dst.restype = None
            lib.nnsemd_oracle_barycentric_dst.argtypes = [
                P, P, P, ctypes.c_int64, P, ctypes.c_int64, ctypes.c_int32, P]
            lib.nnsemd_oracle_barycentric.restype = None
            lib.nnsemd_oracle_barycentric.argtypes = [
                P, P, P, ctypes.c_int64, P, ctypes.c_int64, ctypes.c_int32, P]
            lib.nnsemd_oracle_kmeans.restype = None
            lib.nnsemd_oracle_kmeans.argtypes = [P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, P, P, P]
            lib.nnsemd_oracle_recolour.restype = None
            lib.nnsemd_oracle_recolour.argtypes = [P, P, ctypes.c_int64, P, P]
            lib.nnsemd_oracle_rp_key.restype = ctypes.c_uint64
            lib.nnsemd_oracle_rp_key.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64]
            _lib = lib
    return _lib


def _f64(x, ndim):
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    if ndim == 2 and x.ndim == 1:
        x = x.reshape(-1, 1)
    return x


def _ptr(x):
    return x.ctypes.data_as(ctypes.c_void_p) if x is not None else None


def solve(X, a, Y, b, metric: str = "l2", protocol: str = "greedy", seed: int = 0,
          with_plan: bool = True, max_rounds: int = 0, plan_capacity: int | None = None) -> dict:
    """Run NNS-EMD on one pair (suppliers X,a searched by consumers Y,b).

    Inputs are promoted exactly to FP64 (FP32 and BF16 values are exact in
    FP64).  Returns a dict with the stats fields plus, when requested, the
    plan as ``src``, ``dst``, ``flow`` arrays in (round, supplier, claimant)
    order.
    """
    lib = _load()
    X = _f64(X, 2)
    Y = _f64(Y, 2)
    a = _f64(a, 1)
    b = _f64(b, 1)
    m, d = X.shape
    n = Y.shape[0]
    if Y.shape[1] != d and n > 0 and m > 0:
        raise ValueError("dimension mismatch")
    if m == 0:
        d = Y.shape[1] if Y.ndim == 2 and Y.shape[1] > 0 else max(d, 1)
    st = OracleStats()
    if with_plan:
        cap = max(m + n - 1, 1) if plan_capacity is None else plan_capacity
        src = np.zeros(max(cap, 1), np.int32)
        dst = np.zeros(max(cap, 1), np.int32)
        flow = np.zeros(max(cap, 1), np.float64)
    else:
        cap, src, dst, flow = 0, None, None, None
    lib.nnsemd_oracle_solve(_ptr(X), _ptr(a), m, _ptr(Y), _ptr(b), n, max(d, 1),
                            METRICS[metric], PROTOCOLS[protocol], seed & (2**64 - 1),
                            max_rounds, _ptr(src), _ptr(dst), _ptr(flow), cap,
                            ctypes.byref(st))
    out = st.as_dict()
    out["status_name"] = STATUS.get(out["status"], str(out["status"]))
    if with_plan and out["status"] in (0, -6):
        k = out["nnz"]
        out["src"], out["dst"], out["flow"] = src[:k].copy(), dst[:k].copy(), flow[:k].copy()
    return out


def solve_cost(D, a, b, protocol: str = "greedy", seed: int = 0, with_plan: bool = True,
               max_rounds: int = 0) -> dict:
    """Run NNS-EMD on a given ground-distance matrix D (m x n; Algorithm 1's
    input): suppliers carry masses a (m), consumers b (n).  D_ij is the key
    of the search and of the greedy order and the distance of the cost.
    Same result dict as solve()."""
    lib = _load()
    D = np.ascontiguousarray(np.asarray(D, dtype=np.float64))
    a = _f64(a, 1)
    b = _f64(b, 1)
    m, n = len(a), len(b)
    if D.shape != (m, n):
        raise ValueError("D must be m x n")
    st = OracleStats()
    if with_plan:
        cap = max(m + n - 1, 1)
        src = np.zeros(cap, np.int32)
        dst = np.zeros(cap, np.int32)
        flow = np.zeros(cap, np.float64)
    else:
        cap, src, dst, flow = 0, None, None, None
    lib.nnsemd_oracle_solve_cost(_ptr(D), _ptr(a), m, _ptr(b), n, PROTOCOLS[protocol],
                                 seed & (2**64 - 1), max_rounds, _ptr(src), _ptr(dst), _ptr(flow),
                                 cap, ctypes.byref(st))
    out = st.as_dict()
    out["status_name"] = STATUS.get(out["status"], str(out["status"]))
    if with_plan and out["status"] in (0, -6):
        k = out["nnz"]
        out["src"], out["dst"], out["flow"] = src[:k].copy(), dst[:k].copy(), flow[:k].copy()
    return out


def solve_batched(Xcat, acat, x_off, Ycat, bcat, y_off, pair_x=None, pair_y=None,
                  metric: str = "l2", protocol: str = "greedy", seed: int = 0,
                  num_pairs: int | None = None) -> tuple[list, int]:
    """Solve many pairs (OpenMP over pairs).  Returns (list of stats dicts,
    number of threads used)."""
    lib = _load()
    Xcat = _f64(Xcat, 2)
    Ycat = _f64(Ycat, 2)
    acat = _f64(acat, 1)
    bcat = _f64(bcat, 1)
    x_off = np.ascontiguousarray(x_off, dtype=np.int64)
    y_off = np.ascontiguousarray(y_off, dtype=np.int64)
    px = None if pair_x is None else np.ascontiguousarray(pair_x, dtype=np.int32)
    py = None if pair_y is None else np.ascontiguousarray(pair_y, dtype=np.int32)
    if num_pairs is None:
        num_pairs = len(px) if px is not None else len(x_off) - 1
    d = Xcat.shape[1]
    stats = (OracleStats * max(num_pairs, 1))()
    threads = lib.nnsemd_oracle_solve_batched(
        num_pairs, _ptr(Xcat), _ptr(acat), _ptr(x_off), _ptr(Ycat), _ptr(bcat), _ptr(y_off),
        _ptr(px), _ptr(py), d, METRICS[metric], PROTOCOLS[protocol], seed & (2**64 - 1),
        ctypes.cast(stats, ctypes.c_void_p))
    return [stats[p].as_dict() for p in range(num_pairs)], threads


def barycentric(src, dst, flow, Y, m: int) -> np.ndarray:
    """T_i = sum_j F_ij y_j / sum_j F_ij for every supplier i (NaN if none)."""
    lib = _load()
    src = np.ascontiguousarray(src, np.int32)
    dst = np.ascontiguousarray(dst, np.int32)
    flow = np.ascontiguousarray(flow, np.float64)
    Y = _f64(Y, 2)
    out = np.zeros((m, Y.shape[1]), np.float64)
    lib.nnsemd_oracle_barycentric(_ptr(src), _ptr(dst), _ptr(flow), len(src), _ptr(Y), m,
                                  Y.shape[1], _ptr(out))
    return out


def barycentric_dst(src, dst, flow, X, n: int) -> np.ndarray:
    """T_j = sum_i F_ij x_i / sum_i F_ij for every consumer j (NaN if none)."""
    lib = _load()
    src = np.ascontiguousarray(src, np.int32)
    dst = np.ascontiguousarray(dst, np.int32)
    flow = np.ascontiguousarray(flow, np.float64)
    X = _f64(X, 2)
    out = np.zeros((n, X.shape[1]), np.float64)
    lib.nnsemd_oracle_barycentric_dst(_ptr(src), _ptr(dst), _ptr(flow), len(src), _ptr(X), n,
                                      X.shape[1], _ptr(out))
    return out


def kmeans(pixels, K: int, iters: int):
    """k-means palette of an 8-bit RGB image (pixels: (P, 3) uint8): returns
    (centroids (K, 3) FP64 on the 0..255 scale, counts (K,) int64,
    assignment (P,) int32) -- the reproducible Lloyd iteration of the C file."""
    lib = _load()
    px = np.ascontiguousarray(np.asarray(pixels, np.uint8).reshape(-1, 3))
    P = px.shape[0]
    C = np.zeros((K, 3), np.float64)
    cnt = np.zeros(K, np.int64)
    asg = np.zeros(P, np.int32)
    lib.nnsemd_oracle_kmeans(_ptr(px), P, K, iters, _ptr(C), _ptr(cnt), _ptr(asg))
    return C, cnt, asg


def palette_histogram(C, counts):
    """A palette as a colour histogram: bin colours C / 255 rounded to FP32,
    masses counts / sum(counts) rounded to FP32 (both from FP64)."""
    counts = np.asarray(counts, np.int64)
    pts = (np.asarray(C, np.float64) / 255.0).astype(np.float32)
    mass = (counts.astype(np.float64) / float(counts.sum())).astype(np.float32)
    return pts, mass


def recolour(pixels, assign, colour_map):
    """Pixels recoloured through a per-bin colour map in [0,1]^3 (NaN rows
    keep the pixel's colour); uint8 (P, 3)."""
    lib = _load()
    px = np.ascontiguousarray(np.asarray(pixels, np.uint8).reshape(-1, 3))
    asg = np.ascontiguousarray(assign, np.int32)
    T = np.ascontiguousarray(colour_map, np.float64)
    out = np.zeros_like(px)
    lib.nnsemd_oracle_recolour(_ptr(px), _ptr(asg), px.shape[0], _ptr(T), _ptr(out))
    return out


def colour_transfer(ref_pixels, src_pixels, k_ref: int, k_src: int, iters: int, metric: str = "l2"):
    """Colour transfer (Sec. IV-D) step by step on the host: both palettes,
    NNS-EMD from the reference palette (suppliers) to the source palette
    (consumers), the per-consumer barycentric map, the recoloured source."""
    Cr, nr, _ = kmeans(ref_pixels, k_ref, iters)
    Cs, ns, asg = kmeans(src_pixels, k_src, iters)
    Xr, ar = palette_histogram(Cr, nr)
    Ys, bs = palette_histogram(Cs, ns)
    r = solve(Xr, ar, Ys, bs, metric=metric)
    T = barycentric_dst(r["src"], r["dst"], r["flow"], Xr, k_src)
    return {"ref_palette": Xr, "ref_mass": ar, "src_palette": Ys, "src_mass": bs, "assign": asg,
            "solve": r, "map": T, "image": recolour(src_pixels, asg, T)}


def rp_key(seed: int, round_: int, j: int) -> int:
    """Random-protocol order key (SplitMix64 of the (seed, round, j) counter)."""
    return int(_load().nnsemd_oracle_rp_key(seed & (2**64 - 1), round_, j))
