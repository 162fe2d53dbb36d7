"""Thin ctypes binding of libnnsemd.so (include/nnsemd.h).

Argument marshalling only: every step of NNS-EMD runs in the library's HIP
kernels.  Tensors must already live on the GPU; PyTorch provides the device
memory and the stream.  There is no CPU fallback: if the library or a GPU is
missing the calls raise.
"""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("NNSEMD_LIB") or os.path.join(_PKG, "libnnsemd.so")

STATUS = {
    0: "OK", -1: "INVALID_ARG", -2: "MASS_MISMATCH", -3: "CAPACITY", -4: "OUT_OF_MEMORY",
    -5: "DEVICE", -6: "NOT_CONVERGED", -7: "UNSUPPORTED",
}
METRICS = {"l2": 0, "sqeuclidean": 1, "l1": 2}
PROTOCOLS = {"greedy": 0, "random": 1}
MODES = {"fp32": 0, "bf16_mfma_refine": 1}
DTYPES = {"f32": 0, "bf16": 1, "f64": 2}

# nnsemd_stats_t as a numpy record (64 bytes, written by the device).
STATS_DTYPE = np.dtype([("status", "<i4"), ("rounds", "<i4"), ("nnz", "<i8"), ("work", "<i8"),
                        ("rescored", "<i8"), ("residual_src", "<f8"), ("residual_dst", "<f8"),
                        ("near_ties_nn", "<i8"), ("near_ties_order", "<i8")])
STATS_BYTES = STATS_DTYPE.itemsize

EXPORTS = ["nnsemd_create", "nnsemd_destroy", "nnsemd_status_string", "nnsemd_last_error",
           "emd_approx", "emd_approx_map", "emd_approx_batched", "emd_barycentric_map",
           "emd_approx_cost", "emd_approx_cost_batched", "nnsemd_colour_transfer",
           "emd_approx_batched_noalloc",
           "nnsemd_sg_num_params", "nnsemd_sg_embed", "nnsemd_sg_predict", "nnsemd_sg_loss_grad",
           "nnsemd_sg_train_step", "nnsemd_topk_smallest_f32", "nnsemd_topk_smallest_f64", "nnsemd_sg_retrieve",
           "nnsemd_autotune", "nnsemd_tuning_save", "nnsemd_tuning_load",
           "nnsemd_tuning_clear", "nnsemd_autotune_docs", "nnsemd_tuning_set_docs"]
SG_HIDDEN = 256


class NNSEMDError(RuntimeError):
    def __init__(self, status: int, msg: str = ""):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Options(ctypes.Structure):
    _fields_ = [("protocol", ctypes.c_int32), ("mode", ctypes.c_int32),
                ("max_rounds", ctypes.c_int64), ("seed", ctypes.c_uint64),
                ("threads", ctypes.c_int32), ("schedule", ctypes.c_int32),
                ("path", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class Tuning(ctypes.Structure):
    _fields_ = [("threads", ctypes.c_int32), ("split", ctypes.c_int32),
                ("ms_best", ctypes.c_float), ("ms_default", ctypes.c_float)]


class DocTuning(ctypes.Structure):
    _fields_ = [("split", ctypes.c_int32), ("ms_split", ctypes.c_float), ("ms_fused", ctypes.c_float)]


_lock = threading.Lock()
_lib = None
_handles: dict[int, ctypes.c_void_p] = {}


def load_library():
    """Load libnnsemd.so (raises if it was not built)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() (hipcc, gfx950) first")
        lib = ctypes.CDLL(LIB_PATH)
        P, I32, I64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        lib.nnsemd_create.argtypes = [ctypes.POINTER(P), I32]
        lib.nnsemd_create.restype = I32
        lib.nnsemd_destroy.argtypes = [P]
        lib.nnsemd_destroy.restype = I32
        lib.nnsemd_status_string.argtypes = [I32]
        lib.nnsemd_status_string.restype = ctypes.c_char_p
        lib.nnsemd_last_error.argtypes = [P]
        lib.nnsemd_last_error.restype = ctypes.c_char_p
        lib.emd_approx.argtypes = [P, P, P, I64, P, P, I64, I32, I32, I32, ctypes.POINTER(Options),
                                   P, P, P, P, I64, P, P]
        lib.emd_approx.restype = I32
        lib.emd_approx_batched.argtypes = [P, I64, P, P, P, I64, P, P, P, I64, P, P, I64, I64, I32, I32,
                                           I32, ctypes.POINTER(Options), P, P, P, P, P, P, P]
        lib.emd_approx_batched.restype = I32
        lib.emd_approx_batched_noalloc.argtypes = lib.emd_approx_batched.argtypes
        lib.emd_approx_batched_noalloc.restype = I32
        lib.emd_approx_map.argtypes = [P, P, P, I64, P, P, I64, I32, I32, I32, ctypes.POINTER(Options),
                                       P, P, P, P, P, I64, P, P]
        lib.emd_approx_map.restype = I32
        lib.emd_barycentric_map.argtypes = [P, P, P, P, I64, P, P, I64, I32, I64, I32, P, P]
        lib.emd_barycentric_map.restype = I32
        lib.emd_approx_cost.argtypes = [P, P, I32, P, I64, P, I64, ctypes.POINTER(Options), P, P, P, P, I64, P, P]
        lib.emd_approx_cost.restype = I32
        lib.emd_approx_cost_batched.argtypes = [P, I64, P, P, I32, P, P, P, P, I64, I64, ctypes.POINTER(Options),
                                                P, P, P, P, P, P, P]
        lib.emd_approx_cost_batched.restype = I32
        lib.nnsemd_colour_transfer.argtypes = [P, P, I64, P, I64, I32, I32, I32, I32, ctypes.POINTER(Options), P, P,
                                               P, P, P, P, P, P, P]
        lib.nnsemd_colour_transfer.restype = I32
        F32 = ctypes.c_float
        lib.nnsemd_sg_num_params.argtypes = []
        lib.nnsemd_sg_num_params.restype = I64
        lib.nnsemd_sg_embed.argtypes = [P, P, P, P, P, I64, I64, P, P]
        lib.nnsemd_sg_predict.argtypes = [P, P, P, I64, P, I64, P, P, I64, P, P]
        lib.nnsemd_sg_loss_grad.argtypes = [P, P, P, P, P, I64, I64, P, P, P, P]
        lib.nnsemd_sg_train_step.argtypes = [P, P, P, P, I64, F32, P, P, P, I64, I64, P, P, P, P]
        lib.nnsemd_topk_smallest_f32.argtypes = [P, P, I64, I32, P, P]
        lib.nnsemd_topk_smallest_f64.argtypes = [P, P, I64, I32, P, P]
        lib.nnsemd_sg_retrieve.argtypes = [P, P, P, I64, P, P, I64, P, P, P, I64, I32, I32, P, P, P, P, P]
        lib.nnsemd_autotune.argtypes = [P, I32, I32, I64, I64, I64, ctypes.POINTER(Tuning), P]
        lib.nnsemd_tuning_save.argtypes = [P, ctypes.c_char_p]
        lib.nnsemd_tuning_load.argtypes = [P, ctypes.c_char_p]
        lib.nnsemd_tuning_clear.argtypes = [P]
        lib.nnsemd_autotune_docs.argtypes = [P, I32, I64, I64, I64, ctypes.POINTER(DocTuning), P]
        lib.nnsemd_tuning_set_docs.argtypes = [P, I32, I64, I32]
        for fn in ("nnsemd_autotune", "nnsemd_tuning_save", "nnsemd_tuning_load", "nnsemd_tuning_clear",
                   "nnsemd_autotune_docs", "nnsemd_tuning_set_docs"):
            getattr(lib, fn).restype = I32
        for fn in ("nnsemd_sg_embed", "nnsemd_sg_predict", "nnsemd_sg_loss_grad", "nnsemd_sg_train_step",
                   "nnsemd_topk_smallest_f32", "nnsemd_topk_smallest_f64", "nnsemd_sg_retrieve"):
            getattr(lib, fn).restype = I32
        _lib = lib
        return lib


def handle(device: int = 0):
    """Library handle for a device (created once per process)."""
    lib = load_library()
    with _lock:
        h = _handles.get(device)
        if h is None:
            h = ctypes.c_void_p()
            st = lib.nnsemd_create(ctypes.byref(h), device)
            if st != 0:
                raise NNSEMDError(st, "nnsemd_create failed")
            _handles[device] = h
        return h


def _check(lib, h, st):
    if st != 0:
        raise NNSEMDError(st, lib.nnsemd_last_error(h).decode())


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


SCHEDULES = {"longest_first": 0, "as_given": 1}
PATHS = {"auto": 0, "on_chip": 1, "multi": 2, "multi_no_tail": 3}


def _options(protocol, mode, max_rounds, seed, threads, schedule="longest_first", path="auto"):
    return Options(PROTOCOLS[protocol], MODES[mode], int(max_rounds), int(seed) & (2**64 - 1),
                   int(threads), SCHEDULES[schedule], PATHS[path], 0)


def _stream(torch, device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _require(t, dtype, name):
    if t is None:
        raise ValueError(f"{name} is required")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor (no CPU path exists)")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def stats_numpy(stats_tensor) -> np.ndarray:
    """Copy a device stats buffer to host and view it as STATS_DTYPE records."""
    return stats_tensor.cpu().numpy().view(STATS_DTYPE)


def emd_approx(X, a, Y, b, metric: str = "l2", *, plan: bool = True, protocol: str = "greedy",
               mode: str = "fp32", seed: int = 0, max_rounds: int = 0, threads: int = 0,
               path: str = "auto", out: dict | None = None) -> dict:
    """NNS-EMD of one pair on the GPU.  X (m x d) / a (m): suppliers; Y (n x d)
    / b (n): consumers; FP32 CUDA tensors.  Returns device tensors: cost (1,),
    stats (STATS_BYTES uint8), and with plan=True plan_src/plan_dst/plan_flow of
    capacity m + n - 1 (the first stats.nnz entries are the plan).  Runs
    asynchronously on the current stream."""
    import torch
    lib = load_library()
    dev = X.device.index if X.device.index is not None else torch.cuda.current_device()
    h = handle(dev)
    dt = torch.bfloat16 if mode == "bf16_mfma_refine" else torch.float32
    _require(X, dt, "X")
    _require(Y, dt, "Y")
    _require(a, torch.float32, "a")
    _require(b, torch.float32, "b")
    m, n = X.shape[0], Y.shape[0]
    d = X.shape[1] if X.dim() == 2 else 1
    o = out or {}
    cost = o.get("cost")
    if cost is None:
        cost = torch.empty(1, dtype=torch.float64, device=X.device)
    stats = o.get("stats")
    if stats is None:
        stats = torch.empty(STATS_DTYPE.itemsize, dtype=torch.uint8, device=X.device)
    cap = max(m + n - 1, 1)
    src = dst = flow = None
    if plan:
        src = o.get("plan_src") if o.get("plan_src") is not None else torch.empty(cap, dtype=torch.int32, device=X.device)
        dst = o.get("plan_dst") if o.get("plan_dst") is not None else torch.empty(cap, dtype=torch.int32, device=X.device)
        flow = o.get("plan_flow") if o.get("plan_flow") is not None else torch.empty(cap, dtype=torch.float64, device=X.device)
        cap = src.numel()
    opts = _options(protocol, mode, max_rounds, seed, threads, path=path)
    st = lib.emd_approx(h, _ptr(X), _ptr(a), m, _ptr(Y), _ptr(b), n, d,
                        DTYPES["bf16" if mode == "bf16_mfma_refine" else "f32"], METRICS[metric],
                        ctypes.byref(opts), _ptr(cost), _ptr(src), _ptr(dst), _ptr(flow),
                        cap if plan else 0, _ptr(stats), _stream(torch, dev))
    _check(lib, h, st)
    return {"cost": cost, "stats": stats, "plan_src": src, "plan_dst": dst, "plan_flow": flow}


def emd_approx_map(X, a, Y, b, metric: str = "l2", *, plan: bool = True, protocol: str = "greedy",
                   seed: int = 0, max_rounds: int = 0, path: str = "auto") -> dict:
    """emd_approx plus the per-supplier barycentric map (m x d FP64 device
    tensor 'map').  On chip (asynchronous) when the pair fits one workgroup,
    else on the multi-workgroup path."""
    import torch
    lib = load_library()
    dev = X.device.index if X.device.index is not None else torch.cuda.current_device()
    h = handle(dev)
    for t, nm in ((X, "X"), (Y, "Y"), (a, "a"), (b, "b")):
        _require(t, torch.float32, nm)
    m, n = X.shape[0], Y.shape[0]
    d = X.shape[1] if X.dim() == 2 else 1
    cost = torch.empty(1, dtype=torch.float64, device=X.device)
    mp = torch.empty((max(m, 1), d), dtype=torch.float64, device=X.device)
    stats = torch.empty(STATS_DTYPE.itemsize, dtype=torch.uint8, device=X.device)
    cap = max(m + n - 1, 1)
    src = dst = flow = None
    if plan:
        src = torch.empty(cap, dtype=torch.int32, device=X.device)
        dst = torch.empty(cap, dtype=torch.int32, device=X.device)
        flow = torch.empty(cap, dtype=torch.float64, device=X.device)
    opts = _options(protocol, "fp32", max_rounds, seed, 0, path=path)
    st = lib.emd_approx_map(h, _ptr(X), _ptr(a), m, _ptr(Y), _ptr(b), n, d, DTYPES["f32"], METRICS[metric],
                            ctypes.byref(opts), _ptr(cost), _ptr(mp), _ptr(src), _ptr(dst), _ptr(flow),
                            cap if plan else 0, _ptr(stats), _stream(torch, dev))
    _check(lib, h, st)
    return {"cost": cost, "map": mp[:m], "stats": stats, "plan_src": src, "plan_dst": dst, "plan_flow": flow}


def _d_dtype(D):
    import torch
    if D.dtype == torch.float32:
        return DTYPES["f32"]
    if D.dtype == torch.float64:
        return DTYPES["f64"]
    raise ValueError("D must be float32 or float64")


def emd_approx_cost(D, a, b, *, plan: bool = True, protocol: str = "greedy", seed: int = 0,
                    max_rounds: int = 0, schedule: str = "longest_first", out: dict | None = None) -> dict:
    """NNS-EMD of one pair from its ground-distance matrix D (m x n device
    tensor, FP32 or FP64; Algorithm 1's input) and FP32 masses a (m), b (n).
    Returns device tensors cost (1,), stats and the plan (capacity m+n-1)."""
    import torch
    lib = load_library()
    dev = _dev_of(D)
    h = handle(dev)
    _require(D, D.dtype, "D")
    _require(a, torch.float32, "a")
    _require(b, torch.float32, "b")
    m, n = a.numel(), b.numel()
    if D.numel() != m * n:
        raise ValueError("D must hold m x n entries")
    o = out or {}
    cost = o.get("cost") if o.get("cost") is not None else torch.empty(1, dtype=torch.float64, device=D.device)
    stats = o.get("stats") if o.get("stats") is not None else \
        torch.empty(STATS_BYTES, dtype=torch.uint8, device=D.device)
    cap = max(m + n - 1, 1)
    src = dst = flow = None
    if plan:
        src = torch.empty(cap, dtype=torch.int32, device=D.device)
        dst = torch.empty(cap, dtype=torch.int32, device=D.device)
        flow = torch.empty(cap, dtype=torch.float64, device=D.device)
    opts = _options(protocol, "fp32", max_rounds, seed, 0, schedule)
    st = lib.emd_approx_cost(h, _ptr(D), _d_dtype(D), _ptr(a), m, _ptr(b), n, ctypes.byref(opts), _ptr(cost),
                             _ptr(src), _ptr(dst), _ptr(flow), cap if plan else 0, _ptr(stats), _stream(torch, dev))
    _check(lib, h, st)
    return {"cost": cost, "stats": stats, "plan_src": src, "plan_dst": dst, "plan_flow": flow}


def emd_approx_cost_batched(Dcat, d_off, acat, a_off, bcat, b_off, *, max_m: int, max_n: int, plan_off=None,
                            protocol: str = "greedy", seed: int = 0, max_rounds: int = 0,
                            schedule: str = "longest_first", out: dict | None = None) -> dict:
    """Many pairs of given distance matrices in one launch (offsets are int64
    device tensors of num_pairs + 1 entries).  Asynchronous."""
    import torch
    lib = load_library()
    dev = _dev_of(Dcat)
    h = handle(dev)
    for t, nm in ((d_off, "d_off"), (a_off, "a_off"), (b_off, "b_off")):
        _require(t, torch.int64, nm)
    _require(acat, torch.float32, "acat")
    _require(bcat, torch.float32, "bcat")
    P = a_off.numel() - 1
    o = out or {}
    costs = o.get("costs") if o.get("costs") is not None else \
        torch.empty(max(P, 1), dtype=torch.float64, device=Dcat.device)
    stats = o.get("stats") if o.get("stats") is not None else \
        torch.empty(max(P, 1) * STATS_BYTES, dtype=torch.uint8, device=Dcat.device)
    src = dst = flow = None
    if plan_off is not None:
        _require(plan_off, torch.int64, "plan_off")
        total = int(plan_off[-1].item())
        src = torch.empty(max(total, 1), dtype=torch.int32, device=Dcat.device)
        dst = torch.empty(max(total, 1), dtype=torch.int32, device=Dcat.device)
        flow = torch.empty(max(total, 1), dtype=torch.float64, device=Dcat.device)
    opts = _options(protocol, "fp32", max_rounds, seed, 0, schedule)
    st = lib.emd_approx_cost_batched(h, P, _ptr(Dcat), _ptr(d_off), _d_dtype(Dcat), _ptr(acat), _ptr(a_off),
                                     _ptr(bcat), _ptr(b_off), int(max_m), int(max_n), ctypes.byref(opts),
                                     _ptr(costs), _ptr(src), _ptr(dst), _ptr(flow), _ptr(plan_off), _ptr(stats),
                                     _stream(torch, dev))
    _check(lib, h, st)
    return {"costs": costs, "stats": stats, "plan_src": src, "plan_dst": dst, "plan_flow": flow}


def colour_transfer(ref_rgb, src_rgb, k_ref: int = 256, k_src: int = 256, iters: int = 10, metric: str = "l2",
                    protocol: str = "greedy", seed: int = 0, out: dict | None = None) -> dict:
    """Colour transfer by NNS-EMD (uint8 device images of shape (P, 3) or
    (H, W, 3)): k-means palettes, NNS-EMD reference -> source palette,
    recoloured source through the per-consumer barycentric map.  Returns
    device tensors: image (like src_rgb), palettes, masses, the source
    assignment, cost and stats.  Asynchronous."""
    import torch
    lib = load_library()
    dev = _dev_of(src_rgb)
    h = handle(dev)
    _require(ref_rgb, torch.uint8, "ref_rgb")
    _require(src_rgb, torch.uint8, "src_rgb")
    Pr, Ps = ref_rgb.numel() // 3, src_rgb.numel() // 3
    o = out or {}
    d = src_rgb.device
    img = o.get("image") if o.get("image") is not None else torch.empty_like(src_rgb)
    rp = torch.empty((k_ref, 3), dtype=torch.float32, device=d)
    rm = torch.empty(k_ref, dtype=torch.float32, device=d)
    sp = torch.empty((k_src, 3), dtype=torch.float32, device=d)
    sm = torch.empty(k_src, dtype=torch.float32, device=d)
    asg = torch.empty(Ps, dtype=torch.int32, device=d)
    cost = torch.empty(1, dtype=torch.float64, device=d)
    stats = torch.empty(STATS_BYTES, dtype=torch.uint8, device=d)
    opts = _options(protocol, "fp32", 0, seed, 0)
    st = lib.nnsemd_colour_transfer(h, _ptr(ref_rgb), Pr, _ptr(src_rgb), Ps, k_ref, k_src, iters, METRICS[metric],
                                    ctypes.byref(opts), _ptr(img), _ptr(rp), _ptr(rm), _ptr(sp), _ptr(sm),
                                    _ptr(asg), _ptr(cost), _ptr(stats), _stream(torch, dev))
    _check(lib, h, st)
    return {"image": img, "ref_palette": rp, "ref_mass": rm, "src_palette": sp, "src_mass": sm, "assign": asg,
            "cost": cost, "stats": stats}


MAP_SIDES = {"suppliers": 0, "consumers": 1}


def barycentric_map(plan_src, plan_dst, plan_flow, P, rows: int, side: str = "suppliers", nnz=None, out=None):
    """Barycentric map of a device plan (FP64 rows x d).  side 'suppliers':
    P = consumer points, rows = m; 'consumers': P = supplier points, rows = n.
    nnz: optional device int64 tensor (or view, e.g. of a stats record) with
    the number of plan entries in use; default all of them.  Asynchronous."""
    import torch
    lib = load_library()
    dev = _dev_of(P)
    h = handle(dev)
    _require(P, torch.float32, "P")
    for t, nm, dt in ((plan_src, "plan_src", torch.int32), (plan_dst, "plan_dst", torch.int32),
                      (plan_flow, "plan_flow", torch.float64)):
        _require(t, dt, nm)
    d = P.shape[1] if P.dim() == 2 else 1
    m = out if out is not None else torch.empty((max(rows, 1), d), dtype=torch.float64, device=P.device)
    st = lib.emd_barycentric_map(h, _ptr(plan_src), _ptr(plan_dst), _ptr(plan_flow), plan_src.numel(), _ptr(nnz),
                                 _ptr(P), P.shape[0], d, int(rows), MAP_SIDES[side], _ptr(m), _stream(torch, dev))
    _check(lib, h, st)
    return m[:rows]


def stats_field(stats_tensor, index: int, field: str):
    """Device view of one int64 field of a stats record (e.g. 'nnz'), to pass
    as a device count without a host round trip."""
    off = STATS_DTYPE.fields[field][1] + index * STATS_BYTES
    return stats_tensor[off:off + 8].view(__import__("torch").int64)


def plan_offsets(m_sizes, n_sizes) -> np.ndarray:
    """Host helper: plan_off with capacity m_p + n_p - 1 per pair (int64)."""
    cap = np.maximum(np.asarray(m_sizes, np.int64) + np.asarray(n_sizes, np.int64) - 1, 0)
    off = np.zeros(len(cap) + 1, np.int64)
    off[1:] = np.cumsum(cap)
    return off


def emd_approx_batched(Xcat, acat, x_off, Ycat, bcat, y_off, *, max_m: int, max_n: int,
                       pair_x=None, pair_y=None, num_pairs: int | None = None, metric: str = "l2",
                       plan_off=None, protocol: str = "greedy", mode: str = "fp32", seed: int = 0,
                       max_rounds: int = 0, threads: int = 0, schedule: str = "longest_first",
                       out: dict | None = None, noalloc: bool = False) -> dict:
    """NNS-EMD of many ragged pairs in one persistent launch.  Offsets and
    pair tables are int64/int32 CUDA tensors; max_m/max_n are host bounds on
    the set sizes.  With plan_off (CUDA int64, num_pairs + 1) the plans are
    written too.  Returns device tensors costs (num_pairs,), stats
    (num_pairs * STATS_BYTES uint8) and the plan buffers.  Asynchronous.
    noalloc: the entry point that allocates nothing (point path only).  Pass
    every output in `out` (and plan_total with a plan) so that this binding
    allocates nothing either."""
    import torch
    lib = load_library()
    dev = Xcat.device.index if Xcat.device.index is not None else torch.cuda.current_device()
    h = handle(dev)
    dt = torch.bfloat16 if mode == "bf16_mfma_refine" else torch.float32
    _require(Xcat, dt, "Xcat")
    _require(Ycat, dt, "Ycat")
    _require(acat, torch.float32, "acat")
    _require(bcat, torch.float32, "bcat")
    _require(x_off, torch.int64, "x_off")
    _require(y_off, torch.int64, "y_off")
    if pair_x is not None:
        _require(pair_x, torch.int32, "pair_x")
    if pair_y is not None:
        _require(pair_y, torch.int32, "pair_y")
    nx, ny = x_off.numel() - 1, y_off.numel() - 1
    if num_pairs is None:
        num_pairs = pair_x.numel() if pair_x is not None else nx
    d = Xcat.shape[1] if Xcat.dim() == 2 else 1
    o = out or {}
    costs = o.get("costs")
    if costs is None:
        costs = torch.empty(max(num_pairs, 1), dtype=torch.float64, device=Xcat.device)
    stats = o.get("stats")
    if stats is None:
        stats = torch.empty(max(num_pairs, 1) * STATS_DTYPE.itemsize, dtype=torch.uint8, device=Xcat.device)
    src = dst = flow = None
    if plan_off is not None:
        _require(plan_off, torch.int64, "plan_off")
        total = o.get("plan_total")
        if total is None:
            total = int(plan_off[-1].item())
        src = o.get("plan_src") if o.get("plan_src") is not None else torch.empty(max(total, 1), dtype=torch.int32, device=Xcat.device)
        dst = o.get("plan_dst") if o.get("plan_dst") is not None else torch.empty(max(total, 1), dtype=torch.int32, device=Xcat.device)
        flow = o.get("plan_flow") if o.get("plan_flow") is not None else torch.empty(max(total, 1), dtype=torch.float64, device=Xcat.device)
    opts = _options(protocol, mode, max_rounds, seed, threads, schedule)
    fn = lib.emd_approx_batched_noalloc if noalloc else lib.emd_approx_batched
    st = fn(
        h, num_pairs, _ptr(Xcat), _ptr(acat), _ptr(x_off), nx, _ptr(Ycat), _ptr(bcat), _ptr(y_off), ny,
        _ptr(pair_x), _ptr(pair_y), int(max_m), int(max_n), d,
        DTYPES["bf16" if mode == "bf16_mfma_refine" else "f32"], METRICS[metric], ctypes.byref(opts),
        _ptr(costs), _ptr(src), _ptr(dst), _ptr(flow), _ptr(plan_off), _ptr(stats), _stream(torch, dev))
    _check(lib, h, st)
    return {"costs": costs, "stats": stats, "plan_src": src, "plan_dst": dst, "plan_flow": flow,
            "plan_off": plan_off}


# ---------------------------------------------------------------- surrogate
def _dev_of(t):
    import torch
    return t.device.index if t.device.index is not None else torch.cuda.current_device()


def sg_num_params() -> int:
    return int(load_library().nnsemd_sg_num_params())


def sg_embed(theta, X, a, set_off, out=None):
    """Pooled embeddings (num_sets x 256 FP32) of concatenated 3-D point sets."""
    import torch
    lib = load_library()
    dev = _dev_of(X)
    h = handle(dev)
    _require(theta, torch.float32, "theta")
    _require(X, torch.float32, "X")
    _require(a, torch.float32, "a")
    _require(set_off, torch.int64, "set_off")
    S = set_off.numel() - 1
    E = out if out is not None else torch.empty((max(S, 1), SG_HIDDEN), dtype=torch.float32, device=X.device)
    st = lib.nnsemd_sg_embed(h, _ptr(theta), _ptr(X), _ptr(a), _ptr(set_off), S, X.shape[0], _ptr(E),
                             _stream(torch, dev))
    _check(lib, h, st)
    return E[:S]


def sg_predict(theta, Eq, Ec, q_idx=None, c_idx=None, num_pairs=None, out=None):
    """Surrogate EMD of pairs of embedding rows."""
    import torch
    lib = load_library()
    dev = _dev_of(Eq)
    h = handle(dev)
    for t, nm in ((theta, "theta"), (Eq, "Eq"), (Ec, "Ec")):
        _require(t, torch.float32, nm)
    if num_pairs is None:
        num_pairs = c_idx.numel() if c_idx is not None else Ec.shape[0]
    pred = out if out is not None else torch.empty(max(num_pairs, 1), dtype=torch.float32, device=Eq.device)
    st = lib.nnsemd_sg_predict(h, _ptr(theta), _ptr(Eq), Eq.shape[0], _ptr(Ec), Ec.shape[0], _ptr(q_idx),
                               _ptr(c_idx), num_pairs, _ptr(pred), _stream(torch, dev))
    _check(lib, h, st)
    return pred[:num_pairs]


def sg_loss_grad(theta, X, a, set_off, labels, grad=None):
    """(loss (1,), grad (num_params,)) of one training batch (pair b = sets 2b, 2b+1)."""
    import torch
    lib = load_library()
    dev = _dev_of(X)
    h = handle(dev)
    loss = torch.empty(1, dtype=torch.float32, device=X.device)
    if grad is None:
        grad = torch.empty(sg_num_params(), dtype=torch.float32, device=X.device)
    st = lib.nnsemd_sg_loss_grad(h, _ptr(theta), _ptr(X), _ptr(a), _ptr(set_off), labels.numel(), X.shape[0],
                                 _ptr(labels), _ptr(loss), _ptr(grad), _stream(torch, dev))
    _check(lib, h, st)
    return loss, grad


def sg_train_step(theta, m, v, step, lr, X, a, set_off, labels, loss=None, grad=None):
    """One Adam step on theta (in place); returns the batch loss tensor (1,)."""
    import torch
    lib = load_library()
    dev = _dev_of(X)
    h = handle(dev)
    if loss is None:
        loss = torch.empty(1, dtype=torch.float32, device=X.device)
    st = lib.nnsemd_sg_train_step(h, _ptr(theta), _ptr(m), _ptr(v), int(step), float(lr), _ptr(X), _ptr(a),
                                  _ptr(set_off), labels.numel(), X.shape[0], _ptr(labels), _ptr(loss), _ptr(grad),
                                  _stream(torch, dev))
    _check(lib, h, st)
    return loss


def topk_smallest(values, k: int, out=None):
    """Indices (int32) of the k smallest values, ascending by (value, index)."""
    import torch
    lib = load_library()
    dev = _dev_of(values)
    h = handle(dev)
    idx = out if out is not None else torch.empty(k, dtype=torch.int32, device=values.device)
    if values.dtype == torch.float32:
        st = lib.nnsemd_topk_smallest_f32(h, _ptr(values), values.numel(), k, _ptr(idx), _stream(torch, dev))
    elif values.dtype == torch.float64:
        st = lib.nnsemd_topk_smallest_f64(h, _ptr(values), values.numel(), k, _ptr(idx), _stream(torch, dev))
    else:
        raise ValueError("values must be float32 or float64")
    _check(lib, h, st)
    return idx


def sg_retrieve(theta, index_E, Xq, aq, Ycat, bcat, y_off, max_n: int, keep: int = 1000, top: int = 10,
                out: dict | None = None) -> dict:
    """Surrogate-pruned retrieval: keep the `keep` candidates of smallest
    predicted EMD, re-rank them with NNS-EMD, return the `top` best
    (idx int32, cost float64) plus the kept indices and their stats."""
    import torch
    lib = load_library()
    dev = _dev_of(Xq)
    h = handle(dev)
    o = out or {}
    d = Xq.device
    idx = o.get("idx") if o.get("idx") is not None else torch.empty(top, dtype=torch.int32, device=d)
    cost = o.get("cost") if o.get("cost") is not None else torch.empty(top, dtype=torch.float64, device=d)
    kept = o.get("kept") if o.get("kept") is not None else torch.empty(keep, dtype=torch.int32, device=d)
    kst = o.get("kept_stats") if o.get("kept_stats") is not None else \
        torch.empty(keep * STATS_DTYPE.itemsize, dtype=torch.uint8, device=d)
    st = lib.nnsemd_sg_retrieve(h, _ptr(theta), _ptr(index_E), index_E.shape[0], _ptr(Xq), _ptr(aq), Xq.shape[0],
                                _ptr(Ycat), _ptr(bcat), _ptr(y_off), int(max_n), keep, top, _ptr(idx), _ptr(cost),
                                _ptr(kept), _ptr(kst), _stream(torch, dev))
    _check(lib, h, st)
    return {"idx": idx, "cost": cost, "kept": kept, "kept_stats": kst}


# ---------------------------------------------------------------- autotuning
def autotune(d: int, metric: str, max_m: int, max_n: int, num_pairs: int = 1024, device: int = 0) -> dict:
    """Time the batched point path's launch configurations on synthetic pairs
    of this shape and record the fastest in the device's handle."""
    import torch
    lib = load_library()
    h = handle(device)
    t = Tuning()
    st = lib.nnsemd_autotune(h, d, METRICS[metric], max_m, max_n, num_pairs, ctypes.byref(t),
                             _stream(torch, device))
    _check(lib, h, st)
    return {"threads": t.threads, "split": t.split, "ms_best": t.ms_best, "ms_default": t.ms_default}


def autotune_docs(d: int, max_m: int, max_n: int, num_pairs: int = 1024, device: int = 0) -> dict:
    """Time the BF16 high-dimensional path's launch forms (split key-tile
    kernel, or tiles fused into the rounds kernel) on synthetic pairs of this
    shape and record the faster in the device's handle."""
    import torch
    lib = load_library()
    h = handle(device)
    t = DocTuning()
    st = lib.nnsemd_autotune_docs(h, d, max_m, max_n, num_pairs, ctypes.byref(t), _stream(torch, device))
    _check(lib, h, st)
    return {"form": "split" if t.split else "fused", "ms_split": t.ms_split, "ms_fused": t.ms_fused}


def tuning_set_docs(d: int, max_side: int, form: str, device: int = 0):
    """Record the BF16 high-dimensional path's launch form by hand for the
    (d, max side) class: "split" (its tile pass runs stripe by stripe over a
    supplier set that every pair shares, else per pair), "split_per_pair"
    (the per-pair tile pass always) or "fused"."""
    lib = load_library()
    h = handle(device)
    forms = {"fused": 0, "split": 1, "split_per_pair": 2}
    if form not in forms:
        raise ValueError("form is 'split', 'split_per_pair' or 'fused'")
    _check(lib, h, lib.nnsemd_tuning_set_docs(h, d, max_side, forms[form]))


def tuning_save(path: str, device: int = 0):
    lib = load_library()
    h = handle(device)
    _check(lib, h, lib.nnsemd_tuning_save(h, path.encode()))


def tuning_load(path: str, device: int = 0):
    lib = load_library()
    h = handle(device)
    _check(lib, h, lib.nnsemd_tuning_load(h, path.encode()))


def tuning_reset(device: int = 0):
    """Forget every recorded launch configuration (back to the default)."""
    lib = load_library()
    h = handle(device)
    _check(lib, h, lib.nnsemd_tuning_clear(h))
