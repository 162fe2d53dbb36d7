"""CPU-side checks of the boundary: the library loads without a GPU and
exports every entry point that include/nnsemd.h declares; the binding's
stats record matches the header's struct layout."""
import ctypes
import os
import re

from paper_2401_07378_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    txt = open(os.path.join(ROOT, "include", "nnsemd.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b([a-z_0-9]+)\s*\(", txt)) - {"if", "sizeof"})


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(binding.LIB_PATH)
    names = declared_functions()
    assert "emd_approx" in names and "emd_approx_batched" in names
    for name in names:
        assert hasattr(lib, name), name
    assert set(binding.EXPORTS) <= set(names)


def test_status_strings_without_gpu():
    lib = binding.load_library()
    for code in binding.STATUS:
        assert lib.nnsemd_status_string(code)
    assert lib.nnsemd_last_error(None) == b""


def test_stats_record_layout():
    # int32 status, int32 rounds, int64 nnz, work, rescored, double x2,
    # int64 near_ties_nn, near_ties_order
    assert binding.STATS_DTYPE.itemsize == 64
    assert binding.STATS_DTYPE.fields["residual_dst"][1] == 40
    assert binding.STATS_DTYPE.fields["near_ties_order"][1] == 56
    assert ctypes.sizeof(binding.Options) == 40


def test_null_handle_is_rejected():
    lib = binding.load_library()
    assert lib.emd_approx(None, None, None, 0, None, None, 0, 2, 0, 0, None, None, None, None, None, 0,
                          None, None) == -1
