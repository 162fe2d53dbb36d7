"""Host checks of the measured-traffic figures that bench.py reports
(CPU only).  Each committed rocprofv3 counter summary carries the hash of
the kernel sources it was taken on; bench.py reports its bytes only while
that hash matches the sources, and null after a kernel change."""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _load(path):
    with open(path) as f:
        return json.load(f)


def test_point_path_traffic_file_is_consistent():
    t = _load(bench.TRAFFIC_FILE)
    want = (t["fetch_kib_per_dispatch"] * t["fetch_scale"] + t["write_kib_per_dispatch"] * t["write_scale"]) * 1024
    assert abs(t["bytes_per_launch"] - want) <= 1e-6 * want + 1024
    got = bench.measured_traffic(0)
    if t["source_hash"] == bench.kernel_source_hash():
        assert got == t["bytes_per_launch"]
    else:
        assert got is None


def test_document_traffic_file_is_consistent():
    t = _load(bench.DOC_TRAFFIC_FILE)
    ks = t["kernels"]
    # every kernel of one split-form call: norms, stripe list, tile pass, rounds
    for name in ("doc_xnorm_kernel", "doc_stripe_reset_kernel", "doc_stripe_list_kernel",
                 "doc_tile_shared_kernel", "doc_pair_kernel"):
        assert any(k.startswith(name) for k in ks), name
    want = sum(v["fetch_kib_per_dispatch"] * t["fetch_scale"] + v["write_kib_per_dispatch"] * t["write_scale"]
               for v in ks.values()) * 1024
    assert abs(t["bytes_per_call"] - want) <= 1e-6 * want + 1024
    got = bench.measured_doc_traffic()
    if t["source_hash"] == bench.doc_kernel_source_hash():
        assert got == t["bytes_per_call"]
    else:
        assert got is None


def test_traffic_is_null_for_changed_sources(tmp_path, monkeypatch):
    t = _load(bench.DOC_TRAFFIC_FILE)
    t["source_hash"] = "0" * 16
    p = tmp_path / "doc_traffic.json"
    p.write_text(json.dumps(t))
    monkeypatch.setattr(bench, "DOC_TRAFFIC_FILE", str(p))
    assert bench.measured_doc_traffic() is None
