"""The colour-transfer application (Sec. IV-D) through the C ABI against the
oracle's step-by-step run: k-means palettes (bit-identical centroids as
FP32 bins, masses and pixel assignments), the NNS-EMD plan between the
palettes, and the recoloured source image byte for byte."""
import numpy as np
import pytest

import oracle
from paper_2401_07378_amd import workloads as W
from tests.gpu_helpers import to_dev

pytestmark = pytest.mark.gpu


def _run(ref, src, k_ref, k_src, iters, metric="l2"):
    import torch
    from paper_2401_07378_amd import binding
    r = binding.colour_transfer(to_dev(ref.reshape(-1, 3)), to_dev(src.reshape(-1, 3)), k_ref, k_src, iters, metric)
    torch.cuda.synchronize()
    out = {k: v.cpu().numpy() for k, v in r.items()}
    out["stats"] = binding.stats_numpy(r["stats"])[0]
    return out


@pytest.mark.parametrize("size,k,iters,metric", [((64, 48), 16, 4, "l2"), ((256, 256), 256, 10, "l2"),
                                                 ((200, 120), 100, 6, "sqeuclidean"), ((33, 17), 7, 0, "l1")])
def test_colour_transfer_matches_oracle(size, k, iters, metric):
    ref = W.colour_image(10, *size)
    src = W.colour_image(11, *size)
    g = _run(ref, src, k, k, iters, metric)
    want = oracle.colour_transfer(ref.reshape(-1, 3), src.reshape(-1, 3), k, k, iters, metric)
    np.testing.assert_array_equal(g["ref_palette"], want["ref_palette"])
    np.testing.assert_array_equal(g["ref_mass"], want["ref_mass"])
    np.testing.assert_array_equal(g["src_palette"], want["src_palette"])
    np.testing.assert_array_equal(g["src_mass"], want["src_mass"])
    np.testing.assert_array_equal(g["assign"], want["assign"])
    r = want["solve"]
    st = g["stats"]
    assert int(st["status"]) == 0 and int(st["rounds"]) == r["rounds"] and int(st["nnz"]) == r["nnz"]
    assert abs(float(g["cost"][0]) - r["cost"]) <= 1e-12 * max(r["cost"], 1e-300)
    np.testing.assert_array_equal(g["image"].reshape(-1, 3), want["image"])


def test_colour_transfer_full_size_images():
    """1024 x 1024 images (the paper's transfer size), palettes of 256 bins."""
    ref = W.colour_image(12, 1024, 1024)
    src = W.colour_image(13, 1024, 1024)
    g = _run(ref, src, 256, 256, 10)
    want = oracle.colour_transfer(ref.reshape(-1, 3), src.reshape(-1, 3), 256, 256, 10)
    np.testing.assert_array_equal(g["assign"], want["assign"])
    np.testing.assert_array_equal(g["image"].reshape(-1, 3), want["image"])


def test_colour_transfer_onto_itself():
    img = W.colour_image(14, 96, 64)
    g = _run(img, img, 32, 32, 5)
    assert float(g["cost"][0]) == 0.0 and int(g["stats"]["rounds"]) == 1
    want = oracle.colour_transfer(img.reshape(-1, 3), img.reshape(-1, 3), 32, 32, 5)
    np.testing.assert_array_equal(g["image"].reshape(-1, 3), want["image"])
