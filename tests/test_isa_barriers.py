"""Static check of the compiled solver kernels (CPU only, needs hipcc).

On AMD hardware a workgroup barrier counts wavefronts, not lanes.  If the
structurized code lets a loop back-edge mask some lanes off and fall straight
into a block that starts with a barrier, the remaining lanes of that wave pass
the barrier without the masked lanes, which can livelock the workgroup.  This
test compiles the kernels to gfx950 assembly and rejects that shape."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = "/opt/rocm/bin/hipcc"


def scan(asm: str):
    lines = asm.split("\n")
    labels = {l.split(":")[0]: i for i, l in enumerate(lines) if re.match(r"^\.LBB\d+_\d+:", l)}

    def starts_with_barrier(i):
        k = 0
        for l in lines[i + 1:i + 400]:
            t = l.strip()
            if not t or t.startswith(";") or t.startswith("."):
                continue
            if "s_barrier" in t:
                return True
            if t.startswith(("s_waitcnt", "s_or_b64 exec", "s_nop")):
                continue
            k += 1
            if k > 2:
                return False
        return False

    hits = []
    for i, l in enumerate(lines):
        if "s_andn2_b64 exec, exec" not in l or i + 1 >= len(lines):
            continue
        n0 = lines[i + 1].strip()
        if n0.startswith("s_cbranch_execz") and i + 2 < len(lines):
            if re.match(r"^\.LBB", lines[i + 2]) and starts_with_barrier(i + 2):
                hits.append(lines[i + 2].split(":")[0])
        if n0.startswith("s_cbranch_execnz"):
            tgt = n0.split()[-1]
            if tgt in labels and starts_with_barrier(labels[tgt]):
                hits.append(tgt)
    return hits


def test_scanner_flags_the_bad_shape():
    bad = "\n".join([
        ".LBB0_9:", "\ts_andn2_b64 exec, exec, s[6:7]", "\ts_cbranch_execz .LBB0_20",
        ".LBB0_10:", "; loop header", "\ts_waitcnt lgkmcnt(0)", "\ts_barrier", "\tds_read_b32 v2, v74"])
    assert scan(bad) == [".LBB0_10"]
    good = "\n".join([
        ".LBB0_9:", "\ts_andn2_b64 exec, exec, s[6:7]", "\ts_cbranch_execz .LBB0_20",
        ".LBB0_10:", "\tv_add_u32 v1, v1, v2", "\tv_mul_lo_u32 v3, v1, v1", "\tds_write_b32 v4, v3",
        "\ts_barrier"])
    assert scan(good) == []


@pytest.mark.skipif(not shutil.which(HIPCC) and not os.path.exists(HIPCC), reason="hipcc not available")
@pytest.mark.parametrize("src", ["pair_solver.hip", "large_pair.hip", "doc_solver.hip", "surrogate.hip",
                                 "cost_solver.hip", "transport_map.hip", "colour_transfer.hip"])
def test_solver_kernels_have_no_divergent_back_edge_into_a_barrier(tmp_path, src):
    out = tmp_path / (src + ".s")
    cmd = [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "--offload-device-only", "-S",
           "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(ROOT, "paper_2401_07378_amd", "csrc"),
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           os.path.join(ROOT, "paper_2401_07378_amd", "csrc", src), "-o", str(out)]
    subprocess.run(cmd, check=True, capture_output=True)
    asm = out.read_text()
    assert asm.count("s_barrier") > 0
    assert scan(asm) == []
