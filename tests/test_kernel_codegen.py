"""Code-generation checks of the tile kernels (CPU: hipcc cross-compiles gfx950 assembly).

Two compiler behaviours cost a large share of the MFMA rate and show up only in the assembly:
accumulators copied through a temporary before every MFMA (a serial dependency between all
MFMAs of a step; seen when the accumulators live across two K loops), and register spills.
"""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2605_29752_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def asm(tmp_path_factory):
    if not os.path.exists(HIPCC) and shutil.which("hipcc") is None:
        pytest.skip("hipcc not available")
    out = str(tmp_path_factory.mktemp("asm") / "gemm_tile.s")
    cmd = [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-x", "hip",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "--cuda-device-only", "-S", os.path.join(CSRC, "gemm_tile.hip"), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    return open(out).read()


TILES = [(256, 256), (256, 128), (128, 256), (128, 128), (128, 64), (64, 128), (64, 64)]


def kernel_body(text, name):
    start = text.index("\n" + name + ":")
    end = text.index("s_endpgm", start)
    return text[start:end]


@pytest.mark.parametrize("bm,bn", TILES)
def test_no_accumulator_copies(asm, bm, bn):
    body = kernel_body(asm, "_ZN2sg16sg_gemm_tile_dmaILi%dELi%dEEEvNS_5KArgsE" % (bm, bn))
    assert re.search(r"v_mfma_f32_16x16x32_bf16", body)
    assert "v_accvgpr_mov" not in body, "accumulators copied between MFMAs"


@pytest.mark.parametrize("bm,bn", TILES)
def test_no_spills(asm, bm, bn):
    name = "_ZN2sg16sg_gemm_tile_dmaILi%dELi%dEEEvNS_5KArgsE" % (bm, bn)
    # the kernel's entry in the code-object metadata (one "  - " item per kernel)
    meta = asm[asm.index("amdhsa.kernels:"):]
    entry = [e for e in meta.split("\n  - ") if re.search(r"\.name:\s+" + name + r"\s", e)]
    assert len(entry) == 1
    for key in (".vgpr_spill_count", ".sgpr_spill_count"):
        vals = re.findall(re.escape(key) + r":\s+(\d+)", entry[0])
        assert vals == ["0"], (key, vals)
