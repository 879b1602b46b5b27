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


def _device_asm(tmp_path_factory, src):
    if not os.path.exists(HIPCC) and shutil.which("hipcc") is None:
        pytest.skip("hipcc not available")
    out = str(tmp_path_factory.mktemp("asm") / (src + ".s"))
    cmd = [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-x", "hip",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "--cuda-device-only", "-S", os.path.join(CSRC, src), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    return open(out).read()


@pytest.fixture(scope="module")
def asm(tmp_path_factory):
    return _device_asm(tmp_path_factory, "gemm_tile.hip")


@pytest.fixture(scope="module")
def grouped_asm(tmp_path_factory):
    return _device_asm(tmp_path_factory, "grouped.hip")


TILES = [(256, 256), (256, 128), (128, 256), (128, 128), (128, 64), (64, 128), (64, 64)]


def kernel_body(text, name):
    start = text.index("\n" + name + ":")
    end = text.index("s_endpgm", start)
    return text[start:end]


def _accumulator_copies(body):
    """AGPR-to-AGPR moves whose source is not a register just set to zero (a zero broadcast that
    initialises accumulators is fine; a copy of live accumulator data is what to catch).  A
    linear scan: an AGPR counts as zero from `v_accvgpr_write_b32 aN, 0` (or a move from a zero
    register) until another instruction writes it."""
    zero, bad = set(), []
    for line in body.split("\n"):
        ins = line.strip().split(None, 1)
        if len(ins) < 2 or ins[0].startswith((";", ".")):
            continue
        ops = [o.strip() for o in ins[1].split(",")]
        dst = ops[0]
        regs = set()
        m = re.fullmatch(r"a(\d+)", dst)
        if m:
            regs = {int(m.group(1))}
        m = re.fullmatch(r"a\[(\d+):(\d+)\]", dst)
        if m:
            regs = set(range(int(m.group(1)), int(m.group(2)) + 1))
        if ins[0] == "v_accvgpr_write_b32" and len(ops) > 1 and ops[1] == "0":
            zero |= regs
            continue
        if ins[0].startswith("v_accvgpr_mov"):
            src = re.fullmatch(r"a(\d+)", ops[1])
            if src and int(src.group(1)) in zero:
                zero |= regs
                continue
            bad.append(line.strip())
        zero -= regs
    return bad


@pytest.mark.parametrize("bm,bn", TILES)
def test_no_accumulator_copies(asm, bm, bn):
    body = kernel_body(asm, "_ZN2sg16sg_gemm_tile_dmaILi%dELi%dEEEvNS_5KArgsE" % (bm, bn))
    assert re.search(r"v_mfma_f32_16x16x32_bf16", body)
    bad = _accumulator_copies(body)
    assert not bad, "accumulators copied between MFMAs: %s" % bad[:4]


def test_accumulator_copy_scan_catches_copies():
    """The scan accepts a zero broadcast and rejects a copy of live data."""
    assert _accumulator_copies("\tv_accvgpr_write_b32 a0, 0\n\tv_accvgpr_mov_b32 a1, a0\n") == []
    live = "\tv_mfma_f32_16x16x32_bf16 a[0:3], v[0:3], v[4:7], a[0:3]\n\tv_accvgpr_mov_b32 a4, a0\n"
    assert _accumulator_copies(live) == ["v_accvgpr_mov_b32 a4, a0"]
    rezeroed = ("\tv_accvgpr_write_b32 a0, 0\n\tv_mfma_f32_16x16x32_bf16 a[0:3], v[0:3], v[4:7], a[0:3]\n"
                "\tv_accvgpr_mov_b32 a5, a0\n")
    assert _accumulator_copies(rezeroed) == ["v_accvgpr_mov_b32 a5, a0"]


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


def test_deep_k_kernel_codegen(asm):
    """The 64x64 tile with 128-deep K stages: MFMAs, no accumulator copies, no spills."""
    name = "_ZN2sg21sg_gemm_tile_dma_k128ILi64ELi64EEEvNS_5KArgsE"
    body = kernel_body(asm, name)
    assert re.search(r"v_mfma_f32_16x16x32_bf16", body)
    assert not _accumulator_copies(body)
    meta = asm[asm.index("amdhsa.kernels:"):]
    entry = [e for e in meta.split("\n  - ") if re.search(r"\.name:\s+" + name + r"\s", e)]
    assert len(entry) == 1
    for key in (".vgpr_spill_count", ".sgpr_spill_count"):
        assert re.findall(re.escape(key) + r":\s+(\d+)", entry[0]) == ["0"], key


@pytest.mark.parametrize("bm,bn", TILES)
def test_stream_k_kernel_codegen(asm, bm, bn):
    """The stream-K kernels run the same tile body once per segment of their range: MFMAs, no
    accumulator copies, no spills."""
    name = "_ZN2sg19sg_gemm_tile_dma_skILi%dELi%dEEEvNS_5KArgsENS_6SkArgsE" % (bm, bn)
    body = kernel_body(asm, name)
    assert re.search(r"v_mfma_f32_16x16x32_bf16", body)
    bad = _accumulator_copies(body)
    assert not bad, "accumulators copied between MFMAs: %s" % bad[:4]
    meta = asm[asm.index("amdhsa.kernels:"):]
    entry = [e for e in meta.split("\n  - ") if re.search(r"\.name:\s+" + name + r"\s", e)]
    assert len(entry) == 1
    for key in (".vgpr_spill_count", ".sgpr_spill_count"):
        assert re.findall(re.escape(key) + r":\s+(\d+)", entry[0]) == ["0"], key


def test_grouped_kernels_no_spills(grouped_asm):
    """Every persistent grouped kernel (each tile shape, all-aligned and general bodies) keeps
    its registers: no spills."""
    meta = grouped_asm[grouped_asm.index("amdhsa.kernels:"):]
    entries = [e for e in meta.split("\n  - ") if re.search(r"\.name:\s+_ZN2sg15sg_gemm_grouped", e)]
    assert len(entries) == 2 * len(TILES)
    for e in entries:
        for key in (".vgpr_spill_count", ".sgpr_spill_count"):
            assert re.findall(re.escape(key) + r":\s+(\d+)", e) == ["0"], (key, e[:200])
