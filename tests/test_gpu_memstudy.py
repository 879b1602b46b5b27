"""Buffer read / write kernels of the memory study (paper Sec. 5) through the C ABI: the read
folds every word of the buffer (checked bit-exactly against the host XOR of the same words), the
write stores exactly its pattern and nothing past its length, and the sweep runs every
operation under both allocation modes."""
import numpy as np
import pytest

from gpu_helpers import say

pytestmark = pytest.mark.gpu

sg = pytest.importorskip("paper_2605_29752_amd")


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    return sg.Context(0)


@pytest.mark.parametrize("nbytes", [16, 4096, (1 << 20) + 48, 64 << 20, (3 << 20) + 16 * 1023])
def test_read_folds_every_word(nbytes):
    import torch
    say("read", nbytes)
    rng = np.random.default_rng(nbytes % 1000)
    words = rng.integers(0, 1 << 32, nbytes // 4, dtype=np.uint64).astype(np.uint32)
    buf = torch.from_numpy(words.view(np.int32)).cuda()
    nb = sg.mem_read_blocks(nbytes)
    assert 1 <= nb <= 2048
    sink = torch.full((2048,), -1, dtype=torch.int32, device="cuda")
    sg.mem_read(buf, sink, nbytes)
    torch.cuda.synchronize()
    got = np.bitwise_xor.reduce(sink.cpu().numpy()[:nb].view(np.uint32))
    assert got == np.bitwise_xor.reduce(words)
    assert np.all(sink.cpu().numpy()[nb:] == -1)       # only the documented partials written


@pytest.mark.parametrize("nbytes", [16, 4096 + 16, 16 << 20])
def test_write_pattern_and_extent(nbytes):
    import torch
    seed = 0x1234ABCD
    total = nbytes // 4 + 64                          # room past the written extent
    buf = torch.full((total,), 7, dtype=torch.int32, device="cuda")
    sg.mem_write(buf, seed, nbytes)
    torch.cuda.synchronize()
    got = buf.cpu().numpy().view(np.uint32)
    i = np.arange(nbytes // 4, dtype=np.uint64)
    want = ((i * np.uint64(0x9E3779B1)) & np.uint64(0xFFFFFFFF)).astype(np.uint32) ^ np.uint32(seed)
    assert np.array_equal(got[:nbytes // 4], want)
    assert np.all(got[nbytes // 4:] == 7)


def test_read_write_errors():
    import torch
    buf = torch.zeros(1024, dtype=torch.int32, device="cuda")
    sink = torch.zeros(2048, dtype=torch.int32, device="cuda")
    with pytest.raises(sg.SGError) as e:
        sg.mem_read(buf, sink, 20)                    # not a multiple of 16
    assert e.value.code == sg.SG_EINVAL
    with pytest.raises(sg.SGError) as e:
        sg.mem_write(buf[1:], 0, 64)                  # 4 bytes past a 16-byte boundary
    assert e.value.code == sg.SG_EINVAL


def test_sweep_every_op_and_allocation(ctx):
    shapes = [(128, 128, 128), (1024, 256, 512), (4096, 4096, 4096), (384, 4096, 128)]
    for op in (sg.MEM_READ_A, sg.MEM_READ_B, sg.MEM_READ_C, sg.MEM_WRITE_D):
        for alloc in (sg.MEM_ISOLATED, sg.MEM_COALLOC):
            t = ctx.mem_sweep(shapes, op, alloc, warmup=1, reps=3)
            say("op", op, "alloc", alloc, t)
            assert np.all(np.isfinite(t)) and np.all(t > 0)
    # a 64 MiB FP32 read cannot beat the HBM specification by much (the 256 MB cache aside,
    # nothing streams faster than ~10 TB/s); a sanity bound on the timing, not a target
    t = ctx.mem_sweep([(4096, 4096, 4096)], sg.MEM_READ_A, sg.MEM_ISOLATED, warmup=1, reps=3)[0]
    assert 4096 * 4096 * 4 / t < 20e12
    with pytest.raises(sg.SGError):
        ctx.mem_sweep(shapes, 9, sg.MEM_ISOLATED)
    with pytest.raises(sg.SGError):
        ctx.mem_sweep(shapes, sg.MEM_READ_A, sg.MEM_ISOLATED, elem_bytes=3)
