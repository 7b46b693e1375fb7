"""The streaming-read reference pass (pcal_read_probe, through the C ABI) reads every byte once.

The per-wave XORs of the 64-bit words must combine to the XOR of the whole
buffer, whatever the launch shape (slices of ragged length included), and
invalid arguments are rejected on the host before any launch.
"""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2501_05993_amd import pcal

    pcal.lib()
    return pcal


@pytest.mark.parametrize("nbytes,blocks,threads", [
    ((4 << 20) + 48, 1024, 256),
    ((4 << 20) + 48, 512, 1024),
    (16, 8, 64),
    (160000, 3, 192),
])
def test_read_probe_reads_every_word(pc, nbytes, blocks, threads):
    print("[gpu-test] read probe bytes=%d shape %dx%d" % (nbytes, blocks, threads), flush=True)
    host = np.random.default_rng(nbytes + blocks).integers(0, 256, size=nbytes, dtype=np.uint8)
    dev = torch.from_numpy(host).cuda()
    out = torch.full((blocks * threads // 64,), -1, dtype=torch.int64, device="cuda")
    pc.read_probe(dev, out, blocks, threads)
    torch.cuda.synchronize()
    got = np.bitwise_xor.reduce(out.cpu().numpy().view(np.uint64))
    want = np.bitwise_xor.reduce(host.view(np.uint64))
    assert got == want


def test_read_probe_rejects_bad_arguments(pc):
    dev = torch.zeros(4096, dtype=torch.uint8, device="cuda")
    out = torch.zeros(64, dtype=torch.int64, device="cuda")
    f = pc.lib().pcal_read_probe
    p, o = dev.data_ptr(), ctypes.c_void_p(out.data_ptr())
    assert f(ctypes.c_void_p(p + 8), 4000, 4, 64, o, None, None, None) == pc.EINVAL   # misaligned
    assert f(ctypes.c_void_p(p), 4001, 4, 64, o, None, None, None) == pc.EINVAL       # not a multiple of 16
    assert f(ctypes.c_void_p(p), 4096, 4, 96, o, None, None, None) == pc.EINVAL       # threads not a multiple of 64
    assert f(ctypes.c_void_p(p), 4096, 0, 64, o, None, None, None) == pc.EINVAL       # no workgroups
    assert f(ctypes.c_void_p(p), 4096, 4, 64, None, None, None, None) == pc.EINVAL    # no output
