"""The streaming diagnostic moves exactly the bytes it claims, for both
access widths and several grids: the copy is bitwise, the write leaves
zeros, and the read's per-block XORs combine to the XOR of every word of the
source (each word read once)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("width", [8, 16])
@pytest.mark.parametrize("nbytes,blocks", [(16, 1), (4096 + 16 * 7, 3), (64 << 20, 1024), (64 << 20, 16384)])
def test_copy_read_write(nbytes, blocks, width):
    import torch
    from paper_2010_14823_amd import casim
    rng = np.random.default_rng(nbytes + blocks)
    words = rng.integers(0, 1 << 32, size=nbytes // 4, dtype=np.uint64).astype(np.uint32)
    src = torch.from_numpy(words.view(np.int32)).cuda()
    dst = torch.full_like(src, -1)
    casim.debug_bandwidth(src, dst, nbytes, 0, width, blocks)
    torch.cuda.synchronize()
    assert torch.equal(dst, src)
    casim.debug_bandwidth(None, dst, nbytes, 2, width, blocks)
    torch.cuda.synchronize()
    assert int(torch.count_nonzero(dst)) == 0
    casim.debug_bandwidth(src, dst, nbytes, 1, width, blocks)
    torch.cuda.synchronize()
    per = width // 4
    nb = min(blocks, nbytes // width)
    got = dst.cpu().numpy().view(np.uint32).reshape(-1, per)[:nb]
    want = np.bitwise_xor.reduce(words.reshape(-1, per), axis=0)
    assert np.array_equal(np.bitwise_xor.reduce(got, axis=0), want)
