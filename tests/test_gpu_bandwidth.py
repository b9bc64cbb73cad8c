"""The streaming diagnostic moves exactly the bytes it claims: the copy is
bitwise, the write leaves zeros, and the read's per-block XORs combine to
the XOR of every word of the source (each word read once)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nbytes", [16, 4096 + 16 * 7, 64 << 20])
def test_copy_read_write(nbytes):
    import torch
    from paper_2010_14823_amd import casim
    rng = np.random.default_rng(nbytes)
    words = rng.integers(0, 1 << 32, size=nbytes // 4, dtype=np.uint64).astype(np.uint32)
    src = torch.from_numpy(words.view(np.int32)).cuda()
    dst = torch.full_like(src, -1)
    casim.debug_bandwidth(src, dst, nbytes, 0)
    torch.cuda.synchronize()
    assert torch.equal(dst, src)
    casim.debug_bandwidth(None, dst, nbytes, 2)
    torch.cuda.synchronize()
    assert int(torch.count_nonzero(dst)) == 0
    casim.debug_bandwidth(src, dst, nbytes, 1)
    torch.cuda.synchronize()
    n16 = nbytes // 16
    blocks = min((n16 + 1023) // 1024, 4096)
    got = dst.cpu().numpy().view(np.uint32).reshape(-1, 4)[:blocks]
    want = np.bitwise_xor.reduce(words.reshape(-1, 4), axis=0)
    assert np.array_equal(np.bitwise_xor.reduce(got, axis=0), want)
