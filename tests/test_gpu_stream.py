"""The measurement kernels (streaming copy and spread) element by element,
with a canary past the end of the destination."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gen():
    import torch
    import paper_2606_23348_amd as g
    assert torch.cuda.is_available()
    g.lib()
    return g


def _bytes(n, seed):
    return np.random.default_rng(seed).integers(0, 256, n, dtype=np.uint8)


@pytest.mark.parametrize("chunks", [1, 255, 256, 1000, 65537])
def test_stream_copy(gen, chunks):
    import torch
    src = torch.from_numpy(_bytes(chunks * 16, chunks)).cuda()
    buf = torch.full(((chunks + 32) * 16,), 0xAB, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    gen.gen_stream_copy(buf[:chunks * 16], src)
    torch.cuda.synchronize()
    assert torch.equal(buf[:chunks * 16], src)
    assert bool((buf[chunks * 16:] == 0xAB).all())


@pytest.mark.parametrize("k", [1, 2, 3, 8, 11])
@pytest.mark.parametrize("chunks", [1, 257, 4099])
def test_stream_spread(gen, k, chunks):
    import torch
    n_src = -(-chunks // k)
    host = _bytes(n_src * 16, 7 * k + chunks)
    src = torch.from_numpy(host).cuda()
    buf = torch.full(((chunks + 32) * 16,), 0xAB, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    gen.gen_stream_spread(buf[:chunks * 16], src, k)
    torch.cuda.synchronize()
    expect = host.reshape(n_src, 16)[np.arange(chunks) // k].reshape(-1)
    got = buf.cpu().numpy()
    assert np.array_equal(got[:chunks * 16], expect)
    assert (got[chunks * 16:] == 0xAB).all()


@pytest.mark.parametrize("chunks", [1, 300, 4099])
def test_stream_spread_write_only(gen, chunks):
    """k = 0: zeros written, nothing read (no source buffer)."""
    import torch
    buf = torch.full(((chunks + 32) * 16,), 0xAB, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    gen.gen_stream_spread(buf[:chunks * 16], None, 0)
    torch.cuda.synchronize()
    got = buf.cpu().numpy()
    assert not got[:chunks * 16].any()
    assert (got[chunks * 16:] == 0xAB).all()
