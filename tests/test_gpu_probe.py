"""The streaming-bandwidth probe (he_stream_probe) computes what it says on ragged sizes, so the
bandwidth it reports is that of real reads and writes; and it rejects what it cannot take."""
import numpy as np
import pytest

from paper_2207_04620_amd import inputs as I

pytestmark = pytest.mark.gpu

def partial_words(n):
    """words of partial sums the read mix writes: one pair per 4096 words"""
    return 2 * ((n + 4095) // 4096)


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    from paper_2207_04620_amd import he
    he.lib()
    # the context issues on torch's stream, so the probe is ordered after the inputs' copies
    ctx = he.Context(I.small(log_n=10, n_q=3, alpha=1, q_bits=40, p_bits=50, h_list=(8,)), schedule=0,
                     stream=torch.cuda.current_stream().cuda_stream)
    return torch, he, ctx


def _words(torch, n, seed):
    g = np.random.default_rng(seed)
    return torch.from_numpy(g.integers(-(1 << 63), (1 << 63) - 1, size=n, dtype=np.int64)).cuda()


@pytest.mark.parametrize("n", [2, 2 * 1024 * 4 + 6, (1 << 21) + 2 * 1000])
def test_copy_add_and_read_results(env, n):
    torch, he, ctx = env
    a, b = _words(torch, n, 1), _words(torch, n, 2)
    c = torch.zeros(max(n, partial_words(n)), dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    ms = ctx.stream_probe(1, a, None, c[:n], 2)
    assert ms > 0
    assert torch.equal(c[:n], a)
    ctx.stream_probe(2, a, b, c[:n], 2)
    an, bn, cn = (x.cpu().numpy().view(np.uint64) for x in (a, b, c[:n]))
    assert np.array_equal(cn, an + bn)  # uint64 addition wraps mod 2^64
    c.zero_()
    ctx.stream_probe(0, a, None, c, 1)
    part = c.cpu().numpy().view(np.uint64)
    assert not part[partial_words(n):].any()
    assert int(part.sum(dtype=np.uint64)) == int(an.sum(dtype=np.uint64))


def test_rejections(env):
    torch, he, ctx = env
    a = _words(torch, 8, 3)
    c = torch.zeros(64, dtype=torch.int64, device="cuda")
    for args in [(3, a, None, c[:8], 1), (2, a, None, c[:8], 1), (1, a, None, c[:8], 0),
                 (1, a[:7], None, c[:7], 1), (1, a[1:7], None, c[:6], 1)]:
        with pytest.raises(he.HEError) as e:
            ctx.stream_probe(*args)
        assert e.value.name == "HE_EINVAL", args[0]
