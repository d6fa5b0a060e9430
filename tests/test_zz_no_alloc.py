"""he_rotate_noalloc, the rotation entry point that allocates nothing (its temporaries live in a
static device scratch), against he_rotate on the N=2^15 ring: two calls in a row, the second on
a smaller input (a lower level, fewer limbs), each bit-identical to he_rotate's result; the
allocation cache does not grow during the calls; a missing key and an input beyond the scratch
are refused."""
import numpy as np
import pytest

from paper_2207_04620_amd import inputs as I

pytestmark = pytest.mark.gpu

EKEY, ENOMEM = 5, 2


def _log(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def H():
    import torch
    assert torch.cuda.is_available()
    from paper_2207_04620_amd import he
    he.lib()
    return he


def _to_eval(ctx, words):
    """coefficient-domain residues u64[2][nl][N] -> a device tensor in the evaluation domain"""
    import torch
    nl = words.shape[1]
    t = torch.from_numpy(np.ascontiguousarray(words).reshape(-1, ctx.n).view(np.int64)).cuda()
    ctx.ntt(t, [i for _ in range(2) for i in range(nl)])
    return t


def _to_coeff(ctx, t, nl):
    import torch
    ctx.ntt(t, [i for _ in range(2) for i in range(nl)], inverse=True)
    torch.cuda.synchronize()
    return t.cpu().numpy().view(np.uint64).reshape(2, nl, ctx.n)


def test_rotate_noalloc_matches_rotate(H):
    import torch
    ctx = H.Context(I.C3, h_list=[], stream=torch.cuda.current_stream().cuda_stream)
    for call, (level, k) in enumerate([(13, 5), (4, -64)]):
        _log(f"[noalloc] call {call}: level {level}, k {k}")
        ctx.gen_rotation_key(k)
        A = I.matrix(70 + call, 64).ravel()
        a = ctx.encrypt(A, level=level, nonce=70 + call)
        want = ctx.export(ctx.rotate(a, k))
        inp = _to_eval(ctx, ctx.export(a))
        out = torch.empty_like(inp)
        ctx.sync()
        torch.cuda.synchronize()
        in_use, _ = ctx.pool_stats(reset=True)
        ctx.rotate_noalloc(inp.data_ptr(), level, k, out.data_ptr())
        ctx.sync()
        after, peak = ctx.pool_stats()
        assert after == in_use and peak == in_use, (in_use, after, peak)
        got = _to_coeff(ctx, out, level + 1)
        assert got.shape == want.shape
        bad = np.argwhere(got != want)
        assert bad.size == 0, f"{len(bad)} residues differ, first at {bad[:3].tolist()}"
    _log("[noalloc] missing key")
    with pytest.raises(H.HEError) as e:
        ctx.rotate_noalloc(inp.data_ptr(), 4, 3, out.data_ptr())
    assert e.value.code == EKEY
    ctx.close()


def test_rotate_noalloc_refuses_inputs_beyond_the_scratch(H):
    """N = 2^16 with 17 + 5 limbs at the top level needs 144 N words (75.5 MB) > 64 MiB"""
    import torch
    ctx = H.Context(I.C4, h_list=[])
    buf = torch.empty(2 * 17 * ctx.n, dtype=torch.int64, device="cuda")
    out = torch.empty_like(buf)
    with pytest.raises(H.HEError) as e:
        ctx.rotate_noalloc(buf.data_ptr(), 16, 1, out.data_ptr())
    assert e.value.code == ENOMEM
    ctx.close()
