"""The batched product captured into a HIP graph: every replay, with eager work and host
synchronisations between replays, gives the same residues as the eager batched product; the
graph keeps working after the caller drops its handles, and the context works after the graph
is destroyed."""
import numpy as np
import pytest

from paper_2207_04620_amd import inputs as I

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def H():
    import torch
    assert torch.cuda.is_available()
    from paper_2207_04620_amd import he
    he.lib()
    return he


@pytest.mark.parametrize("schedule", [0, 15])
def test_graph_replays_equal_eager(H, schedule):
    ctx = H.Context(I.small(log_n=12, n_q=6, alpha=2, q_bits=40, p_bits=50, h_list=(8, 16)), schedule=schedule)
    mix = [(8, 5), (16, 5), (8, 4), (16, 5)]
    As, Bs = [], []
    for i, (h, lv) in enumerate(mix):
        A, B = I.matrix_pair(70 + i, h)
        As.append(ctx.encrypt(A.ravel(), level=lv, nonce=2 * i))
        Bs.append(ctx.encrypt(B.ravel(), level=lv, nonce=2 * i + 1))
    hs = [h for h, _ in mix]
    want = [ctx.export(r) for r in ctx.matmul_batch(As, Bs, hs)]
    _log(f"[graph] capture, schedule {schedule}")
    g, outs = ctx.matmul_batch_graph(As, Bs, hs)
    info = g.info()
    assert info["nodes"] > 10 and info["bytes"] > 0
    for rep in range(4):
        if rep:
            g.launch()
        # eager work and synchronisations between the replays
        other = ctx.matmul_batch(As[:2], Bs[:2], hs[:2])
        ctx.sync()
        for o, w in zip(outs, want):
            assert np.array_equal(ctx.export(o), w), rep
        assert np.array_equal(ctx.export(other[1]), want[1])
    # the caller drops its result handles: the graph still owns the buffers it writes
    del outs
    g.launch()
    ctx.sync()
    fresh = ctx.matmul_batch(As, Bs, hs)
    for r, w in zip(fresh, want):
        assert np.array_equal(ctx.export(r), w)
    g.close()
    for r, w in zip(ctx.matmul_batch(As, Bs, hs), want):
        assert np.array_equal(ctx.export(r), w)
    ctx.close()


def test_graph_refused_while_profiling(H):
    ctx = H.Context(I.small(log_n=12, n_q=6, alpha=2, q_bits=40, p_bits=50, h_list=(8,)))
    a = ctx.encrypt(I.matrix(1, 8).ravel(), nonce=1)
    ctx.profile(True)
    try:
        with pytest.raises(H.HEError) as e:
            ctx.matmul_batch_graph([a], [a], [8])
        assert e.value.code == 9
    finally:
        ctx.profile(False)
        ctx.profile_report()
    ctx.close()
