"""The scheduling knobs and their autotuner: results do not depend on the knobs (bit for bit),
and the autotuner applies and caches a timed choice."""
import os

import numpy as np
import pytest

from paper_2207_04620_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    import torch
    assert torch.cuda.is_available()
    from paper_2207_04620_amd import he
    he.lib()
    return he


def test_tunings_do_not_change_results(H):
    """a mixed batch (h = 8 and 16, two levels) under every pair_batch, group cap, overlap and
    concurrent-groups setting gives the same residues as under the defaults"""
    ctx = H.Context(I.small(log_n=12, n_q=6, alpha=2, q_bits=40, p_bits=50, h_list=(8, 16)), schedule=15)
    mix = [(8, 5), (16, 5), (8, 4), (16, 5), (8, 5), (16, 4), (8, 5)]
    As, Bs = [], []
    for i, (h, lv) in enumerate(mix):
        A, B = I.matrix_pair(60 + i, h)
        As.append(ctx.encrypt(A.ravel(), level=lv, nonce=2 * i))
        Bs.append(ctx.encrypt(B.ravel(), level=lv, nonce=2 * i + 1))
    hs = [h for h, _ in mix]
    ref = [ctx.export(r) for r in ctx.matmul_batch(As, Bs, hs)]
    for cg in (0, 1):
        for ov in (0, 1):
            for pb in (1, 2, 8, 16):
                for mg in (1, 2, 32):
                    ctx.set_tuning(pb, mg, ov, cg)
                    for r, w in zip(ctx.matmul_batch(As, Bs, hs), ref):
                        assert np.array_equal(ctx.export(r), w), (pb, mg, ov, cg)
    with pytest.raises(H.HEError):
        ctx.set_tuning(0, 4)
    with pytest.raises(H.HEError):
        ctx.set_tuning(4, 4, 2)
    with pytest.raises(H.HEError):
        ctx.set_tuning(4, 4, 0, 2)
    ctx.close()


def test_autotune_applies_and_caches(H, tmp_path):
    ctx = H.Context(I.small(log_n=12, n_q=6, alpha=2, q_bits=40, p_bits=50, h_list=(16,)), schedule=15)
    path = str(tmp_path / "tune.txt")
    rep = ctx.autotune(16, 5, 16, cache_path=path)
    assert rep["source"] == "timed"
    cands = rep["candidates"]
    assert len(cands) == 9 and all(c["ms"] > 0 for c in cands)
    assert [c["overlap"] for c in cands] == [0] * 8 + [1]
    chosen = rep["chosen"]
    assert chosen["concurrent_groups"] == 1  # not tuned: the context's setting
    keys = ("pair_batch", "max_group", "overlap")
    assert {k: chosen[k] for k in keys} in [{k: c[k] for k in keys} for c in cands]
    assert ctx.tuning() == chosen
    best = min(c["ms"] for c in cands)
    assert next(c["ms"] for c in cands if all(c[k] == chosen[k] for k in keys)) <= best / 0.99 ** 9
    line = open(path).read().split()
    assert line[0] == rep["key"] and [int(x) for x in line[1:4]] == [chosen[k] for k in keys]
    # the same key again: answered from the cache without timing, and applied
    ctx.set_tuning(1, 1, 0, 1)
    again = ctx.autotune(16, 5, 16, cache_path=path)
    assert again["source"] in ("process cache", "file cache") and again["chosen"] == chosen
    assert ctx.tuning() == chosen
    ctx.close()
