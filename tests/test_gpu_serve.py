"""Batched sign and the continuous-batching serving loop, through the C ABI.

Each served result must be bit-identical to the same operation run alone
(the serving loop runs the same operation DAG in lockstep cohorts)."""
import sys
import time

import numpy as np
import pytest

from paper_2207_04620_amd import inputs as I

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    from paper_2207_04620_amd import he
    prm = I.small(log_n=12, n_q=8, alpha=3, q_bits=40, p_bits=50, h_list=(4, 8, 16))
    _log("[serve] context small12")
    return he.Context(prm)


def test_sign_batch_equals_single(ctx):
    X = I.sign_inputs(11, 5, 16)
    xs = [ctx.encrypt(X[i].ravel(), level=7 - (i % 2), nonce=50 + i) for i in range(5)]
    singles = [ctx.export(ctx.sign_approx(x, 3, 1, 0)) for x in xs]
    got = ctx.sign_approx_batch(xs, 3, 1, 0)
    for g, s in zip(got, singles):
        assert np.array_equal(ctx.export(g), s)


def test_serve_mixed_requests_equal_alone(ctx):
    from paper_2207_04620_amd import he
    reqs, alone = [], []
    for i, (h, lvl) in enumerate([(8, 7), (16, 6), (8, 7), (4, 5), (16, 7), (8, 7)]):
        A, B = I.matrix_pair(300 + i, h)
        a = ctx.encrypt(A.ravel(), level=lvl, nonce=400 + 2 * i)
        b = ctx.encrypt(B.ravel(), level=lvl, nonce=401 + 2 * i)
        reqs.append(("mm", h, a, b))
        alone.append(ctx.export(ctx.matmul(a, b, h)))
    X = I.sign_inputs(12, 3, 16)
    for i in range(3):
        x = ctx.encrypt(X[i].ravel(), level=7, nonce=500 + i)
        mode = i % 2
        reqs.append(("sign", mode, x, None))
        alone.append(ctx.export(ctx.sign_approx(x, 3, 1, mode)))
    # the served requests of depth 1 and 2: x^2 (Mul_ct, RS) and x . x^2
    for i, k in enumerate((2, 3, 2)):
        x = ctx.encrypt(X[i].ravel(), level=6 - i, nonce=600 + i)
        x2 = ctx.rescale(ctx.mul(x, x))
        want = x2 if k == 2 else ctx.rescale(ctx.mul(ctx.drop(x, x2.level), x2))
        reqs.append(("pow", k, x, None))
        alone.append(ctx.export(want))
    srv = he.Server(ctx, max_batch=4)
    tickets = []
    for j, r in enumerate(reqs):
        if r[0] == "mm":
            tickets.append(srv.submit(he.REQ_MATMUL, r[2], r[3], h=r[1]))
        elif r[0] == "pow":
            tickets.append(srv.submit(he.REQ_POWER, r[2], k=r[1]))
        else:
            tickets.append(srv.submit(he.REQ_SIGN, r[2], d=3, k=1, mode=r[1]))
        if j % 3 == 2:
            time.sleep(0.01)  # later arrivals join while earlier cohorts run
    results = {}
    deadline = time.time() + 60
    while len(results) < len(tickets) and time.time() < deadline:
        for t in tickets:
            if t in results:
                continue
            got = srv.poll(t)
            if got is not None:
                results[t] = got
        time.sleep(0.002)
    srv.stop()
    assert len(results) == len(tickets)
    for t, want in zip(tickets, alone):
        ct, lat = results[t]
        assert lat > 0
        assert np.array_equal(ctx.export(ct), want)


def test_serve_admission_and_rejections(ctx):
    from paper_2207_04620_amd import he
    A, B = I.matrix_pair(9, 8)
    a = ctx.encrypt(A.ravel(), level=7, nonce=1)
    b = ctx.encrypt(B.ravel(), level=7, nonce=2)
    tiny = he.Server(ctx, mem_budget_bytes=1 << 20)
    with pytest.raises(he.HEError) as e:
        tiny.submit(he.REQ_MATMUL, a, b, h=8)
    assert e.value.name == "HE_ENOMEM"
    tiny.stop()
    srv = he.Server(ctx)
    with pytest.raises(he.HEError) as e:
        srv.submit(he.REQ_MATMUL, a, b, h=6)
    assert e.value.name == "HE_ESHAPE"
    with pytest.raises(he.HEError) as e:
        srv.submit(he.REQ_SIGN, ctx.drop(a, 1), d=3, k=1)
    assert e.value.name == "HE_ELEVEL"
    srv.stop()
    # a budget that fits one product at a time still completes every request
    one = he.Server(ctx, mem_budget_bytes=64 << 20)
    ts = [one.submit(he.REQ_MATMUL, a, b, h=8) for _ in range(3)]
    want = ctx.export(ctx.matmul(a, b, 8))
    done = {}
    deadline = time.time() + 60
    while len(done) < 3 and time.time() < deadline:
        for t in ts:
            if t not in done:
                r = one.poll(t)
                if r is not None:
                    done[t] = r
        time.sleep(0.002)
    one.stop()
    assert len(done) == 3
    for t in ts:
        assert np.array_equal(ctx.export(done[t][0]), want)


def test_serve_across_rings_equal_alone():
    """the serving configuration across rings: one server per context (N = 2^14, 2^15,
    2^16; each with its own stream and request loop, so their work overlaps on the device);
    matmul requests of h in {8, ..., 128} and sign/ReLU requests of depth 3..13, each routed
    to the smallest ring that holds its h and depth, submitted in an interleaved burst.
    Every result equals the same operation run alone on that context, bit for bit."""
    import torch
    assert torch.cuda.is_available()
    from paper_2207_04620_amd import he
    _log("[serve] contexts C2 / C3 / C4")
    rings = [he.Context(I.C2, h_list=[8, 16, 32, 64], schedule=he.SCHED_FAST),
             he.Context(I.C3, h_list=[128], schedule=he.SCHED_FAST),
             he.Context(I.C4, h_list=[], schedule=he.SCHED_FAST)]
    work = [("mm", 8), ("mm", 64), ("mm", 128), ("mm", 16), ("sign", 3, 1, he.SIGN), ("sign", 3, 2, he.RELU),
            ("mm", 32), ("sign", 3, 4, he.RELU), ("sign", 3, 3, he.SIGN), ("mm", 64), ("sign", 3, 4, he.SIGN)]
    reqs = []
    for i, w in enumerate(work):
        if w[0] == "mm":
            ctx = he.smallest_ring(rings, h=w[1], depth=3)
            A, B = I.matrix_pair(800 + i, w[1])
            a = ctx.encrypt(A.ravel(), nonce=2 * i)
            b = ctx.encrypt(B.ravel(), nonce=2 * i + 1)
            want = ctx.export(ctx.matmul(a, b, w[1]))
            reqs.append((ctx, w, a, b, want))
        else:
            _, d, k, mode = w
            depth = he.sign_depth(d, k, mode)
            # the deepest ReLU also runs on the largest ring (the sign configuration's ring)
            ctx = rings[2] if depth == 13 else he.smallest_ring(rings, h=32, depth=depth)
            X = I.sign_inputs(900 + i, 1, 32)[0]
            x = ctx.encrypt(X.ravel(), nonce=2 * i)
            want = ctx.export(ctx.sign_approx(x, d, k, mode))
            reqs.append((ctx, w, x, None, want))
        _log(f"[serve] request {i}: {w} on N=2^{ctx.n.bit_length() - 1}")
    assert {id(r[0]) for r in reqs} == {id(c) for c in rings}
    servers = {id(c): he.Server(c, max_batch=4, min_batch=1) for c in rings}
    tickets = []
    for ctx, w, a, b, _ in reqs:
        srv = servers[id(ctx)]
        if w[0] == "mm":
            tickets.append(srv.submit(he.REQ_MATMUL, a, b, h=w[1]))
        else:
            tickets.append(srv.submit(he.REQ_SIGN, a, d=w[1], k=w[2], mode=w[3]))
    done = {}
    deadline = time.time() + 120
    while len(done) < len(tickets) and time.time() < deadline:
        for j, t in enumerate(tickets):
            if j not in done:
                r = servers[id(reqs[j][0])].poll(t)
                if r is not None:
                    done[j] = r
        time.sleep(0.002)
    for s in servers.values():
        s.stop()
    assert len(done) == len(tickets)
    for j, (ctx, w, _, _, want) in enumerate(reqs):
        assert np.array_equal(ctx.export(done[j][0]), want), (j, w)
    _log("[serve] across rings: every result equals its run alone")


def test_serve_budget_from_measured_footprints():
    """admission by measured footprints on the N=2^15 ring: a burst of 40 h=64 products (16 of
    them first, so that the type is measured, then 24 more) under a budget of 2.5 GB; the
    allocation cache's in-use bytes while serving stay within the budget above what was in use
    before (keys, masks, inputs), every request completes, and results equal the product run
    alone"""
    import torch
    assert torch.cuda.is_available()
    from paper_2207_04620_amd import he
    _log("[serve] budget test: context C3, h=64")
    ctx = he.Context(I.C3, h_list=[64], schedule=he.SCHED_FAST)
    pairs = [I.matrix_pair(950 + i, 64) for i in range(4)]
    As = [ctx.encrypt(A.ravel(), level=13, nonce=2 * i) for i, (A, _) in enumerate(pairs)]
    Bs = [ctx.encrypt(B.ravel(), level=13, nonce=2 * i + 1) for i, (_, B) in enumerate(pairs)]
    want = [ctx.export(ctx.matmul(a, b, 64)) for a, b in zip(As, Bs)]
    ctx.sync()
    base, _ = ctx.pool_stats()
    budget = 2500 << 20
    srv = he.Server(ctx, mem_budget_bytes=budget, max_batch=16, min_batch=1)
    try:
        for wave, n in enumerate((16, 24)):
            ts = [srv.submit(he.REQ_MATMUL, As[i % 4], Bs[i % 4], h=64) for i in range(n)]
            done = {}
            deadline = time.time() + 120
            while len(done) < n and time.time() < deadline:
                for j, t in enumerate(ts):
                    if j not in done:
                        r = srv.poll(t)
                        if r is not None:
                            done[j] = ctx.export(r[0]) if j < 4 else True  # results dropped at once
                time.sleep(0.002)
            assert len(done) == n, wave
            for j in range(4):
                assert np.array_equal(done[j], want[j % 4])
            st = srv.stats()
            _log(f"[serve] wave {wave}: {st}, base {base}")
            assert st["per_member"] and st["inflight"] == 0
            assert st["peak_in_use"] - base <= budget, (st, base)
    finally:
        srv.stop()
    ctx.close()
