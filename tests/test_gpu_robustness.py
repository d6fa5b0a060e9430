"""Error paths of the C ABI, each forced from the host so that every kernel that does run
exits normally: handles from another context (HE_EMISMATCH), a checkpoint with a residue
outside [0, q_i) (HE_EINVAL), a kernel launch failed by the host-side injection before it is
queued (HE_EDEVICE from the call that issued it), and the allocation cache's cap
(HE_ENOMEM from the device pool).  After each, the context (or the server) goes on and its
next results equal the ones computed before the failure."""
import time

import numpy as np
import pytest

from paper_2207_04620_amd import inputs as I

pytestmark = pytest.mark.gpu

EINVAL, ENOMEM, EMISMATCH, EDEVICE = 1, 2, 7, 8


def _log(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def H():
    import torch
    assert torch.cuda.is_available()
    from paper_2207_04620_amd import he
    he.lib()
    return he


@pytest.fixture(scope="module")
def ctx(H):
    _log("[robust] context small12")
    return H.Context(I.small(log_n=12, n_q=8, alpha=3, q_bits=40, p_bits=50, h_list=(8,)))


def _code(H, fn, *a, **kw):
    with pytest.raises(H.HEError) as e:
        fn(*a, **kw)
    return e.value.code


def test_handles_from_another_context(H, ctx):
    other = H.Context(I.small(log_n=12, n_q=8, alpha=3, q_bits=40, p_bits=50, h_list=(8,)))
    A, B = I.matrix_pair(1, 8)
    a, b = ctx.encrypt(A.ravel(), nonce=1), ctx.encrypt(B.ravel(), nonce=2)
    x = other.encrypt(B.ravel(), nonce=2)
    assert _code(H, ctx.add, a, x) == EMISMATCH
    assert _code(H, ctx.rotate, x, 1) == EMISMATCH
    assert _code(H, ctx.matmul, a, x, 8) == EMISMATCH
    assert _code(H, ctx.matmul_batch, [a, a], [b, x], [8, 8]) == EMISMATCH
    assert _code(H, ctx.sign_approx, x, 3, 1) == EMISMATCH
    assert _code(H, ctx.export, x) == EMISMATCH
    srv = H.Server(ctx)
    try:
        assert _code(H, srv.submit, H.REQ_MATMUL, a, x, h=8) == EMISMATCH
    finally:
        srv.stop()
    # nothing was queued by the refused calls: the context still computes the same product
    got = ctx.export(ctx.matmul(a, b, 8))
    assert np.array_equal(got, ctx.export(ctx.matmul(a, b, 8)))
    other.close()


def test_import_rejects_residues_out_of_range(H, ctx):
    a = ctx.encrypt(I.matrix(3, 8).ravel(), nonce=3)
    words = ctx.export(a)
    lv, dg, sc = a.info()
    back = ctx.import_(words, lv, sc, dg)
    assert np.array_equal(ctx.export(back), words)
    for (p, i, t) in [(0, 0, 5), (1, lv, ctx.n - 1)]:
        bad = words.copy()
        bad[p, i, t] = ctx.moduli[i]  # q_i itself: one past the largest residue
        assert _code(H, ctx.import_, bad, lv, sc, dg) == EINVAL
    bad = words.copy()
    bad[0, 1, 0] = np.uint64(2 ** 63)
    assert _code(H, ctx.import_, bad, lv, sc, dg) == EINVAL


def _launches(ctx, fn):
    """kernel launches one call makes (from the launch-timing records)"""
    ctx.profile(True)
    try:
        fn()
        rep = ctx.profile_report()
    finally:
        ctx.profile(False)
    return sum(v["launches"] for v in rep.values())


def test_injected_launch_failure_fails_only_that_call(H, ctx):
    A, B = I.matrix_pair(4, 8)
    a, b = ctx.encrypt(A.ravel(), nonce=4), ctx.encrypt(B.ravel(), nonce=5)
    want = ctx.export(ctx.matmul(a, b, 8))
    n_prod = _launches(ctx, lambda: ctx.matmul(a, b, 8))
    n_batch = _launches(ctx, lambda: ctx.matmul_batch([a, a], [b, b], [8, 8]))
    _log(f"[robust] a product makes {n_prod} launches, a batch of two {n_batch}")
    assert n_prod > 10 and n_batch > 10
    try:
        for n in (1, n_prod // 2, n_prod):  # the first, a middle and the last launch
            _log(f"[robust] launch {n} of a product fails")
            H.fail_launch(n)
            assert _code(H, ctx.matmul, a, b, 8) == EDEVICE
            H.fail_launch(0)
            assert np.array_equal(ctx.export(ctx.matmul(a, b, 8)), want)
        _log(f"[robust] a batch whose launch {n_batch // 2} fails, then the same batch")
        H.fail_launch(n_batch // 2)
        assert _code(H, ctx.matmul_batch, [a, a], [b, b], [8, 8]) == EDEVICE
    finally:
        H.fail_launch(0)
    for r in ctx.matmul_batch([a, a], [b, b], [8, 8]):
        assert np.array_equal(ctx.export(r), want)


def test_injected_failure_in_a_two_stream_batch(H, ctx):
    """a batch of two shapes runs its groups on the context's two streams; a launch that fails
    on either stream fails the call with HE_EDEVICE, the queued work of the other stream drains
    before its buffers return to the cache, and the same batch then gives the residues of a
    clean run"""
    hs = [8, 8, 4, 4]
    As, Bs = [], []
    for i, h in enumerate(hs):
        A, B = I.matrix_pair(40 + i, h)
        As.append(ctx.encrypt(A.ravel(), nonce=40 + 2 * i))
        Bs.append(ctx.encrypt(B.ravel(), nonce=41 + 2 * i))
    ctx.set_tuning(4, 32, 0, 1)
    want = [ctx.export(r) for r in ctx.matmul_batch(As, Bs, hs)]
    n = _launches(ctx, lambda: ctx.matmul_batch(As, Bs, hs))
    _log(f"[robust] a two-shape batch makes {n} launches")
    try:
        for k in (n // 4, n // 2, (3 * n) // 4, n):
            _log(f"[robust] launch {k} of the two-stream batch fails")
            H.fail_launch(k)
            assert _code(H, ctx.matmul_batch, As, Bs, hs) == EDEVICE
            H.fail_launch(0)
            got = [ctx.export(r) for r in ctx.matmul_batch(As, Bs, hs)]
            assert all(np.array_equal(g, w) for g, w in zip(got, want))
    finally:
        H.fail_launch(0)


def test_pool_cap_gives_enomem_then_recovers(H, ctx):
    A, B = I.matrix_pair(6, 8)
    a, b = ctx.encrypt(A.ravel(), nonce=6), ctx.encrypt(B.ravel(), nonce=7)
    want = ctx.export(ctx.matmul(a, b, 8))
    ctx.sync()
    in_use, _ = ctx.pool_stats()
    try:
        # the cap at the bytes in use trims the cache; the product's first working buffer is
        # then beyond it and the call fails cleanly
        _log("[robust] product under a pool cap at the bytes in use")
        ctx.pool_limit(in_use + 1)
        assert _code(H, ctx.matmul, a, b, 8) == ENOMEM
    finally:
        ctx.pool_limit(0)
    assert np.array_equal(ctx.export(ctx.matmul(a, b, 8)), want)


def _wait(srv, tickets, timeout=60.0):
    out = {}
    deadline = time.time() + timeout
    while len(out) < len(tickets) and time.time() < deadline:
        for t in tickets:
            if t in out:
                continue
            try:
                r = srv.poll(t)
            except Exception as e:  # the request's own failure
                out[t] = e
                continue
            if r is not None:
                out[t] = r
        time.sleep(0.002)
    assert len(out) == len(tickets), "requests did not finish"
    return out


def test_server_fails_only_the_cohort_whose_launch_fails(H, ctx):
    """a product and a sign evaluation in flight together: the first launch of the next round
    fails (host-side injection); exactly one of the two requests fails with HE_EDEVICE, the
    other completes bit-identical to running it alone, and the server then serves both again"""
    A, B = I.matrix_pair(8, 8)
    a, b = ctx.encrypt(A.ravel(), level=7, nonce=8), ctx.encrypt(B.ravel(), level=7, nonce=9)
    x = ctx.encrypt(I.sign_inputs(9, 1, 16)[0].ravel(), level=7, nonce=10)
    want = {"mm": ctx.export(ctx.matmul(a, b, 8)), "sg": ctx.export(ctx.sign_approx(x, 3, 1, 0))}
    srv = H.Server(ctx)
    try:
        H.fail_launch(1)
        tm = srv.submit(H.REQ_MATMUL, a, b, h=8)
        ts = srv.submit(H.REQ_SIGN, x, d=3, k=1, mode=0)
        res = _wait(srv, [tm, ts])
        H.fail_launch(0)
        failed = [t for t, r in res.items() if isinstance(r, Exception)]
        assert len(failed) == 1, res
        assert isinstance(res[failed[0]], H.HEError) and res[failed[0]].code == EDEVICE
        for t, key in ((tm, "mm"), (ts, "sg")):
            if t not in failed:
                assert np.array_equal(ctx.export(res[t][0]), want[key])
        _log("[robust] server after the failure")
        t2 = [srv.submit(H.REQ_MATMUL, a, b, h=8), srv.submit(H.REQ_SIGN, x, d=3, k=1, mode=0)]
        res = _wait(srv, t2)
        assert np.array_equal(ctx.export(res[t2[0]][0]), want["mm"])
        assert np.array_equal(ctx.export(res[t2[1]][0]), want["sg"])
    finally:
        H.fail_launch(0)
        srv.stop()
