"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Integer results (every ciphertext residue, exported in the coefficient domain)
must be bit-identical; decrypted values must be within the stated bound of the
FP64 product.  Both sides receive the same seeded inputs from
paper_2207_04620_amd.inputs and derive everything else from the seed.
"""
import math
import os
import sys

import numpy as np
import pytest

import oracle as O
from paper_2207_04620_amd import inputs as I

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def he():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2207_04620_amd import he as H
    H.lib()
    return H


class Pair:
    def __init__(self, H, prm, h_list=None, schedule=0):
        _log(f"[parity] context {prm.name} N=2^{prm.log_n} h={h_list if h_list is not None else prm.h_list}")
        self.prm = prm
        self.g = H.Context(prm, schedule=schedule, h_list=h_list)
        self.o = O.Ctx.from_params(prm)

    def same(self, gct, oct_):
        g = self.g.export(gct)
        o = oct_.export()
        assert g.shape == o.shape, (g.shape, o.shape)
        bad = np.argwhere(g != o)
        assert bad.size == 0, f"{len(bad)} residues differ, first at {bad[:3].tolist()}"
        lv, dg, sc = gct.info()
        assert lv == oct_.level and dg == oct_.degree
        assert sc == pytest.approx(oct_.scale, rel=1e-12)


@pytest.fixture(scope="module")
def small(he):
    return Pair(he, I.small(log_n=12, n_q=6, alpha=2, q_bits=40, p_bits=50), h_list=[4, 8, 16])


@pytest.fixture(scope="module")
def c1p(he):
    return Pair(he, I.C1P)


def test_moduli_match(small):
    assert small.g.moduli == small.o.moduli


@pytest.mark.parametrize("log_n", [8, 10, 11, 12, 13, 14, 15, 16, 17])
def test_ntt_matches_oracle_evaluation_order(he, log_n):
    import torch
    prm = I.Params(f"ntt{log_n}", log_n, [60, 45, 40], [50], 1, 40.0, 3, [])
    _log(f"[parity] ntt log_n={log_n}")
    g = he.Context(prm, h_list=[])
    o = O.Ctx.from_params(prm)
    x = I.residues(log_n, (len(g.moduli), g.n), g.moduli)
    t = torch.from_numpy(x.view(np.int64)).cuda()
    g.ntt(t, list(range(len(g.moduli))))
    torch.cuda.synchronize()
    got = t.cpu().numpy().view(np.uint64)
    for mi in range(len(g.moduli)):
        assert np.array_equal(got[mi], o.eval_bitrev(mi, x[mi])), f"limb {mi}"
    g.ntt(t, list(range(len(g.moduli))), inverse=True)
    torch.cuda.synchronize()
    assert np.array_equal(t.cpu().numpy().view(np.uint64), x)


def test_encode_matches_oracle(small):
    z = I.matrix(3, 16).ravel()
    a = small.g.encode(z)
    b, tie = small.o.encode(z)
    assert tie > 1e-9 and np.array_equal(a, b)


@pytest.mark.parametrize("level", [5, 2, 0])
def test_encrypt_coeffs_parity(small, level):
    m = I.plaintext_poly(level, small.g.n, 2 ** 35)
    gct = small.g.encrypt_coeffs(m, level, 2.0 ** 40, nonce=11 + level)
    oct_ = small.o.encrypt_coeffs(m, level, 2.0 ** 40, nonce=11 + level)
    small.same(gct, oct_)
    assert np.array_equal(small.g.decrypt_coeffs(gct), small.o.decrypt_coeffs(oct_))


def test_encrypt_values_parity_and_roundtrip(small):
    z = I.matrix(4, 16).ravel()
    gct, oct_ = small.g.encrypt(z, nonce=3), small.o.encrypt(z, nonce=3)
    small.same(gct, oct_)
    assert np.abs(small.g.decrypt(gct, 256) - z).max() < 1e-6


def test_add_sub_drop_rescale_parity(small):
    a, b = I.matrix_pair(5, 16)
    ga, gb = small.g.encrypt(a.ravel(), nonce=1), small.g.encrypt(b.ravel(), level=4, nonce=2)
    oa, ob = small.o.encrypt(a.ravel(), nonce=1), small.o.encrypt(b.ravel(), level=4, nonce=2)
    small.same(small.g.add(ga, gb), small.o.add(oa, ob))
    small.same(small.g.sub(ga, gb), small.o.sub(oa, ob))
    small.same(small.g.drop(ga, 3), small.o.drop(oa, 3))
    small.same(small.g.rescale(ga), small.o.rescale(oa))


def test_mul_relin_rescale_parity(small):
    a, b = I.matrix_pair(6, 16)
    ga, gb = small.g.encrypt(a.ravel(), nonce=4), small.g.encrypt(b.ravel(), nonce=5)
    oa, ob = small.o.encrypt(a.ravel(), nonce=4), small.o.encrypt(b.ravel(), nonce=5)
    gt, ot = small.g.tensor(ga, gb), small.o.tensor(oa, ob)
    small.same(gt, ot)
    gr, orr = small.g.relin(gt), small.o.relin(ot)
    small.same(gr, orr)
    gs, os_ = small.g.rescale(gr), small.o.rescale(orr)
    small.same(gs, os_)
    assert np.abs(small.g.decrypt(gs, 256) - (a * b).ravel()).max() < 1e-3


def test_mul_plain_and_int_parity(small):
    a = I.matrix(7, 16).ravel()
    ga, oa = small.g.encrypt(a, nonce=6), small.o.encrypt(a, nonce=6)
    pt = I.plaintext_poly(7, small.g.n, 2 ** 20)
    small.same(small.g.mul_plain(ga, pt, 2.0 ** 20), small.o.mul_plain(oa, pt, 2.0 ** 20))
    for k in (3, -5, 2 ** 44 + 1, -(2 ** 50)):
        small.same(small.g.mul_int(ga, k), small.o.mul_int(oa, k))


@pytest.mark.parametrize("k", [1, 3, -1, -7, 16, 100, 1023, 2047])
def test_rotate_parity(small, k):
    a = I.matrix(8, 16).ravel()
    ga, oa = small.g.encrypt(a, nonce=7), small.o.encrypt(a, nonce=7)
    small.g.gen_rotation_key(k)
    gr, orr = small.g.rotate(ga, k), small.o.rotate(oa, k)
    small.same(gr, orr)
    assert np.abs(small.g.decrypt(gr, 256) - np.roll(a, -k)).max() < 1e-6


def test_rotate_lower_level_parity(small):
    a = I.matrix(9, 16).ravel()
    ga, oa = small.g.drop(small.g.encrypt(a, nonce=8), 1), small.o.drop(small.o.encrypt(a, nonce=8), 1)
    small.g.gen_rotation_key(5)
    small.same(small.g.rotate(ga, 5), small.o.rotate(oa, 5))


def test_missing_key_is_reported(small, he):
    ga = small.g.encrypt(np.zeros(4), nonce=1)
    with pytest.raises(he.HEError) as e:
        small.g.rotate(ga, 777)
    assert e.value.name == "HE_EKEY"


@pytest.mark.parametrize("h", [4, 8, 16])
def test_matmul_parity_small(small, h):
    A, B = I.matrix_pair(20 + h, h)
    _log(f"[parity] matmul small h={h}")
    ga, gb = small.g.encrypt(A.ravel(), nonce=30), small.g.encrypt(B.ravel(), nonce=31)
    oa, ob = small.o.encrypt(A.ravel(), nonce=30), small.o.encrypt(B.ravel(), nonce=31)
    small.g.counters(reset=True)
    small.o.reset_counters()
    gm = small.g.matmul(ga, gb, h)
    om = small.o.matmul(oa, ob, h)
    small.same(gm, om)
    gc, oc = small.g.counters(), small.o.counters()
    for key in ("rot", "keyswitch", "mul_pt", "mul_ct", "rescale"):
        assert gc[key] == oc[key], key
    assert np.abs(small.g.decrypt(gm, h * h).reshape(h, h) - A @ B).max() < 1e-3


def test_modup_conversion_launch_forms(he):
    """one digit per prime (8 digits): at the top level the 8 digits' 72 targets exceed one
    merged ModUp conversion launch, so each digit converts in its own launch; after the first
    rescales the digits fit one launch.  A product through both forms, single and as a batch of
    two, equals the oracle on every residue"""
    prm = I.small(log_n=12, n_q=8, alpha=1, q_bits=40, p_bits=50)
    p = Pair(he, prm, h_list=[4])
    A, B = I.matrix_pair(77, 4)
    ga, gb = p.g.encrypt(A.ravel(), nonce=40), p.g.encrypt(B.ravel(), nonce=41)
    oa, ob = p.o.encrypt(A.ravel(), nonce=40), p.o.encrypt(B.ravel(), nonce=41)
    om = p.o.matmul(oa, ob, 4)
    p.same(p.g.matmul(ga, gb, 4), om)
    A2, B2 = I.matrix_pair(78, 4)
    ga2, gb2 = p.g.encrypt(A2.ravel(), nonce=42), p.g.encrypt(B2.ravel(), nonce=43)
    res = p.g.matmul_batch([ga, ga2], [gb, gb2], [4, 4])
    p.same(res[0], om)
    assert np.abs(p.g.decrypt(res[1], 16).reshape(4, 4) - A2 @ B2).max() < 1e-3


def test_matmul_relin_once_parity(he):
    prm = I.small(log_n=12, n_q=6, alpha=2, q_bits=40, p_bits=50)
    p = Pair(he, prm, h_list=[8], schedule=1)
    A, B = I.matrix_pair(77, 8)
    gm = p.g.matmul(p.g.encrypt(A.ravel(), nonce=1), p.g.encrypt(B.ravel(), nonce=2), 8)
    om = p.o.matmul(p.o.encrypt(A.ravel(), nonce=1), p.o.encrypt(B.ravel(), nonce=2), 8, O.RELIN_ONCE)
    p.same(gm, om)


SCHEDULES = [2, 4, 3, 5, 6, 7, 8, 9, 14, 15]  # flag combinations beyond relin-each / relin-once


@pytest.mark.parametrize("schedule", SCHEDULES)
def test_matmul_schedule_parity(he, schedule):
    """each schedule flag combination is its own reference: the oracle run with the same
    flags must agree on every residue, and on the operation counts"""
    prm = I.small(log_n=12, n_q=6, alpha=2, q_bits=40, p_bits=50)
    p = Pair(he, prm, h_list=[4, 16], schedule=schedule)
    for h in (4, 16):
        _log(f"[parity] matmul schedule={schedule} h={h}")
        A, B = I.matrix_pair(90 + schedule + h, h)
        ga, gb = p.g.encrypt(A.ravel(), nonce=3), p.g.encrypt(B.ravel(), nonce=4)
        oa, ob = p.o.encrypt(A.ravel(), nonce=3), p.o.encrypt(B.ravel(), nonce=4)
        p.g.counters(reset=True)
        p.o.reset_counters()
        gm = p.g.matmul(ga, gb, h)
        om = p.o.matmul(oa, ob, h, schedule)
        p.same(gm, om)
        gc, oc = p.g.counters(), p.o.counters()
        for key in ("rot", "keyswitch", "mul_pt", "mul_ct", "rescale"):
            assert gc[key] == oc[key], (key, gc[key], oc[key])
        assert np.abs(p.g.decrypt(gm, h * h).reshape(h, h) - A @ B).max() < 1e-3
    # a batch of mixed sides and levels under the same schedule equals the single products
    pairs = [(4, 5), (16, 4), (4, 3)]
    As, Bs, hs, singles = [], [], [], []
    for i, (h, lvl) in enumerate(pairs):
        A, B = I.matrix_pair(300 + i, h)
        a = p.g.encrypt(A.ravel(), level=lvl, nonce=10 + 2 * i)
        b = p.g.encrypt(B.ravel(), level=lvl, nonce=11 + 2 * i)
        As.append(a), Bs.append(b), hs.append(h)
        singles.append(p.g.export(p.g.matmul(a, b, h)))
    for r, s in zip(p.g.matmul_batch(As, Bs, hs), singles):
        assert np.array_equal(p.g.export(r), s)


@pytest.mark.parametrize("log_n", [8, 10])
@pytest.mark.parametrize("schedule", [2, 15])
def test_matmul_rings_of_few_blocks(he, log_n, schedule):
    """rings with fewer than eight 256-slot blocks per limb (the rotation-set launches number
    their blocks without the XCD grouping there): single and batched products bit-exact"""
    prm = I.small(log_n=log_n, n_q=5, alpha=2, q_bits=40, p_bits=50, h_list=(4, 8))
    p = Pair(he, prm, schedule=schedule)
    for h in (4, 8):
        _log(f"[parity] matmul N=2^{log_n} schedule={schedule} h={h}")
        A, B = I.matrix_pair(500 + log_n + h, h)
        gm = p.g.matmul(p.g.encrypt(A.ravel(), nonce=1), p.g.encrypt(B.ravel(), nonce=2), h)
        om = p.o.matmul(p.o.encrypt(A.ravel(), nonce=1), p.o.encrypt(B.ravel(), nonce=2), h, schedule)
        p.same(gm, om)
    As, Bs, singles = [], [], []
    for i in range(3):
        A, B = I.matrix_pair(520 + i, 8)
        a, b = p.g.encrypt(A.ravel(), nonce=20 + 2 * i), p.g.encrypt(B.ravel(), nonce=21 + 2 * i)
        As.append(a), Bs.append(b)
        singles.append(p.g.export(p.g.matmul(a, b, 8)))
    for r, s1 in zip(p.g.matmul_batch(As, Bs, [8, 8, 8]), singles):
        assert np.array_equal(p.g.export(r), s1)


def test_c1_as_stated_primitives(he):
    """C1 exactly as stated (N = 2^12, q0 40 bits, q1 30 bits, P 40 bits, scale 2^30: one
    rescale level): encryption of an h = 8 matrix, one multiply (Fig. 1 Mul_ct: tensor +
    relinearisation, then RS) and rotations by 1 and by h, every residue against the oracle;
    the product decrypts to the slot-wise product within 1e-3 of FP64"""
    p = Pair(he, I.C1, h_list=[])
    A, B = I.matrix_pair(11, 8)
    ga, gb = p.g.encrypt(A.ravel(), nonce=1), p.g.encrypt(B.ravel(), nonce=2)
    oa, ob = p.o.encrypt(A.ravel(), nonce=1), p.o.encrypt(B.ravel(), nonce=2)
    p.same(ga, oa)
    gm, om = p.g.rescale(p.g.mul(ga, gb)), p.o.rescale(p.o.mul(oa, ob))
    p.same(gm, om)
    assert gm.info()[0] == 0
    assert np.abs(p.g.decrypt(gm, 64) - (A * B).ravel()).max() < 1e-3
    for k in (1, 8):
        p.g.gen_rotation_key(k)
        p.same(p.g.rotate(ga, k), p.o.rotate(oa, k))


def test_matmul_fast_schedule_c1plus_bound(he):
    """the stated accuracy (1e-3 at scale 2^30, 2^12 ring, h = 8) under all four flags"""
    p = Pair(he, I.C1P, schedule=15)
    A, B = I.matrix_pair(2, 8)
    gm = p.g.matmul(p.g.encrypt(A.ravel(), nonce=1), p.g.encrypt(B.ravel(), nonce=2), 8)
    om = p.o.matmul(p.o.encrypt(A.ravel(), nonce=1), p.o.encrypt(B.ravel(), nonce=2), 8, 15)
    p.same(gm, om)
    assert np.abs(p.g.decrypt(gm, 64).reshape(8, 8) - A @ B).max() < 1e-3


def test_matmul_c1plus_parity_and_bound(c1p):
    """the h=8 product on the 2^12 ring at scale 2^30: bit-exact, and within 1e-3 of FP64"""
    A, B = I.matrix_pair(1, 8)
    gm = c1p.g.matmul(c1p.g.encrypt(A.ravel(), nonce=1), c1p.g.encrypt(B.ravel(), nonce=2), 8)
    om = c1p.o.matmul(c1p.o.encrypt(A.ravel(), nonce=1), c1p.o.encrypt(B.ravel(), nonce=2), 8)
    c1p.same(gm, om)
    err = np.abs(c1p.g.decrypt(gm, 64).reshape(8, 8) - A @ B).max()
    _log(f"[parity] C1+ h=8 max abs error {err:.3e}")
    assert err < 1e-3


def test_matmul_shape_and_level_errors(small, he):
    ga = small.g.encrypt(np.zeros(16), nonce=1)
    with pytest.raises(he.HEError) as e:
        small.g.matmul(ga, ga, 6)
    assert e.value.name == "HE_ESHAPE"
    with pytest.raises(he.HEError) as e:
        small.g.matmul(ga, ga, 64)
    assert e.value.name == "HE_ESHAPE"
    with pytest.raises(he.HEError) as e:
        small.g.matmul(small.g.drop(ga, 2), ga, 4)
    assert e.value.name == "HE_ELEVEL"


def test_matmul_batch_equals_single(small):
    pairs = [(4, 5), (8, 5), (16, 4), (8, 3)]
    As, Bs, hs, singles = [], [], [], []
    for i, (h, lvl) in enumerate(pairs):
        A, B = I.matrix_pair(200 + i, h)
        a = small.g.encrypt(A.ravel(), level=lvl, nonce=100 + 2 * i)
        b = small.g.encrypt(B.ravel(), level=lvl, nonce=101 + 2 * i)
        As.append(a), Bs.append(b), hs.append(h)
        singles.append(small.g.export(small.g.matmul(a, b, h)))
    res = small.g.matmul_batch(As, Bs, hs)
    for r, s in zip(res, singles):
        assert np.array_equal(small.g.export(r), s)


def test_matmul_batch_beyond_group_cap(he):
    """33 products of one shape and level under the headline schedule: a full lockstep group
    of 32 and a ragged group of 1 (the cap on the working set); every result equals the product
    run alone, and the lone member equals the oracle"""
    prm = I.small(log_n=12, n_q=6, alpha=2, q_bits=40, p_bits=50)
    p = Pair(he, prm, h_list=[8], schedule=15)
    As, Bs, mats = [], [], []
    for i in range(33):
        A, B = I.matrix_pair(300 + i, 8)
        mats.append((A, B))
        As.append(p.g.encrypt(A.ravel(), nonce=2 * i))
        Bs.append(p.g.encrypt(B.ravel(), nonce=2 * i + 1))
    res = p.g.matmul_batch(As, Bs, [8] * 33)
    for i in (0, 17, 31, 32):
        assert np.array_equal(p.g.export(res[i]), p.g.export(p.g.matmul(As[i], Bs[i], 8))), i
    for i, (A, B) in enumerate(mats):
        assert np.abs(p.g.decrypt(res[i], 64).reshape(8, 8) - A @ B).max() < 1e-3, i
    A, B = mats[32]
    om = p.o.matmul(p.o.encrypt(A.ravel(), nonce=64), p.o.encrypt(B.ravel(), nonce=65), 8, 15)
    p.same(res[32], om)


# coefficients of x, x^3, x^5, ... of g_1 .. g_4 as printed in Sec. 4.2
GD_COEF = {1: [3 / 2, -1 / 2], 2: [15 / 8, -10 / 8, 3 / 8], 3: [35 / 16, -35 / 16, 21 / 16, -5 / 16],
           4: [315 / 128, -420 / 128, 378 / 128, -180 / 128, 35 / 128]}


def _gdk(d, k, x):
    """g_d^(k) in FP64 from the printed coefficients"""
    y = np.asarray(x, np.float64).copy()
    for _ in range(k):
        y = sum(c * y ** (2 * i + 1) for i, c in enumerate(GD_COEF[d]))
    return y


@pytest.mark.parametrize("d,k,mode", [(3, 1, 0), (1, 2, 0), (2, 1, 0), (3, 1, 1), (4, 1, 0), (4, 1, 1)])
def test_sign_parity(he, d, k, mode):
    """g_d^(k) and ReLU on a 2^12 ring, every residue against the oracle; g_4 is the polynomial
    of the paper's experiments (x^9 term: the powers x^2, x^4, x^8, depth 4 per composition)"""
    prm = I.small(log_n=12, n_q=8, alpha=3, q_bits=40, p_bits=50)
    p = Pair(he, prm, h_list=[])
    X = I.sign_inputs(5, 1, 16)[0].ravel()
    gx, ox = p.g.encrypt(X, nonce=9), p.o.encrypt(X, nonce=9)
    gy, oy = p.g.sign_approx(gx, d, k, mode), p.o.sign(ox, d, k, relu=bool(mode))
    p.same(gy, oy)
    y = _gdk(d, k, X)
    want = (X + X * y) / 2 if mode else y
    assert np.abs(p.g.decrypt(gy, 256) - want).max() < 1e-3


@pytest.mark.parametrize("log_n", [13, 17])
def test_relu_parity_ring_sizes(he, log_n):
    """every relinearisation goes through the fused base conversion + forward column pass;
    N = 2^13 has 2 column stages, N = 2^17 has 6 (the generic column rounds): bit-exact
    residues against the oracle, ModUp digits of 3 limbs, a 2-prime P"""
    prm = I.small(log_n=log_n, n_q=8, alpha=3, q_bits=40, p_bits=50)
    _log(f"[parity] relu d=3 k=1 at N=2^{log_n}")
    p = Pair(he, prm, h_list=[])
    X = I.sign_inputs(5, 1, 16)[0].ravel()
    gx, ox = p.g.encrypt(X, nonce=9), p.o.encrypt(X, nonce=9)
    gy, oy = p.g.sign_approx(gx, 3, 1, 1), p.o.sign(ox, 3, 1, relu=True)
    p.same(gy, oy)
    y = sum(c * X ** (2 * i + 1) for i, c in enumerate([35 / 16, -35 / 16, 21 / 16, -5 / 16]))
    assert np.abs(p.g.decrypt(gy, 256) - (X + X * y) / 2).max() < 1e-3


@pytest.mark.parametrize("schedule", [0, 15])
def test_largest_shape_for_ring_and_empty_batch(he, schedule):
    """h^2 = N/2 (N = 2^13, h = 64): one replica of the matrix, so every Step-2 and Step-3
    rotation spans the whole slot vector; every residue against the oracle under Alg. 3 as
    printed (0) and the headline schedule (15).  An empty batch returns nothing."""
    prm = I.small(log_n=13, n_q=6, alpha=2, q_bits=40, p_bits=50)
    _log(f"[parity] h=64 at N=2^13, schedule {schedule}")
    p = Pair(he, prm, h_list=[64], schedule=schedule)
    assert p.g.matmul_batch([], [], []) == []
    A, B = I.matrix_pair(64 + schedule, 64)
    gm = p.g.matmul(p.g.encrypt(A.ravel(), nonce=40), p.g.encrypt(B.ravel(), nonce=41), 64)
    om = p.o.matmul(p.o.encrypt(A.ravel(), nonce=40), p.o.encrypt(B.ravel(), nonce=41), 64, schedule)
    p.same(gm, om)
    assert np.abs(p.g.decrypt(gm, 64 * 64).reshape(64, 64) - A @ B).max() < 1e-3


# ---------------------------------------------------------------- full-size configurations
def test_c2_h64_matmul_parity(he):
    """N=2^14, 7 x 40-bit Q + 60-bit P, scale 2^40: the whole h=64 product, every residue"""
    p = Pair(he, I.C2)
    A, B = I.matrix_pair(2, 64)
    ga, gb = p.g.encrypt(A.ravel(), nonce=1), p.g.encrypt(B.ravel(), nonce=2)
    oa, ob = p.o.encrypt(A.ravel(), nonce=1), p.o.encrypt(B.ravel(), nonce=2)
    p.same(ga, oa)
    _log("[parity] C2 h=64 GPU matmul")
    gm = p.g.matmul(ga, gb, 64)
    _log("[parity] C2 h=64 oracle matmul")
    om = p.o.matmul(oa, ob, 64)
    p.same(gm, om)
    err = np.abs(p.g.decrypt(gm, 4096).reshape(64, 64) - A @ B).max()
    _log(f"[parity] C2 h=64 max abs error {err:.3e}")
    assert err < 1e-3


def test_c3_rotations_and_h16_matmul_parity(he):
    """N=2^15, Q = 60 + 13 x 45, P = 3 x 60 + 56, alpha 5 (dnum 3), scale 2^45"""
    p = Pair(he, I.C3, h_list=[16])
    A, B = I.matrix_pair(3, 16)
    for lvl in (13, 7, 3):
        ga, oa = p.g.encrypt(A.ravel(), level=lvl, nonce=lvl), p.o.encrypt(A.ravel(), level=lvl, nonce=lvl)
        for k in (1, 16, -15):
            p.same(p.g.rotate(ga, k), p.o.rotate(oa, k))
    ga, gb = p.g.encrypt(A.ravel(), level=9, nonce=40), p.g.encrypt(B.ravel(), level=9, nonce=41)
    oa, ob = p.o.encrypt(A.ravel(), level=9, nonce=40), p.o.encrypt(B.ravel(), level=9, nonce=41)
    _log("[parity] C3 h=16 matmul")
    gm = p.g.matmul(ga, gb, 16)
    om = p.o.matmul(oa, ob, 16)
    p.same(gm, om)
    assert np.abs(p.g.decrypt(gm, 256).reshape(16, 16) - A @ B).max() < 1e-6


@pytest.fixture(scope="module")
def c3_oracle():
    """one oracle context for the N=2^15 configuration, shared by the tests below so that its
    rotation keys (cached per Galois element) are made once"""
    return O.Ctx.from_params(I.C3)


def _oracle_member(o, pairs, i, lvl, h, mode):
    A, B = pairs[i]
    return o.matmul(o.encrypt(A.ravel(), level=lvl, nonce=2 * i), o.encrypt(B.ravel(), level=lvl, nonce=2 * i + 1),
                    h, mode).export()


def _same_residues(gexp, oexp, what):
    assert gexp.shape == oexp.shape, (what, gexp.shape, oexp.shape)
    bad = np.argwhere(gexp != oexp)
    assert bad.size == 0, f"{what}: {len(bad)} residues differ, first at {bad[:3].tolist()}"


@pytest.mark.parametrize("schedule", [15, 0])
def test_c3_h64_batch16_full_size(he, c3_oracle, schedule):
    """the benchmarked configuration itself: a batch of 16 h=64 products on the N=2^15 ring
    from level 13, through the batched entry point the benchmark times, under the headline
    schedule (all four flags) and under Alg. 3 as printed (schedule 0: relinearisation of every
    Step-3 product, one ModDown per rotation, every A^(k) rescaled, Step 3 unsplit).  The
    first and the last member against the oracle in the same schedule on every residue; every
    member within the FP64 bound of A B, and member 5 equal to the same product run alone."""
    prm = I.C3
    g = he.Context(prm, h_list=[64], schedule=schedule)
    pairs = [I.matrix_pair(1000 + i, 64) for i in range(16)]
    As = [g.encrypt(A.ravel(), level=13, nonce=2 * i) for i, (A, _) in enumerate(pairs)]
    Bs = [g.encrypt(B.ravel(), level=13, nonce=2 * i + 1) for i, (_, B) in enumerate(pairs)]
    _log(f"[parity] C3 h=64 batch 16, schedule {schedule}: GPU batch")
    out = g.matmul_batch(As, Bs, [64] * 16)
    for i, (A, B) in enumerate(pairs):
        err = np.abs(g.decrypt(out[i], 4096).reshape(64, 64) - A @ B).max()
        assert err < 1e-5, (i, err)
    _log(f"[parity] C3 h=64 schedule {schedule}: member 5 alone")
    assert np.array_equal(g.export(g.matmul(As[5], Bs[5], 64)), g.export(out[5]))
    for i in (0, 15):
        _log(f"[parity] C3 h=64 schedule {schedule}: oracle, member {i}")
        _same_residues(g.export(out[i]), _oracle_member(c3_oracle, pairs, i, 13, 64, schedule), f"member {i}")
    _log(f"[parity] C3 h=64 schedule {schedule}: bit-exact")
    g.close()


def test_c3_mixed_batch_parity(he, c3_oracle):
    """a batch of products of mixed h in {16, 32, 64} and starting levels in [3, 13] on the
    N=2^15 ring (the mixed-batch configuration, 24 of its members): one batched call; every
    member within the FP64 bound at its own output level, equal to the same product run
    alone, and four members equal to the oracle on every residue: the first h=16 and h=32
    members, the first h=64 member (level 7) and the h=64 member that starts at the lowest
    level a product accepts (3)"""
    prm = I.C3
    g = he.Context(prm, h_list=[16, 32, 64], schedule=15)
    mix = I.batch_mix(3, 24)
    _log(f"[parity] C3 mixed batch: {mix}")
    pairs = [I.matrix_pair(500 + i, h) for i, (h, _) in enumerate(mix)]
    As = [g.encrypt(A.ravel(), level=lv, nonce=2 * i) for i, ((A, _), (_, lv)) in enumerate(zip(pairs, mix))]
    Bs = [g.encrypt(B.ravel(), level=lv, nonce=2 * i + 1) for i, ((_, B), (_, lv)) in enumerate(zip(pairs, mix))]
    out = g.matmul_batch(As, Bs, [h for h, _ in mix])
    for i, ((A, B), (h, lv)) in enumerate(zip(pairs, mix)):
        assert out[i].info()[0] == lv - 3
        err = np.abs(g.decrypt(out[i], h * h).reshape(h, h) - A @ B).max()
        assert err < 1e-5, (i, h, lv, err)
    _log("[parity] C3 mixed batch: singles")
    for i in range(8):
        h = mix[i][0]
        assert np.array_equal(g.export(g.matmul(As[i], Bs[i], h)), g.export(out[i])), i
    picks = [next(j for j, (h, _) in enumerate(mix) if h == want) for want in (16, 32, 64)]
    picks.append(next(j for j, (h, lv) in enumerate(mix) if h == 64 and lv == 3))
    for i in picks:
        h, lv = mix[i]
        _log(f"[parity] C3 mixed batch: oracle member {i} (h={h}, level {lv})")
        _same_residues(g.export(out[i]), _oracle_member(c3_oracle, pairs, i, lv, h, 15), f"member {i}")
    g.close()


def test_c4_sign_relu_then_h32_matmul(he):
    """the sign/ReLU configuration on the N=2^16 ring (Q = 60 + 16 x 45, P = 5 x 60, dnum 3):
    a batch of ReLU(x) = (x + x g_3^(3)(x)) / 2 over 32 x 32 inputs with |x| in [2^-8, 1],
    then an h=32 product of each result with one encrypted W.  Member 0 against the oracle on
    every residue (both stages), and so is the last member; every member within 1e-3 of the FP64
    evaluation"""
    prm = I.C4
    count = 16
    g = he.Context(prm, h_list=[32], schedule=15)
    X = I.sign_inputs(4, count, 32)
    W = np.random.default_rng(4).uniform(-1.0, 1.0, (32, 32))
    xs = [g.encrypt(X[i].ravel(), nonce=i + 1) for i in range(count)]
    _log("[parity] C4 ReLU batch")
    ys = g.sign_approx_batch(xs, 3, 3, he.RELU)
    lvl = ys[0].info()[0]
    w = g.encrypt(W.ravel(), level=lvl, nonce=1000)
    _log(f"[parity] C4 h=32 products at level {lvl}")
    ms = g.matmul_batch(ys, [w] * count, [32] * count)

    def g3(v):
        return (35 * v - 35 * v ** 3 + 21 * v ** 5 - 5 * v ** 7) / 16

    for i in range(count):
        x = X[i]
        s = g3(g3(g3(x)))
        relu = (x + x * s) / 2
        assert np.abs(g.decrypt(ys[i], 1024).reshape(32, 32) - relu).max() < 1e-3, i
        assert np.abs(g.decrypt(ms[i], 1024).reshape(32, 32) - relu @ W).max() < 1e-3, i
    o = O.Ctx.from_params(prm)
    ow = o.encrypt(W.ravel(), level=lvl, nonce=1000)
    for i in (0, count - 1):
        _log(f"[parity] C4 oracle, member {i}")
        oy = o.sign(o.encrypt(X[i].ravel(), nonce=i + 1), 3, 3, relu=True)
        _same_residues(g.export(ys[i]), oy.export(), f"ReLU member {i}")
        _same_residues(g.export(ms[i]), o.matmul(oy, ow, 32, 15).export(), f"product member {i}")
    _log("[parity] C4: bit-exact")
    g.close()


@pytest.mark.parametrize("mode", [0, 1])
def test_c4_g4_sign_and_relu(he, mode):
    """g_4 (the polynomial of the paper's experiments, Sec. 4.2) at k = 1 on the N=2^16 ring:
    a batch of 8 sign (mode 0) or ReLU (mode 1) evaluations over 32 x 32 inputs with |x| in
    [2^-8, 1]; the first and the last member against the oracle on every residue, every member
    within 1e-3 of the FP64 evaluation of the printed polynomial"""
    prm = I.C4
    count = 8
    g = he.Context(prm, h_list=[], schedule=15)
    X = I.sign_inputs(44, count, 32)
    xs = [g.encrypt(X[i].ravel(), nonce=i + 1) for i in range(count)]
    _log(f"[parity] C4 g_4 k=1 mode {mode}: GPU batch")
    ys = g.sign_approx_batch(xs, 4, 1, mode)
    for i in range(count):
        x = X[i].ravel()
        y = _gdk(4, 1, x)
        want = (x + x * y) / 2 if mode else y
        assert np.abs(g.decrypt(ys[i], 1024) - want).max() < 1e-3, i
    o = O.Ctx.from_params(prm)
    for i in (0, count - 1):
        _log(f"[parity] C4 g_4 mode {mode}: oracle member {i}")
        oy = o.sign(o.encrypt(X[i].ravel(), nonce=i + 1), 4, 1, relu=bool(mode))
        _same_residues(g.export(ys[i]), oy.export(), f"member {i}")
    g.close()


# ---------------------------------------------------------------- App. C, D, E
def _packed(beta, h, seed):
    rng = np.random.default_rng(seed)
    return [rng.uniform(-1.0, 1.0, (h, h)) for _ in range(beta)]


@pytest.mark.parametrize("schedule", [0, 15])
def test_transpose_rect_packed_parity(he, schedule):
    """transposition (App. C), HE-RMatMult (Alg. 6) and iota_beta packing (App. E) on a 2^12
    ring: every result against the oracle on every residue (same schedule flags), decrypting
    to the FP64 transpose / product; mixed shapes in one batch equal their single runs"""
    prm = I.small(log_n=12, n_q=6, alpha=2, q_bits=40, p_bits=50)
    p = Pair(he, prm, h_list=[], schedule=schedule)
    H = he
    for h, beta in ((4, 1), (8, 1), (16, 1), (8, 4), (4, 8)):
        _log(f"[parity] transpose h={h} beta={beta} schedule={schedule}")
        mats = _packed(beta, h, 10 * h + beta)
        v = H.pack_beta(mats)
        g = p.g.transpose(p.g.encrypt(v, nonce=5), h, beta)
        o = p.o.transpose(p.o.encrypt(v, nonce=5), h, beta, schedule)
        p.same(g, o)
        got = p.g.decrypt(g, beta * h * h)
        for m in range(beta):
            assert np.abs(got[m::beta].reshape(h, h) - mats[m].T).max() < 1e-6
    shapes = [(8, 2, 1), (16, 4, 1), (16, 1, 1), (8, 8, 4), (8, 4, 2), (4, 4, 8)]
    As, Bs, want, sing = [], [], [], []
    for n_, (h, t, beta) in enumerate(shapes):
        _log(f"[parity] shaped product h={h} t={t} beta={beta} schedule={schedule}")
        rng = np.random.default_rng(100 + n_)
        A = [rng.uniform(-1, 1, (t, h)) for _ in range(beta)]
        B = [rng.uniform(-1, 1, (h, h)) for _ in range(beta)]
        va = H.pack_beta([np.tile(x, (h // t, 1)) for x in A])
        vb = H.pack_beta(B)
        ga, gb = p.g.encrypt(va, nonce=2 * n_), p.g.encrypt(vb, nonce=2 * n_ + 1)
        g = p.g.matmul_ex(ga, gb, h, t, beta)
        o = p.o.matmul_ex(p.o.encrypt(va, nonce=2 * n_), p.o.encrypt(vb, nonce=2 * n_ + 1), h, t, beta, schedule)
        p.same(g, o)
        got = p.g.decrypt(g, beta * h * h)
        for m in range(beta):
            M = got[m::beta].reshape(h, h)
            for blk in range(h // t):
                assert np.abs(M[blk * t:(blk + 1) * t] - A[m] @ B[m]).max() < 1e-3
        As.append(ga), Bs.append(gb), sing.append(p.g.export(g))
    batch = p.g.matmul_batch_ex(As, Bs, shapes)
    for r, s_ in zip(batch, sing):
        assert np.array_equal(p.g.export(r), s_)


def test_c3_packed_h64_beta4_full_size(he):
    """four h=64 products in one ciphertext pair on the N=2^15 ring (iota_4 fills all 16384
    slots): against the oracle on every residue under the headline schedule, and each of the
    four products within 1e-5 of FP64"""
    prm = I.C3
    g = he.Context(prm, h_list=[], schedule=15)
    As, Bs = _packed(4, 64, 31), _packed(4, 64, 32)
    va, vb = he.pack_beta(As), he.pack_beta(Bs)
    _log("[parity] C3 packed beta=4 h=64: GPU")
    gm = g.matmul_ex(g.encrypt(va, nonce=1), g.encrypt(vb, nonce=2), 64, 64, 4)
    got = g.decrypt(gm, 4 * 4096)
    for m in range(4):
        assert np.abs(got[m::4].reshape(64, 64) - As[m] @ Bs[m]).max() < 1e-5
    _log("[parity] C3 packed beta=4 h=64: oracle")
    o = O.Ctx.from_params(prm)
    om = o.matmul_ex(o.encrypt(va, nonce=1), o.encrypt(vb, nonce=2), 64, 64, 4, 15)
    assert np.array_equal(g.export(gm), om.export())
    g.close()


# ---------------------------------------------------------------- Alg. 5 AppMax, pooling; Alg. 6
def _appmax64(a, b, k, d=3):
    m = a - b
    return ((a + b) + m * _gdk(d, k, m)) / 2


def test_appmax_maxpool_flupdate_parity(he):
    """AppMax (Alg. 5) with g_3 and g_4, 2 x 2 max pooling and the aggregation step of Alg. 6 on a 2^12 ring:
    every result against the oracle on every residue, and within 1e-6 of the FP64 evaluation;
    batched AppMax equals single"""
    prm = I.small(log_n=12, n_q=14, alpha=2, q_bits=40, p_bits=50)
    p = Pair(he, prm, h_list=[])
    rng = np.random.default_rng(41)
    a, b = rng.uniform(-0.5, 0.5, 256), rng.uniform(-0.5, 0.5, 256)
    ga, gb = p.g.encrypt(a, nonce=1), p.g.encrypt(b, nonce=2)
    oa, ob = p.o.encrypt(a, nonce=1), p.o.encrypt(b, nonce=2)
    for k in (1, 3):
        _log(f"[parity] appmax d=3 k={k}")
        g = p.g.appmax(ga, gb, 3, k)
        p.same(g, p.o.appmax(oa, ob, 3, k))
        assert np.abs(p.g.decrypt(g, 256) - _appmax64(a, b, k)).max() < 1e-6
    for k in (1, 2):
        _log(f"[parity] appmax d=4 k={k}")
        g = p.g.appmax(ga, gb, 4, k)
        p.same(g, p.o.appmax(oa, ob, 4, k))
        assert np.abs(p.g.decrypt(g, 256) - _appmax64(a, b, k, 4)).max() < 1e-6
    gl = p.g.encrypt(b, level=9, nonce=3)
    batch = p.g.appmax_batch([ga, gb, ga], [gb, ga, gl], 3, 1)
    for r, (x, y) in zip(batch, [(ga, gb), (gb, ga), (ga, gl)]):
        assert np.array_equal(p.g.export(r), p.g.export(p.g.appmax(x, y, 3, 1)))
    _log("[parity] maxpool2 h=16")
    h = 16
    X = rng.uniform(-0.5, 0.5, (h, h))
    g = p.g.maxpool2(p.g.encrypt(X.ravel(), nonce=4), h, 3, 1)
    p.same(g, p.o.maxpool2(p.o.encrypt(X.ravel(), nonce=4), h, 3, 1))
    v = X.ravel()
    m1 = _appmax64(v, np.roll(v, -1), 1)
    assert np.abs(p.g.decrypt(g, h * h) - _appmax64(m1, np.roll(m1, -h), 1)).max() < 1e-6
    _log("[parity] fl_update n=20")
    n, coeff = 20, 0.1 / (16 * 20)
    W = rng.uniform(-1, 1, 512)
    G = [rng.uniform(-1, 1, 512) for _ in range(n)]
    gw = p.g.encrypt(W, nonce=100)
    gg = [p.g.encrypt(x, level=12 if i % 3 else 13, nonce=101 + i) for i, x in enumerate(G)]
    ow = p.o.encrypt(W, nonce=100)
    og = [p.o.encrypt(x, level=12 if i % 3 else 13, nonce=101 + i) for i, x in enumerate(G)]
    g = p.g.fl_update(gw, gg, coeff)
    p.same(g, p.o.fl_update(ow, og, coeff))
    assert np.abs(p.g.decrypt(g, 512) - (W - coeff * np.sum(G, axis=0))).max() < 1e-6
