"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Nothing here compares the oracle with itself: each check is a printed value of
the paper (tests/golden/, each file citing its passage), a closed form, an
invariant, brute force on tiny inputs, or an independent library (sympy, Python
big integers, numpy float64 at sizes where it is exact).
"""
import json
import math
import os
from decimal import Decimal, getcontext
from fractions import Fraction

import numpy as np
import pytest
import sympy

import ckks_noise as CN
import oracle as O
from paper_2207_04620_amd import inputs as I

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


@pytest.fixture(scope="module")
def tiny():
    # N = 16, a few 20/24-bit primes: brute force is cheap here
    return O.Ctx(4, [24, 20, 20], [24, 24], 1, 12.0, 11)


@pytest.fixture(scope="module")
def small():
    return O.Ctx.from_params(I.small(log_n=10, n_q=5, alpha=2))


# ---------------------------------------------------------------- integers
def test_mulmod_matches_python_ints():
    rng = np.random.default_rng(0)
    for _ in range(2000):
        q = int(rng.integers(3, 2 ** 62)) | 1
        a, b = int(rng.integers(0, q)), int(rng.integers(0, q))
        assert O.mulmod(a, b, q) == a * b % q


def test_is_prime_brute_force_and_sympy():
    small_primes = {n for n in range(2, 20000) if all(n % d for d in range(2, int(n ** 0.5) + 1))}
    for n in range(20000):
        assert O.is_prime(n) == (n in small_primes)
    rng = np.random.default_rng(1)
    for _ in range(300):
        n = int(rng.integers(2 ** 40, 2 ** 62)) | 1
        assert O.is_prime(n) == sympy.isprime(n)


@pytest.mark.parametrize("prm", [I.C1, I.C1P, I.C2, I.C3, I.C4], ids=lambda p: p.name)
def test_prime_chain(prm):
    """largest unused primes below 2^bits with q = 1 mod 2N, Q list then P list"""
    c = O.Ctx.from_params(prm, threads=2)
    m2n = 2 * prm.n
    used = []
    for q, bits in zip(c.moduli, prm.q_bits + prm.p_bits):
        assert sympy.isprime(q) and q % m2n == 1 and q < 2 ** bits and q > 2 ** (bits - 1)
        # no larger admissible prime of that size was skipped
        cand = (2 ** bits - 1) // m2n * m2n + 1
        while cand > q:
            assert cand in used or not sympy.isprime(cand)
            cand -= m2n
        used.append(q)
    assert len(set(c.moduli)) == len(c.moduli)


def test_psi_is_smallest_primitive_root(tiny):
    for i, q in enumerate(tiny.moduli):
        psi = tiny.psi(i)
        n = tiny.n
        assert pow(psi, n, q) == q - 1
        roots = [x for x in range(1, q) if pow(x, n, q) == q - 1]
        assert psi == min(roots)


# ---------------------------------------------------------------- NTT
def naive_negacyclic(a, b, q):
    n = len(a)
    out = [0] * n
    for i in range(n):
        for j in range(n):
            k = i + j
            if k < n:
                out[k] = (out[k] + a[i] * b[j]) % q
            else:
                out[k - n] = (out[k - n] - a[i] * b[j]) % q
    return out


@pytest.mark.parametrize("log_n", [3, 4, 5, 6])
def test_poly_mul_is_negacyclic_convolution(log_n):
    c = O.Ctx(log_n, [40, 30], [45], 1, 20.0, 5)
    rng = np.random.default_rng(log_n)
    for mi, q in enumerate(c.moduli):
        a = rng.integers(0, q, size=c.n, dtype=np.uint64)
        b = rng.integers(0, q, size=c.n, dtype=np.uint64)
        got = c.poly_mul(mi, a, b)
        want = naive_negacyclic([int(x) for x in a], [int(x) for x in b], q)
        assert [int(x) for x in got] == want


def test_eval_bitrev_is_evaluation_at_odd_powers(tiny):
    rng = np.random.default_rng(3)
    L = tiny.log_n
    for mi, q in enumerate(tiny.moduli):
        a = [int(x) for x in rng.integers(0, q, size=tiny.n)]
        got = tiny.eval_bitrev(mi, np.array(a, np.uint64))
        psi = tiny.psi(mi)
        for j in range(tiny.n):
            br = int(format(j, f"0{L}b")[::-1], 2)
            x = pow(psi, 2 * br + 1, q)
            assert int(got[j]) == sum(ai * pow(x, i, q) for i, ai in enumerate(a)) % q


# ---------------------------------------------------------------- ChaCha20 and samplers
def test_chacha20_rfc8439_block():
    g = gold("chacha20_rfc8439.json")
    out = O.chacha20_block(g["key_words"], g["counter"], g["nonce_words"])
    assert [format(x, "08x") for x in out] == g["out_words_hex"]


def test_stream_word_layout():
    # word w of (seed, purpose, index) = words 2(w%8), 2(w%8)+1 of block w/8
    seed, purpose, index = 0x1234_5678_9ABC_DEF0, 4, (7 << 16) | 3
    key = [seed & 0xFFFFFFFF, seed >> 32, 0, 0, 0, 0, 0, 0]
    nonce = [purpose, index & 0xFFFFFFFF, index >> 32]
    for w in (0, 1, 7, 8, 13, 1000):
        blk = O.chacha20_block(key, w // 8, nonce)
        assert O.word(seed, purpose, index, w) == blk[2 * (w % 8)] | (blk[2 * (w % 8) + 1] << 32)


def test_gauss_table_matches_decimal():
    getcontext().prec = 60
    sigma = Decimal("3.2")
    rho = [(-(Decimal(x * x)) / (2 * sigma * sigma)).exp() for x in range(20)]
    tot = rho[0] + 2 * sum(rho[1:])
    cum = rho[0]
    want = []
    for k in range(19):
        if k:
            cum += 2 * rho[k]
        want.append(int((cum / tot * (Decimal(2) ** 63)).to_integral_value(rounding="ROUND_FLOOR")))
    assert [int(x) for x in O.gauss_table()] == want


def test_sampler_distributions():
    n = 1 << 18
    t = O.sample_ternary(9, 1, 0, n)
    assert set(np.unique(t)) <= {-1, 0, 1}
    frac = [np.mean(t == v) for v in (-1, 0, 1)]
    assert max(abs(f - 1 / 3) for f in frac) < 0.01
    e = O.sample_gauss(9, 3, 0, n)
    assert np.abs(e).max() <= 19
    assert abs(e.mean()) < 0.03 and abs(e.std() - 3.2) < 0.03
    # chi-square against the discrete Gaussian on [-19, 19]
    xs = np.arange(-12, 13)
    p = np.exp(-(xs ** 2) / (2 * 3.2 ** 2))
    p /= np.exp(-(np.arange(-19, 20) ** 2) / (2 * 3.2 ** 2)).sum()
    obs = np.array([(e == x).sum() for x in xs])
    chi2 = ((obs - n * p) ** 2 / (n * p)).sum()
    assert chi2 < 60  # 25 bins; the 0.9999 quantile is about 58
    q = (1 << 45) + 12345
    u = O.sample_uniform(9, 2, 0, q, n)
    assert int(u.max()) < q and abs(u.astype(np.float64).mean() / q - 0.5) < 0.005


# ---------------------------------------------------------------- base conversion
def test_base_conversion_is_crt_lift_within_alpha_half(small):
    rng = np.random.default_rng(5)
    src = [1, 2]
    D = small.moduli[1] * small.moduli[2]
    for dst in (0, 3, len(small.q)):
        t = small.moduli[dst]
        x_int = [int(v) for v in rng.integers(0, D, size=small.n, dtype=np.uint64)] if D < 2 ** 63 else \
            [int.from_bytes(rng.bytes(16), "little") % D for _ in range(small.n)]
        res = np.array([[v % small.moduli[s] for v in x_int] for s in src], np.uint64)
        got = small.base_conv(src, dst, res)
        for v, g in zip(x_int[:512], got[:512]):
            # the lift is x + u D for an integer |u| <= len(src)/2
            ok = any((v + u * D - int(g)) % t == 0 for u in range(-1, 2))
            assert ok


def test_base_conversion_exact_for_small_centered_values(small):
    rng = np.random.default_rng(6)
    src = [1, 2, 3]
    D = math.prod(small.moduli[s] for s in src)
    vals = [int(v) for v in rng.integers(-(2 ** 40), 2 ** 40, size=small.n)]
    res = np.array([[v % small.moduli[s] for v in vals] for s in src], np.uint64)
    got = small.base_conv(src, 0, res)
    q0 = small.moduli[0]
    # |x| << D / (2 n_src): the centered lift sum y_s D/q_s equals x + u D with u in {-1,0,1};
    # the oracle's result must be one of these residues.
    for v, g in zip(vals, got):
        assert any((v + u * D) % q0 == int(g) for u in (-1, 0, 1))


# ---------------------------------------------------------------- encoding
def test_encode_constant_is_constant_polynomial(small):
    m, _ = small.encode(np.full(7, 0.25), scale=2.0 ** 30)
    assert m[0] == 2 ** 28 and not np.any(m[1:])


def test_encode_matches_direct_formula_float64(tiny):
    # N = 16: m_i = (2/N) sum_j z_j cos(pi * (5^j i mod 2N) / N), exact enough in float64
    rng = np.random.default_rng(8)
    z = rng.uniform(-1, 1, size=tiny.n // 2)
    scale = 2.0 ** 20
    m, tie = tiny.encode(z, scale)
    N = tiny.n
    want = []
    for i in range(N):
        s = sum(z[j] * math.cos(math.pi * ((pow(5, j, 2 * N) * i) % (2 * N)) / N) for j in range(N // 2))
        want.append(2.0 / N * s * scale)
    assert tie > 1e-6
    assert list(m) == [int(round(w)) for w in want]


def test_encode_rotation_is_automorphism(small):
    """Ecd(R(z, r)) = sigma_{5^r}(Ecd(z)): pins slot j <-> zeta^(5^j) and the left rotation"""
    rng = np.random.default_rng(9)
    z = rng.uniform(-1, 1, size=small.n // 2)
    m, tie = small.encode(z)
    assert tie > 1e-9
    N = small.n
    for r in (1, 3, 17):
        mr, _ = small.encode(np.roll(z, -r))
        g = pow(5, r, 2 * N)
        perm = np.zeros(N, np.int64)
        for i in range(N):
            e = i * g % (2 * N)
            if e < N:
                perm[e] = m[i]
            else:
                perm[e - N] = -m[i]
        assert np.array_equal(mr, perm)


def test_decode_inverts_encode(small):
    rng = np.random.default_rng(10)
    z = rng.uniform(-1, 1, size=small.n // 2)
    m, _ = small.encode(z)
    back = small.decode(m.astype(np.float64), small.scale)
    assert np.abs(back - z).max() < 1e-6


def test_slotwise_product_of_polynomial_product(small):
    """the canonical embedding turns negacyclic products into slot products"""
    rng = np.random.default_rng(11)
    a, b = rng.uniform(-1, 1, size=small.n // 2), rng.uniform(-1, 1, size=small.n // 2)
    ma, _ = small.encode(a, 2.0 ** 20)
    mb, _ = small.encode(b, 2.0 ** 20)
    prod = naive_negacyclic_int([int(x) for x in ma], [int(x) for x in mb])
    back = small.decode(np.array(prod, np.float64), 2.0 ** 40)
    assert np.abs(back - a * b).max() < 1e-4


def naive_negacyclic_int(a, b):
    n = len(a)
    aa, bb = np.array(a, dtype=object), np.array(b, dtype=object)
    out = [0] * n
    for i in range(n):
        if aa[i] == 0:
            continue
        for j in range(n):
            k = i + j
            if k < n:
                out[k] += aa[i] * bb[j]
            else:
                out[k - n] -= aa[i] * bb[j]
    return out


# ---------------------------------------------------------------- encryption and Fig. 1 operations
def test_encrypt_decrypt_roundtrip_noise_bound(small):
    rng = np.random.default_rng(12)
    m = rng.integers(-(2 ** 30), 2 ** 30, size=small.n)
    for level in (small.max_level, 2):
        ct = small.encrypt_coeffs(m, level, small.scale, nonce=3)
        got = small.decrypt_coeffs(ct)
        noise = got - m
        # |v e_pk + e0 + e1 s| <= 19 (N + 1 + N) for ternary v, s
        assert np.abs(noise).max() <= 19 * (2 * small.n + 1)
        assert np.abs(noise).max() > 0


def test_rotation_matches_slot_rotation(small):
    rng = np.random.default_rng(13)
    z = rng.uniform(-1, 1, size=small.n // 2)
    ct = small.encrypt(z, nonce=4)
    for k in (1, 5, -3, 64, small.n // 2 - 1):
        got = small.decrypt(small.rotate(ct, k))
        assert np.abs(got - np.roll(z, -k)).max() < 1e-3


def test_hoisted_rotation_is_bit_identical(small):
    rng = np.random.default_rng(14)
    ct = small.encrypt(rng.uniform(-1, 1, size=64), nonce=5)
    ks = [1, 2, 7, -8, 40]
    for k, r in zip(ks, small.rotate_hoisted(ct, ks)):
        assert np.array_equal(r.export(), small.rotate(ct, k).export())


def test_mul_relin_rescale(small):
    rng = np.random.default_rng(15)
    a, b = rng.uniform(-1, 1, size=small.n // 2), rng.uniform(-1, 1, size=small.n // 2)
    ca, cb = small.encrypt(a, nonce=6), small.encrypt(b, nonce=7)
    t = small.tensor(ca, cb)
    assert t.degree == 2
    assert np.abs(small.decrypt(t) - a * b).max() < 1e-3  # degree-2 decryption with s^2
    r = small.rescale(small.relin(t))
    assert r.level == ca.level - 1
    assert abs(r.scale - ca.scale * cb.scale / small.q[ca.level]) < 1e-6 * r.scale
    assert np.abs(small.decrypt(r) - a * b).max() < 1e-3


def test_add_level_min_scale_max(small):
    z = np.linspace(-1, 1, 32)
    a = small.encrypt(z, nonce=8)
    b = small.drop(small.encrypt(z, nonce=9), 2)
    s = small.add(a, b)
    assert s.level == 2 and s.scale == max(a.scale, b.scale)
    assert np.abs(small.decrypt(s, 32) - 2 * z).max() < 1e-3


# ---------------------------------------------------------------- Sec. 3: masks and permutations
def perm_from_rows(rows, vec):
    return np.array([vec[c] for c in rows])


def test_fig2_masks_and_permutations():
    g = gold("fig2_3x3.json")
    h = g["h"]
    for k, v in g["u_mu"].items():
        assert list(O.mask_slots(0, h, int(k))) == v
    for k, v in g["u_zeta"].items():
        assert list(O.mask_slots(1, h, int(k) // h)) == v
    for k, v in g["v"].items():
        k = int(k)
        kind, kk = (2, k) if k > 0 else (3, k + h)
        assert list(O.mask_slots(kind, h, kk)) == v
    a = np.arange(9)
    # Eq. 1: U a = sum_k u_k . R(a, k) with R(m,k)[t] = m[t+k]
    ua = sum(O.mask_slots(0, h, k) * np.roll(a, -k) for k in range(-h + 1, h))
    assert list(ua.astype(int)) == g["U_mu_a"] == g["perm_rows"]["U_mu"]
    zb = sum(O.mask_slots(1, h, k) * np.roll(a, -h * k) for k in range(h))
    assert list(zb.astype(int)) == g["U_zeta_b"] == g["perm_rows"]["U_zeta"]
    mu = np.array(g["U_mu_a"])
    zt = np.array(g["U_zeta_b"])
    for k in (1, 2):
        vk = O.mask_slots(2, h, k) * np.roll(mu, -k) + O.mask_slots(3, h, k) * np.roll(mu, -(k - h))
        assert vk.astype(int).reshape(h, h).tolist() == g[f"phi{k}_mu_A"]
        assert list(vk.astype(int)) == list(perm_from_rows(g["perm_rows"][f"V{k}"], mu))
        pk = np.roll(zt, -h * k)
        assert pk.reshape(h, h).tolist() == g[f"pi{k}_zeta_B"]
        assert list(pk) == list(perm_from_rows(g["perm_rows"][f"P{k}"], zt))


@pytest.mark.parametrize("h", [2, 4, 8, 16])
def test_eq2_with_oracle_masks(h):
    """masks reproduce mu, zeta, phi^k, pi^k (Sec. 3.3 definitions) and Eq. 2 gives A B"""
    rng = np.random.default_rng(h)
    A, B = rng.uniform(-1, 1, (h, h)), rng.uniform(-1, 1, (h, h))
    a, b = A.ravel(), B.ravel()
    mu_def = np.array([[A[i, (i + j) % h] for j in range(h)] for i in range(h)])
    zeta_def = np.array([[B[(i + j) % h, j] for j in range(h)] for i in range(h)])
    mu = sum(O.mask_slots(0, h, k) * np.roll(a, -k) for k in range(-h + 1, h))
    zt = sum(O.mask_slots(1, h, k) * np.roll(b, -h * k) for k in range(h))
    assert np.array_equal(mu, mu_def.ravel()) and np.array_equal(zt, zeta_def.ravel())
    total = mu * zt
    for k in range(1, h):
        phi = O.mask_slots(2, h, k) * np.roll(mu, -k) + O.mask_slots(3, h, k) * np.roll(mu, -(k - h))
        pi = np.roll(zt, -h * k)
        phi_def = np.array([[mu_def[i, (j + k) % h] for j in range(h)] for i in range(h)])
        pi_def = np.array([[zeta_def[(i + k) % h, j] for j in range(h)] for i in range(h)])
        assert np.array_equal(phi, phi_def.ravel()) and np.array_equal(pi, pi_def.ravel())
        total = total + phi * pi
    assert np.abs(total.reshape(h, h) - A @ B).max() < 1e-12
    assert np.array_equal(O.mask_slots(2, h, 0), np.ones(h * h))


# ---------------------------------------------------------------- Alg. 3 end to end
def expected_rotations(h):
    b = 1 << ((int(math.log2(h)) + 1) // 2)
    giant1 = len([i for i in range(-((h - 1 + b - 1) // b), (h + b - 1) // b) if i != 0])
    giant2 = len([i for i in range(1, (h + b - 1) // b)])
    return (b - 1) + giant1 + (b - 1) + giant2 + 3 * (h - 1)


def test_rotation_count_h64_vs_table1():
    g = gold("gd_coefficients.json")
    h = 64
    # Table I: 3h + 5 sqrt(h) = 232 rotations; the corrected BSGS index range uses 225
    assert 3 * h + 5 * int(math.isqrt(h)) == g["rotations_h64"]
    assert expected_rotations(64) == 225 <= g["rotations_h64"]


@pytest.mark.parametrize("h,keys", [(8, 22), (16, 46), (32, 94), (64, 190)])
def test_distinct_rotation_keys(h, keys):
    c = O.Ctx(14, [40, 40], [50], 1, 30.0, 1)
    assert len(c.matmul_rotations(h)) == keys


@pytest.mark.parametrize("h", [4, 8, 16])
def test_matmul_decrypts_to_product_and_counts(small, h):
    A, B = I.matrix_pair(100 + h, h)
    ca, cb = small.encrypt(A.ravel(), nonce=20), small.encrypt(B.ravel(), nonce=21)
    small.reset_counters()
    cm = small.matmul(ca, cb, h)
    cnt = small.counters()
    assert cm.level == ca.level - 3
    got = small.decrypt(cm, h * h).reshape(h, h)
    assert np.abs(got - A @ B).max() < 1e-3
    # replicas in the other slots hold the same product (tiled layout)
    full = small.decrypt(cm)
    for r in range(small.n // 2 // (h * h)):
        assert np.abs(full[r * h * h:(r + 1) * h * h].reshape(h, h) - A @ B).max() < 1e-3
    assert cnt["rot"] == expected_rotations(h)
    assert cnt["mul_ct"] == h
    assert cnt["mul_pt"] == (2 * h - 1) + h + (2 * (h - 1) + 1)
    assert cnt["keyswitch"] == expected_rotations(h) + h
    assert cnt["rescale"] == 2 + h + 1  # Step 1-1, Step 1-2, each A^(k), the final sum


def test_c1_as_stated_one_multiply():
    """C1 as stated (40 + 30-bit chain, 40-bit P, scale 2^30): one Mul_ct + RS decrypts to the
    slot-wise product of two h = 8 matrices within 1e-3, and rotations by 1 and h rotate the
    slots; the packed product (depth 3) is refused on this one-level chain"""
    c = O.Ctx.from_params(I.C1)
    A, B = I.matrix_pair(11, 8)
    a, b = c.encrypt(A.ravel(), nonce=1), c.encrypt(B.ravel(), nonce=2)
    m = c.rescale(c.mul(a, b))
    assert m.level == 0
    assert np.abs(c.decrypt(m, 64) - (A * B).ravel()).max() < 1e-3
    v = A.ravel()
    for k in (1, 8):
        assert np.abs(c.decrypt(c.rotate(a, k), 64) - np.roll(v, -k)).max() < 1e-3
    with pytest.raises(ValueError):
        c.matmul(a, b, 8)


def test_matmul_c1plus_bound():
    """the stated accuracy: max abs error <= 1e-3 at scale 2^30 (C1+ ring, h = 8)"""
    c = O.Ctx.from_params(I.C1P)
    A, B = I.matrix_pair(1, 8)
    cm = c.matmul(c.encrypt(A.ravel(), nonce=1), c.encrypt(B.ravel(), nonce=2), 8)
    assert np.abs(c.decrypt(cm, 64).reshape(8, 8) - A @ B).max() < 1e-3


def test_matmul_relin_once(small):
    h = 8
    A, B = I.matrix_pair(7, h)
    ca, cb = small.encrypt(A.ravel(), nonce=30), small.encrypt(B.ravel(), nonce=31)
    small.reset_counters()
    once = small.matmul(ca, cb, h, O.RELIN_ONCE)
    assert small.counters()["keyswitch"] == expected_rotations(h) + 1
    each = small.matmul(ca, cb, h, O.RELIN_EACH)
    assert np.abs(small.decrypt(once, 64).reshape(h, h) - A @ B).max() < 1e-3
    assert not np.array_equal(once.export(), each.export())


MODES = [O.RELIN_EACH, O.RELIN_ONCE, O.HOIST_MODDOWN, O.RESCALE_LATE,
         O.RELIN_ONCE | O.HOIST_MODDOWN, O.RELIN_ONCE | O.HOIST_MODDOWN | O.RESCALE_LATE,
         O.STEP3_BSGS, O.STEP3_BSGS | O.RELIN_ONCE, O.FAST]


def step3_counts(h, mode):
    """(rotations, relinearisations) of Steps 2-3: 2(h-1) rotations of A0; with the Step-3
    split (bg baby steps, bg = 2^ceil((log2 h + 1)/2) capped at h) bg - 1 rotations of B0 and
    h/bg - 1 giant-step rotations, else h - 1 rotations of B0; one relinearisation per
    product, or per block sum under relin-once"""
    bg = min(h, 2 ** ((int(math.log2(h)) + 2) // 2)) if mode & O.STEP3_BSGS else h
    rots = 2 * (h - 1) + (bg - 1) + (h // bg - 1)
    relins = h // bg if mode & O.RELIN_ONCE else h
    return rots, relins


def step1_rotations(h):
    b = 2 ** ((int(math.log2(h)) + 1) // 2)
    giant11 = len([i for i in range((1 - h) // b, (h - 1) // b + 1) if i != 0])
    return (b - 1) + giant11 + (b - 1) + (len(range(0, h, b)) - 1)


def test_step3_count_helpers_match_default_formula():
    for h in (4, 8, 16, 32, 64):
        assert step1_rotations(h) + step3_counts(h, 0)[0] == expected_rotations(h)


@pytest.mark.parametrize("mode", MODES)
def test_matmul_schedules_decrypt_and_counts(small, mode):
    """every schedule computes A B at the same depth; the op counts follow from what
    each flag moves (one relinearisation per block instead of per product, ModDown shared
    by a mask pair, two rescales at the end instead of one per A^(k), fewer B0 rotations)"""
    for h in (8, 16):
        A, B = I.matrix_pair(40 + mode, h)
        ca, cb = small.encrypt(A.ravel(), nonce=50), small.encrypt(B.ravel(), nonce=51)
        small.reset_counters()
        cm = small.matmul(ca, cb, h, mode)
        cnt = small.counters()
        assert cm.level == ca.level - 3
        assert abs(cm.scale / ca.scale - 1) < 1e-3
        full = small.decrypt(cm)
        for r in range(small.n // 2 // (h * h)):
            assert np.abs(full[r * h * h:(r + 1) * h * h].reshape(h, h) - A @ B).max() < 1e-3
        rots, relins = step3_counts(h, mode)
        assert cnt["rot"] == step1_rotations(h) + rots
        assert cnt["keyswitch"] == step1_rotations(h) + rots + relins
        assert cnt["mul_pt"] == (2 * h - 1) + h + (2 * (h - 1) + 1)
        assert cnt["mul_ct"] == h
        assert cnt["rescale"] == 2 + (2 if mode & O.RESCALE_LATE else h + 1)
        # every rotation the product performs has a key in the schedule's rotation list
        assert len(small.matmul_rotations(h, mode)) <= cnt["rot"]


@pytest.mark.parametrize("h,keys", [(16, 44), (32, 79), (64, 160)])
def test_step3_bsgs_rotation_keys(h, keys):
    """distinct rotation amounts under the Step-3 split (A-side amounts k - s, k - h - s with
    the giant shift s, B0 baby steps h j, giant steps h bg i, and Step 1's)"""
    c = O.Ctx(14, [40, 40], [50], 1, 30.0, 1)
    got = c.matmul_rotations(h, O.STEP3_BSGS)
    assert len(got) == keys
    b = 2 ** ((int(math.log2(h)) + 1) // 2)
    bg = min(h, 2 ** ((int(math.log2(h)) + 2) // 2))
    half = c.n // 2
    want = set()
    for j in range(1, b):
        want |= {j, h * j}
    for i in range((1 - h) // b, (h - 1) // b + 1):
        if i:
            want.add((b * i) % half)
    for i in range(1, (h + b - 1) // b):
        want.add(h * b * i)
    for k in range(1, h):
        s = h * bg * (k // bg)
        want |= {(k - s) % half, (k - h - s) % half}
    for j in range(1, bg):
        want.add(h * j)
    for i in range(1, h // bg):
        want.add(h * bg * i)
    want.discard(0)
    assert sorted(want) == got


def test_matmul_schedules_agree_at_coefficient_level(small):
    """the schedules differ only in where rounding happens: at h = 8 on a 2^10 ring the
    decrypted coefficient vectors of every flag combination differ from Alg. 3 as printed by
    no more than the rounding noise the schedule noise model gives (7 standard deviations of
    V_X + V_0; mean square within the 15 % sampling spread of 1024 coefficients), and each
    schedule is a different bit pattern"""
    h = 8
    prm = I.small(log_n=10, n_q=5, alpha=2)
    M = _noise_model(small, prm)
    frac = CN.mask_fractions(O.mask_slots, h)
    A, B = I.matrix_pair(77, h)
    ca, cb = small.encrypt(A.ravel(), nonce=60), small.encrypt(B.ravel(), nonce=61)
    outs = {m: small.matmul(ca, cb, h, m) for m in MODES}
    ref = small.decrypt_coeffs(outs[O.RELIN_EACH])
    mu = float(np.mean(A ** 2)), float(np.mean(B ** 2))
    V0 = M.matmul(h, 0, ca.level, *mu, frac)
    for m, ct in outs.items():
        VX = M.matmul(h, m, ca.level, *mu, frac)
        assert abs(VX.s / ct.scale - 1) < 1e-12, m
        d = small.decrypt_coeffs(ct) - ref
        sd = math.sqrt(VX.v + V0.v)
        assert float(np.sqrt(np.mean(d ** 2))) <= 1.15 * sd, (m, sd)
        assert float(np.abs(d).max()) <= 7 * sd, (m, sd)
    assert len({ct.export().tobytes() for ct in outs.values()}) == len(MODES)


# ---------------------------------------------------------------- schedules vs Alg. 3 as printed
def _automorph_coeffs(m, g):
    """sigma_g on the coefficient vector of an element of Z[X]/(X^N + 1): X^i -> X^(i g)"""
    n = m.size
    idx = (np.arange(n) * g) % (2 * n)
    out = np.zeros_like(m)
    out[idx % n] = np.where(idx >= n, -1.0, 1.0) * m
    return out


def _noise_model(c, prm):
    hs = int(np.count_nonzero(O.sample_ternary(prm.seed, 1, 0, c.n)))  # the secret, purpose 1
    return CN.ScheduleNoise(c.n, c.q, c.p, prm.alpha, 2.0 ** prm.log_scale, hs)


@pytest.mark.parametrize("p_bits,alpha", [([50, 50], 2), ([60], 2)])
def test_noise_model_rounding_terms(p_bits, alpha):
    """the rounding terms of the schedule noise model, measured one by one: the decrypted
    coefficients after a rescale, a rotation and a relinearisation differ from the exact
    result (the decryption divided by q, the automorphism of the decryption, the degree-2
    decryption) by centred noise of the modelled variance, within 15 %: over N = 4096
    coefficients the mean square of the rounding terms has a spread of about 2 %, and a
    key-switching term, weighted by the spectrum of one key's error polynomial, about 4 %.  With P = 2 x 50 bits the ModDown rounding dominates the key switch; with one
    60-bit P below the 90-bit digits the key-switching term dominates."""
    prm = I.Params("noise", 12, [50, 40, 40, 40, 40], p_bits, alpha, 40.0, 17, [])
    c = O.Ctx.from_params(prm)
    M = _noise_model(c, prm)
    rng = np.random.default_rng(5)
    ct = c.encrypt(rng.uniform(-1, 1, 2048), nonce=1)
    ct2 = c.encrypt(rng.uniform(-1, 1, 2048), nonce=2)
    base = c.decrypt_coeffs(ct)

    def ratio(d, v):
        return float(np.mean(d ** 2)) / v

    r = ratio(c.decrypt_coeffs(c.rescale(ct)) - base / c.q[ct.level], M.v_rs)
    assert abs(r - 1) < 0.15, r
    for k in (3, 100):
        g = pow(5, k, 2 * c.n)
        d = c.decrypt_coeffs(c.rotate(ct, k)) - _automorph_coeffs(base, g)
        r = ratio(d, M.v_ks(ct.level) + M.v_md)
        assert abs(r - 1) < 0.15, (k, r)
    # the degree-2 ciphertext at a small scale, so that its decryption is exact in float64
    t = c.tensor(c.rescale(ct), c.rescale(ct2))
    d = c.decrypt_coeffs(c.relin(t)) - c.decrypt_coeffs(t)
    r = ratio(d, M.v_ks(t.level) + M.v_md)
    assert abs(r - 1) < 0.15, r


def test_fused_schedules_tied_to_alg3_as_printed_h64():
    """each fused schedule (relin-once 1, ModDown hoisting 2, late rescale 4, Step-3 split 8,
    all four 15) against Alg. 3 as printed (0) for an h = 64 product on a 2^13 ring (one
    replica: every rotation spans the whole slot vector): the decrypted coefficients differ by
    the rounding terms the flags move and by nothing else.  The noise model follows each
    schedule's operations (its output scale equals the oracle's to double rounding) and gives
    the variance V of each schedule's rounding noise; the difference of two schedules has
    variance at most V_X + V_0, so its mean square must not exceed that by more than the
    sampling spread (10 % over 8192 coefficients) and no coefficient may exceed 7 standard
    deviations (probability below 10^-8 for 8192 Gaussian coefficients)."""
    prm = I.small(log_n=13, n_q=5, alpha=2, q_bits=40, p_bits=50, h_list=())
    c = O.Ctx.from_params(prm)
    M = _noise_model(c, prm)
    h = 64
    A, B = I.matrix_pair(64, h)
    ca, cb = c.encrypt(A.ravel(), nonce=1), c.encrypt(B.ravel(), nonce=2)
    frac = CN.mask_fractions(O.mask_slots, h)
    ref_ct = c.matmul(ca, cb, h, 0)
    ref = c.decrypt_coeffs(ref_ct)
    V0 = M.matmul(h, 0, ca.level, float(np.mean(A ** 2)), float(np.mean(B ** 2)), frac)
    assert V0.lvl == ref_ct.level and abs(V0.s / ref_ct.scale - 1) < 1e-12
    for mode in (1, 2, 4, 8, 15):
        ct = c.matmul(ca, cb, h, mode)
        VX = M.matmul(h, mode, ca.level, float(np.mean(A ** 2)), float(np.mean(B ** 2)), frac)
        assert VX.lvl == ct.level and abs(VX.s / ct.scale - 1) < 1e-12, mode
        d = c.decrypt_coeffs(ct) - ref
        sd = math.sqrt(VX.v + V0.v)
        assert np.any(d != 0), mode  # a distinct rounding pattern, not the same computation
        assert float(np.sqrt(np.mean(d ** 2))) <= 1.1 * sd, (mode, np.sqrt(np.mean(d ** 2)), sd)
        assert float(np.abs(d).max()) <= 7 * sd, (mode, np.abs(d).max(), sd)
        # far below the output scale: the schedules agree to about 2^-30 relative
        assert 7 * sd < ct.scale * 2.0 ** -27


def test_matmul_fast_schedule_c1plus_bound():
    """the stated accuracy (1e-3 at scale 2^30, C1+ ring, h = 8) also holds for the
    schedule with all three flags"""
    c = O.Ctx.from_params(I.C1P)
    A, B = I.matrix_pair(2, 8)
    cm = c.matmul(c.encrypt(A.ravel(), nonce=1), c.encrypt(B.ravel(), nonce=2), 8, O.FAST)
    assert np.abs(c.decrypt(cm, 64).reshape(8, 8) - A @ B).max() < 1e-3


def test_matmul_rejects_bad_shapes(small):
    ct = small.encrypt(np.zeros(4), nonce=1)
    with pytest.raises(ValueError):
        small.matmul(ct, ct, 6)             # not a power of two
    with pytest.raises(ValueError):
        small.matmul(ct, ct, 32)            # h^2 > N/2
    with pytest.raises(ValueError):
        small.matmul(small.drop(ct, 2), ct, 4)  # level below depth 3


# ---------------------------------------------------------------- Sec. 4: g_d
def gd_from_definition(d):
    m = sympy.symbols("m")
    g = sum(Fraction(math.comb(2 * i, i), 4 ** i) * m * (1 - m ** 2) ** i for i in range(d + 1))
    return sympy.Poly(sympy.expand(g), m), m


@pytest.mark.parametrize("d", [1, 2, 3, 4])
def test_gd_printed_coefficients_and_properties(d):
    g = gold("gd_coefficients.json")["g"][str(d)]
    poly, m = gd_from_definition(d)
    coeffs = {int(k): sympy.Rational(v[0], v[1]) for k, v in g.items()}
    got = {mon[0]: c for mon, c in zip(poly.monoms(), poly.coeffs())}
    assert got == coeffs
    # each coefficient is n / 2^(2d-1) with n an integer (Sec. 4.2)
    assert all((c * 2 ** (2 * d - 1)).q == 1 for c in coeffs.values())
    expr = poly.as_expr()
    assert expr.subs(m, 1) == 1 and expr.subs(m, -1) == -1                    # Prop. II
    assert sympy.expand(expr.subs(m, -m) + expr) == 0                         # Prop. I
    p_d = sympy.Rational(2 * d + 1, 4 ** d) * math.comb(2 * d, d)             # Lemma 4.1
    assert coeffs[1] == p_d == sum(sympy.Rational(math.comb(2 * i, i), 4 ** i) for i in range(d + 1))
    assert sympy.expand(sympy.diff(expr, m) - p_d * (1 - m ** 2) ** d) == 0   # Prop. III


@pytest.mark.parametrize("d", [1, 2, 3, 4])
def test_lemmas_4_2_4_3(d):
    poly, m = gd_from_definition(d)
    f = sympy.lambdify(m, poly.as_expr(), "numpy")
    p_d = (2 * d + 1) / 4 ** d * math.comb(2 * d, d)
    x = np.linspace(0, 1, 20001)
    one_minus = 1 - f(x)
    assert np.all(one_minus >= -1e-15)
    assert np.all(one_minus <= (1 - x) ** p_d + 1e-12)
    assert np.all(one_minus <= 2 ** d * (1 - x) ** (d + 1) + 1e-12)


def min_k(d, sigma, delta):
    poly, m = gd_from_definition(d)
    f = sympy.lambdify(m, poly.as_expr(), "numpy")
    x = np.concatenate([np.geomspace(delta, 1, 200001)])
    for k in range(1, 60):
        x = f(x)
        if np.max(1 - x) <= 2.0 ** -sigma:
            return k
    return None


def test_theorem_3_5_k_table():
    """the minimal k with g_d^(k) (sigma, delta)-close, against the theorem's leading terms"""
    k = min_k(4, 20, 2.0 ** -20)
    p4 = 315 / 128
    lead = math.log2(2 ** 20) / math.log2(p4) + math.log2(19) / math.log2(5)
    assert k == 17 and abs(k - lead) < 2
    assert min_k(3, 8, 2.0 ** -8) == 9


def gd_eval(d, x):
    g = gold("gd_coefficients.json")["g"][str(d)]
    return sum(v[0] / v[1] * x ** int(p) for p, v in g.items())


@pytest.mark.parametrize("d,k", [(1, 1), (2, 1), (3, 1), (1, 2)])
def test_sign_decrypts_to_composite_polynomial(d, k):
    c = O.Ctx.from_params(I.small(log_n=10, n_q=8, alpha=2, q_bits=40, log_scale=40.0))
    X = I.sign_inputs(5, 1, 16)[0].ravel()
    x = c.encrypt(X, nonce=40)
    y = c.sign(x, d, k)
    want = X.copy()
    for _ in range(k):
        want = gd_eval(d, want)
    nb = int(math.floor(math.log2(d))) + 1
    assert y.level == x.level - k * (nb + 1)
    assert np.abs(c.decrypt(y, 256) - want).max() < 1e-3
    # scale matching: every term of the sum lands on the input's scale, so the
    # compositions do not drift (output scale = input scale to double rounding) and the
    # error stays at the encryption/rescale noise level (2^-40 here) times the Lipschitz
    # growth of g_d^(k), far below the stated bound
    assert abs(y.scale / x.scale - 1) < 1e-12
    assert np.abs(c.decrypt(y, 256) - want).max() < 1e-6


@pytest.mark.parametrize("d", [1, 2, 3, 4])
def test_gd_numerators_are_printed_coefficients(d):
    """the integer numerators the oracle evaluates g_d with, over 2^(2d-1), are the printed
    coefficients of Sec. 4.2 (g_4: 315, -420, 378, -180, 35 over 128)"""
    g = gold("gd_coefficients.json")["g"][str(d)]
    num = O.gd_numerators(d)
    den = 2 ** (2 * d - 1)
    assert len(num) == d + 1
    for i, n in enumerate(num):
        p, q = g[str(2 * i + 1)]
        assert Fraction(n, den) == Fraction(p, q), (d, i)


@pytest.mark.parametrize("k,mode", [(1, "sign"), (2, "sign"), (1, "relu"), (1, "appmax")])
def test_g4_decrypts_to_printed_polynomial(k, mode):
    """g_4, the polynomial of the paper's experiments (Sec. 4.2; Sec. 6.1 uses d = 4): sign at
    k = 1 and 2, ReLU and AppMax (Alg. 5) at k = 1, against the FP64 composition of the printed
    coefficients (not the oracle's numerators); depth 1 + floor(log2 4) + 1 = 4 per composition
    (powers x^2, x^4, x^8 for the x^9 term), plus one level for ReLU and AppMax"""
    c = O.Ctx.from_params(I.small(log_n=10, n_q=10, alpha=2, q_bits=40, log_scale=40.0))
    X = I.sign_inputs(45, 1, 16)[0].ravel()
    x = c.encrypt(X, nonce=46)
    want = X.copy()
    for _ in range(k):
        want = gd_eval(4, want)
    if mode == "sign":
        y = c.sign(x, 4, k)
        assert y.level == x.level - 4 * k
        assert abs(y.scale / x.scale - 1) < 1e-12
    elif mode == "relu":
        y = c.sign(x, 4, k, relu=True)
        want = (X + X * want) / 2
        assert y.level == x.level - 4 * k - 1
    else:
        rng = np.random.default_rng(47)
        a, b = rng.uniform(-0.5, 0.5, 256), rng.uniform(-0.5, 0.5, 256)
        y = c.appmax(c.encrypt(a, nonce=48), c.encrypt(b, nonce=49), 4, k)
        X, want = a, appmax_fp64(a, b, 4, k)
        assert y.level == x.level - 4 * k - 1
    got = c.decrypt(y, X.size)
    assert np.abs(got - want).max() < 1e-6
    # Lemma 4.2 (1 - g_d(x) <= (1 - x)^(p_d) on [0, 1], p_4 = 315/128), applied k times:
    # |x| >= 1/4 ends within 0.75^(p_4^k) of sgn(x)
    if mode == "sign":
        far = np.abs(X) >= 0.25
        assert np.abs(np.abs(got[far]) - 1).max() < 0.75 ** ((315 / 128) ** k) + 1e-6


def test_relu_decrypts(small):
    c = O.Ctx.from_params(I.small(log_n=10, n_q=6, alpha=2, q_bits=40, log_scale=40.0))
    X = I.sign_inputs(6, 1, 16)[0].ravel()
    y = c.sign(c.encrypt(X, nonce=41), 3, 1, relu=True)
    g = gd_eval(3, X)
    assert np.abs(c.decrypt(y, 256) - (X + X * g) / 2).max() < 1e-3
    # the last composition lands on the prime the product x g rescales by, so x + x g adds
    # equal scales and the ReLU output carries exactly twice the input's scale
    assert abs(y.scale / (2 * c.encrypt(X, nonce=41).scale) - 1) < 1e-12
    assert np.abs(c.decrypt(y, 256) - (X + X * g) / 2).max() < 1e-6


def test_sign_rejects_shallow_level(small):
    x = small.drop(small.encrypt(np.zeros(4), nonce=1), 2)
    with pytest.raises(ValueError):
        small.sign(x, 3, 1)


# ---------------------------------------------------------------- App. C, D, E
@pytest.mark.parametrize("h", [2, 3, 4, 8, 16])
def test_transpose_diagonals_from_definition(h):
    """kind-4 masks t_{(h-1)k}: sum_k t_{(h-1)k} . R(a, (h-1)k) is the transpose of the
    row-major matrix a (plaintext, numpy); for k >= 0 they match App. C's printed formula
    t - k = (h+1) j, 0 <= j < h - k; for k < 0 the printed t + k = (h+1) j does not (h > 2),
    the reading t + h k = (h+1) j, 0 <= j < h + k does"""
    n = h * h
    a = np.random.default_rng(h).standard_normal(n)
    out = np.zeros(n)
    for k in range(1 - h, h):
        m = O.mask_slots(4, h, k) if (h & (h - 1)) == 0 else None
        if m is None:  # the oracle's masks are for powers of two; rebuild the definition
            m = np.array([1.0 if (t % h) - (t // h) == k else 0.0 for t in range(n)])
        out += m * np.roll(a, -(h - 1) * k)
        printed = np.array([1.0 if any(t - k == (h + 1) * j for j in range(0, h - k)) else 0.0 for t in range(n)]) \
            if k >= 0 else np.array([1.0 if any(t + k == (h + 1) * j for j in range(0, h + k)) else 0.0
                                     for t in range(n)])
        reading = np.array([1.0 if any(t + h * k == (h + 1) * j for j in range(0, h + k)) else 0.0
                            for t in range(n)])
        if k >= 0:
            assert np.array_equal(m, printed)
        else:
            assert np.array_equal(m, reading)
            if h > 2:
                assert not np.array_equal(m, printed)
    assert np.allclose(out, a.reshape(h, h).T.ravel())


def pack_beta(mats):
    """iota_beta^-1 (App. E): matrix m's entry (i, j) at position beta (h i + j) + m"""
    beta, h = len(mats), mats[0].shape[0]
    v = np.zeros(beta * h * h)
    for m, M in enumerate(mats):
        v[m::beta] = M.ravel()
    return v


def test_packing_rotation_is_matrixwise():
    """App. E: a rotation of the packed vector by beta r rotates every matrix by r"""
    h, beta = 4, 4
    mats = [np.random.default_rng(m).standard_normal((h, h)) for m in range(beta)]
    v = pack_beta(mats)
    for r in (1, 3, h, 5):
        w = np.roll(v, -beta * r)
        for m in range(beta):
            assert np.array_equal(w[m::beta], np.roll(mats[m].ravel(), -r))


@pytest.mark.parametrize("h,beta", [(4, 1), (8, 1), (16, 1), (4, 2), (8, 4)])
def test_transpose_decrypts(small, h, beta):
    mats = [np.random.default_rng(10 * h + m).uniform(-1, 1, (h, h)) for m in range(beta)]
    ct = small.encrypt(pack_beta(mats), nonce=70)
    small.reset_counters()
    tt = small.transpose(ct, h, beta)
    cnt = small.counters()
    assert tt.level == ct.level - 1
    got = small.decrypt(tt, beta * h * h)
    for m in range(beta):
        assert np.abs(got[m::beta].reshape(h, h) - mats[m].T).max() < 1e-6
    b = 2 ** ((int(math.log2(h)) + 1) // 2)
    giants = len([i for i in range((1 - h) // b, (h - 1) // b + 1) if i != 0])
    assert cnt["rot"] == (b - 1) + giants
    assert cnt["mul_pt"] == 2 * h - 1
    assert len(small.transpose_rotations(h, beta)) == (b - 1) + giants


@pytest.mark.parametrize("h,t", [(8, 1), (8, 2), (8, 4), (16, 4), (16, 8)])
def test_rectangular_product_decrypts(small, h, t):
    """Alg. 6: A~ = h/t vertical copies of the t x h matrix A; the result holds h/t copies of
    the t x h product A B; t - 1 rounds of Steps 2-3 and log2(h/t) fold rotations"""
    rng = np.random.default_rng(h + t)
    A = rng.uniform(-1, 1, (t, h))
    B = rng.uniform(-1, 1, (h, h))
    ca = small.encrypt(np.tile(A, (h // t, 1)).ravel(), nonce=80)
    cb = small.encrypt(B.ravel(), nonce=81)
    small.reset_counters()
    cm = small.matmul_ex(ca, cb, h, t)
    cnt = small.counters()
    assert cm.level == ca.level - 3
    got = small.decrypt(cm, h * h).reshape(h, h)
    for blk in range(h // t):
        assert np.abs(got[blk * t:(blk + 1) * t] - A @ B).max() < 1e-3
    b = 2 ** ((int(math.log2(h)) + 1) // 2)
    step1 = step1_rotations(h)
    fold = int(math.log2(h // t))
    assert cnt["rot"] == step1 + 3 * (t - 1) + fold
    assert cnt["mul_ct"] == t
    assert cnt["mul_pt"] == (2 * h - 1) + h + (2 * (t - 1) + 1)


@pytest.mark.parametrize("h,beta,mode", [(4, 4, O.RELIN_EACH), (8, 2, O.FAST), (8, 4, O.RELIN_ONCE)])
def test_packed_products_decrypt(small, h, beta, mode):
    """beta products in one ciphertext pair (App. E), same op counts as one product"""
    rng = np.random.default_rng(h * beta)
    As = [rng.uniform(-1, 1, (h, h)) for _ in range(beta)]
    Bs = [rng.uniform(-1, 1, (h, h)) for _ in range(beta)]
    ca, cb = small.encrypt(pack_beta(As), nonce=90), small.encrypt(pack_beta(Bs), nonce=91)
    small.reset_counters()
    cm = small.matmul_ex(ca, cb, h, h, beta, mode)
    cnt = small.counters()
    got = small.decrypt(cm, beta * h * h)
    for m in range(beta):
        assert np.abs(got[m::beta].reshape(h, h) - As[m] @ Bs[m]).max() < 1e-3
    rots, relins = step3_counts(h, mode)
    assert cnt["rot"] == step1_rotations(h) + rots


@pytest.mark.parametrize("h,t,beta,mode", [(16, 16, 2, 0), (16, 4, 1, O.FAST), (8, 2, 4, O.STEP3_BSGS)])
def test_shaped_rotation_keys(h, t, beta, mode):
    """the rotation amounts of a shaped product, built independently: Step 1-1 (unit 1),
    Step 1-2 (unit h), Steps 2-3 over t rounds (A-side k - s and k - h - s, B0 baby h j and
    giant h bg i), the fold t h 2^s; all times beta, mod N/2"""
    c = O.Ctx(14, [40, 40], [50], 1, 30.0, 1)
    half = c.n // 2
    b = 2 ** ((int(math.log2(h)) + 1) // 2)
    bg = min(t, 2 ** ((int(math.log2(t)) + 2) // 2)) if mode & O.STEP3_BSGS else t
    want = set()
    for j in range(1, b):
        want |= {j, h * j}
    for i in range((1 - h) // b, (h - 1) // b + 1):
        if i:
            want.add(b * i)
    for i in range(1, (h + b - 1) // b):
        want.add(h * b * i)
    for k in range(1, t):
        s = h * bg * (k // bg)
        want |= {k - s, k - h - s}
    for j in range(1, bg):
        want.add(h * j)
    for i in range(1, t // bg):
        want.add(h * bg * i)
    s = 0
    while (t << s) < h:
        want.add((t * h) << s)
        s += 1
    want = {(beta * x) % half for x in want} - {0}
    assert sorted(want) == c.matmul_rotations_ex(h, t, beta, mode)


# ---------------------------------------------------------------- Alg. 5 AppMax, pooling; Alg. 6
def appmax_fp64(a, b, d, k):
    m = a - b
    g = m.copy()
    for _ in range(k):
        g = gd_eval(d, g)
    return ((a + b) + m * g) / 2


def test_appmax_decrypts_and_approaches_max():
    """Alg. 5 against its FP64 evaluation (tight), against max(a, b) where |a - b| >= 1/4 (the
    composite sign has converged there for d = 3, k = 3), and ReLU as the case b = 0"""
    c = O.Ctx.from_params(I.small(log_n=10, n_q=12, alpha=3, q_bits=40, log_scale=40.0))
    rng = np.random.default_rng(21)
    a, b = rng.uniform(-0.5, 0.5, 256), rng.uniform(-0.5, 0.5, 256)
    ca, cb = c.encrypt(a, nonce=1), c.encrypt(b, nonce=2)
    y = c.appmax(ca, cb, 3, 3)
    got = c.decrypt(y, 256)
    assert np.abs(got - appmax_fp64(a, b, 3, 3)).max() < 1e-6
    far = np.abs(a - b) >= 0.25
    assert np.abs(got[far] - np.maximum(a, b)[far]).max() < 2e-3
    assert y.level == ca.level - (3 * 3 + 1)
    assert abs(y.scale / (2 * ca.scale) - 1) < 1e-12
    z = c.appmax(ca, c.encrypt(np.zeros(256), nonce=3), 3, 2)
    r = c.sign(ca, 3, 2, relu=True)
    assert np.abs(c.decrypt(z, 256) - c.decrypt(r, 256)).max() < 1e-6


def test_maxpool2_matches_window_formula():
    # alpha = 2: every key-switching digit (<= 90 bits) stays below P (100 bits); rotations
    # with wider digits carry digit / P times more noise
    c = O.Ctx.from_params(I.small(log_n=10, n_q=12, alpha=2, q_bits=40, log_scale=40.0))
    h = 8
    X = np.random.default_rng(22).uniform(-0.5, 0.5, (h, h))
    y = c.maxpool2(c.encrypt(X.ravel(), nonce=4), h, 3, 1)
    v = X.ravel()
    m1 = appmax_fp64(v, np.roll(v, -1), 3, 1)
    m2 = appmax_fp64(m1, np.roll(m1, -h), 3, 1)
    got = c.decrypt(y, h * h)
    assert np.abs(got - m2).max() < 1e-6
    # the stride-2 outputs are window maxima up to the method's error (window spreads >= 1/4)
    W = np.array([[X[i:i + 2, j:j + 2].max() for j in range(0, h, 2)] for i in range(0, h, 2)])
    G = got.reshape(h, h)[::2, ::2]
    assert np.abs(G - W).max() < 0.2


def test_fl_update_decrypts():
    """Alg. 6 aggregation: W - eta / (B N) sum_i G_i, one level"""
    c = O.Ctx.from_params(I.small(log_n=10, n_q=5, alpha=2))
    rng = np.random.default_rng(23)
    n, coeff = 5, 0.05 / (10 * 5)
    W = rng.uniform(-1, 1, 64)
    G = [rng.uniform(-1, 1, 64) for _ in range(n)]
    cw = c.encrypt(W, nonce=1)
    cg = [c.encrypt(g, nonce=10 + i) for i, g in enumerate(G)]
    r = c.fl_update(cw, cg, coeff)
    assert r.level == cw.level - 1
    assert abs(r.scale / cw.scale - 1) < 1e-12  # the product lands on the gradients' scale
    assert np.abs(c.decrypt(r, 64) - (W - coeff * np.sum(G, axis=0))).max() < 1e-7
