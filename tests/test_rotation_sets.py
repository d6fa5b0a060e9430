"""Host-side facts the rotation-set inner product relies on (no GPU needed).

The launch that serves several rotations of one lift numbers its blocks by the source block
they gather. That is valid because sigma_g, acting on the bit-reversed evaluation layout,
maps every aligned block of 256 slots onto one aligned block of 256 slots. The output block of
a set is then sigma_{g^-1} of the source block, with g^-1 mod 2N from Newton's iteration.
"""
import pytest

BLOCK = 256


def brev(x, bits):
    return int(format(x, f"0{bits}b")[::-1], 2)


def perm_g(j, g, log_n):
    """position j of the bit-reversed layout holds a(psi^(2 brev(j) + 1)); sigma_g reads the
    position whose exponent is g times that one (mod 2N)"""
    e = 2 * brev(j, log_n) + 1
    e2 = (e * g) % (2 << log_n)
    return brev((e2 - 1) >> 1, log_n)


def newton_inverse(g, log_n):
    """g^-1 mod 2N as the library computes it: x <- x (2 - g x) mod 2^64, six times from x = g"""
    x = g
    for _ in range(6):
        x = (x * (2 - g * x)) % (1 << 64)
    return x % (2 << log_n)


def galois(k, log_n):
    """5^k mod 2N (rotation by k slots; negative k through the order N/2 of 5)"""
    half = 1 << (log_n - 1)
    return pow(5, k % half, 2 << log_n)


@pytest.mark.parametrize("log_n", [8, 10, 12, 15])
def test_automorphism_maps_aligned_blocks_onto_aligned_blocks(log_n):
    n = 1 << log_n
    for k in (1, 3, 7, 17, 64, 63 - 64, 1000, -1, -(n // 4) + 5):
        g = galois(k, log_n)
        for blk in range(n // BLOCK):
            src = {perm_g(blk * BLOCK + t, g, log_n) // BLOCK for t in range(BLOCK)}
            assert len(src) == 1, (log_n, k, blk, sorted(src)[:4])


@pytest.mark.parametrize("log_n", [8, 12, 15, 17])
def test_newton_inverse_and_output_block(log_n):
    n = 1 << log_n
    for k in (1, 2, 5, 64, -64, -1, 12345):
        g = galois(k, log_n)
        gi = newton_inverse(g, log_n)
        assert (g * gi) % (2 * n) == 1
        # the output block of source block R: every slot of it gathers from R
        for R in range(0, n // BLOCK, max(1, n // BLOCK // 16)):
            xo = perm_g(R * BLOCK, gi, log_n) // BLOCK
            assert all(perm_g(xo * BLOCK + t, g, log_n) // BLOCK == R for t in range(BLOCK))


def test_pairs_of_a_step2_block_gather_the_same_source_block():
    """the two rotations of a Step-2 mask pair (k and k - h, h = 64, N = 2^15) read the same
    source block for every output block: 5^64 = 1 modulo 2^8"""
    log_n, h = 15, 64
    for k in (1, 17, 63):
        g1, g2 = galois(k, log_n), galois(k - h, log_n)
        for blk in range((1 << log_n) // BLOCK):
            i = blk * BLOCK
            assert perm_g(i, g1, log_n) // BLOCK == perm_g(i, g2, log_n) // BLOCK
