"""Average-case rounding-noise model of the packed product, used to bound how far two
schedules of the same product may decrypt apart.

The schedules of HE-MatMult (Alg. 3 with App. B's baby-step/giant-step split) compute the same
exact rational function of the two input ciphertexts: with exact divisions in place of every
rescale and ModDown, and no key-switching noise, they would decrypt to the same polynomial,
input encryption noise included.  They differ only in the rounding terms each one adds and in
where it adds them.  This module follows the operation sequence of one schedule and tracks the
variance per coefficient of the rounding noise accumulated in every ciphertext (absolute
coefficient units at that ciphertext's scale), so that the decrypted coefficients of two
schedules X and Y differ by a centred sum of many independent terms of variance at most
V_X + V_Y.

Rounding terms (s the ternary secret with h_s nonzero coefficients, K special primes, sigma the
error deviation):
  rescale by q:   (r0 + r1 s) / q with r_i the centred residues mod q, each coefficient of
                  r_i / q uniform on (-1/2, 1/2): variance (1 + h_s) / 12;
  ModDown by P:   the centred base conversion of the P part leaves sum_k y_k / p_k per
                  component (y_k centred mod p_k): variance K (1 + h_s) / 12;
  key switching:  (sum_j d~_j e_j) / P over the digits j of the switched polynomial; d~_j is the
                  centred ModUp of the digit, sum_{i in I_j} y_i (D_j / q_i) with y_i centred mod
                  q_i, so each coefficient has variance |I_j| D_j^2 / 12, and the negacyclic
                  product with the Gaussian e_j has variance N sigma^2 |I_j| D_j^2 / 12.
Propagation: a rotation permutes coefficients up to sign (variance kept); a product with a
plaintext m multiplies the variance by ||m||_2^2, which for an encoding at scale S of slot
values z is S^2 mean|z|^2 (Parseval over the N primitive roots); a tensor product of a and b
gives S_b^2 mu_b v_a + S_a^2 mu_a v_b (mu the mean squared slot value); a rescale by q divides
by q^2 and adds its own rounding.  Terms from different rotations, or from one error read at
different slots, are independent, so variances add.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

RELIN_ONCE, HOIST_MODDOWN, RESCALE_LATE, STEP3_BSGS = 1, 2, 4, 8


@dataclass
class Nz:
    v: float      # noise variance per coefficient, at this ciphertext's scale
    s: float      # scale
    lvl: int
    mu: float = 0.0  # mean squared slot value of the message (for tensor products)


def ilog2(h):
    return (h - 1).bit_length()


class ScheduleNoise:
    def __init__(self, n, q, p, alpha, delta, h_s, sigma=3.2):
        self.n, self.q, self.p, self.alpha, self.delta = n, list(q), list(p), alpha, delta
        self.P = float(math.prod(self.p))
        self.v_rs = (1 + h_s) / 12.0
        self.v_md = len(self.p) * (1 + h_s) / 12.0
        self.sigma = sigma

    # rounding terms ---------------------------------------------------------------
    def v_ks(self, lvl):
        tot = 0.0
        for lo in range(0, lvl + 1, self.alpha):
            hi = min(lo + self.alpha, lvl + 1)
            d = float(math.prod(self.q[lo:hi]))
            tot += (hi - lo) * (d / self.P) ** 2
        return self.n * self.sigma ** 2 * tot / 12.0

    # operations --------------------------------------------------------------------
    def rot(self, a):
        return Nz(a.v + self.v_ks(a.lvl) + self.v_md, a.s, a.lvl, a.mu)

    def mulpt(self, a, f):
        return Nz(f * self.delta ** 2 * a.v, a.s * self.delta, a.lvl, a.mu)

    @staticmethod
    def add(a, b):
        if a is None:
            return b
        return Nz(a.v + b.v, max(a.s, b.s), min(a.lvl, b.lvl), max(a.mu, b.mu))

    def rs(self, a):
        q = float(self.q[a.lvl])
        return Nz(a.v / q ** 2 + self.v_rs, a.s / q, a.lvl - 1, a.mu)

    @staticmethod
    def drop(a):
        return Nz(a.v, a.s, a.lvl - 1, a.mu)

    @staticmethod
    def tensor(a, b):
        return Nz(b.s ** 2 * b.mu * a.v + a.s ** 2 * a.mu * b.v, a.s * b.s, min(a.lvl, b.lvl), a.mu * b.mu)

    def relin(self, a):
        return Nz(a.v + self.v_ks(a.lvl) + self.v_md, a.s, a.lvl, a.mu)

    def rot_sum_hoisted(self, terms):
        """sum of rotations sharing one ModDown: each term's key-switch inner product (and its
        ciphertext's noise) times its mask in the extended basis, one ModDown at the end"""
        v, s = 0.0, 0.0
        for a, f in terms:
            w = 1.0 if f is None else f * self.delta ** 2
            v += w * (a.v + self.v_ks(a.lvl))
            s = max(s, a.s * (1.0 if f is None else self.delta))
        return Nz(v + self.v_md, s, terms[0][0].lvl, terms[0][0].mu)

    # the product ---------------------------------------------------------------------
    def lintrans(self, a, fr, dlo, dhi, b, hoist):
        baby = [a] + [self.rot(a) for _ in range(1, b)]
        acc, giants = None, []
        for i in range(dlo // b, dhi // b + 1):
            inner = None
            for j in range(b):
                d = b * i + j
                if dlo <= d <= dhi:
                    inner = self.add(inner, self.mulpt(baby[j], fr(d)))
            if inner is None:
                continue
            if i and hoist:
                giants.append((inner, None))
                continue
            acc = self.add(acc, self.rot(inner) if i else inner)
        if giants:
            acc = self.add(acc, self.rot_sum_hoisted(giants))
        return acc

    def matmul(self, h, mode, lvl, mu_a, mu_b, mask_frac):
        """variance of the rounding noise of the product of two fresh ciphertexts at level lvl
        (scale delta, message mean squares mu_a, mu_b); mask_frac(kind, k) is the fraction of
        ones of a diagonal mask (the mean of its squared 0/1 slot values)"""
        once, hoist, late = mode & RELIN_ONCE, mode & HOIST_MODDOWN, mode & RESCALE_LATE
        b = 1 << ((ilog2(h) + 1) // 2)
        A = Nz(0.0, self.delta, lvl, mu_a)
        B = Nz(0.0, self.delta, lvl, mu_b)
        A0 = self.rs(self.lintrans(A, lambda d: mask_frac(0, d), 1 - h, h - 1, b, hoist))
        B0 = self.rs(self.lintrans(B, lambda d: mask_frac(1, d), 0, h - 1, b, hoist))
        if not late:
            B0 = self.drop(B0)
        bg = h
        if mode & STEP3_BSGS:
            bg = min(h, 1 << ((ilog2(h) + 2) // 2))
        bj = [B0] + [self.rot(B0) for _ in range(1, bg)]
        acc, giants = None, []
        for i in range(h // bg):
            S = None
            for j in range(bg):
                k = bg * i + j
                if k == 0:
                    Ak = self.mulpt(A0, mask_frac(2, 0))
                elif hoist:
                    Ak = self.rot_sum_hoisted([(A0, mask_frac(2, k)), (A0, mask_frac(3, k))])
                else:
                    Ak = self.add(self.mulpt(self.rot(A0), mask_frac(2, k)),
                                  self.mulpt(self.rot(A0), mask_frac(3, k)))
                if not late:
                    Ak = self.rs(Ak)
                prod = self.tensor(Ak, bj[j])
                if not once:
                    prod = self.relin(prod)
                S = self.add(S, prod)
            if once:
                S = self.relin(S)
            if i and hoist:
                giants.append((S, None))
                continue
            acc = self.add(acc, self.rot(S) if i else S)
        if giants:
            acc = self.add(acc, self.rot_sum_hoisted(giants))
        res = self.rs(acc)
        if late:
            res = self.rs(res)
        return res


def mask_fractions(mask_slots, h):
    """mask_frac(kind, k) from slot-domain 0/1 diagonal vectors of length h^2"""
    cache = {}

    def frac(kind, k):
        if (kind, k) not in cache:
            u = np.asarray(mask_slots(kind, h, k), np.float64)
            cache[(kind, k)] = float(np.mean(u * u))
        return cache[(kind, k)]

    return frac
