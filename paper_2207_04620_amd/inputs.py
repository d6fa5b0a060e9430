"""Seeded synthetic inputs and parameter presets shared by the tests, the smoke
check and the benchmark.

This module holds no homomorphic arithmetic: only parameter choices (ring
degree, prime bit sizes, digit width, scale, seed) and numpy generators for the
plaintext matrices.  The paper's own inputs are dataset activations and model
weights; matrices with entries uniform in [-1, 1] of the paper's shapes stand in
for them (Sec. 3.6 multiplies h x h matrices; matrices are zero-padded to powers
of two, as in the experiments section).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List

import numpy as np


@dataclass(frozen=True)
class Params:
    name: str
    log_n: int
    q_bits: List[int]
    p_bits: List[int]
    alpha: int
    log_scale: float
    seed: int
    h_list: List[int] = field(default_factory=list)

    @property
    def n(self) -> int:
        return 1 << self.log_n

    @property
    def max_level(self) -> int:
        return len(self.q_bits) - 1

    @property
    def dnum(self) -> int:
        return -(-len(self.q_bits) // self.alpha)


# N=2^12, q0 40-bit, q1 30-bit, P 40-bit, scale 2^30: one multiplicative level.
C1 = Params("C1", 12, [40, 30], [40], 1, 30.0, 1, [8])
# The h=8 product needs depth 3: the same ring, q0 and P with q1 replaced by three
# 30-bit primes.
C1P = Params("C1+", 12, [40, 30, 30, 30], [40], 1, 30.0, 1, [8])
# N=2^14, 7 x 40-bit Q primes, one 60-bit special prime, scale 2^40 (dnum = 7).
C2 = Params("C2", 14, [40] * 7, [60], 1, 40.0, 2, [64])
# N=2^15, Q = 60 + 13 x 45 bits (14 limbs), P = 3 x 60 + 56 bits, alpha = 5 (dnum = 3).
C3 = Params("C3", 15, [60] + [45] * 13, [60, 60, 60, 56], 5, 45.0, 3, [16, 32, 64])
# N=2^16, Q = 60 + 16 x 45 bits (17 limbs), P = 5 x 60 bits, alpha = 6 (dnum = 3).
C4 = Params("C4", 16, [60] + [45] * 16, [60] * 5, 6, 45.0, 4, [32])

PRESETS = {p.name: p for p in (C1, C1P, C2, C3, C4)}


def small(log_n: int = 10, n_q: int = 5, q_bits: int = 40, p_bits: int = 50, alpha: int = 2,
          log_scale: float = 40.0, seed: int = 7, h_list=(4, 8)) -> Params:
    """A small ring for fast functional tests (not a security parameter set)."""
    return Params(f"small{log_n}", log_n, [q_bits + 10] + [q_bits] * (n_q - 1), [p_bits] * 2, alpha,
                  log_scale, seed, list(h_list))


def matrix(seed: int, h: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """h x h matrix with entries uniform in [lo, hi] (row-major, the encoding iota of Sec. 3.4)."""
    return np.random.default_rng(seed).uniform(lo, hi, size=(h, h))


def matrix_pair(seed: int, h: int):
    rng = np.random.default_rng(seed)
    return rng.uniform(-1, 1, size=(h, h)), rng.uniform(-1, 1, size=(h, h))


def sign_inputs(seed: int, count: int, h: int) -> np.ndarray:
    """count matrices of h x h entries with |x| ~ U[2^-8, 1] and a random sign."""
    rng = np.random.default_rng(seed)
    mag = rng.uniform(2.0 ** -8, 1.0, size=(count, h, h))
    sgn = np.where(rng.random(size=(count, h, h)) < 0.5, -1.0, 1.0)
    return mag * sgn


def batch_mix(seed: int, count: int, h_choices=(16, 32, 64), levels=(3, 13)):
    """(h, level) for each member of a mixed batch: h uniform over h_choices,
    starting level uniform over [levels[0], levels[1]]."""
    rng = np.random.default_rng(seed)
    hs = rng.choice(np.asarray(h_choices), size=count)
    lv = rng.integers(levels[0], levels[1] + 1, size=count)
    return [(int(h), int(l)) for h, l in zip(hs, lv)]


def plaintext_poly(seed: int, n: int, bound: int) -> np.ndarray:
    """an integer polynomial with coefficients uniform in [-bound, bound]."""
    return np.random.default_rng(seed).integers(-bound, bound + 1, size=n, dtype=np.int64)


def residues(seed: int, shape, moduli) -> np.ndarray:
    """uniform residues: last axis N, second-to-last axis one limb per modulus."""
    rng = np.random.default_rng(seed)
    out = np.empty(shape, np.uint64)
    for i, q in enumerate(moduli):
        out[..., i, :] = rng.integers(0, q, size=out[..., i, :].shape, dtype=np.uint64)
    return out


def poisson_arrivals(seed: int, rate_per_s: float, count: int) -> np.ndarray:
    """arrival times (seconds from 0) of a Poisson process with the given rate"""
    return np.cumsum(np.random.default_rng(seed).exponential(1.0 / rate_per_s, size=count))
