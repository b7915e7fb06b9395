"""Pins for the oracle's constants: hash keys, mixer, Poisson thresholds, t(k)
and the region tables.  Each is checked against a published value or an
independent high-precision computation, not against the oracle's own code."""
import math
import os
from decimal import Decimal, getcontext
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

from oracle import oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden")
M64 = (1 << 64) - 1


def _rows(name):
    out = []
    for line in open(os.path.join(GOLD, name)):
        line = line.strip()
        if line and not line.startswith("#"):
            out.append(line.split())
    return out


def test_mt19937_64_standard_value():
    # C++ [rand.predef]: 10000th output of default-seeded mt19937_64.
    for seed, n, val in _rows("mt19937_64.txt"):
        assert O.mt19937_64(int(seed), int(n))[-1] == int(val)


def test_mixer_is_splitmix64_finaliser():
    # The oracle's mixer, driven as the SplitMix64 generator, reproduces the
    # generator's published outputs.
    for seed, n, val in _rows("splitmix64.txt"):
        state = (int(seed) + int(n) * 0x9E3779B97F4A7C15) & M64
        assert O.mix64(state) == int(val, 0)


def test_mixer_is_a_bijection():
    # Invert each step (xor-shift and odd multiplication) and recover the input.
    def unxorshift(z, s):
        x = z
        for _ in range(64 // s + 1):
            x = z ^ (x >> s)
        return x & M64

    inv1 = pow(0xBF58476D1CE4E5B9, -1, 1 << 64)
    inv2 = pow(0x94D049BB133111EB, -1, 1 << 64)
    rng = np.random.default_rng(5)
    for v in [0, 1, M64, 1 << 63] + [int(x) for x in rng.integers(0, 2**63, 200)]:
        z = O.mix64(v)
        z = unxorshift(z, 31)
        z = (z * inv2) & M64
        z = unxorshift(z, 27)
        z = (z * inv1) & M64
        z = unxorshift(z, 30)
        assert z == v


def test_poisson_thresholds_high_precision():
    # floor(2^64 * P[Poi(1) <= n]) with e^-1 from 60-digit decimal arithmetic.
    getcontext().prec = 60
    einv = Decimal(-1).exp()
    C = O.poisson_thresholds()
    assert len(C) == 20
    acc = Decimal(0)
    fact = Decimal(1)
    for n in range(20):
        if n:
            fact *= n
        acc += 1 / fact
        v = einv * acc * (Decimal(2) ** 64)
        assert int(v) == C[n], n  # v > 0, int() is floor
    # strictly increasing, below 2^64, and the increments follow 1/n!
    assert all(C[n] < C[n + 1] for n in range(19)) and C[19] < 2 ** 64
    assert C[0] == 6786177901268885274  # floor(2^64 / e)
    for n in range(1, 12):
        ratio = (C[n] - C[n - 1]) / (C[n - 1] - (C[n - 2] if n > 1 else 0))
        assert abs(ratio - 1.0 / n) < 1e-9
    # agrees with a library CDF to double precision
    for n in range(20):
        assert abs(stats.poisson.cdf(n, 1.0) * 2.0 ** 64 - C[n]) < 2.0 ** 13


def test_t_of_k():
    for k, t in _rows("t_of_k.txt"):
        assert O.t_of_k(int(k)) == int(t)
    # agreement with a double-precision evaluation wherever k ln k is not
    # within 1e-9 of an integer, and the bound lambda = t/k >= 1 + ln k that
    # the proof of Theorem 1 needs
    for k in range(1, 4097):
        v = k * math.log(k)
        t = O.t_of_k(k)
        if abs(v - round(v)) > 1e-9:
            assert t == math.ceil(v) + k
        assert t / k >= 1 + math.log(k) - 1e-12


def test_region_tables():
    for t in (1, 4, 331, 1676, 8122, 512):
        W, R, u = O.tables(t)
        assert u == float(Fraction(1, t))
        for nu in range(54):
            assert W[nu] == float(Fraction(2 ** nu - 1, t))  # correctly rounded
            assert R[nu] == 2.0 ** nu - 1
        assert len(W) == len(R) == 1024
        for nu in range(1023):
            assert W[nu] < W[nu + 1] and R[nu] < R[nu + 1]
            rel = abs(Fraction(W[nu + 1]) - Fraction(2 ** (nu + 1) - 1, t)) / Fraction(2 ** (nu + 1) - 1, t)
            assert rel <= Fraction(1, 2 ** 52)
