"""Pins of the reading behind the fused-Laplacian heat form (no GPU).

The binary64 heat sub-timestep (paper, Section 4) is defined as
u' = u + r*((u[i-1] + u[i+1]) - 2u) with every operation rounded.  The GPU's
stage kernels may evaluate the Laplacian as fma(-2, u, s), s = u[i-1] +
u[i+1], which rounds the exact s - 2u once.  The canonical form rounds
s - fl(2u), and fl(2u) = 2u exactly whenever it is finite, so the two agree
for every |u| <= DBL_MAX/2.  The library allows the fused form only for
0 <= r <= 1/2 and |u0| <= DBL_MAX/16, relying on the update being a convex
combination of its inputs, so that the largest magnitude of a level exceeds
the previous level's by a few roundings at most.

These tests pin both halves with exact rational arithmetic (correctly rounded
conversion, ties to even) and with the oracle's own runs.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import workloads
from tests.test_oracle_fma_pins import round32

DMAX = np.finfo(np.float64).max
FMAX = np.finfo(np.float32).max
EPS = 2.0 ** -53                    # unit roundoff of binary64
EPS32 = 2.0 ** -24                  # unit roundoff of binary32


def fma_exact(a: float, b: float, c: float) -> float:
    """a*b + c computed exactly and rounded once to binary64 (ties to even)."""
    x = Fraction(a) * Fraction(b) + Fraction(c)
    return x.numerator / x.denominator


def random_doubles(rng, n, lo_exp, hi_exp):
    """Signed doubles with exponents spread over [lo_exp, hi_exp] (binary),
    including subnormals when lo_exp < -1022."""
    e = rng.integers(lo_exp, hi_exp + 1, n)
    m = rng.uniform(1.0, 2.0, n)
    s = rng.choice([-1.0, 1.0], n)
    return [float(si * math.ldexp(mi, int(ei))) for si, mi, ei in zip(s, m, e)]


@pytest.mark.parametrize("lo,hi", [(-1074, -1000), (-60, 10), (-3, 3), (900, 1021)])
def test_canonical_laplacian_equals_the_fused_one(lo, hi):
    """s - fl(2u) == fma(-2, u, s) for |u| <= DBL_MAX/2 across magnitudes,
    subnormals included, and for neighbouring values where the subtraction
    cancels."""
    rng = np.random.default_rng(lo + 2000)
    us = random_doubles(rng, 3000, lo, hi)
    ss = random_doubles(rng, 3000, lo, hi)
    for u, s in zip(us, ss):
        for s2 in (s, 2.0 * u, np.nextafter(2.0 * u, math.inf), s + 2.0 * u):
            if not math.isfinite(s2) or abs(u) > DMAX / 2 or abs(s2) > DMAX / 2:
                continue
            assert (s2 - 2.0 * u) == fma_exact(-2.0, u, s2)


@pytest.mark.parametrize("lo,hi", [(-149, -120), (-30, 10), (-3, 3), (100, 125)])
def test_canonical_laplacian_equals_the_fused_one_binary32(lo, hi):
    """The same identity in binary32: s - fl32(2u) == fl32(s - 2u exactly)
    for |u| <= FLT_MAX/2, subnormals included."""
    rng = np.random.default_rng(lo + 3000)
    us = np.array(random_doubles(rng, 3000, lo, hi)).astype(np.float32)
    ss = np.array(random_doubles(rng, 3000, lo, hi)).astype(np.float32)
    two = np.float32(2.0)
    for u, s in zip(us, ss):
        for s2 in (s, two * u, np.nextafter(two * u, np.float32(np.inf)), s + two * u):
            if not np.isfinite(s2) or abs(u) > FMAX / 2 or abs(s2) > FMAX / 2:
                continue
            exact = Fraction(float(s2)) - 2 * Fraction(float(u))
            assert float(np.float32(s2 - two * u)) == round32(exact)


def test_the_forms_differ_only_past_half_the_largest_value():
    u, s = 0.6 * DMAX, DMAX
    assert math.isinf(s - 2.0 * u)              # 2u overflows
    assert fma_exact(-2.0, u, s) == pytest.approx(-0.2 * DMAX)
    u = DMAX / 2                                # the largest u whose double is finite
    assert s - 2.0 * u == fma_exact(-2.0, u, s) == 0.0


@pytest.mark.parametrize("r", [0.5, 0.25, 0.1, 0.0])
def test_the_largest_magnitude_stays_bounded(oracle_mod, r):
    """For 0 <= r <= 1/2 the oracle's run keeps max|u| within
    max|u0| * (1 + 7 eps)^n (each update is a convex combination of its three
    inputs, evaluated with four roundings), even for fields at the check's
    bound DBL_MAX/16 with neighbours of equal and opposite sign."""
    n, steps = 512, 2000
    rng = np.random.default_rng(11)
    u0 = (DMAX / 16) * rng.choice([-1.0, 1.0], n) * rng.uniform(0.999, 1.0, n)
    u0[::7] = DMAX / 16
    m0 = np.max(np.abs(u0))
    bound = m0 * (1.0 + 7.0 * EPS) ** steps
    u = u0
    for _ in range(steps // 200):
        u = oracle_mod.heat(u, 200, r)
        assert np.all(np.isfinite(u))
        assert np.max(np.abs(u)) <= bound


@pytest.mark.parametrize("r", [0.5, 0.25, 0.1])
def test_the_largest_magnitude_stays_bounded_binary32(oracle_mod, r):
    """The binary32 run at the check's bound FLT_MAX/16: max|u| stays within
    max|u0| * (1 + 7 eps32)^n."""
    n, steps = 512, 2000
    rng = np.random.default_rng(12)
    u0 = ((FMAX / 16) * rng.choice([-1.0, 1.0], n) * rng.uniform(0.999, 1.0, n)).astype(np.float32)
    u0[::7] = np.float32(FMAX / 16)
    bound = float(np.max(np.abs(u0))) * (1.0 + 7.0 * EPS32) ** steps
    u = u0
    for _ in range(steps // 200):
        u = oracle_mod.heat(u, 200, r)
        assert u.dtype == np.float32 and np.all(np.isfinite(u))
        assert float(np.max(np.abs(u))) <= bound


def test_white_noise_workload_is_far_inside_the_bound():
    """The benchmark's fields (U[-1, 1] heat inputs) pass the range check."""
    u0 = workloads.initial("heat_large")
    assert np.max(np.abs(u0)) <= 1.0 < DMAX / 16
