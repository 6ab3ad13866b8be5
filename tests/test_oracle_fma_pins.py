"""Pins for the contraction-on forms of the oracle (heat_fma, ks_fma): the
schemes with each multiply-add fused, the form in which the paper's Section 4
counts the heat sub-timestep as 3 FLOPs.

Each operation of these definitions is an IEEE operation with one rounding
(add, sub, mul, or a fused multiply-add rounded once), so a brute force that
evaluates every operation exactly in rationals and rounds it to the nearest
binary64 (or binary32) value, ties to even, must give the oracle's bits.
That holds for any r and any data, not only in an exact regime, so it also
tells a fused from an unfused multiply-add.  The heat form is further pinned
by the Fourier closed form of the scheme.
"""
from fractions import Fraction

import numpy as np
import pytest

import workloads
from tests.conftest import same_bits
from tests.test_oracle_pins import EPS32, EPS64, heat_closed_form


def round64(x: Fraction) -> float:
    """Nearest binary64 value, ties to even (int / int true division in
    Python is correctly rounded)."""
    return x.numerator / x.denominator


def round32(x: Fraction) -> float:
    """Nearest binary32 value, ties to even: the binary64 rounding can be off
    by double rounding, so compare it with its binary32 neighbours exactly."""
    f = np.float32(round64(x))
    best = None
    for c in (np.nextafter(f, np.float32(-np.inf)), f, np.nextafter(f, np.float32(np.inf))):
        d = abs(Fraction(float(c)) - x)
        if best is None or d < best[0] or \
                (d == best[0] and int(np.array(c).view(np.uint32)) % 2 == 0):
            best = (d, c)
    return float(best[1])


class Arith:
    """IEEE binary64 or binary32 operations, each rounded once."""

    def __init__(self, rnd):
        self.rnd = rnd

    def v(self, x):
        return Fraction(self.rnd(Fraction(x)))

    def add(self, a, b):
        return Fraction(self.rnd(a + b))

    def sub(self, a, b):
        return Fraction(self.rnd(a - b))

    def mul(self, a, b):
        return Fraction(self.rnd(a * b))

    def fma(self, a, b, c):
        return Fraction(self.rnd(a * b + c))


def heat_fma_brute(u0, nsteps, r, ar):
    u = [ar.v(float(x)) for x in u0]
    r = ar.v(r)
    n = len(u)
    for _ in range(nsteps):
        u = [ar.fma(r, ar.fma(Fraction(-2), u[i], ar.add(u[i - 1], u[(i + 1) % n])), u[i])
             for i in range(n)]
    return u


@pytest.mark.parametrize("r", [0.3, 0.1, 0.25])
def test_heat_fma_brute_force_f64(oracle_mod, r):
    n, steps = 11, 7
    u0 = workloads.white_noise(n, seed=31)
    want = np.array([float(x) for x in heat_fma_brute(u0, steps, r, Arith(round64))])
    assert same_bits(oracle_mod.heat_fma(u0, steps, r), want)


def test_heat_fma_brute_force_f32(oracle_mod):
    n, steps = 9, 6
    u0 = workloads.white_noise(n, seed=32).astype(np.float32)
    r = float(np.float32(0.3))
    want = np.array([float(x) for x in heat_fma_brute(u0, steps, r, Arith(round32))],
                    dtype=np.float32)
    assert same_bits(oracle_mod.heat_fma(u0, steps, 0.3), want)


def test_heat_fma_differs_from_the_unfused_scheme(oracle_mod):
    """At r = 0.3 the product r*lap is inexact, so fusing changes bits: the
    brute force above tells the two apart."""
    u0 = workloads.white_noise(64, seed=33)
    assert not same_bits(oracle_mod.heat_fma(u0, 20, 0.3), oracle_mod.heat(u0, 20, 0.3))


@pytest.mark.parametrize("r", [0.25, 0.3, 0.1])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_heat_fma_fourier_decay(oracle_mod, r, dtype):
    n, steps = 256, 500
    u0 = workloads.white_noise(n, seed=34).astype(dtype)
    got = oracle_mod.heat_fma(u0, steps, r)
    rr = float(np.float32(r)) if dtype == np.float32 else r
    want = heat_closed_form(u0, steps, rr)
    eps = EPS32 if dtype == np.float32 else EPS64
    tol = 4.0 * steps * eps * np.abs(u0).max() + 1e-13
    assert np.abs(got - want).max() <= tol


def ks_fma_brute(u0, nsteps, dt, dx, ar):
    """The KS scheme with fused multiply-adds, every operation rounded once:
    D2(a) = fma(-2, a, a[i-1] + a[i+1]) * c2, D1(a) = (a[i+1] - a[i-1]) * c1,
    F(a,b) = -(fma(a, D1 a, b) + D2 b), v = fma(h, F(u,w), u), u' = fma(dt, F(v,z), u),
    with c1 = 1/(2dx), c2 = 1/(dx dx), h = dt/2 rounded once."""
    n = len(u0)
    c1 = ar.v(1.0 / (2.0 * dx))
    c2 = ar.v(1.0 / (dx * dx))
    h = ar.v(0.5 * dt)
    dtq = ar.v(dt)
    u = [ar.v(float(x)) for x in u0]

    def d2(a, i):
        return ar.mul(ar.fma(Fraction(-2), a[i], ar.add(a[i - 1], a[(i + 1) % n])), c2)

    def F(a, b, i):
        d1 = ar.mul(ar.sub(a[(i + 1) % n], a[i - 1]), c1)
        return -ar.add(ar.fma(a[i], d1, b[i]), d2(b, i))

    for _ in range(nsteps):
        w = [d2(u, i) for i in range(n)]
        v = [ar.fma(h, F(u, w, i), u[i]) for i in range(n)]
        z = [d2(v, i) for i in range(n)]
        u = [ar.fma(dtq, F(v, z, i), u[i]) for i in range(n)]
    return u


@pytest.mark.parametrize("dx", [0.5, 0.7])
def test_ks_fma_brute_force(oracle_mod, dx):
    n, steps = 10, 3
    u0 = workloads.white_noise(n, seed=35)
    want = np.array([float(x) for x in ks_fma_brute(u0, steps, 0.005, dx, Arith(round64))])
    got = oracle_mod.ks_fma(u0, steps, 0.005, dx)
    assert same_bits(got, want)
    assert not same_bits(got, oracle_mod.ks(u0, steps, 0.005, dx))


def test_ks_fma_close_to_the_unfused_scheme(oracle_mod):
    """Over a short horizon the two forms differ by rounding only."""
    u0 = workloads.smoothed_noise(512, seed=36)
    a = oracle_mod.ks_fma(u0, 200, 0.005, 0.5)
    b = oracle_mod.ks(u0, 200, 0.005, 0.5)
    assert 0 < np.abs(a - b).max() <= 1e-13 * np.abs(b).max()
