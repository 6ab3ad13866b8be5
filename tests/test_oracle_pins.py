"""Pins for the CPU oracle: each check compares the oracle with something other
than itself -- a closed form, an exact rational computation, an invariant or a
symmetry of the discrete scheme -- chosen so that a dropped term, a wrong sign
or index, or a misplaced constant fails at least one of them.

Schemes (paper Section 4 for the 3-point heat sub-timestep; Section 6 for KS
by finite differences and explicit RK2, split into radius-1 sub-timesteps as
in Section 2).
"""
from fractions import Fraction
import math

import os

import numpy as np
import pytest

import workloads

EPS64 = np.finfo(np.float64).eps
EPS32 = float(np.finfo(np.float32).eps)


# ------------------------------------------------------------------ helpers

def heat_closed_form(u0: np.ndarray, nsteps: int, r: float) -> np.ndarray:
    """Each discrete Fourier mode m of the periodic 3-point scheme is an
    eigenvector with eigenvalue g_m = 1 - 4 r sin^2(pi m / N)."""
    n = u0.size
    m = np.arange(n)
    g = 1.0 - 4.0 * r * np.sin(np.pi * m / n) ** 2
    return np.real(np.fft.ifft(np.fft.fft(u0.astype(np.float64)) * g ** nsteps))


def heat_rational(u0, nsteps, r):
    """Exact rational time stepping of u' = u + r (u[i-1] - 2u[i] + u[i+1])."""
    u = [Fraction(float(x)) for x in u0]
    r = Fraction(r)
    n = len(u)
    for _ in range(nsteps):
        u = [u[i] + r * (u[i - 1] - 2 * u[i] + u[(i + 1) % n]) for i in range(n)]
    return u


def ks_rational_step(u0, dt, dx):
    """One exact RK2-midpoint step of u_t = -u u_x - u_xx - u_xxxx with central
    differences: D1 a = (a[i+1]-a[i-1])/(2dx), D2 a = (a[i-1]-2a[i]+a[i+1])/dx^2,
    u_xxxx = D2(D2 u); v = u + dt/2 f(u), u' = u + dt f(v)."""
    n = len(u0)
    dt, dx = Fraction(dt), Fraction(dx)

    def d1(a):
        return [(a[(i + 1) % n] - a[i - 1]) / (2 * dx) for i in range(n)]

    def d2(a):
        return [(a[i - 1] - 2 * a[i] + a[(i + 1) % n]) / (dx * dx) for i in range(n)]

    def f(a):
        a1, a2 = d1(a), d2(a)
        a4 = d2(a2)
        return [-a[i] * a1[i] - a2[i] - a4[i] for i in range(n)]

    u = [Fraction(float(x)) for x in u0]
    fu = f(u)
    v = [u[i] + dt / 2 * fu[i] for i in range(n)]
    fv = f(v)
    return [u[i] + dt * fv[i] for i in range(n)]


# ----------------------------------------------------------------- heat f64

@pytest.mark.parametrize("r", [0.25, 0.3, 0.1])
def test_heat_fourier_decay_f64(oracle_mod, r):
    n, steps = 256, 500
    u0 = workloads.white_noise(n, seed=7)
    got = oracle_mod.heat(u0, steps, r)
    want = heat_closed_form(u0, steps, r)
    # coefficients r, 1-2r, r are >= 0 here, so the step is non-expansive and
    # rounding errors add at most ~2 eps |u|_inf per step.
    tol = 4.0 * steps * EPS64 * np.abs(u0).max() + 1e-13
    assert np.abs(got - want).max() <= tol


def test_heat_small_workload_mode_decay(oracle_mod):
    """The 4096-point, 10,000-step sine-mode workload: every mode decays by
    exactly g_m^n (closed form applied to the rounded input array)."""
    w = workloads.WORKLOADS["heat_small"]
    u0 = workloads.initial("heat_small")
    got = oracle_mod.heat(u0, w["nsteps"], w["r"])
    want = heat_closed_form(u0, w["nsteps"], w["r"])
    tol = 4.0 * w["nsteps"] * EPS64 * np.abs(u0).max()
    assert np.abs(got - want).max() <= tol
    # the decay factors of the extreme modes, from the closed form
    g1 = (1 - math.sin(math.pi / 4096) ** 2) ** 10_000
    g64 = (1 - math.sin(64 * math.pi / 4096) ** 2) ** 10_000
    assert abs(g1 - 0.99413) < 1e-5 and abs(g64 / 3.40e-11 - 1) < 1e-2


@pytest.mark.parametrize("n,steps", [(16, 12), (37, 9), (64, 12)])
def test_heat_exact_rational_f64(oracle_mod, n, steps):
    """Integers |u| <= 2^20 with r = 1/4: every intermediate fits in 53 bits,
    so IEEE binary64 must agree with exact rational arithmetic bit for bit."""
    u0 = workloads.integer_field(n, seed=n, amp=1 << 20)
    got = oracle_mod.heat(u0, steps, 0.25)
    want = np.array([float(x) for x in heat_rational(u0, steps, Fraction(1, 4))])
    assert np.array_equal(got, want)
    # and the periodic sum is conserved exactly
    assert math.fsum(got) == math.fsum(u0)


def test_heat_conservation_f64(oracle_mod):
    n, steps = 1000, 300
    u0 = workloads.white_noise(n, seed=3)
    got = oracle_mod.heat(u0, steps, 0.25)
    assert abs(math.fsum(got) - math.fsum(u0)) <= 4 * steps * n * EPS64


def test_heat_special_cases(oracle_mod):
    u0 = workloads.white_noise(101, seed=5)
    assert np.array_equal(oracle_mod.heat(u0, 17, 0.0), u0)           # r = 0: identity
    c = np.full(64, 0.7)
    assert np.array_equal(oracle_mod.heat(c, 50, 0.25), c)              # constants are fixed
    nyq = np.array([(-1.0) ** j for j in range(64)])
    assert np.array_equal(oracle_mod.heat(nyq, 1, 0.25), np.zeros(64))  # g_{N/2} = 0 at r = 1/4
    assert np.array_equal(oracle_mod.heat(u0, 0, 0.25), u0)             # zero steps


def test_heat_reflection_and_translation(oracle_mod):
    n, steps = 96, 40
    u0 = workloads.white_noise(n, seed=11)
    base = oracle_mod.heat(u0, steps, 0.3)
    # reflection i -> -i commutes with the symmetric stencil, bit for bit
    refl = oracle_mod.heat(np.roll(u0[::-1], 1), steps, 0.3)
    assert np.array_equal(refl, np.roll(base[::-1], 1))
    # translation equivariance
    assert np.array_equal(oracle_mod.heat(np.roll(u0, 13), steps, 0.3), np.roll(base, 13))


def test_heat_thread_count_independent(oracle_mod):
    u0 = workloads.white_noise(5000, seed=2)
    a = oracle_mod.heat(u0, 50, 0.25, threads=1)
    b = oracle_mod.heat(u0, 50, 0.25, threads=4)
    assert np.array_equal(a, b)


def test_heat_cone_points_match_full(oracle_mod):
    n, steps = 300, 70
    u0 = workloads.white_noise(n, seed=9)
    full = oracle_mod.heat(u0, steps, 0.25)
    idx = np.array([0, 1, 149, 298, 299])
    assert np.array_equal(oracle_mod.heat_points(u0, steps, 0.25, idx), full[idx])
    # cone wider than the grid (wrap-around)
    full2 = oracle_mod.heat(u0[:50], 40, 0.25)
    assert np.array_equal(oracle_mod.heat_points(u0[:50], 40, 0.25, [0, 7, 49]),
                          full2[[0, 7, 49]])


# ----------------------------------------------------------------- heat f32

def test_heat_fourier_decay_f32(oracle_mod):
    n, steps = 256, 400
    u0 = workloads.white_noise(n, seed=8, dtype=np.float32)
    got = oracle_mod.heat(u0, steps, 0.25)
    assert got.dtype == np.float32
    want = heat_closed_form(u0.astype(np.float64), steps, 0.25)
    assert np.abs(got - want).max() <= 4.0 * steps * EPS32 * np.abs(u0).max()


@pytest.mark.parametrize("n", [16, 29])
def test_heat_exact_rational_f32(oracle_mod, n):
    """Integers |u| <= 2^8, r = 1/4, 6 steps: all values fit in 24 bits."""
    u0 = workloads.integer_field(n, seed=n, amp=1 << 8, dtype=np.float32)
    got = oracle_mod.heat(u0, 6, 0.25)
    want = np.array([float(x) for x in heat_rational(u0, 6, Fraction(1, 4))], dtype=np.float32)
    assert np.array_equal(got, want)


def test_heat_f32_rounds_every_operation(oracle_mod):
    """With a non-dyadic r the binary32 result depends on per-operation
    rounding; numpy float32 elementwise arithmetic is correctly rounded per
    operation, so it fixes the expected bits (a float64 evaluation rounded at
    the end, or a fused multiply-add, would differ)."""
    u0 = workloads.white_noise(200, seed=4, dtype=np.float32)
    r = np.float32(0.3)
    u = u0.copy()
    for _ in range(25):
        left, right = np.roll(u, 1), np.roll(u, -1)
        u = (u + r * ((left + right) - np.float32(2.0) * u)).astype(np.float32)
    got = oracle_mod.heat(u0, 25, 0.3)
    assert np.array_equal(got, u)
    wide = oracle_mod.heat(u0.astype(np.float64), 25, float(r)).astype(np.float32)
    assert not np.array_equal(got, wide)


# ----------------------------------------------------------------------- KS

def ks_symbol(m, n, dx):
    """Eigenvalue of the linear part -D2 - D2 D2 on mode m."""
    s = math.sin(math.pi * m / n) ** 2
    return 4.0 * s / dx ** 2 - 16.0 * s * s / dx ** 4


@pytest.mark.parametrize("m", [1, 3, 7])
def test_ks_linear_growth(oracle_mod, m):
    """Small-amplitude cosine: u^n = R(dt lam)^n u0 with R(z) = 1 + z + z^2/2
    (RK2 midpoint) and lam the discrete symbol of -u_xx - u_xxxx.  The
    nonlinear term only feeds other harmonics at O(A^2)."""
    n, dt, dx, steps, amp = 64, 0.005, 0.5, 200, 1e-6
    j = np.arange(n)
    u0 = amp * np.cos(2 * np.pi * m * j / n)
    got = oracle_mod.ks(u0, steps, dt, dx)
    z = dt * ks_symbol(m, n, dx)
    want_amp = amp * (1 + z + z * z / 2) ** steps
    proj = 2.0 / n * np.dot(got, np.cos(2 * np.pi * m * j / n))
    assert abs(proj / want_amp - 1) < 1e-8
    # forward Euler (1+z)^n, or dt in place of dt/2 in the midpoint, would be
    # off by far more than the tolerance above
    assert abs((1 + z) ** steps / (1 + z + z * z / 2) ** steps - 1) > 1e-6


def test_ks_nonlinear_second_harmonic(oracle_mod):
    """-u u_x on A cos(t j) with the central difference gives exactly
    (A^2 sin t / (2 dx)) sin(2 t j); after one short step the sin(2 t j)
    coefficient is dt times that, to O(dt)."""
    n, dt, dx, amp, m = 64, 1e-4, 0.5, 0.5, 3
    th = 2 * np.pi * m / n
    j = np.arange(n)
    u0 = amp * np.cos(th * j)
    got = oracle_mod.ks(u0, 1, dt, dx)
    coef = 2.0 / n * np.dot(got, np.sin(2 * th * j))
    want = dt * amp * amp * math.sin(th) / (2 * dx)
    assert abs(coef / want - 1) < 1e-2


@pytest.mark.parametrize("amp", [1 << 8, 1 << 10])
def test_ks_exact_rational_one_step(oracle_mod, amp):
    """Integers |u| <= 2^10, dx = 1/2, dt = 2^-8: one RK2 step needs at most
    ~49 significant bits, so binary64 equals exact rational arithmetic."""
    n = 32
    u0 = workloads.integer_field(n, seed=amp, amp=amp)
    got = oracle_mod.ks(u0, 1, 2.0 ** -8, 0.5)
    want = np.array([float(x) for x in ks_rational_step(u0, Fraction(1, 256), Fraction(1, 2))])
    assert np.array_equal(got, want)
    assert math.fsum(got) == math.fsum(u0)


def test_ks_conservation(oracle_mod):
    n, steps = 512, 400
    u0 = workloads.smoothed_noise(n, seed=12)
    got = oracle_mod.ks(u0, steps, 0.005, 0.5)
    assert np.all(np.isfinite(got))
    assert abs(math.fsum(got) - math.fsum(u0)) <= 1e-12 * steps


def test_ks_symmetries(oracle_mod):
    """KS is invariant under (x, u) -> (-x, -u), and the central scheme keeps
    that bit for bit; a one-sided difference would not.  Also translation
    equivariance and fixed constants."""
    n, steps = 128, 60
    u0 = workloads.smoothed_noise(n, seed=21)
    base = oracle_mod.ks(u0, steps, 0.005, 0.5)
    flip = oracle_mod.ks(-np.roll(u0[::-1], 1), steps, 0.005, 0.5)
    assert np.array_equal(flip, -np.roll(base[::-1], 1))
    assert np.array_equal(oracle_mod.ks(np.roll(u0, 17), steps, 0.005, 0.5), np.roll(base, 17))
    c = np.full(40, -1.25)
    assert np.array_equal(oracle_mod.ks(c, 30, 0.005, 0.5), c)


def test_ks_cone_points_match_full(oracle_mod):
    n, steps = 200, 20
    u0 = workloads.smoothed_noise(n, seed=13)
    full = oracle_mod.ks(u0, steps, 0.005, 0.5)
    idx = np.array([0, 5, 100, 199])
    assert np.array_equal(oracle_mod.ks_points(u0, steps, 0.005, 0.5, idx), full[idx])


def test_ks_literal_domain_blows_up(oracle_mod):
    """The literal 128*pi domain at N = 2^20 gives dx = 3.8e-4: explicit RK2
    is violently unstable there (|R(dt lam)| ~ 1e24 for the top mode); a short
    run on the same dx at a small N already overflows.  This is why the
    workloads use dx = 0.5."""
    dx = 128 * math.pi / (1 << 20)
    z = 0.005 * ks_symbol(32, 64, dx)
    assert abs(1 + z + z * z / 2) > 1e20
    u0 = workloads.smoothed_noise(64, seed=1)
    out = oracle_mod.ks(u0, 5, 0.005, dx)
    assert not np.all(np.isfinite(out))


# ------------------------------------------------------------ discrete adjoint

def _window_J(step_fn, u0, nsteps, n0, wgt, cot=None):
    u = u0.copy()
    total = wgt * float(np.dot(u, u)) if n0 <= 0 else 0.0
    for j in range(1, nsteps + 1):
        u = step_fn(u)
        if j >= n0:
            total += wgt * float(np.dot(u, u))
    if cot is not None:
        total += float(np.dot(cot, u))
    return total


@pytest.mark.parametrize("stencil", ["heat", "ks"])
def test_adjoint_matches_finite_differences(oracle_mod, stencil):
    """<dJ/du0, v> equals the central difference of J along v, computed with
    the (separately pinned) forward oracle only."""
    n, nsteps, n0 = 64, 60, 45
    wgt = 1.0 / (16 * n)
    if stencil == "heat":
        u0 = workloads.white_noise(n, seed=31)
        step = lambda u: oracle_mod.heat(u, 1, 0.3)
        g = oracle_mod.heat_adjoint(u0, nsteps, 0.3, n0, wgt)
    else:
        u0 = 3 * workloads.smoothed_noise(n, seed=32)
        step = lambda u: oracle_mod.ks(u, 1, 0.005, 0.5)
        g = oracle_mod.ks_adjoint(u0, nsteps, 0.005, 0.5, n0, wgt)
    rng = workloads.rng(33)
    for _ in range(4):
        v = rng.standard_normal(n)
        v /= np.linalg.norm(v)
        eps = 1e-5
        fd = (_window_J(step, u0 + eps * v, nsteps, n0, wgt) -
              _window_J(step, u0 - eps * v, nsteps, n0, wgt)) / (2 * eps)
        assert abs(fd - np.dot(g, v)) <= 1e-7 * abs(fd) + 1e-13


def test_heat_adjoint_closed_form(oracle_mod):
    """For the heat scheme A is symmetric, so dJ/du0 = 2w sum_j A^{2j} u0 +
    A^n c; in Fourier space every mode m is scaled by g_m = 1 - 4r sin^2(pi m/N)."""
    n, nsteps, n0, r = 128, 200, 150, 0.25
    wgt = 1.0 / n
    u0 = workloads.white_noise(n, seed=34)
    c = workloads.white_noise(n, seed=35)
    got = oracle_mod.heat_adjoint(u0, nsteps, r, n0, wgt, c)
    m = np.arange(n)
    gm = 1.0 - 4.0 * r * np.sin(np.pi * m / n) ** 2
    scale = sum(2 * wgt * gm ** (2 * j) for j in range(n0, nsteps + 1))
    want = np.real(np.fft.ifft(np.fft.fft(u0) * scale + np.fft.fft(c) * gm ** nsteps))
    assert np.abs(got - want).max() <= 1e-12 * max(1.0, np.abs(want).max())


def test_heat_adjoint_is_the_forward_step(oracle_mod):
    """Self-adjointness: with no window term the adjoint of n heat steps
    applied to c is n forward steps of c, bit for bit."""
    n, nsteps = 77, 41
    c = workloads.white_noise(n, seed=36)
    got = oracle_mod.heat_adjoint(workloads.white_noise(n, seed=37), nsteps, 0.3, nsteps + 1, 0.0, c)
    assert np.array_equal(got, oracle_mod.heat(c, nsteps, 0.3))


def test_ks_adjoint_linear_regime(oracle_mod):
    """Around u0 = 0 the KS step is linear and symmetric (R(dt L) with
    L = -D2 - D2 D2), so the adjoint of a cosine mode is R(dt lam)^n times it."""
    n, nsteps, m = 64, 100, 5
    j = np.arange(n)
    c = np.cos(2 * np.pi * m * j / n)
    got = oracle_mod.ks_adjoint(np.zeros(n), nsteps, 0.005, 0.5, nsteps + 1, 0.0, c)
    z = 0.005 * ks_symbol(m, n, 0.5)
    assert np.abs(got - (1 + z + z * z / 2) ** nsteps * c).max() < 1e-12


def _ks_jvp(u0, v, nsteps, dt, dx, n0, wgt, cot):
    """J and its derivative along v by forward-mode (dual-number) stepping of
    the KS scheme written out here: per RK2 step w = D2 u, p = u + (dt/2) F(u,w),
    z = D2 p, u' = u + dt F(p,z), F(a,b) = -(a D1 a + b + D2 b)."""
    c1, c2 = 1.0 / (2.0 * dx), 1.0 / (dx * dx)

    def d1(a):
        return (np.roll(a, -1) - np.roll(a, 1)) * c1

    def d2(a):
        return ((np.roll(a, 1) + np.roll(a, -1)) - 2.0 * a) * c2

    def F(a, da, b, db):
        return (-(a * d1(a) + b + d2(b)),
                -(da * d1(a) + a * d1(da) + db + d2(db)))

    u, du = u0.copy(), v.copy()
    J = dJ = 0.0
    if n0 <= 0:
        J += wgt * np.dot(u, u)
        dJ += 2 * wgt * np.dot(u, du)
    for j in range(1, nsteps + 1):
        w, dw = d2(u), d2(du)
        f, df = F(u, du, w, dw)
        p, dp = u + 0.5 * dt * f, du + 0.5 * dt * df
        z, dz = d2(p), d2(dp)
        f, df = F(p, dp, z, dz)
        u, du = u + dt * f, du + dt * df
        if j >= n0:
            J += wgt * np.dot(u, u)
            dJ += 2 * wgt * np.dot(u, du)
    if cot is not None:
        J += np.dot(cot, u)
        dJ += np.dot(cot, du)
    return J, dJ


@pytest.mark.parametrize("n,nsteps,n0,with_cot", [(16, 5, 2, True), (40, 30, 20, False),
                                                  (9, 12, 0, True)])
def test_ks_adjoint_matches_forward_mode(oracle_mod, n, nsteps, n0, with_cot):
    """Reverse mode (the oracle's adjoint) against forward mode (dual numbers
    through the scheme, no truncation error): <dJ/du0, v> = dJ(u0; v) to
    rounding, for random directions v."""
    u0 = 3 * workloads.smoothed_noise(n, seed=n + 5)
    cot = workloads.white_noise(n, seed=n + 6) if with_cot else None
    wgt = 1.0 / (5 * n)
    g = oracle_mod.ks_adjoint(u0, nsteps, 0.005, 0.5, n0, wgt, cot)
    rng = workloads.rng(n + 7)
    for _ in range(5):
        v = rng.standard_normal(n)
        _, dJ = _ks_jvp(u0, v, nsteps, 0.005, 0.5, n0, wgt, cot)
        assert abs(np.dot(g, v) - dJ) <= 1e-11 * (abs(dJ) + np.abs(g).sum() * np.abs(v).max())


@pytest.mark.parametrize("n,nsteps,n0,with_cot", [(16, 5, 2, True), (40, 30, 20, False),
                                                  (9, 12, 0, True)])
def test_ks_tlm_matches_dual_numbers(oracle_mod, n, nsteps, n0, with_cot):
    """The oracle's tangent-linear model along several directions at once
    against the test's own forward-mode (dual-number) stepping."""
    g = workloads.rng(200 + n)
    u0 = 3 * workloads.smoothed_noise(n, seed=n)
    dirs = g.standard_normal((5, n))
    cot = g.standard_normal(n) if with_cot else None
    wgt = 0.37
    got = oracle_mod.ks_tlm(u0, nsteps, 0.005, 0.5, n0, wgt, dirs, cot, threads=1)
    for q in range(dirs.shape[0]):
        _, dJ = _ks_jvp(u0, dirs[q], nsteps, 0.005, 0.5, n0, wgt, cot)
        assert abs(got[q] - dJ) <= 1e-12 * max(abs(dJ), 1e-300) + 1e-15, (q, got[q], dJ)


def test_ks_tlm_against_finite_differences_and_the_adjoint(oracle_mod):
    """Along random directions the tangent-linear derivative equals a
    Richardson-extrapolated central difference of the (pinned) forward
    oracle, and the (pinned) adjoint's <g, v>."""
    n, nsteps, n0 = 64, 200, 150
    u0 = 3 * workloads.smoothed_noise(n, seed=9)
    dirs = workloads.rng(9).standard_normal((3, n))
    wgt = 1.0 / ((nsteps - n0 + 1) * n)
    got = oracle_mod.ks_tlm(u0, nsteps, 0.005, 0.5, n0, wgt, dirs, threads=1)

    def J(u):
        out = 0.0
        u = oracle_mod.ks(u, n0 - 1, 0.005, 0.5, threads=1)
        for _ in range(n0, nsteps + 1):
            u = oracle_mod.ks(u, 1, 0.005, 0.5, threads=1)
            out += wgt * math.fsum(u * u)
        return out

    g = oracle_mod.ks_adjoint(u0, nsteps, 0.005, 0.5, n0, wgt, threads=1)
    for q in range(3):
        v = dirs[q]
        e = 1e-4
        d1 = (J(u0 + e * v) - J(u0 - e * v)) / (2 * e)
        d2 = (J(u0 + 0.5 * e * v) - J(u0 - 0.5 * e * v)) / e
        fd = (4 * d2 - d1) / 3
        assert abs(got[q] - fd) <= 1e-8 * abs(got[q]), (q, got[q], fd)
        assert abs(got[q] - float(np.dot(g, v))) <= 1e-12 * np.abs(g).sum() * np.abs(v).max()


# ------------------------------------------------------------------- Euler
GAMMA = 1.4


def euler_state(rho, u, p, gamma=GAMMA):
    rho, u, p = np.broadcast_arrays(np.asarray(rho, float), np.asarray(u, float),
                                    np.asarray(p, float))
    return np.stack([rho, rho * u, p / (gamma - 1) + 0.5 * rho * u * u], axis=-1)


def euler_primitive(q, gamma=GAMMA):
    rho = q[:, 0]
    u = q[:, 1] / rho
    return rho, u, (gamma - 1) * (q[:, 2] - 0.5 * rho * u * u)


def exact_riemann(left, right, xi, gamma=GAMMA):
    """Exact solution of the 1D Riemann problem (left/right = (rho, u, p)) at
    similarity coordinates xi = x/t: the star pressure from the two-rarefaction
    / two-shock pressure functions (found by bisection), then the wave pattern
    sampled at each xi (the textbook construction, e.g. Toro, Riemann Solvers
    and Numerical Methods for Fluid Dynamics, ch. 4)."""
    g = gamma
    rl, ul, pl = left
    rr, ur, pr = right
    cl, cr = np.sqrt(g * pl / rl), np.sqrt(g * pr / rr)

    def fk(p, rk, pk, ck):
        if p > pk:       # shock
            A, B = 2 / ((g + 1) * rk), (g - 1) / (g + 1) * pk
            return (p - pk) * np.sqrt(A / (p + B))
        return 2 * ck / (g - 1) * ((p / pk) ** ((g - 1) / (2 * g)) - 1)

    def fsum(p):
        return fk(p, rl, pl, cl) + fk(p, rr, pr, cr) + (ur - ul)

    lo, hi = 1e-12, 10 * max(pl, pr)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if fsum(mid) > 0:
            hi = mid
        else:
            lo = mid
    ps = 0.5 * (lo + hi)
    us = 0.5 * (ul + ur) + 0.5 * (fk(ps, rr, pr, cr) - fk(ps, rl, pl, cl))

    def side(xi_, rk, uk, pk, ck, sgn):
        # sgn = -1 for the left wave, +1 for the right wave; xi_ measured as is
        if ps > pk:      # shock
            rs = rk * ((ps / pk + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / pk + 1))
            S = uk + sgn * ck * np.sqrt((g + 1) / (2 * g) * ps / pk + (g - 1) / (2 * g))
            if sgn * (xi_ - S) > 0:
                return rk, uk, pk
            return rs, us, ps
        rs = rk * (ps / pk) ** (1 / g)
        cs = ck * (ps / pk) ** ((g - 1) / (2 * g))
        head, tail = uk + sgn * ck, us + sgn * cs
        if sgn * (xi_ - head) > 0:
            return rk, uk, pk
        if sgn * (xi_ - tail) < 0:
            return rs, us, ps
        # inside the fan
        u = 2 / (g + 1) * (-sgn * ck + (g - 1) / 2 * uk + xi_)
        c = sgn * (xi_ - u)
        rho = rk * (c / ck) ** (2 / (g - 1))
        return rho, u, pk * (c / ck) ** (2 * g / (g - 1))

    out = np.empty((len(xi), 3))
    for j, x in enumerate(xi):
        out[j] = side(x, rl, ul, pl, cl, -1) if x < us else side(x, rr, ur, pr, cr, +1)
    return out


def mirrored_sod(n):
    """The periodic Sod problem: rho = 0.125, u = 0, p = 0.1 on the left half
    of [0, 1), rho = 1, u = 0, p = 1 on the right half."""
    x = (np.arange(n) + 0.5) / n
    lowside = x < 0.5
    return euler_state(np.where(lowside, 0.125, 1.0), 0.0, np.where(lowside, 0.1, 1.0))


def test_euler_uniform_state_is_exact(oracle_mod):
    q0 = np.tile(euler_state(0.8, 0.7, 1.3), (37, 1))
    assert np.array_equal(oracle_mod.euler(q0, 60, 0.01, 1 / 37, GAMMA), q0)


def test_euler_conservation(oracle_mod):
    n = 256
    x = (np.arange(n) + 0.5) / n
    q0 = euler_state(1 + 0.3 * np.sin(2 * np.pi * x), 0.5 * np.cos(4 * np.pi * x),
                     1 + 0.2 * np.sin(6 * np.pi * x))
    q = oracle_mod.euler(q0, 200, 0.2 / n, 1 / n, GAMMA)
    assert np.allclose(q.sum(axis=0), q0.sum(axis=0), rtol=1e-13, atol=1e-12)
    assert not np.allclose(q, q0)


def test_euler_mirror_symmetry_is_exact(oracle_mod):
    """Reflection about x = 1/4 (cell i <-> cell n/2-1-i) with u -> -u maps
    the mirrored Sod problem to itself; every operation of the scheme commutes
    with it exactly, so the result is symmetric bit for bit."""
    n = 96
    q = oracle_mod.euler(mirrored_sod(n), 120, 0.2 / n, 1 / n, GAMMA)
    j = (n // 2 - 1 - np.arange(n)) % n
    assert np.array_equal(q[:, 0], q[j, 0])
    assert np.array_equal(q[:, 1], -q[j, 1])
    assert np.array_equal(q[:, 2], q[j, 2])
    assert np.abs(q[:, 1]).max() > 0.1


def test_euler_translation_is_exact(oracle_mod):
    n = 64
    q0 = mirrored_sod(n)
    a = oracle_mod.euler(np.roll(q0, 11, axis=0), 50, 0.2 / n, 1 / n, GAMMA)
    b = np.roll(oracle_mod.euler(q0, 50, 0.2 / n, 1 / n, GAMMA), 11, axis=0)
    assert np.array_equal(a, b)


def _sod_error(oracle_mod, n, t=0.1, cfl=0.2):
    dx = 1 / n
    nsteps = int(round(t / (cfl * dx)))
    dt = t / nsteps
    q = oracle_mod.euler(mirrored_sod(n), nsteps, dt, dx, GAMMA)
    x = (np.arange(n) + 0.5) / n
    # two Riemann problems: at x = 1/2 (low | high) and at x = 0 = 1 (high | low)
    low, high = (0.125, 0.0, 0.1), (1.0, 0.0, 1.0)
    near_half = np.abs(x - 0.5) < 0.25
    want = np.empty((n, 3))
    want[near_half] = exact_riemann(low, high, (x[near_half] - 0.5) / t)
    xd = np.where(x[~near_half] > 0.5, x[~near_half] - 1.0, x[~near_half])
    want[~near_half] = exact_riemann(high, low, xd / t)
    rho, u, p = euler_primitive(q)
    return (np.abs(rho - want[:, 0]).mean(), np.abs(u - want[:, 1]).mean(),
            np.abs(p - want[:, 2]).mean())


def test_euler_sod_against_exact_riemann(oracle_mod):
    """Density, velocity and pressure at t = 0.1 against the exact solutions
    of the two Riemann problems (they have not met yet), with the L1 error
    falling as the grid is refined."""
    e200 = _sod_error(oracle_mod, 200)
    e800 = _sod_error(oracle_mod, 800)
    assert e800[0] < 4e-3 and e800[1] < 1e-2 and e800[2] < 4e-3
    for a, b in zip(e200, e800):
        assert b < a / 2.2


def test_euler_smooth_convergence(oracle_mod):
    """An entropy wave (rho = 1 + 0.2 sin 2 pi x, u = 1, p = 1) is carried
    unchanged at speed 1; the scheme converges at about second order (minmod
    clips the extrema, so the L1 order is a little below 2)."""
    errs = []
    for n in (64, 128, 256):
        x = (np.arange(n) + 0.5) / n
        t, nsteps = 0.25, n
        q0 = euler_state(1 + 0.2 * np.sin(2 * np.pi * x), 1.0, 1.0)
        q = oracle_mod.euler(q0, nsteps, t / nsteps, 1 / n, GAMMA)
        # exact cell averages of the translated wave
        xa, xb = x - 0.5 / n - t, x + 0.5 / n - t
        avg = 1 + 0.2 * (np.cos(2 * np.pi * xa) - np.cos(2 * np.pi * xb)) / (2 * np.pi / n)
        errs.append(np.abs(q[:, 0] - avg).mean())
    assert errs[0] / errs[1] > 2.8 and errs[1] / errs[2] > 2.8


def roe_average(qL, qR, gamma=GAMMA):
    """Roe's averaged velocity and total enthalpy of two states (paper,
    Section 7 names the Roe matrix): the square-root-of-density weighted
    means, written from their definition and pinned below by the property
    that defines them, not by the oracle."""
    rl, rr = qL[0], qR[0]
    ul, ur = qL[1] / rl, qR[1] / rr
    pl = (gamma - 1) * (qL[2] - 0.5 * rl * ul * ul)
    pr = (gamma - 1) * (qR[2] - 0.5 * rr * ur * ur)
    hl, hr = (qL[2] + pl) / rl, (qR[2] + pr) / rr
    a, b = math.sqrt(rl), math.sqrt(rr)
    return (a * ul + b * ur) / (a + b), (a * hl + b * hr) / (a + b)


def euler_jacobian(u, H, gamma=GAMMA):
    """The flux Jacobian df/dq of the 1D Euler equations written in the
    velocity u and total enthalpy H."""
    g = gamma
    return np.array([[0.0, 1.0, 0.0],
                     [0.5 * (g - 3) * u * u, (3 - g) * u, g - 1],
                     [u * (0.5 * (g - 1) * u * u - H), H - (g - 1) * u * u, g * u]])


def euler_flux(q, gamma=GAMMA):
    rho, m, E = q
    u = m / rho
    p = (gamma - 1) * (E - 0.5 * m * u)
    return np.array([m, m * u + p, (E + p) * u])


def _roe_property_residual(avg):
    rng = np.random.default_rng(71)
    worst = 0.0
    for _ in range(200):
        qL = euler_state(rng.uniform(0.1, 2.0), rng.uniform(-1.5, 1.5), rng.uniform(0.1, 3.0))
        qR = euler_state(rng.uniform(0.1, 2.0), rng.uniform(-1.5, 1.5), rng.uniform(0.1, 3.0))
        u, H = avg(qL, qR)
        lhs = euler_jacobian(u, H) @ (qR - qL)
        rhs = euler_flux(qR) - euler_flux(qL)
        worst = max(worst, float(np.abs(lhs - rhs).max() / np.abs(rhs).max()))
    return worst


def test_roe_average_satisfies_the_roe_property():
    """A(u~, H~)(qR - qL) = f(qR) - f(qL) is the property that defines Roe's
    average; the test's roe_average meets it on random state pairs, and the
    plausible slips (weights swapped between the sides, plain arithmetic
    means) do not, so the property pins the weighting."""
    assert _roe_property_residual(roe_average) < 1e-12

    def enthalpy(q):
        u = q[1] / q[0]
        p = (GAMMA - 1) * (q[2] - 0.5 * q[0] * u * u)
        return (q[2] + p) / q[0]

    def swapped(qL, qR):
        a, b = math.sqrt(qL[0]), math.sqrt(qR[0])
        return (b * qL[1] / qL[0] + a * qR[1] / qR[0]) / (a + b), \
            (b * enthalpy(qL) + a * enthalpy(qR)) / (a + b)

    def arithmetic(qL, qR):
        return 0.5 * (qL[1] / qL[0] + qR[1] / qR[0]), 0.5 * (enthalpy(qL) + enthalpy(qR))

    assert _roe_property_residual(swapped) > 1e-2
    assert _roe_property_residual(arithmetic) > 1e-2


def _oracle_face_speed(oracle_mod, left, right, n=16):
    """The dissipation speed the oracle uses at the face between two flat
    states.  Cells 0..n/2-1 hold `left`, the rest `right`; all minmod slopes
    vanish, so at face n/2 - 1/2 the first flux sub-timestep sees exactly
    qL = left, qR = right, and the face i - 1/2 of cell i = n/2 - 1 carries the
    plain flux f(left).  One step with dt = 1e-7 dx changes the density of that
    cell by -(dt/dx)(F - f(left)) up to O(dt^2): solve for the speed in
    F = (f(qL) + f(qR))/2 - (speed/2)(qR - qL)."""
    q0 = np.concatenate([np.tile(euler_state(*left), (n // 2, 1)),
                         np.tile(euler_state(*right), (n // 2, 1))])
    dx = 1.0 / n
    dt = 1e-7 * dx
    q = oracle_mod.euler(q0, 1, dt, dx, GAMMA)
    i = n // 2 - 1
    F_rho = q0[i, 1] - (q[i, 0] - q0[i, 0]) * dx / dt      # f(left)[rho] = m_left
    qL, qR = q0[i], q0[i + 1]
    return (0.5 * (qL[1] + qR[1]) - F_rho) / (0.5 * (qR[0] - qL[0]))


def test_euler_oracle_roe_speed_at_a_stationary_contact(oracle_mod):
    """At a contact at rest (u = 0, uniform p, rho = 1 | 0.25) the physical
    fluxes agree, so the density change of one step is the dissipation term
    alone: it recovers the oracle's speed |u~| + c~, which must be Roe's.
    (Weights swapped between the sides give a speed 22% off, arithmetic
    means 12% off.)"""
    left, right = (1.0, 0.0, 1.0), (0.25, 0.0, 1.0)
    got = _oracle_face_speed(oracle_mod, left, right)
    u, H = roe_average(euler_state(*left), euler_state(*right))
    want = abs(u) + math.sqrt((GAMMA - 1) * (H - 0.5 * u * u))
    assert abs(got - want) <= 1e-6 * want, (got, want)


def test_euler_oracle_roe_speed_at_a_general_jump(oracle_mod):
    """The same for two flat states that differ in density, velocity and
    pressure, so that the velocity's weighting matters too."""
    for left, right in (((1.0, 0.3, 1.0), (0.3, -0.4, 0.6)),
                        ((0.2, -0.7, 0.3), (1.4, 0.5, 2.0))):
        got = _oracle_face_speed(oracle_mod, left, right)
        u, H = roe_average(euler_state(*left), euler_state(*right))
        want = abs(u) + math.sqrt((GAMMA - 1) * (H - 0.5 * u * u))
        assert abs(got - want) <= 1e-6 * want, (left, right, got, want)


def test_exact_riemann_reference_values():
    """The test's exact Riemann solver reproduces the published star state of
    Sod's problem (rho, u, p) = (1, 0, 1) | (0.125, 0, 0.1), gamma = 1.4
    (tests/golden/sod_star_state.json, with its source)."""
    import json
    with open(os.path.join(os.path.dirname(__file__), "golden", "sod_star_state.json")) as fh:
        ref = json.load(fh)
    tol = ref["tolerance"]
    left, right = (1.0, 0.0, 1.0), (0.125, 0.0, 0.1)
    a, b = exact_riemann(left, right, np.array([0.9, 1.0]))
    assert abs(a[2] - ref["p_star"]) < tol and abs(a[1] - ref["u_star"]) < tol
    assert abs(a[0] - ref["rho_star_left"]) < tol and abs(b[0] - ref["rho_star_right"]) < tol


def test_oracle_regression_record():
    """The oracle still gives the bits recorded in
    tests/golden/oracle_regression.json (written by make_oracle_regression.py
    from the oracle itself): a change to its arithmetic must come with a new
    record, and with the reading of the paper that justifies it."""
    import json
    import importlib.util
    here = os.path.join(os.path.dirname(__file__), "golden")
    spec = importlib.util.spec_from_file_location("make_oracle_regression",
                                                  os.path.join(here, "make_oracle_regression.py"))
    gen = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(gen)
    with open(os.path.join(here, "oracle_regression.json")) as fh:
        rec = json.load(fh)
    names = []
    for name, fn in gen.cases():
        names.append(name)
        got = np.asarray(fn())
        want = rec[name]
        assert str(got.dtype) == want["dtype"] and list(got.shape) == want["shape"], name
        vals = np.array([float.fromhex(h) for h in want["values"]]).astype(got.dtype)
        assert np.array_equal(got.ravel().view(np.uint8), vals.view(np.uint8)), name
    assert sorted(names) == sorted(rec)
