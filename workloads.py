"""Seeded synthetic inputs for the swept-rule workloads.

This module holds only input generation (random numbers, initial fields and
run sizes); none of the method's arithmetic lives here.  Both the CPU oracle
side (tests) and the HIP side (tests, bench) draw their inputs from it, so the
two sides see identical bytes.

Generator: numpy ``Generator(PCG64(seed))``; workload i uses seed 1000 + i
unless a test passes its own seed.

Workloads (sizes and distributions of the five benchmark configurations):

* ``heat_small``   heat, N=4096, float64, r=0.25, 10,000 steps; u0 is a sum
  of 8 sine modes with N(0,1) amplitudes and distinct mode numbers in [1, 64].
* ``heat_large``   heat, N=2**24, float64 and float32, r=0.25, 20,000 steps;
  u0 ~ U[-1, 1] iid (the float32 field is the float64 one rounded).
* ``ks``           Kuramoto-Sivashinsky, N=2**20, float64, dt=0.005, 50,000
  RK2 steps; u0 = 9-point periodic box filter of 0.1*N(0,1) noise.  Grid
  spacing dx=0.5 (the literal domain length 128*pi gives dx=3.8e-4, for which
  explicit RK2 is unstable by twelve orders of magnitude; the kernel work does
  not depend on dx).
* ``batch``        4096 instances, half heat (r=0.25) half KS (dt=0.005,
  dx=0.5), N log-uniform in [256, 65536] (odd N occurs), steps uniform in
  [1000, 20000], u0 ~ U[-1, 1].
* ``ks_adjoint``   KS at N=2**16, 20,000 steps, u0 as for ``ks``.
* ``euler``        1D Euler equations, N=2**20 cells on [0, 1) (dx = 1/N),
  gamma = 1.4, dt = 0.2 dx, 10,000 midpoint steps; the periodic Sod problem:
  rho = 0.125, u = 0, p = 0.1 on the left half, rho = 1, u = 0, p = 1 on the
  right half (no randomness).  Parity tests also use ``euler_smooth``: seeded
  random Fourier modes in rho, u, p around (1, 0, 1).
* ``euler_small``  the same problem on N=4096 cells, 10,000 steps (a grid
  small enough that each stage is latency-bound).
"""
from __future__ import annotations

from dataclasses import dataclass
import numpy as np

KS_DT = 0.005
KS_DX = 0.5
HEAT_R = 0.25


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def sine_modes(n: int, seed: int, modes: int = 8, max_mode: int = 64) -> np.ndarray:
    """u0_j = sum_q a_q sin(2 pi m_q j / n), a_q ~ N(0,1), m_q distinct in [1, max_mode]."""
    g = rng(seed)
    m = g.choice(np.arange(1, max_mode + 1), size=modes, replace=False)
    a = g.standard_normal(modes)
    j = np.arange(n, dtype=np.float64)
    u = np.zeros(n, dtype=np.float64)
    for aq, mq in zip(a, m):
        u += aq * np.sin(2.0 * np.pi * float(mq) * j / n)
    return u


def white_noise(n: int, seed: int, dtype=np.float64) -> np.ndarray:
    """u0 ~ U[-1, 1] iid, drawn in float64 and rounded to dtype."""
    return rng(seed).uniform(-1.0, 1.0, size=n).astype(dtype)


def smoothed_noise(n: int, seed: int, amp: float = 0.1, width: int = 9) -> np.ndarray:
    """u0 = periodic box filter (width points, centred) of amp * N(0,1) noise."""
    y = amp * rng(seed).standard_normal(n)
    h = width // 2
    acc = np.zeros(n, dtype=np.float64)
    for d in range(-h, h + 1):
        acc += np.roll(y, -d)
    return acc / float(width)


def integer_field(n: int, seed: int, amp: int, dtype=np.float64) -> np.ndarray:
    """Integers in [-amp, amp]: small-integer data keeps the schemes exact."""
    return rng(seed).integers(-amp, amp + 1, size=n).astype(dtype)


@dataclass
class Instance:
    stencil: str      # "heat" or "ks"
    n: int
    nsteps: int
    u0: np.ndarray


def batch(count: int = 4096, seed: int = 1003, nmin: int = 256, nmax: int = 65536,
          smin: int = 1000, smax: int = 20000, with_data: bool = True):
    """Ensemble of independent instances: N log-uniform in [nmin, nmax]
    (rounded to integers, so odd N occurs), steps uniform over the integers in
    [smin, smax], the first half (after a seeded shuffle) heat, the rest KS."""
    g = rng(seed)
    n = np.rint(np.exp(g.uniform(np.log(nmin), np.log(nmax), size=count))).astype(np.int64)
    steps = g.integers(smin, smax + 1, size=count).astype(np.int64)
    kinds = np.array(["heat"] * (count // 2) + ["ks"] * (count - count // 2))
    g.shuffle(kinds)
    out = []
    for q in range(count):
        u0 = g.uniform(-1.0, 1.0, size=int(n[q])) if with_data else None
        out.append(Instance(str(kinds[q]), int(n[q]), int(steps[q]), u0))
    return out


EULER_GAMMA = 1.4
EULER_CFL = 0.2


def euler_state(rho, u, p, gamma: float = EULER_GAMMA) -> np.ndarray:
    """Conserved variables (rho, rho u, E) per cell, shape (N, 3)."""
    rho, u, p = np.broadcast_arrays(np.asarray(rho, float), np.asarray(u, float),
                                    np.asarray(p, float))
    return np.ascontiguousarray(np.stack([rho, rho * u, p / (gamma - 1) + 0.5 * rho * u * u],
                                         axis=-1))


def euler_mirrored_sod(n: int) -> np.ndarray:
    """The periodic Sod problem on n cells of [0, 1)."""
    x = (np.arange(n) + 0.5) / n
    low = x < 0.5
    return euler_state(np.where(low, 0.125, 1.0), 0.0, np.where(low, 0.1, 1.0))


def euler_smooth(n: int, seed: int, modes: int = 6) -> np.ndarray:
    """rho, u, p = (1, 0, 1) plus seeded random low Fourier modes (rho and p
    stay within [0.5, 1.5])."""
    g = rng(seed)
    x = (np.arange(n) + 0.5) / n
    fields = []
    for base, amp in ((1.0, 0.5), (0.0, 0.5), (1.0, 0.5)):
        f = np.zeros(n)
        for m in g.choice(np.arange(1, 9), size=modes, replace=True):
            f += g.uniform(-1, 1) * np.sin(2 * np.pi * m * x + g.uniform(0, 2 * np.pi))
        fields.append(base + amp * f / max(1.0, np.abs(f).max()))
    return euler_state(*fields)


WORKLOADS = {
    "heat_small": dict(stencil="heat", n=4096, nsteps=10_000, r=HEAT_R, seed=1000),
    "heat_large": dict(stencil="heat", n=1 << 24, nsteps=20_000, r=HEAT_R, seed=1001),
    "ks": dict(stencil="ks", n=1 << 20, nsteps=50_000, dt=KS_DT, dx=KS_DX, seed=1002),
    "batch": dict(count=4096, seed=1003),
    "ks_adjoint": dict(stencil="ks", n=1 << 16, nsteps=20_000, dt=KS_DT, dx=KS_DX, seed=1004),
    "euler": dict(stencil="euler", n=1 << 20, nsteps=10_000, gamma=EULER_GAMMA, cfl=EULER_CFL,
                  seed=1005),
    "euler_small": dict(stencil="euler", n=4096, nsteps=10_000, gamma=EULER_GAMMA,
                        cfl=EULER_CFL, seed=1006),
}


KS_ADJOINT_WINDOW = 2000   # J = mean of u^2 over the final 2,000 steps


def adjoint_directions(n: int, count: int = 16, seed: int = 1104) -> np.ndarray:
    """Seeded unit directions for checks of a gradient: row q is z / |z|_2
    with z ~ N(0, I) (the q-th draw of n normals)."""
    g = rng(seed)
    out = np.empty((count, n))
    for q in range(count):
        z = g.standard_normal(n)
        out[q] = z / np.linalg.norm(z)
    return out


def initial(name: str, dtype=np.float64, n: int | None = None) -> np.ndarray:
    """Initial field of a named workload (optionally at another size n)."""
    w = WORKLOADS[name]
    size = w["n"] if n is None else n
    if name == "heat_small":
        return sine_modes(size, w["seed"]).astype(dtype)
    if name == "heat_large":
        return white_noise(size, w["seed"], dtype)
    if name in ("ks", "ks_adjoint"):
        return smoothed_noise(size, w["seed"]).astype(dtype)
    if name in ("euler", "euler_small"):
        return euler_mirrored_sod(size)
    raise KeyError(name)
