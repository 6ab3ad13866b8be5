"""The fused-Laplacian evaluation of heat (binary64 and binary32) in
swept_advance.

(u[i-1] + u[i+1]) - 2u equals fma(-2, u, u[i-1] + u[i+1]) bit for bit while
2u is finite; the library takes the fused form only after its range check
(0 <= r <= 1/2, every finite |u0| <= MAX/16 for the type's largest finite
value MAX), which keeps every point far from MAX/2 (paper, Section 4: the
heat sub-timestep).  Both forms must
give the oracle's bits; the checks here also make sure the fused form is the
one taken where it is allowed, that data or parameters outside the allowed
range take the five operations as written, and that one call's failed check
does not stick to later calls."""
import numpy as np
import pytest

import workloads
from tests.conftest import gpu_available, same_bits

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

DMAX = np.finfo(np.float64).max
FMAX = np.finfo(np.float32).max


@pytest.fixture(scope="module")
def sw():
    import paper_1504_01380_amd as swept
    swept.init(0)
    yield swept
    swept.set_tuning(0, 0, swept.MODE_AUTO)
    swept.set_heat_form(swept.FORM_AUTO)


@pytest.fixture(autouse=True)
def _reset(sw):
    sw.set_tuning(0, 0, sw.MODE_AUTO)
    sw.set_heat_form(sw.FORM_AUTO)
    yield
    sw.set_tuning(0, 0, sw.MODE_AUTO)
    sw.set_heat_form(sw.FORM_AUTO)


def run(sw, u0, nsteps, r, fn=None):
    import torch
    u = torch.from_numpy(np.ascontiguousarray(u0)).to("cuda")
    (fn or sw.advance)(u, nsteps, "heat", [r])
    torch.cuda.synchronize()
    sw.sync()
    return u.cpu().numpy()


def same_bits_up_to_nan(a, b):
    """Byte equality except that any two NaNs match (the payload a NaN
    carries is not part of the scheme)."""
    na, nb = np.isnan(a), np.isnan(b)
    return np.array_equal(na, nb) and same_bits(a[~na], b[~nb])


# (label, nx, nsteps, tuning): the continuous and banded kernels (equal
# tiles), the lane-frame kernel (few tiles) and the unequal tiling (odd nx on
# its two-fold cover, and an even nx with no good even divisor)
PLANS = [("cont_W1024_P4", 1 << 16, 1500, (1024, 4, 1)),
         ("cont_W512_P2", 3 << 12, 777, (512, 2, 1)),
         ("banded", 1 << 14, 600, (256, 1, 3)),
         ("lane", 4096, 1000, (64, 0, 4)),
         ("ragged_odd", 1001, 700, (0, 0, 0)),
         ("ragged_8198", 8198, 513, (0, 0, 0)),
         ("auto", 5000, 300, (0, 0, 0))]


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("label,nx,nsteps,tuning", PLANS)
def test_fused_form_is_taken_and_exact(sw, oracle_mod, label, nx, nsteps, tuning, dtype):
    u0 = workloads.white_noise(nx, seed=nx + 3, dtype=dtype)
    want = oracle_mod.heat(u0, nsteps, 0.25)
    sw.set_tuning(*tuning)
    got = run(sw, u0, nsteps, 0.25)
    assert sw.last_heat_form() == sw.FORM_FUSED
    assert same_bits(got, want)
    sw.set_heat_form(sw.FORM_CANONICAL)
    got = run(sw, u0, nsteps, 0.25)
    assert sw.last_heat_form() == sw.FORM_CANONICAL
    assert same_bits(got, want)


@pytest.mark.parametrize("dtype,r", [(dt, r) for dt in (np.float64, np.float32)
                                     for r in (0.0, 0.1, 0.3, 0.5)] +
                         [(np.float32, 0.5000000000000001)])
def test_fused_form_over_the_allowed_r(sw, oracle_mod, r, dtype):
    """0 <= r <= 1/2 as the field's type rounds it (the double just above
    1/2 rounds to 1/2 in binary32)."""
    u0 = workloads.white_noise(1 << 14, seed=77, dtype=dtype)
    sw.set_tuning(256, 2, 1)
    got = run(sw, u0, 900, r)
    assert sw.last_heat_form() == sw.FORM_FUSED
    assert same_bits(got, oracle_mod.heat(u0, 900, r))


@pytest.mark.parametrize("dtype,r", [(np.float64, -0.05), (np.float64, 0.5000000000000001),
                                     (np.float64, 0.6), (np.float64, 1.0),
                                     (np.float32, -0.05), (np.float32, 0.50000006),
                                     (np.float32, 0.6)])
def test_r_outside_the_range_takes_the_canonical_form(sw, oracle_mod, dtype, r):
    u0 = workloads.white_noise(1 << 14, seed=78, dtype=dtype)
    sw.set_tuning(256, 2, 1)
    got = run(sw, u0, 120, r)
    assert sw.last_heat_form() == sw.FORM_CANONICAL
    assert same_bits_up_to_nan(got, oracle_mod.heat(u0, 120, r))


@pytest.mark.parametrize("dtype,big", [(np.float64, DMAX), (np.float32, FMAX)])
def test_values_near_the_overflow_take_the_canonical_form(sw, oracle_mod, dtype, big):
    """Values of 0.4..0.6 MAX: 2u overflows for half of them, so the
    oracle's run fills with infinities and NaNs, which the fused form would
    not produce.  The range check must send the call to the canonical form."""
    rng = np.random.default_rng(5)
    u0 = (big * (0.5 + 0.1 * rng.uniform(-1.0, 1.0, 1 << 14))).astype(dtype)
    want = oracle_mod.heat(u0, 40, 0.25)
    assert not np.all(np.isfinite(want))        # the case separates the two forms
    sw.set_tuning(256, 2, 1)
    got = run(sw, u0, 40, 0.25)
    assert sw.last_heat_form() == sw.FORM_CANONICAL
    assert same_bits_up_to_nan(got, want)


@pytest.mark.parametrize("dtype,big", [(np.float64, DMAX), (np.float32, FMAX)])
def test_the_bound_is_a_sixteenth_of_the_largest_value(sw, oracle_mod, dtype, big):
    u0 = workloads.white_noise(1 << 14, seed=79, dtype=dtype)
    sw.set_tuning(256, 2, 1)
    lim = dtype(big / 16)
    for scale, form in ((lim, sw.FORM_FUSED),
                        (np.nextafter(lim, dtype(np.inf)), sw.FORM_CANONICAL)):
        v = u0.copy()
        v[123] = scale
        got = run(sw, v, 200, 0.25)
        assert sw.last_heat_form() == form
        assert same_bits(got, oracle_mod.heat(v, 200, 0.25))


def test_non_finite_values_pass_the_check(sw, oracle_mod):
    """Infinities in the field allow the fused form: a non-finite input only
    makes non-finite outputs, the same in both forms."""
    u0 = workloads.white_noise(1 << 14, seed=80)
    u0[[10, 5000]] = [np.inf, -np.inf]
    sw.set_tuning(256, 2, 1)
    got = run(sw, u0, 300, 0.25)
    assert sw.last_heat_form() == sw.FORM_FUSED
    want = oracle_mod.heat(u0, 300, 0.25)
    assert same_bits_up_to_nan(got, want)
    assert np.isnan(want).any() and np.isfinite(want).any()


def test_a_failed_check_does_not_stick(sw, oracle_mod):
    good = workloads.white_noise(1 << 14, seed=81)
    bad = good.copy()
    bad[7] = DMAX / 4
    sw.set_tuning(256, 2, 1)
    for u0, form in ((good, sw.FORM_FUSED), (bad, sw.FORM_CANONICAL),
                     (good, sw.FORM_FUSED), (bad, sw.FORM_CANONICAL)):
        got = run(sw, u0, 250, 0.25)
        assert sw.last_heat_form() == form
        assert same_bits_up_to_nan(got, oracle_mod.heat(u0, 250, 0.25))


def test_naive_and_noalloc_report_their_forms(sw, oracle_mod):
    u0 = workloads.white_noise(1 << 14, seed=82)
    want = oracle_mod.heat(u0, 300, 0.25)
    got = run(sw, u0, 300, 0.25, fn=sw.advance_noalloc)
    assert sw.last_heat_form() == sw.FORM_FUSED
    assert same_bits(got, want)
    sw.set_tuning(0, 0, sw.MODE_NAIVE)
    got = run(sw, u0, 300, 0.25)
    assert sw.last_heat_form() == sw.FORM_CANONICAL
    assert same_bits(got, want)
