"""Pins of the oracle's entropic KBC-type collision (Sec. III-C "Entropic
KBC Models"): the update is the independently pinned weighted MRT with the
cell's own higher-order rate; that rate maximises the quadratic expansion of
the entropy (checked by brute-force search, not by the closed form); it
tends to the exact entropy maximiser as the non-equilibrium shrinks;
conservation; and no higher-order non-equilibrium leaves the MRT result."""

import numpy as np
import pytest
from scipy.optimize import minimize_scalar

from oracle import collision as col
from oracle.equilibrium import equilibrium
from oracle.lattice import velocity_set

STENCILS = ["D2Q9", "D3Q19", "D3Q27"]
RATES = dict(omega=1 / 0.6, omega_bulk=1.2, omega_odd=0.0, magic=0.0, omega_hi=(1.0, 1.0, 1.0, 1.0))


def _cells(lat, n, seed, amp, umax=0.05):
    """n random cells: equilibrium at random rho, u times (1 + amp * noise)."""
    rng = np.random.default_rng(seed)
    rho = 1.0 + 0.02 * rng.uniform(-1, 1, n)
    u = umax * rng.uniform(-1, 1, (3, n))
    if lat.d == 2:
        u[2] = 0.0
    feq = equilibrium(lat, rho, u, 1.0, True)
    return feq * (1.0 + amp * rng.uniform(-1, 1, feq.shape))


def _force(lat, n, seed):
    rng = np.random.default_rng(seed)
    F = 1e-3 * rng.uniform(-1, 1, (3, n))
    if lat.d == 2:
        F[2] = 0.0
    return F


@pytest.mark.parametrize("name", STENCILS)
@pytest.mark.parametrize("forced", [False, True])
def test_kbc_is_mrt_with_the_cells_higher_order_rate(name, forced):
    lat = velocity_set(name)
    f = _cells(lat, 40, 1, 0.05)
    F = _force(lat, 40, 2) if forced else None
    out = col.kbc(lat, f, RATES, F)
    omh = col.kbc_parts(lat, f, RATES, F)[4]
    assert np.all(np.isfinite(omh)) and np.ptp(omh) > 0   # a genuinely local rate
    for i in range(f.shape[1]):
        r = dict(RATES, omega_hi=(omh[i],) * 4)
        ref = col.mrt(lat, f[:, i:i + 1], r, None if F is None else F[:, i:i + 1])
        np.testing.assert_allclose(out[:, i], ref[:, 0], rtol=0, atol=1e-14)


@pytest.mark.parametrize("name", STENCILS)
def test_kbc_rate_maximises_quadratic_entropy(name):
    """With ln x ~ x - 1 the entropy of f' is, up to a constant,
    -1/2 sum (f' - f^eq)^2 / f^eq; a grid search over omega_h finds its
    maximum where the closed form puts it."""
    lat = velocity_set(name)
    f = _cells(lat, 12, 3, 0.05)
    ds, db, dh, feq, omh, _, _ = col.kbc_parts(lat, f, RATES)
    for i in range(f.shape[1]):
        grid = omh[i] + np.linspace(-0.5, 0.5, 100001)
        post = (f[:, i:i + 1] - RATES["omega"] * ds[:, i:i + 1] - RATES["omega_bulk"] * db[:, i:i + 1]
                - grid[None, :] * dh[:, i:i + 1])
        s2 = -0.5 * ((post - feq[:, i:i + 1]) ** 2 / feq[:, i:i + 1]).sum(axis=0)
        assert abs(grid[np.argmax(s2)] - omh[i]) <= 1.5e-5


@pytest.mark.parametrize("name", STENCILS)
def test_kbc_rate_tends_to_exact_entropy_maximiser(name):
    """The closed form linearises the logarithm; the exact maximiser of
    -sum f' ln(f'/f^eq) differs from it by an amount that shrinks with the
    non-equilibrium amplitude."""
    lat = velocity_set(name)
    gaps = []
    for amp in (0.04, 0.004):
        f = _cells(lat, 8, 4, amp)
        ds, db, dh, feq, omh, _, _ = col.kbc_parts(lat, f, RATES)
        gap = 0.0
        for i in range(f.shape[1]):
            def neg_entropy(w):
                post = f[:, i] - RATES["omega"] * ds[:, i] - RATES["omega_bulk"] * db[:, i] - w * dh[:, i]
                return float((post * np.log(post / feq[:, i])).sum())
            res = minimize_scalar(neg_entropy, bounds=(omh[i] - 1.0, omh[i] + 1.0), method="bounded",
                                  options=dict(xatol=1e-12))
            gap = max(gap, abs(res.x - omh[i]))
        gaps.append(gap)
    assert gaps[0] < 0.05
    assert gaps[1] < gaps[0] / 5, gaps


@pytest.mark.parametrize("name", STENCILS)
def test_kbc_conserves(name):
    lat = velocity_set(name)
    f = _cells(lat, 30, 5, 0.05)
    F = _force(lat, 30, 6)
    c = lat.c.astype(float)
    for force in (None, F):
        out = col.kbc(lat, f, RATES, force)
        np.testing.assert_allclose(out.sum(axis=0), f.sum(axis=0), rtol=0, atol=1e-14)
        dj = c.T @ out - c.T @ f
        np.testing.assert_allclose(dj, 0 if force is None else force, rtol=0, atol=1e-14)


@pytest.mark.parametrize("name", STENCILS)
def test_kbc_higher_order_correction_is_bounded(name):
    """(omega_h - 1) dh is the E-projection of (1 - omega) ds + (1 - omega_b) db
    onto the line of dh, so by Cauchy-Schwarz its E-norm is at most
    |1 - omega| |ds|_E + |1 - omega_b| |db|_E, however small dh is.  (The
    operator has no limit as dh -> 0: the correction keeps this size and
    turns with the direction of dh.)"""
    lat = velocity_set(name)
    for amp in (0.05, 1e-6):
        f = _cells(lat, 50, 9, amp)
        ds, db, dh, feq, omh, _, _ = col.kbc_parts(lat, f, RATES)

        def norm_e(a):
            return np.sqrt((a * a / feq).sum(axis=0))

        lhs = norm_e((omh - 1.0) * dh)
        rhs = abs(1 - RATES["omega"]) * norm_e(ds) + abs(1 - RATES["omega_bulk"]) * norm_e(db)
        assert np.all(lhs <= rhs * (1 + 1e-12) + 1e-300)
        assert np.max(lhs / rhs) > 0.05   # and it is not negligible
