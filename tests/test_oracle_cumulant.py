"""Pin of the oracle's cumulant operator against an exact-rational brute
force of the paper's definition (Eq. 9: cumulants are derivatives of
K(xi) = ln sum f exp(c.xi) at xi = 0), computed here with truncated power
series and an exact linear solve; plus the closed-form product equilibrium."""

import math
from fractions import Fraction

import numpy as np
import pytest
import sympy as sp

from oracle import collision, equilibrium as eqm, lattice, moments


# ---- truncated multivariate power series in xi with exact coefficients ----
def _mul(a, b, d):
    out = {}
    for ea, ca in a.items():
        for eb, cb in b.items():
            e = tuple(x + y for x, y in zip(ea, eb))
            if max(e) > 2:
                continue            # only exponents <= 2 per variable are needed
            out[e] = out.get(e, 0) + ca * cb
    return out


def _add(a, b, s=1):
    out = dict(a)
    for e, c in b.items():
        out[e] = out.get(e, 0) + s * c
    return out


def _scale(a, s):
    return {e: c * s for e, c in a.items()}


def _series_log1p(X, d, nmax):
    out, P = {}, {(0,) * 3: Fraction(1)}
    for n in range(1, nmax + 1):
        P = _mul(P, X, d)
        out = _add(out, _scale(P, Fraction((-1) ** (n + 1), n)))
    return out


def _series_exp(Y, nmax):
    out, P = {(0,) * 3: Fraction(1)}, {(0,) * 3: Fraction(1)}
    for n in range(1, nmax + 1):
        P = _mul(P, Y, 3)
        out = _add(out, _scale(P, Fraction(1, math.factorial(n))))
    return out


def _fact(e):
    return math.factorial(e[0]) * math.factorial(e[1]) * math.factorial(e[2])


def brute_force_cumulant(lat, f, om_s, om_b, hi):
    """Exact-rational cumulant collision of one cell."""
    cs2 = lattice.CS2_EXACT
    d = lat.d
    # moment generating function, each exp(c xi) truncated per variable
    Mser = {}
    for fq, c in zip(f, lat.c):
        term = {(0, 0, 0): fq}
        for a in range(3):
            ca = int(c[a])
            fac = {(0, 0, 0): Fraction(1)}
            if ca != 0:
                e1 = [0, 0, 0]; e1[a] = 1
                e2 = [0, 0, 0]; e2[a] = 2
                fac[tuple(e1)] = Fraction(ca)
                fac[tuple(e2)] = Fraction(ca * ca, 2)
            term = _mul(term, fac, 3)
        Mser = _add(Mser, term)
    rho = Mser[(0, 0, 0)]
    X = {e: c / rho for e, c in Mser.items() if e != (0, 0, 0)}
    K = _series_log1p(X, 3, 2 * d)
    exps = moments.monomial_exponents(lat)
    kap = {e: K.get(e, 0) * _fact(e) for e in exps if sum(e) > 0}
    diag = [e for e in exps if sum(e) == 2 and max(e) == 2]
    tr = sum(kap[e] for e in diag)
    tr_post = tr + om_b * (d * cs2 - tr)
    post = {}
    for e in kap:
        n = sum(e)
        if n == 1:
            post[e] = kap[e]
        elif n == 2 and max(e) == 1:
            post[e] = kap[e] * (1 - om_s)
        elif n == 2:
            post[e] = (1 - om_s) * (kap[e] - tr / d) + tr_post / d
        else:
            post[e] = kap[e] * (1 - hi[n - 3])
    Y = {e: c / _fact(e) for e, c in post.items()}
    E = _series_exp(Y, 2 * d)
    m = [rho * E.get(e, 0) * _fact(e) if sum(e) else rho for e in exps]
    Mmat = sp.Matrix([[sp.Rational(int(np.prod([int(c[a]) ** e[a] for a in range(3)])))
                       for c in lat.c] for e in exps])
    sol = Mmat.LUsolve(sp.Matrix([sp.Rational(v.numerator, v.denominator) for v in m]))
    return [Fraction(int(s.p), int(s.q)) for s in sol]


def _rational_cell(lat, seed):
    rng = np.random.default_rng(seed)
    return [w * (1 + Fraction(int(rng.integers(-40, 41)), 1000)) for w in lat.wf]


@pytest.mark.parametrize("name", ["D2Q9", "D3Q27"])
@pytest.mark.parametrize("hi", [(1, 1, 1, 1), (Fraction(3, 2), Fraction(6, 5), Fraction(4, 5), Fraction(1, 2))])
def test_cumulant_matches_exact_series(name, hi):
    lat = lattice.velocity_set(name)
    om_s, om_b = Fraction(20, 11), Fraction(6, 5)
    for seed in (1, 2):
        f = _rational_cell(lat, seed)
        want = brute_force_cumulant(lat, f, om_s, om_b, hi)
        rates = dict(omega=float(om_s), omega_bulk=float(om_b), omega_hi=tuple(float(h) for h in hi))
        got = collision.cumulant(lat, np.array([[float(v)] for v in f]), rates)[:, 0]
        np.testing.assert_allclose(got, [float(v) for v in want], rtol=1e-13, atol=1e-16)


@pytest.mark.parametrize("name", ["D2Q9", "D3Q27"])
def test_cumulant_all_rates_one_is_product_equilibrium(name):
    """All rates 1: the post-collision state is the factorised equilibrium
    rho prod_a phi(c_a; u_a), phi(0) = 1 - c_s^2 - u^2,
    phi(+-1) = (c_s^2 + u^2 +- u)/2."""
    lat = lattice.velocity_set(name)
    rng = np.random.default_rng(4)
    rho = 1 + 0.05 * rng.standard_normal(6)
    u = 0.05 * rng.standard_normal((3, 6))
    if lat.d == 2:
        u[2] = 0
    f = eqm.equilibrium(lat, rho, u) * (1 + 0.03 * rng.standard_normal((lat.Q, 6)))
    r, j = eqm.density_momentum(lat, f)
    uu = j / r
    cs2 = 1.0 / 3.0
    phi = {0: lambda v: 1 - cs2 - v * v, 1: lambda v: (cs2 + v * v + v) / 2, -1: lambda v: (cs2 + v * v - v) / 2}
    want = np.array([r * np.prod([phi[int(c[a])](uu[a]) for a in range(lat.d)], axis=0) for c in lat.c])
    got = collision.cumulant(lat, f, dict(omega=1.0, omega_bulk=1.0, omega_hi=(1.0,) * 4))
    np.testing.assert_allclose(got, want, rtol=1e-13, atol=1e-16)


@pytest.mark.parametrize("name", ["D2Q9", "D3Q27"])
def test_cumulant_conserves(name):
    lat = lattice.velocity_set(name)
    rng = np.random.default_rng(6)
    rho = 1 + 0.05 * rng.standard_normal(8)
    u = 0.05 * rng.standard_normal((3, 8))
    if lat.d == 2:
        u[2] = 0
    f = eqm.equilibrium(lat, rho, u) * (1 + 0.03 * rng.standard_normal((lat.Q, 8)))
    out = collision.cumulant(lat, f, dict(omega=1.7, omega_bulk=1.1, omega_hi=(0.8, 1.2, 1.0, 1.4)))
    r0, j0 = eqm.density_momentum(lat, f)
    r1, j1 = eqm.density_momentum(lat, out)
    np.testing.assert_allclose(r1, r0, rtol=1e-14)
    np.testing.assert_allclose(j1, j0, atol=1e-15)
