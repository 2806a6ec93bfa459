"""Pins of the oracle's lattice, equilibrium, forcing and moment bases
against what the paper and the mathematics fix (CPU only)."""

import itertools
from fractions import Fraction

import numpy as np
import pytest
import sympy as sp

from oracle import collision, equilibrium as eqm, lattice, moments
from tests.golden_tables import read_table, rho as s_rho, u0 as s_u0, u1 as s_u1, x as s_x, y as s_y

STENCILS = ["D2Q9", "D3Q19", "D3Q27"]


# ------------------------------------------------------------------ lattice
@pytest.mark.parametrize("name", STENCILS)
def test_isotropy_exact(name):
    """Standard weights: sum w = 1, sum w c = 0, sum w c_a c_b = c_s^2 delta,
    fourth moment = c_s^4 (dd + dd + dd), odd moments vanish (exact)."""
    lat = lattice.velocity_set(name)
    d = lat.d
    cs2 = lattice.CS2_EXACT
    assert sum(lat.wf) == 1
    for a in range(3):
        assert sum(w * int(c[a]) for w, c in zip(lat.wf, lat.c)) == 0
    for a, b in itertools.product(range(d), repeat=2):
        s = sum(w * int(c[a]) * int(c[b]) for w, c in zip(lat.wf, lat.c))
        assert s == (cs2 if a == b else 0)
    for a, b, g in itertools.product(range(d), repeat=3):
        assert sum(w * int(c[a] * c[b] * c[g]) for w, c in zip(lat.wf, lat.c)) == 0
    for a, b, g, e in itertools.product(range(d), repeat=4):
        s = sum(w * int(c[a] * c[b] * c[g] * c[e]) for w, c in zip(lat.wf, lat.c))
        dl = lambda i, j: 1 if i == j else 0
        assert s == cs2 * cs2 * (dl(a, b) * dl(g, e) + dl(a, g) * dl(b, e) + dl(a, e) * dl(b, g))


@pytest.mark.parametrize("name", STENCILS)
def test_opposites_and_sizes(name):
    lat = lattice.velocity_set(name)
    assert lat.Q == int(name.split("Q")[1])
    assert len({tuple(v) for v in lat.c}) == lat.Q
    for q in range(lat.Q):
        assert (lat.c[lat.opp[q]] == -lat.c[q]).all()


@pytest.mark.parametrize("name", ["D2Q9", "D3Q27"])
def test_product_weights(name):
    """D2Q9/D3Q27 weights are products of the 1-D weights (2/3, 1/6, 1/6)."""
    lat = lattice.velocity_set(name)
    w1 = {0: Fraction(2, 3), 1: Fraction(1, 6), -1: Fraction(1, 6)}
    for w, c in zip(lat.wf, lat.c):
        assert w == np.prod([w1[int(c[a])] for a in range(lat.d)])


# ------------------------------------------------------------- equilibrium
def _rand_state(rng, lat, n=7):
    rho = 1.0 + 0.1 * rng.standard_normal(n)
    u = 0.05 * rng.standard_normal((3, n))
    if lat.d == 2:
        u[2] = 0
    return rho, u


def test_equilibrium_matches_paper_trt_table():
    """The D2Q9 equilibrium moments printed in the paper's TRT table equal
    the raw moments of Eq. (3) (paper: identical on D2Q9)."""
    lat = lattice.velocity_set("D2Q9")
    rng = np.random.default_rng(11)
    rho, u = _rand_state(rng, lat)
    feq = eqm.equilibrium(lat, rho, u)
    for poly, eq_expr, _ in read_table("d2q9_trt_table.txt"):
        fpoly = sp.lambdify((s_x, s_y), poly)
        row = np.array([float(fpoly(int(c[0]), int(c[1]))) for c in lat.c])
        got = row @ feq
        want = sp.lambdify((s_rho, s_u0, s_u1), eq_expr)(rho, u[0], u[1]) * np.ones_like(rho)
        np.testing.assert_allclose(got, want, rtol=0, atol=1e-15)


def test_trt_table_rate_parity():
    """Paper's TRT table: omega_e on even-order, omega_o on odd-order moments."""
    for poly, _, r in read_table("d2q9_trt_table.txt"):
        order = sp.Poly(poly, s_x, s_y).total_degree()
        assert r == ("e" if order % 2 == 0 else "o")


@pytest.mark.parametrize("name", ["D2Q9", "D3Q27"])
def test_equilibrium_equals_truncated_maxwellian_exact(name):
    """On D2Q9 and D3Q27 every monomial moment of Eq. (3) equals the
    continuous Maxwellian moment truncated at O(u^2) (Eqs. 7-8), exactly."""
    lat = lattice.velocity_set(name)
    rho = Fraction(21, 20)
    u = [Fraction(3, 100), Fraction(-7, 100), Fraction(2, 50) if lat.d == 3 else Fraction(0)]
    cs2 = lattice.CS2_EXACT
    feq = []
    for w, c in zip(lat.wf, lat.c):
        cu = sum(int(c[a]) * u[a] for a in range(3))
        usq = sum(v * v for v in u)
        feq.append(w * rho + w * rho * (cu / cs2 + cu * cu / (2 * cs2 * cs2) - usq / (2 * cs2)))
    for e in moments.monomial_exponents(lat):
        m = sum(int(np.prod([int(c[a]) ** e[a] for a in range(3)])) * f for c, f in zip(lat.c, feq))
        assert m == eqm.gaussian_raw_moment(e, rho, u), e
    # float path of the oracle agrees with the exact rationals
    fl = eqm.equilibrium(lat, np.array([float(rho)]), np.array([[float(v)] for v in u]))
    np.testing.assert_allclose(fl[:, 0], [float(v) for v in feq], rtol=1e-15, atol=0)


@pytest.mark.parametrize("name", STENCILS)
def test_equilibrium_conserves(name):
    lat = lattice.velocity_set(name)
    rho, u = _rand_state(np.random.default_rng(3), lat)
    feq = eqm.equilibrium(lat, rho, u)
    r, j = eqm.density_momentum(lat, feq)
    np.testing.assert_allclose(r, rho, rtol=1e-15)
    np.testing.assert_allclose(j, rho * u, rtol=0, atol=1e-16)


@pytest.mark.parametrize("name", STENCILS)
def test_guo_source_moments(name):
    """Textbook moments of Guo's source: sum S = 0, sum c S = F,
    sum c_a c_b S = u_a F_b + F_a u_b."""
    lat = lattice.velocity_set(name)
    rng = np.random.default_rng(5)
    rho, u = _rand_state(rng, lat)
    F = 1e-3 * rng.standard_normal((3, u.shape[1]))
    if lat.d == 2:
        F[2] = 0
    S = eqm.guo_source(lat, u, F)
    c = lat.c.astype(float)
    np.testing.assert_allclose(S.sum(0), 0, atol=1e-18)
    np.testing.assert_allclose(c.T @ S, F, rtol=1e-13, atol=1e-19)
    for a, b in itertools.product(range(lat.d), repeat=2):
        np.testing.assert_allclose((c[:, a] * c[:, b]) @ S, u[a] * F[b] + F[a] * u[b], rtol=1e-12, atol=1e-19)


# ----------------------------------------------------------------- moments
def test_monomial_counts():
    """D3Q19 keeps 19 of the 27 monomials (8 zero rows dropped); the others
    keep all; every monomial matrix is invertible."""
    for name, n in (("D2Q9", 9), ("D3Q19", 19), ("D3Q27", 27)):
        lat = lattice.velocity_set(name)
        M, exps = moments.raw_moment_matrix(lat)
        assert len(exps) == n
        assert abs(np.linalg.det(M)) > 1e-6
    lat = lattice.velocity_set("D3Q19")
    exps = moments.monomial_exponents(lat)
    dropped = {e for e in itertools.product(range(3), repeat=3)} - set(exps)
    assert (1, 1, 1) in dropped and (2, 1, 1) in dropped and len(dropped) == 8


def test_gram_schmidt_reproduces_paper_mrt_table():
    """Weighted Gram-Schmidt of the split D2Q9 monomials gives, up to scale,
    the nine polynomials printed in the paper's MRT table, in the same rate
    groups, and the incompressible equilibrium moments of that table."""
    lat = lattice.velocity_set("D2Q9")
    M, groups, rows = moments.orthogonal_mrt_basis(lat)
    table = read_table("d2q9_mrt_table.txt")
    used = set()
    rng = np.random.default_rng(2)
    rho, u = _rand_state(rng, lat, n=3)
    feq = eqm.equilibrium(lat, rho, u, rho0=1.0, compressible=False)
    group_map = {"c": ("o0", "o1")}
    for poly, eq_expr, grp in table:
        fpoly = sp.lambdify((s_x, s_y), poly)
        vec = [sp.Rational(fpoly(int(c[0]), int(c[1]))) for c in lat.c]
        match = None
        for k, r in enumerate(rows):
            ratio = None
            ok = True
            for a, b in zip(vec, r):
                b = sp.Rational(b.numerator, b.denominator)
                if a == 0 and b == 0:
                    continue
                if a == 0 or b == 0:
                    ok = False
                    break
                ratio = b / a if ratio is None else ratio
                if b / a != ratio:
                    ok = False
                    break
            if ok:
                match = k
                break
        assert match is not None, poly
        used.add(match)
        assert groups[match] in group_map.get(grp, (grp,))
        want = sp.lambdify((s_rho, s_u0, s_u1), eq_expr)(rho, u[0], u[1]) * np.ones_like(rho)
        np.testing.assert_allclose(np.array(vec, dtype=float) @ feq, want, atol=1e-15)
    assert len(used) == 9


@pytest.mark.parametrize("name", STENCILS)
def test_basis_weighted_orthogonal(name):
    """Rows are w-orthogonal: M W M^T is diagonal."""
    lat = lattice.velocity_set(name)
    M, groups, rows = moments.orthogonal_mrt_basis(lat)
    for i, j in itertools.combinations(range(lat.Q), 2):
        assert sum(w * a * b for w, a, b in zip(lat.wf, rows[i], rows[j])) == 0
    assert groups.count("bulk") == 1
    assert groups.count("shear") == (2 if lat.d == 2 else 5)


# --------------------------------------------------------------- operators
def _random_pdfs(lat, n, rng, scale=0.02):
    rho, u = _rand_state(rng, lat, n)
    f = eqm.equilibrium(lat, rho, u) * (1.0 + scale * rng.standard_normal((lat.Q, n)))
    return f


RATES = dict(omega=1.25, omega_bulk=1.4, omega_odd=0.0, magic=3.0 / 16.0,
             omega_hi=(1.1, 0.9, 1.3, 1.7))


@pytest.mark.parametrize("name", STENCILS)
@pytest.mark.parametrize("method", ["SRT", "TRT", "MRT"])
def test_collision_conserves(name, method):
    lat = lattice.velocity_set(name)
    rng = np.random.default_rng(7)
    f = _random_pdfs(lat, 11, rng)
    F = 1e-4 * rng.standard_normal((3, 11))
    if lat.d == 2:
        F[2] = 0
    for force in (None, F):
        out = collision.collide(method, lat, f, RATES, force)
        r0, j0 = eqm.density_momentum(lat, f)
        r1, j1 = eqm.density_momentum(lat, out)
        np.testing.assert_allclose(r1, r0, rtol=4e-16 * lat.Q)
        jf = j0 if force is None else j0 + force
        np.testing.assert_allclose(j1, jf, rtol=0, atol=1e-15)


@pytest.mark.parametrize("name", STENCILS)
def test_mrt_all_rates_equal_is_srt(name):
    """With every group at the same rate, Eq. (4) reduces to Eq. (1)."""
    lat = lattice.velocity_set(name)
    rng = np.random.default_rng(8)
    f = _random_pdfs(lat, 9, rng)
    F = 1e-4 * rng.standard_normal((3, 9))
    if lat.d == 2:
        F[2] = 0
    r = dict(RATES, omega=1.37, omega_bulk=1.37, omega_hi=(1.37,) * 4)
    for force in (None, F):
        for comp in (True, False):
            a = collision.mrt(lat, f, r, force, compressible=comp)
            b = collision.srt(lat, f, r, force, compressible=comp)
            np.testing.assert_allclose(a, b, rtol=0, atol=2e-15)


@pytest.mark.parametrize("name", STENCILS)
def test_mrt_even_odd_rates_is_trt(name):
    """Pins which moment order each higher-order rate acts on: MRT with the
    even rate on the shear, bulk, order-4 and order-6 groups and the odd rate
    on orders 3 and 5 is TRT(even, odd) (Sec. III-C "SRT, TRT" and "MRT":
    even-order polynomials are symmetric in c, odd-order ones antisymmetric,
    and the weighted Gram-Schmidt never mixes the two).  Negative control:
    the order-3 and order-4 rates swapped is not TRT."""
    lat = lattice.velocity_set(name)
    rng = np.random.default_rng(18)
    f = _random_pdfs(lat, 11, rng)
    F = 1e-4 * rng.standard_normal((3, 11))
    if lat.d == 2:
        F[2] = 0
    we, wo = 1.37, 1.81
    trt = dict(RATES, omega=we, omega_odd=wo)
    mrt = dict(RATES, omega=we, omega_bulk=we, omega_hi=(wo, we, wo, we))
    for force in (None, F):
        a = collision.mrt(lat, f, mrt, force)
        b = collision.trt(lat, f, trt, force)
        np.testing.assert_allclose(a, b, rtol=0, atol=2e-15)
    swapped = dict(mrt, omega_hi=(we, wo, wo, we))
    assert np.max(np.abs(collision.mrt(lat, f, swapped) - collision.trt(lat, f, trt))) > 1e-6


@pytest.mark.parametrize("name", ["D2Q9", "D3Q27"])
def test_trt_population_form_equals_paper_moment_form(name):
    """The +/- population TRT equals the paper's TRT built from raw
    monomial moments with Maxwellian equilibrium moments (D2Q9, D3Q27)."""
    lat = lattice.velocity_set(name)
    f = _random_pdfs(lat, 13, np.random.default_rng(9))
    for r in (RATES, dict(RATES, omega=0.6, omega_odd=1.7)):
        a = collision.trt(lat, f, r)
        b = collision.trt_moment_form(lat, f, r)
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-14)


def test_trt_magic_parameter():
    r = dict(omega=1.0 / 0.8, magic=3.0 / 16.0, omega_odd=0.0)
    wo = collision.trt_odd_rate(r)
    assert abs((1 / r["omega"] - 0.5) * (1 / wo - 0.5) - 3.0 / 16.0) < 1e-15
    assert abs(1 / wo - 1.125) < 1e-14


# -------------------------------------------------------------- Smagorinsky
@pytest.mark.parametrize("name", STENCILS)
def test_smagorinsky_rate_solves_paper_equations(name):
    """The local rate satisfies the paper's Eq. (14) with |S| from Eq. (12)
    (both written out here separately) for random non-equilibrium states."""
    lat = lattice.velocity_set(name)
    rng = np.random.default_rng(12)
    f = _random_pdfs(lat, 50, rng, scale=0.05)
    rho, u = eqm.macroscopic(lat, f)
    feq = eqm.equilibrium(lat, rho, u)
    cs, om0 = 0.17, 1.0 / 0.52
    om = collision.smagorinsky_rate(lat, f, feq, rho, om0, cs)
    c = lat.c.astype(float)
    Pi = np.einsum("qa,qb,qn->abn", c, c, f - feq)
    S = -3.0 * om / (2.0 * rho) * Pi                      # Eq. (12)
    Snorm = np.sqrt(2.0 * (S * S).sum(axis=(0, 1)))
    nu0 = (1.0 / om0 - 0.5) / 3.0
    np.testing.assert_allclose(om, 2.0 / (6.0 * cs * cs * Snorm + 6.0 * nu0 + 1.0), rtol=1e-13)   # Eq. (14)
    assert np.all(om < om0) and np.all(om > 0)


@pytest.mark.parametrize("name,method", [("D2Q9", "SRT"), ("D3Q19", "SRT"), ("D3Q19", "MRT"), ("D3Q27", "MRT")])
def test_smagorinsky_zero_constant_and_conservation(name, method):
    lat = lattice.velocity_set(name)
    rng = np.random.default_rng(13)
    f = _random_pdfs(lat, 9, rng, scale=0.05)
    F = 1e-4 * rng.standard_normal((3, 9))
    if lat.d == 2:
        F[2] = 0
    base = collision.collide(method, lat, f, RATES, F)
    np.testing.assert_array_equal(collision.collide(method, lat, f, dict(RATES, cs_smag=0.0), F), base)
    out = collision.collide(method, lat, f, dict(RATES, cs_smag=0.2), F)
    r0, j0 = eqm.density_momentum(lat, f)
    r1, j1 = eqm.density_momentum(lat, out)
    np.testing.assert_allclose(r1, r0, rtol=1e-14)
    np.testing.assert_allclose(j1, j0 + F, atol=1e-15)
    assert np.max(np.abs(out - base)) > 1e-6      # the model changes the result
