"""Pins of the C++17 / OpenMP FP64 oracle (``oracle/lbm_oracle.cpp``), CPU only.

The C++ oracle is a second implementation of the forward path written
independently of the numpy oracle (its own lattice tables, Gram-Schmidt in
double, the closed-form inverse of the weighted-orthogonal basis, cumulants
from restricted-growth-string set partitions, the per-axis inverse of the
moment map).  It is pinned two ways: element-wise equality with the numpy
oracle on ragged lattices with walls, forces and moving walls, and the
physical closed forms and invariants the method fixes, evaluated on the C++
oracle itself."""

import math

import numpy as np
import pytest

from oracle import cpu, run as orun
from paper_2001_11806_amd import inputs
from tests.golden_tables import read_table, x as s_x, y as s_y

CS2 = 1.0 / 3.0
RATES = dict(omega=1 / 0.8, omega_bulk=1.2, omega_odd=0.0, magic=3 / 16, omega_hi=(1.0, 1.0, 1.0, 1.0))
GEN = dict(RATES, omega_bulk=1.3, omega_hi=(1.1, 1.2, 0.9, 1.3))

CASES = [(s, m) for s in ("D2Q9", "D3Q19", "D3Q27") for m in ("SRT", "TRT", "MRT", "CUMULANT")
         if not (m == "CUMULANT" and s == "D3Q19")]


def _fields(stencil, dims, seed, with_mask=True, amp=2e-2):
    nx, ny, nz = dims
    rng = np.random.default_rng(seed)
    mask = None
    if with_mask:
        mask = (rng.random((nz, ny, nx)) < 0.12).astype(np.uint8)
        mask[:, 0, :] = 1
    rho = 1.0 + 0.01 * rng.uniform(-1, 1, (nz, ny, nx))
    u = inputs.uniform_noise_velocity(dims, amp, seed + 100, mask)
    if stencil == "D2Q9":
        u[2] = 0
    return mask, rho, u


@pytest.mark.parametrize("storage", ["f64", "f32", "bf16", "f16"])
@pytest.mark.parametrize("stencil,method", CASES)
def test_cpp_equals_numpy_oracle(stencil, method, storage):
    """Five steps on a ragged lattice (walls, random solid cells, a per-row
    force profile) from the same initial state: the two oracles agree to
    1e-14 in every stored value and readout, the totals to 1e-13.  The cumulant case runs
    general higher-order rates, no walls and no force (the operator is
    defined for periodic, unforced lattices here)."""
    dims = (23, 7, 1) if stencil == "D2Q9" else (23, 7, 5)
    cum = method == "CUMULANT"
    mask, rho, u = _fields(stencil, dims, 5, with_mask=not cum)
    rates = GEN if cum else RATES
    prof = None
    if not cum:
        prof = np.stack([2e-4 * np.sin(np.arange(dims[1])), -1e-4 * np.ones(dims[1]),
                         np.zeros(dims[1]) if stencil == "D2Q9" else 5e-5 * np.cos(np.arange(dims[1]))], axis=1)
    cfg = orun.Config(stencil, method, rates, storage=storage)
    P0 = orun.init_equilibrium(cfg, rho, u, mask)
    np.testing.assert_array_equal(cpu.init_equilibrium(cfg, rho, u, mask), P0)
    Ff = orun.force_field(prof, dims) if prof is not None else None
    want = orun.run(cfg, P0, 5, mask, Ff)
    got = cpu.run(cfg, P0, 5, mask, prof)
    assert np.max(np.abs(got - want)) <= 1e-14
    r1, u1 = orun.readout(cfg, want, mask, Ff)
    r2, u2 = cpu.readout(cfg, got, mask, prof)
    assert np.max(np.abs(r1 - r2)) <= 1e-14 and np.max(np.abs(u1 - u2)) <= 1e-14
    c1, c2 = orun.conserved(cfg, want, mask), cpu.conserved(cfg, got, mask)
    # totals of N*Q values summed in another order: within N*Q rounding units
    assert np.max(np.abs(c1 - c2)) <= 1e-13 * np.abs(c1).max()


@pytest.mark.parametrize("method", ["SRT", "TRT", "MRT"])
def test_cpp_equals_numpy_oracle_moving_walls(method):
    """Velocity bounce-back from two moving wall types and a resting wall."""
    dims = (17, 9, 4)
    mask, rho, u = _fields("D3Q19", dims, 8)
    rng = np.random.default_rng(9)
    solid = np.nonzero(mask.reshape(-1))[0]
    mask.reshape(-1)[rng.choice(solid, solid.size // 2, replace=False)] = rng.integers(2, 4, solid.size // 2)
    table = np.zeros((4, 3))
    table[2] = (1e-2, -5e-3, 2e-3)
    table[3] = (-3e-3, 0.0, 7e-3)
    cfg = orun.Config("D3Q19", method, RATES)
    P0 = orun.init_equilibrium(cfg, rho, u, mask)
    want = orun.run(cfg, P0, 4, mask, None, table)
    got = cpu.run(cfg, P0, 4, mask, None, table)
    assert np.max(np.abs(got - want)) <= 1e-14


# ------------------------------------------------------------------ closed forms on the C++ oracle
@pytest.mark.parametrize("stencil,method", CASES)
def test_cpp_collision_conserves_mass_and_momentum(stencil, method):
    """Each collision keeps rho and gains exactly F of momentum (Guo)."""
    cfg = orun.Config(stencil, method, GEN if method == "CUMULANT" else RATES)
    rng = np.random.default_rng(3)
    g = cfg.lat.w[:, None] * (1 + 0.05 * rng.standard_normal((cfg.lat.Q, 200)))
    F = None if method == "CUMULANT" else np.array([1e-4, -2e-4, 0.0 if stencil == "D2Q9" else 3e-4])
    out = cpu.collide_cells(cfg, g, F)
    c = cfg.lat.c.astype(float)
    # a few ulp of the O(1) sums
    np.testing.assert_allclose(out.sum(0), g.sum(0), rtol=0, atol=2e-15)
    gain = c.T @ out - c.T @ g
    want = np.zeros((3, 1)) if F is None else F.reshape(3, 1)
    np.testing.assert_allclose(gain, np.broadcast_to(want, gain.shape), rtol=0, atol=2e-15)


@pytest.mark.parametrize("stencil", ["D2Q9", "D3Q27"])
def test_cpp_cumulant_unit_rates_give_product_equilibrium(stencil):
    """With every relaxation rate 1 the post-collision cumulants are the
    Maxwellian ones (u, c_s^2, 0), whose populations are the product form
    rho prod_a phi(c_a; u_a), phi(0) = 1 - c_s^2 - u^2,
    phi(+-1) = (c_s^2 + u^2 +- u) / 2."""
    cfg = orun.Config(stencil, "CUMULANT", dict(omega=1.0, omega_bulk=1.0, omega_hi=(1.0,) * 4))
    rng = np.random.default_rng(7)
    g = cfg.lat.w[:, None] * (1 + 0.1 * rng.standard_normal((cfg.lat.Q, 50)))
    out = cpu.collide_cells(cfg, g)
    c = cfg.lat.c.astype(float)
    rho = g.sum(0)
    u = (c.T @ g) / rho
    want = np.ones_like(g) * rho
    for a in range(3 if stencil == "D3Q27" else 2):
        ca = c[:, a][:, None]
        ua = u[a][None, :]
        phi = np.where(ca == 0, 1 - CS2 - ua * ua, 0.5 * (CS2 + ua * ua + ca * ua))
        want = want * phi
    np.testing.assert_allclose(out, want, rtol=0, atol=1e-15)


def test_cpp_cumulants_of_a_product_distribution_vanish():
    """A distribution whose three axes are independent three-point laws has
    zero mixed cumulants, and on D3Q27 every cumulant of order >= 3 is mixed
    (exponents are at most 2 per axis).  With shear and bulk rates 1 the
    collision therefore returns the Gaussian product equilibrium whatever the
    higher-order rates: a wrong sign, coefficient or block in the partition
    sums leaves a non-zero higher-order cumulant that the non-unit rates
    would carry into the result."""
    cfg = orun.Config("D3Q27", "CUMULANT", dict(omega=1.0, omega_bulk=1.0, omega_hi=(1.7, 0.3, 1.9, 0.6)))
    rng = np.random.default_rng(2)
    c = cfg.lat.c
    cols = []
    for _ in range(20):
        ax = [rng.uniform(0.2, 0.5, 3) for _ in range(3)]
        cols.append([ax[0][c[q, 0] + 1] * ax[1][c[q, 1] + 1] * ax[2][c[q, 2] + 1] for q in range(27)])
    g = np.array(cols).T
    out = cpu.collide_cells(cfg, g)
    rho = g.sum(0)
    u = (c.T.astype(float) @ g) / rho
    want = np.ones_like(g) * rho
    for a in range(3):
        ca = c[:, a][:, None].astype(float)
        phi = np.where(ca == 0, 1 - CS2 - u[a] ** 2, 0.5 * (CS2 + u[a] ** 2 + ca * u[a]))
        want = want * phi
    np.testing.assert_allclose(out, want, rtol=0, atol=2e-15)
    # negative control: a non-product input carries mixed cumulants, which the
    # non-unit higher-order rates leave partly in place
    g2 = g * (1 + 0.05 * rng.standard_normal(g.shape))
    out2 = cpu.collide_cells(cfg, g2)
    rho2 = g2.sum(0)
    u2 = (c.T.astype(float) @ g2) / rho2
    want2 = np.ones_like(g2) * rho2
    for a in range(3):
        ca = c[:, a][:, None].astype(float)
        want2 = want2 * np.where(ca == 0, 1 - CS2 - u2[a] ** 2, 0.5 * (CS2 + u2[a] ** 2 + ca * u2[a]))
    assert np.max(np.abs(out2 - want2)) > 1e-5


def test_cpp_mrt_basis_reproduces_paper_d2q9_table():
    """The C++ Gram-Schmidt on D2Q9 gives the paper's weighted-orthogonal
    polynomials (Sec. III-C "MRT" table) up to scale, with their rate groups."""
    cfg = orun.Config("D2Q9", "MRT", dict(RATES, omega=1.1, omega_bulk=1.2, omega_hi=(1.3, 1.4, 1.0, 1.0)))
    M, s = cpu.mrt_basis(cfg)
    rows = read_table("d2q9_mrt_table.txt")
    c = cfg.lat.c
    group_rate = {"c": 0.0, "shear": 1.1, "bulk": 1.2, "o3": 1.3, "o4": 1.4}
    assert len(rows) == 9
    used = set()
    for poly, _, grp in rows:
        vals = np.array([float(poly.subs({s_x: int(c[q, 0]), s_y: int(c[q, 1])})) for q in range(9)])
        match = [k for k in range(9)
                 if np.allclose(M[k] * (vals @ M[k]) / (M[k] @ M[k]), vals, atol=1e-13)]
        assert len(match) == 1, (poly, match)
        assert s[match[0]] == group_rate[grp]
        used.add(match[0])
    assert used == set(range(9))


@pytest.mark.parametrize("stencil", ["D2Q9", "D3Q19", "D3Q27"])
def test_cpp_mrt_basis_weighted_orthogonal_and_equal_rates_give_srt(stencil):
    cfg = orun.Config(stencil, "MRT", dict(RATES, omega=1.3, omega_bulk=1.3, omega_hi=(1.3,) * 4))
    M, _ = cpu.mrt_basis(cfg)
    G = (M * cfg.lat.w[None, :]) @ M.T
    off = G - np.diag(np.diag(G))
    assert np.max(np.abs(off)) < 1e-13 * np.max(np.abs(G))
    rng = np.random.default_rng(11)
    g = cfg.lat.w[:, None] * (1 + 0.05 * rng.standard_normal((cfg.lat.Q, 40)))
    F = np.array([1e-4, 2e-4, 0.0 if stencil == "D2Q9" else -1e-4])
    srt = orun.Config(stencil, "SRT", dict(omega=1.3))
    np.testing.assert_allclose(cpu.collide_cells(cfg, g, F), cpu.collide_cells(srt, g, F), rtol=0, atol=1e-15)


@pytest.mark.parametrize("stencil", ["D2Q9", "D3Q19", "D3Q27"])
def test_cpp_mrt_even_odd_rates_is_trt(stencil):
    """MRT with the even rate on shear, bulk, orders 4 and 6 and the odd rate
    on orders 3 and 5 equals TRT(even, odd) (Sec. III-C "SRT, TRT", "MRT"):
    pins the C++ oracle's mapping of the higher-order rates to moment orders.
    Negative control: order-3 and order-4 rates swapped."""
    we, wo = 1.37, 1.81
    mrt = orun.Config(stencil, "MRT", dict(RATES, omega=we, omega_bulk=we, omega_hi=(wo, we, wo, we)))
    trt = orun.Config(stencil, "TRT", dict(RATES, omega=we, omega_odd=wo))
    rng = np.random.default_rng(19)
    g = mrt.lat.w[:, None] * (1 + 0.05 * rng.standard_normal((mrt.lat.Q, 40)))
    F = np.array([1e-4, 2e-4, 0.0 if stencil == "D2Q9" else -1e-4])
    np.testing.assert_allclose(cpu.collide_cells(mrt, g, F), cpu.collide_cells(trt, g, F), rtol=0, atol=2e-15)
    bad = orun.Config(stencil, "MRT", dict(RATES, omega=we, omega_bulk=we, omega_hi=(we, wo, wo, we)))
    assert np.max(np.abs(cpu.collide_cells(bad, g, F) - cpu.collide_cells(trt, g, F))) > 1e-6


def test_cpp_poiseuille_trt_magic_exact_and_srt_slip():
    """Steady Poiseuille between halfway walls: exact with TRT, Lambda = 3/16
    (Ginzburg's result); SRT at tau = 0.8 slips (negative control)."""
    H, F = 16, 1e-5
    ny = H + 2
    mask = inputs.channel_mask(1, ny, 1)
    y = np.arange(1, H + 1)
    nu = CS2 * (0.8 - 0.5)
    exact = F / (2 * nu) * (y - 0.5) * (H + 0.5 - y)
    errs = {}
    for method in ("TRT", "SRT"):
        cfg = orun.Config("D3Q19", method, dict(omega=1 / 0.8, magic=3 / 16, omega_odd=0.0))
        P = cpu.init_equilibrium(cfg, None, np.zeros((3, 1, ny, 1)), mask)
        P = cpu.run(cfg, P, 8000, mask, [F, 0, 0], threads=1)
        _, u = cpu.readout(cfg, P, mask, [F, 0, 0])
        errs[method] = np.max(np.abs(u[0, 0, 1:H + 1, 0] / exact - 1))
    assert errs["TRT"] < 1e-9
    assert errs["SRT"] > 1e-4


@pytest.mark.parametrize("stencil,method", [("D3Q19", "SRT"), ("D3Q19", "TRT"), ("D3Q27", "MRT"),
                                            ("D3Q27", "CUMULANT"), ("D2Q9", "MRT"), ("D2Q9", "CUMULANT")])
def test_cpp_shear_wave_viscosity(stencil, method):
    """u_y = A sin(k x) decays as exp(-nu k^2 t), nu = c_s^2 (1/omega - 1/2)."""
    n, T, A = 96, 300, 1e-6
    om = 1.0 / 0.7
    cfg = orun.Config(stencil, method, dict(omega=om, omega_bulk=1.1, omega_odd=0.0, magic=3 / 16,
                                            omega_hi=(1.0,) * 4))
    x = np.arange(n)
    u = np.zeros((3, 1, 1, n))
    k = 2 * np.pi / n
    u[1, 0, 0] = A * np.sin(k * x)
    P = cpu.init_equilibrium(cfg, None, u)
    P = cpu.run(cfg, P, T, threads=1)
    _, uu = cpu.readout(cfg, P)
    amp = 2 * (uu[1, 0, 0] * np.sin(k * x)).mean()
    nu = CS2 * (1 / om - 0.5)
    assert abs(-math.log(amp / A) / (k * k * T) / nu - 1) < 5e-3


def test_cpp_taylor_green_c1():
    """C1 on the C++ oracle: D2Q9 SRT tau 0.8, 64^2, 1000 steps: energy
    ratio within the O(k^2) error of exp(-2 nu |k|^2 t), mass to roundoff."""
    n, tau, T = 64, 0.8, 1000
    cfg = orun.Config("D2Q9", "SRT", dict(omega=1 / tau))
    rho, u = inputs.taylor_green_2d(n, 0.01)
    P = cpu.init_equilibrium(cfg, rho, u)
    m0 = cpu.conserved(cfg, P)[0]

    def energy(P):
        r, uu = cpu.readout(cfg, P)
        return float((r * (uu ** 2).sum(0)).sum())
    E0 = energy(P)
    P = cpu.run(cfg, P, T)
    k = 2 * np.pi / n
    nu = CS2 * (tau - 0.5)
    assert abs(energy(P) / E0 / np.exp(-2 * nu * 2 * k * k * T) - 1) < 2e-2
    assert abs(cpu.conserved(cfg, P)[0] / m0 - 1) < 1e-13


@pytest.mark.parametrize("method", ["SRT", "TRT"])
def test_cpp_couette_moving_wall_exact(method):
    """A lid at y = H + 0.5 moving with U over a resting wall at y = 0.5:
    the steady profile is u_x = U (y - 0.5) / H exactly."""
    H, U = 12, 0.01
    ny = H + 2
    cfg = orun.Config("D3Q19", method, dict(omega=1 / 0.8, magic=3 / 16, omega_odd=0.0))
    mask = inputs.channel_mask(1, ny, 1)
    mask[:, ny - 1, :] = 2
    table = np.zeros((3, 3))
    table[2] = (U, 0.0, 0.0)
    P = cpu.init_equilibrium(cfg, None, np.zeros((3, 1, ny, 1)), mask)
    P = cpu.run(cfg, P, 6000, mask, None, table, threads=1)
    _, u = cpu.readout(cfg, P, mask)
    y = np.arange(1, H + 1)
    np.testing.assert_allclose(u[0, 0, 1:H + 1, 0], U * (y - 0.5) / H, rtol=1e-9, atol=1e-14)


def test_cpp_storage_rounding_matches_numpy_casts():
    """Emulated FP32 / FP16 rounding of the shifted values equals numpy's
    IEEE casts, BF16 the bit-level round-to-nearest-even (one step from a
    state whose deviations span many binades, ties included)."""
    rng = np.random.default_rng(12)
    u = rng.uniform(-0.05, 0.05, (3, 4, 4, 64)) * 10.0 ** rng.integers(-6, 0, (3, 4, 4, 64))
    for storage in ("f32", "f16", "bf16"):
        cfg = orun.Config("D3Q19", "SRT", dict(omega=1.0), storage=storage)
        P = cpu.init_equilibrium(cfg, None, u)
        dev = P - cfg.lat.w.reshape(-1, 1, 1, 1)
        np.testing.assert_array_equal(dev, orun.round_storage(dev, storage))
        P64 = orun.init_equilibrium(orun.Config("D3Q19", "SRT", dict(omega=1.0)), np.ones(u.shape[1:]), u)
        np.testing.assert_array_equal(P, orun.quantize(cfg, P64))


@pytest.mark.parametrize("stencil,method", CASES)
def test_cpp_long_double_build_is_the_same_method(stencil, method):
    """The long double build (the reference of the FP64 GPU parity tests) is
    the same method: from the same rounded FP64 state, five steps agree with
    the FP64 build to the FP64 rounding of the state (1e-14), and with the
    numpy oracle run on np.longdouble arrays (exact-rational weights) to
    1e-16, well below FP64 rounding.  (The numpy run keeps c_s^2 as the
    float64 1/3, a 2e-17 relative difference.)"""
    dims = (23, 7, 1) if stencil == "D2Q9" else (23, 7, 5)
    cum = method == "CUMULANT"
    mask, rho, u = _fields(stencil, dims, 7, with_mask=not cum)
    rates = GEN if cum else RATES
    F = None if cum else np.array([2e-4, -1e-4, 0.0 if stencil == "D2Q9" else 5e-5])
    cfg = orun.Config(stencil, method, rates)
    P0 = cpu.init_equilibrium(cfg, rho, u, mask)
    P64 = cpu.run(cfg, P0, 5, mask, F)
    Pld = cpu.run(cfg, P0, 5, mask, F, precision="ld")
    assert Pld.dtype == np.longdouble
    assert np.max(np.abs((P64 - Pld).astype(np.float64))) < 1e-14
    assert np.max(np.abs((P64 - Pld).astype(np.float64))) > 0          # really another precision
    if method != "CUMULANT":                                           # numpy cumulant inverts by LAPACK (no long double)
        ld = np.longdouble
        lcfg = orun.Config(stencil, method, rates)
        lcfg.lat = lcfg.lat._replace(w=np.array([ld(f.numerator) / ld(f.denominator) for f in lcfg.lat.wf]))
        Ff = None if F is None else orun.force_field(F, dims).astype(ld)
        Pn = orun.run(lcfg, P0.astype(ld), 5, mask, Ff)
        assert np.max(np.abs((Pn - Pld).astype(np.float64))) < 1e-16
