"""Physics pins of the oracle: closed forms and invariants (CPU only)."""

import numpy as np
import pytest

from oracle import equilibrium as eqm, lattice, run, stream
from paper_2001_11806_amd import inputs

CS2 = 1.0 / 3.0


def _linear_shear_rate(lat, omega, k):
    """Decay factor per step of the slowest non-propagating mode of the
    linearised SRT lattice operator at wave vector k (textbook linearisation
    around rest: f^eq_q ~ w_q (rho + c_q.j / c_s^2))."""
    c = lat.c.astype(float)
    W = lat.w[:, None] * (1.0 + (c @ c.T) / CS2)          # d f^eq_q / d f_p
    J = (1 - omega) * np.eye(lat.Q) + omega * W
    D = np.diag(np.exp(-1j * (c @ k)))
    ev = np.linalg.eigvals(J @ D)
    real = ev[np.abs(ev.imag) < 1e-10].real
    return real[np.argmax(real)]


def test_taylor_green_c1_energy_decay():
    """D2Q9 SRT tau=0.8, 64^2, u0=0.01, 1000 steps: kinetic energy decays at
    the linear lattice shear eigenvalue (to the O(u0^2) nonlinear level), and
    within the O(k^2) discretisation error of exp(-2 nu |k|^2 t),
    nu = c_s^2 (tau - 1/2); mass is conserved to roundoff."""
    n, tau, T = 64, 0.8, 1000
    cfg = run.Config("D2Q9", "SRT", dict(omega=1 / tau))
    rho, u = inputs.taylor_green_2d(n, 0.01)
    P = run.init_equilibrium(cfg, rho, u)
    m0 = run.conserved(cfg, P)[0]

    def energy(P):
        r, uu = run.readout(cfg, P)
        return float((r * (uu ** 2).sum(0)).sum())
    E0 = energy(P)
    P = run.run(cfg, P, 200)
    E200 = energy(P)
    P = run.run(cfg, P, T - 200)
    ratio = energy(P) / E0
    k = 2 * np.pi / n
    lam = _linear_shear_rate(cfg.lat, 1 / tau, np.array([k, k, 0.0]))
    # after the start-up layer the decay rate is the lattice eigenvalue up to
    # the nonlinear O(u0^2) ~ 1e-4 effect
    assert abs(energy(P) / E200 / lam ** (2 * (T - 200)) - 1) < 1e-4
    nu = CS2 * (tau - 0.5)
    assert abs(ratio / np.exp(-2 * nu * 2 * k * k * T) - 1) < 2e-2
    assert abs(run.conserved(cfg, P)[0] / m0 - 1) < 1e-13


@pytest.mark.parametrize("name,method", [("D3Q19", "SRT"), ("D3Q19", "TRT"), ("D3Q27", "MRT"),
                                          ("D3Q27", "CUMULANT"), ("D2Q9", "MRT"), ("D2Q9", "CUMULANT"),
                                          ("D2Q9", "KBC"), ("D3Q19", "KBC"), ("D3Q27", "KBC")])
def test_shear_wave_viscosity(name, method):
    """A small shear wave u_y = A sin(k x) decays as exp(-nu k^2 t) with
    nu = c_s^2 (1/omega - 1/2) of the shear rate (paper, Eq. 14 at |S| = 0)."""
    n, T, A = 96, 300, 1e-6
    om = 1.0 / 0.7
    cfg = run.Config(name, method, dict(omega=om, omega_bulk=1.1, omega_odd=0.0, magic=3 / 16,
                                        omega_hi=(1.0, 1.0, 1.0, 1.0)))
    x = np.arange(n)
    u = np.zeros((3, 1, 1, n))
    k = 2 * np.pi / n
    u[1, 0, 0] = A * np.sin(k * x)
    P = run.init_equilibrium(cfg, np.ones((1, 1, n)), u)
    P = run.run(cfg, P, T)
    _, uu = run.readout(cfg, P)
    amp = 2 * (uu[1, 0, 0] * np.sin(k * x)).mean()
    nu = CS2 * (1 / om - 0.5)
    measured = -np.log(amp / A) / (k * k * T)
    assert abs(measured / nu - 1) < 5e-3, (measured, nu)


def _poiseuille(method, H=16, F=1e-5, steps=8000):
    ny = H + 2
    cfg = run.Config("D3Q19", method, dict(omega=1 / 0.8, magic=3 / 16, omega_odd=0.0))
    mask = inputs.channel_mask(1, ny, 1)
    Ff = run.force_field(np.array([F, 0, 0]), (1, ny, 1))
    P = run.init_equilibrium(cfg, np.ones((1, ny, 1)), np.zeros((3, 1, ny, 1)), mask)
    P = run.run(cfg, P, steps, mask, Ff)
    _, u = run.readout(cfg, P, mask, Ff)
    y = np.arange(1, H + 1)
    nu = CS2 * (0.8 - 0.5)
    exact = F / (2 * nu) * (y - 0.5) * (H + 0.5 - y)
    return u[0, 0, 1:H + 1, 0], exact


def test_poiseuille_trt_magic_exact():
    """TRT with Lambda = 3/16 and halfway bounce-back reproduces the parabolic
    profile with walls half-way between cells exactly (Ginzburg's result)."""
    got, exact = _poiseuille("TRT")
    assert np.max(np.abs(got / exact - 1)) < 1e-9


def test_poiseuille_srt_slip_negative_control():
    """SRT at tau = 0.8 has a tau-dependent wall slip: the same check fails."""
    got, exact = _poiseuille("SRT")
    assert np.max(np.abs(got / exact - 1)) > 1e-4


def test_gather_at_matches_stream_pull():
    lat = lattice.velocity_set("D3Q19")
    rng = np.random.default_rng(1)
    dims = (7, 5, 4)
    P = rng.standard_normal((lat.Q, 4, 5, 7))
    solid = (rng.random((4, 5, 7)) < 0.2).astype(np.uint8)
    full = stream.stream_pull(lat, P, solid)
    cells = np.arange(7 * 5 * 4)
    part = stream.gather_at(lat, lambda q, idx: P[q].reshape(-1)[idx], cells, dims, solid)
    np.testing.assert_array_equal(part, full.reshape(lat.Q, -1))


@pytest.mark.parametrize("name,method", [("D3Q19", "SRT"), ("D3Q19", "TRT"), ("D3Q27", "MRT"), ("D2Q9", "TRT")])
def test_mass_conserved_with_mask_and_force(name, method):
    """Streaming with bounce-back is a permutation of fluid links and the
    collision conserves mass: total mass stays put to roundoff."""
    cfg = run.Config(name, method, dict(omega=1.6, omega_bulk=1.2, magic=3 / 16, omega_odd=0.0,
                                        omega_hi=(1.0, 1.1, 0.9, 1.0)))
    nz = 1 if name == "D2Q9" else 6
    dims = (10, 8, nz)
    rng = np.random.default_rng(3)
    solid = (rng.random((nz, 8, 10)) < 0.15).astype(np.uint8)
    u = inputs.uniform_noise_velocity(dims, 0.02, 1, solid)
    if name == "D2Q9":
        u[2] = 0
    P = run.init_equilibrium(cfg, np.ones((nz, 8, 10)), u, solid)
    F = run.force_field(np.array([1e-4, -2e-5, 0.0 if name == "D2Q9" else 3e-5]), dims)
    m0 = run.conserved(cfg, P, solid)[0]
    P = run.run(cfg, P, 40, solid, F)
    assert abs(run.conserved(cfg, P, solid)[0] / m0 - 1) < 1e-14


def test_momentum_gain_is_force_periodic():
    """No walls: every step adds exactly F per fluid cell to the momentum."""
    cfg = run.Config("D3Q27", "MRT", dict(omega=1.8, omega_bulk=1.2, omega_hi=(1.0,) * 4))
    dims = (6, 5, 4)
    u = inputs.uniform_noise_velocity(dims, 0.02, 2)
    P = run.init_equilibrium(cfg, np.ones((4, 5, 6)), u)
    Fv = np.array([1e-4, 2e-4, -3e-4])
    F = run.force_field(Fv, dims)
    c0 = run.conserved(cfg, P)
    P = run.run(cfg, P, 10, None, F)
    c1 = run.conserved(cfg, P)
    np.testing.assert_allclose(c1[1:] - c0[1:], 10 * 120 * Fv, rtol=1e-10)


def test_round_bf16_matches_bit_rounding():
    """Emulated bf16 rounding equals round-to-nearest-even on float32 bits
    (for values already representable in float32), incl. exact ties."""
    rng = np.random.default_rng(0)
    x = (rng.standard_normal(20000) * 10.0 ** rng.integers(-30, 5, 20000)).astype(np.float32)
    ties = (np.arange(1, 200, dtype=np.uint32) << 16 | 0x8000).view(np.float32)   # exact halfway cases
    x = np.concatenate([x, ties, -ties])
    b = x.view(np.uint32).astype(np.uint64)
    r = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    want = r.astype(np.uint32).view(np.float32).astype(np.float64)
    np.testing.assert_array_equal(run.round_bf16(x.astype(np.float64)), want)


def test_quantize_round_trip_and_bound():
    cfg = run.Config("D3Q19", "SRT", dict(omega=1.0), storage="f16")
    rng = np.random.default_rng(4)
    P = cfg.lat.w.reshape(-1, 1) * (1 + 0.01 * rng.standard_normal((19, 100)))
    Q = run.quantize(cfg, P)
    dev = P - cfg.lat.w.reshape(-1, 1)
    assert np.all(np.abs(Q - P) <= np.abs(dev) * 2.0 ** -11 + 2.0 ** -25)
    np.testing.assert_array_equal(run.quantize(cfg, Q), Q)


@pytest.mark.parametrize("method", ["SRT", "TRT"])
def test_couette_moving_wall_exact(method):
    """Velocity bounce-back: a wall at y = H + 0.5 moving with U along x over
    a resting wall at y = 0.5 gives the linear Couette profile
    u_x = U (y - 0.5) / H exactly at steady state (halfway bounce-back is
    exact for linear flows)."""
    H, U = 12, 0.01
    ny = H + 2
    cfg = run.Config("D3Q19", method, dict(omega=1 / 0.8, magic=3 / 16, omega_odd=0.0))
    mask = inputs.channel_mask(1, ny, 1)
    mask[:, ny - 1, :] = 2
    table = np.zeros((3, 3))
    table[2] = (U, 0.0, 0.0)
    P = run.init_equilibrium(cfg, np.ones((1, ny, 1)), np.zeros((3, 1, ny, 1)), mask)
    P = run.run(cfg, P, 6000, mask, None, table)
    _, u = run.readout(cfg, P, mask)
    y = np.arange(1, H + 1)
    np.testing.assert_allclose(u[0, 0, 1:H + 1, 0], U * (y - 0.5) / H, rtol=1e-9, atol=1e-14)
    # the moving wall drags: momentum enters through it
    assert run.conserved(cfg, P, mask)[1] > 0


def lid_driven_cavity(N, U, steps, tau=1.0):
    """D2Q9 SRT cavity: resting walls at x = 0, x = N-1, y = 0; the top row
    y = N-1 is a lid (wall type 2) moving with U along x."""
    cfg = run.Config("D2Q9", "SRT", dict(omega=1 / tau))
    mask = np.zeros((1, N, N), dtype=np.uint8)
    mask[0, 0, :] = 1
    mask[0, :, 0] = 1
    mask[0, :, N - 1] = 1
    mask[0, N - 1, :] = 2
    table = np.zeros((3, 3))
    table[2] = (U, 0.0, 0.0)
    P = run.init_equilibrium(cfg, np.ones((1, N, N)), np.zeros((3, 1, N, N)), mask)
    P = run.run(cfg, P, steps, mask, None, table)
    _, u = run.readout(cfg, P, mask)
    return u[:2, 0], mask, table


def _asymmetry(u):
    """Departure from the Stokes-flow symmetry u_x(x, y) = u_x(L - x, y),
    u_y(x, y) = -u_y(L - x, y), relative to max |u|."""
    ux, uy = u
    return max(np.max(np.abs(ux - ux[:, ::-1])), np.max(np.abs(uy + uy[:, ::-1]))) / np.max(np.abs(u))


def test_lid_driven_cavity_stokes_symmetry():
    """Creeping lid-driven cavity.  Stokes flow is linear and reversible, so
    reflecting x and reversing the flow maps the solution to itself: the
    steady field is mirror-symmetric about the vertical centre line.  At
    Re = 0.002 the departure is the O(Re) inertia; at Re = 2 it is a hundred
    times larger (negative control).  The lid drags the fluid along below it
    and the return flow runs the other way near the bottom."""
    u_slow = lid_driven_cavity(24, 1e-4, 6000)[0]
    u_fast = lid_driven_cavity(24, 1e-2, 6000)[0]
    a_slow, a_fast = _asymmetry(u_slow), _asymmetry(u_fast)
    assert a_slow < 2e-4, a_slow
    assert a_fast > 50 * a_slow, (a_slow, a_fast)
    assert u_slow[0][-2, 12] > 0 > u_slow[0][1, 12]
