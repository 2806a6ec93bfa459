"""Pins of the oracle's tangent-linear and adjoint maps (CPU only):
central finite differences of the forward run, the dot-product identity
between tangent and adjoint, and the O(h^2) Taylor remainder."""

import numpy as np
import pytest

from oracle import adjoint, run
from paper_2001_11806_amd import inputs


RATES = {"SRT": dict(omega=1 / 0.6),
         "TRT": dict(omega=1 / 0.6, magic=3 / 16, omega_odd=0.0),
         "MRT": dict(omega=1 / 0.6, omega_bulk=1.2, omega_hi=(1.3, 0.9, 1.1, 1.2))}
METHODS = ["SRT", "TRT", "MRT"]


def _setup(nx=8, ny=10, nz=6, T=12, seed=4, method="SRT"):
    cfg = run.Config("D3Q19", method, RATES[method])
    mask = inputs.channel_mask(nx, ny, nz)
    mask[2:4, 4:6, 3:5] = 1                      # a small obstacle
    u0 = inputs.uniform_noise_velocity((nx, ny, nz), 2e-2, seed, mask)
    rho = np.ones((nz, ny, nx))
    F = np.array([1e-3, 2e-4, -1e-4])
    return cfg, mask, rho, u0, F, T


def _loss(cfg, rho, u0, mask, F, T):
    Ps = adjoint.trajectory(cfg, rho, u0, mask, F, T)
    return adjoint.outlet_loss(cfg, Ps[T], mask, F)[0]


@pytest.mark.parametrize("method", METHODS)
def test_trajectory_equals_run_step(method):
    """The adjoint module's forward trajectory is the ordinary time step."""
    cfg, mask, rho, u0, F, T = _setup(T=5, method=method)
    Ps = adjoint.trajectory(cfg, rho, u0, mask, F, T)
    P = run.init_equilibrium(cfg, rho, u0, mask)
    P = run.run(cfg, P, T, mask, run.force_field(F, (8, 10, 6)))
    np.testing.assert_array_equal(Ps[T], P)


@pytest.mark.parametrize("method", METHODS)
def test_tangent_matches_central_differences(method):
    cfg, mask, rho, u0, F, T = _setup(method=method)
    rng = np.random.default_rng(1)
    du = rng.standard_normal(u0.shape) * (mask == 0)
    dF = rng.standard_normal(3)
    tl = adjoint.tangent(cfg, rho, u0, mask, F, T, du, dF)
    h = 1e-6
    fd = (_loss(cfg, rho, u0 + h * du, mask, F + h * dF, T)
          - _loss(cfg, rho, u0 - h * du, mask, F - h * dF, T)) / (2 * h)
    assert abs(tl / fd - 1) < 1e-6


@pytest.mark.parametrize("method", METHODS)
def test_adjoint_dot_product_identity(method):
    """<dL/dp, v> from the reverse sweep equals the tangent along v."""
    cfg, mask, rho, u0, F, T = _setup(method=method)
    L, gu, grho, gF = adjoint.gradient(cfg, rho, u0, mask, F, T)
    rng = np.random.default_rng(2)
    for _ in range(3):
        du = rng.standard_normal(u0.shape) * (mask == 0)
        dF = rng.standard_normal(3)
        tl = adjoint.tangent(cfg, rho, u0, mask, F, T, du, dF)
        rev = float((gu * du).sum() + gF @ dF)
        assert abs(rev / tl - 1) < 1e-12


@pytest.mark.parametrize("method", METHODS)
def test_gradient_matches_finite_differences_and_taylor_order(method):
    cfg, mask, rho, u0, F, T = _setup(method=method)
    L, gu, grho, gF = adjoint.gradient(cfg, rho, u0, mask, F, T)
    rng = np.random.default_rng(3)
    fluid = np.argwhere((mask == 0))
    picks = fluid[rng.choice(len(fluid), 6, replace=False)]
    for (z, y, x) in picks:
        for a in range(3):
            e = np.zeros_like(u0)
            e[a, z, y, x] = 1.0
            # h = 1e-5 balances truncation (~1e-12) against the roundoff
            # of the 12-step run (~1e-17 / h)
            h = 1e-5
            fd = (_loss(cfg, rho, u0 + h * e, mask, F, T) - _loss(cfg, rho, u0 - h * e, mask, F, T)) / (2 * h)
            assert abs(gu[a, z, y, x] - fd) <= 1e-6 * abs(fd) + 1e-11
    for b in range(3):
        e = np.zeros(3)
        e[b] = 1.0
        h = 1e-5
        fd = (_loss(cfg, rho, u0, mask, F + h * e, T) - _loss(cfg, rho, u0, mask, F - h * e, T)) / (2 * h)
        assert abs(gF[b] - fd) <= 1e-6 * abs(fd) + 1e-11
    # Taylor remainder of first order decays as h^2
    d = rng.standard_normal(u0.shape) * (mask == 0) * 1e-3
    r = []
    for h in (1.0, 0.5, 0.25):
        r.append(abs(_loss(cfg, rho, u0 + h * d, mask, F, T) - L - h * float((gu * d).sum())))
    assert 3.0 < r[0] / r[1] < 5.0 and 3.0 < r[1] / r[2] < 5.0


def test_solid_cells_have_zero_gradient():
    cfg, mask, rho, u0, F, T = _setup()
    _, gu, grho, _ = adjoint.gradient(cfg, rho, u0, mask, F, T)
    assert not gu[:, mask.astype(bool)].any()
    assert not grho[mask.astype(bool)].any()


def test_moving_wall_gradient_matches_finite_differences():
    """With a moving wall the gather adds a constant: the adjoint still
    matches finite differences of the forward run."""
    cfg, mask, rho, u0, F, T = _setup()
    mask = mask.copy()
    mask[:, -1, :] = 2
    u0 = u0 * (mask == 0)
    table = np.zeros((3, 3))
    table[2] = (0.03, 0.0, 0.01)
    L, gu, grho, gF = adjoint.gradient(cfg, rho, u0, mask, F, T, wall_velocity=table)

    def loss(uu, FF):
        Ps = adjoint.trajectory(cfg, rho, uu, mask, FF, T, table)
        return adjoint.outlet_loss(cfg, Ps[T], mask, FF)[0]
    h = 1e-5
    fd = (loss(u0, F + [h, 0, 0]) - loss(u0, F - [h, 0, 0])) / (2 * h)
    assert abs(gF[0] - fd) <= 1e-6 * abs(fd) + 1e-11
    e = np.zeros_like(u0)
    e[0, 2, 5, 7] = 1.0
    fd = (loss(u0 + h * e, F) - loss(u0 - h * e, F)) / (2 * h)
    assert abs(gu[0, 2, 5, 7] - fd) <= 1e-6 * abs(fd) + 1e-11


def test_relaxation_matrices_reproduce_the_collisions():
    """P* = g - A (g - f^eq) + B S with the adjoint's constant matrices is the
    collision the forward run applies (SRT, TRT, MRT), so the Jacobian is
    taken of the right map."""
    from oracle import collision
    from oracle.equilibrium import equilibrium, guo_source, macroscopic
    rng = np.random.default_rng(6)
    for method in METHODS:
        cfg = run.Config("D3Q19", method, RATES[method])
        lat = cfg.lat
        rho = 1 + 0.01 * rng.uniform(-1, 1, 20)
        u = 0.03 * rng.uniform(-1, 1, (3, 20))
        g = equilibrium(lat, rho, u) * (1 + 0.05 * rng.uniform(-1, 1, (lat.Q, 20)))
        F = 1e-3 * rng.uniform(-1, 1, (3, 20))
        A, B = adjoint.relaxation_matrices(cfg)
        r, uu = macroscopic(lat, g, F)
        want = g - A @ (g - equilibrium(lat, r, uu)) + B @ guo_source(lat, uu, F)
        np.testing.assert_allclose(collision.collide(method, lat, g, cfg.rates, F), want, rtol=0, atol=1e-15)


@pytest.mark.parametrize("method", METHODS)
def test_adjoint_matches_complex_step_tangent(method):
    """Dot-product identity against a tangent that shares nothing with the
    hand-derived Jacobian: the complex-step derivative of the forward run
    itself.  <dL/dp, v> from the reverse sweep equals Im L(p + i h v) / h
    to rounding, for random directions v in (u0, F), with a moving wall as
    well as resting ones."""
    cfg, mask, rho, u0, F, T = _setup(method=method)
    mask = mask.copy()
    mask[:, -1, :] = 2
    u0 = u0 * (mask == 0)
    table = np.zeros((3, 3))
    table[2] = (0.03, 0.0, 0.01)
    L, gu, grho, gF = adjoint.gradient(cfg, rho, u0, mask, F, T, wall_velocity=table)
    rng = np.random.default_rng(12)
    for _ in range(3):
        du = rng.standard_normal(u0.shape) * (mask == 0)
        dF = rng.standard_normal(3)
        cs = adjoint.tangent_complex_step(cfg, rho, u0, mask, F, T, du, dF, wall_velocity=table)
        rev = float((gu * du).sum() + gF @ dF)
        assert abs(rev / cs - 1) < 1e-12, (rev, cs)


def test_complex_step_identity_catches_a_wrong_jacobian(monkeypatch):
    """Negative control: a relaxation matrix off by 1e-3 in one rate (a
    mistake confined to the Jacobian, with the forward run untouched)
    breaks the identity against the complex-step tangent by far more than
    its 1e-12 bar."""
    cfg, mask, rho, u0, F, T = _setup(method="TRT")
    good = adjoint.relaxation_matrices

    def wrong(c):
        A, B = good(c)
        return A * (1 + 1e-3), B
    monkeypatch.setattr(adjoint, "relaxation_matrices", wrong)
    L, gu, grho, gF = adjoint.gradient(cfg, rho, u0, mask, F, T)
    rng = np.random.default_rng(13)
    du = rng.standard_normal(u0.shape) * (mask == 0)
    dF = rng.standard_normal(3)
    cs = adjoint.tangent_complex_step(cfg, rho, u0, mask, F, T, du, dF)
    rev = float((gu * du).sum() + gF @ dF)
    assert abs(rev / cs - 1) > 1e-6


@pytest.mark.parametrize("stencil", ["D2Q9", "D3Q19", "D3Q27"])
def test_transpose_gather_is_a_permutation_of_fluid_slots(stencil):
    """Write-count check of the adjoint's reverse streaming: pushing a 1
    back along every link of every fluid cell lands exactly one 1 in every
    slot of every fluid cell (each slot is read by exactly one link: its own
    pull, or the bounce-back of its cell) and nothing in solid cells; and
    <gather(P), H> = <P, transpose(H)> on fluid cells for random P, H."""
    from oracle.lattice import velocity_set
    from oracle.stream import stream_pull
    lat = velocity_set(stencil)
    dims = (9, 8, 1) if stencil == "D2Q9" else (7, 8, 5)
    rng = np.random.default_rng(21)
    solid = (rng.random(dims[::-1]) < 0.2).astype(np.uint8)
    solid[..., 0, :] = 1
    fl = solid == 0
    ones = np.where(fl[None], 1.0, 0.0) * np.ones((lat.Q,) + dims[::-1])
    got = adjoint.transpose_gather(lat, ones, solid)
    assert np.array_equal(got[:, fl], np.ones((lat.Q, int(fl.sum()))))
    assert not got[:, ~fl].any()
    P = rng.standard_normal((lat.Q,) + dims[::-1])
    H = rng.standard_normal(P.shape) * fl[None]
    lhs = float((stream_pull(lat, P, solid) * H).sum())
    rhs = float((P * adjoint.transpose_gather(lat, H, solid) * fl[None]).sum())
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))
