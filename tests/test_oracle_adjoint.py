"""Pins of the oracle's tangent-linear and adjoint maps (CPU only):
central finite differences of the forward run, the dot-product identity
between tangent and adjoint, and the O(h^2) Taylor remainder."""

import numpy as np
import pytest

from oracle import adjoint, run
from paper_2001_11806_amd import inputs


def _setup(nx=8, ny=10, nz=6, T=12, seed=4):
    cfg = run.Config("D3Q19", "SRT", dict(omega=1 / 0.6))
    mask = inputs.channel_mask(nx, ny, nz)
    mask[2:4, 4:6, 3:5] = 1                      # a small obstacle
    u0 = inputs.uniform_noise_velocity((nx, ny, nz), 2e-2, seed, mask)
    rho = np.ones((nz, ny, nx))
    F = np.array([1e-3, 2e-4, -1e-4])
    return cfg, mask, rho, u0, F, T


def _loss(cfg, rho, u0, mask, F, T):
    Ps = adjoint.trajectory(cfg, rho, u0, mask, F, T)
    return adjoint.outlet_loss(cfg, Ps[T], mask, F)[0]


def test_trajectory_equals_run_step():
    """The adjoint module's forward trajectory is the ordinary time step."""
    cfg, mask, rho, u0, F, T = _setup(T=5)
    Ps = adjoint.trajectory(cfg, rho, u0, mask, F, T)
    P = run.init_equilibrium(cfg, rho, u0, mask)
    P = run.run(cfg, P, T, mask, run.force_field(F, (8, 10, 6)))
    np.testing.assert_array_equal(Ps[T], P)


def test_tangent_matches_central_differences():
    cfg, mask, rho, u0, F, T = _setup()
    rng = np.random.default_rng(1)
    du = rng.standard_normal(u0.shape) * (mask == 0)
    dF = rng.standard_normal(3)
    tl = adjoint.tangent(cfg, rho, u0, mask, F, T, du, dF)
    h = 1e-6
    fd = (_loss(cfg, rho, u0 + h * du, mask, F + h * dF, T)
          - _loss(cfg, rho, u0 - h * du, mask, F - h * dF, T)) / (2 * h)
    assert abs(tl / fd - 1) < 1e-6


def test_adjoint_dot_product_identity():
    """<dL/dp, v> from the reverse sweep equals the tangent along v."""
    cfg, mask, rho, u0, F, T = _setup()
    L, gu, grho, gF = adjoint.gradient(cfg, rho, u0, mask, F, T)
    rng = np.random.default_rng(2)
    for _ in range(3):
        du = rng.standard_normal(u0.shape) * (mask == 0)
        dF = rng.standard_normal(3)
        tl = adjoint.tangent(cfg, rho, u0, mask, F, T, du, dF)
        rev = float((gu * du).sum() + gF @ dF)
        assert abs(rev / tl - 1) < 1e-12


def test_gradient_matches_finite_differences_and_taylor_order():
    cfg, mask, rho, u0, F, T = _setup()
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
