"""Tangent-linear and discrete adjoint of the SRT + Guo + bounce-back time
step (test infrastructure only; see ``oracle/__init__.py``).

The paper does not treat differentiation; this module is derived by hand
from the forward map that ``run`` implements, compressible Eq. (3)
equilibrium, uniform body force F:

    P^0      = f^eq(rho_init, u_init)                          (fluid cells)
    g(x)     = pull-gather of P^t with halfway bounce-back      (a permutation)
    rho, u   = sum g,  (sum c g + F/2) / rho
    P^{t+1}  = g - omega (g - f^eq(rho, u)) + (1 - omega/2) S(u, F)
    readout  : rho_T = sum P^T,  u_T = (sum c P^T - F/2) / rho_T

Jacobian of the collision at one cell, J[q, p] = dP*_q / dg_p:

    (1 - omega) delta_qp + omega f^eq_q / rho
        + sum_a (omega df^eq_q/du_a + dS_q/du_a) (c_pa - u_a) / rho

The adjoint state lambda^t = dL/dP^t is propagated by h = J^T lambda^{t+1}
at every fluid cell followed by the transpose of the gather (each slot of
lambda^t receives exactly one h value).  Parity pins: tangent vs central
finite differences, adjoint vs tangent (dot-product identity), gradient vs
finite differences of the loss.
"""

import numpy as np

from .equilibrium import density_momentum, equilibrium
from .lattice import CS2
from .stream import _shift, stream_pull


def _local_derivs(lat, g, omega, F):
    """rho, u and the per-cell derivative blocks for pre-collision g (Q, n)."""
    c = lat.c.astype(np.float64)                      # (Q, 3)
    F = np.asarray(F, dtype=np.float64).reshape(3, 1)
    rho, j = density_momentum(lat, g)
    u = (j + 0.5 * F) / rho                           # (3, n)
    feq = equilibrium(lat, rho, u)                    # (Q, n)
    cu = c @ u                                        # (Q, n)
    cF = c @ F                                        # (Q, 1)
    w = lat.w[:, None]
    # df^eq_q/du_a  (Q, 3, n)
    dfeq_du = (w * rho)[:, None, :] * (c[:, :, None] / CS2
                                       + cu[:, None, :] * c[:, :, None] / CS2 ** 2
                                       - u[None, :, :] / CS2)
    # dS_q/du_a including (1 - omega/2)   (Q, 3, 1)
    dS_du = (1 - 0.5 * omega) * w[:, :, None] * (-F.reshape(1, 3, 1) / CS2
                                                 + c[:, :, None] * cF[:, :, None] / CS2 ** 2)
    dS_du = np.broadcast_to(dS_du, dfeq_du.shape)
    # dS_q/dF_b at fixed u, including (1 - omega/2)   (Q, 3, n)
    dS_dF = (1 - 0.5 * omega) * w[:, :, None] * ((c[:, :, None] - u[None, :, :]) / CS2
                                                 + cu[:, None, :] * c[:, :, None] / CS2 ** 2)
    return rho, u, feq, dfeq_du, dS_du, dS_dF


def collision_jacobian(lat, g, omega, F):
    """J[q, p, n] = dP*_q/dg_p and B[q, b, n] = dP*_q/dF_b at each cell."""
    rho, u, feq, dfeq_du, dS_du, dS_dF = _local_derivs(lat, g, omega, F)
    c = lat.c.astype(np.float64)
    du_dg = (c.T[:, :, None] - u[:, None, :]) / rho   # (3, Q_p, n)
    A = omega * dfeq_du + dS_du                       # (Q, 3, n)
    J = np.einsum("qan,apn->qpn", A, du_dg)
    J = J + omega * (feq / rho)[:, None, :]
    J = J + (1.0 - omega) * np.eye(lat.Q)[:, :, None]
    B = dS_dF + A / (2.0 * rho)
    return J, B


def trajectory(cfg, rho_init, u_init, solid, F, T, wall_velocity=None):
    """Forward states P^0 .. P^T (float64, no storage rounding)."""
    lat = cfg.lat
    s = solid.astype(bool)
    P = equilibrium(lat, rho_init, u_init)
    P = np.where(s[None], lat.w.reshape(-1, 1, 1, 1) * cfg.rho0, P)
    Ps = [P]
    Ff = np.broadcast_to(np.asarray(F, float).reshape(3, 1, 1, 1), (3,) + s.shape)
    from .collision import srt
    for _ in range(T):
        g = stream_pull(lat, P, solid, wall_velocity, cfg.rho0)
        post = srt(lat, g, cfg.rates, Ff)
        P = np.where(s[None], P, post)
        Ps.append(P)
    return Ps


def readout_u(cfg, P, solid, F):
    rho, j = density_momentum(cfg.lat, P)
    u = (j - 0.5 * np.asarray(F, float).reshape(3, 1, 1, 1)) / rho
    return rho, np.where(solid[None].astype(bool), 0.0, u)


def outlet_loss(cfg, P, solid, F):
    """L = sum of u_x^2 over fluid cells of the last x-plane (reading of the
    'outlet plane' of a periodic channel), and dL/du (3, nz, ny, nx)."""
    rho, u = readout_u(cfg, P, solid, F)
    sel = np.zeros(solid.shape, dtype=bool)
    sel[:, :, -1] = True
    sel &= ~solid.astype(bool)
    L = float((u[0][sel] ** 2).sum())
    dL_du = np.zeros_like(u)
    dL_du[0][sel] = 2.0 * u[0][sel]
    return L, dL_du


def seed(cfg, P, solid, F, dL_du, dL_drho=None):
    """lambda^T = dL/dP^T through the readout, and the readout's direct
    contribution to dL/dF (u_T depends on F through -F/2)."""
    lat = cfg.lat
    c = lat.c.astype(np.float64)
    rho, u = readout_u(cfg, P, solid, F)
    fl = ~solid.astype(bool)
    lam = np.zeros_like(P)
    for q in range(lat.Q):
        v = sum(dL_du[a] * (c[q, a] - u[a]) for a in range(3)) / np.where(fl, rho, 1.0)
        if dL_drho is not None:
            v = v + dL_drho
        lam[q] = np.where(fl, v, 0.0)
    dF = np.array([-(dL_du[a][fl] / (2.0 * rho[fl])).sum() for a in range(3)])
    return lam, dF


def adjoint_step(cfg, P_t, lam_next, solid, F, wall_velocity=None):
    """lambda^t from lambda^{t+1}, plus this step's dL/dF contribution.  The
    moving-wall term of the gather is a constant: it shifts the state at which
    the Jacobian is taken but adds nothing to the transpose."""
    lat = cfg.lat
    s = solid.astype(bool)
    fl = ~s
    g = stream_pull(lat, P_t, solid, wall_velocity, cfg.rho0)
    shp = g.shape[1:]
    J, B = collision_jacobian(lat, g.reshape(lat.Q, -1), cfg.rates["omega"], F)
    lam2 = lam_next.reshape(lat.Q, -1)
    h = np.einsum("qpn,qn->pn", J, lam2).reshape(g.shape)
    dF_cell = np.einsum("qbn,qn->bn", B, lam2).reshape((3,) + shp)
    dF = np.array([dF_cell[b][fl].sum() for b in range(3)])
    lam = np.zeros_like(lam_next)
    lam[:, s] = lam_next[:, s]             # identity map at solid cells
    for q in range(lat.Q):
        src_solid = _shift(s, lat.c[q])
        link = fl & ~src_solid
        bb = fl & src_solid
        lam[q] += _shift(np.where(link, h[q], 0.0), -lat.c[q])
        lam[lat.opp[q]] += np.where(bb, h[q], 0.0)
    return lam, dF


def init_gradient(cfg, rho_init, u_init, lam0, solid):
    """dL/du_init and dL/drho_init through P^0 = f^eq(rho, u)."""
    lat = cfg.lat
    c = lat.c.astype(np.float64)
    fl = ~solid.astype(bool)
    rho = np.asarray(rho_init, float)
    cu = np.tensordot(c, u_init, axes=(1, 0))
    w = lat.w.reshape(-1, 1, 1, 1)
    feq = equilibrium(lat, rho, u_init)
    du = np.zeros_like(u_init)
    for a in range(3):
        dfeq = w * rho * (c[:, a].reshape(-1, 1, 1, 1) / CS2
                          + cu * c[:, a].reshape(-1, 1, 1, 1) / CS2 ** 2 - u_init[a] / CS2)
        du[a] = np.where(fl, (lam0 * dfeq).sum(0), 0.0)
    drho = np.where(fl, (lam0 * feq / rho).sum(0), 0.0)
    return du, drho


def gradient(cfg, rho_init, u_init, solid, F, T, loss=outlet_loss, wall_velocity=None):
    """Full reverse sweep: returns (L, dL/du_init, dL/drho_init, dL/dF)."""
    Ps = trajectory(cfg, rho_init, u_init, solid, F, T, wall_velocity)
    L, dL_du = loss(cfg, Ps[T], solid, F)
    lam, dF = seed(cfg, Ps[T], solid, F, dL_du)
    for t in range(T - 1, -1, -1):
        lam, dFt = adjoint_step(cfg, Ps[t], lam, solid, F, wall_velocity)
        dF = dF + dFt
    du, drho = init_gradient(cfg, rho_init, u_init, lam, solid)
    return L, du, drho, dF


def tangent(cfg, rho_init, u_init, solid, F, T, du0, dF, loss=outlet_loss, wall_velocity=None):
    """Forward-mode derivative of the loss along (du0, dF)."""
    lat = cfg.lat
    s = solid.astype(bool)
    fl = ~s
    c = lat.c.astype(np.float64)
    w = lat.w.reshape(-1, 1, 1, 1)
    cu = np.tensordot(c, u_init, axes=(1, 0))
    dP = np.zeros((lat.Q,) + s.shape)
    for a in range(3):
        dfeq = w * rho_init * (c[:, a].reshape(-1, 1, 1, 1) / CS2
                               + cu * c[:, a].reshape(-1, 1, 1, 1) / CS2 ** 2 - u_init[a] / CS2)
        dP += dfeq * du0[a]
    dP = np.where(fl[None], dP, 0.0)
    Ps = trajectory(cfg, rho_init, u_init, solid, F, T, wall_velocity)
    dFv = np.asarray(dF, float)
    for t in range(T):
        g = stream_pull(lat, Ps[t], solid, wall_velocity, cfg.rho0)
        dg = stream_pull(lat, dP, s)
        J, B = collision_jacobian(lat, g.reshape(lat.Q, -1), cfg.rates["omega"], F)
        new = np.einsum("qpn,pn->qn", J, dg.reshape(lat.Q, -1)) + np.einsum("qbn,b->qn", B, dFv)
        dP = np.where(s[None], dP, new.reshape(dP.shape))
    L, dL_du = loss(cfg, Ps[T], solid, F)
    rho, j = density_momentum(lat, Ps[T])
    u = (j - 0.5 * np.asarray(F, float).reshape(3, 1, 1, 1)) / rho
    drho_T, dj = density_momentum(lat, dP)
    du_T = (dj - 0.5 * dFv.reshape(3, 1, 1, 1) - u * drho_T) / rho
    return float((dL_du * np.where(fl[None], du_T, 0.0)).sum())
