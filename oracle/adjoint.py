"""Tangent-linear and discrete adjoint of the SRT / TRT / MRT + Guo +
bounce-back time step (test infrastructure only; see ``oracle/__init__.py``).

The paper does not treat differentiation; this module is derived by hand
from the forward map that ``run`` implements, compressible Eq. (3)
equilibrium, uniform body force F:

    P^0      = f^eq(rho_init, u_init)                          (fluid cells)
    g(x)     = pull-gather of P^t with halfway bounce-back      (a permutation)
    rho, u   = sum g,  (sum c g + F/2) / rho
    P^{t+1}  = g - A (g - f^eq(rho, u)) + B S(u, F)
    readout  : rho_T = sum P^T,  u_T = (sum c P^T - F/2) / rho_T

with constant Q x Q matrices: SRT A = omega I, B = (1 - omega/2) I; TRT
A = omega_e P+ + omega_o P-, B = (1 - omega_e/2) P+ + (1 - omega_o/2) P-
(P+- the symmetric / antisymmetric parts of each (q, opp q) pair); MRT
A = M^-1 S M, B = M^-1 (I - S/2) M (rates 0 on the conserved moments), the
forms ``collision`` evaluates.  Jacobian of the collision at one cell,
J[q, p] = dP*_q / dg_p:

    delta_qp - A_qp + sum_k A_qk [f^eq_k / rho + sum_a df^eq_k/du_a (c_pa - u_a) / rho]
        + sum_k B_qk sum_a dS_k/du_a (c_pa - u_a) / rho

(SRT: (1 - omega) delta_qp + omega f^eq_q / rho + sum_a (omega df^eq_q/du_a
+ (1 - omega/2) dS_q/du_a) (c_pa - u_a) / rho.)

The adjoint state lambda^t = dL/dP^t is propagated by h = J^T lambda^{t+1}
at every fluid cell followed by the transpose of the gather (each slot of
lambda^t receives exactly one h value).  Parity pins: tangent vs central
finite differences, adjoint vs tangent (dot-product identity), gradient vs
finite differences of the loss.  A second tangent, ``tangent_complex_step``,
owes nothing to these hand derivations: it runs the forward map itself on
complex inputs, so the dot-product identity against it pins the Jacobian J
and not only its transposition.
"""

import numpy as np

from .equilibrium import density_momentum, equilibrium
from .lattice import CS2
from .stream import _shift, stream_pull


def relaxation_matrices(cfg):
    """The constant matrices A (relaxation) and B (source weighting) of the
    collision P* = g - A (g - f^eq) + B S for SRT, TRT and MRT."""
    from .collision import _group_rates, _mrt_tables, trt_odd_rate
    lat, r = cfg.lat, cfg.rates
    I = np.eye(lat.Q)
    if cfg.method == "SRT":
        return r["omega"] * I, (1.0 - 0.5 * r["omega"]) * I
    if cfg.method == "TRT":
        Pi = I[lat.opp]                    # (Pi v)_q = v_opp(q)
        Pp, Pm = 0.5 * (I + Pi), 0.5 * (I - Pi)
        we, wo = r["omega"], trt_odd_rate(r)
        return we * Pp + wo * Pm, (1.0 - 0.5 * we) * Pp + (1.0 - 0.5 * wo) * Pm
    if cfg.method == "MRT":
        M, groups, Minv = _mrt_tables(lat.name)
        s = _group_rates(groups, r)
        return Minv @ np.diag(s) @ M, Minv @ np.diag(1.0 - 0.5 * s) @ M
    raise ValueError("no adjoint for " + cfg.method)


def _local_derivs(lat, g, F):
    """rho, u and the per-cell derivative blocks for pre-collision g (Q, n)
    (S is the Guo source without its rate factor)."""
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
    # dS_q/du_a   (Q, 3, 1)
    dS_du = w[:, :, None] * (-F.reshape(1, 3, 1) / CS2 + c[:, :, None] * cF[:, :, None] / CS2 ** 2)
    dS_du = np.broadcast_to(dS_du, dfeq_du.shape)
    # dS_q/dF_b at fixed u   (Q, 3, n)
    dS_dF = w[:, :, None] * ((c[:, :, None] - u[None, :, :]) / CS2 + cu[:, None, :] * c[:, :, None] / CS2 ** 2)
    return rho, u, feq, dfeq_du, dS_du, dS_dF


def collision_jacobian(cfg, g, F):
    """J[q, p, n] = dP*_q/dg_p and B[q, b, n] = dP*_q/dF_b at each cell."""
    lat = cfg.lat
    Amat, Bmat = relaxation_matrices(cfg)
    rho, u, feq, dfeq_du, dS_du, dS_dF = _local_derivs(lat, g, F)
    c = lat.c.astype(np.float64)
    du_dg = (c.T[:, :, None] - u[:, None, :]) / rho   # (3, Q_p, n)
    dfeq_dg = np.einsum("kan,apn->kpn", dfeq_du, du_dg) + (feq / rho)[:, None, :]
    dS_dg = np.einsum("kan,apn->kpn", dS_du, du_dg)
    J = (np.eye(lat.Q) - Amat)[:, :, None] + np.einsum("qk,kpn->qpn", Amat, dfeq_dg) \
        + np.einsum("qk,kpn->qpn", Bmat, dS_dg)
    # dP*/dF: the source at fixed u, and u = (j + F/2) / rho
    du_term = np.einsum("qk,kan->qan", Amat, dfeq_du) + np.einsum("qk,kan->qan", Bmat, dS_du)
    B = np.einsum("qk,kbn->qbn", Bmat, dS_dF) + du_term / (2.0 * rho)
    return J, B


def trajectory(cfg, rho_init, u_init, solid, F, T, wall_velocity=None):
    """Forward states P^0 .. P^T (float64, no storage rounding)."""
    lat = cfg.lat
    s = solid.astype(bool)
    P = equilibrium(lat, rho_init, u_init)
    P = np.where(s[None], lat.w.reshape(-1, 1, 1, 1) * cfg.rho0, P)
    Ps = [P]
    F = np.asarray(F)
    Ff = np.broadcast_to(F.astype(complex if np.iscomplexobj(F) else float).reshape(3, 1, 1, 1), (3,) + s.shape)
    from .collision import collide
    for _ in range(T):
        g = stream_pull(lat, P, solid, wall_velocity, cfg.rho0)
        post = collide(cfg.method, lat, g, cfg.rates, Ff, cfg.rho0, cfg.compressible)
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


def transpose_gather(lat, h, solid):
    """Transpose of the pull gather with halfway bounce-back (``stream_pull``):
    the value h_q(x) that a fluid cell x pulled along link q goes back to the
    slot it was read from, (x - c_q, q) for an ordinary link or (x, opp q)
    when x - c_q is solid.  Each fluid slot is read by exactly one link, so
    this is a permutation of fluid slots; solid-cell slots receive nothing."""
    s = solid.astype(bool)
    fl = ~s
    out = np.zeros_like(h)
    for q in range(lat.Q):
        src_solid = _shift(s, lat.c[q])
        link = fl & ~src_solid
        bb = fl & src_solid
        out[q] += _shift(np.where(link, h[q], 0.0), -lat.c[q])
        out[lat.opp[q]] += np.where(bb, h[q], 0.0)
    return out


def adjoint_step(cfg, P_t, lam_next, solid, F, wall_velocity=None):
    """lambda^t from lambda^{t+1}, plus this step's dL/dF contribution.  The
    moving-wall term of the gather is a constant: it shifts the state at which
    the Jacobian is taken but adds nothing to the transpose."""
    lat = cfg.lat
    s = solid.astype(bool)
    fl = ~s
    g = stream_pull(lat, P_t, solid, wall_velocity, cfg.rho0)
    shp = g.shape[1:]
    J, B = collision_jacobian(cfg, g.reshape(lat.Q, -1), F)
    lam2 = lam_next.reshape(lat.Q, -1)
    h = np.einsum("qpn,qn->pn", J, lam2).reshape(g.shape)
    dF_cell = np.einsum("qbn,qn->bn", B, lam2).reshape((3,) + shp)
    dF = np.array([dF_cell[b][fl].sum() for b in range(3)])
    lam = transpose_gather(lat, h, solid)
    lam[:, s] = lam_next[:, s]             # identity map at solid cells (no fluid link writes there)
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
        J, B = collision_jacobian(cfg, g.reshape(lat.Q, -1), F)
        new = np.einsum("qpn,pn->qn", J, dg.reshape(lat.Q, -1)) + np.einsum("qbn,b->qn", B, dFv)
        dP = np.where(s[None], dP, new.reshape(dP.shape))
    L, dL_du = loss(cfg, Ps[T], solid, F)
    rho, j = density_momentum(lat, Ps[T])
    u = (j - 0.5 * np.asarray(F, float).reshape(3, 1, 1, 1)) / rho
    drho_T, dj = density_momentum(lat, dP)
    du_T = (dj - 0.5 * dFv.reshape(3, 1, 1, 1) - u * drho_T) / rho
    return float((dL_du * np.where(fl[None], du_T, 0.0)).sum())


def tangent_complex_step(cfg, rho_init, u_init, solid, F, T, du0, dF, h=1e-30, wall_velocity=None):
    """Directional derivative of the outlet loss along (du0, dF) by the
    complex-step method (Squire and Trapp 1998; Martins, Sturdza and Alonso
    2003): for a map that is real-analytic in its inputs,
    dL/dp . v = Im L(p + i h v) / h + O(h^2), with no difference of nearly
    equal numbers, so h = 1e-30 gives the derivative to rounding.  The forward
    trajectory (equilibrium initialisation, pull streaming with bounce-back,
    the collision itself) and the readout run unchanged on complex values;
    the loss is written with u_x^2 (not |u_x|^2) so that it stays analytic.
    Shares no formula with ``collision_jacobian`` / ``tangent``."""
    s = solid.astype(bool)
    u_c = np.asarray(u_init, dtype=complex) + 1j * h * np.asarray(du0, dtype=float)
    F_c = np.asarray(F, dtype=complex) + 1j * h * np.asarray(dF, dtype=float)
    Ps = trajectory(cfg, rho_init, u_c, solid, F_c, T, wall_velocity)
    rho, j = density_momentum(cfg.lat, Ps[T])
    ux = (j[0] - 0.5 * F_c[0]) / rho
    sel = np.zeros(s.shape, dtype=bool)
    sel[:, :, -1] = True
    sel &= ~s
    L = (ux[sel] * ux[sel]).sum()
    return float(L.imag / h)
