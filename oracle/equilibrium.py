"""Macroscopic moments, equilibrium, forcing (test infrastructure only).

Array convention: populations ``f`` have shape (Q, ...) and vector fields
(velocity, force) have shape (3, ...); the trailing "..." is any cell shape.
"""

import itertools
from fractions import Fraction

import numpy as np

from .lattice import CS2, CS2_EXACT


def _real_or_complex(a):
    """The input as a float64 array, keeping a wider or complex floating
    type: the complex-step derivative (``adjoint.tangent_complex_step``)
    runs the forward map on complex values, and the FP64 rounding floor of
    the oracle is measured against a run in extended precision
    (``np.longdouble``).  Integer and float64 inputs give float64."""
    a = np.asarray(a)
    return a.astype(np.result_type(a.dtype, np.float64), copy=False)


def _bcast(a, ndim):
    """Reshape a (3,)- or (3, ...)-array so it broadcasts against (3, *cells)."""
    a = _real_or_complex(a)
    return a.reshape(a.shape + (1,) * (ndim + 1 - a.ndim))


def density_momentum(lat, f):
    """Eq. (2) numerators: rho = sum_q f_q and j = sum_q c_q f_q."""
    rho = f.sum(axis=0)
    j = np.tensordot(lat.c.T.astype(np.float64), f, axes=(1, 0))
    return rho, j


def macroscopic(lat, f, force=None, rho0=1.0, compressible=True):
    """Eq. (2) with the Guo half-force shift.

    rho = sum f;  u = (sum c f + F/2) / rho_0, where rho_0 = rho for the
    compressible method and the constant reference density otherwise
    (Eq. (3) discussion).  The F/2 term is Guo's velocity definition
    (reading: the paper only cites the forcing scheme, Sec. I).
    """
    rho, j = density_momentum(lat, f)
    if force is not None:
        j = j + 0.5 * _bcast(force, rho.ndim)
    denom = rho if compressible else rho0
    return rho, j / denom


def equilibrium(lat, rho, u, rho0=1.0, compressible=True):
    """Eq. (3) truncated at second order in u.

    f_q^eq = w_q rho + w_q rho_0 [c.u/c_s^2 + (c.u)^2/(2 c_s^4) - u.u/(2 c_s^2)],
    rho_0 = rho (compressible) or the reference density (incompressible).
    The (c.u)^2 / u.u pair is the paper's u_a u_b (c_a c_b - c_s^2 delta_ab)
    term written out.
    """
    rho = _real_or_complex(rho)
    u = _real_or_complex(u)
    cu = np.tensordot(lat.c.astype(np.float64), u, axes=(1, 0))
    usq = (u * u).sum(axis=0)
    r0 = rho if compressible else rho0
    w = lat.w.reshape((lat.Q,) + (1,) * rho.ndim)
    return w * rho + w * r0 * (cu / CS2 + cu * cu / (2.0 * CS2 * CS2) - usq / (2.0 * CS2))


def guo_source(lat, u, force):
    """Guo's discrete forcing term without its (1 - omega/2) prefactor.

    S_q = w_q [ (c_q - u).F / c_s^2 + (c_q.u)(c_q.F) / c_s^4 ].
    Its moments are sum S = 0, sum c S = F, sum c_a c_b S = u_a F_b + F_a u_b.
    """
    u = _real_or_complex(u)
    F = _bcast(force, u.ndim - 1) * np.ones_like(u)
    c = lat.c.astype(np.float64)
    cu = np.tensordot(c, u, axes=(1, 0))
    cF = np.tensordot(c, F, axes=(1, 0))
    uF = (u * F).sum(axis=0)
    w = lat.w.reshape((lat.Q,) + (1,) * (u.ndim - 1))
    return w * ((cF - uF) / CS2 + cu * cF / (CS2 * CS2))


def gaussian_raw_moment(exps, rho, u):
    """Raw moment of the continuous Maxwellian (Eqs. 7-8), truncated at O(u^2).

    For a monomial x^a y^b z^c the Maxwellian factorises per axis into
    E[xi^e] with E[xi^0]=1, E[xi]=u, E[xi^2]=c_s^2+u^2 (e <= 2 suffices on
    first-neighbour stencils).  The product is expanded and every term of
    total degree > 2 in u is dropped.  Exact rationals in, exact rationals out
    when ``rho`` and ``u`` are ``Fraction`` objects.
    """
    # per-axis polynomial in u_a as {degree: coefficient}
    per_axis = []
    for e in exps:
        if e == 0:
            per_axis.append({0: Fraction(1)})
        elif e == 1:
            per_axis.append({1: Fraction(1)})
        elif e == 2:
            per_axis.append({0: CS2_EXACT, 2: Fraction(1)})
        else:
            raise ValueError("exponent > 2 aliases a lower moment")
    total = 0
    for combo in itertools.product(*[sorted(p.items()) for p in per_axis]):
        deg = sum(dg for dg, _ in combo)
        if deg > 2:
            continue
        term = rho
        for axis, (dg, coef) in enumerate(combo):
            term = term * coef * (u[axis] ** dg)
        total = total + term
    return total
