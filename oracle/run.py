"""Initialisation, time stepping, readout, storage rounding (test
infrastructure only; see ``oracle/__init__.py``).

State: post-collision populations P with shape (Q, nz, ny, nx).  One time
step is pull streaming (with bounce-back) followed by the collision at every
fluid cell; solid cells keep their values and are never read by fluid cells.

Readout convention (reading; the paper does not fix it): the stored state is
post-collision, so rho = sum P and u = (sum c P - F/2)/rho, which equals the
Guo velocity used in the collision that produced P.  Solid cells read out
rho = u = 0.

Shifted storage (not in the paper): the stored quantity is
P - w_q rho_0, rounded to nearest-even in the storage type after every
write.  ``quantize`` emulates that rounding in float64.
"""

import numpy as np

from .collision import collide
from .equilibrium import density_momentum, equilibrium
from .lattice import velocity_set
from .stream import gather_at, stream_pull


class Config:
    """Plain description of one run (the oracle's own, independent of any
    binding): stencil, method, rates, reference density, compressibility,
    storage type name ("f64", "f32", "bf16", "f16")."""

    def __init__(self, stencil, method, rates, rho0=1.0, compressible=True, storage="f64"):
        self.lat = velocity_set(stencil)
        self.method = method
        self.rates = dict(rates)
        self.rho0 = float(rho0)
        self.compressible = bool(compressible)
        self.storage = storage


def force_field(force, dims):
    """Broadcast a force given as None, (3,) or a per-y profile (ny, 3) to an
    array of shape (3, nz, ny, nx) (or None)."""
    if force is None:
        return None
    nx, ny, nz = dims
    F = np.asarray(force, dtype=np.float64)
    if F.shape == (3,):
        return np.broadcast_to(F.reshape(3, 1, 1, 1), (3, nz, ny, nx)).copy()
    if F.shape == (ny, 3):
        return np.broadcast_to(F.T.reshape(3, 1, ny, 1), (3, nz, ny, nx)).copy()
    raise ValueError("force must be (3,) or (ny, 3)")


# ---------------------------------------------------------------- rounding
def round_bf16(x):
    """Round float64 values to the nearest bfloat16 (8 significant bits),
    ties to even, with the float32 exponent range (no overflow handling)."""
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)                       # x = m 2^e, 0.5 <= |m| < 1
    r = np.ldexp(np.rint(np.ldexp(m, 8)), e - 8)
    # below the smallest normal bf16 the spacing is fixed at 2^-133
    tiny = np.abs(x) < 2.0 ** -126
    r = np.where(tiny, np.ldexp(np.rint(np.ldexp(x, 133)), -133), r)
    return r


def round_storage(x, storage):
    """Round-to-nearest-even into the storage type, returned as float64."""
    if storage == "f64":
        return np.asarray(x, dtype=np.float64)
    if storage == "f32":
        return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)
    if storage == "f16":
        return np.asarray(x, dtype=np.float64).astype(np.float16).astype(np.float64)
    if storage == "bf16":
        return round_bf16(x)
    raise ValueError(storage)


def quantize(cfg, P):
    """Emulate shifted storage: round (P - w rho_0) and add the shift back."""
    if cfg.storage == "f64":
        return P
    w = cfg.lat.w.reshape((cfg.lat.Q,) + (1,) * (P.ndim - 1))
    return round_storage(P - w * cfg.rho0, cfg.storage) + w * cfg.rho0


# ---------------------------------------------------------------- stepping
def init_equilibrium(cfg, rho, u, solid=None):
    """P^0 = f^eq(rho, u) (Eq. 3) at fluid cells, w rho_0 at solid cells;
    then storage rounding.  ``rho``: (nz, ny, nx); ``u``: (3, nz, ny, nx)."""
    P = equilibrium(cfg.lat, rho, u, cfg.rho0, cfg.compressible)
    if solid is not None:
        rest = cfg.lat.w.reshape(-1, 1, 1, 1) * cfg.rho0
        P = np.where(solid[None].astype(bool), rest, P)
    return quantize(cfg, P)


def step(cfg, P, solid=None, force=None, wall_velocity=None):
    """One stream-pull-collide step (two-array pattern).

    ``force``: None or an array (3, nz, ny, nx) from ``force_field``;
    ``wall_velocity``: None or a table (K, 3) indexed by the mask value.
    """
    g = stream_pull(cfg.lat, P, solid, wall_velocity, cfg.rho0)
    post = collide(cfg.method, cfg.lat, g, cfg.rates, force, cfg.rho0, cfg.compressible)
    post = quantize(cfg, post)
    if solid is not None:
        post = np.where(solid[None].astype(bool), P, post)
    return post


def run(cfg, P, nsteps, solid=None, force=None, wall_velocity=None):
    for _ in range(nsteps):
        P = step(cfg, P, solid, force, wall_velocity)
    return P


def readout(cfg, P, solid=None, force=None):
    """rho, u of the stored post-collision state (see module docstring)."""
    rho, j = density_momentum(cfg.lat, P)
    if force is not None:
        j = j - 0.5 * force
    u = j / (rho if cfg.compressible else cfg.rho0)
    if solid is not None:
        s = solid.astype(bool)
        rho = np.where(s, 0.0, rho)
        u = np.where(s[None], 0.0, u)
    return rho, u


def conserved(cfg, P, solid=None):
    """Total mass and momentum of the stored populations over fluid cells."""
    rho, j = density_momentum(cfg.lat, P)
    if solid is not None:
        s = solid.astype(bool)
        rho = np.where(s, 0.0, rho)
        j = np.where(s[None], 0.0, j)
    return np.array([rho.sum(), j[0].sum(), j[1].sum(), j[2].sum()])


def step_at_cells(cfg, P_of, cells, dims, solid=None, force=None, wall_velocity=None):
    """One step evaluated only at ``cells`` (linear indices, x fastest).

    ``P_of(q, idx)`` gives the stored state at linear cell indices.
    ``force`` is None, (3,) or a per-y profile (ny, 3).  Returns (Q, ncells).
    """
    g = gather_at(cfg.lat, P_of, cells, dims, solid, wall_velocity, cfg.rho0)
    F = None
    if force is not None:
        F = np.asarray(force, dtype=np.float64)
        if F.shape == (3,):
            F = np.broadcast_to(F.reshape(3, 1), (3, cells.size))
        else:
            y = (cells // dims[0]) % dims[1]
            F = F[y].T
    post = collide(cfg.method, cfg.lat, g, cfg.rates, F, cfg.rho0, cfg.compressible)
    return quantize(cfg, post)
