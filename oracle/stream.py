"""Streaming and bounce-back (test infrastructure only).

Lattice arrays have shape (Q, nz, ny, nx): x is the last axis.  Sec. IV-B
(Fig. "stream-pull-collide"): with two arrays, cell x pulls population q
from its upstream neighbour, g_q(x) = P(x - c_q, q), with periodic wrap.
Halfway velocity bounce-back (Sec. III-C "Boundary Conditions"): when
x - c_q is solid the missing population is the cell's own outgoing
population in the opposite direction minus 2 w (c . u_w) / c_s^2, where c
points from the fluid cell to the wall (here c = -c_q) and u_w is the wall
velocity: g_q(x) = P(x, opp(q)) + 2 w_q rho_0 (c_q . u_w) / c_s^2.  The
paper's rule carries no density factor; rho_0 (1 in all workloads) is the
reading used for other reference densities.  Mask values: 0 fluid, 1 resting
wall, k >= 2 a moving wall whose velocity is row k of a velocity table.
"""

import numpy as np

from .lattice import CS2


def _shift(a, c):
    """Return b with b(x) = a(x - c) on a periodic (nz, ny, nx) lattice."""
    return np.roll(a, shift=(int(c[2]), int(c[1]), int(c[0])), axis=(-3, -2, -1))


def wall_term(lat, q, wall_id, wall_velocity, rho0):
    """2 w_q rho_0 (c_q . u_w) / c_s^2 for the wall type(s) ``wall_id``."""
    if wall_velocity is None:
        return 0.0
    uw = np.asarray(wall_velocity, dtype=np.float64)[np.asarray(wall_id, dtype=np.int64)]
    return 2.0 * lat.w[q] * rho0 * (uw @ lat.c[q].astype(np.float64)) / CS2


def stream_pull(lat, P, solid=None, wall_velocity=None, rho0=1.0):
    """Pull streaming with periodic wrap and halfway (velocity) bounce-back.

    ``solid``: mask (nz, ny, nx), 0 fluid, >= 1 solid; ``wall_velocity``:
    table (K, 3) indexed by the mask value, or None (all walls at rest)."""
    g = np.empty_like(P)
    for q in range(lat.Q):
        g[q] = _shift(P[q], lat.c[q])
        if solid is not None:
            src = _shift(solid, lat.c[q])
            g[q] = np.where(src != 0, P[lat.opp[q]] + wall_term(lat, q, src, wall_velocity, rho0), g[q])
    return g


def gather_at(lat, P_of, cells, dims, solid=None, wall_velocity=None, rho0=1.0):
    """Pull-gather for a list of cells only.

    ``P_of(q, cellidx)`` returns population q at linear cell indices
    (x fastest); ``cells`` is an int array of linear indices; ``dims`` is
    (nx, ny, nz).  Same rule as ``stream_pull``; used to check single cells
    of very large lattices without building the whole array.
    """
    nx, ny, nz = dims
    x = cells % nx
    y = (cells // nx) % ny
    z = cells // (nx * ny)
    g = np.empty((lat.Q, cells.size))
    for q in range(lat.Q):
        cx, cy, cz = (int(v) for v in lat.c[q])
        src = ((z - cz) % nz * ny + (y - cy) % ny) * nx + (x - cx) % nx
        val = P_of(q, src)
        if solid is not None:
            sid = solid.reshape(-1)[src]
            bb = sid != 0
            if bb.any():
                own = P_of(int(lat.opp[q]), cells) + wall_term(lat, q, sid, wall_velocity, rho0)
                val = np.where(bb, own, val)
        g[q] = val
    return g
