"""Streaming and bounce-back (test infrastructure only).

Lattice arrays have shape (Q, nz, ny, nx): x is the last axis.  Sec. IV-B
(Fig. "stream-pull-collide"): with two arrays, cell x pulls population q
from its upstream neighbour, g_q(x) = P(x - c_q, q), with periodic wrap.
Halfway bounce-back for a resting wall (Sec. III-C "Boundary Conditions",
wall velocity zero; the link direction points from the fluid cell to the
wall): when x - c_q is solid the missing population is the cell's own
outgoing population in the opposite direction, g_q(x) = P(x, opp(q)).
"""

import numpy as np


def _shift(a, c):
    """Return b with b(x) = a(x - c) on a periodic (nz, ny, nx) lattice."""
    return np.roll(a, shift=(int(c[2]), int(c[1]), int(c[0])), axis=(-3, -2, -1))


def stream_pull(lat, P, solid=None):
    """Pull streaming with periodic wrap and halfway bounce-back."""
    g = np.empty_like(P)
    for q in range(lat.Q):
        g[q] = _shift(P[q], lat.c[q])
        if solid is not None:
            from_solid = _shift(solid, lat.c[q])
            g[q] = np.where(from_solid, P[lat.opp[q]], g[q])
    return g


def gather_at(lat, P_of, cells, dims, solid=None):
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
            bb = solid.reshape(-1)[src].astype(bool)
            if bb.any():
                own = P_of(int(lat.opp[q]), cells)
                val = np.where(bb, own, val)
        g[q] = val
    return g
