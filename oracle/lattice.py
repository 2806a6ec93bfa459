"""Velocity sets (test infrastructure only; see ``oracle/__init__.py``).

Sec. III-A: a DdQq stencil is a sequence of integer velocity vectors; each
cell holds q populations f_q.  The paper prints neither the weights nor a
direction order.  Reading used here: the standard lattice weights of the
first-neighbourhood sets, speed of sound c_s^2 = 1/3 (Sec. III-A, "Equilibrium
State"), and this direction order:

    index 0          the rest vector
    indices 1..h     one vector of each +/- pair (the list below)
    indices h+1..2h  their negatives, so opp(q) = q +/- h with h = (Q-1)/2

Vectors are always stored with three components (c_z = 0 for D2Q9) so that
one 3-D code path serves every stencil.
"""

from collections import namedtuple
from fractions import Fraction

import numpy as np

CS2 = 1.0 / 3.0                 # lattice speed of sound squared, float
CS2_EXACT = Fraction(1, 3)      # same, exact

_HALF = {
    "D2Q9": [(1, 0, 0), (0, 1, 0), (1, 1, 0), (1, -1, 0)],
    "D3Q19": [(1, 0, 0), (0, 1, 0), (0, 0, 1),
              (1, 1, 0), (1, -1, 0), (1, 0, 1), (1, 0, -1), (0, 1, 1), (0, 1, -1)],
    "D3Q27": [(1, 0, 0), (0, 1, 0), (0, 0, 1),
              (1, 1, 0), (1, -1, 0), (1, 0, 1), (1, 0, -1), (0, 1, 1), (0, 1, -1),
              (1, 1, 1), (1, 1, -1), (1, -1, 1), (1, -1, -1)],
}

# standard weights by squared speed |c|^2
_WEIGHTS = {
    "D2Q9": {0: Fraction(4, 9), 1: Fraction(1, 9), 2: Fraction(1, 36)},
    "D3Q19": {0: Fraction(1, 3), 1: Fraction(1, 18), 2: Fraction(1, 36)},
    "D3Q27": {0: Fraction(8, 27), 1: Fraction(2, 27), 2: Fraction(1, 54), 3: Fraction(1, 216)},
}

Lattice = namedtuple("Lattice", "name d Q c w wf opp")


def velocity_set(name):
    """Return the ``Lattice`` for ``name`` in {"D2Q9", "D3Q19", "D3Q27"}."""
    half = _HALF[name]
    vecs = [(0, 0, 0)] + half + [tuple(-v for v in h) for h in half]
    c = np.array(vecs, dtype=np.int64)
    Q = len(vecs)
    h = len(half)
    wf = [_WEIGHTS[name][int((v * v).sum())] for v in c]
    w = np.array([float(x) for x in wf])
    opp = np.array([0] + [q + h for q in range(1, h + 1)] + [q - h for q in range(h + 1, Q)])
    d = 2 if name == "D2Q9" else 3
    return Lattice(name, d, Q, c, w, wf, opp)
