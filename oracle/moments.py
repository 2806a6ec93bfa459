"""Moment bases (test infrastructure only; see ``oracle/__init__.py``).

Sec. III-A "Moment Space": a moment is sum_q P(c_q) f_q for a polynomial P in
the velocity components (Eq. 5); the moment matrix is M_kq = P_k(c_q).  On
first-neighbour stencils exponents above 2 alias lower ones, so candidate
monomials are x^a y^b z^c with a, b, c in {0, 1, 2}; on D3Q19 the 8 monomials
that vanish on every direction are dropped.  Sec. III-C "MRT": the second
order monomials are split into a bulk part (x^2+y^2+z^2) and shear parts
before a Gram-Schmidt orthogonalisation, here with the lattice-weighted
product <p, r>_w = sum_q w_q p(c_q) r(c_q).  Inputs are sorted by order.

All basis construction is done in exact rationals (``fractions.Fraction``).
"""

import itertools
from fractions import Fraction

import numpy as np


def monomial_exponents(lat):
    """Non-aliased monomial exponents (a, b, c), each in {0,1,2}, that give a
    non-zero row on ``lat``, sorted by order then lexicographically."""
    axes = [range(3)] * lat.d + [range(1)] * (3 - lat.d)
    out = []
    for e in itertools.product(*axes):
        row = [int(np.prod([int(cq[i]) ** e[i] for i in range(3)])) for cq in lat.c]
        if any(row):
            out.append(tuple(e))
    out.sort(key=lambda e: (sum(e), e))
    return out


def monomial_row(lat, e):
    """Exact row P(c_q) for the monomial with exponents ``e``."""
    return [Fraction(int(np.prod([int(cq[i]) ** e[i] for i in range(3)]))) for cq in lat.c]


def raw_moment_matrix(lat):
    """Monomial moment matrix (float) and its exponent list."""
    exps = monomial_exponents(lat)
    M = np.array([[float(v) for v in monomial_row(lat, e)] for e in exps])
    return M, exps


def split_shear_bulk(lat, exps):
    """Replace the diagonal second-order monomials by the bulk moment
    x^2+y^2(+z^2) and the shear differences x^2-y^2 (, x^2-z^2); the
    off-diagonal second-order monomials stay and are shear moments.

    Returns a list of (row, group) with group in
    {"o0", "o1", "shear", "bulk", "o3", "o4", "o5", "o6"}.
    """
    rows = []
    diag = [e for e in exps if sum(e) == 2 and max(e) == 2]
    for e in exps:
        order = sum(e)
        if order == 2:
            continue
        rows.append((monomial_row(lat, e), "o%d" % order))
    second = []
    off = [e for e in exps if sum(e) == 2 and max(e) == 1]
    dr = [monomial_row(lat, e) for e in diag]
    for k in range(1, len(dr)):
        second.append(([a - b for a, b in zip(dr[0], dr[k])], "shear"))
    for e in off:
        second.append((monomial_row(lat, e), "shear"))
    second.append(([sum(col) for col in zip(*dr)], "bulk"))
    # keep the order-sorted sequence: orders 0, 1, then 2 (shear, bulk), then 3+
    low = [r for r in rows if r[1] in ("o0", "o1")]
    high = [r for r in rows if r[1] not in ("o0", "o1")]
    return low + second + high


def weighted_gram_schmidt(lat, rows):
    """Gram-Schmidt over rows (lists of Fractions) with <p,r>_w = sum w p r.

    Returns new rows, each orthogonal (in the weighted product) to every
    earlier row.  Exact arithmetic.
    """
    w = lat.wf
    out = []
    for r in rows:
        v = list(r)
        for u in out:
            num = sum(wi * vi * ui for wi, vi, ui in zip(w, v, u))
            den = sum(wi * ui * ui for wi, ui in zip(w, u))
            v = [vi - num / den * ui for vi, ui in zip(v, u)]
        out.append(v)
    return out


def orthogonal_mrt_basis(lat):
    """Weighted-orthogonal MRT basis (Sec. III-C "MRT").

    Returns (M, groups): M is a (Q, Q) float matrix whose rows are w-orthogonal
    polynomials evaluated on the stencil, ``groups`` the rate group of each row.
    """
    exps = monomial_exponents(lat)
    split = split_shear_bulk(lat, exps)
    rows = weighted_gram_schmidt(lat, [r for r, _ in split])
    M = np.array([[float(v) for v in r] for r in rows])
    groups = [g for _, g in split]
    return M, groups, rows
