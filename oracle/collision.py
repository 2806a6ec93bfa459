"""Collision operators (test infrastructure only; see ``oracle/__init__.py``).

Every operator maps pre-collision populations f (shape (Q, ...)) to
post-collision populations, in float64, with no blocking or fusion.

Rates are passed as a plain dict with keys
    omega       SRT rate; TRT even rate; MRT/cumulant shear rate
    omega_bulk  MRT/cumulant bulk rate
    omega_odd   TRT odd rate (<= 0: derived from ``magic``)
    magic       TRT parameter Lambda = (1/omega_e - 1/2)(1/omega_o - 1/2)
    omega_hi    MRT/cumulant rates of the moment orders 3, 4, 5, 6
    cs_smag     Smagorinsky constant C_S (optional; > 0 makes the SRT rate and
                the MRT shear rate local)
"""

import functools
import math

import numpy as np

from .equilibrium import equilibrium, guo_source, macroscopic
from .lattice import CS2
from .moments import monomial_exponents, orthogonal_mrt_basis, raw_moment_matrix


def trt_odd_rate(rates):
    """Odd TRT rate: given directly, or from Lambda = (1/w_e - 1/2)(1/w_o - 1/2)."""
    if rates.get("omega_odd", 0.0) > 0.0:
        return rates["omega_odd"]
    we = rates["omega"]
    return 1.0 / (rates["magic"] / (1.0 / we - 0.5) + 0.5)


def nonequilibrium_stress(lat, f, feq):
    """Pi^neq_ab = sum_q c_qa c_qb (f_q - f^eq_q) (Sec. III-C, Eq. 13);
    returns an array (3, 3, ...)."""
    c = lat.c.astype(np.float64)
    d = f - feq
    return np.einsum("qa,qb,q...->ab...", c, c, d)


def smagorinsky_rate(lat, f, feq, rho, omega0, cs):
    """Local relaxation rate of the Smagorinsky model (Sec. III-C, Eqs. 11-14).

    nu = nu_0 + (C_S Delta)^2 |S| with Delta = 1, |S| = sqrt(2 S:S),
    S = -3 omega / (2 rho) Pi^neq and omega = 2 / (6 nu + 1).  With
    P = sqrt(2 Pi^neq : Pi^neq) this is the quadratic
    (9 C_S^2 P / rho) omega^2 + 2 tau_0 omega - 2 = 0 (tau_0 = 1 / omega_0),
    whose positive root is returned.
    """
    Pi = nonequilibrium_stress(lat, f, feq)
    P = np.sqrt(2.0 * (Pi * Pi).sum(axis=(0, 1)))
    tau0 = 1.0 / omega0
    a = 9.0 * cs * cs * P / rho
    disc = np.sqrt(tau0 * tau0 + 2.0 * a)
    return np.where(a > 0, (disc - tau0) / np.where(a > 0, a, 1.0), 1.0 / tau0)


def srt(lat, f, rates, force=None, rho0=1.0, compressible=True):
    """Eq. (1): f* = f - omega (f - f^eq), plus Guo's (1 - omega/2) S; with
    C_S > 0 omega is the local Smagorinsky rate."""
    om = rates["omega"]
    rho, u = macroscopic(lat, f, force, rho0, compressible)
    feq = equilibrium(lat, rho, u, rho0, compressible)
    if rates.get("cs_smag", 0.0) > 0.0:
        om = smagorinsky_rate(lat, f, feq, rho, om, rates["cs_smag"])
    out = f - om * (f - feq)
    if force is not None:
        out = out + (1.0 - 0.5 * om) * guo_source(lat, u, force)
    return out


def trt(lat, f, rates, force=None, rho0=1.0, compressible=True):
    """TRT (Sec. III-C): even moments relax with omega_e, odd with omega_o.

    Written in the equivalent population form: even moments vanish on the
    antisymmetric part f^- = (f_q - f_opp(q))/2 and odd moments on the
    symmetric part f^+, so relaxing the two parts with omega_e / omega_o is
    the same operator.  The Guo source is split the same way.
    """
    we = rates["omega"]
    wo = trt_odd_rate(rates)
    rho, u = macroscopic(lat, f, force, rho0, compressible)
    feq = equilibrium(lat, rho, u, rho0, compressible)
    o = lat.opp
    fp, fm = 0.5 * (f + f[o]), 0.5 * (f - f[o])
    ep, em = 0.5 * (feq + feq[o]), 0.5 * (feq - feq[o])
    out = f - we * (fp - ep) - wo * (fm - em)
    if force is not None:
        S = guo_source(lat, u, force)
        out = out + (1.0 - 0.5 * we) * 0.5 * (S + S[o]) + (1.0 - 0.5 * wo) * 0.5 * (S - S[o])
    return out


def maxwellian_moments(exps, rho, u):
    """Float version of ``equilibrium.gaussian_raw_moment`` over cell arrays:
    per-axis Maxwellian moments (1, u_a, c_s^2 + u_a^2) multiplied out with
    every term above second order in u dropped."""
    out = []
    for e in exps:
        terms = [(0, np.ones_like(rho))]
        for a, ea in enumerate(e):
            if ea == 0:
                fac = [(0, 1.0)]
            elif ea == 1:
                fac = [(1, u[a])]
            else:
                fac = [(0, CS2), (2, u[a] * u[a])]
            terms = [(d1 + d2, t1 * t2) for d1, t1 in terms for d2, t2 in fac if d1 + d2 <= 2]
        out.append(rho * sum(t for _, t in terms))
    return np.array(out)


def trt_moment_form(lat, f, rates):
    """TRT exactly as the paper builds it (Sec. III-C "SRT, TRT"): raw
    monomial moments, Maxwellian equilibrium moments truncated at O(u^2), rate
    omega_e for even and omega_o for odd moments, then Eq. (4).  No forcing.
    Used as an independent cross-check of ``trt``."""
    M, exps = raw_moment_matrix(lat)
    we, wo = rates["omega"], trt_odd_rate(rates)
    s = np.array([we if sum(e) % 2 == 0 else wo for e in exps])
    rho, u = macroscopic(lat, f)
    meq = maxwellian_moments(exps, rho, u)
    shp = f.shape
    m = M @ f.reshape(lat.Q, -1)
    post = m - s[:, None] * (m - meq.reshape(lat.Q, -1))
    return np.linalg.solve(M, post).reshape(shp)


def _group_rates(groups, rates):
    table = {"o0": 0.0, "o1": 0.0, "shear": rates["omega"], "bulk": rates["omega_bulk"]}
    for k in range(4):
        table["o%d" % (k + 3)] = rates["omega_hi"][k]
    return np.array([table[g] for g in groups])


@functools.lru_cache(maxsize=None)
def _mrt_tables(name):
    from .lattice import velocity_set
    lat = velocity_set(name)
    M, groups, _ = orthogonal_mrt_basis(lat)
    return M, tuple(groups), np.linalg.inv(M)


def mrt(lat, f, rates, force=None, rho0=1.0, compressible=True):
    """Eq. (4) with the weighted-orthogonal basis of ``moments`` (with C_S > 0
    the shear rate is the local Smagorinsky rate).

    m = M f, m^eq = M f^eq (Eq. 3), f* = f - M^-1 S (m - m^eq); the Guo
    source enters in moment space as M^-1 (I - S/2) M S.  Conserved moments
    (orders 0, 1) get rate 0, as in the paper's MRT table; with Guo forcing
    their rate does not change the result.
    """
    M, groups, Minv = _mrt_tables(lat.name)
    shp = f.shape
    rho, u = macroscopic(lat, f, force, rho0, compressible)
    feq = equilibrium(lat, rho, u, rho0, compressible)
    f2 = f.reshape(lat.Q, -1)
    s = np.repeat(_group_rates(groups, rates)[:, None], f2.shape[1], axis=1)
    if rates.get("cs_smag", 0.0) > 0.0:
        om = smagorinsky_rate(lat, f, feq, rho, rates["omega"], rates["cs_smag"]).reshape(-1)
        for k, g in enumerate(groups):
            if g == "shear":
                s[k] = om
    neq = M @ (f2 - feq.reshape(lat.Q, -1))
    out = f2 - Minv @ (s * neq)
    if force is not None:
        S = guo_source(lat, u, force).reshape(lat.Q, -1)
        out = out + Minv @ ((1.0 - 0.5 * s) * (M @ S))
    return out.reshape(shp)


def set_partitions(items):
    """All set partitions of the list ``items`` (blocks are lists)."""
    if not items:
        yield []
        return
    first, rest = items[0], items[1:]
    for part in set_partitions(rest):
        for i in range(len(part)):
            yield part[:i] + [[first] + part[i]] + part[i + 1:]
        yield [[first]] + part


@functools.lru_cache(maxsize=None)
def _partitions_of(e):
    """Set partitions of the multiset x^a y^b z^c, each block returned as
    its own exponent triple."""
    labels = [0] * e[0] + [1] * e[1] + [2] * e[2]
    out = []
    for part in set_partitions(list(range(len(labels)))):
        blocks = []
        for blk in part:
            cnt = [0, 0, 0]
            for pos in blk:
                cnt[labels[pos]] += 1
            blocks.append(tuple(cnt))
        out.append(tuple(blocks))
    return tuple(out)


def cumulants_from_moments(mu, exps):
    """Faa di Bruno / moment-cumulant relation (Sec. III-B).

    ``mu[e]`` are raw moments of the normalised distribution f/rho.  For
    order >= 1: kappa_S = sum over set partitions pi of S of
    (-1)^(|pi|-1) (|pi|-1)! prod_{B in pi} mu_B.
    """
    kap = {}
    for e in exps:
        if sum(e) == 0:
            continue
        tot = 0.0
        for blocks in _partitions_of(e):
            k = len(blocks)
            term = (-1.0) ** (k - 1) * math.factorial(k - 1)
            prod = 1.0
            for b in blocks:
                prod = prod * mu[b]
            tot = tot + term * prod
        kap[e] = tot
    return kap


def moments_from_cumulants(kap, exps):
    """Inverse relation: mu_S = sum over set partitions of prod kappa_B."""
    mu = {}
    for e in exps:
        if sum(e) == 0:
            mu[e] = 1.0
            continue
        tot = 0.0
        for blocks in _partitions_of(e):
            prod = 1.0
            for b in blocks:
                prod = prod * kap[b]
            tot = tot + prod
        mu[e] = tot
    return mu


def cumulant(lat, f, rates, force=None, rho0=1.0, compressible=True):
    """Cumulant collision (Sec. III-B, Eq. 9), D2Q9 and D3Q27.

    populations -> raw moments m_e = sum c^e f (all exponents <= 2)
    -> cumulants of f/rho (partition formula) -> relaxation
    kappa* = kappa + omega (kappa^eq - kappa) with the Maxwellian
    equilibrium: kappa^eq = u (order 1, conserved), c_s^2 delta (order 2),
    0 (order >= 3).  Order 2 is split into shear (off-diagonal and deviatoric
    diagonal, rate omega) and bulk (trace, rate omega_bulk); order n >= 3
    uses omega_hi[n-3].  Then cumulants -> moments -> populations by the
    inverse of the monomial moment matrix.
    """
    if force is not None:
        raise NotImplementedError("forcing is not defined for the cumulant operator here")
    if not compressible:
        raise NotImplementedError("the cumulant operator is compressible by construction")
    if lat.name not in ("D2Q9", "D3Q27"):
        raise NotImplementedError("cumulant collision needs a tensor-product stencil")
    M, exps = raw_moment_matrix(lat)
    shp = f.shape
    f2 = f.reshape(lat.Q, -1)
    m = M @ f2
    rho = m[exps.index((0, 0, 0))]
    mu = {e: m[i] / rho for i, e in enumerate(exps)}
    kap = cumulants_from_moments(mu, exps)
    om_s, om_b, hi = rates["omega"], rates["omega_bulk"], rates["omega_hi"]
    D = lat.d
    post = {}
    diag = [e for e in exps if sum(e) == 2 and max(e) == 2]
    tr = sum(kap[e] for e in diag)
    tr_post = tr + om_b * (D * CS2 - tr)
    for e in exps:
        n = sum(e)
        if n == 0:
            continue
        if n == 1:
            post[e] = kap[e]
        elif n == 2 and max(e) == 1:
            post[e] = kap[e] - om_s * kap[e]
        elif n == 2:
            dev = kap[e] - tr / D
            post[e] = (1.0 - om_s) * dev + tr_post / D
        else:
            post[e] = kap[e] - hi[n - 3] * kap[e]
    mu_post = moments_from_cumulants(post, exps)
    m_post = np.array([rho * mu_post[e] for e in exps])
    return np.linalg.solve(M, m_post).reshape(shp)


def kbc_parts(lat, f, rates, force=None, rho0=1.0, compressible=True):
    """Pieces of the entropic KBC-type collision (Sec. III-C "Entropic KBC
    Models").

    The method is the weighted-orthogonal MRT of ``mrt`` with two kinds of
    rates: fixed ones for the second-order moments (shear omega, bulk
    omega_bulk) and one rate omega_h for every moment of order >= 3, chosen
    per cell.  The non-equilibrium f - f^eq is split by projecting onto the
    basis groups: ds (shear), db (bulk), dh (orders >= 3); the conserved
    orders carry none without a force (with Guo's force the order-1 part is
    the half-force shift, which no rate acts on).  The post-collision state
    f' = f - omega ds - omega_b db - omega_h dh.  omega_h makes the entropy
    -sum f' ln(f'/f^eq) stationary with ln x replaced by x - 1, i.e.
    sum_q dh_q f'_q / f^eq_q = 0, whose solution is
        omega_h = 1 + [(1 - omega) <ds, dh>_E + (1 - omega_b) <db, dh>_E] / <dh, dh>_E
    with <a, b>_E = sum_q a_q b_q / f^eq_q.  For omega_b = omega this is the
    paper's closed form; keeping the bulk moments in their own group with
    their own fixed rate is the reading used here.  <dh, dh>_E = 0 (no
    higher-order non-equilibrium) gives omega_h = 1.  The correction
    (omega_h - 1) dh is the E-projection of (1 - omega) ds + (1 - omega_b) db
    onto the line of dh: its size does not vanish with dh, so the operator
    has no limit at dh = 0 and results at rounding-level dh depend on the
    rounding.  The paper adds no safeguard, and none is added here.

    Returns (ds, db, dh, feq, omega_h, rho, u), populations as (Q, ncells).
    """
    M, groups, Minv = _mrt_tables(lat.name)
    rho, u = macroscopic(lat, f, force, rho0, compressible)
    feq = equilibrium(lat, rho, u, rho0, compressible).reshape(lat.Q, -1)
    m = M @ (f.reshape(lat.Q, -1) - feq)

    def part(keep):
        rows = [k for k, g in enumerate(groups) if keep(g)]
        return Minv[:, rows] @ m[rows]

    ds = part(lambda g: g == "shear")
    db = part(lambda g: g == "bulk")
    dh = part(lambda g: g not in ("o0", "o1", "shear", "bulk"))

    def dot_e(a, b):
        return (a * b / feq).sum(axis=0)

    hh = dot_e(dh, dh)
    num = (1.0 - rates["omega"]) * dot_e(ds, dh) + (1.0 - rates["omega_bulk"]) * dot_e(db, dh)
    omh = np.where(hh > 0, 1.0 + num / np.where(hh > 0, hh, 1.0), 1.0)
    return ds, db, dh, feq, omh, rho, u


def kbc(lat, f, rates, force=None, rho0=1.0, compressible=True):
    """Entropic KBC-type collision (Sec. III-C "Entropic KBC Models"); see
    ``kbc_parts``.  Guo forcing as in ``mrt``: the source lies in orders 1
    and 2 only, so it enters with the fixed rates and never with omega_h."""
    shp = f.shape
    ds, db, dh, feq, omh, rho, u = kbc_parts(lat, f, rates, force, rho0, compressible)
    out = f.reshape(lat.Q, -1) - rates["omega"] * ds - rates["omega_bulk"] * db - omh * dh
    if force is not None:
        M, groups, Minv = _mrt_tables(lat.name)
        s = _group_rates(groups, dict(rates, omega_hi=(0.0, 0.0, 0.0, 0.0)))
        S = guo_source(lat, u, force).reshape(lat.Q, -1)
        out = out + Minv @ ((1.0 - 0.5 * s)[:, None] * (M @ S))
    return out.reshape(shp)


OPERATORS = {"SRT": srt, "TRT": trt, "MRT": mrt, "CUMULANT": cumulant, "KBC": kbc}


def collide(method, lat, f, rates, force=None, rho0=1.0, compressible=True):
    """Dispatch on the method name."""
    return OPERATORS[method](lat, f, rates, force, rho0, compressible)
