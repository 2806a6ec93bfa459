// Plain FP64 CPU oracle of the lattice Boltzmann stream-collide step, in C++17
// with OpenMP over lattice rows.
//
// TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the CPU
// baseline of the benchmark load this library.  It shares no code, tables or
// constants with the HIP library, and it is written for clarity, not speed:
// one cell at a time, the method's steps in the order the paper states them,
// dense loops over directions and moments, double precision throughout.  The
// same source also builds with long double (64-bit significand) for every
// value and argument: that build serves only to measure how far the FP64
// oracle's own rounding moves a result.
//
// What it computes (paper: "lbmpy: Automatic code generation for efficient
// parallel lattice Boltzmann methods"):
//   - DdQq velocity sets with the standard weights and c_s^2 = 1/3
//     (Sec. III-A).  Direction order: rest vector first, then one vector of
//     each +/- pair, then their negatives (opp(q) = q +/- h);
//   - pull streaming with periodic wrap and halfway velocity bounce-back
//     (Sec. IV-B, Fig. "stream-pull-collide"; Sec. III-C "Boundary
//     Conditions"): g_q(x) = P(x - c_q, q), or P(x, opp q) + 2 w_q rho_0
//     (c_q . u_w) / c_s^2 when x - c_q is solid;
//   - density and velocity (Eq. 2) with Guo's half-force shift, the
//     second-order equilibrium (Eq. 3), Guo's source term;
//   - collisions: SRT (Eq. 1), TRT (Sec. III-C, even / odd parts of each
//     direction pair), MRT (Eq. 4) in the lattice-weighted Gram-Schmidt basis
//     of the monomials sorted by order with the second order split into
//     shear and bulk parts (Sec. III-C "MRT"), cumulants (Eq. 9, Sec. III-B)
//     by the set-partition relation between raw moments and cumulants;
//   - shifted storage emulation (not in the paper): after every write the
//     value P - w_q rho_0 is rounded to nearest-even in FP32, BF16 or FP16.
// State: unshifted post-collision populations P[q][z][y][x] (x fastest).
// Solid cells keep their values and never act as fluid.

#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

// Floating-point type of every value and argument: double, or long double
// (x87 extended, 64-bit significand) in the build that measures the FP64
// rounding floor (-DORC_REAL="long double").
#ifndef ORC_REAL
#define ORC_REAL double
#endif
typedef ORC_REAL real;

namespace {

constexpr real CS2 = real(1) / 3;

// ------------------------------------------------------------------ lattice
struct Lattice {
  int d = 0, Q = 0, h = 0;
  int c[27][3] = {};
  real w[27] = {};
  int opp[27] = {};
};

bool make_lattice(int stencil, Lattice& L) {
  static const int half2[4][3] = {{1, 0, 0}, {0, 1, 0}, {1, 1, 0}, {1, -1, 0}};
  static const int half3[13][3] = {{1, 0, 0},  {0, 1, 0},  {0, 0, 1},  {1, 1, 0},   {1, -1, 0},
                                   {1, 0, 1},  {1, 0, -1}, {0, 1, 1},  {0, 1, -1},  {1, 1, 1},
                                   {1, 1, -1}, {1, -1, 1}, {1, -1, -1}};
  const int(*half)[3];
  if (stencil == 0) {
    L.d = 2;
    L.h = 4;
    half = half2;
  } else if (stencil == 1) {
    L.d = 3;
    L.h = 9;
    half = half3;
  } else if (stencil == 2) {
    L.d = 3;
    L.h = 13;
    half = half3;
  } else {
    return false;
  }
  L.Q = 2 * L.h + 1;
  for (int a = 0; a < 3; ++a) L.c[0][a] = 0;
  for (int i = 0; i < L.h; ++i)
    for (int a = 0; a < 3; ++a) {
      L.c[1 + i][a] = half[i][a];
      L.c[1 + L.h + i][a] = -half[i][a];
    }
  for (int q = 0; q < L.Q; ++q) {
    L.opp[q] = q == 0 ? 0 : (q <= L.h ? q + L.h : q - L.h);
    const int s = L.c[q][0] * L.c[q][0] + L.c[q][1] * L.c[q][1] + L.c[q][2] * L.c[q][2];
    if (stencil == 0) {
      L.w[q] = s == 0 ? real(4) / 9 : (s == 1 ? real(1) / 9 : real(1) / 36);
    } else if (stencil == 1) {
      L.w[q] = s == 0 ? real(1) / 3 : (s == 1 ? real(1) / 18 : real(1) / 36);
    } else {
      L.w[q] = s == 0 ? real(8) / 27 : (s == 1 ? real(2) / 27 : (s == 2 ? real(1) / 54 : real(1) / 216));
    }
  }
  return true;
}

// integer power of a velocity component (exponent 0, 1 or 2)
real ipow(int c, int e) {
  real r = 1.0;
  for (int i = 0; i < e; ++i) r *= c;
  return r;
}

// ------------------------------------------------------------------ config
enum { SRT = 0, TRT = 1, MRT = 2, CUMULANT = 3 };

struct Method {
  Lattice L;
  int method = 0, storage = 0, compressible = 1;
  real omega = 0, omega_bulk = 0, omega_odd = 0, hi[4] = {0, 0, 0, 0}, rho0 = 1;
  // MRT: weighted-orthogonal basis rows M[k][q], their inverse, per-row rate
  std::vector<real> M, Minv, rate;
  // cumulants: monomial exponents and, per exponent, its set partitions
  // (each partition a list of block exponents)
  std::vector<int> ex;                                   // n_ex * 3
  std::vector<std::vector<std::vector<int>>> parts;      // [e][partition] -> block exponent indices
};

// exponent index of (a, b, c) in the cumulant exponent list, -1 if absent
int ex_index(const Method& m, int a, int b, int c) {
  const int n = (int)m.ex.size() / 3;
  for (int i = 0; i < n; ++i)
    if (m.ex[3 * i] == a && m.ex[3 * i + 1] == b && m.ex[3 * i + 2] == c) return i;
  return -1;
}

// Weighted-orthogonal MRT basis (Sec. III-C "MRT"): the monomials x^a y^b z^c
// with exponents in {0, 1, 2} that do not vanish on every direction, sorted by
// order and then lexicographically; the second-order diagonal monomials are
// replaced by the differences x^2 - y^2 (, x^2 - z^2) (shear) and the sum
// x^2 + y^2 (+ z^2) (bulk), the off-diagonal ones stay (shear); then
// Gram-Schmidt with <p, r>_w = sum_q w_q p(c_q) r(c_q).  Rows of order 0 and 1
// are conserved (rate 0), shear rows relax with omega, the bulk row with
// omega_bulk, order n >= 3 with hi[n - 3].  The inverse follows from the
// weighted orthogonality: (M^-1)[q][k] = w_q M[k][q] / <M_k, M_k>_w.
void build_mrt(Method& m) {
  const Lattice& L = m.L;
  const int Q = L.Q;
  struct Row {
    std::vector<real> v;
    int group;   // 0 conserved, 1 shear, 2 bulk, 3.. order
  };
  std::vector<int> exps;   // candidate exponent triples
  const int zmax = L.d == 3 ? 2 : 0;
  for (int order = 0; order <= 6; ++order)
    for (int a = 0; a <= 2; ++a)
      for (int b = 0; b <= 2; ++b)
        for (int c = 0; c <= zmax; ++c) {
          if (a + b + c != order) continue;
          bool nonzero = false;
          for (int q = 0; q < Q; ++q) nonzero |= ipow(L.c[q][0], a) * ipow(L.c[q][1], b) * ipow(L.c[q][2], c) != 0;
          if (!nonzero) continue;
          exps.push_back(a);
          exps.push_back(b);
          exps.push_back(c);
        }
  auto mono = [&](int i) {
    std::vector<real> v(Q);
    for (int q = 0; q < Q; ++q)
      v[q] = ipow(L.c[q][0], exps[3 * i]) * ipow(L.c[q][1], exps[3 * i + 1]) * ipow(L.c[q][2], exps[3 * i + 2]);
    return v;
  };
  const int ne = (int)exps.size() / 3;
  std::vector<Row> low, second, high;
  std::vector<int> diag;
  for (int i = 0; i < ne; ++i) {
    const int ord = exps[3 * i] + exps[3 * i + 1] + exps[3 * i + 2];
    const int mx = std::max(exps[3 * i], std::max(exps[3 * i + 1], exps[3 * i + 2]));
    if (ord <= 1) low.push_back({mono(i), 0});
    else if (ord == 2 && mx == 2) diag.push_back(i);
    else if (ord >= 3) high.push_back({mono(i), ord});
  }
  std::vector<real> d0 = mono(diag[0]);
  for (size_t k = 1; k < diag.size(); ++k) {
    std::vector<real> dk = mono(diag[k]), v(Q);
    for (int q = 0; q < Q; ++q) v[q] = d0[q] - dk[q];
    second.push_back({v, 1});
  }
  for (int i = 0; i < ne; ++i) {
    const int ord = exps[3 * i] + exps[3 * i + 1] + exps[3 * i + 2];
    const int mx = std::max(exps[3 * i], std::max(exps[3 * i + 1], exps[3 * i + 2]));
    if (ord == 2 && mx == 1) second.push_back({mono(i), 1});
  }
  std::vector<real> bulk(Q, 0.0);
  for (int i : diag) {
    std::vector<real> v = mono(i);
    for (int q = 0; q < Q; ++q) bulk[q] += v[q];
  }
  second.push_back({bulk, 2});
  std::vector<Row> rows = low;
  rows.insert(rows.end(), second.begin(), second.end());
  rows.insert(rows.end(), high.begin(), high.end());
  // weighted Gram-Schmidt
  for (size_t k = 0; k < rows.size(); ++k)
    for (size_t j = 0; j < k; ++j) {
      real num = 0, den = 0;
      for (int q = 0; q < Q; ++q) {
        num += L.w[q] * rows[k].v[q] * rows[j].v[q];
        den += L.w[q] * rows[j].v[q] * rows[j].v[q];
      }
      for (int q = 0; q < Q; ++q) rows[k].v[q] -= num / den * rows[j].v[q];
    }
  m.M.assign((size_t)Q * Q, 0.0);
  m.Minv.assign((size_t)Q * Q, 0.0);
  m.rate.assign(Q, 0.0);
  for (int k = 0; k < Q; ++k) {
    real dk = 0;
    for (int q = 0; q < Q; ++q) {
      m.M[(size_t)k * Q + q] = rows[k].v[q];
      dk += L.w[q] * rows[k].v[q] * rows[k].v[q];
    }
    for (int q = 0; q < Q; ++q) m.Minv[(size_t)q * Q + k] = L.w[q] * rows[k].v[q] / dk;
    const int g = rows[k].group;
    m.rate[k] = g == 0 ? 0.0 : (g == 1 ? m.omega : (g == 2 ? m.omega_bulk : m.hi[g - 3]));
  }
}

// All set partitions of n labelled elements, as restricted growth strings
// (element i goes to block r[i]; r[0] = 0, r[i] <= 1 + max(r[0..i-1])).
void set_partitions(int n, std::vector<std::vector<int>>& out) {
  std::vector<int> r(n, 0);
  if (n == 0) {
    out.push_back(r);
    return;
  }
  while (true) {
    out.push_back(r);
    // next restricted growth string
    int i = n - 1;
    while (i > 0) {
      int mx = 0;
      for (int j = 0; j < i; ++j) mx = std::max(mx, r[j]);
      if (r[i] <= mx) {
        r[i] += 1;
        for (int j = i + 1; j < n; ++j) r[j] = 0;
        break;
      }
      --i;
    }
    if (i == 0) return;
  }
}

// Cumulant tables (Sec. III-B): every exponent (a, b, c), each in {0, 1, 2}
// (c = 0 on D2Q9), and for each the set partitions of the multiset
// {x^a, y^b, z^c}, each block mapped to its own exponent triple.
void build_cumulant(Method& m) {
  const int zmax = m.L.d == 3 ? 2 : 0;
  for (int a = 0; a <= 2; ++a)
    for (int b = 0; b <= 2; ++b)
      for (int c = 0; c <= zmax; ++c) {
        m.ex.push_back(a);
        m.ex.push_back(b);
        m.ex.push_back(c);
      }
  const int ne = (int)m.ex.size() / 3;
  m.parts.resize(ne);
  for (int e = 0; e < ne; ++e) {
    std::vector<int> labels;
    for (int k = 0; k < m.ex[3 * e]; ++k) labels.push_back(0);
    for (int k = 0; k < m.ex[3 * e + 1]; ++k) labels.push_back(1);
    for (int k = 0; k < m.ex[3 * e + 2]; ++k) labels.push_back(2);
    const int n = (int)labels.size();
    if (n == 0) continue;
    std::vector<std::vector<int>> rgs;
    set_partitions(n, rgs);
    for (const auto& r : rgs) {
      int nb = 0;
      for (int v : r) nb = std::max(nb, v + 1);
      std::vector<int> cnt(3 * nb, 0);
      for (int i = 0; i < n; ++i) cnt[3 * r[i] + labels[i]] += 1;
      std::vector<int> blocks;
      for (int b = 0; b < nb; ++b) blocks.push_back(ex_index(m, cnt[3 * b], cnt[3 * b + 1], cnt[3 * b + 2]));
      m.parts[e].push_back(blocks);
    }
  }
}

// ------------------------------------------------------------------ storage
// Round to nearest, ties to even, keeping `bits` significant bits; below
// 2^min_normal the spacing is fixed at 2^quantum (subnormals).
real round_bits(real x, int bits, int min_normal, int quantum) {
  if (x == 0.0 || !std::isfinite(x)) return x;
  if (std::fabs(x) < std::ldexp(1.0, min_normal)) return std::ldexp(std::nearbyint(std::ldexp(x, -quantum)), quantum);
  int e = 0;
  const real mant = std::frexp(x, &e);   // x = mant 2^e, 0.5 <= |mant| < 1
  return std::ldexp(std::nearbyint(std::ldexp(mant, bits)), e - bits);
}

real round_storage(real x, int storage) {
  switch (storage) {
    case 1: return (real)(float)x;                  // FP32 (IEEE conversion rounds to nearest even)
    case 2: return round_bits(x, 8, -126, -133);      // BF16
    case 3: return round_bits(x, 11, -14, -24);       // FP16
    default: return x;
  }
}

// ------------------------------------------------------------------ one cell
// Equilibrium, Eq. (3) at second order:
// f^eq_q = w_q rho + w_q rho_0 [c.u / c_s^2 + (c.u)^2 / (2 c_s^4) - u.u / (2 c_s^2)].
void equilibrium(const Lattice& L, real rho, const real u[3], real r0, real* feq) {
  const real uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  for (int q = 0; q < L.Q; ++q) {
    const real cu = L.c[q][0] * u[0] + L.c[q][1] * u[1] + L.c[q][2] * u[2];
    feq[q] = L.w[q] * rho + L.w[q] * r0 * (cu / CS2 + cu * cu / (2 * CS2 * CS2) - uu / (2 * CS2));
  }
}

// Guo's source without its rate factor:
// S_q = w_q [(c_q - u).F / c_s^2 + (c_q.u)(c_q.F) / c_s^4].
void guo(const Lattice& L, const real u[3], const real F[3], real* S) {
  const real uF = u[0] * F[0] + u[1] * F[1] + u[2] * F[2];
  for (int q = 0; q < L.Q; ++q) {
    const real cu = L.c[q][0] * u[0] + L.c[q][1] * u[1] + L.c[q][2] * u[2];
    const real cF = L.c[q][0] * F[0] + L.c[q][1] * F[1] + L.c[q][2] * F[2];
    S[q] = L.w[q] * ((cF - uF) / CS2 + cu * cF / (CS2 * CS2));
  }
}

// Eq. (2) with Guo's shift: rho = sum g, u = (sum c g + F/2) / rho_0.
void macroscopic(const Method& m, const real* g, const real F[3], real& rho, real u[3]) {
  const Lattice& L = m.L;
  rho = 0;
  real j[3] = {0, 0, 0};
  for (int q = 0; q < L.Q; ++q) {
    rho += g[q];
    for (int a = 0; a < 3; ++a) j[a] += L.c[q][a] * g[q];
  }
  const real den = m.compressible ? rho : m.rho0;
  for (int a = 0; a < 3; ++a) u[a] = (j[a] + 0.5 * F[a]) / den;
}

// Cumulant collision (Eq. 9, Sec. III-B) of one cell.  Raw moments
// m_e = sum_q c^e g_q; cumulants of the normalised distribution by the
// set-partition relation kappa_S = sum_pi (-1)^(|pi|-1) (|pi|-1)! prod_B mu_B;
// relaxation kappa* = kappa + omega (kappa^eq - kappa) towards the Maxwellian
// cumulants (u, c_s^2 delta, 0) with the second order split into shear
// (off-diagonal and deviatoric diagonal) and bulk (trace) parts; raw moments
// back by mu_S = sum_pi prod_B kappa*_B; populations by inverting the
// moment map axis by axis: on each axis (f_-, f_0, f_+) -> (m_0, m_1, m_2) =
// (f_- + f_0 + f_+, f_+ - f_-, f_+ + f_-), whose inverse is
// f_- = (m_2 - m_1)/2, f_0 = m_0 - m_2, f_+ = (m_2 + m_1)/2.
void collide_cumulant(const Method& m, const real* g, real* out) {
  const Lattice& L = m.L;
  const int ne = (int)m.ex.size() / 3;
  real mom[27], mu[27], kap[27], post[27], mup[27];
  for (int e = 0; e < ne; ++e) {
    real s = 0;
    for (int q = 0; q < L.Q; ++q)
      s += ipow(L.c[q][0], m.ex[3 * e]) * ipow(L.c[q][1], m.ex[3 * e + 1]) * ipow(L.c[q][2], m.ex[3 * e + 2]) * g[q];
    mom[e] = s;
  }
  const int e0 = ex_index(m, 0, 0, 0);
  const real rho = mom[e0];
  for (int e = 0; e < ne; ++e) mu[e] = mom[e] / rho;
  for (int e = 0; e < ne; ++e) {
    if (e == e0) continue;
    real tot = 0;
    for (const auto& blocks : m.parts[e]) {
      const int k = (int)blocks.size();
      real fact = 1;
      for (int i = 2; i < k; ++i) fact *= i;     // (k - 1)!
      real prod = ((k - 1) % 2 == 0 ? 1.0 : -1.0) * fact;
      for (int b : blocks) prod *= mu[b];
      tot += prod;
    }
    kap[e] = tot;
  }
  const int D = L.d;
  real tr = 0;
  for (int e = 0; e < ne; ++e) {
    const int a = m.ex[3 * e], b = m.ex[3 * e + 1], c = m.ex[3 * e + 2];
    if (a + b + c == 2 && std::max(a, std::max(b, c)) == 2) tr += kap[e];
  }
  const real tr_post = tr + m.omega_bulk * (D * CS2 - tr);
  for (int e = 0; e < ne; ++e) {
    if (e == e0) continue;
    const int a = m.ex[3 * e], b = m.ex[3 * e + 1], c = m.ex[3 * e + 2];
    const int n = a + b + c;
    if (n == 1) {
      post[e] = kap[e];
    } else if (n == 2 && std::max(a, std::max(b, c)) == 1) {
      post[e] = kap[e] - m.omega * kap[e];
    } else if (n == 2) {
      const real dev = kap[e] - tr / D;
      post[e] = (1 - m.omega) * dev + tr_post / D;
    } else {
      post[e] = kap[e] - m.hi[n - 3] * kap[e];
    }
  }
  for (int e = 0; e < ne; ++e) {
    if (e == e0) {
      mup[e] = 1.0;
      continue;
    }
    real tot = 0;
    for (const auto& blocks : m.parts[e]) {
      real prod = 1;
      for (int b : blocks) prod *= post[b];
      tot += prod;
    }
    mup[e] = tot;
  }
  // moments [a][b][c] -> populations [x][y][z] (index 0, 1, 2 = velocity -1, 0, +1)
  const int nz = L.d == 3 ? 3 : 1;
  real A[3][3][3] = {}, B[3][3][3] = {};
  for (int e = 0; e < ne; ++e) A[m.ex[3 * e]][m.ex[3 * e + 1]][m.ex[3 * e + 2]] = rho * mup[e];
  auto inv1 = [](real m0, real m1, real m2, real* f) {
    f[0] = 0.5 * (m2 - m1);
    f[1] = m0 - m2;
    f[2] = 0.5 * (m2 + m1);
  };
  if (nz == 3) {   // along z: A[a][b][c] -> B[a][b][vz]
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        real f[3];
        inv1(A[a][b][0], A[a][b][1], A[a][b][2], f);
        for (int v = 0; v < 3; ++v) B[a][b][v] = f[v];
      }
  } else {
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) B[a][b][0] = A[a][b][0];
  }
  for (int a = 0; a < 3; ++a)      // along y: B[a][b][vz] -> A[a][vy][vz]
    for (int v = 0; v < nz; ++v) {
      real f[3];
      inv1(B[a][0][v], B[a][1][v], B[a][2][v], f);
      for (int k = 0; k < 3; ++k) A[a][k][v] = f[k];
    }
  for (int k = 0; k < 3; ++k)      // along x: A[a][vy][vz] -> B[vx][vy][vz]
    for (int v = 0; v < nz; ++v) {
      real f[3];
      inv1(A[0][k][v], A[1][k][v], A[2][k][v], f);
      for (int i = 0; i < 3; ++i) B[i][k][v] = f[i];
    }
  for (int q = 0; q < L.Q; ++q) {
    const int zi = nz == 3 ? L.c[q][2] + 1 : 0;
    out[q] = B[L.c[q][0] + 1][L.c[q][1] + 1][zi];
  }
}

// Collision of one cell: pre-collision g -> post-collision out.
void collide(const Method& m, const real* g, const real F[3], real* out) {
  const Lattice& L = m.L;
  const int Q = L.Q;
  if (m.method == CUMULANT) {
    collide_cumulant(m, g, out);
    return;
  }
  real rho, u[3], feq[27], S[27];
  macroscopic(m, g, F, rho, u);
  equilibrium(L, rho, u, m.compressible ? rho : m.rho0, feq);
  guo(L, u, F, S);
  if (m.method == SRT) {
    // Eq. (1) plus Guo's source: f* = g - omega (g - f^eq) + (1 - omega/2) S
    for (int q = 0; q < Q; ++q) out[q] = g[q] - m.omega * (g[q] - feq[q]) + (1 - 0.5 * m.omega) * S[q];
  } else if (m.method == TRT) {
    // even (symmetric) and odd (antisymmetric) parts of each (q, opp q) pair
    // relax with omega_e and omega_o; the source is split the same way
    const real we = m.omega, wo = m.omega_odd;
    for (int q = 0; q < Q; ++q) {
      const int o = L.opp[q];
      const real gp = 0.5 * (g[q] + g[o]), gm = 0.5 * (g[q] - g[o]);
      const real ep = 0.5 * (feq[q] + feq[o]), em = 0.5 * (feq[q] - feq[o]);
      const real sp = 0.5 * (S[q] + S[o]), sm = 0.5 * (S[q] - S[o]);
      out[q] = g[q] - we * (gp - ep) - wo * (gm - em) + (1 - 0.5 * we) * sp + (1 - 0.5 * wo) * sm;
    }
  } else {
    // Eq. (4): f* = g - M^-1 S M (g - f^eq) + M^-1 (I - S/2) M S_Guo
    real mneq[27], msrc[27];
    for (int k = 0; k < Q; ++k) {
      real a = 0, b = 0;
      for (int q = 0; q < Q; ++q) {
        a += m.M[(size_t)k * Q + q] * (g[q] - feq[q]);
        b += m.M[(size_t)k * Q + q] * S[q];
      }
      mneq[k] = m.rate[k] * a;
      msrc[k] = (1 - 0.5 * m.rate[k]) * b;
    }
    for (int q = 0; q < Q; ++q) {
      real a = 0;
      for (int k = 0; k < Q; ++k) a += m.Minv[(size_t)q * Q + k] * (msrc[k] - mneq[k]);
      out[q] = g[q] + a;
    }
  }
}

// Periodic wrap of a coordinate at most one cell outside [0, n).
int wrap(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

int nthreads_of(int32_t n) {
#ifdef _OPENMP
  return n > 0 ? n : omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}

}  // namespace

extern "C" {

// Description of one oracle run.  storage: 0 FP64 (no rounding), 1 FP32,
// 2 BF16, 3 FP16 (emulated shifted storage).  omega_odd <= 0: derived from
// magic = (1/omega - 1/2)(1/omega_odd - 1/2).
typedef struct {
  int32_t stencil, method, storage, compressible;
  int32_t nx, ny, nz;
  real omega, omega_bulk, omega_odd, magic, omega_hi[4];
  real rho0;
} orc_config;

}  // extern "C"

namespace {

bool setup(const orc_config* cfg, Method& m) {
  if (!cfg || !make_lattice(cfg->stencil, m.L)) return false;
  if (cfg->method < SRT || cfg->method > CUMULANT) return false;
  if (cfg->method == CUMULANT && cfg->stencil == 1) return false;   // needs a tensor-product stencil
  m.method = cfg->method;
  m.storage = cfg->storage;
  m.compressible = cfg->compressible;
  m.omega = cfg->omega;
  m.omega_bulk = cfg->omega_bulk;
  m.omega_odd = cfg->omega_odd > 0 ? cfg->omega_odd : 1.0 / (cfg->magic / (1.0 / cfg->omega - 0.5) + 0.5);
  for (int i = 0; i < 4; ++i) m.hi[i] = cfg->omega_hi[i];
  m.rho0 = cfg->rho0;
  if (m.method == MRT) build_mrt(m);
  if (m.method == CUMULANT) build_cumulant(m);
  return true;
}

}  // namespace

extern "C" {

// P (Q*N) = f^eq(rho, u) (Eq. 3) at fluid cells, w_q rho_0 at solid cells,
// then the storage rounding.  rho: N values or NULL (rho_0); u: 3*N values
// (component-major) or NULL (rest); mask: N bytes (0 fluid) or NULL.
int32_t orc_init(const orc_config* cfg, const uint8_t* mask, const real* rho, const real* u, real* P) {
  Method m;
  if (!setup(cfg, m) || !P) return -1;
  const int64_t N = (int64_t)cfg->nx * cfg->ny * cfg->nz;
  const int Q = m.L.Q;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < N; ++i) {
    real feq[27];
    if (mask && mask[i]) {
      for (int q = 0; q < Q; ++q) feq[q] = m.L.w[q] * m.rho0;
    } else {
      const real r = rho ? rho[i] : m.rho0;
      const real uu[3] = {u ? u[i] : 0.0, u ? u[N + i] : 0.0, u ? u[2 * N + i] : 0.0};
      equilibrium(m.L, r, uu, m.compressible ? r : m.rho0, feq);
    }
    for (int q = 0; q < Q; ++q) {
      const real sh = m.L.w[q] * m.rho0;
      P[q * N + i] = m.storage ? round_storage(feq[q] - sh, m.storage) + sh : feq[q];
    }
  }
  return 0;
}

// nsteps stream-pull-collide steps on P (Q*N, updated in place).
// force_y: 3*ny doubles, force of row y at [3*y + a], or NULL (no force);
// wall_u: 3*128 doubles, velocity of wall type k at [3*k + a], or NULL (all
// walls at rest); nthreads <= 0: all available.
int32_t orc_run(const orc_config* cfg, const uint8_t* mask, const real* force_y, const real* wall_u, real* P,
                int32_t nsteps, int32_t nthreads) {
  Method m;
  if (!setup(cfg, m) || !P || nsteps < 0) return -1;
  if (m.method == CUMULANT && force_y) return -2;
  const int nx = cfg->nx, ny = cfg->ny, nz = cfg->nz;
  const int64_t N = (int64_t)nx * ny * nz;
  const int Q = m.L.Q;
  std::vector<real> other((size_t)Q * N);
  real* src = P;
  real* dst = other.data();
  const int nt = nthreads_of(nthreads);
  for (int t = 0; t < nsteps; ++t) {
#pragma omp parallel for collapse(2) schedule(static) num_threads(nt)
    for (int z = 0; z < nz; ++z)
      for (int y = 0; y < ny; ++y) {
        real g[27], out[27];
        const real F[3] = {force_y ? force_y[3 * y] : 0.0, force_y ? force_y[3 * y + 1] : 0.0,
                             force_y ? force_y[3 * y + 2] : 0.0};
        for (int x = 0; x < nx; ++x) {
          const int64_t i = ((int64_t)z * ny + y) * nx + x;
          if (mask && mask[i]) {
            for (int q = 0; q < Q; ++q) dst[q * N + i] = src[q * N + i];
            continue;
          }
          for (int q = 0; q < Q; ++q) {
            const int xs = wrap(x - m.L.c[q][0], nx);
            const int ys = wrap(y - m.L.c[q][1], ny);
            const int zs = wrap(z - m.L.c[q][2], nz);
            const int64_t s = ((int64_t)zs * ny + ys) * nx + xs;
            if (mask && mask[s]) {
              real cu = 0;
              if (wall_u)
                for (int a = 0; a < 3; ++a) cu += m.L.c[q][a] * wall_u[3 * mask[s] + a];
              g[q] = src[m.L.opp[q] * N + i] + 2 * m.L.w[q] * m.rho0 * cu / CS2;
            } else {
              g[q] = src[q * N + s];
            }
          }
          collide(m, g, F, out);
          for (int q = 0; q < Q; ++q) {
            const real sh = m.L.w[q] * m.rho0;
            dst[q * N + i] = m.storage ? round_storage(out[q] - sh, m.storage) + sh : out[q];
          }
        }
      }
    std::swap(src, dst);
  }
  if (src != P) std::memcpy(P, src, sizeof(real) * (size_t)Q * N);
  return 0;
}

// Readout of the stored post-collision state: rho = sum P,
// u = (sum c P - F/2) / rho_0 (rho_0 = rho when compressible); solid cells
// read rho = u = 0.  rho: N or NULL, u: 3*N or NULL.
int32_t orc_readout(const orc_config* cfg, const uint8_t* mask, const real* force_y, const real* P, real* rho,
                    real* u) {
  Method m;
  if (!setup(cfg, m) || !P) return -1;
  const int nx = cfg->nx, ny = cfg->ny;
  const int64_t N = (int64_t)nx * ny * cfg->nz;
  const int Q = m.L.Q;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < N; ++i) {
    const int y = (int)((i / nx) % ny);
    real r = 0, j[3] = {0, 0, 0};
    for (int q = 0; q < Q; ++q) {
      r += P[q * N + i];
      for (int a = 0; a < 3; ++a) j[a] += m.L.c[q][a] * P[q * N + i];
    }
    const bool solid = mask && mask[i];
    const real den = m.compressible ? r : m.rho0;
    if (rho) rho[i] = solid ? 0.0 : r;
    if (u)
      for (int a = 0; a < 3; ++a) {
        const real F = force_y ? force_y[3 * y + a] : 0.0;
        u[a * N + i] = solid ? 0.0 : (j[a] - 0.5 * F) / den;
      }
  }
  return 0;
}

// Totals over fluid cells: out = (sum rho, sum j_x, sum j_y, sum j_z).
int32_t orc_conserved(const orc_config* cfg, const uint8_t* mask, const real* P, real* out) {
  Method m;
  if (!setup(cfg, m) || !P || !out) return -1;
  const int64_t N = (int64_t)cfg->nx * cfg->ny * cfg->nz;
  const int Q = m.L.Q;
  real s0 = 0, s1 = 0, s2 = 0, s3 = 0;
#pragma omp parallel for schedule(static) reduction(+ : s0, s1, s2, s3)
  for (int64_t i = 0; i < N; ++i) {
    if (mask && mask[i]) continue;
    for (int q = 0; q < Q; ++q) {
      const real v = P[q * N + i];
      s0 += v;
      s1 += m.L.c[q][0] * v;
      s2 += m.L.c[q][1] * v;
      s3 += m.L.c[q][2] * v;
    }
  }
  out[0] = s0;
  out[1] = s1;
  out[2] = s2;
  out[3] = s3;
  return 0;
}

// One collision of `n` independent cells: g (Q*n, cell-major: g[c*Q + q]) ->
// out (same layout); F: 3 doubles or NULL.  For single-cell pins.
int32_t orc_collide_cells(const orc_config* cfg, const real* g, const real* F, int64_t n, real* out) {
  Method m;
  if (!setup(cfg, m) || !g || !out) return -1;
  const real F0[3] = {F ? F[0] : 0.0, F ? F[1] : 0.0, F ? F[2] : 0.0};
  if (m.method == CUMULANT && F && (F[0] != 0 || F[1] != 0 || F[2] != 0)) return -2;
  const int Q = m.L.Q;
  for (int64_t c = 0; c < n; ++c) collide(m, g + c * Q, F0, out + c * Q);
  return 0;
}

// MRT basis of the stencil (rows M[k][q]) and its per-row rates, for pins.
int32_t orc_mrt_basis(const orc_config* cfg, real* M, real* rate) {
  Method m;
  orc_config c = *cfg;
  c.method = MRT;
  if (!setup(&c, m) || !M || !rate) return -1;
  std::memcpy(M, m.M.data(), sizeof(real) * m.M.size());
  std::memcpy(rate, m.rate.data(), sizeof(real) * m.rate.size());
  return 0;
}

int32_t orc_num_threads(void) { return nthreads_of(0); }

}  // extern "C"
