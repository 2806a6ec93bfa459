// Discrete adjoint of the SRT + Guo + bounce-back time step.
//
// Forward step (the sweep): g = pull-gather(P^t) with bounce-back,
// rho = sum g, u = (sum c g + F/2)/rho, P^{t+1} = g - omega (g - f^eq) + (1 - omega/2) S.
// Its transpose, per fluid cell x, with lambda = lambda^{t+1}(x, .):
//   e_q    = f^eq_q / rho = w_q (1 + 3 c.u + 4.5 (c.u)^2 - 1.5 u.u)
//   alpha  = omega sum_q lambda_q e_q
//   beta_a = sum_q lambda_q [omega df^eq_q/du_a + dS_q/du_a]
//          = sum_q c_qa t_q - 3 (omega rho u_a + (1 - omega/2) F_a) s0,
//            t_q = lambda_q w_q (3 omega rho (1 + 3 c.u) + 9 (1 - omega/2) c.F),
//            s0 = sum_q lambda_q w_q
//   h_p    = (1 - omega) lambda_p + alpha + (c_p - u).beta / rho
// and h_p goes back along the link it was pulled through: to the entry
// lambda^t(x - c_p, p), or lambda^t(x, opp(p)) if that link was bounced.
// dL/dF collects, per cell,
//   sum_q lambda_q dS_q/dF_b + beta_b / (2 rho)
//   = (1 - omega/2) [sum_q c_qb lambda_q w_q (3 + 9 c.u) - 3 u_b s0] + beta_b / (2 rho),
// reduced per block in FP64.
//
// Storage of lambda: one array, laid out like the state of an AA run
// (Sec. IV-B) at the same time, whichever pattern the forward run used (the
// forward states come from the tape in the two-array layout either way).
// Each AA kernel reads and writes the same set of slots per cell, so its
// transpose does as well: the adjoint of the even kernel reads lambda from
// the cell's own slots opp(q) and writes h to its own slots q; the adjoint
// of the odd kernel reads lambda from the slots the forward kernel pushed
// to, (x + c_q, q) or (x, opp q) at a wall, and writes h to the slots it
// pulled from, (x - c_q, opp q) or (x, q) at a wall.  Both run in place
// without races, and lambda needs one array instead of two.
#include <type_traits>

#include "sweep.h"

namespace lbm {

bool adjoint_supported(int stencil, int method) {
  return (method == M_SRT || method == M_TRT || method == M_MRT) && stencil >= 0 && stencil <= 2;
}

template <int W>
__device__ __forceinline__ void block_sum_adj(double (&v)[W]) {
  __shared__ double red[W][16];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < W; ++c) {
    double s = v[c];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
    if (lane == 0) red[c][wid] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int c = 0; c < W; ++c) {
      double s = 0.0;
      for (int i = 0; i < nw; ++i) s += red[c][i];
      v[c] = s;
    }
  }
}

__device__ __forceinline__ double ld_f(const void* p, size_t i, int fdt) {
  return fdt == 0 ? ((const double*)p)[i] : (double)((const float*)p)[i];
}
__device__ __forceinline__ void st_f(void* p, size_t i, double v, int fdt) {
  if (fdt == 0)
    ((double*)p)[i] = v;
  else
    ((float*)p)[i] = (float)v;
}

// Linear index (plane * N + cell) of the slot that holds population q of the
// fluid cell c in a stored layout (0 two arrays; 1 AA inverted; 2 AA
// streamed, see load_post).
template <class L>
__device__ __forceinline__ size_t post_slot(int layout, int q, const CellIdx& c, const Geo& g,
                                            const uint8_t* flags, int has_mask) {
  const size_t N = (size_t)g.N;
  if (layout == 0) return (size_t)q * N + c.cell;
  if (layout == 1) return (size_t)opp<L>(q) * N + c.cell;
  LBM_NEIGHBOURS(c, g)
  const int d = upstream<L>(opp<L>(q), c, g, xm, xp, ym, yp, zm, zp);  // x + c_q
  // a neighbour can be solid only where the cell's own flag says so
  const bool bounced = q > 0 && has_mask && (flags[c.cell] & 2) && (flags[d] & 1);
  return bounced ? (size_t)opp<L>(q) * N + c.cell : (size_t)q * N + d;
}

// ------------------------------------------------------------------ seed
// lambda^T_q = dL/drho + sum_a dL/du_a (c_qa - u_a)/rho with the readout
// rho = sum P, u = (sum c P - F/2)/rho; the readout also gives dL/dF its
// direct term -sum_x dL/du(x) / (2 rho(x)).
// The seed writes every slot: solid cells' own slots get 0, and the fluid
// values land on the fluid slots one to one in every layout.
template <class L, class T>
__global__ __launch_bounds__(512) void k_adj_seed(const T* __restrict__ P, const uint8_t* __restrict__ flags,
                                                  int has_mask, int layout, int lam_layout,
                                                  const typename Storage<T>::R* __restrict__ force_y,
                                                  const void* dL_drho, const void* dL_du, int fdt,
                                                  typename Storage<T>::R* __restrict__ lam,
                                                  double* __restrict__ partials, Geo g, double rho0) {
  using R = typename Storage<T>::R;
  const CellIdx c = cell_of(g);
  const size_t N = (size_t)g.N;
  double dF[3] = {0, 0, 0};
  if (c.valid) {
    const bool solid = has_mask && (flags[c.cell] & 1);
    if (solid) {
#pragma unroll
      for (int q = 0; q < L::Q; ++q) lam[q * N + c.cell] = R(0);
    } else {
      R f[L::Q];
      if (layout == 0) {
#pragma unroll
        for (int q = 0; q < L::Q; ++q) f[q] = Storage<T>::load(P + q * N + c.cell);
      } else {
        double v[L::Q];
        load_post<L, T>(P, flags, has_mask, layout, c, g, v);
#pragma unroll
        for (int q = 0; q < L::Q; ++q) f[q] = R(v[q]);
      }
      R drho, jx, jy, jz;
      density_momentum<L>(f, drho, jx, jy, jz);
      const R rho = R(rho0) + drho;
      const R inv = R(1) / rho;
      const R ux = (jx - R(0.5) * force_y[3 * c.y]) * inv;
      const R uy = (jy - R(0.5) * force_y[3 * c.y + 1]) * inv;
      const R uz = (jz - R(0.5) * force_y[3 * c.y + 2]) * inv;
      const R gx = R(ld_f(dL_du, c.cell, fdt)), gy = R(ld_f(dL_du, N + c.cell, fdt)),
              gz = R(ld_f(dL_du, 2 * N + c.cell, fdt));
      const R gr = dL_drho ? R(ld_f(dL_drho, c.cell, fdt)) : R(0);
      const R base = gr - (gx * ux + gy * uy + gz * uz) * inv;
#pragma unroll
      for (int q = 0; q < L::Q; ++q)
        lam[post_slot<L>(lam_layout, q, c, g, flags, has_mask)] = base + cdot<L>(q, gx, gy, gz) * inv;
      dF[0] = -(double)gx / (2.0 * (double)rho);
      dF[1] = -(double)gy / (2.0 * (double)rho);
      dF[2] = -(double)gz / (2.0 * (double)rho);
    }
  }
  block_sum_adj<3>(dF);
  if (threadIdx.x == 0)
    for (int k = 0; k < 3; ++k) partials[(size_t)blockIdx.x * 3 + k] = dF[k];
}

// ------------------------------------------------------------------ sweep
// a = A^T lambda and b = B^T lambda for the collision's constant matrices
// (P* = g - A (g - f^eq) + B S): SRT A = omega I, B = (1 - omega/2) I; TRT
// A = omega_e P+ + omega_o P-, B = (1 - omega_e/2) P+ + (1 - omega_o/2) P-,
// with P+- the symmetric and antisymmetric parts of each (q, opp q) pair
// (symmetric matrices, so A^T = A); MRT A = M^-1 S M, B = M^-1 (I - S/2) M
// in the weighted-orthogonal basis, where M^-1 = W M^T D^-1 gives
//   (A^T lambda)_p = sum_k m_k(c_p) s_k (sum_q m_k(c_q) w_q lambda_q) / d_k,
// d_k = sum_q w_q m_k(c_q)^2, s_k the rate of row k (0 on conserved rows);
// the same basis the forward MRT operator relaxes in (on D2Q9 and D3Q27 the
// forward kernel uses the equivalent tensor-product form).
template <class L, int M, class R>
__device__ __forceinline__ void relax_transpose(const R* lam, R* a, R* b, const CollideParams<R>& p) {
  if constexpr (M == M_TRT) {
    const R we = p.om, wo = p.om_o, fe = R(1) - R(0.5) * we, fo = R(1) - R(0.5) * wo;
    a[0] = we * lam[0];
    b[0] = fe * lam[0];
#pragma unroll
    for (int q = 1; q <= L::H; ++q) {
      const int o = q + L::H;
      const R lp = R(0.5) * (lam[q] + lam[o]), lm = R(0.5) * (lam[q] - lam[o]);
      a[q] = we * lp + wo * lm;
      a[o] = we * lp - wo * lm;
      b[q] = fe * lp + fo * lm;
      b[o] = fe * lp - fo * lm;
    }
  } else if constexpr (M == M_MRT) {
    constexpr MrtBasis<L::Q> B = make_mrt_basis<L>();
    R mom[L::Q];
#pragma unroll
    for (int k = 0; k < L::Q; ++k) {
      R acc = R(0);
#pragma unroll
      for (int q = 0; q < L::Q; ++q)
        if (B.m[k][q] != 0.0) acc += R(B.m[k][q] * weight<L>(q)) * lam[q];
      mom[k] = acc * R(B.inv_norm[k]);
    }
    R sa[L::Q], sbv[L::Q];
#pragma unroll
    for (int k = 0; k < L::Q; ++k) {
      const int grp = B.group[k];
      const R rate = grp == 0 ? R(0) : (grp == 1 ? p.om : (grp == 2 ? p.om_b : p.hi[grp - 3]));
      sa[k] = rate * mom[k];
      sbv[k] = (R(1) - R(0.5) * rate) * mom[k];
    }
#pragma unroll
    for (int q = 0; q < L::Q; ++q) {
      R x = R(0), y = R(0);
#pragma unroll
      for (int k = 0; k < L::Q; ++k)
        if (B.m[k][q] != 0.0) {
          x += R(B.m[k][q]) * sa[k];
          y += R(B.m[k][q]) * sbv[k];
        }
      a[q] = x;
      b[q] = y;
    }
  } else {
    const R om = p.om, fs = R(1) - R(0.5) * p.om;
#pragma unroll
    for (int q = 0; q < L::Q; ++q) {
      a[q] = om * lam[q];
      b[q] = fs * lam[q];
    }
  }
}

// One fluid cell: lam (lambda^{t+1} of the cell, Q values) becomes h = J^T lam
// in place, for the pre-collision populations f; dF receives the cell's
// dL/dF contribution.  With a = A^T lam, b = B^T lam:
//   h_p = lam_p - a_p + alpha + (c_p - u).beta / rho,
//   alpha = sum_q a_q f^eq_q / rho,
//   beta  = sum_q [a_q df^eq_q/du + b_q dS_q/du],
//   dL/dF += sum_q b_q dS_q/dF (at fixed u) + beta / (2 rho).
template <class L, int M, class R>
__device__ __forceinline__ void adj_cell(const R* f, R* lam, R F0, R F1, R F2, const CollideParams<R>& p,
                                         double* dF) {
  R drho, jx, jy, jz;
  density_momentum<L>(f, drho, jx, jy, jz);
  const R rho = p.rho0 + drho;
  const R inv = R(1) / rho;
  const R ux = (jx + R(0.5) * F0) * inv, uy = (jy + R(0.5) * F1) * inv, uz = (jz + R(0.5) * F2) * inv;
  const R usq = R(1.5) * (ux * ux + uy * uy + uz * uz);
  if constexpr (M == M_SRT) {   // a = omega lam, b = (1 - omega/2) lam: the factors come out of the sums
    const R om = p.om, fs = R(1) - R(0.5) * p.om;
    const R omr3 = R(3) * om * rho;
    R alpha = R(0), s0 = R(0), bx = R(0), by = R(0), bz = R(0), sx = R(0), sy = R(0), sz = R(0);
#pragma unroll
    for (int q = 0; q < L::Q; ++q) {
      const R w = R(weight<L>(q));
      const R cu = cdot<L>(q, ux, uy, uz);
      const R cF = cdot<L>(q, F0, F1, F2);
      const R lw = lam[q] * w;
      alpha += lw * (R(1) + R(3) * cu + R(4.5) * cu * cu - usq);
      s0 += lw;
      const R t = lw * (omr3 * (R(1) + R(3) * cu) + R(9) * fs * cF);
      const R sf = lw * (R(3) + R(9) * cu);
      if (L::c(q, 0) == 1) { bx += t; sx += sf; }
      if (L::c(q, 0) == -1) { bx -= t; sx -= sf; }
      if (L::c(q, 1) == 1) { by += t; sy += sf; }
      if (L::c(q, 1) == -1) { by -= t; sy -= sf; }
      if (L::c(q, 2) == 1) { bz += t; sz += sf; }
      if (L::c(q, 2) == -1) { bz -= t; sz -= sf; }
    }
    alpha *= om;
    bx -= R(3) * (om * rho * ux + fs * F0) * s0;
    by -= R(3) * (om * rho * uy + fs * F1) * s0;
    bz -= R(3) * (om * rho * uz + fs * F2) * s0;
    const R base = alpha - (bx * ux + by * uy + bz * uz) * inv;
    const R one_m = R(1) - om;
#pragma unroll
    for (int q = 0; q < L::Q; ++q) lam[q] = one_m * lam[q] + base + cdot<L>(q, bx, by, bz) * inv;
    dF[0] = (double)(fs * (sx - R(3) * ux * s0) + bx * R(0.5) * inv);
    dF[1] = (double)(fs * (sy - R(3) * uy * s0) + by * R(0.5) * inv);
    dF[2] = (double)(fs * (sz - R(3) * uz * s0) + bz * R(0.5) * inv);
    return;
  }
  R a[L::Q], b[L::Q];
  relax_transpose<L, M, R>(lam, a, b, p);
  const R r3 = R(3) * rho;
  R alpha = R(0), sa = R(0), sb = R(0), bx = R(0), by = R(0), bz = R(0), sx = R(0), sy = R(0), sz = R(0);
#pragma unroll
  for (int q = 0; q < L::Q; ++q) {
    const R w = R(weight<L>(q));
    const R cu = cdot<L>(q, ux, uy, uz);
    const R cF = cdot<L>(q, F0, F1, F2);
    const R aw = a[q] * w, bw = b[q] * w;
    alpha += aw * (R(1) + R(3) * cu + R(4.5) * cu * cu - usq);
    sa += aw;
    sb += bw;
    const R t = aw * (r3 * (R(1) + R(3) * cu)) + bw * (R(9) * cF);
    const R sf = bw * (R(3) + R(9) * cu);
    if (L::c(q, 0) == 1) { bx += t; sx += sf; }
    if (L::c(q, 0) == -1) { bx -= t; sx -= sf; }
    if (L::c(q, 1) == 1) { by += t; sy += sf; }
    if (L::c(q, 1) == -1) { by -= t; sy -= sf; }
    if (L::c(q, 2) == 1) { bz += t; sz += sf; }
    if (L::c(q, 2) == -1) { bz -= t; sz -= sf; }
  }
  bx -= r3 * ux * sa + R(3) * F0 * sb;
  by -= r3 * uy * sa + R(3) * F1 * sb;
  bz -= r3 * uz * sa + R(3) * F2 * sb;
  const R base = alpha - (bx * ux + by * uy + bz * uz) * inv;
#pragma unroll
  for (int q = 0; q < L::Q; ++q) lam[q] = lam[q] - a[q] + base + cdot<L>(q, bx, by, bz) * inv;
  dF[0] = (double)(sx - R(3) * ux * sb + bx * R(0.5) * inv);
  dF[1] = (double)(sy - R(3) * uy * sb + by * R(0.5) * inv);
  dF[2] = (double)(sz - R(3) * uz * sb + bz * R(0.5) * inv);
}

// A wave-uniform plane pointer the compiler cannot see through.  The adjoint
// kernels read lambda from the slots they then write (the same addresses in
// another order); left alone, the compiler builds the 19 64-bit addresses
// once in vector registers and keeps them from the loads to the stores
// (111 VGPRs for the even D3Q19 FP32 kernel).  Passing each load's plane base
// through an empty inline-asm statement that pins it to scalar registers
// keeps every access in the scalar-base plus 32-bit lane-offset form: 76
// VGPRs (83 for the odd kernel), and C4's backward 29.6 -> 29.2 ms in both
// patterns (alternating processes, three rounds).
template <class T>
__device__ __forceinline__ T* opaque_uniform(T* p) {
  asm volatile("" : "+s"(p));
  return p;
}

// One lambda array (AA pattern), in place; ODD selects the adjoint of the
// odd kernel.  P is the forward state of the reversed step in the two-array
// layout (the tape and the recomputed segment hold that layout).
template <class L, class T, int ODD, int M>
__global__ __launch_bounds__(512) void k_adj_sweep_aa(const T* __restrict__ P, const uint8_t* __restrict__ flags,
                                                      int has_mask,
                                                      const typename Storage<T>::R* __restrict__ force_y,
                                                      typename Storage<T>::R* A, double* __restrict__ partials,
                                                      Geo g, CollideParams<typename Storage<T>::R> p) {
  using R = typename Storage<T>::R;
  const CellIdx c = cell_of(g);
  const size_t N = (size_t)g.N;
  double dF[3] = {0, 0, 0};
  int fl = 0;
  if (c.valid && has_mask) fl = flags[c.cell];
  if (c.valid && !(fl & 1)) {
    R f[L::Q];
    uint32_t bb = 0;   // bit q: x - c_q is solid (so x + c_opp(q) is solid)
    load_phase_begin<T>();
    gather<L, T>(P, flags, fl, c, g, f, &bb, p);
    LBM_NEIGHBOURS(c, g)
    const uint32_t ox[3] = {(uint32_t)xp * (uint32_t)sizeof(R), (uint32_t)c.x * (uint32_t)sizeof(R),
                            (uint32_t)xm * (uint32_t)sizeof(R)};  // x - c_x for c_x = -1, 0, +1
    R* own = A + (size_t)(c.z * g.ny + c.y) * (size_t)g.nx;
    R lam[L::Q];
    if (!ODD) {
#pragma unroll
      for (int q = 0; q < L::Q; ++q) lam[q] = *at_bytes(opaque_uniform(own + (size_t)opp<L>(q) * N), ox[1]);
    } else {
      // forward push slot of q: (x + c_q, q), or (x, opp q) when x + c_q is solid
#pragma unroll
      for (int q = 0; q < L::Q; ++q)
        lam[q] = *at_bytes(opaque_uniform(plane_row<L>(A, q, opp<L>(q), c, ym, yp, zm, zp, g)),
                           ox[L::c(opp<L>(q), 0) + 1]);
      if (bb) {
#pragma unroll
        for (int q = 1; q < L::Q; ++q)
          if ((bb >> opp<L>(q)) & 1u) lam[q] = *at_bytes(own + (size_t)opp<L>(q) * N, ox[1]);
      }
    }
    load_phase_end<T>();
    adj_cell<L, M, R>(f, lam, force_y[3 * c.y], force_y[3 * c.y + 1], force_y[3 * c.y + 2], p, dF);
    if (!ODD) {
#pragma unroll
      for (int q = 0; q < L::Q; ++q) *at_bytes(own + (size_t)q * N, ox[1]) = lam[q];
    } else {
      // forward pull slot of q: (x - c_q, opp q), or (x, q) when x - c_q is solid
#pragma unroll
      for (int q = 0; q < L::Q; ++q) {
        if ((bb >> q) & 1u)
          *at_bytes(own + (size_t)q * N, ox[1]) = lam[q];
        else
          *at_bytes(plane_row<L>(A, opp<L>(q), q, c, ym, yp, zm, zp, g), ox[L::c(q, 0) + 1]) = lam[q];
      }
    }
  }
  block_sum_adj<3>(dF);
  if (threadIdx.x == 0)
    for (int k = 0; k < 3; ++k) partials[(size_t)blockIdx.x * 3 + k] += dF[k];
}

// ------------------------------------------------------------------ init
// P^0 = f^eq(rho, u): dL/du_a = sum_q lambda_q w_q rho (3 c_qa + 9 (c.u) c_qa - 3 u_a),
//                      dL/drho = sum_q lambda_q w_q (1 + 3 c.u + 4.5 (c.u)^2 - 1.5 u.u).
template <class L, class R>
__global__ __launch_bounds__(512) void k_adj_init_grad(const R* __restrict__ lam, const uint8_t* __restrict__ flags,
                                                       int has_mask, int layout, const R* __restrict__ init_fields,
                                                       void* dL_du0, void* dL_drho0, int fdt, Geo g) {
  const CellIdx c = cell_of(g);
  if (!c.valid) return;
  const size_t N = (size_t)g.N;
  double gx = 0, gy = 0, gz = 0, gr = 0;
  if (!(has_mask && (flags[c.cell] & 1))) {
    const R rho = init_fields[c.cell];
    const R ux = init_fields[N + c.cell], uy = init_fields[2 * N + c.cell], uz = init_fields[3 * N + c.cell];
    const R usq = R(1.5) * (ux * ux + uy * uy + uz * uz);
    R ax = 0, ay = 0, az = 0, s0 = 0, r = 0;
#pragma unroll
    for (int q = 0; q < L::Q; ++q) {
      const R lw = lam[post_slot<L>(layout, q, c, g, flags, has_mask)] * R(weight<L>(q));
      const R cu = cdot<L>(q, ux, uy, uz);
      r += lw * (R(1) + R(3) * cu + R(4.5) * cu * cu - usq);
      s0 += lw;
      const R t = lw * (R(3) + R(9) * cu);
      if (L::c(q, 0) == 1) ax += t;
      if (L::c(q, 0) == -1) ax -= t;
      if (L::c(q, 1) == 1) ay += t;
      if (L::c(q, 1) == -1) ay -= t;
      if (L::c(q, 2) == 1) az += t;
      if (L::c(q, 2) == -1) az -= t;
    }
    gx = (double)(rho * (ax - R(3) * ux * s0));
    gy = (double)(rho * (ay - R(3) * uy * s0));
    gz = (double)(rho * (az - R(3) * uz * s0));
    gr = (double)r;
  }
  if (dL_du0) {
    st_f(dL_du0, c.cell, gx, fdt);
    st_f(dL_du0, N + c.cell, gy, fdt);
    st_f(dL_du0, 2 * N + c.cell, gz, fdt);
  }
  if (dL_drho0) st_f(dL_drho0, c.cell, gr, fdt);
}

template <class R>
__global__ __launch_bounds__(512) void k_store_init_fields(const void* rho, const void* u, int fdt,
                                                           R* __restrict__ out, Geo g, double rho0) {
  const CellIdx c = cell_of(g);
  if (!c.valid) return;
  const size_t N = (size_t)g.N;
  out[c.cell] = R(rho ? ld_f(rho, c.cell, fdt) : rho0);
  for (int a = 0; a < 3; ++a) out[(a + 1) * N + c.cell] = R(u ? ld_f(u, a * N + c.cell, fdt) : 0.0);
}

// ------------------------------------------------------------------ launchers
template <class F>
static hipError_t by_stencil_dtype(int stencil, int dtype, F&& fn) {
  auto by_dtype = [&](auto lat) -> hipError_t {
    switch (dtype) {
      case 0: return fn(lat, double());
      case 1: return fn(lat, float());
      case 2: return fn(lat, __bf16());
      case 3: return fn(lat, _Float16());
    }
    return hipErrorInvalidValue;
  };
  switch (stencil) {
    case 0: return by_dtype(D2Q9());
    case 1: return by_dtype(D3Q19());
    case 2: return by_dtype(D3Q27());
  }
  return hipErrorInvalidValue;
}

hipError_t launch_adjoint_seed(int stencil, int dtype, const void* P, const uint8_t* flags, int has_mask,
                               int layout, int lam_layout, const void* force_y, const void* dL_drho,
                               const void* dL_du, int field_dtype, void* lam, double* partials, const Geo& g,
                               const Params& p, hipStream_t s) {
  return by_stencil_dtype(stencil, dtype, [&](auto lat, auto tag) -> hipError_t {
    using L = decltype(lat);
    using T = decltype(tag);
    using R = typename Storage<T>::R;
    hipLaunchKernelGGL((k_adj_seed<L, T>), dim3((unsigned)num_blocks(g)), dim3(g.bx), 0, s, (const T*)P, flags,
                       has_mask, layout, lam_layout, (const R*)force_y, dL_drho, dL_du, field_dtype, (R*)lam,
                       partials, g, p.rho0);
    return hipGetLastError();
  });
}

hipError_t launch_adjoint_sweep(int stencil, int method, int dtype, int phase, const void* P,
                                const uint8_t* flags, int has_mask, const void* force_y, void* lam,
                                double* partials, const Geo& g, const Params& p, hipStream_t s) {
  return by_stencil_dtype(stencil, dtype, [&](auto lat, auto tag) -> hipError_t {
    using L = decltype(lat);
    using T = decltype(tag);
    using R = typename Storage<T>::R;
    const CollideParams<R> cp = to_collide_params<R>(p);
    const dim3 grid((unsigned)num_blocks(g)), block(g.bx);
    auto go = [&](auto odd, auto meth) {
      hipLaunchKernelGGL((k_adj_sweep_aa<L, T, decltype(odd)::value, decltype(meth)::value>), grid, block, 0, s,
                         (const T*)P, flags, has_mask, (const R*)force_y, (R*)lam, partials, g, cp);
    };
    using Z = std::integral_constant<int, 0>;
    using O = std::integral_constant<int, 1>;
    using SRT = std::integral_constant<int, M_SRT>;
    using TRT = std::integral_constant<int, M_TRT>;
    using MRT = std::integral_constant<int, M_MRT>;
    if (method == M_TRT) {
      if (phase == 0) go(Z(), TRT()); else go(O(), TRT());
    } else if (method == M_MRT || method == M_MRT_UNIT) {   // the same operator
      if (phase == 0) go(Z(), MRT()); else go(O(), MRT());
    } else {
      if (phase == 0) go(Z(), SRT()); else go(O(), SRT());
    }
    return hipGetLastError();
  });
}

hipError_t launch_adjoint_init_grad(int stencil, int dtype, const void* lam, const uint8_t* flags, int has_mask,
                                    int layout, const void* init_fields, void* dL_du0, void* dL_drho0,
                                    int field_dtype, const Geo& g, const Params& p, hipStream_t s) {
  (void)p;
  auto run = [&](auto lat, auto rtag) -> hipError_t {
    using L = decltype(lat);
    using R = decltype(rtag);
    hipLaunchKernelGGL((k_adj_init_grad<L, R>), dim3((unsigned)num_blocks(g)), dim3(g.bx), 0, s, (const R*)lam,
                       flags, has_mask, layout, (const R*)init_fields, dL_du0, dL_drho0, field_dtype, g);
    return hipGetLastError();
  };
  const bool dbl = dtype == 0;
  switch (stencil) {
    case 0: return dbl ? run(D2Q9(), double()) : run(D2Q9(), float());
    case 1: return dbl ? run(D3Q19(), double()) : run(D3Q19(), float());
    case 2: return dbl ? run(D3Q27(), double()) : run(D3Q27(), float());
  }
  return hipErrorInvalidValue;
}

hipError_t launch_store_init_fields(int dtype, const void* rho, const void* u, int field_dtype, void* init_fields,
                                    const Geo& g, const Params& p, hipStream_t s) {
  if (dtype == 0) {
    hipLaunchKernelGGL((k_store_init_fields<double>), dim3((unsigned)num_blocks(g)), dim3(g.bx), 0, s, rho, u,
                       field_dtype, (double*)init_fields, g, p.rho0);
  } else {
    hipLaunchKernelGGL((k_store_init_fields<float>), dim3((unsigned)num_blocks(g)), dim3(g.bx), 0, s, rho, u,
                       field_dtype, (float*)init_fields, g, p.rho0);
  }
  return hipGetLastError();
}

}  // namespace lbm
