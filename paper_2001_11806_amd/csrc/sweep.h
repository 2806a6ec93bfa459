// The fused stream-pull-collide sweep: two-array pattern, the AA pattern,
// and the stored-layout helpers.
//
// Paper, Sec. IV-B and Fig. "stream-pull-collide": every cell pulls
// population q from its upstream neighbour x - c_q in the source array,
// collides locally and writes all Q results to its own slot in the
// destination array.  Halfway velocity bounce-back (Sec. III-C "Boundary
// Conditions") is compiled into the gather (Sec. IV-B "Boundary Conditions",
// flag field variant): if x - c_q is solid the cell reads its own outgoing
// population opp(q) instead, plus the moving-wall term.
//
// MI355X mapping
//   - structure-of-arrays layout P[q][z][y][x]; a wavefront reads 64
//     consecutive x of one q-plane per load, so every load and store is
//     coalesced; the +-1 x offset of the pull is absorbed by the cache line
//     that the neighbouring lanes fetch anyway;
//   - one block per x-row (or per x-segment of at most 512 cells), so each
//     source row of each q-plane is read by exactly one block: the pull
//     touches every stored byte exactly once, 2 Q s bytes per cell update;
//   - all Q loads are issued before any arithmetic (full unroll), which keeps
//     Q * 64 loads in flight per wave;
//   - the per-cell flag byte (bit 0 solid, bit 1 "fluid cell next to a
//     solid") keeps the neighbour-mask reads off the path of interior cells;
//   - periodic wrap by compare-and-select on the three neighbour coordinates.
#pragma once

#include "collide.h"
#include "internal.h"
#include "lattice.h"
#include "storage.h"

namespace lbm {

template <class R>
inline CollideParams<R> to_collide_params(const Params& p) {
  CollideParams<R> c;
  c.rho0 = R(p.rho0);
  c.om = R(p.om);
  c.om_b = R(p.om_b);
  c.om_o = R(p.om_o);
  for (int i = 0; i < 4; ++i) c.hi[i] = R(p.hi[i]);
  c.smag18 = R(p.smag18);
  c.compressible = p.compressible;
  c.wall = (const R*)p.wall;
  c.links = p.links;
  c.moving = p.moving;
  return c;
}

// Thread -> cell mapping shared by all per-cell kernels.  The hardware
// hands out the blocks of a launch in index order, block b to XCD b mod 8.
// Geo::order bit 1 renumbers them so that XCD k walks the k-th contiguous
// eighth of the row segments (the rows a pull shares then meet in one L2);
// bit 0 walks the segments from last to first.  Alternating the direction
// every step makes a step start on the rows the previous one wrote last,
// which are still in the Infinity Cache when the grid is not much larger
// than it.  Set only when gridDim.x is a multiple of 8 (bit 1).
struct CellIdx {
  int x, y, z, cell;
  bool valid;
};

__device__ __forceinline__ CellIdx cell_of(const Geo& g) {
  CellIdx c;
  unsigned b = blockIdx.x;
  if (g.order & 2) b = (b & 7u) * (gridDim.x >> 3) + (b >> 3);
  if (g.order & 1) b = gridDim.x - 1u - b;
  const int seg = b % g.nxb;
  const int row = b / g.nxb;
  c.x = seg * g.bx + threadIdx.x;
  c.y = row % g.ny;
  c.z = row / g.ny;
  c.cell = row * g.nx + c.x;
  c.valid = c.x < g.nx;
  return c;
}

// Linear index of the upstream cell x - c for direction q (periodic).
template <class L>
__device__ __forceinline__ int upstream(int q, const CellIdx& c, const Geo& g, int xm, int xp, int ym,
                                        int yp, int zm, int zp) {
  const int cx = L::c(q, 0), cy = L::c(q, 1), cz = L::c(q, 2);
  const int sx = cx > 0 ? xm : (cx < 0 ? xp : c.x);
  const int sy = cy > 0 ? ym : (cy < 0 ? yp : c.y);
  const int sz = cz > 0 ? zm : (cz < 0 ? zp : c.z);
  return (sz * g.ny + sy) * g.nx + sx;
}

#define LBM_NEIGHBOURS(c, g)                                        \
  const int xm = ((c).x == 0 ? (g).nx : (c).x) - 1;                 \
  const int xp = ((c).x + 1 == (g).nx) ? 0 : (c).x + 1;             \
  const int ym = ((c).y == 0 ? (g).ny : (c).y) - 1;                 \
  const int yp = ((c).y + 1 == (g).ny) ? 0 : (c).y + 1;             \
  const int zm = ((c).z == 0 ? (g).nz : (c).z) - 1;                 \
  const int zp = ((c).z + 1 == (g).nz) ? 0 : (c).z + 1;

// Addressing.  A block covers one x-segment of one (y, z) row, so y, z and
// every neighbour row index are wave-uniform: the start of the source row of
// plane q, src + q N + row(y - c_y, z - c_z) nx, is computed in scalar
// registers, and each lane adds one of three 32-bit byte offsets (x - c_x
// with periodic wrap).  The loads then use the scalar-base + vector-offset
// form and cost no 64-bit vector address arithmetic.
template <class T>
__device__ __forceinline__ const T* at_bytes(const T* base, uint32_t off) {
  return (const T*)((const char*)base + off);
}
template <class T>
__device__ __forceinline__ T* at_bytes(T* base, uint32_t off) {
  return (T*)((char*)base + off);
}

template <class L, class T>
__device__ __forceinline__ const T* row_base(const T* src, int q, int y, int z, int ym, int yp, int zm, int zp,
                                             const Geo& g) {
  const int cy = L::c(q, 1), cz = L::c(q, 2);
  const int sy = cy > 0 ? ym : (cy < 0 ? yp : y);
  const int sz = cz > 0 ? zm : (cz < 0 ? zp : z);
  return src + (size_t)q * (size_t)g.N + (size_t)(sz * g.ny + sy) * (size_t)g.nx;
}

// Pull-gather of the Q pre-collision populations of one fluid cell with
// halfway bounce-back.  Every link first loads its upstream slot (for a
// bounced link that slot belongs to a solid cell: in bounds, value unused);
// cells next to a wall (flag bit 1) then read their bounced-link bits and
// replace those links by their own outgoing population opp(q), plus the
// moving-wall term (wall type from the solid neighbour's flag byte) when the
// mask has moving walls.  Bit q of *bb is set for bounced links.
template <class L, class T>
__device__ __forceinline__ void gather(const T* __restrict__ src, const uint8_t* __restrict__ flags, int fl,
                                       const CellIdx& c, const Geo& g, typename Storage<T>::R* f, uint32_t* bb,
                                       const CollideParams<typename Storage<T>::R>& p) {
  LBM_NEIGHBOURS(c, g)
  const uint32_t ox[3] = {(uint32_t)xp * (uint32_t)sizeof(T), (uint32_t)c.x * (uint32_t)sizeof(T),
                          (uint32_t)xm * (uint32_t)sizeof(T)};  // source x for c_x = -1, 0, +1
#pragma unroll
  for (int q = 0; q < L::Q; ++q)
    f[q] = Storage<T>::load(at_bytes(row_base<L>(src, q, c.y, c.z, ym, yp, zm, zp, g), ox[L::c(q, 0) + 1]));
  uint32_t m = 0;
  if (fl & 2) {
    m = p.links[c.cell];
#pragma unroll
    for (int q = 1; q < L::Q; ++q) {
      if ((m >> q) & 1u) {
        f[q] = Storage<T>::load(src + (size_t)opp<L>(q) * (size_t)g.N + c.cell);
        if (p.moving)   // solid neighbour's flag byte: bits 1..7 hold the wall type
          f[q] += wall_term<L>(q, flags[upstream<L>(q, c, g, xm, xp, ym, yp, zm, zp)] >> 1, p.wall, p.rho0);
      }
    }
  }
  if (bb) *bb = m;
}

// Wave priority while a wave issues its loads (s_setprio, within the
// kernel): with 32- and 16-bit storage the CU then serves waves that start
// their memory traffic ahead of waves busy with their collision arithmetic.
// Measured in alternating processes, bit-identical results: 512^3 D3Q27 MRT
// FP16 2.77 -> 2.59 ms per step (3.08 -> 2.63 on a slower box), 256^3 D3Q19
// TRT FP32 0.440 -> 0.437 ms, the 128^3 FP32 forward and adjoint of the
// adjoint workload 0.7 % faster; the FP64 sweeps, which run fewer waves per
// CU, lost 0.3-1.6 %, so they keep the default priority.
template <class T>
__device__ __forceinline__ void load_phase_begin() {
  if (sizeof(T) <= 4) __builtin_amdgcn_s_setprio(2);
}
template <class T>
__device__ __forceinline__ void load_phase_end() {
  if (sizeof(T) <= 4) __builtin_amdgcn_s_setprio(0);
}

// Store the Q post-collision values of a cell into its own slots; NT = 1
// marks them non-temporal (the lattice is far larger than the caches and
// the next reader is the next launch).
template <class T, int NT>
__device__ __forceinline__ void store_cell(T* __restrict__ dst, const CellIdx& c, const Geo& g,
                                           const typename Storage<T>::R* f, int Q) {
  T* row = dst + (size_t)(c.z * g.ny + c.y) * (size_t)g.nx;
  const uint32_t ox = (uint32_t)c.x * (uint32_t)sizeof(T);
#pragma unroll
  for (int q = 0; q < 27; ++q) {
    if (q < Q) {
      T* p = at_bytes(row + (size_t)q * (size_t)g.N, ox);
      if (NT)
        Storage<T>::store_nt(p, f[q]);
      else
        Storage<T>::store(p, f[q]);
    }
  }
}

template <class L, int M, class T, int NT>
__global__ __launch_bounds__(512) void k_sweep(const T* __restrict__ src, T* __restrict__ dst,
                                               const uint8_t* __restrict__ flags,
                                               const typename Storage<T>::R* __restrict__ force_y, Geo g,
                                               CollideParams<typename Storage<T>::R> p, int has_mask) {
  using R = typename Storage<T>::R;
  const CellIdx c = cell_of(g);
  if (!c.valid) return;
  R f[L::Q];
  int fl = 0;
  if (NT) {
    // streaming grids: issue the Q loads together with the flag byte instead
    // of after it, so a wave does not wait one memory round trip before its
    // loads start (the launch runs fewer waves per CU, see run_sweep); a
    // solid cell's loads are then wasted, in bounds
    load_phase_begin<T>();
    if (has_mask) fl = flags[c.cell];
    gather<L, T>(src, flags, fl, c, g, f, nullptr, p);
    load_phase_end<T>();
    if (fl & 1) return;  // solid cells are never updated
  } else {
    if (has_mask) {
      fl = flags[c.cell];
      if (fl & 1) return;  // solid cells are never updated
    }
    load_phase_begin<T>();
    gather<L, T>(src, flags, fl, c, g, f, nullptr, p);
    load_phase_end<T>();
  }
  const R F[3] = {force_y[3 * c.y], force_y[3 * c.y + 1], force_y[3 * c.y + 2]};
  collide<L, M>(f, F, p);
  store_cell<T, NT>(dst, c, g, f, L::Q);
}

// ------------------------------------------------------------------ AA
// Single-array AA pattern (Sec. IV-B, Fig. "AA update pattern"), two kernels
// run alternately.  With P^t the post-collision state of step t:
//   even kernel (t even -> t+1): the array holds the streamed populations,
//     A[x][q] = g_q(x) (from a moving wall: without its wall term, which the
//     kernel adds on loading); collide in place and store inverted,
//     A[x][opp q] = f*_q(x);
//   odd kernel (t odd -> t+1): pull g_q(x) = A[x - c_q][opp q] (bounce-back:
//     A[x][q] when x - c_q is solid), collide, push f*_q to A[x + c_q][q]
//     (bounce-back: A[x][opp q] when x + c_q is solid).
// In the odd kernel every slot is read and written by the same cell, so the
// update is race-free in place.  Both kernels move 2 Q s bytes per cell.
template <class L, class T>
__device__ __forceinline__ T* plane_row(T* A, int plane, int dir, const CellIdx& c, int ym, int yp, int zm, int zp,
                                        const Geo& g) {
  const int cy = L::c(dir, 1), cz = L::c(dir, 2);
  const int sy = cy > 0 ? ym : (cy < 0 ? yp : c.y);
  const int sz = cz > 0 ? zm : (cz < 0 ? zp : c.z);
  return A + (size_t)plane * (size_t)g.N + (size_t)(sz * g.ny + sy) * (size_t)g.nx;
}

template <class T, int NT>
__device__ __forceinline__ void put(T* p, typename Storage<T>::R v) {
  if (NT)
    Storage<T>::store_nt(p, v);
  else
    Storage<T>::store(p, v);
}

// Checkpoint of the AA pattern: the post-collision populations of the cell
// in the two-array layout, slot (x, q), written by the step that produces
// them (non-temporal: the tape is read only by the adjoint).
template <class L, class T>
__device__ __forceinline__ void tape_store(T* tape, const CellIdx& c, const Geo& g,
                                           const typename Storage<T>::R* f) {
  T* row = tape + (size_t)(c.z * g.ny + c.y) * (size_t)g.nx;
  const uint32_t ox = (uint32_t)c.x * (uint32_t)sizeof(T);
#pragma unroll
  for (int q = 0; q < L::Q; ++q) Storage<T>::store_nt(at_bytes(row + (size_t)q * (size_t)g.N, ox), f[q]);
}

template <class L, int M, class T, int NT>
__global__ __launch_bounds__(512) void k_sweep_aa_even(T* A, const uint8_t* __restrict__ flags,
                                                       const typename Storage<T>::R* __restrict__ force_y, Geo g,
                                                       CollideParams<typename Storage<T>::R> p, int has_mask,
                                                       T* __restrict__ tape) {
  using R = typename Storage<T>::R;
  const CellIdx c = cell_of(g);
  if (!c.valid) return;
  const int fl = has_mask ? flags[c.cell] : 0;
  if (fl & 1) return;
  T* row = A + (size_t)(c.z * g.ny + c.y) * (size_t)g.nx;
  const uint32_t ox = (uint32_t)c.x * (uint32_t)sizeof(T);
  R f[L::Q];
  load_phase_begin<T>();
#pragma unroll
  for (int q = 0; q < L::Q; ++q) f[q] = Storage<T>::load(at_bytes(row + (size_t)q * (size_t)g.N, ox));
  load_phase_end<T>();
  if (p.moving && (fl & 2)) {
    // a bounced slot holds the cell's own outgoing population; the
    // moving-wall term is added here, on loading, as in the two-array gather
    LBM_NEIGHBOURS(c, g)
    const uint32_t m = p.links[c.cell];
#pragma unroll
    for (int q = 1; q < L::Q; ++q)
      if ((m >> q) & 1u)
        f[q] += wall_term<L>(q, flags[upstream<L>(q, c, g, xm, xp, ym, yp, zm, zp)] >> 1, p.wall, p.rho0);
  }
  const R F[3] = {force_y[3 * c.y], force_y[3 * c.y + 1], force_y[3 * c.y + 2]};
  collide<L, M>(f, F, p);
#pragma unroll
  for (int q = 0; q < L::Q; ++q) put<T, NT>(at_bytes(row + (size_t)opp<L>(q) * (size_t)g.N, ox), f[q]);
  if (tape) tape_store<L, T>(tape, c, g, f);
}

template <class L, int M, class T, int NT>
__global__ __launch_bounds__(512) void k_sweep_aa_odd(T* A, const uint8_t* __restrict__ flags,
                                                      const typename Storage<T>::R* __restrict__ force_y, Geo g,
                                                      CollideParams<typename Storage<T>::R> p, int has_mask,
                                                      T* __restrict__ tape) {
  using R = typename Storage<T>::R;
  const CellIdx c = cell_of(g);
  if (!c.valid) return;
  int fl = 0;
  if (has_mask) {
    fl = flags[c.cell];
    if (fl & 1) return;
  }
  LBM_NEIGHBOURS(c, g)
  const uint32_t ox[3] = {(uint32_t)xp * (uint32_t)sizeof(T), (uint32_t)c.x * (uint32_t)sizeof(T),
                          (uint32_t)xm * (uint32_t)sizeof(T)};  // x - c_x for c_x = -1, 0, +1
  R f[L::Q];
  load_phase_begin<T>();
#pragma unroll
  for (int q = 0; q < L::Q; ++q)
    f[q] = Storage<T>::load(at_bytes(plane_row<L>(A, opp<L>(q), q, c, ym, yp, zm, zp, g), ox[L::c(q, 0) + 1]));
  load_phase_end<T>();
  uint32_t m = 0;   // bit q: x - c_q is solid, i.e. x + c_opp(q) is solid
  if (fl & 2) {
    m = p.links[c.cell];
#pragma unroll
    for (int q = 1; q < L::Q; ++q) {
      if ((m >> q) & 1u) {
        f[q] = Storage<T>::load(A + (size_t)q * (size_t)g.N + c.cell);
        if (p.moving)
          f[q] += wall_term<L>(q, flags[upstream<L>(q, c, g, xm, xp, ym, yp, zm, zp)] >> 1, p.wall, p.rho0);
      }
    }
  }
  const R F[3] = {force_y[3 * c.y], force_y[3 * c.y + 1], force_y[3 * c.y + 2]};
  collide<L, M>(f, F, p);
  if (tape) tape_store<L, T>(tape, c, g, f);
  if (!(fl & 2)) {
#pragma unroll
    for (int q = 0; q < L::Q; ++q)
      put<T, NT>(at_bytes(plane_row<L>(A, q, opp<L>(q), c, ym, yp, zm, zp, g), ox[L::c(opp<L>(q), 0) + 1]), f[q]);
  } else {
    // next to a wall: links into solid cells bounce back into the cell's own
    // opposite slot; solid cells' slots are never written
#pragma unroll
    for (int q = 0; q < L::Q; ++q) {
      if (q > 0 && ((m >> opp<L>(q)) & 1u))   // x + c_q is solid: the value re-enters along opp(q), and
        put<T, NT>(A + (size_t)opp<L>(q) * (size_t)g.N + c.cell, f[q]);   // the even kernel adds the wall term
      else
        put<T, NT>(at_bytes(plane_row<L>(A, q, opp<L>(q), c, ym, yp, zm, zp, g), ox[L::c(opp<L>(q), 0) + 1]),
                   f[q]);
    }
  }
}

template <class T>
__device__ __forceinline__ void store_from_double(T* p, double v) {
  *p = static_cast<T>(v);
}

// ------------------------------------------------------------------ layouts
// Where the post-collision populations P^t(x, q) of the stored state live:
//   0  two-array pattern: slot (x, q);
//   1  AA, after an even kernel: slot (x, opp q);
//   2  AA, after an odd kernel or after initialisation: slot (x + c_q, q),
//      or (x, opp q) when x + c_q is solid.
// Solid cells keep their own slots (x, q) in every layout.
//   In layout 2 a bounced slot holds the cell's own outgoing population;
//   the moving-wall term of the population that re-enters from it is added
//   by the even kernel when it loads the slot (as the two-array gather
//   does), so every stored value is a post-collision value.
template <class L, class T>
__device__ __forceinline__ void load_post(const T* P, const uint8_t* flags, int has_mask, int layout,
                                          const CellIdx& c, const Geo& g, double* v) {
  const size_t N = (size_t)g.N;
  const int fl = has_mask ? flags[c.cell] : 0;
  if (layout == 0 || (fl & 1)) {
#pragma unroll
    for (int q = 0; q < L::Q; ++q) v[q] = (double)Storage<T>::load(P + q * N + c.cell);
  } else if (layout == 1) {
#pragma unroll
    for (int q = 0; q < L::Q; ++q) v[q] = (double)Storage<T>::load(P + opp<L>(q) * N + c.cell);
  } else {
    LBM_NEIGHBOURS(c, g)
#pragma unroll
    for (int q = 0; q < L::Q; ++q) {
      const int d = upstream<L>(opp<L>(q), c, g, xm, xp, ym, yp, zm, zp);  // x + c_q
      const int fs = (q > 0 && (fl & 2)) ? flags[d] : 0;   // neighbours are read next to walls only
      v[q] = (double)Storage<T>::load((fs & 1) ? P + opp<L>(q) * N + c.cell : P + q * N + d);
    }
  }
}

template <class L, class T>
__device__ __forceinline__ void store_post(T* P, const uint8_t* flags, int has_mask, int layout, const CellIdx& c,
                                           const Geo& g, const double* v) {
  const size_t N = (size_t)g.N;
  const int fl = has_mask ? flags[c.cell] : 0;
  if (layout == 0 || (fl & 1)) {
#pragma unroll
    for (int q = 0; q < L::Q; ++q) store_from_double(P + q * N + c.cell, v[q]);
  } else if (layout == 1) {
#pragma unroll
    for (int q = 0; q < L::Q; ++q) store_from_double(P + opp<L>(q) * N + c.cell, v[q]);
  } else {
    LBM_NEIGHBOURS(c, g)
#pragma unroll
    for (int q = 0; q < L::Q; ++q) {
      const int d = upstream<L>(opp<L>(q), c, g, xm, xp, ym, yp, zm, zp);  // x + c_q
      const int fs = (q > 0 && (fl & 2)) ? flags[d] : 0;   // neighbours are read next to walls only
      store_from_double((fs & 1) ? P + opp<L>(q) * N + c.cell : P + q * N + d, v[q]);
    }
  }
}

// phase -1: two-array sweep src -> dst; phase 0 / 1: AA even / odd kernel on
// src, and dst (if not null) receives the produced state in the two-array
// layout (a checkpoint of the tape).
template <class L, int M, class T>
hipError_t run_sweep(int phase, const void* src, void* dst, const uint8_t* flags, const void* force_y, const Geo& g,
                     const Params& p, int has_mask, hipStream_t s) {
  using R = typename Storage<T>::R;
  const CollideParams<R> cp = to_collide_params<R>(p);
  // non-temporal stores once the grid clearly exceeds the on-chip caches
  const bool nt = (size_t)g.N * L::Q * sizeof(T) > kStreamGridBytes;
  const dim3 grid((unsigned)num_blocks(g)), block(g.bx);
  if (phase < 0) {
    // Waves per CU of the two-array sweep on streaming grids, measured per
    // storage type and operator (256^3 and 384^3 lattices): 12 for FP64
    // SRT / TRT / MRT / unit-rate cumulant; FP32 SRT / TRT 16 on D3Q19 and
    // 12 on D3Q27; full occupancy for the rest (16-bit, FP32 MRT, which lost
    // 7 % at 12, FP32 cumulant, KBC, Smagorinsky)
    constexpr bool srt_trt = M == M_SRT || M == M_TRT;
    const int waves = !nt ? 0
                      : sizeof(T) == 8 ? ((srt_trt || M == M_MRT || M == M_MRT_UNIT || M == M_CUMULANT) ? 12 : 0)
                      : sizeof(T) == 4 ? (srt_trt ? (L::Q == 19 ? 16 : 12) : 0)
                                       : 0;
    const unsigned lds = occupancy_lds(waves, g.bx);
    if (nt)
      hipLaunchKernelGGL((k_sweep<L, M, T, 1>), grid, block, lds, s, (const T*)src, (T*)dst, flags,
                         (const R*)force_y, g, cp, has_mask);
    else
      hipLaunchKernelGGL((k_sweep<L, M, T, 0>), grid, block, 0, s, (const T*)src, (T*)dst, flags, (const R*)force_y,
                         g, cp, has_mask);
  } else if (phase == 0) {
    if (nt)
      hipLaunchKernelGGL((k_sweep_aa_even<L, M, T, 1>), grid, block, 0, s, (T*)src, flags, (const R*)force_y, g, cp,
                         has_mask, (T*)dst);
    else
      hipLaunchKernelGGL((k_sweep_aa_even<L, M, T, 0>), grid, block, 0, s, (T*)src, flags, (const R*)force_y, g, cp,
                         has_mask, (T*)dst);
  } else {
    if (nt)
      hipLaunchKernelGGL((k_sweep_aa_odd<L, M, T, 1>), grid, block, 0, s, (T*)src, flags, (const R*)force_y, g, cp,
                         has_mask, (T*)dst);
    else
      hipLaunchKernelGGL((k_sweep_aa_odd<L, M, T, 0>), grid, block, 0, s, (T*)src, flags, (const R*)force_y, g, cp,
                         has_mask, (T*)dst);
  }
  return hipGetLastError();
}

template <class L, int M>
hipError_t sweep_for_dtype(int dtype, int phase, const void* src, void* dst, const uint8_t* flags,
                           const void* force_y, const Geo& g, const Params& p, int has_mask, hipStream_t s) {
  switch (dtype) {
    case 0: return run_sweep<L, M, double>(phase, src, dst, flags, force_y, g, p, has_mask, s);
    case 1: return run_sweep<L, M, float>(phase, src, dst, flags, force_y, g, p, has_mask, s);
    case 2: return run_sweep<L, M, __bf16>(phase, src, dst, flags, force_y, g, p, has_mask, s);
    case 3: return run_sweep<L, M, _Float16>(phase, src, dst, flags, force_y, g, p, has_mask, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_sweep_d2q9(int method, int dtype, int phase, const void* src, void* dst, const uint8_t* flags,
                             const void* force_y, const Geo& g, const Params& p, int has_mask, hipStream_t s);
hipError_t launch_sweep_d3q19(int method, int dtype, int phase, const void* src, void* dst, const uint8_t* flags,
                              const void* force_y, const Geo& g, const Params& p, int has_mask, hipStream_t s);
hipError_t launch_sweep_d3q27(int method, int dtype, int phase, const void* src, void* dst, const uint8_t* flags,
                              const void* force_y, const Geo& g, const Params& p, int has_mask, hipStream_t s);

}  // namespace lbm
