// Velocity sets as compile-time tables for the device code.
//
// DdQq stencils of the paper (Sec. III-A) with the standard weights and
// c_s^2 = 1/3.  Direction order (shared with the C ABI, see include/lbm.h):
// q = 0 rest, q = 1..H one vector of each +/- pair, q = H+1..2H the
// negatives, so opp(q) = q +/- H.  All accessors are constexpr so that fully
// unrolled loops over q fold every coefficient into an immediate.
#pragma once

#include <hip/hip_runtime.h>

namespace lbm {

struct D2Q9 {
  static constexpr int Q = 9, H = 4, DIM = 2, ID = 0;
  __host__ __device__ static constexpr int c(int q, int a) {
    constexpr int t[9][3] = {{0, 0, 0},  {1, 0, 0},  {0, 1, 0},   {1, 1, 0},  {1, -1, 0},
                             {-1, 0, 0}, {0, -1, 0}, {-1, -1, 0}, {-1, 1, 0}};
    return t[q][a];
  }
};

struct D3Q19 {
  static constexpr int Q = 19, H = 9, DIM = 3, ID = 1;
  __host__ __device__ static constexpr int c(int q, int a) {
    constexpr int t[19][3] = {{0, 0, 0},  {1, 0, 0},   {0, 1, 0},   {0, 0, 1},  {1, 1, 0},
                              {1, -1, 0}, {1, 0, 1},   {1, 0, -1},  {0, 1, 1},  {0, 1, -1},
                              {-1, 0, 0}, {0, -1, 0},  {0, 0, -1},  {-1, -1, 0}, {-1, 1, 0},
                              {-1, 0, -1}, {-1, 0, 1}, {0, -1, -1}, {0, -1, 1}};
    return t[q][a];
  }
};

struct D3Q27 {
  static constexpr int Q = 27, H = 13, DIM = 3, ID = 2;
  __host__ __device__ static constexpr int c(int q, int a) {
    constexpr int t[27][3] = {
        {0, 0, 0},    {1, 0, 0},   {0, 1, 0},    {0, 0, 1},    {1, 1, 0},   {1, -1, 0},  {1, 0, 1},
        {1, 0, -1},   {0, 1, 1},   {0, 1, -1},   {1, 1, 1},    {1, 1, -1},  {1, -1, 1},  {1, -1, -1},
        {-1, 0, 0},   {0, -1, 0},  {0, 0, -1},   {-1, -1, 0},  {-1, 1, 0},  {-1, 0, -1}, {-1, 0, 1},
        {0, -1, -1},  {0, -1, 1},  {-1, -1, -1}, {-1, -1, 1},  {-1, 1, -1}, {-1, 1, 1}};
    return t[q][a];
  }
};

template <class L>
__host__ __device__ constexpr int opp(int q) {
  return q == 0 ? 0 : (q <= L::H ? q + L::H : q - L::H);
}

template <class L>
__host__ __device__ constexpr int csq(int q) {  // |c_q|^2
  return L::c(q, 0) * L::c(q, 0) + L::c(q, 1) * L::c(q, 1) + L::c(q, 2) * L::c(q, 2);
}

// Standard weights by |c|^2.  D2Q9 / D3Q27 are products of the 1-D weights
// (2/3, 1/6, 1/6); D3Q19 uses 1/3, 1/18, 1/36.
template <class L>
__host__ __device__ constexpr double weight(int q) {
  if (L::ID == 0) return csq<L>(q) == 0 ? 4.0 / 9.0 : (csq<L>(q) == 1 ? 1.0 / 9.0 : 1.0 / 36.0);
  if (L::ID == 1) return csq<L>(q) == 0 ? 1.0 / 3.0 : (csq<L>(q) == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
  return csq<L>(q) == 0 ? 8.0 / 27.0
                        : (csq<L>(q) == 1 ? 2.0 / 27.0 : (csq<L>(q) == 2 ? 1.0 / 54.0 : 1.0 / 216.0));
}

// Index of the direction with components (x, y, z); -1 if absent.
template <class L>
__host__ __device__ constexpr int qindex(int x, int y, int z) {
  for (int q = 0; q < L::Q; ++q)
    if (L::c(q, 0) == x && L::c(q, 1) == y && L::c(q, 2) == z) return q;
  return -1;
}

}  // namespace lbm
