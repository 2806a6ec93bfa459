// Per-cell kernels around the sweep: flag building, initialisation,
// macroscopic readout, FP64 conservation totals, PDF import/export, the
// Q-stream copy bandwidth reference, and small reduction helpers.
//
// These run once per run or once per readout, not per time step, so they
// compute in FP64 regardless of the storage type.
#include <algorithm>
#include <mutex>

#include "sweep.h"

namespace lbm {

// --------------------------------------------------------------- dispatch
bool sweep_supported(int stencil, int method) {   // kernel method code
  if (method == M_SRT || method == M_TRT || method == M_MRT || method == M_KBC || method == M_SRT_SMAG ||
      method == M_MRT_SMAG)
    return stencil >= 0 && stencil <= 2;
  if (method == M_CUMULANT || method == M_CUMULANT_GEN || method == M_MRT_UNIT) return stencil == 0 || stencil == 2;
  return false;
}

hipError_t launch_sweep(int stencil, int method, int dtype, int phase, const void* src, void* dst,
                        const uint8_t* flags, const void* force_y, const Geo& g, const Params& p, int has_mask,
                        hipStream_t s) {
  switch (stencil) {
    case 0: return launch_sweep_d2q9(method, dtype, phase, src, dst, flags, force_y, g, p, has_mask, s);
    case 1: return launch_sweep_d3q19(method, dtype, phase, src, dst, flags, force_y, g, p, has_mask, s);
    case 2: return launch_sweep_d3q27(method, dtype, phase, src, dst, flags, force_y, g, p, has_mask, s);
  }
  return hipErrorInvalidValue;
}

#define LBM_STENCIL_SWITCH(stencil, CALL) \
  switch (stencil) {                      \
    case 0: { using L = D2Q9; CALL; }     \
    case 1: { using L = D3Q19; CALL; }    \
    case 2: { using L = D3Q27; CALL; }    \
  }                                       \
  return hipErrorInvalidValue;

#define LBM_DTYPE_SWITCH(dtype, CALL)          \
  switch (dtype) {                             \
    case 0: { using T = double; CALL; }        \
    case 1: { using T = float; CALL; }         \
    case 2: { using T = __bf16; CALL; }        \
    case 3: { using T = _Float16; CALL; }      \
  }                                            \
  return hipErrorInvalidValue;

template <class FT>
__device__ __forceinline__ double ld_field(const void* p, size_t i) {
  return (double)((const FT*)p)[i];
}

__device__ __forceinline__ double ld_any(const void* p, size_t i, int field_dtype) {
  return field_dtype == 0 ? ((const double*)p)[i] : (double)((const float*)p)[i];
}

__device__ __forceinline__ void st_any(void* p, size_t i, double v, int field_dtype) {
  if (field_dtype == 0)
    ((double*)p)[i] = v;
  else
    ((float*)p)[i] = (float)v;
}

// Block-wide sum of `v` for every component; result valid in thread 0.
template <int W>
__device__ __forceinline__ void block_sum(double (&v)[W]) {
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


// --------------------------------------------------------------- flags
// bit 0: solid (bits 1..7 then hold the wall type); for fluid cells bit 1:
// at least one solid upstream neighbour.  links: for fluid cells bit q set
// when x - c_q is solid (the links the sweep bounces back), else 0.
template <class L>
__global__ __launch_bounds__(512) void k_build_flags(const uint8_t* __restrict__ solid, uint8_t* __restrict__ flags,
                                                     uint32_t* __restrict__ links, Geo g) {
  const CellIdx c = cell_of(g);
  if (!c.valid) return;
  LBM_NEIGHBOURS(c, g)
  // solid cells: bit 0 set, bits 1..7 = wall type (the mask value)
  uint8_t f = solid[c.cell] ? (uint8_t)(1u | ((unsigned)solid[c.cell] << 1)) : 0;
  uint32_t m = 0;
  if (!f) {
#pragma unroll
    for (int q = 1; q < L::Q; ++q)
      if (solid[upstream<L>(q, c, g, xm, xp, ym, yp, zm, zp)] != 0) m |= 1u << q;
    if (m) f |= 2;
  }
  flags[c.cell] = f;
  links[c.cell] = m;
}

hipError_t launch_build_flags(int stencil, const uint8_t* solid, uint8_t* flags, uint32_t* links, const Geo& g,
                              hipStream_t s) {
  LBM_STENCIL_SWITCH(stencil, {
    hipLaunchKernelGGL(k_build_flags<L>, dim3((unsigned)num_blocks(g)), dim3(g.bx), 0, s, solid, flags, links, g);
    return hipGetLastError();
  })
}

// --------------------------------------------------------------- init
// P = f^eq(rho, u) (Eq. 3, second order), stored shifted by w rho_0.
template <class L, class T>
__global__ __launch_bounds__(512) void k_init(T* P, const uint8_t* __restrict__ flags, int has_mask, int layout,
                                              const void* rho, const void* u, int fdt, Geo g, double rho0,
                                              int compressible) {
  const CellIdx c = cell_of(g);
  if (!c.valid) return;
  const size_t N = (size_t)g.N;
  const bool solid = has_mask && (flags[c.cell] & 1);
  const double r = rho ? ld_any(rho, c.cell, fdt) : rho0;
  double ux = 0, uy = 0, uz = 0;
  if (u) {
    ux = ld_any(u, c.cell, fdt);
    uy = ld_any(u, N + c.cell, fdt);
    uz = ld_any(u, 2 * N + c.cell, fdt);
  }
  const double rr = compressible ? r : rho0;
  const double usq = 1.5 * (ux * ux + uy * uy + uz * uz);
  double v[L::Q];
#pragma unroll
  for (int q = 0; q < L::Q; ++q) {
    v[q] = 0.0;
    if (!solid) {
      const double cu = cdot<L>(q, ux, uy, uz);
      v[q] = weight<L>(q) * ((r - rho0) + rr * (3.0 * cu + 4.5 * cu * cu - usq));
    }
  }
  store_post<L, T>(P, flags, has_mask, layout, c, g, v);
}

hipError_t launch_init(int stencil, int dtype, void* P, const uint8_t* flags, int has_mask, int layout,
                       const void* rho, const void* u, int field_dtype, const Geo& g, const Params& p, hipStream_t s) {
  LBM_STENCIL_SWITCH(stencil, {
    LBM_DTYPE_SWITCH(dtype, {
      hipLaunchKernelGGL((k_init<L, T>), dim3((unsigned)num_blocks(g)), dim3(g.bx), 0, s, (T*)P, flags, has_mask,
                         layout, rho, u, field_dtype, g, p.rho0, p.compressible);
      return hipGetLastError();
    })
  })
}

// --------------------------------------------------------------- readout
// Stored state is post-collision: rho = sum f, u = (sum c f - F/2) / rho_0.
template <class L, class T>
__global__ __launch_bounds__(512) void k_readout(const T* __restrict__ P, const uint8_t* __restrict__ flags,
                                                 int has_mask, int layout, const typename Storage<T>::R* __restrict__ force_y,
                                                 void* rho_out, void* u_out, int fdt, Geo g, double rho0,
                                                 int compressible) {
  const CellIdx c = cell_of(g);
  if (!c.valid) return;
  const size_t N = (size_t)g.N;
  double r = 0, ux = 0, uy = 0, uz = 0;
  if (!(has_mask && (flags[c.cell] & 1))) {
    double f[L::Q];
    load_post<L, T>(P, flags, has_mask, layout, c, g, f);
    double d = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
    for (int q = 0; q < L::Q; ++q) {
      const double v = f[q];
      d += v;
      jx += L::c(q, 0) * v;
      jy += L::c(q, 1) * v;
      jz += L::c(q, 2) * v;
    }
    r = rho0 + d;
    const double inv = 1.0 / (compressible ? r : rho0);
    ux = (jx - 0.5 * (double)force_y[3 * c.y]) * inv;
    uy = (jy - 0.5 * (double)force_y[3 * c.y + 1]) * inv;
    uz = (jz - 0.5 * (double)force_y[3 * c.y + 2]) * inv;
  }
  if (rho_out) st_any(rho_out, c.cell, r, fdt);
  if (u_out) {
    st_any(u_out, c.cell, ux, fdt);
    st_any(u_out, N + c.cell, uy, fdt);
    st_any(u_out, 2 * N + c.cell, uz, fdt);
  }
}

hipError_t launch_readout(int stencil, int dtype, const void* P, const uint8_t* flags, int has_mask, int layout,
                          const void* force_y, void* rho, void* u, int field_dtype, const Geo& g, const Params& p,
                          hipStream_t s) {
  LBM_STENCIL_SWITCH(stencil, {
    LBM_DTYPE_SWITCH(dtype, {
      using R = typename Storage<T>::R;
      hipLaunchKernelGGL((k_readout<L, T>), dim3((unsigned)num_blocks(g)), dim3(g.bx), 0, s, (const T*)P, flags,
                         has_mask, layout, (const R*)force_y, rho, u, field_dtype, g, p.rho0, p.compressible);
      return hipGetLastError();
    })
  })
}

// --------------------------------------------------------------- totals
template <class L, class T>
__global__ __launch_bounds__(512) void k_conserved(const T* __restrict__ P, const uint8_t* __restrict__ flags,
                                                   int has_mask, int layout, double* __restrict__ partials, Geo g,
                                                   double rho0) {
  const CellIdx c = cell_of(g);
  double v[4] = {0, 0, 0, 0};
  if (c.valid && !(has_mask && (flags[c.cell] & 1))) {
    double pf[L::Q];
    load_post<L, T>(P, flags, has_mask, layout, c, g, pf);
    double d = 0;
#pragma unroll
    for (int q = 0; q < L::Q; ++q) {
      const double f = pf[q];
      d += f;
      v[1] += L::c(q, 0) * f;
      v[2] += L::c(q, 1) * f;
      v[3] += L::c(q, 2) * f;
    }
    v[0] = rho0 + d;
  }
  block_sum<4>(v);
  if (threadIdx.x == 0)
    for (int k = 0; k < 4; ++k) partials[(size_t)blockIdx.x * 4 + k] = v[k];
}

// Single-block reduction of nparts rows of `width` doubles into acc.
__global__ __launch_bounds__(256) void k_sum_partials(const double* __restrict__ partials, int64_t nparts,
                                                      int width, double* __restrict__ acc, int accumulate) {
  for (int k = 0; k < width; ++k) {
    double v[1] = {0.0};
    for (int64_t i = threadIdx.x; i < nparts; i += blockDim.x) v[0] += partials[i * width + k];
    block_sum<1>(v);
    if (threadIdx.x == 0) acc[k] = accumulate ? acc[k] + v[0] : v[0];
    __syncthreads();
  }
}

hipError_t launch_sum_partials(const double* partials, int64_t nparts, int width, double* acc, int accumulate,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, partials, nparts, width, acc, accumulate);
  return hipGetLastError();
}

hipError_t launch_conserved(int stencil, int dtype, const void* P, const uint8_t* flags, int has_mask, int layout,
                            double* partials, double* out4, const Geo& g, const Params& p, hipStream_t s) {
  hipError_t e = hipSuccess;
  auto body = [&](auto lat, auto tag) -> hipError_t {
    using L = decltype(lat);
    using T = decltype(tag);
    hipLaunchKernelGGL((k_conserved<L, T>), dim3((unsigned)num_blocks(g)), dim3(g.bx), 0, s, (const T*)P, flags,
                       has_mask, layout, partials, g, p.rho0);
    return hipGetLastError();
  };
  auto by_dtype = [&](auto lat) -> hipError_t {
    switch (dtype) {
      case 0: return body(lat, double());
      case 1: return body(lat, float());
      case 2: return body(lat, __bf16());
      case 3: return body(lat, _Float16());
    }
    return hipErrorInvalidValue;
  };
  switch (stencil) {
    case 0: e = by_dtype(D2Q9()); break;
    case 1: e = by_dtype(D3Q19()); break;
    case 2: e = by_dtype(D3Q27()); break;
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  return launch_sum_partials(partials, num_blocks(g), 4, out4, 0, s);
}

// --------------------------------------------------------------- totals without allocation
// Scratch of lbm_conserved_noalloc: one row of four FP64 partial totals per
// block of a strided reduction, for callers that cannot allocate device
// memory.  Every GPU holds its own copy for the life of the process.  Host
// code never names this array in a launch or copy: it uses the device
// address that noalloc_scratch_setup records for each device.
__device__ __align__(256) double scratch[kNoAllocSlots * 4];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_dev[device]) return hipSuccess;
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return e;
  if (cur != device) return hipErrorInvalidDevice;   // the symbol address is per device: look it up there
  void* p = nullptr;
  e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!p) return hipErrorInvalidSymbol;
  g_scratch_dev[device] = p;
  return hipSuccess;
}

double* noalloc_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return (double*)g_scratch_dev[device];
}

// The totals of k_conserved with a bounded grid: block b sums the row
// segments b, b + gridDim.x, ... (plain order), so gridDim.x partial rows
// cover any lattice.
template <class L, class T>
__global__ __launch_bounds__(512) void k_conserved_strided(const T* __restrict__ P, const uint8_t* __restrict__ flags,
                                                           int has_mask, int layout, double* __restrict__ partials,
                                                           Geo g, double rho0) {
  double v[4] = {0, 0, 0, 0};
  const int64_t nblk = (int64_t)g.nxb * g.ny * g.nz;
  for (int64_t b = blockIdx.x; b < nblk; b += gridDim.x) {
    CellIdx c;
    const int64_t row = b / g.nxb;
    c.x = (int)(b % g.nxb) * g.bx + (int)threadIdx.x;
    c.y = (int)(row % g.ny);
    c.z = (int)(row / g.ny);
    c.cell = (int)(row * g.nx) + c.x;
    c.valid = c.x < g.nx;
    if (!c.valid || (has_mask && (flags[c.cell] & 1))) continue;
    double pf[L::Q];
    load_post<L, T>(P, flags, has_mask, layout, c, g, pf);
    double d = 0;
#pragma unroll
    for (int q = 0; q < L::Q; ++q) {
      const double f = pf[q];
      d += f;
      v[1] += L::c(q, 0) * f;
      v[2] += L::c(q, 1) * f;
      v[3] += L::c(q, 2) * f;
    }
    v[0] += rho0 + d;
  }
  block_sum<4>(v);
  if (threadIdx.x == 0)
    for (int k = 0; k < 4; ++k) partials[(size_t)blockIdx.x * 4 + k] = v[k];
}

hipError_t launch_conserved_noalloc(int stencil, int dtype, const void* P, const uint8_t* flags, int has_mask,
                                    int layout, double* scratch_dev, int nslots, double* out4, const Geo& g,
                                    const Params& p, hipStream_t s) {
  if (!scratch_dev || nslots < 1 || nslots > kNoAllocSlots) return hipErrorInvalidValue;
  auto body = [&](auto lat, auto tag) -> hipError_t {
    using L = decltype(lat);
    using T = decltype(tag);
    hipLaunchKernelGGL((k_conserved_strided<L, T>), dim3((unsigned)nslots), dim3(g.bx), 0, s, (const T*)P, flags,
                       has_mask, layout, scratch_dev, g, p.rho0);
    return hipGetLastError();
  };
  auto by_dtype = [&](auto lat) -> hipError_t {
    switch (dtype) {
      case 0: return body(lat, double());
      case 1: return body(lat, float());
      case 2: return body(lat, __bf16());
      case 3: return body(lat, _Float16());
    }
    return hipErrorInvalidValue;
  };
  hipError_t e = hipErrorInvalidValue;
  switch (stencil) {
    case 0: e = by_dtype(D2Q9()); break;
    case 1: e = by_dtype(D3Q19()); break;
    case 2: e = by_dtype(D3Q27()); break;
  }
  if (e != hipSuccess) return e;
  return launch_sum_partials(scratch_dev, nslots, 4, out4, 0, s);
}

// --------------------------------------------------------------- PDF I/O
template <class L, class T>
__global__ __launch_bounds__(512) void k_get_pdfs(const T* __restrict__ P, const T* __restrict__ P_solid,
                                                  const uint8_t* __restrict__ flags, int has_mask, int layout,
                                                  double* __restrict__ out, Geo g, double rho0) {
  const CellIdx c = cell_of(g);
  if (!c.valid) return;
  const size_t N = (size_t)g.N;
  double v[L::Q];
  if (has_mask && (flags[c.cell] & 1)) {   // solid cells keep their own slots in every layout
#pragma unroll
    for (int q = 0; q < L::Q; ++q) v[q] = (double)Storage<T>::load(P_solid + q * N + c.cell);
  } else {
    load_post<L, T>(P, flags, has_mask, layout, c, g, v);
  }
#pragma unroll
  for (int q = 0; q < L::Q; ++q) out[q * N + c.cell] = v[q] + weight<L>(q) * rho0;
}

template <class L, class T>
__global__ __launch_bounds__(512) void k_set_pdfs(T* P, const uint8_t* __restrict__ flags, int has_mask, int layout,
                                                  const double* __restrict__ in, Geo g, double rho0) {
  const CellIdx c = cell_of(g);
  if (!c.valid) return;
  const size_t N = (size_t)g.N;
  double v[L::Q];
#pragma unroll
  for (int q = 0; q < L::Q; ++q) v[q] = in[q * N + c.cell] - weight<L>(q) * rho0;
  store_post<L, T>(P, flags, has_mask, layout, c, g, v);
}

hipError_t launch_get_pdfs(int stencil, int dtype, const void* P, const void* P_solid, const uint8_t* flags,
                           int has_mask, int layout, double* out, const Geo& g, const Params& p, hipStream_t s) {
  LBM_STENCIL_SWITCH(stencil, {
    LBM_DTYPE_SWITCH(dtype, {
      hipLaunchKernelGGL((k_get_pdfs<L, T>), dim3((unsigned)num_blocks(g)), dim3(g.bx), 0, s, (const T*)P,
                         (const T*)P_solid, flags, has_mask, layout, out, g, p.rho0);
      return hipGetLastError();
    })
  })
}

hipError_t launch_set_pdfs(int stencil, int dtype, void* P, const uint8_t* flags, int has_mask, int layout,
                           const double* in, const Geo& g, const Params& p, hipStream_t s) {
  LBM_STENCIL_SWITCH(stencil, {
    LBM_DTYPE_SWITCH(dtype, {
      hipLaunchKernelGGL((k_set_pdfs<L, T>), dim3((unsigned)num_blocks(g)), dim3(g.bx), 0, s, (T*)P, flags,
                         has_mask, layout, in, g, p.rho0);
      return hipGetLastError();
    })
  })
}

// --------------------------------------------------------------- relayout
// Copy a stored state from `layout` into the two-array layout of another
// buffer, in the storage type (the adjoint tape of the AA pattern); every
// value is copied bit for bit (each slot holds a post-collision value).
template <class L, class T>
__global__ __launch_bounds__(512) void k_relayout(const T* __restrict__ P, const uint8_t* __restrict__ flags,
                                                  int has_mask, int layout, T* __restrict__ out, Geo g) {
  const CellIdx c = cell_of(g);
  if (!c.valid) return;
  const size_t N = (size_t)g.N;
  double v[L::Q];
  load_post<L, T>(P, flags, has_mask, layout, c, g, v);
#pragma unroll
  for (int q = 0; q < L::Q; ++q) store_from_double(out + q * N + c.cell, v[q]);
}

hipError_t launch_relayout(int stencil, int dtype, const void* P, const uint8_t* flags, int has_mask, int layout,
                           void* out, const Geo& g, const Params& p, hipStream_t s) {
  LBM_STENCIL_SWITCH(stencil, {
    LBM_DTYPE_SWITCH(dtype, {
      hipLaunchKernelGGL((k_relayout<L, T>), dim3((unsigned)num_blocks(g)), dim3(g.bx), 0, s, (const T*)P, flags,
                         has_mask, layout, (T*)out, g);
      return hipGetLastError();
    })
  })
}

// The reference kernels raise their wave priority while they issue their
// loads where that makes them faster, as the sweeps do: with 2-byte
// elements (512^3, 27 planes: pull 4.8-5.1 -> 5.6-5.9 TB/s, copy 5.0-5.2 ->
// 5.4-5.5 TB/s in alternating processes); 4-byte lines were not faster.
template <class E>
__device__ __forceinline__ void ref_load_begin() {
  if (sizeof(E) == 2) __builtin_amdgcn_s_setprio(2);
}
template <class E>
__device__ __forceinline__ void ref_load_end() {
  if (sizeof(E) == 2) __builtin_amdgcn_s_setprio(0);
}

// --------------------------------------------------------------- copy-Q
// Bandwidth reference: same thread layout and access pattern as the sweep
// (all Q loads, then all Q stores; blocks of the sweep's row length), without
// the gather offsets or arithmetic.  Arrays larger than the caches store
// non-temporally, as the sweep does.
template <class E, int Q, int NT>
__global__ __launch_bounds__(512) void k_copy_q(const E* __restrict__ src, E* __restrict__ dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  E v[Q];
  ref_load_begin<E>();
#pragma unroll
  for (int q = 0; q < Q; ++q) v[q] = src[q * n + i];
  ref_load_end<E>();
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    if (NT)
      __builtin_nontemporal_store(v[q], dst + q * n + i);
    else
      dst[q * n + i] = v[q];
  }
}

template <class E, int NT>
__global__ __launch_bounds__(512) void k_copy_generic(const E* __restrict__ src, E* __restrict__ dst, int64_t n,
                                                      int Q) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int q = 0; q < Q; ++q) {
    if (NT)
      __builtin_nontemporal_store(src[q * n + i], dst + q * n + i);
    else
      dst[q * n + i] = src[q * n + i];
  }
}

// The copy reference runs with the occupancy and block size the caller names
// (the launch shape of the sweep it is compared with): at most waves_per_cu
// wavefronts per CU (0 = full occupancy), block_threads per block.
template <class E, int NT>
hipError_t copy_q_nt(const void* src, void* dst, int64_t n, int q, int waves_per_cu, int block_threads,
                     hipStream_t s) {
  const dim3 grid((unsigned)((n + block_threads - 1) / block_threads)), block(block_threads);
  const unsigned lds = occupancy_lds(waves_per_cu, block_threads);
  switch (q) {
    case 9: hipLaunchKernelGGL((k_copy_q<E, 9, NT>), grid, block, lds, s, (const E*)src, (E*)dst, n); break;
    case 19: hipLaunchKernelGGL((k_copy_q<E, 19, NT>), grid, block, lds, s, (const E*)src, (E*)dst, n); break;
    case 27: hipLaunchKernelGGL((k_copy_q<E, 27, NT>), grid, block, lds, s, (const E*)src, (E*)dst, n); break;
    default: hipLaunchKernelGGL((k_copy_generic<E, NT>), grid, block, lds, s, (const E*)src, (E*)dst, n, q);
  }
  return hipGetLastError();
}

template <class E>
hipError_t copy_q_typed(const void* src, void* dst, int64_t n, int q, int waves_per_cu, int block_threads,
                        hipStream_t s) {
  if ((size_t)n * (size_t)q * sizeof(E) > kStreamGridBytes)
    return copy_q_nt<E, 1>(src, dst, n, q, waves_per_cu, block_threads, s);
  return copy_q_nt<E, 0>(src, dst, n, q, waves_per_cu, block_threads, s);
}

// Pull-streaming reference: the sweep's access pattern without its
// arithmetic.  Every cell pulls plane q from its periodic upstream neighbour
// x - c_q and stores it in its own slot, dst[q][x] = src[q][x - c_q], with
// the sweep's addressing (scalar row bases, one block per row segment) and
// store type, so its rate is what the sweep's loads and stores reach with no
// collision in between.
template <class L, class E, int NT>
__global__ __launch_bounds__(512) void k_stream_q(const E* __restrict__ src, E* __restrict__ dst, Geo g) {
  const CellIdx c = cell_of(g);
  if (!c.valid) return;
  LBM_NEIGHBOURS(c, g)
  const uint32_t ox[3] = {(uint32_t)xp * (uint32_t)sizeof(E), (uint32_t)c.x * (uint32_t)sizeof(E),
                          (uint32_t)xm * (uint32_t)sizeof(E)};  // source x for c_x = -1, 0, +1
  E v[L::Q];
  ref_load_begin<E>();
#pragma unroll
  for (int q = 0; q < L::Q; ++q)
    v[q] = *at_bytes(row_base<L>(src, q, c.y, c.z, ym, yp, zm, zp, g), ox[L::c(q, 0) + 1]);
  ref_load_end<E>();
  E* row = dst + (size_t)(c.z * g.ny + c.y) * (size_t)g.nx;
#pragma unroll
  for (int q = 0; q < L::Q; ++q) {
    E* d = at_bytes(row + (size_t)q * (size_t)g.N, ox[1]);
    if (NT)
      __builtin_nontemporal_store(v[q], d);
    else
      *d = v[q];
  }
}

template <class L, class E>
hipError_t stream_q_typed(const void* src, void* dst, const Geo& g, int waves_per_cu, hipStream_t s) {
  const dim3 grid((unsigned)num_blocks(g)), block(g.bx);
  const unsigned lds = occupancy_lds(waves_per_cu, g.bx);
  if ((size_t)g.N * L::Q * sizeof(E) > kStreamGridBytes)
    hipLaunchKernelGGL((k_stream_q<L, E, 1>), grid, block, lds, s, (const E*)src, (E*)dst, g);
  else
    hipLaunchKernelGGL((k_stream_q<L, E, 0>), grid, block, lds, s, (const E*)src, (E*)dst, g);
  return hipGetLastError();
}

template <class L>
hipError_t stream_q_stencil(const void* src, void* dst, const Geo& g, int elem_bytes, int waves_per_cu,
                            hipStream_t s) {
  switch (elem_bytes) {
    case 2: return stream_q_typed<L, uint16_t>(src, dst, g, waves_per_cu, s);
    case 4: return stream_q_typed<L, uint32_t>(src, dst, g, waves_per_cu, s);
    case 8: return stream_q_typed<L, uint64_t>(src, dst, g, waves_per_cu, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_stream_q(const void* src, void* dst, int stencil, const Geo& g, int elem_bytes,
                           int waves_per_cu, hipStream_t s) {
  switch (stencil) {
    case 0: return stream_q_stencil<D2Q9>(src, dst, g, elem_bytes, waves_per_cu, s);
    case 1: return stream_q_stencil<D3Q19>(src, dst, g, elem_bytes, waves_per_cu, s);
    case 2: return stream_q_stencil<D3Q27>(src, dst, g, elem_bytes, waves_per_cu, s);
  }
  return hipErrorInvalidValue;
}

// AA-pattern reference: the two in-place kernels of the AA sweep with no
// collision in between (Sec. IV-B, Fig. "AA update pattern").  The even
// kernel reads a cell's own slots and writes them back inverted, A[opp q][x]
// = A[q][x]; the odd kernel reads A[opp q][x - c_q] and writes the value to
// A[q][x + c_q] (periodic).  Each cell reads exactly the slots it writes, so
// both are race-free in place, with the AA kernels' addressing, block order
// and store type.
template <class L, class E, int ODD, int NT>
__global__ __launch_bounds__(512) void k_stream_aa_q(E* A, Geo g) {
  const CellIdx c = cell_of(g);
  if (!c.valid) return;
  E v[L::Q];
  if (!ODD) {
    E* row = A + (size_t)(c.z * g.ny + c.y) * (size_t)g.nx;
    const uint32_t ox = (uint32_t)c.x * (uint32_t)sizeof(E);
    ref_load_begin<E>();
#pragma unroll
    for (int q = 0; q < L::Q; ++q) v[q] = *at_bytes(row + (size_t)q * (size_t)g.N, ox);
    ref_load_end<E>();
#pragma unroll
    for (int q = 0; q < L::Q; ++q) {
      E* d = at_bytes(row + (size_t)opp<L>(q) * (size_t)g.N, ox);
      if (NT)
        __builtin_nontemporal_store(v[q], d);
      else
        *d = v[q];
    }
  } else {
    LBM_NEIGHBOURS(c, g)
    const uint32_t ox[3] = {(uint32_t)xp * (uint32_t)sizeof(E), (uint32_t)c.x * (uint32_t)sizeof(E),
                            (uint32_t)xm * (uint32_t)sizeof(E)};  // x - c_x for c_x = -1, 0, +1
    ref_load_begin<E>();
#pragma unroll
    for (int q = 0; q < L::Q; ++q)
      v[q] = *at_bytes(plane_row<L>(A, opp<L>(q), q, c, ym, yp, zm, zp, g), ox[L::c(q, 0) + 1]);
    ref_load_end<E>();
#pragma unroll
    for (int q = 0; q < L::Q; ++q) {
      E* d = at_bytes(plane_row<L>(A, q, opp<L>(q), c, ym, yp, zm, zp, g), ox[L::c(opp<L>(q), 0) + 1]);
      if (NT)
        __builtin_nontemporal_store(v[q], d);
      else
        *d = v[q];
    }
  }
}

template <class L, class E>
hipError_t stream_aa_q_typed(void* buf, const Geo& g, int odd, int waves_per_cu, hipStream_t s) {
  const dim3 grid((unsigned)num_blocks(g)), block(g.bx);
  const unsigned lds = occupancy_lds(waves_per_cu, g.bx);
  const bool nt = (size_t)g.N * L::Q * sizeof(E) > kStreamGridBytes;
  if (odd) {
    if (nt)
      hipLaunchKernelGGL((k_stream_aa_q<L, E, 1, 1>), grid, block, lds, s, (E*)buf, g);
    else
      hipLaunchKernelGGL((k_stream_aa_q<L, E, 1, 0>), grid, block, lds, s, (E*)buf, g);
  } else {
    if (nt)
      hipLaunchKernelGGL((k_stream_aa_q<L, E, 0, 1>), grid, block, lds, s, (E*)buf, g);
    else
      hipLaunchKernelGGL((k_stream_aa_q<L, E, 0, 0>), grid, block, lds, s, (E*)buf, g);
  }
  return hipGetLastError();
}

template <class L>
hipError_t stream_aa_q_stencil(void* buf, const Geo& g, int elem_bytes, int odd, int waves_per_cu, hipStream_t s) {
  switch (elem_bytes) {
    case 2: return stream_aa_q_typed<L, uint16_t>(buf, g, odd, waves_per_cu, s);
    case 4: return stream_aa_q_typed<L, uint32_t>(buf, g, odd, waves_per_cu, s);
    case 8: return stream_aa_q_typed<L, uint64_t>(buf, g, odd, waves_per_cu, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_stream_aa_q(void* buf, int stencil, const Geo& g, int elem_bytes, int odd, int waves_per_cu,
                              hipStream_t s) {
  switch (stencil) {
    case 0: return stream_aa_q_stencil<D2Q9>(buf, g, elem_bytes, odd, waves_per_cu, s);
    case 1: return stream_aa_q_stencil<D3Q19>(buf, g, elem_bytes, odd, waves_per_cu, s);
    case 2: return stream_aa_q_stencil<D3Q27>(buf, g, elem_bytes, odd, waves_per_cu, s);
  }
  return hipErrorInvalidValue;
}

unsigned occupancy_lds(int waves_per_cu, int block_threads) {
  static int lds_per_cu[64];   // LDS bytes per CU of each device, queried once
  int dev = 0;
  if (waves_per_cu <= 0 || hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0u;
  if (lds_per_cu[dev] <= 0) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess || v <= 0)
      return 0u;
    lds_per_cu[dev] = v;
  }
  const int blocks = waves_per_cu / ((block_threads + 63) / 64);   // resident blocks per CU wanted
  if (blocks < 2) return 0u;
  const int lds = std::min(65536, lds_per_cu[dev] / blocks);
  return lds_per_cu[dev] / lds == blocks ? (unsigned)lds : 0u;
}

hipError_t launch_copy_q(const void* src, void* dst, int64_t n, int q, int elem_bytes, int waves_per_cu,
                         int block_threads, hipStream_t s) {
  switch (elem_bytes) {
    case 2: return copy_q_typed<uint16_t>(src, dst, n, q, waves_per_cu, block_threads, s);
    case 4: return copy_q_typed<uint32_t>(src, dst, n, q, waves_per_cu, block_threads, s);
    case 8: return copy_q_typed<uint64_t>(src, dst, n, q, waves_per_cu, block_threads, s);
  }
  return hipErrorInvalidValue;
}

// --------------------------------------------------------------- zero fill
__global__ __launch_bounds__(256) void k_fill_zero(uint32_t* __restrict__ p, int64_t words) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < words; i += (int64_t)gridDim.x * 256) p[i] = 0u;
}

hipError_t launch_fill_zero(void* p, int64_t bytes, hipStream_t s) {
  const int64_t words = bytes / 4;  // every buffer here is a multiple of 4 bytes
  int64_t blocks = (words + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)blocks), dim3(256), 0, s, (uint32_t*)p, words);
  return hipGetLastError();
}

}  // namespace lbm
