// Host-side launch interface between the runtime (runtime.hip) and the
// kernels (sweep.hip, aux.hip, adjoint.hip).  Every launcher enqueues on the
// given stream and returns the launch status.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

// Geometry of one launch: one thread per cell, each block covers one
// contiguous x-segment of one (y, z) row; nxb segments per row.
struct Geo {
  int nx, ny, nz;
  int nxb;        // x-segments per row
  int bx;         // threads per block (multiple of 64)
  int64_t N;      // nx * ny * nz
  int order;      // block -> row-segment order, see cell_of: bit 0 reversed, bit 1 XCD slabs
};

// Grids of at most this many bytes are swept with cached stores and the
// cache-friendly block order; larger ones stream with non-temporal stores.
constexpr size_t kStreamGridBytes = size_t(512) << 20;

// Dynamic LDS bytes to request (and leave unused) so that at most
// `waves_per_cu` wavefronts of blocks of `block_threads` threads share a CU;
// 0 (no limit) when the request cannot express that.  A streaming kernel at
// full occupancy keeps more loads in flight than HBM needs, and fewer
// resident waves measured faster for some of them.
unsigned occupancy_lds(int waves_per_cu, int block_threads);

// Runtime parameters in FP64; each launcher converts to its compute type.
struct Params {
  double rho0;
  double om, om_b, om_o;
  double hi[4];
  double smag18;   // 18 C_S^2 (Smagorinsky), 0 = off
  int compressible;
  const void* wall; // device table [128][3] of wall velocities (compute type), row = wall id
  const uint32_t* links;  // per-cell bounced-link bits (NULL without a mask)
  int moving;             // the mask holds moving-wall types
};

inline int64_t num_blocks(const Geo& g) { return (int64_t)g.nxb * g.ny * g.nz; }

// Record the thread-local message lbm_last_error() returns (printf format)
// and return `code`.
int32_t set_last_error(int32_t code, const char* fmt, ...);

// forward
// phase -1: two-array sweep src -> dst; 0 / 1: AA even / odd kernel in place on src,
// with dst (if not null) receiving the produced state in the two-array layout
hipError_t launch_sweep(int stencil, int method, int dtype, int phase, const void* src, void* dst,
                        const uint8_t* flags, const void* force_y, const Geo& g, const Params& p,
                        int has_mask, hipStream_t s);
bool sweep_supported(int stencil, int method);   // method: kernel code (collide.h)

// auxiliary (aux.hip)
// flags (one byte per cell) and the bounced-link bits of every cell
hipError_t launch_build_flags(int stencil, const uint8_t* solid, uint8_t* flags, uint32_t* links,
                              const Geo& g, hipStream_t s);
// layout of the stored state: 0 two-array; 1 AA after an even kernel;
// 2 AA streamed (after an odd kernel or initialisation)
hipError_t launch_init(int stencil, int dtype, void* P, const uint8_t* flags, int has_mask, int layout,
                       const void* rho, const void* u, int field_dtype, const Geo& g,
                       const Params& p, hipStream_t s);
hipError_t launch_readout(int stencil, int dtype, const void* P, const uint8_t* flags, int has_mask, int layout,
                          const void* force_y, void* rho, void* u, int field_dtype, const Geo& g,
                          const Params& p, hipStream_t s);
hipError_t launch_conserved(int stencil, int dtype, const void* P, const uint8_t* flags,
                            int has_mask, int layout, double* partials, double* out4, const Geo& g,
                            const Params& p, hipStream_t s);
// The same totals through the library's static scratch (no allocation):
// at most kNoAllocSlots partial rows of 4 doubles on each device.
constexpr int kNoAllocSlots = 4096;
constexpr int kMaxDevices = 64;
// Record the device address of the scratch on `device` (which must be the
// current device); idempotent.  Called by lbm_create.
hipError_t noalloc_scratch_setup(int device);
// That address, or NULL before setup.
double* noalloc_scratch(int device);
hipError_t launch_conserved_noalloc(int stencil, int dtype, const void* P, const uint8_t* flags, int has_mask,
                                    int layout, double* scratch_dev, int nslots, double* out4, const Geo& g,
                                    const Params& p, hipStream_t s);
// Solid cells are read from P_solid (the buffer that keeps their values).
hipError_t launch_get_pdfs(int stencil, int dtype, const void* P, const void* P_solid, const uint8_t* flags,
                           int has_mask, int layout, double* out, const Geo& g, const Params& p, hipStream_t s);
hipError_t launch_set_pdfs(int stencil, int dtype, void* P, const uint8_t* flags, int has_mask, int layout,
                           const double* in, const Geo& g, const Params& p, hipStream_t s);
hipError_t launch_relayout(int stencil, int dtype, const void* P, const uint8_t* flags, int has_mask,
                           int layout, void* out, const Geo& g, const Params& p, hipStream_t s);
hipError_t launch_copy_q(const void* src, void* dst, int64_t n, int q, int elem_bytes, int waves_per_cu,
                         int block_threads, hipStream_t s);
// pull-streaming reference over the row-segment launch shape of g
hipError_t launch_stream_q(const void* src, void* dst, int stencil, const Geo& g, int elem_bytes,
                           int waves_per_cu, hipStream_t s);
hipError_t launch_stream_aa_q(void* buf, int stencil, const Geo& g, int elem_bytes, int odd, int waves_per_cu,
                              hipStream_t s);
hipError_t launch_sum_partials(const double* partials, int64_t nparts, int width, double* acc,
                               int accumulate, hipStream_t s);
hipError_t launch_fill_zero(void* p, int64_t bytes, hipStream_t s);

// adjoint (adjoint.hip)
bool adjoint_supported(int stencil, int method);
// Layouts as for the stored state (0 two arrays, 1 AA inverted, 2
// streamed): the seed reads P in `layout` and places lambda in `lam_layout`
// (the AA layout of the seeded time); the init gradient reads lambda in
// `layout`.
hipError_t launch_adjoint_seed(int stencil, int dtype, const void* P, const uint8_t* flags,
                               int has_mask, int layout, int lam_layout, const void* force_y,
                               const void* dL_drho, const void* dL_du, int field_dtype, void* lam,
                               double* partials, const Geo& g, const Params& p, hipStream_t s);
// Transpose of one time step: phase 0 / 1 = of the AA even / odd kernel, in
// place on lam.  P is the forward state of the reversed step in the
// two-array layout (the tape and the recomputed segment hold that layout).
hipError_t launch_adjoint_sweep(int stencil, int method, int dtype, int phase, const void* P,
                                const uint8_t* flags, int has_mask, const void* force_y, void* lam,
                                double* partials, const Geo& g, const Params& p, hipStream_t s);
hipError_t launch_adjoint_init_grad(int stencil, int dtype, const void* lam, const uint8_t* flags,
                                    int has_mask, int layout, const void* init_fields, void* dL_du0,
                                    void* dL_drho0, int field_dtype, const Geo& g,
                                    const Params& p, hipStream_t s);
hipError_t launch_store_init_fields(int dtype, const void* rho, const void* u, int field_dtype,
                                   void* init_fields, const Geo& g, const Params& p,
                                   hipStream_t s);

}  // namespace lbm
