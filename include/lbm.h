/*
 * lbm.h -- C ABI of the MI355X (gfx950) lattice Boltzmann stream-collide
 * library.  Plain C types only: host or device pointers and sizes.
 *
 * Method (paper: "lbmpy: Automatic code generation for efficient parallel
 * lattice Boltzmann methods", Bauer, Koestler, Ruede):
 *   - lattice: DdQq velocity sets on a regular periodic grid (Sec. III-A);
 *   - one time step = pull streaming from the upstream neighbours followed by
 *     the local collision, fused in one kernel over two arrays
 *     (Sec. IV-B, Fig. "stream-pull-collide"), or in place in one array with
 *     the AA pattern (Sec. IV-B, Fig. "AA update pattern");
 *   - collision: SRT (Eq. 1), TRT (Sec. III-C), MRT in a lattice-weighted
 *     orthogonal moment basis (Eq. 4, Sec. III-C "MRT"), cumulant (Eq. 9,
 *     Sec. III-B), the Smagorinsky model (Sec. III-C "Turbulence models",
 *     Eqs. 11-14) and the entropic KBC model (Sec. III-C "Entropic KBC
 *     Models"); equilibrium Eq. (3) at second order, density and velocity
 *     from Eq. (2); body force by Guo's scheme (cited in Sec. I);
 *   - walls: halfway velocity bounce-back (Sec. III-C "Boundary Conditions")
 *     for resting and moving walls, compiled into the sweep from a solid mask
 *     (Sec. IV-B "Boundary Conditions").
 * Extensions not in the paper: PDFs stored shifted by w_q rho_0 in FP32, BF16
 * or FP16 with FP32 collision arithmetic; a discrete adjoint sweep with a
 * checkpoint tape.
 *
 * Conventions for every call
 *   - Return value: lbm_status; LBM_OK (0) on success.  On failure nothing
 *     has been enqueued and lbm_last_error() describes the problem.
 *   - Arguments are validated on the host before any device work, so
 *     argument errors never touch the GPU.
 *   - Device pointers ("_dev") must be on the context's device.  Work is
 *     enqueued on the stream given to lbm_create (NULL = the null stream)
 *     and is asynchronous unless the function says "synchronises".
 *   - Field layout: x fastest, then y, then z.  Cell index
 *     i = (z * ny + y) * nx + x, N = nx * ny * nz.  Vector fields are
 *     component-major: component a of cell i at [a * N + i].
 *   - PDF layout (lbm_get_pdfs / lbm_set_pdfs): [q * N + i], unshifted FP64.
 *     Direction order: q = 0 is the rest vector; q = 1..h are the vectors
 *     listed below, q = h+1..2h their negatives (opposite(q) = q +/- h):
 *       D2Q9  (h=4):  (1,0) (0,1) (1,1) (1,-1)
 *       D3Q19 (h=9):  (1,0,0) (0,1,0) (0,0,1) (1,1,0) (1,-1,0) (1,0,1)
 *                     (1,0,-1) (0,1,1) (0,1,-1)
 *       D3Q27 (h=13): the D3Q19 list, then (1,1,1) (1,1,-1) (1,-1,1) (1,-1,-1)
 *   - A context is not thread-safe.  The context owns its device memory
 *     (PDF grids, tape, adjoint state); the caller owns every buffer it
 *     passes in.
 */
#ifndef LBM_MI355X_H
#define LBM_MI355X_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx;

/* Status, stencil, method and storage-type codes are plain int32_t values
 * (fixed width across compilers); the typedefs name what a value means. */
typedef int32_t lbm_status;
typedef int32_t lbm_stencil;
typedef int32_t lbm_method;
typedef int32_t lbm_dtype;

/* stencils (Sec. III-A) */
enum { LBM_D2Q9 = 0, LBM_D3Q19 = 1, LBM_D3Q27 = 2 };
/* collision operators: Eq. (1); Sec. III-C TRT; Eq. (4); Eq. (9); Sec. III-C
 * "Entropic KBC Models" (MRT with a per-cell higher-order rate) */
enum { LBM_SRT = 0, LBM_TRT = 1, LBM_MRT = 2, LBM_CUMULANT = 3, LBM_KBC = 4 };
/* PDF storage type (FP64 computes in FP64, the others in FP32); also used
 * to describe caller field buffers (only LBM_F64 / LBM_F32 there) */
enum { LBM_F64 = 0, LBM_F32 = 1, LBM_BF16 = 2, LBM_F16 = 3 };
/* status codes (lbm_status) */
enum {
  LBM_OK = 0,
  LBM_EINVAL = -1,        /* bad argument                                  */
  LBM_EUNSUPPORTED = -2,  /* valid request this library does not implement  */
  LBM_ENOMEM = -3,        /* device allocation failed                      */
  LBM_EHIP = -4,          /* a HIP runtime call failed                     */
  LBM_ESTATE = -5,        /* call not valid in the context's current state */
  LBM_ENONFINITE = -6     /* a reduction found NaN or Inf                  */
};

/* Relaxation rates (Sec. III-A "Relaxation rates"; runtime constants). */
typedef struct {
  double omega;       /* SRT omega = 1/tau; TRT even rate; MRT/cumulant/KBC shear rate */
  double omega_bulk;  /* MRT/cumulant/KBC bulk rate (trace of the 2nd-order moments) */
  double omega_odd;   /* TRT odd rate; if <= 0 it is derived from `magic`          */
  double magic;       /* TRT Lambda = (1/omega_even - 1/2)(1/omega_odd - 1/2)      */
  double omega_hi[4]; /* MRT/cumulant rates of moment orders 3, 4, 5, 6            */
  double cs_smag;     /* Smagorinsky constant C_S (Sec. III-C "Turbulence models");
                         > 0 makes the SRT rate / MRT shear rate local:
                         omega = 2 / (tau0 + sqrt(tau0^2 + 18 C_S^2 P / rho)),
                         P = sqrt(2 Pi^neq : Pi^neq), tau0 = 1 / omega.  0 = off  */
} lbm_rates;

typedef struct {
  lbm_stencil stencil;      /* LBM_D2Q9 | LBM_D3Q19 | LBM_D3Q27                    */
  lbm_method method;        /* LBM_SRT | LBM_TRT | LBM_MRT | LBM_CUMULANT | LBM_KBC */
  lbm_dtype dtype;          /* PDF storage type                                     */
  int32_t nx, ny, nz;       /* lattice size; nz == 1 for D2Q9; N < 2^31            */
  lbm_rates rates;          /* every used rate must lie in (0, 2)                   */
  double rho0;              /* reference density: storage shift and Eq. (3) rho_0  */
  int32_t compressible;     /* 1: rho_0 = rho in Eq. (3) (default); 0: incompressible */
  int32_t pattern;          /* 0: two arrays, stream-pull-collide (Sec. IV-B);
                               1: AA pattern in one array (Sec. IV-B, Fig. "AA update
                               pattern"): half the memory; with a tape the adjoint
                               state is one array as well                           */
  int32_t checkpoint_every; /* k > 0 enables the adjoint tape (PDF copy every k steps) */
  int32_t max_tape_steps;   /* longest forward run the tape covers (adjoint only)   */
  int32_t launch_mode;      /* 0: automatic -- lattices of at most 64 MiB per grid without a
                               tape replay a captured HIP graph of 32 sweeps (launch latency
                               dominates there); 1: one direct launch per step      */
} lbm_config;

/* Supported combinations: SRT, TRT, MRT on all stencils (MRT rates: orders
 * 3..6 on D3Q27, orders 3 and 4 on D2Q9 and D3Q19; when all of them are 1 on
 * D2Q9 / D3Q27 with FP32 or 16-bit storage, a kernel that rebuilds the
 * post-collision populations from their moments of order <= 2 runs instead,
 * the same operator of Eq. (4));
 * CUMULANT on D2Q9 and D3Q27, compressible and without body force (higher-order
 * rates all 1 use a Gaussian-reconstruction kernel, other rates a general FP64
 * cumulant kernel); KBC on all stencils (shear and bulk rates fixed, one
 * entropic rate per cell for orders >= 3:
 *   omega_h = 1 + [(1 - omega) <ds, dh>_E + (1 - omega_bulk) <db, dh>_E] / <dh, dh>_E,
 *   <a, b>_E = sum_q a_q b_q / f^eq_q, ds / db / dh the shear, bulk and
 *   higher-order parts of f - f^eq; omega_h = 1 when dh = 0);
 * both patterns for every method; the adjoint tape for compressible SRT, TRT
 * and MRT with either pattern.  Others return LBM_EUNSUPPORTED. */

/* Create a context: validates cfg, allocates two PDF grids (plus the tape when
 * checkpoint_every > 0) and copies the solid mask in.
 * solid_mask_host: N bytes on the host: 0 = fluid, 1 = resting wall,
 *   2..127 = moving-wall types (see lbm_set_wall_velocity), or NULL (all fluid,
 *   fully periodic); larger values are LBM_EINVAL.  Solid cells are never
 *   updated and read out as rho = u = 0.
 * hip_stream: a hipStream_t of the current device, or NULL.
 * On success *out owns all allocations; release with lbm_destroy.
 * The PDFs are initialised to rest at rho0 (shifted zero). */
lbm_status lbm_create(const lbm_config* cfg, const uint8_t* solid_mask_host,
                   void* hip_stream, lbm_ctx** out);

/* Free everything the context owns (synchronises its stream). NULL is a no-op. */
lbm_status lbm_destroy(lbm_ctx* ctx);

/* Body force (Guo scheme).  F: 3 host doubles, a force constant in space; or
 * F == NULL and profile_y = ny*3 host doubles, force (Fx, Fy, Fz) of row y at
 * [3*y + a] (uniform in x and z).  Invalidates a recorded tape. */
lbm_status lbm_set_force(lbm_ctx* ctx, const double* F, const double* profile_y);

/* Velocity of the moving-wall type `wall_type` (2..127): solid cells whose mask
 * value is wall_type act as a wall moving with u (3 host doubles).  A
 * population re-entering along link q from such a wall is the cell's own
 * outgoing opposite population plus 2 w_q rho0 (c_q . u) / c_s^2 (velocity
 * bounce-back, Sec. III-C "Boundary Conditions").  Mask value 1 is the resting
 * wall; all types start at rest.  With pattern 1 call it before
 * lbm_init_equilibrium / lbm_set_pdfs.  Invalidates a recorded tape. */
lbm_status lbm_set_wall_velocity(lbm_ctx* ctx, int32_t wall_type, const double* u);

/* P = f^eq(rho, u) (Eq. 3) at fluid cells; resets the step counter and tape.
 * rho_dev: N values or NULL (rho0 everywhere); u_dev: 3*N values or NULL
 * (at rest); both of type field_dtype (LBM_F64 or LBM_F32). */
lbm_status lbm_init_equilibrium(lbm_ctx* ctx, const void* rho_dev, const void* u_dev,
                             lbm_dtype field_dtype);

/* Advance n >= 0 time steps.  One step is the pull streaming of Sec. IV-B
 * (Fig. "stream-pull-collide": each cell gathers population q from its
 * upstream neighbour x - c_q, with the bounce-back rule at solid neighbours)
 * fused with the collision of the configured method, one launch per step;
 * with pattern 1 the AA even and odd kernels of Sec. IV-B alternate on one
 * array (Fig. "AA update pattern").  With launch_mode 0
 * small lattices replay a captured graph of 32 launches).  With the tape
 * enabled, the state at every multiple of k steps below max_tape_steps is
 * kept in the tape, in the two-array layout (the sweep that produces it
 * writes it there directly), and so are the states of the last k-step
 * segment below max_tape_steps, which an adjoint started in or at the end of
 * that segment then need not recompute. */
lbm_status lbm_step(lbm_ctx* ctx, int32_t n);

/* Readout of the stored (post-collision) state by Eq. (2): rho = sum f,
 * u = (sum c f - F/2) / rho_0 (rho_0 = rho when compressible; the F/2 term
 * makes u the Guo velocity of the collision that produced the state).
 * rho_dev: N or NULL, u_dev: 3*N or NULL, of type field_dtype. */
lbm_status lbm_get_macroscopic(lbm_ctx* ctx, void* rho_dev, void* u_dev, lbm_dtype field_dtype);

/* FP64 totals over fluid cells of the moments of Eq. (2): out[0] = sum of
 * rho = sum_q f_q, out[1..3] = sum of the momentum sum_q c_q f_q (without
 * the F/2 shift).  Synchronises.  LBM_ENONFINITE if any total is NaN/Inf
 * (out is still written). */
lbm_status lbm_conserved(lbm_ctx* ctx, double out[4]);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the totals
 * of lbm_conserved, written to totals_dev (4 doubles of device memory that
 * the caller owns) on the context's stream, with no allocation, no host copy
 * and no synchronisation; the caller checks them for NaN / Inf.  The partial
 * sums go to a static device scratch of 4096 rows of 4 doubles (128 KiB,
 * one per GPU, held until the process ends) shared by every call on that
 * GPU: any lattice fits (its row segments are reduced in strides over at
 * most 4096 blocks), nothing in it needs clearing, and calls on one GPU that
 * overlap in time (on other streams or threads) race on it.
 * LBM_EINVAL for NULL arguments. */
lbm_status lbm_conserved_noalloc(lbm_ctx* ctx, double* totals_dev);

/* Copy the state out / in as unshifted FP64 PDFs, layout [q*N + i] in the
 * documented direction order.  lbm_set_pdfs rounds into the storage type and
 * resets the step counter; on a context with a tape (checkpoint_every > 0) it
 * returns LBM_ESTATE, since the adjoint needs the initial fields rho, u that
 * lbm_init_equilibrium takes.  lbm_get_pdfs synchronises. */
lbm_status lbm_get_pdfs(lbm_ctx* ctx, double* pdfs_dev);
lbm_status lbm_set_pdfs(lbm_ctx* ctx, const double* pdfs_dev);

/* Number of steps taken since the last init / set_pdfs. */
lbm_status lbm_get_time(lbm_ctx* ctx, int64_t* t);

/* ---- discrete adjoint (SRT, TRT and MRT, compressible) ------------------
 * Forward map: P^0 = f^eq(rho_init, u_init) from lbm_init_equilibrium,
 * P^{t+1} = collide(pull-gather(P^t)), readout as lbm_get_macroscopic.
 * The adjoint state lambda^t = dL/dP^t runs backwards through the transposed
 * collision Jacobian and the transposed gather (reverse streaming).  With
 * pattern 1 the tape stores each checkpoint in the two-array layout and
 * lambda lives in one array, updated in place by the transposes of the AA
 * kernels; the gradients equal those of pattern 0.
 *
 * Seed lambda^T from dL/drho and dL/du at the current step T (fields of type
 * field_dtype, dL_drho_dev may be NULL).  Needs checkpoint_every > 0 and
 * T <= max_tape_steps, else LBM_ESTATE. */
lbm_status lbm_adjoint_seed(lbm_ctx* ctx, const void* dL_drho_dev, const void* dL_du_dev,
                         lbm_dtype field_dtype);
/* Run n adjoint steps backwards (n <= steps remaining, else LBM_ESTATE);
 * recomputes the forward states of each k-step segment from the tape. */
lbm_status lbm_adjoint_step(lbm_ctx* ctx, int32_t n);
/* Once the adjoint has reached t = 0: dL/du_init (3*N), dL/drho_init (N,
 * or NULL) of type field_dtype, and dL/dF (3 host doubles, accumulated in
 * FP64, or NULL).  Synchronises when dL_dF != NULL. */
lbm_status lbm_adjoint_grads(lbm_ctx* ctx, void* dL_du0_dev, void* dL_drho0_dev,
                          lbm_dtype field_dtype, double* dL_dF);

/* Bandwidth reference: copy Q planes of n elements of elem_bytes (2, 4 or 8)
 * from src to dst with the sweep's thread layout (one thread per cell, Q
 * loads and Q stores, non-temporal stores once the arrays exceed 512 MiB as
 * in the sweep).  The analogue of the paper's multi-stream copy benchmark
 * (Sec. V-A, Tab. III).  waves_per_cu: 0 = full occupancy, k > 0 = at most k
 * wavefronts per CU (the launch shape of a sweep that runs so; values the
 * LDS split cannot express fall back to full occupancy), < 0 or > 32 is
 * LBM_EINVAL.  block_threads: threads per block, 0 = 256, else a multiple of
 * 64 in 64..512 (a sweep's row-segment length), otherwise LBM_EINVAL.
 * hip_stream as in lbm_create. */
lbm_status lbm_copy_q(const void* src_dev, void* dst_dev, int64_t n, int32_t q,
                   int32_t elem_bytes, int32_t waves_per_cu, int32_t block_threads, void* hip_stream);

/* Bandwidth reference for the pull access pattern: periodic pull streaming
 * of the stencil's Q planes with no collision and no walls,
 * dst[q][x] = src[q][x - c_q] (the streaming half of Eq. (1), Sec. IV-B), in
 * the sweep's launch shape: one block per x-row segment of block_threads
 * cells (0 = the sweep's own segmentation, rows of up to 512 cells), the
 * sweep's addressing, and non-temporal stores once the Q planes exceed
 * 512 MiB.  src_dev and dst_dev hold Q planes of nx*ny*nz elements of
 * elem_bytes (2, 4 or 8; layout [q][z][y][x]) and must not overlap.  Its
 * rate is what the sweep's loads and stores reach without arithmetic.
 * waves_per_cu as in lbm_copy_q.  Errors (LBM_EINVAL, before any device
 * work): NULL buffer, unknown stencil, dims < 1 or nx*ny*nz >= 2^31, nz != 1
 * with D2Q9, elem_bytes, waves_per_cu or block_threads out of range.
 * hip_stream as in lbm_create. */
lbm_status lbm_stream_q(const void* src_dev, void* dst_dev, int32_t nx, int32_t ny, int32_t nz,
                     lbm_stencil stencil, int32_t elem_bytes, int32_t waves_per_cu,
                     int32_t block_threads, void* hip_stream);

/* Bandwidth reference for the AA pattern (Sec. IV-B, Fig. "AA update
 * pattern"): the data movement of its two in-place kernels with no
 * collision and no walls, on one buffer buf_dev of Q planes of nx*ny*nz
 * elements (layout [q][z][y][x]).  phase 0 (even): every cell writes its own
 * slots back inverted, A[opp q][x] = A[q][x]; phase 1 (odd): every cell reads
 * A[opp q][x - c_q] and writes it to A[q][x + c_q] (periodic), i.e. plane q
 * becomes plane opp(q) shifted by 2 c_q.  Launch shape, addressing, block
 * order and store type are those of the AA sweep; waves_per_cu and
 * block_threads as in lbm_stream_q.  Errors (LBM_EINVAL, before any device
 * work): as lbm_stream_q, and phase other than 0 or 1.  hip_stream as in
 * lbm_create. */
lbm_status lbm_stream_aa_q(void* buf_dev, int32_t nx, int32_t ny, int32_t nz, lbm_stencil stencil,
                        int32_t elem_bytes, int32_t phase, int32_t waves_per_cu, int32_t block_threads,
                        void* hip_stream);

/* Thread-local description of the last error. */
const char* lbm_last_error(void);

/* Library version (major*10000 + minor*100 + patch). */
int32_t lbm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LBM_MI355X_H */
