// Host runtime behind the C ABI of include/lbm.h: argument validation,
// device buffers, the step loop, the checkpoint tape and the adjoint driver.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/lbm.h"
#include "internal.h"

using namespace lbm;

namespace {

thread_local std::string g_last_error;

int32_t fail(int32_t code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

}  // namespace

int32_t lbm::set_last_error(int32_t code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

namespace {

int32_t hip_fail(hipError_t e, const char* what) {
  return fail(LBM_EHIP, "%s: %s", what, hipGetErrorString(e));
}

int q_of(int stencil) { return stencil == LBM_D2Q9 ? 9 : (stencil == LBM_D3Q19 ? 19 : 27); }
size_t storage_bytes(int dtype) { return dtype == LBM_F64 ? 8 : (dtype == LBM_F32 ? 4 : 2); }
size_t compute_bytes(int dtype) { return dtype == LBM_F64 ? 8 : 4; }
bool rate_ok(double w) { return std::isfinite(w) && w > 0.0 && w < 2.0; }

}  // namespace

struct lbm_ctx {
  lbm_config cfg{};
  int Q = 0;
  int kmethod = 0;  // kernel method code: the ABI method, or its Smagorinsky variant
  Geo g{};
  Params p{};
  hipStream_t stream = nullptr;
  int device = 0;              // device current at creation (its stream's device)
  size_t grid_bytes = 0;
  void* grid[2] = {nullptr, nullptr};
  // Buffer holding the current state: grid[0] with AA; with two arrays one
  // of the grids, or a tape slot while a tape is recorded.  Solid cells keep
  // their values in the grids only (the sweep never writes them).
  void* state = nullptr;
  uint8_t* flags = nullptr;
  uint32_t* links = nullptr;   // bounced-link bits per cell (with a mask)
  int has_mask = 0;
  void* force = nullptr;       // compute type, 3 * ny
  void* wall = nullptr;        // compute type, [128][3] wall velocities by wall type
  double* partials = nullptr;  // 4 doubles per block
  double* acc = nullptr;       // [0..2] adjoint dL/dF, [4..7] conservation totals
  double* adj_acc = nullptr;   // 3 doubles per block: dL/dF accumulated over adjoint steps
  int64_t t = 0;
  // tape
  int k = 0;
  int nslots = 0;
  void* tape = nullptr;        // nslots grids: P^0, P^k, ...
  void* seg = nullptr;         // k - 1 grids: recomputed states of one segment
  int64_t seg_id = -1;
  int64_t seg_fwd_lo = INT64_MAX;  // the forward wrote the last segment's states from this time on
  int64_t taped_t = -1;        // AA: time of the last state written to the tape by its sweep
  bool tape_ok = false;
  void* init_fields = nullptr; // compute type: rho, ux, uy, uz
  void* lam = nullptr;         // compute type, Q * N: lambda in the AA layout of its time
  int64_t adj_t = -1;
  int64_t adj_T = -1;
  // graph replay for small lattices: one executable graph per starting grid
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t graph_exec[2] = {nullptr, nullptr};
};

namespace {

constexpr int kGraphSteps = 32;                 // even: the current grid is unchanged after a replay
constexpr size_t kGraphMaxGridBytes = size_t(64) << 20;

void free_ctx(lbm_ctx* c) {
  for (auto& ge : c->graph_exec)
    if (ge) (void)hipGraphExecDestroy(ge);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  void* bufs[] = {c->grid[0], c->grid[1], c->flags, c->links, c->force,       c->wall,   c->partials, c->acc,
                  c->adj_acc, c->tape,    c->seg,   c->init_fields, c->lam};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  delete c;
}

// Kernel method code (collide.h): the ABI method, its Smagorinsky variant,
// the general-rate cumulant kernel, or KBC.
int kernel_method(const lbm_config* cfg) {
  if (cfg->rates.cs_smag > 0) return cfg->method == LBM_SRT ? 4 : 5;
  if (cfg->method == LBM_KBC) return 7;
  const int nhi = cfg->stencil == LBM_D2Q9 ? 2 : 4;   // orders 3..4 (D2Q9) or 3..6 (D3Q27) exist
  bool unit_hi = true;
  for (int i = 0; i < nhi; ++i) unit_hi = unit_hi && cfg->rates.omega_hi[i] == 1.0;
  // unit higher-order rates: the Gaussian-reconstruction cumulant kernel, and
  // on the tensor-product stencils with FP32 or 16-bit storage the MRT kernel
  // that rebuilds f* from orders <= 2 (512^3 D3Q27 FP16: 2.779 -> 2.749 ms per
  // step; FP64, which is far from its VALU limit, measured 1.2 % slower with
  // it, so FP64 keeps the general kernel)
  if (cfg->method == LBM_CUMULANT) return unit_hi ? 3 : 6;
  if (cfg->method == LBM_MRT && cfg->stencil != LBM_D3Q19 && unit_hi && cfg->dtype != LBM_F64) return 8;
  return cfg->method;
}

int32_t validate(const lbm_config* cfg) {
  if (!cfg) return fail(LBM_EINVAL, "cfg is NULL");
  if (cfg->stencil < 0 || cfg->stencil > 2) return fail(LBM_EINVAL, "unknown stencil %d", cfg->stencil);
  if (cfg->method < 0 || cfg->method > 4) return fail(LBM_EINVAL, "unknown method %d", cfg->method);
  if (cfg->dtype < 0 || cfg->dtype > 3) return fail(LBM_EINVAL, "unknown dtype %d", cfg->dtype);
  if (cfg->nx < 1 || cfg->ny < 1 || cfg->nz < 1)
    return fail(LBM_EINVAL, "lattice dims must be >= 1 (got %d x %d x %d)", cfg->nx, cfg->ny, cfg->nz);
  const int64_t N = (int64_t)cfg->nx * cfg->ny * cfg->nz;
  if (N >= (int64_t(1) << 31)) return fail(LBM_EINVAL, "lattice has %lld cells; the limit is 2^31 - 1", (long long)N);
  if (cfg->stencil == LBM_D2Q9 && cfg->nz != 1) return fail(LBM_EINVAL, "D2Q9 needs nz == 1");
  if (!(std::isfinite(cfg->rho0) && cfg->rho0 > 0)) return fail(LBM_EINVAL, "rho0 must be positive");
  if (cfg->compressible != 0 && cfg->compressible != 1) return fail(LBM_EINVAL, "compressible must be 0 or 1");
  const lbm_rates& r = cfg->rates;
  if (!rate_ok(r.omega)) return fail(LBM_EINVAL, "omega = %g is outside (0, 2)", r.omega);
  if (cfg->method == LBM_TRT) {
    if (r.omega_odd <= 0) {
      if (!(std::isfinite(r.magic) && r.magic > 0)) return fail(LBM_EINVAL, "TRT needs omega_odd > 0 or magic > 0");
      const double wo = 1.0 / (r.magic / (1.0 / r.omega - 0.5) + 0.5);
      if (!rate_ok(wo)) return fail(LBM_EINVAL, "TRT odd rate from magic = %g is outside (0, 2)", wo);
    } else if (!rate_ok(r.omega_odd)) {
      return fail(LBM_EINVAL, "omega_odd = %g is outside (0, 2)", r.omega_odd);
    }
  }
  if (cfg->method == LBM_KBC && !rate_ok(r.omega_bulk))
    return fail(LBM_EINVAL, "omega_bulk = %g is outside (0, 2)", r.omega_bulk);
  if (cfg->method == LBM_MRT || cfg->method == LBM_CUMULANT) {
    if (!rate_ok(r.omega_bulk)) return fail(LBM_EINVAL, "omega_bulk = %g is outside (0, 2)", r.omega_bulk);
    const int nhi = cfg->stencil == LBM_D3Q27 ? 4 : 2;   // highest moment order 2 DIM, or 4 on D3Q19
    for (int i = 0; i < nhi; ++i)
      if (!rate_ok(r.omega_hi[i])) return fail(LBM_EINVAL, "omega_hi[%d] = %g is outside (0, 2)", i, r.omega_hi[i]);
  }
  if (!(std::isfinite(r.cs_smag) && r.cs_smag >= 0)) return fail(LBM_EINVAL, "cs_smag must be >= 0");
  if (r.cs_smag > 0 && cfg->method != LBM_SRT && cfg->method != LBM_MRT)
    return fail(LBM_EUNSUPPORTED, "the Smagorinsky model is implemented for SRT and MRT");
  if (r.cs_smag > 0 && cfg->checkpoint_every > 0)
    return fail(LBM_EUNSUPPORTED, "the adjoint of the Smagorinsky model is not implemented");
  if (cfg->pattern != 0 && cfg->pattern != 1) return fail(LBM_EINVAL, "pattern must be 0 (two arrays) or 1 (AA)");
  if (!sweep_supported(cfg->stencil, kernel_method(cfg)))
    return fail(LBM_EUNSUPPORTED, "method %d is not implemented on stencil %d", cfg->method, cfg->stencil);
  if (cfg->method == LBM_CUMULANT && !cfg->compressible)
    return fail(LBM_EUNSUPPORTED, "the cumulant operator is compressible only");
  if (cfg->launch_mode != 0 && cfg->launch_mode != 1) return fail(LBM_EINVAL, "launch_mode must be 0 or 1");
  if (cfg->checkpoint_every < 0) return fail(LBM_EINVAL, "checkpoint_every must be >= 0");
  if (cfg->checkpoint_every > 0) {
    if (cfg->max_tape_steps < 1) return fail(LBM_EINVAL, "max_tape_steps must be >= 1 with a tape");
    if (!adjoint_supported(cfg->stencil, cfg->method) || !cfg->compressible)
      return fail(LBM_EUNSUPPORTED, "the adjoint is implemented for the compressible SRT, TRT and MRT methods only");
  }
  return LBM_OK;
}

Geo make_geo(const lbm_config& c) {
  Geo g{};
  g.nx = c.nx;
  g.ny = c.ny;
  g.nz = c.nz;
  g.nxb = (c.nx + 511) / 512;
  // The 16-bit D3Q27 cumulant kernel is close to its VALU limit and needs
  // full occupancy: when the row's block would hold a number of wavefronts
  // that does not divide the 32 a CU can hold (384 cells: 6), use 128-cell
  // segments (2 wavefronts) instead (384^3: +1.2 %; the FP32 / FP64 cumulant
  // measured slower split)
  const bool half = c.dtype == LBM_BF16 || c.dtype == LBM_F16;
  if (half && c.method == LBM_CUMULANT && c.stencil == LBM_D3Q27 && g.nxb == 1 && c.nx % 128 == 0 &&
      32 % (c.nx / 64) != 0)
    g.nxb = c.nx / 128;
  // The FP64 MRT kernels on D3Q27 (with or without the Smagorinsky model)
  // need 135-150 VGPRs per lane, so a SIMD holds 3 of their wavefronts (12
  // per CU): a 512-cell row block (8 wavefronts) leaves a third of them
  // empty, 256-cell segments fill all 12 (512^3: 11.24 -> 11.01 ms per step,
  // alternating processes)
  if (c.dtype == LBM_F64 && c.stencil == LBM_D3Q27 && c.method == LBM_MRT && g.nxb == 1 && c.nx > 256)
    g.nxb = (c.nx + 255) / 256;
  const int per = (c.nx + g.nxb - 1) / g.nxb;
  g.bx = ((per + 63) / 64) * 64;
  g.N = (int64_t)c.nx * c.ny * c.nz;
  return g;
}

Params make_params(const lbm_config& c) {
  Params p{};
  p.rho0 = c.rho0;
  p.om = c.rates.omega;
  p.om_b = c.rates.omega_bulk;
  p.om_o = c.rates.omega_odd > 0 ? c.rates.omega_odd
                                  : 1.0 / (c.rates.magic / (1.0 / c.rates.omega - 0.5) + 0.5);
  for (int i = 0; i < 4; ++i) p.hi[i] = c.rates.omega_hi[i];
  p.smag18 = 18.0 * c.rates.cs_smag * c.rates.cs_smag;
  p.compressible = c.compressible;
  return p;
}

#define HIP_TRY(expr, what)                 \
  do {                                      \
    hipError_t e_ = (expr);                 \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

int32_t alloc(void** p, size_t bytes, const char* what) {
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return fail(LBM_ENOMEM, "hipMalloc of %zu bytes for %s failed: %s", bytes, what, hipGetErrorString(e));
  }
  return LBM_OK;
}

bool is_aa(const lbm_ctx* c) { return c->cfg.pattern == 1; }

// Geometry of the sweep (or adjoint sweep) of time step t.  Grids within
// reach of the caches use the XCD-slab block order and alternate the
// traversal direction every step.  Larger grids keep the plain order (the
// slabs and the reversal measured slower there), except the forward AA
// kernels (aa_forward), which update one array in place: alternating the
// direction makes each step start on the rows the previous step wrote last
// (measured 2-4 % faster on 256^3).
Geo sweep_geo(const lbm_ctx* c, int64_t t, bool aa_forward = false) {
  Geo g = c->g;
  if (c->grid_bytes <= kStreamGridBytes)
    g.order = (num_blocks(g) % 8 == 0 ? 2 : 0) | (int)(t & 1);
  else if (aa_forward)
    g.order = (int)(t & 1);
  return g;
}

char* tape_slot(const lbm_ctx* c, int64_t j) { return (char*)c->tape + (size_t)j * c->grid_bytes; }
char* seg_slot(const lbm_ctx* c, int64_t i) { return (char*)c->seg + (size_t)i * c->grid_bytes; }
bool in_seg(const lbm_ctx* c, const void* p) {
  return c->seg && p >= c->seg && (const char*)p < seg_slot(c, c->k - 1);
}

// Tape slot of a checkpoint, or the segment slot of a state of the last
// segment below max_tape_steps, for the state of time s; else nullptr.  The
// forward keeps the last segment's states in the segment buffer, so an
// adjoint started at max_tape_steps (or inside that segment) skips its
// recompute.  (Keeping every segment there made the forward slower, 29 cold
// destination buffers instead of two grids, by as much as the backward
// gained; for the last segment alone it costs a fraction of the recompute.)
void* tape_place(const lbm_ctx* c, int64_t s) {
  if (c->k <= 0 || s >= c->cfg.max_tape_steps) return nullptr;
  const int64_t j = s / c->k, r = s % c->k;
  if (r == 0) return j < c->nslots ? tape_slot(c, j) : nullptr;
  const int64_t last = (c->cfg.max_tape_steps - 1) / c->k;
  return (j == last && c->seg && r - 1 < c->k - 1) ? seg_slot(c, r - 1) : nullptr;
}

// Where the two-array sweep stores the state of time s: its tape or segment
// slot (no copy), else the grid that does not hold the source.
void* place(const lbm_ctx* c, int64_t s, const void* src) {
  if (void* p = tape_place(c, s)) return p;
  return src == c->grid[0] ? c->grid[1] : c->grid[0];
}

// Two-array sweep src -> dst of time step t.
int32_t sweep_once(lbm_ctx* c, const void* src, void* dst, int64_t t) {
  HIP_TRY(launch_sweep(c->cfg.stencil, c->kmethod, c->cfg.dtype, -1, src, dst, c->flags, c->force,
                       sweep_geo(c, t), c->p, c->has_mask, c->stream),
          "sweep launch");
  return LBM_OK;
}


// Layout of the stored state (see aux.hip): two arrays 0; AA 2 after an even
// number of steps (streamed), 1 after an odd number (inverted).
int layout_of(const lbm_ctx* c) { return is_aa(c) ? ((c->t & 1) ? 1 : 2) : 0; }

// One forward step on the context's stream.
int32_t step_once(lbm_ctx* c) {
  if (is_aa(c)) {
    // the sweep that produces a checkpoint (or a state of the last segment)
    // also writes it, in the two-array layout, into its tape (segment) slot
    const int64_t s = c->t + 1;
    void* tape = tape_place(c, s);
    HIP_TRY(launch_sweep(c->cfg.stencil, c->kmethod, c->cfg.dtype, (int)(c->t & 1), c->grid[0], tape, c->flags,
                         c->force, sweep_geo(c, c->t, true), c->p, c->has_mask, c->stream),
            "AA sweep launch");
    if (tape && !in_seg(c, tape)) c->taped_t = s;
    if (tape && in_seg(c, tape) && s % c->k == 1) c->seg_fwd_lo = s;
  } else {
    void* dst = place(c, c->t + 1, c->state);
    if (!dst || dst == c->state) return fail(LBM_EHIP, "internal: no buffer for the state of step %lld",
                                             (long long)(c->t + 1));
    int32_t st = sweep_once(c, c->state, dst, c->t);
    if (st != LBM_OK) return st;
    if (in_seg(c, dst) && (c->t + 1) % c->k == 1) c->seg_fwd_lo = c->t + 1;
    c->state = dst;
  }
  c->t += 1;
  return LBM_OK;
}

bool graph_replay(const lbm_ctx* c) {
  return c->cfg.launch_mode == 0 && c->k == 0 && c->grid_bytes <= kGraphMaxGridBytes;
}

// Capture kGraphSteps sweeps starting from grid `parity` on a private stream
// (capture is not possible on the legacy null stream); the executable graph
// is then launched on the context's stream.  Kernels only: no memset nodes.
int32_t ensure_graph(lbm_ctx* c, int parity) {
  if (c->graph_exec[parity]) return LBM_OK;
  if (!c->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking), "capture stream");
  HIP_TRY(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal), "begin capture");
  int cur = parity;
  hipError_t e = hipSuccess;
  for (int i = 0; i < kGraphSteps && e == hipSuccess; ++i) {
    if (is_aa(c))   // parity = time parity: even / odd kernels alternate on one array
      e = launch_sweep(c->cfg.stencil, c->kmethod, c->cfg.dtype, cur, c->grid[0], nullptr, c->flags, c->force,
                       sweep_geo(c, cur, true), c->p, c->has_mask, c->cap_stream);
    else            // parity = current grid
      e = launch_sweep(c->cfg.stencil, c->kmethod, c->cfg.dtype, -1, c->grid[cur], c->grid[cur ^ 1], c->flags,
                       c->force, sweep_geo(c, i), c->p, c->has_mask, c->cap_stream);
    cur ^= 1;
  }
  hipGraph_t graph = nullptr;
  hipError_t e2 = hipStreamEndCapture(c->cap_stream, &graph);
  if (e != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return hip_fail(e, "captured sweep launch");
  }
  if (e2 != hipSuccess) return hip_fail(e2, "end capture");
  e = hipGraphInstantiate(&c->graph_exec[parity], graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) {
    c->graph_exec[parity] = nullptr;
    return hip_fail(e, "graph instantiate");
  }
  return LBM_OK;
}

// Both grids must hold the same values at solid cells: the sweep never
// writes them, and lbm_get_pdfs reports them from whichever grid is current.
int32_t mirror_grid(lbm_ctx* c) {
  if (is_aa(c)) return LBM_OK;
  HIP_TRY(hipMemcpyAsync(c->grid[1], c->grid[0], c->grid_bytes, hipMemcpyDeviceToDevice, c->stream), "grid mirror");
  return LBM_OK;
}

void reset_time(lbm_ctx* c) {
  c->t = 0;
  c->seg_id = -1;
  c->seg_fwd_lo = INT64_MAX;
  c->taped_t = -1;
  c->tape_ok = c->k > 0;
  c->adj_t = -1;
  c->adj_T = -1;
}

int32_t check_field_dtype(int32_t fdt) {
  if (fdt != LBM_F64 && fdt != LBM_F32) return fail(LBM_EINVAL, "field_dtype must be LBM_F64 or LBM_F32");
  return LBM_OK;
}

}  // namespace

extern "C" {

int32_t lbm_version(void) { return 10000; }

const char* lbm_last_error(void) { return g_last_error.c_str(); }

int32_t lbm_create(const lbm_config* cfg, const uint8_t* solid_mask_host, void* hip_stream, lbm_ctx** out) {
  if (!out) return fail(LBM_EINVAL, "out is NULL");
  *out = nullptr;
  int32_t st = validate(cfg);
  if (st != LBM_OK) return st;
  int moving = 0;
  if (solid_mask_host) {
    const size_t n = (size_t)cfg->nx * cfg->ny * cfg->nz;
    for (size_t i = 0; i < n; ++i) {
      if (solid_mask_host[i] > 127)
        return fail(LBM_EINVAL, "mask value %d at cell %zu: wall types are 1..127", solid_mask_host[i], i);
      moving |= solid_mask_host[i] >= 2;
    }
  }
  lbm_ctx* c = new lbm_ctx();
  c->cfg = *cfg;
  c->Q = q_of(cfg->stencil);
  c->kmethod = kernel_method(cfg);
  c->g = make_geo(*cfg);
  c->p = make_params(*cfg);
  c->p.moving = moving;
  c->stream = (hipStream_t)hip_stream;
  {
    hipError_t e0 = hipGetDevice(&c->device);
    if (e0 == hipSuccess) e0 = noalloc_scratch_setup(c->device);
    if (e0 != hipSuccess) {
      delete c;
      return hip_fail(e0, "device scratch lookup");
    }
  }
  const size_t N = (size_t)c->g.N;
  c->grid_bytes = (size_t)c->Q * N * storage_bytes(cfg->dtype);
  const size_t rb = compute_bytes(cfg->dtype);
  const int64_t nblk = num_blocks(c->g);
  auto bail = [&](int32_t s) {
    free_ctx(c);
    return s;
  };
  for (int i = 0; i < (cfg->pattern == 1 ? 1 : 2); ++i)
    if ((st = alloc(&c->grid[i], c->grid_bytes, "PDF grid")) != LBM_OK) return bail(st);
  c->state = c->grid[0];
  if ((st = alloc(&c->force, 3 * (size_t)cfg->ny * rb, "force table")) != LBM_OK) return bail(st);
  if ((st = alloc(&c->wall, 3 * 128 * rb, "wall velocity table")) != LBM_OK) return bail(st);
  c->p.wall = c->wall;
  if ((st = alloc((void**)&c->partials, (size_t)nblk * 4 * sizeof(double), "reduction partials")) != LBM_OK)
    return bail(st);
  if ((st = alloc((void**)&c->acc, 8 * sizeof(double), "accumulators")) != LBM_OK) return bail(st);
  if (cfg->checkpoint_every > 0) {
    c->k = cfg->checkpoint_every;
    c->nslots = (cfg->max_tape_steps - 1) / c->k + 1;
    if ((st = alloc(&c->tape, c->grid_bytes * (size_t)c->nslots, "checkpoint tape")) != LBM_OK) return bail(st);
    if (c->k > 1 && (st = alloc(&c->seg, c->grid_bytes * (size_t)(c->k - 1), "segment buffer")) != LBM_OK)
      return bail(st);
    if ((st = alloc(&c->init_fields, 4 * N * rb, "initial fields")) != LBM_OK) return bail(st);
    if ((st = alloc((void**)&c->adj_acc, (size_t)nblk * 3 * sizeof(double), "dL/dF accumulators")) != LBM_OK)
      return bail(st);
    // one lambda array, updated in place by the transposed AA kernels
    if ((st = alloc(&c->lam, (size_t)c->Q * N * rb, "adjoint state")) != LBM_OK) return bail(st);
  }
  hipError_t e;
  if ((e = launch_fill_zero(c->force, 3 * (size_t)cfg->ny * rb, c->stream)) != hipSuccess)
    return bail(hip_fail(e, "force table init"));
  if ((e = launch_fill_zero(c->wall, 3 * 128 * rb, c->stream)) != hipSuccess)
    return bail(hip_fail(e, "wall table init"));
  if ((e = launch_fill_zero(c->acc, 8 * sizeof(double), c->stream)) != hipSuccess)
    return bail(hip_fail(e, "accumulator init"));
  if (solid_mask_host) {
    c->has_mask = 1;
    if ((st = alloc((void**)&c->flags, N, "flag field")) != LBM_OK) return bail(st);
    if ((st = alloc((void**)&c->links, N * sizeof(uint32_t), "bounced-link bits")) != LBM_OK) return bail(st);
    c->p.links = c->links;
    uint8_t* solid_dev = nullptr;
    if ((st = alloc((void**)&solid_dev, N, "solid mask staging")) != LBM_OK) return bail(st);
    e = hipMemcpy(solid_dev, solid_mask_host, N, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = launch_build_flags(cfg->stencil, solid_dev, c->flags, c->links, c->g, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    (void)hipFree(solid_dev);
    if (e != hipSuccess) return bail(hip_fail(e, "solid mask upload"));
  }
  if ((e = launch_init(cfg->stencil, cfg->dtype, c->grid[0], c->flags, c->has_mask, cfg->pattern == 1 ? 2 : 0,
                       nullptr, nullptr, LBM_F64, c->g, c->p, c->stream)) != hipSuccess)
    return bail(hip_fail(e, "initial state"));
  if ((st = mirror_grid(c)) != LBM_OK) return bail(st);
  reset_time(c);
  if (c->k > 0) {
    e = launch_store_init_fields(cfg->dtype, nullptr, nullptr, LBM_F64, c->init_fields, c->g, c->p, c->stream);
    if (e != hipSuccess) return bail(hip_fail(e, "initial fields"));
  }
  *out = c;
  return LBM_OK;
}

int32_t lbm_destroy(lbm_ctx* ctx) {
  if (!ctx) return LBM_OK;
  hipError_t e = hipStreamSynchronize(ctx->stream);
  free_ctx(ctx);
  if (e != hipSuccess) return hip_fail(e, "destroy");
  return LBM_OK;
}

int32_t lbm_set_force(lbm_ctx* ctx, const double* F, const double* profile_y) {
  if (!ctx) return fail(LBM_EINVAL, "ctx is NULL");
  const int ny = ctx->cfg.ny;
  std::vector<double> tab(3 * (size_t)ny, 0.0);
  if (F) {
    for (int a = 0; a < 3; ++a)
      if (!std::isfinite(F[a])) return fail(LBM_EINVAL, "force component %d is not finite", a);
    for (int y = 0; y < ny; ++y)
      for (int a = 0; a < 3; ++a) tab[3 * (size_t)y + a] = F[a];
  } else if (profile_y) {
    for (size_t i = 0; i < tab.size(); ++i) {
      if (!std::isfinite(profile_y[i])) return fail(LBM_EINVAL, "force profile entry %zu is not finite", i);
      tab[i] = profile_y[i];
    }
  }
  if (ctx->cfg.stencil == LBM_D2Q9)
    for (int y = 0; y < ny; ++y)
      if (tab[3 * (size_t)y + 2] != 0.0) return fail(LBM_EINVAL, "D2Q9 force must have Fz = 0");
  if (ctx->cfg.method == LBM_CUMULANT)
    for (double v : tab)
      if (v != 0.0) return fail(LBM_EUNSUPPORTED, "body forces are not implemented for the cumulant sweep");
  hipError_t e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_fail(e, "set_force sync");
  if (ctx->cfg.dtype == LBM_F64) {
    e = hipMemcpy(ctx->force, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice);
  } else {
    std::vector<float> tf(tab.begin(), tab.end());
    e = hipMemcpy(ctx->force, tf.data(), tf.size() * sizeof(float), hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) return hip_fail(e, "force upload");
  ctx->tape_ok = false;  // a recorded trajectory no longer matches the force
  ctx->adj_t = -1;
  return LBM_OK;
}

int32_t lbm_set_wall_velocity(lbm_ctx* ctx, int32_t wall_type, const double* u) {
  if (!ctx || !u) return fail(LBM_EINVAL, "NULL argument");
  if (wall_type < 2 || wall_type > 127) return fail(LBM_EINVAL, "wall_type must be in 2..127 (1 is the resting wall)");
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(u[a])) return fail(LBM_EINVAL, "wall velocity component %d is not finite", a);
  if (ctx->cfg.stencil == LBM_D2Q9 && u[2] != 0.0) return fail(LBM_EINVAL, "D2Q9 wall velocity must have u_z = 0");
  hipError_t e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_fail(e, "set_wall_velocity sync");
  const size_t off = 3 * (size_t)wall_type;
  if (ctx->cfg.dtype == LBM_F64) {
    e = hipMemcpy((double*)ctx->wall + off, u, 3 * sizeof(double), hipMemcpyHostToDevice);
  } else {
    const float uf[3] = {(float)u[0], (float)u[1], (float)u[2]};
    e = hipMemcpy((float*)ctx->wall + off, uf, 3 * sizeof(float), hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) return hip_fail(e, "wall velocity upload");
  ctx->tape_ok = false;  // a recorded trajectory no longer matches the walls
  ctx->adj_t = -1;
  return LBM_OK;
}

int32_t lbm_init_equilibrium(lbm_ctx* ctx, const void* rho_dev, const void* u_dev, int32_t field_dtype) {
  if (!ctx) return fail(LBM_EINVAL, "ctx is NULL");
  int32_t st = check_field_dtype(field_dtype);
  if (st != LBM_OK) return st;
  ctx->state = ctx->grid[0];
  ctx->t = 0;
  HIP_TRY(launch_init(ctx->cfg.stencil, ctx->cfg.dtype, ctx->grid[0], ctx->flags, ctx->has_mask, layout_of(ctx),
                      rho_dev, u_dev, field_dtype, ctx->g, ctx->p, ctx->stream),
          "init launch");
  int32_t ms = mirror_grid(ctx);
  if (ms != LBM_OK) return ms;
  if (ctx->k > 0)
    HIP_TRY(launch_store_init_fields(ctx->cfg.dtype, rho_dev, u_dev, field_dtype, ctx->init_fields, ctx->g, ctx->p,
                                     ctx->stream),
            "init fields");
  reset_time(ctx);
  return LBM_OK;
}

int32_t lbm_step(lbm_ctx* ctx, int32_t n) {
  if (!ctx) return fail(LBM_EINVAL, "ctx is NULL");
  if (n < 0) return fail(LBM_EINVAL, "n must be >= 0");
  int32_t i = 0;
  if (graph_replay(ctx)) {
    for (; n - i >= kGraphSteps; i += kGraphSteps) {
      const int key = is_aa(ctx) ? (int)(ctx->t & 1) : (ctx->state == ctx->grid[0] ? 0 : 1);
      int32_t st = ensure_graph(ctx, key);
      if (st != LBM_OK) return st;
      HIP_TRY(hipGraphLaunch(ctx->graph_exec[key], ctx->stream), "graph launch");
      ctx->t += kGraphSteps;
    }
  }
  for (; i < n; ++i) {
    if (ctx->k > 0 && ctx->t < ctx->cfg.max_tape_steps && ctx->t % ctx->k == 0) {
      // the tape holds two-array layout: the segment recompute and the
      // adjoint gather read it with the two-array kernels
      char* slot = tape_slot(ctx, ctx->t / ctx->k);
      if (is_aa(ctx)) {
        if (ctx->taped_t != ctx->t)   // the initial state; later checkpoints are written by their sweeps
          HIP_TRY(launch_relayout(ctx->cfg.stencil, ctx->cfg.dtype, ctx->grid[0], ctx->flags, ctx->has_mask,
                                  layout_of(ctx), slot, ctx->g, ctx->p, ctx->stream),
                  "tape relayout");
      } else if (ctx->state != slot)   // the initial state; later checkpoints are swept into their slots
        HIP_TRY(hipMemcpyAsync(slot, ctx->state, ctx->grid_bytes, hipMemcpyDeviceToDevice, ctx->stream),
                "tape copy");
    }
    int32_t st = step_once(ctx);
    if (st != LBM_OK) return st;
  }
  ctx->adj_t = -1;
  return LBM_OK;
}

int32_t lbm_get_time(lbm_ctx* ctx, int64_t* t) {
  if (!ctx || !t) return fail(LBM_EINVAL, "NULL argument");
  *t = ctx->t;
  return LBM_OK;
}

int32_t lbm_get_macroscopic(lbm_ctx* ctx, void* rho_dev, void* u_dev, int32_t field_dtype) {
  if (!ctx) return fail(LBM_EINVAL, "ctx is NULL");
  int32_t st = check_field_dtype(field_dtype);
  if (st != LBM_OK) return st;
  if (!rho_dev && !u_dev) return LBM_OK;
  HIP_TRY(launch_readout(ctx->cfg.stencil, ctx->cfg.dtype, ctx->state, ctx->flags, ctx->has_mask,
                         layout_of(ctx), ctx->force,
                         rho_dev, u_dev, field_dtype, ctx->g, ctx->p, ctx->stream),
          "readout launch");
  return LBM_OK;
}

int32_t lbm_conserved(lbm_ctx* ctx, double out[4]) {
  if (!ctx || !out) return fail(LBM_EINVAL, "NULL argument");
  HIP_TRY(launch_conserved(ctx->cfg.stencil, ctx->cfg.dtype, ctx->state, ctx->flags, ctx->has_mask,
                           layout_of(ctx), ctx->partials, ctx->acc + 4, ctx->g, ctx->p, ctx->stream),
          "conservation launch");
  HIP_TRY(hipMemcpyAsync(out, ctx->acc + 4, 4 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream), "totals copy");
  HIP_TRY(hipStreamSynchronize(ctx->stream), "totals sync");
  for (int i = 0; i < 4; ++i)
    if (!std::isfinite(out[i])) return fail(LBM_ENONFINITE, "conservation total %d is not finite", i);
  return LBM_OK;
}

int32_t lbm_conserved_noalloc(lbm_ctx* ctx, double* totals_dev) {
  if (!ctx || !totals_dev) return fail(LBM_EINVAL, "NULL argument");
  double* scr = noalloc_scratch(ctx->device);
  if (!scr) return fail(LBM_ESTATE, "no scratch address recorded for device %d", ctx->device);
  const int64_t nslots = std::min<int64_t>(num_blocks(ctx->g), kNoAllocSlots);
  HIP_TRY(launch_conserved_noalloc(ctx->cfg.stencil, ctx->cfg.dtype, ctx->state, ctx->flags, ctx->has_mask,
                                   layout_of(ctx), scr, (int)nslots, totals_dev, ctx->g, ctx->p, ctx->stream),
          "conservation launch (no allocation)");
  return LBM_OK;
}

int32_t lbm_get_pdfs(lbm_ctx* ctx, double* pdfs_dev) {
  if (!ctx || !pdfs_dev) return fail(LBM_EINVAL, "NULL argument");
  // solid cells are reported from grid[0], which alone keeps their values
  HIP_TRY(launch_get_pdfs(ctx->cfg.stencil, ctx->cfg.dtype, ctx->state, ctx->grid[0], ctx->flags, ctx->has_mask,
                          layout_of(ctx), pdfs_dev, ctx->g, ctx->p, ctx->stream),
          "get_pdfs launch");
  HIP_TRY(hipStreamSynchronize(ctx->stream), "get_pdfs sync");
  return LBM_OK;
}

int32_t lbm_set_pdfs(lbm_ctx* ctx, const double* pdfs_dev) {
  if (!ctx || !pdfs_dev) return fail(LBM_EINVAL, "NULL argument");
  if (ctx->k > 0) return fail(LBM_ESTATE, "set_pdfs is not available with the adjoint tape (no initial fields)");
  ctx->state = ctx->grid[0];
  ctx->t = 0;
  HIP_TRY(launch_set_pdfs(ctx->cfg.stencil, ctx->cfg.dtype, ctx->grid[0], ctx->flags, ctx->has_mask, layout_of(ctx),
                          pdfs_dev, ctx->g, ctx->p, ctx->stream),
          "set_pdfs launch");
  int32_t ms = mirror_grid(ctx);
  if (ms != LBM_OK) return ms;
  reset_time(ctx);
  return LBM_OK;
}

// ------------------------------------------------------------------ adjoint
int32_t lbm_adjoint_seed(lbm_ctx* ctx, const void* dL_drho_dev, const void* dL_du_dev, int32_t field_dtype) {
  if (!ctx) return fail(LBM_EINVAL, "ctx is NULL");
  int32_t st = check_field_dtype(field_dtype);
  if (st != LBM_OK) return st;
  if (!dL_du_dev) return fail(LBM_EINVAL, "dL_du_dev is NULL");
  if (ctx->k <= 0) return fail(LBM_ESTATE, "the context was created without a tape (checkpoint_every = 0)");
  if (!ctx->tape_ok) return fail(LBM_ESTATE, "the tape is invalid (force changed after initialisation)");
  if (ctx->t > ctx->cfg.max_tape_steps)
    return fail(LBM_ESTATE, "%lld steps exceed max_tape_steps = %d", (long long)ctx->t, ctx->cfg.max_tape_steps);
  // lambda^T goes into the AA layout of time T (1 after an odd number of
  // steps, 2 after an even one) whatever the forward pattern; the seed
  // writes every slot
  HIP_TRY(launch_adjoint_seed(ctx->cfg.stencil, ctx->cfg.dtype, ctx->state, ctx->flags, ctx->has_mask,
                              layout_of(ctx), (ctx->t & 1) ? 1 : 2, ctx->force, dL_drho_dev, dL_du_dev,
                              field_dtype, ctx->lam, ctx->adj_acc, ctx->g, ctx->p, ctx->stream),
          "adjoint seed launch");
  ctx->adj_T = ctx->t;
  ctx->adj_t = ctx->t;
  ctx->seg_id = -1;
  if (ctx->t > 0 && ctx->k > 1) {
    // the forward left the states of the last segment in the segment buffer
    const int64_t J = (ctx->t - 1) / ctx->k;
    if (ctx->seg_fwd_lo == J * ctx->k + 1) ctx->seg_id = J;
    // the recompute of earlier segments overwrites that buffer: a two-array
    // current state kept there moves to grid[1] (free while a tape is recorded)
    if (in_seg(ctx, ctx->state)) {
      HIP_TRY(hipMemcpyAsync(ctx->grid[1], ctx->state, ctx->grid_bytes, hipMemcpyDeviceToDevice, ctx->stream),
              "state copy");
      ctx->state = ctx->grid[1];
    }
  }
  return LBM_OK;
}

namespace {

// Forward state P^s for the adjoint: a tape slot, or a recomputed state of
// the k-step segment that contains s.
int32_t forward_state(lbm_ctx* c, int64_t s, const void** out) {
  const int64_t j = s / c->k, r = s % c->k;
  const char* slot = (const char*)c->tape + (size_t)j * c->grid_bytes;
  if (r == 0) {
    *out = slot;
    return LBM_OK;
  }
  if (c->seg_id != j) {
    c->seg_fwd_lo = INT64_MAX;
    const int64_t last = std::min<int64_t>(c->k - 1, c->adj_T - 1 - j * c->k);
    const void* src = slot;
    for (int64_t i = 1; i <= last; ++i) {
      void* dst = (char*)c->seg + (size_t)(i - 1) * c->grid_bytes;
      int32_t st = sweep_once(c, src, dst, j * c->k + i - 1);
      if (st != LBM_OK) return st;
      src = dst;
    }
    c->seg_id = j;
  }
  *out = (const char*)c->seg + (size_t)(r - 1) * c->grid_bytes;
  return LBM_OK;
}

}  // namespace

int32_t lbm_adjoint_step(lbm_ctx* ctx, int32_t n) {
  if (!ctx) return fail(LBM_EINVAL, "ctx is NULL");
  if (n < 0) return fail(LBM_EINVAL, "n must be >= 0");
  if (ctx->adj_t < 0) return fail(LBM_ESTATE, "no adjoint seeded (or the forward state changed since)");
  if (n > ctx->adj_t) return fail(LBM_ESTATE, "%d adjoint steps requested, %lld remain", n, (long long)ctx->adj_t);
  for (int32_t i = 0; i < n; ++i) {
    const int64_t s = ctx->adj_t - 1;
    const void* P = nullptr;
    int32_t st = forward_state(ctx, s, &P);
    if (st != LBM_OK) return st;
    // transpose of the AA even (s even) or odd kernel, in place on lambda
    HIP_TRY(launch_adjoint_sweep(ctx->cfg.stencil, ctx->kmethod, ctx->cfg.dtype, (int)(s & 1), P, ctx->flags,
                                 ctx->has_mask, ctx->force, ctx->lam, ctx->adj_acc, sweep_geo(ctx, s), ctx->p,
                                 ctx->stream),
            "adjoint sweep launch");
    ctx->adj_t -= 1;
  }
  return LBM_OK;
}

int32_t lbm_adjoint_grads(lbm_ctx* ctx, void* dL_du0_dev, void* dL_drho0_dev, int32_t field_dtype, double* dL_dF) {
  if (!ctx) return fail(LBM_EINVAL, "ctx is NULL");
  int32_t st = check_field_dtype(field_dtype);
  if (st != LBM_OK) return st;
  if (ctx->adj_t != 0) return fail(LBM_ESTATE, "the adjoint has not reached t = 0");
  if (dL_du0_dev || dL_drho0_dev)
    HIP_TRY(launch_adjoint_init_grad(ctx->cfg.stencil, ctx->cfg.dtype, ctx->lam, ctx->flags,
                                     ctx->has_mask, 2, ctx->init_fields, dL_du0_dev, dL_drho0_dev,
                                     field_dtype, ctx->g, ctx->p, ctx->stream),
            "init gradient launch");
  if (dL_dF) {
    HIP_TRY(launch_sum_partials(ctx->adj_acc, num_blocks(ctx->g), 3, ctx->acc, 0, ctx->stream), "dL/dF reduction");
    HIP_TRY(hipMemcpyAsync(dL_dF, ctx->acc, 3 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream), "dL/dF copy");
    HIP_TRY(hipStreamSynchronize(ctx->stream), "dL/dF sync");
  }
  return LBM_OK;
}

int32_t lbm_copy_q(const void* src_dev, void* dst_dev, int64_t n, int32_t q, int32_t elem_bytes,
                   int32_t waves_per_cu, int32_t block_threads, void* hip_stream) {
  if (!src_dev || !dst_dev) return fail(LBM_EINVAL, "NULL buffer");
  if (n < 1 || q < 1) return fail(LBM_EINVAL, "n and q must be >= 1");
  if (elem_bytes != 2 && elem_bytes != 4 && elem_bytes != 8) return fail(LBM_EINVAL, "elem_bytes must be 2, 4 or 8");
  if (waves_per_cu < 0 || waves_per_cu > 32) return fail(LBM_EINVAL, "waves_per_cu must be in 0..32");
  if (block_threads == 0) block_threads = 256;
  if (block_threads < 64 || block_threads > 512 || block_threads % 64 != 0)
    return fail(LBM_EINVAL, "block_threads must be 0 or a multiple of 64 in 64..512");
  if ((n + block_threads - 1) / block_threads > 0x7fffffff) return fail(LBM_EINVAL, "n too large for one launch");
  HIP_TRY(launch_copy_q(src_dev, dst_dev, n, q, elem_bytes, waves_per_cu, block_threads, (hipStream_t)hip_stream),
          "copy_q launch");
  return LBM_OK;
}

int32_t lbm_stream_q(const void* src_dev, void* dst_dev, int32_t nx, int32_t ny, int32_t nz, lbm_stencil stencil,
                     int32_t elem_bytes, int32_t waves_per_cu, int32_t block_threads, void* hip_stream) {
  if (!src_dev || !dst_dev) return fail(LBM_EINVAL, "NULL buffer");
  if (stencil < 0 || stencil > 2) return fail(LBM_EINVAL, "unknown stencil %d", stencil);
  if (nx < 1 || ny < 1 || nz < 1) return fail(LBM_EINVAL, "lattice dims must be >= 1 (got %d x %d x %d)", nx, ny, nz);
  const int64_t N = (int64_t)nx * ny * nz;
  if (N >= (int64_t(1) << 31)) return fail(LBM_EINVAL, "lattice has %lld cells; the limit is 2^31 - 1", (long long)N);
  if (stencil == LBM_D2Q9 && nz != 1) return fail(LBM_EINVAL, "D2Q9 needs nz == 1");
  if (elem_bytes != 2 && elem_bytes != 4 && elem_bytes != 8) return fail(LBM_EINVAL, "elem_bytes must be 2, 4 or 8");
  if (waves_per_cu < 0 || waves_per_cu > 32) return fail(LBM_EINVAL, "waves_per_cu must be in 0..32");
  if (block_threads < 0 || block_threads > 512 || block_threads % 64 != 0)
    return fail(LBM_EINVAL, "block_threads must be 0 or a multiple of 64 in 64..512");
  Geo g{};
  g.nx = nx;
  g.ny = ny;
  g.nz = nz;
  // 0: the sweep's default segmentation (rows of up to 512 cells in equal segments)
  g.nxb = block_threads ? (nx + block_threads - 1) / block_threads : (nx + 511) / 512;
  g.bx = block_threads ? block_threads : (((nx + g.nxb - 1) / g.nxb + 63) / 64) * 64;
  g.N = N;
  HIP_TRY(launch_stream_q(src_dev, dst_dev, stencil, g, elem_bytes, waves_per_cu, (hipStream_t)hip_stream),
          "stream_q launch");
  return LBM_OK;
}

int32_t lbm_stream_aa_q(void* buf_dev, int32_t nx, int32_t ny, int32_t nz, lbm_stencil stencil, int32_t elem_bytes,
                        int32_t phase, int32_t waves_per_cu, int32_t block_threads, void* hip_stream) {
  if (!buf_dev) return fail(LBM_EINVAL, "NULL buffer");
  if (stencil < 0 || stencil > 2) return fail(LBM_EINVAL, "unknown stencil %d", stencil);
  if (nx < 1 || ny < 1 || nz < 1) return fail(LBM_EINVAL, "lattice dims must be >= 1 (got %d x %d x %d)", nx, ny, nz);
  const int64_t N = (int64_t)nx * ny * nz;
  if (N >= (int64_t(1) << 31)) return fail(LBM_EINVAL, "lattice has %lld cells; the limit is 2^31 - 1", (long long)N);
  if (stencil == LBM_D2Q9 && nz != 1) return fail(LBM_EINVAL, "D2Q9 needs nz == 1");
  if (elem_bytes != 2 && elem_bytes != 4 && elem_bytes != 8) return fail(LBM_EINVAL, "elem_bytes must be 2, 4 or 8");
  if (phase != 0 && phase != 1) return fail(LBM_EINVAL, "phase must be 0 (even) or 1 (odd)");
  if (waves_per_cu < 0 || waves_per_cu > 32) return fail(LBM_EINVAL, "waves_per_cu must be in 0..32");
  if (block_threads < 0 || block_threads > 512 || block_threads % 64 != 0)
    return fail(LBM_EINVAL, "block_threads must be 0 or a multiple of 64 in 64..512");
  Geo g{};
  g.nx = nx;
  g.ny = ny;
  g.nz = nz;
  g.nxb = block_threads ? (nx + block_threads - 1) / block_threads : (nx + 511) / 512;
  g.bx = block_threads ? block_threads : (((nx + g.nxb - 1) / g.nxb + 63) / 64) * 64;
  g.N = N;
  // the AA sweep's block order: direction alternating with the phase, and
  // XCD slabs on grids within cache reach
  const size_t bytes = (size_t)N * (size_t)q_of(stencil) * (size_t)elem_bytes;
  g.order = (bytes <= kStreamGridBytes && num_blocks(g) % 8 == 0 ? 2 : 0) | phase;
  HIP_TRY(launch_stream_aa_q(buf_dev, stencil, g, elem_bytes, phase, waves_per_cu, (hipStream_t)hip_stream),
          "stream_aa_q launch");
  return LBM_OK;
}

}  // extern "C"
