"""lbm_conserved_noalloc (the entry point for callers that cannot allocate)
against lbm_conserved, through the C ABI on the GPU: two calls in a row, the
second on a smaller lattice, each compared with the allocating entry point on
the same state.  The first lattice has more row segments (8448) than the
scratch has rows (4096), so its reduction runs in strides; the second is
small and uses 6 rows, so stale rows of the first call must not leak in."""

import numpy as np
import pytest

from tests.gpu_common import RATES, make_gpu, need_gpu, seeded_fields, torch

pytestmark = pytest.mark.gpu


def _case(stencil, method, dtype, dims, pattern, steps, seed):
    mask, rho, u = seeded_fields(stencil, dims, seed)
    g = make_gpu(stencil, method, dtype, dims, mask, RATES, pattern=pattern)
    g.set_force([1e-4, -2e-5, 0.0 if stencil == "D2Q9" else 3e-5])
    g.init_equilibrium(torch.tensor(rho), torch.tensor(u))
    g.step(steps)
    return g, int((mask == 0).sum())


def _check(g, fluid, out):
    want = g.conserved()
    out.fill_(float("nan"))
    g.conserved_noalloc(out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()[:4]
    print("noalloc", got, "conserved", want, flush=True)
    # same FP64 values summed in another order: mass to 1e-13 relative;
    # momentum totals (which cancel) to 1e-13 of the mass scale
    assert abs(got[0] - want[0]) <= 1e-13 * abs(want[0])
    assert np.all(np.abs(got[1:] - want[1:]) <= 1e-13 * fluid)


def test_conserved_noalloc_matches_conserved_two_calls():
    need_gpu()
    out = torch.empty(4, dtype=torch.float64, device="cuda")
    print("case 1: D3Q19 TRT f32 two arrays 150 x 96 x 88, 7 steps", flush=True)
    g1, f1 = _case("D3Q19", "TRT", "f32", (150, 96, 88), 0, 7, 11)
    assert g1.dims[1] * g1.dims[2] > 4096
    _check(g1, f1, out)
    print("case 2: D2Q9 SRT f64 AA 141 x 6, 5 steps", flush=True)
    g2, f2 = _case("D2Q9", "SRT", "f64", (141, 6, 1), 1, 5, 12)
    _check(g2, f2, out)
    print("case 3: back to the first lattice after 3 more steps", flush=True)
    g1.step(3)
    _check(g1, f1, out)
    g1.close()
    g2.close()
