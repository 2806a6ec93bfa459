"""A lattice on a HIP stream of its own (not torch's current stream).

The binding orders every call that reads or writes torch tensors against
torch's current stream: inputs made there are read only once they are
ready, and outputs are used there only once they are written.  Each side is
held up by a few milliseconds of unrelated work queued ahead of the call, so
that a missing wait would show as wrong values; the results must equal, bit
for bit, those of the same run on the current stream."""

import numpy as np
import pytest

from tests.gpu_common import RATES, need_gpu, torch
from paper_2001_11806_amd import inputs
from paper_2001_11806_amd.lbm import LBM

pytestmark = pytest.mark.gpu

DIMS = (70, 12, 6)


def _busy():
    """About ten milliseconds of elementwise work on the current stream."""
    x = torch.ones(1 << 26, dtype=torch.float32, device="cuda")
    for _ in range(24):
        x.mul_(1.0000001)
    return x


def _made_late(a):
    """A device copy of `a` whose values are written behind `_busy` on the
    current stream."""
    t = torch.from_numpy(np.ascontiguousarray(a)).cuda()
    _busy()
    return t * 1.0


def _inputs():
    mask = inputs.channel_mask(*DIMS)
    u0 = inputs.uniform_noise_velocity(DIMS, 1e-2, 5, mask)
    rho = 1.0 + 1e-3 * np.random.default_rng(6).uniform(-1, 1, DIMS[::-1])
    return mask, rho, u0


def _forward(stream):
    mask, rho, u0 = _inputs()
    g = LBM("D3Q19", "TRT", "f64", DIMS, RATES["omega"], magic=RATES["magic"], mask=mask, stream=stream,
            checkpoint_every=4, max_tape_steps=8)
    g.set_force([1e-5, 0.0, 0.0])
    g.init_equilibrium(_made_late(rho), _made_late(u0))
    g.step(8)
    if stream is not None:
        with torch.cuda.stream(stream):
            _busy()
    rho_t, u_t = g.macroscopic()
    out = [rho_t.cpu().numpy(), u_t.cpu().numpy()]
    return g, out


def _backward(g, stream):
    seed = np.random.default_rng(8).standard_normal((3,) + DIMS[::-1])
    g.adjoint_seed(_made_late(seed))
    g.adjoint_step(8)
    if stream is not None:
        with torch.cuda.stream(stream):
            _busy()
    du, _, dF = g.adjoint_grads()
    return [du.cpu().numpy(), dF]


def test_lattice_on_a_side_stream_equals_the_current_stream():
    need_gpu()
    results = []
    for stream in (None, torch.cuda.Stream()):
        g, out = _forward(stream)
        out += _backward(g, stream)
        g.close()
        # PDFs in and out (a lattice without a tape accepts them)
        h = LBM("D3Q19", "TRT", "f64", DIMS, RATES["omega"], magic=RATES["magic"], mask=_inputs()[0],
                stream=stream)
        P = 0.05 + 0.01 * np.random.default_rng(9).random((19,) + DIMS[::-1])
        h.set_pdfs(_made_late(P))    # read after the current stream has written it
        h.step(3)
        if stream is not None:
            with torch.cuda.stream(stream):
                _busy()
        out.append(h.get_pdfs().cpu().numpy())
        out.append(h.conserved())
        h.close()
        results.append(out)
    a, b = results
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    assert np.abs(a[1]).max() > 1e-4 and np.abs(a[2]).max() > 0   # a flow and a gradient, not zeros
