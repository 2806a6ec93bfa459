"""Shared helpers for the GPU parity tests: run a case through the HIP C ABI
and the same case through the CPU oracle on identical seeded inputs."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import equilibrium as oeq, run as orun  # noqa: E402
from paper_2001_11806_amd import inputs  # noqa: E402
from paper_2001_11806_amd.lbm import LBM  # noqa: E402

ULP_BITS = {"f32": 24, "bf16": 8, "f16": 11}

RATES = dict(omega=1 / 0.8, omega_bulk=1.2, omega_odd=0.0, magic=3.0 / 16.0, omega_hi=(1.0, 1.0, 1.0, 1.0))


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def case_dims(stencil):
    """Small ragged lattice: several 64-wide tiles in x plus a ragged tail."""
    return (141, 9, 1) if stencil == "D2Q9" else (141, 7, 5)


def seeded_fields(stencil, dims, seed, amp=2e-2, with_mask=True):
    nx, ny, nz = dims
    rng = np.random.default_rng(seed)
    mask = None
    if with_mask:
        mask = (rng.random((nz, ny, nx)) < 0.12).astype(np.uint8)
        mask[:, 0, :] = 1
    rho = 1.0 + 0.01 * rng.uniform(-1, 1, (nz, ny, nx))
    u = inputs.uniform_noise_velocity(dims, amp, seed + 100, mask)
    if stencil == "D2Q9":
        u[2] = 0
    return mask, rho, u


def make_gpu(stencil, method, dtype, dims, mask, rates=RATES, **kw):
    kw.setdefault("cs_smag", rates.get("cs_smag", 0.0))
    return LBM(stencil, method, dtype, dims, rates["omega"], rates["omega_bulk"], rates["omega_odd"],
               rates["magic"], rates["omega_hi"], mask=mask, **kw)


def oracle_cfg(stencil, method, dtype, rates=RATES):
    return orun.Config(stencil, method, rates, storage=dtype)


def to_np(t):
    return t.detach().to("cpu").numpy()


def ulp_of(x, dtype):
    """Spacing of the storage format at |x| (normal range; subnormal floor)."""
    bits = ULP_BITS[dtype]
    ax = np.abs(x)
    e = np.floor(np.log2(np.where(ax > 0, ax, 1e-300)))
    spacing = 2.0 ** (e - (bits - 1))
    floor = {"f32": 2.0 ** -149, "bf16": 2.0 ** -133, "f16": 2.0 ** -24}[dtype]
    return np.maximum(spacing, floor)


def rho_spacing_bar(rho_ref, bar=1e-12):
    """Bar for the relative L2 error of rho - 1 when rho is returned in FP64:
    ``bar``, or one FP64 spacing of rho (2^-52 near 1) per cell in the RMS,
    whichever is larger.  No FP64 value of rho, however accurate, carries
    rho - 1 more finely than that spacing, and |rho - 1| is small (1e-6 ..
    1e-3) in these flows."""
    d = np.asarray(rho_ref, dtype=np.float64).ravel() - 1.0
    return max(bar, 2.0 ** -52 * np.sqrt(d.size) / max(np.linalg.norm(d), 1e-300))


def rel_l2(a, b):
    """||a - b|| / ||b||; the difference is taken in the wider of the two
    floating types (long double references keep their extra bits)."""
    t = np.result_type(np.asarray(a).dtype, np.asarray(b).dtype, np.float64)
    d = (np.asarray(a, dtype=t) - np.asarray(b, dtype=t)).astype(np.float64)
    return float(np.linalg.norm(d.ravel()) / max(np.linalg.norm(np.asarray(b, dtype=np.float64).ravel()), 1e-300))
