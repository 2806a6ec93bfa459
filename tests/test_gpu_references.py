"""The bandwidth references of the C ABI, checked bit for bit (pure data
movement): lbm_copy_q (Q planes copied), lbm_stream_q (periodic pull
streaming, dst[q][x] = src[q][x - c_q], the streaming half of Eq. (1)) and
lbm_stream_aa_q (the AA pattern's two in-place kernels without collision),
against numpy's roll on small ragged lattices and torch's roll on lattices
above the 512 MiB non-temporal-store threshold.  Payloads are random integers
of the element width, so any misplaced, dropped or doubled element shows."""

import numpy as np
import pytest

from tests.gpu_common import need_gpu, torch
from oracle import lattice
from paper_2001_11806_amd.lbm import copy_q, stream_aa_q, stream_q

pytestmark = pytest.mark.gpu

_INT = {2: (np.int16, torch.int16), 4: (np.int32, torch.int32), 8: (np.int64, torch.int64)}


def _payload(shape, elem_bytes, seed):
    nt, _ = _INT[elem_bytes]
    info = np.iinfo(nt)
    return np.random.default_rng(seed).integers(info.min, info.max, size=shape, dtype=nt, endpoint=True)


def _pull(src, c):
    """dst[q] = src[q] shifted by +c_q with periodic wrap (array axes z, y, x)."""
    return np.stack([np.roll(src[q], shift=(int(v[2]), int(v[1]), int(v[0])), axis=(0, 1, 2))
                     for q, v in enumerate(c)])


@pytest.mark.parametrize("elem_bytes", [2, 4, 8])
@pytest.mark.parametrize("stencil,dims,block", [
    ("D2Q9", (141, 9, 1), 0), ("D2Q9", (1, 1, 1), 0), ("D2Q9", (64, 3, 1), 64),
    ("D3Q19", (141, 7, 5), 0), ("D3Q19", (141, 7, 5), 64), ("D3Q19", (600, 3, 2), 0),
    ("D3Q19", (2, 1, 3), 0), ("D3Q27", (141, 7, 5), 128), ("D3Q27", (600, 3, 2), 256),
    ("D3Q27", (384, 4, 3), 128)])
def test_stream_q_is_periodic_pull(stencil, dims, block, elem_bytes):
    need_gpu()
    lat = lattice.velocity_set(stencil)
    nx, ny, nz = dims
    src = _payload((lat.Q, nz, ny, nx), elem_bytes, seed=nx + 7 * ny + elem_bytes)
    _, tt = _INT[elem_bytes]
    s = torch.from_numpy(src).cuda()
    d = torch.zeros_like(s)
    st = torch.cuda.current_stream()
    stream_q(s, d, dims, stencil, elem_bytes, st, waves_per_cu=0, block_threads=block)
    torch.cuda.synchronize()
    assert np.array_equal(d.cpu().numpy(), _pull(src, lat.c))


def test_stream_q_streaming_size_nontemporal():
    """D3Q19 FP64-sized planes at 256 x 256 x 96 (0.96 GB, non-temporal
    stores) in the headline launch shape (12 waves per CU, 256-cell rows),
    and D3Q27 2-byte planes at 512 x 64 x 160 (0.88 GB) in 512-cell rows:
    equal to torch's roll."""
    need_gpu()
    st = torch.cuda.current_stream()
    for stencil, (nx, ny, nz), eb, waves, block in [("D3Q19", (256, 256, 96), 8, 12, 256),
                                                   ("D3Q27", (512, 64, 160), 2, 0, 512)]:
        lat = lattice.velocity_set(stencil)
        _, tt = _INT[eb]
        g = torch.Generator(device="cuda").manual_seed(11)
        info = torch.iinfo(tt)
        s = torch.randint(info.min, info.max, (lat.Q, nz, ny, nx), dtype=tt, device="cuda", generator=g)
        d = torch.empty_like(s)
        stream_q(s, d, (nx, ny, nz), stencil, eb, st, waves_per_cu=waves, block_threads=block)
        torch.cuda.synchronize()
        for q, v in enumerate(lat.c):
            ref = torch.roll(s[q], shifts=(int(v[2]), int(v[1]), int(v[0])), dims=(0, 1, 2))
            assert torch.equal(d[q], ref), (stencil, q)
        del s, d
        torch.cuda.empty_cache()


def _aa(src, lat, phase):
    """Even: plane q <- plane opp(q).  Odd: A[q][x + c_q] <- A[opp q][x - c_q],
    plane q <- plane opp(q) shifted by 2 c_q (periodic)."""
    if phase == 0:
        return src[lat.opp]
    return np.stack([np.roll(src[lat.opp[q]], shift=(2 * int(v[2]), 2 * int(v[1]), 2 * int(v[0])), axis=(0, 1, 2))
                     for q, v in enumerate(lat.c)])


@pytest.mark.parametrize("elem_bytes", [2, 4, 8])
@pytest.mark.parametrize("stencil,dims,block", [
    ("D2Q9", (141, 9, 1), 0), ("D2Q9", (1, 1, 1), 0), ("D2Q9", (2, 3, 1), 64),
    ("D3Q19", (141, 7, 5), 0), ("D3Q19", (141, 7, 5), 64), ("D3Q19", (600, 3, 2), 0),
    ("D3Q19", (2, 1, 3), 0), ("D3Q19", (256, 4, 2), 256), ("D3Q27", (141, 7, 5), 128),
    ("D3Q27", (600, 3, 2), 256), ("D3Q27", (384, 4, 3), 128), ("D3Q27", (1, 2, 1), 0)])
def test_stream_aa_q_is_the_aa_data_movement(stencil, dims, block, elem_bytes):
    """Five launches in a row (even, odd, even, odd, odd: the last two are
    two odd moves in a row), each in place on one buffer."""
    need_gpu()
    lat = lattice.velocity_set(stencil)
    nx, ny, nz = dims
    expect = _payload((lat.Q, nz, ny, nx), elem_bytes, seed=3 * nx + ny + elem_bytes)
    buf = torch.from_numpy(expect).cuda()
    st = torch.cuda.current_stream()
    for phase in (0, 1, 0, 1, 1):
        stream_aa_q(buf, dims, stencil, elem_bytes, phase, st, waves_per_cu=0, block_threads=block)
        expect = _aa(expect, lat, phase)
    torch.cuda.synchronize()
    assert np.array_equal(buf.cpu().numpy(), expect)


def test_stream_aa_q_streaming_size_nontemporal():
    """D3Q19 8-byte planes at 256 x 256 x 96 (0.96 GB, non-temporal stores)
    in the AA sweep's launch shape (16 waves per CU, 256-cell rows) and
    D3Q27 2-byte planes at 512 x 64 x 160 in 512-cell rows: an even then an
    odd move leave plane q shifted by 2 c_q."""
    need_gpu()
    st = torch.cuda.current_stream()
    for stencil, (nx, ny, nz), eb, waves, block in [("D3Q19", (256, 256, 96), 8, 16, 256),
                                                   ("D3Q27", (512, 64, 160), 2, 0, 512)]:
        lat = lattice.velocity_set(stencil)
        _, tt = _INT[eb]
        g = torch.Generator(device="cuda").manual_seed(13)
        info = torch.iinfo(tt)
        s = torch.randint(info.min, info.max, (lat.Q, nz, ny, nx), dtype=tt, device="cuda", generator=g)
        a = s.clone()
        stream_aa_q(a, (nx, ny, nz), stencil, eb, 0, st, waves_per_cu=waves, block_threads=block)
        stream_aa_q(a, (nx, ny, nz), stencil, eb, 1, st, waves_per_cu=waves, block_threads=block)
        torch.cuda.synchronize()
        for q, v in enumerate(lat.c):
            ref = torch.roll(s[q], shifts=(2 * int(v[2]), 2 * int(v[1]), 2 * int(v[0])), dims=(0, 1, 2))
            assert torch.equal(a[q], ref), (stencil, q)
        del s, a
        torch.cuda.empty_cache()


@pytest.mark.parametrize("elem_bytes", [2, 4, 8])
@pytest.mark.parametrize("q,n,block,waves", [(19, 1000, 0, 0), (27, 4097, 64, 0), (9, 130, 512, 16),
                                             (5, 77, 128, 12), (1, 1, 0, 0)])
def test_copy_q_copies_every_plane(q, n, block, waves, elem_bytes):
    need_gpu()
    src = torch.from_numpy(_payload((q, n), elem_bytes, seed=q * n)).cuda()
    dst = torch.zeros_like(src)
    copy_q(src, dst, n, q, elem_bytes, torch.cuda.current_stream(), waves, block)
    torch.cuda.synchronize()
    assert torch.equal(src, dst)


def test_copy_q_streaming_size_nontemporal():
    """19 planes of 4M 8-byte elements (0.64 GB, non-temporal stores)."""
    need_gpu()
    n, q = 1 << 22, 19
    g = torch.Generator(device="cuda").manual_seed(5)
    src = torch.randint(-2 ** 62, 2 ** 62, (q, n), dtype=torch.int64, device="cuda", generator=g)
    dst = torch.zeros_like(src)
    copy_q(src, dst, n, q, 8, torch.cuda.current_stream(), 12, 256)
    torch.cuda.synchronize()
    assert torch.equal(src, dst)
