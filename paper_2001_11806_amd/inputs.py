"""Seeded synthetic inputs for the lattice Boltzmann workloads.

This module holds no arithmetic of the method itself: it only produces
initial macroscopic fields, solid masks and body-force profiles with numpy's
PCG64 generator (``numpy.random.default_rng(seed)``).  Tests hand the same
arrays to the HIP library and to the CPU oracle.

Array conventions: scalar fields (nz, ny, nx), vector fields (3, nz, ny, nx),
x fastest in memory; masks are uint8 with 1 = solid; force profiles are
(ny, 3).  The workloads mirror the paper's synthetic setups (a periodic box
and a channel, Sec. V); there is no dataset.
"""

import functools

import numpy as np


def taylor_green_2d(n=64, u0=0.01, rho0=1.0):
    """Taylor-Green vortex on an n x n periodic lattice, one wavelength per
    axis: u_x = -u0 cos(kx) sin(ky), u_y = u0 sin(kx) cos(ky), k = 2 pi / n,
    with the matching pressure field folded into rho:
    rho = rho0 - 3 rho0 u0^2 / 4 (cos 2kx + cos 2ky)."""
    k = 2.0 * np.pi / n
    x = np.arange(n, dtype=np.float64)[None, :]
    y = np.arange(n, dtype=np.float64)[:, None]
    u = np.zeros((3, 1, n, n))
    u[0, 0] = -u0 * np.cos(k * x) * np.sin(k * y)
    u[1, 0] = u0 * np.sin(k * x) * np.cos(k * y)
    rho = rho0 - 0.75 * rho0 * u0 * u0 * (np.cos(2 * k * x) + np.cos(2 * k * y))
    return rho.reshape(1, n, n), u


def channel_mask(nx, ny, nz):
    """Solid cell planes at y = 0 and y = ny - 1, periodic in x and z."""
    m = np.zeros((nz, ny, nx), dtype=np.uint8)
    m[:, 0, :] = 1
    m[:, ny - 1, :] = 1
    return m


def uniform_noise_velocity(dims, amp, seed, mask=None, dtype=np.float64):
    """i.i.d. uniform(-amp, amp) per component and cell; zero at solid cells."""
    nx, ny, nz = dims
    rng = np.random.default_rng(seed)
    u = rng.uniform(-amp, amp, size=(3, nz, ny, nx)).astype(dtype)
    if mask is not None:
        u[:, mask.astype(bool)] = 0
    return u


def channel_flow(n=256, seed=2, amp=1e-3, nx=None, nz=None):
    """Channel workload: walls at y = 0 and y = n-1, rho = 1, u uniform noise
    of amplitude ``amp`` on fluid cells.  Returns (mask, rho, u)."""
    nx = n if nx is None else nx
    nz = n if nz is None else nz
    mask = channel_mask(nx, n, nz)
    u = uniform_noise_velocity((nx, n, nz), amp, seed, mask)
    rho = np.ones((nz, n, nx))
    return mask, rho, u


def sphere_channel_mask(n=128, seed=4, radius=8.0, fraction=0.05, nx=None, nz=None):
    """Channel walls (y = 0, y = ny-1) plus spheres of the given radius whose
    centres are seeded uniformly (periodic in x and z, inside the walls in y),
    added until the solid fraction of the interior reaches ``fraction``."""
    nx = n if nx is None else nx
    nz = n if nz is None else nz
    ny = n
    rng = np.random.default_rng(seed)
    mask = channel_mask(nx, ny, nz)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    interior = (y > 0) & (y < ny - 1)
    target = fraction * interior.sum()
    while mask[interior].sum() < target:
        cx, cz = rng.uniform(0, nx), rng.uniform(0, nz)
        cy = rng.uniform(1 + radius, ny - 1 - radius)
        dx = np.abs(x - cx)
        dx = np.minimum(dx, nx - dx)
        dz = np.abs(z - cz)
        dz = np.minimum(dz, nz - dz)
        inside = dx * dx + (y - cy) ** 2 + dz * dz <= radius * radius
        mask[inside] = 1
    return mask


@functools.lru_cache(maxsize=None)
def solenoidal_modes(seed=3, nmodes=32, kmax=4, umax=0.05, n_norm=384):
    """Random Fourier modes for a divergence-free field:
    u(x) = sum_m a_m cos(2 pi k_m . x / n + phi_m), integer k_m in
    [-kmax, kmax]^3 without 0, a_m perpendicular to k_m, scaled so that the
    largest speed |u| on the n_norm^3 lattice is umax (smaller lattices
    sample the same field more coarsely, so their largest speed is at most
    umax)."""
    rng = np.random.default_rng(seed)
    ks, amps, phis = [], [], []
    while len(ks) < nmodes:
        k = rng.integers(-kmax, kmax + 1, size=3)
        if not k.any():
            continue
        a = rng.normal(size=3)
        kk = k.astype(np.float64)
        a = a - kk * (a @ kk) / (kk @ kk)
        ks.append(k)
        amps.append(a)
        phis.append(rng.uniform(0, 2 * np.pi))
    amps = np.array(amps)
    amps /= np.linalg.norm(amps, axis=1).sum()
    modes = (np.array(ks), amps, np.array(phis))
    u = solenoidal_velocity(n_norm, modes)
    speed = np.sqrt((u * u).sum(axis=0)).max()
    del u
    return modes[0], amps * (umax / speed), modes[2]


def solenoidal_velocity(n, modes, dtype=np.float64):
    """Evaluate ``solenoidal_modes`` on the full n^3 periodic lattice.

    Each mode factorises as exp(i k_z z') exp(i (k_y y' + k_x x')), so the
    sum over modes is one complex matrix product per component."""
    ks, amps, phis = modes
    r = np.arange(n, dtype=np.float64) * (2 * np.pi / n)
    Ez = np.exp(1j * (np.outer(ks[:, 2], r) + phis[:, None]))                  # (M, nz)
    Exy = (np.exp(1j * np.outer(ks[:, 1], r))[:, :, None]
           * np.exp(1j * np.outer(ks[:, 0], r))[:, None, :]).reshape(len(ks), -1)   # (M, ny*nx)
    u = np.empty((3, n, n, n), dtype=dtype)
    for c in range(3):
        u[c] = (((amps[:, c:c + 1] * Ez).T @ Exy).real).reshape(n, n, n)
    return u


def solenoidal_velocity_at(n, modes, cells):
    """Evaluate ``solenoidal_modes`` at linear cell indices only (float64)."""
    ks, amps, phis = modes
    x = (cells % n).astype(np.float64)
    y = ((cells // n) % n).astype(np.float64)
    z = (cells // (n * n)).astype(np.float64)
    u = np.zeros((3, cells.size))
    for k, a, ph in zip(ks, amps, phis):
        phase = np.cos(2 * np.pi * (k[0] * x + k[1] * y + k[2] * z) / n + ph)
        u += a[:, None] * phase[None, :]
    return u


def kolmogorov_force_profile(ny, amp=1e-6):
    """Per-y body force F_x(y) = amp sin(2 pi y / ny), F_y = F_z = 0."""
    F = np.zeros((ny, 3))
    F[:, 0] = amp * np.sin(2 * np.pi * np.arange(ny) / ny)
    return F


def sample_cells(dims, count, seed, include_corners=True):
    """Seeded sample of linear cell indices, including the eight lattice
    corners (where every periodic wrap is exercised)."""
    nx, ny, nz = dims
    rng = np.random.default_rng(seed)
    cells = rng.integers(0, nx * ny * nz, size=count)
    if include_corners:
        corners = [((z * ny + y) * nx + x) for z in (0, nz - 1) for y in (0, ny - 1) for x in (0, nx - 1)]
        cells = np.concatenate([cells, np.array(corners)])
    return np.unique(cells)
