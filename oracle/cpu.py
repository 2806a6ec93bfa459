"""ctypes binding of the C++17 / OpenMP FP64 oracle (``lbm_oracle.cpp``).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).  The C++ oracle is a
second, independent implementation of the forward path (pull streaming with
velocity bounce-back, SRT / TRT / MRT / cumulant collisions, Guo forcing,
equilibrium initialisation, readout and shifted-storage rounding) written as
plain loops over cells; it runs on all host cores and serves the lattices the
numpy oracle is too slow for.  It is pinned against the numpy oracle and the
physical closed forms in ``tests/test_oracle_cpp.py``.

Arrays follow the numpy oracle: populations (Q, nz, ny, nx) unshifted FP64,
scalar fields (nz, ny, nx), vector fields (3, nz, ny, nx), masks uint8
(nz, ny, nx) with 0 = fluid; a force is None, (3,) or a per-row profile
(ny, 3); a wall-velocity table is (K, 3) indexed by the mask value.
"""

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbm_oracle.cpp")
LIB = os.path.join(HERE, "liblbm_oracle.so")
# the same source with long double for every value (x87 extended precision,
# 64-bit significand): measures the FP64 oracle's own rounding floor
LIB_LD = os.path.join(HERE, "liblbm_oracle_ld.so")
FLAGS = ["-std=c++17", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra"]

STENCIL = {"D2Q9": 0, "D3Q19": 1, "D3Q27": 2}
METHOD = {"SRT": 0, "TRT": 1, "MRT": 2, "CUMULANT": 3}
STORAGE = {"f64": 0, "f32": 1, "bf16": 2, "f16": 3}


def _config_type(R):
    class OrcConfig(ctypes.Structure):
        _fields_ = [("stencil", ctypes.c_int32), ("method", ctypes.c_int32), ("storage", ctypes.c_int32),
                    ("compressible", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                    ("nz", ctypes.c_int32), ("omega", R), ("omega_bulk", R), ("omega_odd", R), ("magic", R),
                    ("omega_hi", R * 4), ("rho0", R)]
    return OrcConfig


# ctypes struct and numpy element type per precision ("f64" or "ld")
CONFIG = {"f64": _config_type(ctypes.c_double), "ld": _config_type(ctypes.c_longdouble)}
REAL = {"f64": np.float64, "ld": np.longdouble}
OrcConfig = CONFIG["f64"]


def build_sanitized():
    """The FP64 oracle with AddressSanitizer and UndefinedBehaviorSanitizer
    (g++), for the host-sanitizer test; loaded in place of the plain build
    when LBM_ORACLE_LIB names it (with gcc's ASan runtime preloaded)."""
    out = os.path.join(HERE, "liblbm_oracle_san.so")
    subprocess.check_call(["g++", *FLAGS, "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=undefined", SRC, "-o", out])
    return out


def build(verbose=True):
    """Compile the oracle library (FP64, and the long double variant) with
    g++ and OpenMP; always recompiles."""
    for lib, extra in ((LIB, []), (LIB_LD, ["-DORC_REAL=long double"])):
        tmp = lib + ".tmp"
        subprocess.check_call(["g++", *FLAGS, *extra, SRC, "-o", tmp])
        os.replace(tmp, lib)
        if verbose:
            print("built", lib)
    return LIB


_libs = {}


def load(precision="f64"):
    """Load the oracle library of the given precision ("f64" or "ld"),
    building it first if it is not there."""
    if precision in _libs:
        return _libs[precision]
    path = {"f64": os.environ.get("LBM_ORACLE_LIB", LIB), "ld": LIB_LD}[precision]
    if not os.path.exists(path):
        build(verbose=False)
    lib = ctypes.CDLL(path)
    P, I32, I64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    C = ctypes.POINTER(CONFIG[precision])
    for name, args in {"orc_init": [C, P, P, P, P], "orc_run": [C, P, P, P, P, I32, I32],
                       "orc_readout": [C, P, P, P, P, P], "orc_conserved": [C, P, P, P],
                       "orc_collide_cells": [C, P, P, I64, P], "orc_mrt_basis": [C, P, P]}.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = I32
    lib.orc_num_threads.argtypes = []
    lib.orc_num_threads.restype = I32
    _libs[precision] = lib
    return lib


def num_threads():
    """Threads an OpenMP region of the oracle uses by default."""
    return int(load().orc_num_threads())


def _cfg(cfg, dims, precision="f64"):
    """Translate an ``oracle.run.Config`` and lattice dims into the C struct."""
    r = cfg.rates
    c = CONFIG[precision]()
    c.stencil = STENCIL[cfg.lat.name]
    c.method = METHOD[cfg.method]
    c.storage = STORAGE[cfg.storage]
    c.compressible = 1 if cfg.compressible else 0
    c.nx, c.ny, c.nz = (int(v) for v in dims)
    c.omega = float(r["omega"])
    c.omega_bulk = float(r.get("omega_bulk", 1.0))
    c.omega_odd = float(r.get("omega_odd", 0.0))
    c.magic = float(r.get("magic", 0.0))
    for i, v in enumerate(r.get("omega_hi", (1.0,) * 4)):
        c.omega_hi[i] = float(v)
    c.rho0 = float(cfg.rho0)
    return c


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _dims_of(arr):
    nz, ny, nx = arr.shape[-3:]
    return nx, ny, nz


def _mask(mask):
    return None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)


def _force(force, ny, precision="f64"):
    if force is None:
        return None
    F = np.asarray(force, dtype=REAL[precision])
    if F.shape == (3,):
        F = np.broadcast_to(F, (ny, 3))
    if F.shape != (ny, 3):
        raise ValueError("force must be (3,) or (ny, 3)")
    return np.ascontiguousarray(F)


def _walls(wall_velocity, precision="f64"):
    if wall_velocity is None:
        return None
    W = np.zeros((128, 3), dtype=REAL[precision])
    w = np.asarray(wall_velocity, dtype=np.float64)
    W[:w.shape[0]] = w
    return W


def _check(st, what):
    if st != 0:
        raise ValueError("C++ oracle %s failed (status %d)" % (what, st))


def init_equilibrium(cfg, rho, u, mask=None, precision="f64"):
    """P^0 = f^eq(rho, u) (Eq. 3) at fluid cells, w rho_0 at solid cells,
    rounded into the storage type.  rho may be None (rho_0 everywhere).
    ``precision`` "ld" computes in long double and returns np.longdouble."""
    R = REAL[precision]
    u = np.ascontiguousarray(u, dtype=R)
    dims = _dims_of(u)
    r = None if rho is None else np.ascontiguousarray(np.broadcast_to(rho, u.shape[1:]), dtype=R)
    P = np.empty((cfg.lat.Q,) + u.shape[1:], dtype=R)
    _check(load(precision).orc_init(ctypes.byref(_cfg(cfg, dims, precision)), _ptr(_mask(mask)), _ptr(r), _ptr(u),
                                    _ptr(P)), "init")
    return P


def run(cfg, P, nsteps, mask=None, force=None, wall_velocity=None, threads=0, precision="f64"):
    """``nsteps`` stream-pull-collide steps from P; returns the new state
    (P itself is not modified)."""
    P = np.array(P, dtype=REAL[precision], order="C", copy=True)
    dims = _dims_of(P)
    st = load(precision).orc_run(ctypes.byref(_cfg(cfg, dims, precision)), _ptr(_mask(mask)),
                                 _ptr(_force(force, dims[1], precision)), _ptr(_walls(wall_velocity, precision)),
                                 _ptr(P), int(nsteps), int(threads))
    _check(st, "run")
    return P


def readout(cfg, P, mask=None, force=None, precision="f64"):
    """rho, u of a stored post-collision state (solid cells read 0)."""
    R = REAL[precision]
    P = np.ascontiguousarray(P, dtype=R)
    dims = _dims_of(P)
    rho = np.empty(P.shape[1:], dtype=R)
    u = np.empty((3,) + P.shape[1:], dtype=R)
    st = load(precision).orc_readout(ctypes.byref(_cfg(cfg, dims, precision)), _ptr(_mask(mask)),
                                     _ptr(_force(force, dims[1], precision)), _ptr(P), _ptr(rho), _ptr(u))
    _check(st, "readout")
    return rho, u


def conserved(cfg, P, mask=None):
    """FP64 totals (sum rho, sum j) over fluid cells."""
    P = np.ascontiguousarray(P, dtype=np.float64)
    out = np.empty(4)
    _check(load().orc_conserved(ctypes.byref(_cfg(cfg, _dims_of(P))), _ptr(_mask(mask)), _ptr(P), _ptr(out)),
           "conserved")
    return out


def collide_cells(cfg, g, force=None):
    """One collision of independent cells: g (Q, n) -> (Q, n)."""
    g = np.asarray(g, dtype=np.float64)
    gc = np.ascontiguousarray(g.T)
    out = np.empty_like(gc)
    F = None if force is None else np.ascontiguousarray(force, dtype=np.float64).reshape(3)
    st = load().orc_collide_cells(ctypes.byref(_cfg(cfg, (1, 1, 1))), _ptr(gc), _ptr(F), g.shape[1], _ptr(out))
    _check(st, "collide")
    return out.T.copy()


def mrt_basis(cfg):
    """The C++ oracle's weighted-orthogonal basis (Q, Q) and per-row rates."""
    Q = cfg.lat.Q
    M = np.empty((Q, Q))
    s = np.empty(Q)
    _check(load().orc_mrt_basis(ctypes.byref(_cfg(cfg, (1, 1, 1))), _ptr(M), _ptr(s)), "mrt_basis")
    return M, s
