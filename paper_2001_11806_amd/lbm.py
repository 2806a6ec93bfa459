"""ctypes binding of the HIP library (``include/lbm.h``).

Argument marshalling only: every step of the method runs in the library's
kernels.  Torch supplies device memory for caller-side fields and the HIP
stream the library enqueues on.  If the shared library is missing the import
of this module still works, but creating an ``LBM`` raises: there is no CPU
fallback.
"""

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("LBM_MI355X_LIB", os.path.join(_HERE, "liblbm_mi355x.so"))

STENCILS = {"D2Q9": 0, "D3Q19": 1, "D3Q27": 2}
QS = {"D2Q9": 9, "D3Q19": 19, "D3Q27": 27}
METHODS = {"SRT": 0, "TRT": 1, "MRT": 2, "CUMULANT": 3, "KBC": 4}
DTYPES = {"f64": 0, "f32": 1, "bf16": 2, "f16": 3}
STORAGE_BYTES = {"f64": 8, "f32": 4, "bf16": 2, "f16": 2}

OK, EINVAL, EUNSUPPORTED, ENOMEM, EHIP, ESTATE, ENONFINITE = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "LBM_OK", -1: "LBM_EINVAL", -2: "LBM_EUNSUPPORTED", -3: "LBM_ENOMEM",
                -4: "LBM_EHIP", -5: "LBM_ESTATE", -6: "LBM_ENONFINITE"}


class Rates(ctypes.Structure):
    _fields_ = [("omega", ctypes.c_double), ("omega_bulk", ctypes.c_double),
                ("omega_odd", ctypes.c_double), ("magic", ctypes.c_double),
                ("omega_hi", ctypes.c_double * 4), ("cs_smag", ctypes.c_double)]


class Config(ctypes.Structure):
    _fields_ = [("stencil", ctypes.c_int32), ("method", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("rates", Rates), ("rho0", ctypes.c_double), ("compressible", ctypes.c_int32),
                ("pattern", ctypes.c_int32), ("checkpoint_every", ctypes.c_int32),
                ("max_tape_steps", ctypes.c_int32), ("launch_mode", ctypes.c_int32)]


_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_DP = ctypes.POINTER(ctypes.c_double)

SIGNATURES = {
    "lbm_create": ([ctypes.POINTER(Config), _P, _P, ctypes.POINTER(_P)], _I32),
    "lbm_destroy": ([_P], _I32),
    "lbm_set_force": ([_P, _DP, _DP], _I32),
    "lbm_set_wall_velocity": ([_P, _I32, _DP], _I32),
    "lbm_init_equilibrium": ([_P, _P, _P, _I32], _I32),
    "lbm_step": ([_P, _I32], _I32),
    "lbm_get_macroscopic": ([_P, _P, _P, _I32], _I32),
    "lbm_conserved": ([_P, _DP], _I32),
    "lbm_get_pdfs": ([_P, _P], _I32),
    "lbm_set_pdfs": ([_P, _P], _I32),
    "lbm_get_time": ([_P, ctypes.POINTER(_I64)], _I32),
    "lbm_adjoint_seed": ([_P, _P, _P, _I32], _I32),
    "lbm_adjoint_step": ([_P, _I32], _I32),
    "lbm_adjoint_grads": ([_P, _P, _P, _I32, _DP], _I32),
    "lbm_conserved_noalloc": ([_P, _P], _I32),
    "lbm_copy_q": ([_P, _P, _I64, _I32, _I32, _I32, _I32, _P], _I32),
    "lbm_stream_q": ([_P, _P, _I32, _I32, _I32, _I32, _I32, _I32, _I32, _P], _I32),
    "lbm_stream_aa_q": ([_P, _I32, _I32, _I32, _I32, _I32, _I32, _I32, _I32, _P], _I32),
    "lbm_last_error": ([], ctypes.c_char_p),
    "lbm_version": ([], _I32),
}

_lib = None


def load_library(path=None):
    """Load the shared library once; raise if it has not been built."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError("HIP library %s not found: build it with `python -m paper_2001_11806_amd.build` "
                           "(there is no CPU fallback)" % p)
    lib = ctypes.CDLL(p)
    for name, (args, res) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    if path is None:
        _lib = lib
    return lib


class LBMError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


def _check(status):
    if status != OK:
        raise LBMError(status, _lib.lbm_last_error().decode())


def make_config(stencil, method, dtype, dims, omega, omega_bulk=1.0, omega_odd=0.0, magic=0.0,
                omega_hi=(1.0, 1.0, 1.0, 1.0), rho0=1.0, compressible=True, pattern=0,
                checkpoint_every=0, max_tape_steps=0, launch_mode=0, cs_smag=0.0):
    nx, ny, nz = dims
    cfg = Config()
    cfg.stencil = STENCILS[stencil]
    cfg.method = METHODS[method]
    cfg.dtype = DTYPES[dtype]
    cfg.nx, cfg.ny, cfg.nz = int(nx), int(ny), int(nz)
    cfg.rates.omega = float(omega)
    cfg.rates.omega_bulk = float(omega_bulk)
    cfg.rates.omega_odd = float(omega_odd)
    cfg.rates.magic = float(magic)
    for i in range(4):
        cfg.rates.omega_hi[i] = float(omega_hi[i])
    cfg.rates.cs_smag = float(cs_smag)
    cfg.rho0 = float(rho0)
    cfg.compressible = 1 if compressible else 0
    cfg.pattern = int(pattern)
    cfg.checkpoint_every = int(checkpoint_every)
    cfg.max_tape_steps = int(max_tape_steps)
    cfg.launch_mode = int(launch_mode)
    return cfg


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class LBM:
    """One lattice on one GPU.

    dims = (nx, ny, nz); mask: numpy uint8 array (nz, ny, nx), 1 = solid.
    Fields use torch tensors on ``device``: scalars (nz, ny, nx), vectors
    (3, nz, ny, nx), PDFs (Q, nz, ny, nx).
    """

    def __init__(self, stencil, method, dtype, dims, omega, omega_bulk=1.0, omega_odd=0.0, magic=0.0,
                 omega_hi=(1.0, 1.0, 1.0, 1.0), rho0=1.0, compressible=True, mask=None,
                 checkpoint_every=0, max_tape_steps=0, device="cuda:0", stream=None, pattern=0,
                 launch_mode=0, cs_smag=0.0):
        import torch
        self.torch = torch
        self.lib = load_library()
        self.device = torch.device(device)
        self.stencil, self.method, self.dtype = stencil, method, dtype
        self.dims = tuple(int(d) for d in dims)
        self.Q = QS[stencil]
        self.N = self.dims[0] * self.dims[1] * self.dims[2]
        self.cfg = make_config(stencil, method, dtype, dims, omega, omega_bulk, omega_odd, magic, omega_hi,
                               rho0, compressible, pattern, checkpoint_every, max_tape_steps, launch_mode,
                               cs_smag)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        mptr = None
        self._mask = None
        if mask is not None:
            m = np.ascontiguousarray(mask, dtype=np.uint8)
            if m.size != self.N:
                raise ValueError("mask has %d cells, lattice has %d" % (m.size, self.N))
            self._mask = m
            mptr = m.ctypes.data_as(ctypes.c_void_p)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(self.lib.lbm_create(ctypes.byref(self.cfg), mptr, ctypes.c_void_p(stream.cuda_stream),
                                       ctypes.byref(h)))
        self.h = h
        # bumped by every call that changes the forward trajectory, so that a
        # pending autograd graph can tell whether the lattice still holds it
        self.generation = 0

    # ------------------------------------------------------------ helpers
    def _shape3(self):
        nx, ny, nz = self.dims
        return (nz, ny, nx)

    def _call(self, fn, *args):
        """Run an asynchronous library call that reads or writes torch tensors.
        The lattice's stream first waits for torch's current stream (whose
        work made the inputs), and the current stream then waits for the
        lattice's stream, so that no input is freed and reused, and no output
        read, before the call has run.  Nothing to do when they are one stream."""
        cur = self.torch.cuda.current_stream(self.device)
        same = cur == self.stream
        if not same:
            self.stream.wait_stream(cur)
        _check(fn(*args))
        if not same:
            cur.wait_stream(self.stream)

    def _field(self, t, comps, what):
        torch = self.torch
        if t is None:
            return None, None
        if not isinstance(t, torch.Tensor):
            t = torch.as_tensor(np.asarray(t))
        if t.dtype not in (torch.float64, torch.float32):
            t = t.to(torch.float64)
        t = t.to(self.device).contiguous()
        if t.numel() != comps * self.N:
            raise ValueError("%s has %d values, expected %d" % (what, t.numel(), comps * self.N))
        return t, (0 if t.dtype == torch.float64 else 1)

    def close(self):
        if getattr(self, "h", None):
            self.lib.lbm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ API
    def set_force(self, F=None, profile=None):
        self.generation += 1
        if F is not None:
            arr = (ctypes.c_double * 3)(*[float(v) for v in np.asarray(F, dtype=np.float64).reshape(3)])
            _check(self.lib.lbm_set_force(self.h, arr, None))
        elif profile is not None:
            prof = np.ascontiguousarray(profile, dtype=np.float64).reshape(-1)
            if prof.size != 3 * self.dims[1]:
                raise ValueError("profile must have ny*3 values")
            _check(self.lib.lbm_set_force(self.h, None, prof.ctypes.data_as(_DP)))
        else:
            _check(self.lib.lbm_set_force(self.h, None, None))

    def set_wall_velocity(self, wall_type, u):
        self.generation += 1
        arr = (ctypes.c_double * 3)(*[float(v) for v in np.asarray(u, dtype=np.float64).reshape(3)])
        _check(self.lib.lbm_set_wall_velocity(self.h, int(wall_type), arr))

    def init_equilibrium(self, rho=None, u=None):
        self.generation += 1
        r, dr = self._field(rho, 1, "rho")
        v, dv = self._field(u, 3, "u")
        dt = dr if dr is not None else (dv if dv is not None else 0)
        if r is not None and v is not None and r.dtype != v.dtype:
            r = r.to(v.dtype)
            dt = dv
        self._call(self.lib.lbm_init_equilibrium, self.h, _ptr(r), _ptr(v), dt)

    def step(self, n=1):
        self.generation += 1
        _check(self.lib.lbm_step(self.h, int(n)))

    @property
    def time(self):
        t = ctypes.c_int64()
        _check(self.lib.lbm_get_time(self.h, ctypes.byref(t)))
        return t.value

    def macroscopic(self, dtype=None):
        torch = self.torch
        dtype = dtype or torch.float64
        rho = torch.empty(self._shape3(), dtype=dtype, device=self.device)
        u = torch.empty((3,) + self._shape3(), dtype=dtype, device=self.device)
        self._call(self.lib.lbm_get_macroscopic, self.h, _ptr(rho), _ptr(u), 0 if dtype == torch.float64 else 1)
        return rho, u

    def conserved(self):
        out = (ctypes.c_double * 4)()
        _check(self.lib.lbm_conserved(self.h, out))
        return np.array(list(out))

    def conserved_noalloc(self, out):
        """Enqueue the totals of ``conserved`` into ``out`` (4 float64 on the
        lattice's device) without allocating; no synchronisation."""
        torch = self.torch
        if out.dtype != torch.float64 or out.numel() < 4 or not out.is_contiguous() or out.device != self.device:
            raise ValueError("out must be a contiguous float64 tensor of >= 4 elements on " + str(self.device))
        self._call(self.lib.lbm_conserved_noalloc, self.h, _ptr(out))
        return out

    def get_pdfs(self):
        torch = self.torch
        P = torch.empty((self.Q,) + self._shape3(), dtype=torch.float64, device=self.device)
        self._call(self.lib.lbm_get_pdfs, self.h, _ptr(P))
        return P

    def set_pdfs(self, P):
        self.generation += 1
        P, _ = self._field(P, self.Q, "pdfs")
        P = P.to(self.torch.float64).contiguous()
        self._call(self.lib.lbm_set_pdfs, self.h, _ptr(P))

    # ------------------------------------------------------------ adjoint
    def adjoint_seed(self, dL_du, dL_drho=None):
        g, dt = self._field(dL_du, 3, "dL_du")
        r, _ = self._field(dL_drho, 1, "dL_drho")
        if r is not None:
            r = r.to(g.dtype)
        self._call(self.lib.lbm_adjoint_seed, self.h, _ptr(r), _ptr(g), dt)

    def adjoint_step(self, n):
        _check(self.lib.lbm_adjoint_step(self.h, int(n)))

    def adjoint_grads(self, dtype=None, want_rho=False):
        torch = self.torch
        dtype = dtype or torch.float64
        du = torch.empty((3,) + self._shape3(), dtype=dtype, device=self.device)
        dr = torch.empty(self._shape3(), dtype=dtype, device=self.device) if want_rho else None
        dF = (ctypes.c_double * 3)()
        self._call(self.lib.lbm_adjoint_grads, self.h, _ptr(du), _ptr(dr), 0 if dtype == torch.float64 else 1, dF)
        return du, dr, np.array(list(dF))


def copy_q(src, dst, n, q, elem_bytes, stream, waves_per_cu=0, block_threads=0):
    """Q-stream copy bandwidth reference (see include/lbm.h); waves_per_cu
    0 = full occupancy, block_threads 0 = 256."""
    lib = load_library()
    _check(lib.lbm_copy_q(_ptr(src), _ptr(dst), int(n), int(q), int(elem_bytes), int(waves_per_cu),
                          int(block_threads), ctypes.c_void_p(stream.cuda_stream)))


def stream_q(src, dst, dims, stencil, elem_bytes, stream, waves_per_cu=0, block_threads=0):
    """Pull-streaming bandwidth reference (see include/lbm.h): dst[q][x] =
    src[q][x - c_q], periodic, in the sweep's launch shape; dims = (nx, ny,
    nz), block_threads 0 = the sweep's own row segmentation."""
    lib = load_library()
    nx, ny, nz = (int(d) for d in dims)
    _check(lib.lbm_stream_q(_ptr(src), _ptr(dst), nx, ny, nz, STENCILS[stencil], int(elem_bytes),
                            int(waves_per_cu), int(block_threads), ctypes.c_void_p(stream.cuda_stream)))


def stream_aa_q(buf, dims, stencil, elem_bytes, phase, stream, waves_per_cu=0, block_threads=0):
    """AA-pattern bandwidth reference (see include/lbm.h), in place on buf:
    phase 0 inverts every cell's slots, phase 1 moves A[opp q][x - c_q] to
    A[q][x + c_q]; dims = (nx, ny, nz)."""
    lib = load_library()
    nx, ny, nz = (int(d) for d in dims)
    _check(lib.lbm_stream_aa_q(_ptr(buf), nx, ny, nz, STENCILS[stencil], int(elem_bytes), int(phase),
                               int(waves_per_cu), int(block_threads), ctypes.c_void_p(stream.cuda_stream)))
