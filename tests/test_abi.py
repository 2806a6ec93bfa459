"""C ABI checks that need no GPU: the built library loads, exports every
function ``include/lbm.h`` declares, its config struct layout matches the C
compiler's, and argument validation rejects bad requests before any device
work."""

import ctypes
import os
import re
import subprocess
import tempfile

import pytest

from paper_2001_11806_amd import lbm as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_0-9]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(B.LIB_PATH):
        pytest.fail("library not built: run __graft_entry__.build()")
    return B.load_library()


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(B.SIGNATURES), "binding and header disagree"


def test_config_layout_matches_c(tmp_path):
    src = tmp_path / "layout.c"
    src.write_text('#include <stddef.h>\n#include <stdio.h>\n#include "lbm.h"\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu\\n", sizeof(lbm_config), '
                   'offsetof(lbm_config, rates), offsetof(lbm_config, rho0), '
                   'offsetof(lbm_config, checkpoint_every), sizeof(lbm_rates));return 0;}\n')
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    want = [ctypes.sizeof(B.Config), B.Config.rates.offset, B.Config.rho0.offset,
            B.Config.checkpoint_every.offset, ctypes.sizeof(B.Rates)]
    assert got == want


def _create(lib, **kw):
    args = dict(stencil="D3Q19", method="SRT", dtype="f64", dims=(8, 8, 8), omega=1.2)
    args.update(kw)
    cfg = B.make_config(**args)
    h = ctypes.c_void_p()
    st = lib.lbm_create(ctypes.byref(cfg), None, None, ctypes.byref(h))
    return st, lib.lbm_last_error().decode()


@pytest.mark.parametrize("kw,code,msg", [
    (dict(omega=2.0), B.EINVAL, "omega"),
    (dict(omega=0.0), B.EINVAL, "omega"),
    (dict(omega=float("nan")), B.EINVAL, "omega"),
    (dict(dims=(0, 8, 8)), B.EINVAL, "dims"),
    (dict(dims=(2048, 2048, 1024)), B.EINVAL, "2^31"),
    (dict(stencil="D2Q9", dims=(8, 8, 2)), B.EINVAL, "nz"),
    (dict(rho0=-1.0), B.EINVAL, "rho0"),
    (dict(method="TRT", magic=0.0, omega_odd=0.0), B.EINVAL, "TRT"),
    (dict(method="TRT", omega_odd=2.5), B.EINVAL, "omega_odd"),
    (dict(method="MRT", omega_bulk=2.2), B.EINVAL, "omega_bulk"),
    (dict(method="MRT", stencil="D3Q27", omega_hi=(1, 1, 2.0, 1)), B.EINVAL, "omega_hi"),
    (dict(method="MRT", omega_hi=(1, 2.5, 1, 1)), B.EINVAL, "omega_hi[1]"),
    (dict(method="CUMULANT"), B.EUNSUPPORTED, "not implemented"),
    (dict(method="CUMULANT", stencil="D3Q27", omega_hi=(1, 2.2, 1, 1)), B.EINVAL, "omega_hi[1]"),
    (dict(method="CUMULANT", stencil="D3Q27", compressible=False), B.EUNSUPPORTED, "compressible"),
    (dict(method="KBC", omega_bulk=2.5), B.EINVAL, "omega_bulk"),
    (dict(method="KBC", cs_smag=0.1), B.EUNSUPPORTED, "Smagorinsky"),
    (dict(method="KBC", checkpoint_every=2, max_tape_steps=4), B.EUNSUPPORTED, "adjoint"),
    (dict(pattern=2), B.EINVAL, "pattern"),
    (dict(pattern=1, method="CUMULANT", stencil="D3Q27", checkpoint_every=5, max_tape_steps=10), B.EUNSUPPORTED,
     "adjoint"),
    (dict(launch_mode=3), B.EINVAL, "launch_mode"),
    (dict(cs_smag=-0.1), B.EINVAL, "cs_smag"),
    (dict(method="TRT", magic=3 / 16, cs_smag=0.1), B.EUNSUPPORTED, "Smagorinsky"),
    (dict(cs_smag=0.1, checkpoint_every=2, max_tape_steps=4), B.EUNSUPPORTED, "Smagorinsky"),
    (dict(method="KBC", omega_bulk=1.2, checkpoint_every=5, max_tape_steps=10), B.EUNSUPPORTED, "adjoint"),
    (dict(checkpoint_every=5, max_tape_steps=0), B.EINVAL, "max_tape_steps"),
    (dict(checkpoint_every=-1), B.EINVAL, "checkpoint_every"),
])
def test_validation_before_device_work(lib, kw, code, msg):
    st, err = _create(lib, **kw)
    assert st == code, err
    assert msg in err


def test_null_arguments(lib):
    assert lib.lbm_step(None, 1) == B.EINVAL
    assert lib.lbm_destroy(None) == B.OK
    assert lib.lbm_copy_q(None, None, 10, 19, 8, 0, 0, None) == B.EINVAL
    fake = ctypes.c_void_p(4096)        # never dereferenced: validation comes first
    assert lib.lbm_copy_q(fake, fake, 10, 19, 8, 33, 0, None) == B.EINVAL
    assert lib.lbm_copy_q(fake, fake, 10, 19, 8, -1, 0, None) == B.EINVAL
    assert lib.lbm_copy_q(fake, fake, 10, 19, 3, 0, 0, None) == B.EINVAL
    assert lib.lbm_copy_q(fake, fake, 10, 19, 8, 0, 96, None) == B.EINVAL
    assert lib.lbm_copy_q(fake, fake, 10, 19, 8, 0, 1024, None) == B.EINVAL
    assert lib.lbm_stream_q(None, fake, 8, 8, 8, 1, 8, 0, 0, None) == B.EINVAL
    assert lib.lbm_stream_q(fake, fake, 8, 8, 8, 3, 8, 0, 0, None) == B.EINVAL      # stencil
    assert lib.lbm_stream_q(fake, fake, 0, 8, 8, 1, 8, 0, 0, None) == B.EINVAL      # dims
    assert lib.lbm_stream_q(fake, fake, 2048, 2048, 512, 1, 8, 0, 0, None) == B.EINVAL   # 2^31 cells
    assert lib.lbm_stream_q(fake, fake, 8, 8, 2, 0, 8, 0, 0, None) == B.EINVAL      # D2Q9, nz != 1
    assert lib.lbm_stream_q(fake, fake, 8, 8, 8, 1, 1, 0, 0, None) == B.EINVAL      # elem_bytes
    assert lib.lbm_stream_q(fake, fake, 8, 8, 8, 1, 8, 33, 0, None) == B.EINVAL     # waves
    assert lib.lbm_stream_q(fake, fake, 8, 8, 8, 1, 8, 0, 100, None) == B.EINVAL    # block
    assert lib.lbm_stream_q(fake, fake, 8, 8, 8, 1, 8, 0, 576, None) == B.EINVAL
    assert lib.lbm_stream_aa_q(None, 8, 8, 8, 1, 8, 0, 0, 0, None) == B.EINVAL
    assert lib.lbm_stream_aa_q(fake, 8, 8, 8, 1, 8, 2, 0, 0, None) == B.EINVAL     # phase
    assert lib.lbm_stream_aa_q(fake, 8, 8, 8, 1, 8, -1, 0, 0, None) == B.EINVAL
    assert lib.lbm_stream_aa_q(fake, 8, 8, 8, 4, 8, 0, 0, 0, None) == B.EINVAL     # stencil
    assert lib.lbm_stream_aa_q(fake, 8, 0, 8, 1, 8, 0, 0, 0, None) == B.EINVAL     # dims
    assert lib.lbm_stream_aa_q(fake, 2048, 2048, 512, 1, 8, 0, 0, 0, None) == B.EINVAL
    assert lib.lbm_stream_aa_q(fake, 8, 8, 3, 0, 8, 0, 0, 0, None) == B.EINVAL     # D2Q9, nz != 1
    assert lib.lbm_stream_aa_q(fake, 8, 8, 8, 1, 6, 0, 0, 0, None) == B.EINVAL     # elem_bytes
    assert lib.lbm_stream_aa_q(fake, 8, 8, 8, 1, 8, 0, 40, 0, None) == B.EINVAL    # waves
    assert lib.lbm_stream_aa_q(fake, 8, 8, 8, 1, 8, 0, 0, 65, None) == B.EINVAL    # block
    assert lib.lbm_create(None, None, None, None) == B.EINVAL
    assert lib.lbm_version() >= 10000


def test_no_cpu_fallback_when_library_missing(tmp_path):
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        B.load_library(str(tmp_path / "missing.so"))
