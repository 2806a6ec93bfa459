"""Write ``c3_storage_floor.txt``: the storage-only error of shifted FP32 /
FP16 / BF16 PDF storage on the D3Q27 cumulant workload, from the oracle alone.

The C++ oracle runs the workload twice per storage type: plain FP64, and
FP64 arithmetic with every stored value P - w rho_0 rounded to nearest-even
in the storage type after each step.  The relative L2 distance of the two
readouts is the error that the storage rounding alone causes; an FP32-storage
kernel whose error is far above it is limited by its arithmetic, not by its
storage.

Workload: the cumulant collision of Eq. (9) with every higher-order rate and
the bulk rate 1, shear rate 1/0.55; the divergence-free Fourier field of the
384^3 benchmark (32 seeded modes, max |u| 0.05 on 384^3) sampled on a 48^3
periodic box; rho = 1.  Run from the repository root:

    python tests/golden/c3_storage_floor.py
"""

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import cpu, run as orun  # noqa: E402
from paper_2001_11806_amd import inputs  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c3_storage_floor.txt")
N = 48
TIMES = (100, 200, 500)
RATES = dict(omega=1 / 0.55, omega_bulk=1.0, omega_hi=(1.0,) * 4)


def trajectory(storage, u):
    cfg = orun.Config("D3Q27", "CUMULANT", RATES, storage=storage)
    P = cpu.init_equilibrium(cfg, None, u)
    out, t = {}, 0
    for T in TIMES:
        P = cpu.run(cfg, P, T - t)
        t = T
        out[T] = cpu.readout(cfg, P)
    return out


def main():
    u = inputs.solenoidal_velocity(N, inputs.solenoidal_modes(seed=3))
    t0 = time.time()
    ref = trajectory("f64", u)
    lines = ["# storage-only error of shifted storage, D3Q27 cumulant (unit higher-order and bulk rates,",
             "# shear rate 1/0.55), 48^3 sample of the 384^3 solenoidal field; C++ FP64 oracle with",
             "# emulated round-to-nearest-even storage vs plain FP64.  Written by c3_storage_floor.py.",
             "# storage steps rel_l2_u rel_l2_rho_minus_1"]
    for storage in ("f32", "f16", "bf16"):
        got = trajectory(storage, u)
        for T in TIMES:
            r0, u0 = ref[T]
            r1, u1 = got[T]
            eu = np.linalg.norm(u1 - u0) / np.linalg.norm(u0)
            er = np.linalg.norm(r1 - r0) / np.linalg.norm(r0 - 1)
            lines.append("%s %d %.3e %.3e" % (storage, T, eu, er))
            print(lines[-1], flush=True)
    with open(OUT, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("wrote %s (%.0f s, %d threads)" % (OUT, time.time() - t0, cpu.num_threads()))


def read_floor():
    """{(storage, steps): (rel_l2_u, rel_l2_rho_minus_1)} from the stored file."""
    out = {}
    with open(OUT) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            s, T, eu, er = line.split()
            out[(s, int(T))] = (float(eu), float(er))
    return out


if __name__ == "__main__":
    main()
