"""Plain FP64 CPU oracle for the lattice Boltzmann stream-collide method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code, tables or
constants with the HIP library; the only thing both sides consume is the
seeded synthetic input generator (``paper_2001_11806_amd/inputs.py``), which
holds none of the method's arithmetic.

Everything here is written for clarity, not speed: numpy arrays over whole
lattices or over lists of cells (or plain loops over cells in the C++
oracle), float64 throughout, with the method's steps in the order the paper
states them.

Module map
----------
lattice      velocity sets DdQq, weights, opposite directions    (Sec. III-A)
equilibrium  density/velocity (Eq. 2), discrete equilibrium (Eq. 3),
             Guo forcing source, truncated Maxwellian moments (Eqs. 7-8)
moments      monomial moment bases, shear/bulk split, weighted
             Gram-Schmidt (Sec. III-A "Moment Space", III-C "MRT")
collision    SRT (Eq. 1), TRT (Sec. III-C), MRT (Eq. 4),
             cumulant (Eq. 9, Sec. III-B), Smagorinsky (Eqs. 11-14),
             entropic KBC (Sec. III-C "Entropic KBC Models")
stream       pull streaming, halfway bounce-back (Sec. IV-B, Fig. stream-pull)
run          initialisation, time stepping, readout, storage rounding
adjoint      tangent-linear and discrete-adjoint maps of the SRT / TRT / MRT +
             Guo + bounce-back time step (not in the paper; derived by hand
             from the forward map)
cpu          ctypes binding of lbm_oracle.cpp: a second, independent forward
             oracle in plain C++17 loops with OpenMP over lattice rows (all
             host cores), for lattices the numpy code is too slow for

Functions without an independent pin say "parity unpinned" in their
docstring.  All functions listed above are pinned by ``tests/test_oracle_*.py``.
"""

from . import lattice, equilibrium, moments, collision, stream, run, adjoint  # noqa: F401
