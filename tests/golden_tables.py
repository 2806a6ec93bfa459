"""Reader for the hand-transcribed paper tables under tests/golden/."""
import os

import sympy as sp

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
x, y, rho, u0, u1 = sp.symbols("x y rho u0 u1")


def read_table(name):
    rows = []
    with open(os.path.join(HERE, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            a, b, c = [s.strip() for s in line.split("|")]
            rows.append((sp.sympify(a, locals={"x": x, "y": y}),
                         sp.sympify(b, locals={"rho": rho, "u0": u0, "u1": u1}), c))
    return rows
