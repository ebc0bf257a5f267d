"""Writes forchheimer_32cube.txt: the FP64 oracle's steady superficial
velocities of a three-point pressure-drop sweep on one simple-cubic cell, and
their Forchheimer fit (eq. (Forchheimer)), the reference of the reduced-precision
sweep test.  Calls only the oracle.

    python tests/golden/make_forchheimer_reference.py

Cell: 32^3 with a centred sphere of diameter 20, TRT (Lambda = 3/16, tau =
0.8), CLI walls.  Pressure drops from the Darcy estimate for Re_p = 0.01, 3 and
15 with a permeability guess of 40: delta_rho = 3 nx nu^2 Re / (D K)
(U = Re nu / D, grad p = nu U / K, dp = delta_rho / 3).  Each run starts at
rest and stops when the relative change of U over 100 steps stays below
1e-10 three times in a row.  Fit: grad p / U = nu / K_D + beta U by least
squares with grad p = delta_rho / (3 nx).
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402

EDGE, D, TAU, MAGIC = 32, 20.0, 0.8, 3 / 16
RE = (0.01, 3.0, 15.0)
K_GUESS = 40.0


def main() -> None:
    oracle.build(force=False)
    oracle.set_threads(os.cpu_count() or 1)
    nu = (TAU - 0.5) / 3
    shape = (EDGE,) * 3
    c = (EDGE - 1) / 2.0
    sphere = np.array([[c, c, c, D / 2]])
    rows = []
    for re in RE:
        drho = 3 * EDGE * nu * nu * re / (D * K_GUESS)
        o = oracle.Oracle(shape, tau=TAU, magic=MAGIC, delta_rho=drho, collision="trt",
                          wall="cli", spheres=sphere)
        o.init()
        st, n, res = o.run_to_residual(1e-10, 400000, interval=100)
        assert st == "converged", (re, st, n)
        U = float(o.mean_velocity()[0])
        rows.append((re, drho, U, n))
        print(f"Re {re}: delta_rho {drho!r} U {U!r} after {n} steps", flush=True)
    g = np.array([r[1] / (3 * EDGE) for r in rows])
    U = np.array([r[2] for r in rows])
    A = np.stack([np.ones_like(U), U], axis=1)
    (a, b), *_ = np.linalg.lstsq(A, g / U, rcond=None)
    K, beta = float(nu / a), float(b)
    with open(os.path.join(HERE, "forchheimer_32cube.txt"), "w") as f:
        f.write("# FP64 oracle, 32^3 cell, centred sphere D = 20, TRT Lambda = 3/16, tau = 0.8,\n")
        f.write("# CLI walls, each run from rest to a 1e-10 residual (written by\n")
        f.write("# make_forchheimer_reference.py, which calls only the oracle).\n")
        f.write(f"# fit of eq. (Forchheimer): K_D = {K!r} beta = {beta!r}\n")
        f.write("# re_target delta_rho U steps\n")
        for r in rows:
            f.write(f"{r[0]!r} {r[1]!r} {r[2]!r} {r[3]}\n")
        f.write(f"# K_D {K!r}\n# beta {beta!r}\n")


if __name__ == "__main__":
    main()
