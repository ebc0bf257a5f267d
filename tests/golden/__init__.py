"""Stored reference values for the tests, each file citing its source."""
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))


def load_drag_series(c: float) -> float:
    """F / (6 pi mu a U) of a simple-cubic sphere array at solid fraction c,
    from the truncated series in simple_cubic_drag.txt."""
    tab = np.loadtxt(os.path.join(_HERE, "simple_cubic_drag.txt"), comments="#")
    S = float(np.sum(tab[:, 1] * c ** tab[:, 0]))
    return 1.0 / S


def load_forchheimer_reference():
    """The oracle's three-point pressure-drop sweep of forchheimer_32cube.txt:
    dict with arrays re, delta_rho, U, steps and the fitted K_D and beta."""
    path = os.path.join(_HERE, "forchheimer_32cube.txt")
    tab = np.loadtxt(path, comments="#", ndmin=2)
    out = dict(re=tab[:, 0], delta_rho=tab[:, 1], U=tab[:, 2], steps=tab[:, 3].astype(int))
    for line in open(path):
        parts = line.split()
        if len(parts) == 3 and parts[0] == "#" and parts[1] in ("K_D", "beta"):
            out[parts[1]] = float(parts[2])
    return out
