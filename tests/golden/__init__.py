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
