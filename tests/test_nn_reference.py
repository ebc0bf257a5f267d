"""Pins of the FP64 network reference (oracle/nn_reference.py): the periodic
convolution equals scipy's wrap-mode correlation; every backward formula
matches central finite differences of its forward."""
import numpy as np
import pytest
from scipy import ndimage

from oracle import nn_reference as R


def _rand(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


def test_conv3d_is_periodic_correlation():
    x = _rand((2, 5, 4, 6, 3), 1)
    w = _rand((4, 27, 3), 2)
    b = _rand(4, 3)
    y = R.conv3d(x, w, b)
    for n in range(2):
        for o in range(4):
            ref = b[o] + sum(
                ndimage.correlate(x[n, ..., i], w[o, :, i].reshape(3, 3, 3), mode="wrap")
                for i in range(3))
            assert np.allclose(y[n, ..., o], ref, atol=1e-12)


def _fd_check(f, x, g_analytic, eps=1e-6, n_probe=12, seed=0):
    rng = np.random.default_rng(seed)
    for _ in range(n_probe):
        idx = tuple(rng.integers(0, s) for s in x.shape)
        xp = x.copy()
        xm = x.copy()
        xp[idx] += eps
        xm[idx] -= eps
        fd = (f(xp) - f(xm)) / (2 * eps)
        assert abs(fd - g_analytic[idx]) < 1e-6 * max(1.0, abs(fd)), (idx, fd, g_analytic[idx])


def test_conv3d_backward_by_finite_differences():
    x = _rand((1, 4, 3, 5, 2), 4)
    w = _rand((3, 27, 2), 5)
    b = _rand(3, 6)
    dy = _rand((1, 4, 3, 5, 3), 7)
    dx, dw, db = R.conv3d_backward(x, w, dy)
    loss = lambda xx, ww, bb: float(np.sum(R.conv3d(xx, ww, bb) * dy))  # noqa: E731
    _fd_check(lambda xx: loss(xx, w, b), x, dx)
    _fd_check(lambda ww: loss(x, ww, b), w, dw)
    _fd_check(lambda bb: loss(x, w, bb), b, db)


def test_pool_and_upsample_adjoints():
    x = _rand((2, 4, 6, 2, 3), 8)
    dy = _rand((2, 2, 3, 1, 3), 9)
    assert np.isclose(np.sum(R.pool2(x) * dy), np.sum(x * R.pool2_backward(dy)))
    xc = _rand((1, 2, 3, 2, 2), 10)
    dyf = _rand((1, 4, 6, 4, 2), 11)
    assert np.isclose(np.sum(R.up2(xc) * dyf), np.sum(xc * R.up2_backward(dyf)))
    # pooling averages each 2x2x2 block
    assert np.isclose(R.pool2(x)[1, 1, 2, 0, 2], x[1, 2:4, 4:6, 0:2, 2].mean())


@pytest.mark.parametrize("v", [1.0, 1.00390625, 1.005859375, -3.14159, 1e-30, 65504.0])
def test_bf16_rounding(v):
    r = R.bf16(np.array([v]))[0]
    # 8 significant bits: r is within half a unit in the last place
    if v != 0:
        e = np.floor(np.log2(abs(v)))
        assert abs(r - v) <= 2.0 ** (e - 8) + 1e-300
    assert R.bf16(np.array([r]))[0] == r
