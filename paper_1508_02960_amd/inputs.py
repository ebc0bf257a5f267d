"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module only draws numbers and lays out sphere packs; it contains none of
the lattice Boltzmann arithmetic.  Every generator takes an explicit seed.
Spheres are rows ``(cx, cy, cz, r)`` in lattice units, node ``(x, y, z)``
sitting at position ``(x, y, z)``; shapes are ``(nz, ny, nx)``.
"""
from __future__ import annotations

import numpy as np


def centred_sphere(shape, diameter: float) -> np.ndarray:
    """One sphere at the centre of the box (simple-cubic unit cell)."""
    nz, ny, nx = shape
    return np.array([[(nx - 1) / 2.0, (ny - 1) / 2.0, (nz - 1) / 2.0, diameter / 2.0]])


def simple_cubic_array(cells_per_axis: int, cell: int, diameter: float) -> np.ndarray:
    """A (cells_per_axis)^3 block of simple-cubic unit cells of edge `cell`,
    each with one sphere at its centre."""
    out = []
    c0 = (cell - 1) / 2.0
    for iz in range(cells_per_axis):
        for iy in range(cells_per_axis):
            for ix in range(cells_per_axis):
                out.append([c0 + ix * cell, c0 + iy * cell, c0 + iz * cell, diameter / 2.0])
    return np.array(out)


def random_spheres(shape, n: int, r_range, seed: int) -> np.ndarray:
    """n spheres with uniform random centres in the box and radii in r_range."""
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    c = rng.uniform(0.0, 1.0, size=(n, 3)) * np.array([nx, ny, nz])
    r = rng.uniform(r_range[0], r_range[1], size=(n, 1))
    return np.hstack([c, r])


def random_mask(shape, solid_fraction: float, seed: int) -> np.ndarray:
    """Independent Bernoulli solid nodes (uint8, 1 = solid)."""
    rng = np.random.default_rng(seed)
    return (rng.uniform(size=shape) < solid_fraction).astype(np.uint8)


def random_populations(shape, scale: float, seed: int) -> np.ndarray:
    """Random deviation populations g[19, nz, ny, nx], uniform in [-scale, scale]."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-scale, scale, size=(19,) + tuple(shape))


def random_velocity(shape, amplitude: float, seed: int) -> np.ndarray:
    """Velocity field u[3, nz, ny, nx] with i.i.d. components in [-amplitude, amplitude]."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-amplitude, amplitude, size=(3,) + tuple(shape))


def batch_cell_draws(seed: int, edge: int = 64):
    """Endless seeded draws for one-sphere cells: diameter U[40, 60] (scaled
    by edge / 64), centre U[0, edge)^3, tau U[0.55, 1.0], log10 Re_p
    U[-3, log10 300].  The caller decides which draws to keep."""
    rng = np.random.default_rng(seed)
    s = edge / 64.0
    while True:
        d = rng.uniform(40.0, 60.0) * s
        c = rng.uniform(0.0, 1.0, size=3) * edge
        tau = rng.uniform(0.55, 1.0)
        log_re = rng.uniform(-3.0, np.log10(300.0))
        yield dict(diameter=d, centre=c, tau=tau, re_p=10.0 ** log_re)


def pack_draws(seed: int, edge: int, n_range, phi_range):
    """Endless seeded draws for random packs of overlapping spheres of one
    common radius: sphere count U{n_range}, centres U[0, edge)^3, target
    porosity U[phi_range].  The caller fits the radius to the porosity."""
    rng = np.random.default_rng(seed)
    while True:
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        c = rng.uniform(0.0, float(edge), size=(n, 3))
        phi = rng.uniform(phi_range[0], phi_range[1])
        yield dict(centres=c, porosity=phi)
