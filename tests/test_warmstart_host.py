"""Host-side pieces of the warm-start study: pack fitting, percolation and the
target units, checked without a GPU."""
import numpy as np
import pytest

from paper_1508_02960_amd import inputs, lbm
from paper_1508_02960_amd import warmstart as W
from paper_1508_02960_amd import warmstart_study as S


@pytest.mark.parametrize("edge,n_range", [(32, (1, 4)), (48, (8, 27))])
def test_fitted_pack_hits_porosity_and_matches_library_mask(edge, n_range):
    draws = inputs.pack_draws(3, edge, n_range, S.POROSITY)
    for _ in range(3):
        dr = next(draws)
        spheres, fluid = S.fit_pack(dr, edge)
        assert abs(fluid.mean() - dr["porosity"]) <= 1.0 / fluid.size + 1e-12
        d = lbm.Domain((edge,) * 3, tau=0.8, spheres=spheres, bind=False)
        lib_fluid = d.mask() == 0
        d.close()
        # the library's strict-inside rule gives the same nodes (up to ties)
        assert np.mean(lib_fluid != fluid) < 1e-4


def test_percolation():
    f = np.ones((6, 6, 6), bool)
    f[:, :, 3] = False  # a solid wall across x
    assert not W.percolates_x(f)
    f[2, 4, 3] = True   # one hole
    assert W.percolates_x(f)
    g = np.zeros((6, 6, 6), bool)
    g[0, 0, :] = True   # a single x channel
    assert W.percolates_x(g)
    # a channel that reaches x = nx-1 only through the periodic z face
    h = np.zeros((6, 6, 6), bool)
    h[5, 2, 0:3] = True
    h[0:5, 2, 2] = True
    h[0, 2, 2:6] = True
    assert W.percolates_x(h)


def test_target_units_round_trip():
    rng = np.random.default_rng(0)
    shape = (8, 6, 10)
    fluid = rng.uniform(size=shape) > 0.3
    drho = np.where(fluid, rng.normal(size=shape) * 1e-6, 0)
    u = np.where(fluid[None], rng.normal(size=(3,) + shape) * 1e-5, 0)
    # the density's fluid mean is lost in the round trip (t_p has zero mean)
    x = np.arange(10) - 4.5
    lin = -(2e-5 / 10) * x
    drho = np.where(fluid, drho - (drho - lin)[fluid].mean(), 0)
    t = W.fields_to_targets(drho, u, 2e-5, 0.9, fluid)
    d2, u2 = W.targets_to_fields(t, 2e-5, 0.9, fluid)
    assert np.allclose(d2, drho, atol=1e-12, rtol=1e-5)
    assert np.allclose(u2, u, atol=1e-14, rtol=1e-5)
    # a pure linear profile maps to t_p = 0, and Darcy scaling of u
    t = W.fields_to_targets(np.where(fluid, lin, 0), u, 2e-5, 0.9, fluid)
    assert np.max(np.abs(t[..., 3])) < 1e-9
    G = 2e-5 / 3 / 10
    nu = (0.9 - 0.5) / 3
    assert np.allclose(t[..., 0], np.where(fluid, u[0] * nu / G, 0), rtol=1e-6)


def test_coarse_fluid_is_the_pack_at_half_resolution():
    """Coarse node j sits at fine position 2j + 1/2 and is solid iff that
    point lies strictly inside a sphere or a periodic image (brute force)."""
    from paper_1508_02960_amd import warmstart as W

    rng = np.random.default_rng(3)
    edge = 16
    sp = np.hstack([rng.uniform(0, edge, (3, 3)), rng.uniform(1.5, 4.0, (3, 1))])
    got = W.coarse_fluid(sp, edge)
    ec = edge // 2
    want = np.ones((ec, ec, ec), bool)
    for z in range(ec):
        for y in range(ec):
            for x in range(ec):
                p = np.array([2 * x + 0.5, 2 * y + 0.5, 2 * z + 0.5])
                for cx, cy, cz, r in sp:
                    for o in np.ndindex(3, 3, 3):
                        c = np.array([cx, cy, cz]) + (np.array(o) - 1) * edge
                        if np.sum((p - c) ** 2) < r * r:
                            want[z, y, x] = False
    assert np.array_equal(got, want)


def test_prolongate2_interpolates_linear_fields_and_scales_lengths():
    """Trilinear interpolation at fine nodes (coarse coordinate (i - 1/2)/2)
    is exact for a field linear in each coordinate away from the periodic
    seam; velocity targets scale by 4 (length^2), density targets by 2."""
    from paper_1508_02960_amd import warmstart as W

    ec = 6
    z, y, x = np.meshgrid(np.arange(ec), np.arange(ec), np.arange(ec), indexing="ij")
    t = np.stack([x + 2.0 * y, 3.0 * z, np.ones_like(x, float), 1.0 * x - z], axis=-1)
    f = W.prolongate2(t)
    assert f.shape == (2 * ec, 2 * ec, 2 * ec, 4)
    fz, fy, fx = np.meshgrid(*(np.arange(2 * ec),) * 3, indexing="ij")
    cz, cy, cx = (fz - 0.5) / 2, (fy - 0.5) / 2, (fx - 0.5) / 2
    inner = (fz > 0) & (fz < 2 * ec - 1) & (fy > 0) & (fy < 2 * ec - 1) & (fx > 0) & (fx < 2 * ec - 1)
    want = np.stack([4 * (cx + 2 * cy), 4 * 3 * cz, 4 * np.ones_like(cx), 2 * (cx - cz)], axis=-1)
    assert np.allclose(f[inner], want[inner], atol=1e-5)
