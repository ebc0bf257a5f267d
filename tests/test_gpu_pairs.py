"""Two cells per lane (16-bit storage): step_pair_kernel against the one-cell
step kernel on the same domain (lbm_set_step_shape), bit for bit, and
against the FP64 oracle through the format tolerance of test_gpu_precision.

Both kernels round every cell with the same counter-based random word (cell
address and step seed), so their stored states must be identical.  The
partial sums of the residual checks add the cells in another order, so U
agrees to rounding only.
"""
import numpy as np
import pytest

from paper_1508_02960_amd import inputs, lbm

pytestmark = pytest.mark.gpu

STORAGES = ["fp16", "bf16", "fp16_rne", "bf16_rne"]


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    lbm.library()


def _pair_and_single(shape, storage, steps, *, residual_run=False, large=False, **kw):
    states, us = [], []
    rng = np.random.default_rng(5)
    if large:
        u0 = rng.uniform(-1e-3, 1e-3, size=(3,) + tuple(shape))
        drho0 = rng.uniform(-1e-3, 1e-3, size=tuple(shape))
    else:
        g0 = inputs.random_populations(shape, 1e-3, seed=5)
    for pairs in (True, False):
        d = lbm.Domain(shape, storage=storage, **kw)
        waves, rows, default_pairs = d.step_shape()
        # states beyond 1 GiB pair cells by default, smaller ones do not
        assert default_pairs == large
        d.set_step_shape(waves, rows, pairs)
        assert d.step_shape() == (waves, rows, pairs)
        if large:
            d.init_equilibrium(drho0, u0)
        else:
            d.set_state(g0)
        if residual_run:
            d.run_to_residual(0.0, steps)
            us.append(d.mean_velocity()[0])
        else:
            d.step(steps)
        # the large box: density and velocity fields (equal states give
        # equal fields; the small boxes compare the states themselves)
        states.append(np.concatenate([f.ravel() for f in d.macroscopic()]) if large
                      else d.get_state())
        d.close()
    return states, us


@pytest.mark.parametrize("storage", STORAGES)
@pytest.mark.parametrize("collision,wall", [("trt", "cli"), ("srt", "sbb"), ("mrt", "cli")])
def test_pair_kernel_equals_one_cell_kernel(storage, collision, wall):
    """64-wide rows (one tile per row, so the x wrap is at the DPP-row and
    tile edges), random spheres cutting many pairs, the periodic pressure
    jump, 5 steps."""
    shape = (7, 10, 64)
    kw = dict(tau=0.7, magic=0.21, delta_rho=3e-3, collision=collision, wall=wall,
              spheres=inputs.random_spheres(shape, 5, (1.5, 3.5), seed=41))
    (a, b), _ = _pair_and_single(shape, storage, 5, **kw)
    assert np.array_equal(a, b)


def test_pair_kernel_residual_checks():
    """run_to_residual (steps with the fused reductions) in both shapes: the
    same state, U within rounding of the FP64 sums."""
    shape = (9, 12, 128)
    kw = dict(tau=0.8, magic=3 / 16, delta_rho=1e-3, collision="trt", wall="cli",
              spheres=inputs.random_spheres(shape, 6, (2.0, 4.0), seed=42), check_interval=10)
    (a, b), (ua, ub) = _pair_and_single(shape, "fp16", 60, residual_run=True, **kw)
    assert np.array_equal(a, b)
    assert np.max(np.abs(np.asarray(ua) - np.asarray(ub))) <= 1e-12 * np.max(np.abs(ub))


def test_pair_kernel_large_state_tiles():
    """A state beyond 1 GiB uses 32 x 4 tiles (one per wavefront) and
    non-temporal stores; ny = 255 leaves a padding row in the last tile row.
    The one-cell kernel takes half a tile per wavefront there."""
    shape = (224, 255, 256)
    kw = dict(tau=0.6, magic=3 / 16, delta_rho=1e-3, collision="trt", wall="cli",
              spheres=inputs.random_spheres(shape, 40, (8.0, 30.0), seed=43))
    d = lbm.Domain(shape, storage="fp16", bind=False, **kw)
    assert (d.info.tile_width, d.info.tile_height) == (32, 4)
    d.close()
    (a, b), _ = _pair_and_single(shape, "fp16", 4, large=True, **kw)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("storage,wall", [("fp32", "cli"), ("fp64", "iebb"), ("fp16", "sbb")])
def test_workgroup_shapes_give_identical_states(storage, wall):
    """Every workgroup shape (wavefronts across x tile rows, one or two cells
    per lane) stores the same state bit for bit, through plain, graph and
    checked steps."""
    shape = (6, 24, 64)
    kw = dict(tau=0.75, magic=0.2, delta_rho=2e-3, collision="trt", wall=wall,
              spheres=inputs.random_spheres(shape, 4, (2.0, 4.0), seed=44), check_interval=20)
    g0 = inputs.random_populations(shape, 1e-3, seed=45)
    shapes = [(4, 1, False), (8, 2, False), (16, 8, False), (2, 2, False)]
    if storage == "fp16":
        shapes += [(2, 1, True), (8, 4, True)]
    states = []
    for waves, rows, pairs in shapes:
        d = lbm.Domain(shape, storage=storage, **kw)
        d.set_step_shape(waves, rows, pairs)
        d.set_state(g0)
        d.step(40)
        d.run_to_residual(0.0, 40)
        states.append(d.get_state())
        d.close()
    for s in states[1:]:
        assert np.array_equal(s, states[0])


def test_pair_shape_rejected_where_it_cannot_run():
    shape = (4, 6, 70)  # nx not a multiple of the 64-cell rows
    d = lbm.Domain(shape, tau=0.8, storage="fp16", mask=np.zeros(shape, np.uint8))
    assert d.step_shape()[2] is False
    with pytest.raises(lbm.LbmError):
        d.set_step_shape(4, 4, True)
    d.close()
    d = lbm.Domain((4, 6, 64), tau=0.8, storage="fp16", mask=np.zeros((4, 6, 64), np.uint8))
    d.set_step_shape(2, 2, True)
    assert d.step_shape() == (2, 2, True)
    d.close()
    d = lbm.Domain((4, 6, 64), tau=0.8, storage="fp32", mask=np.zeros((4, 6, 64), np.uint8))
    with pytest.raises(lbm.LbmError):
        d.set_step_shape(4, 4, True)  # pairs need 16-bit storage
    with pytest.raises(lbm.LbmError):
        d.set_step_shape(3, 1, False)  # waves not a power of two
    with pytest.raises(lbm.LbmError):
        d.set_step_shape(4, 3, False)  # rows must divide waves
    d.close()


def test_pair_kernel_matches_oracle_on_large_state_tiles(orc):
    """One step of a state beyond 1 GiB (32 x 4 tiles, a padding row in the
    last tile row, streaming stores) from the state the GPU holds, against
    the FP64 oracle: within one spacing of the format plus half a spacing of
    the stored CLI coefficient, as on the small boxes."""
    spacing = 2.0 ** -10
    shape = (256, 250, 224)
    sp = inputs.random_spheres(shape, 30, (8.0, 24.0), seed=49)
    kw = dict(tau=0.7, magic=0.21, delta_rho=3e-3, collision="trt", wall="cli", spheres=sp)
    d = lbm.Domain(shape, storage="fp16", **kw)
    assert (d.info.tile_width, d.info.tile_height) == (32, 4) and d.step_shape()[2]
    d.set_state(inputs.random_populations(shape, 1e-3, seed=50))
    g_held = d.get_state()
    o = orc.Oracle(shape, **kw)
    o.set_state(g_held)
    del g_held
    o.step(1)
    d.step(1)
    fluid = o.mask == 0
    got = d.get_state()
    r = float(np.max(np.abs(got[..., fluid] - o.g[..., fluid])) / np.max(np.abs(o.g[..., fluid])))
    assert r < 2 * spacing + 1e-5, r
    d.close()


def test_one_cell_kernel_on_large_state_without_pairs(orc):
    """A 16-bit state beyond 1 GiB whose nx (200) is not a multiple of the
    32-cell tiles: one cell per lane on 32 x 2 tiles with a padded last
    tile per row and streaming stores; one step against the FP64 oracle."""
    spacing = 2.0 ** -10
    shape = (280, 256, 200)
    sp = inputs.random_spheres(shape, 30, (8.0, 24.0), seed=51)
    kw = dict(tau=0.7, magic=0.21, delta_rho=3e-3, collision="trt", wall="cli", spheres=sp)
    d = lbm.Domain(shape, storage="fp16", **kw)
    assert (d.info.tile_width, d.info.tile_height) == (32, 2) and not d.step_shape()[2]
    d.set_state(inputs.random_populations(shape, 1e-3, seed=52))
    g_held = d.get_state()
    o = orc.Oracle(shape, **kw)
    o.set_state(g_held)
    del g_held
    o.step(1)
    d.step(1)
    fluid = o.mask == 0
    got = d.get_state()
    r = float(np.max(np.abs(got[..., fluid] - o.g[..., fluid])) / np.max(np.abs(o.g[..., fluid])))
    assert r < 2 * spacing + 1e-5, r
    d.close()


@pytest.mark.parametrize("storage", ["fp16", "bf16"])
def test_pair_kernel_matches_oracle(orc, storage):
    """One step of the pair kernel from the state the GPU holds, stepped by
    the FP64 oracle: within one spacing of the format plus half a spacing of
    the stored CLI coefficient (as for the one-cell kernel)."""
    spacing = {"fp16": 2.0 ** -10, "bf16": 2.0 ** -7}[storage]
    shape = (9, 13, 64)
    sp = inputs.random_spheres(shape, 6, (1.5, 4.0), seed=21)
    kw = dict(tau=0.7, magic=0.21, delta_rho=3e-3, collision="trt", wall="cli", spheres=sp)
    d = lbm.Domain(shape, storage=storage, **kw)
    d.set_step_shape(4, 4, True)
    d.set_state(inputs.random_populations(shape, 1e-3, seed=22))
    g_held = d.get_state()
    o = orc.Oracle(shape, **kw)
    o.set_state(g_held)
    o.step(1)
    d.step(1)
    fluid = o.mask == 0
    got, ref = d.get_state()[..., fluid], o.g[..., fluid]
    r = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
    assert r < 2 * spacing + 1e-5, r
    d.close()
