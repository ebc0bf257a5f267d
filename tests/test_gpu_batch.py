"""Batches of independent cells (one launch per step, per-cell parameters,
device-side convergence) against the oracle run cell by cell."""
import numpy as np
import pytest

from paper_1508_02960_amd import inputs, lbm

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    lbm.library()


CELL = (12, 10, 14)


def _cells(n, seed, drho_scale=1e-3):
    rng = np.random.default_rng(seed)
    out = []
    for b in range(n):
        sp = inputs.random_spheres(CELL, int(rng.integers(1, 4)), (1.5, 3.5), seed=seed * 100 + b)
        out.append(dict(spheres=sp, tau=float(rng.uniform(0.6, 1.2)),
                        magic=float(rng.uniform(0.1, 0.3)),
                        delta_rho=float(rng.uniform(-1, 1) * drho_scale)))
    return out


def _oracle(orc, c, wall="cli", collision="trt"):
    return orc.Oracle(CELL, tau=c["tau"], magic=c["magic"], delta_rho=c["delta_rho"],
                      collision=collision, wall=wall, spheres=c["spheres"])


@pytest.mark.parametrize("collision,wall", [("srt", "cli"), ("trt", "cli"), ("mrt", "cli"),
                                            ("trt", "libb"), ("trt", "qibb"), ("mrt", "iebb"),
                                            ("trt", "mr")])
def test_batch_steps_match_cells(orc, collision, wall):
    """Each cell of a batch evolves exactly as the same cell alone (FP64):
    per-cell parameters, z wrap inside the cell, wall coefficients."""
    cells = _cells(4, seed=1)
    b = lbm.Batch(CELL, cells, collision=collision, wall=wall, storage="fp64")
    assert np.array_equal(b.mask()[2], orc.voxelise(CELL, cells[2]["spheres"]))
    g0 = inputs.random_populations((4,) + CELL, 1e-3, seed=2)
    b.set_state(g0)
    b.step(5)
    g = b.get_state()
    for i, c in enumerate(cells):
        o = _oracle(orc, c, collision=collision, wall=wall)
        o.set_state(g0[:, i])
        o.step(5)
        fluid = o.mask == 0
        err = np.max(np.abs(g[:, i][:, fluid] - o.g[:, fluid])) / np.max(np.abs(o.g[:, fluid]))
        assert err < 1e-12, (i, err)
    b.close()


def test_batch_run_to_residual_per_cell(orc):
    """Device-side convergence: every cell stops at its own check, with the
    oracle's step count and permeability (FP64); the frozen cells keep their
    final state while the others continue."""
    cells = _cells(3, seed=3, drho_scale=1e-5)
    for c in cells:
        c["delta_rho"] = abs(c["delta_rho"]) + 1e-6
    b = lbm.Batch(CELL, cells, wall="cli", storage="fp64", check_interval=50)
    st, steps, res = b.run_to_residual(1e-9, 100000)
    assert st == "converged"
    r = b.results()
    g = b.get_state()
    assert len(set(r["steps"].tolist())) > 1  # cells stopped at different checks
    for i, c in enumerate(cells):
        o = _oracle(orc, c)
        o.init()
        so, no, _ = o.run_to_residual(1e-9, 100000, interval=50)
        assert so == "converged" and r["status"][i] == "converged"
        assert r["steps"][i] == no
        assert abs(r["K_D"][i] / o.permeability() - 1) < 1e-10
        fluid = o.mask == 0
        err = np.max(np.abs(g[:, i][:, fluid] - o.g[:, fluid])) / np.max(np.abs(o.g[:, fluid]))
        assert err < 1e-10
    b.close()


def test_batch_run_shrinks_to_running_cells():
    """As cells stop, a run launches blocks for the running cells only (the
    device-side list of running cells, graphs sized to the next power of two
    at or above their count): every cell's status, stopping step and final
    state equal those of the same cell run alone, bit for bit, also for cells
    listed behind stopped ones."""
    shape = (16, 16, 16)
    rng = np.random.default_rng(12)
    cells = [dict(spheres=inputs.random_spheres(shape, 2, (2.0, 4.0), seed=120 + i),
                  tau=float(t), magic=3 / 16, delta_rho=float(rng.uniform(0.5, 1.5) * 1e-5))
             for i, t in enumerate([1.5, 0.7, 1.2, 0.9, 1.4, 0.8])]
    b = lbm.Batch(shape, cells, wall="cli", storage="fp64", check_interval=20)
    b.run_to_residual(1e-6, 20000)
    r = b.results()
    g = b.get_state()
    b.close()
    assert len(set(r["steps"].tolist())) >= 4
    for i, c in enumerate(cells):
        b1 = lbm.Batch(shape, [c], wall="cli", storage="fp64", check_interval=20)
        b1.run_to_residual(1e-6, 20000)
        r1 = b1.results()
        assert r1["status"][0] == r["status"][i] and r1["steps"][0] == r["steps"][i], i
        assert np.array_equal(b1.get_state()[:, 0], g[:, i]), i
        b1.close()


def test_batch_residual_with_largest_workgroups(orc):
    """Regression test of the per-block FP64 reduction at the largest batch
    workgroup (16 wavefronts, 1024 threads, every wavefront holding fluid
    cells): per-cell stopping steps equal the oracle's and K_D agrees to
    1e-10 (FP64), as with the default shape."""
    shape = (4, 32, 32)  # 16 tiles of 8 x 8 per plane: one plane per workgroup
    rng = np.random.default_rng(11)
    cells = []
    for i in range(3):
        sp = inputs.random_spheres(shape, 3, (3.0, 5.0), seed=110 + i)
        sp[:, 3] = np.minimum(sp[:, 3], 3.9)  # radii below the smallest edge
        cells.append(dict(spheres=sp, tau=float(rng.uniform(1.0, 1.3)), magic=3 / 16,
                          delta_rho=float(rng.uniform(0.5, 1.5) * 1e-6)))
    b = lbm.Batch(shape, cells, wall="cli", storage="fp64", check_interval=50)
    b.set_shape(16, 2)
    st, _, _ = b.run_to_residual(1e-7, 60000)
    assert st == "converged"
    r = b.results()
    for i, c in enumerate(cells):
        o = orc.Oracle(shape, tau=c["tau"], magic=c["magic"], delta_rho=c["delta_rho"],
                       collision="trt", wall="cli", spheres=c["spheres"])
        o.init()
        so, no, _ = o.run_to_residual(1e-7, 60000, interval=50)
        assert so == "converged" and r["status"][i] == "converged"
        assert r["steps"][i] == no, (i, r["steps"][i], no)
        assert abs(r["K_D"][i] / o.permeability() - 1) < 1e-10
    b.close()


def test_batch_shapes_give_identical_bits():
    """The launch shape and solid-write mode chosen by the autotuner change
    scheduling only."""
    shape = (16, 10, 14)
    cells = [dict(spheres=inputs.random_spheres(shape, 2, (1.5, 3.0), seed=40 + i),
                  tau=0.6 + 0.2 * i, magic=0.2, delta_rho=1e-3 * (i + 1)) for i in range(3)]
    u0 = inputs.random_velocity((3 * 16, 10, 14), 1e-2, seed=5)
    outs = []
    for by, zp, mode in [(1, 1, 0), (4, 2, 0), (2, 4, 0), (1, 1, 1), (2, 4, 2)]:
        b = lbm.Batch(shape, cells, wall="cli", storage="fp32", check_interval=10)
        b.set_shape(by, zp)
        b.set_solid_writes(mode)
        b.init_equilibrium(u0=u0)
        b.step(20)
        st, _, _ = b.run_to_residual(1e-30, 30)
        outs.append((b.get_state(), b.results()["U"]))
        b.close()
    for g, U in outs[1:]:
        assert np.array_equal(outs[0][0], g) and np.array_equal(outs[0][1], U)


@pytest.mark.parametrize("storage,wall", [("fp64", "cli"), ("fp32", "mr"), ("fp32", "sbb"),
                                          ("fp64", "libb")])
def test_batch_solid_write_modes_give_identical_bits(storage, wall):
    """Rows of 64 cells (one wavefront) cut by spheres: every solid-write
    mode gives the same state, through CLI and MR also the same wall-link
    slots."""
    shape = (8, 12, 64)
    cells = [dict(spheres=inputs.random_spheres(shape, 3, (3.0, 6.0), seed=70 + i), tau=0.7,
                  delta_rho=1e-3) for i in range(2)]
    u0 = inputs.random_velocity((2 * 8, 12, 64), 1e-2, seed=7)
    outs = []
    for mode in (0, 1, 2):
        b = lbm.Batch(shape, cells, wall=wall, storage=storage)
        b.set_solid_writes(mode)
        b.init_equilibrium(u0=u0)
        b.step(15)
        outs.append(b.get_state())
        b.close()
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])


def test_batch_autotune_and_unstable_cell():
    """The autotuner returns an admissible shape and resets to rest; an
    unstable cell is flagged while the others converge."""
    cells = _cells(3, seed=6, drho_scale=1e-5)
    for c in cells:
        c["delta_rho"] = abs(c["delta_rho"]) + 1e-6
    cells[1].update(tau=0.5001, magic=0.25, delta_rho=0.5)
    b = lbm.Batch((16, 10, 14), [dict(c, spheres=inputs.random_spheres((16, 10, 14), 2, (1.5, 3.0), seed=60 + i))
                                 for i, c in enumerate(cells)], wall="cli", storage="fp32",
                  check_interval=20)
    by, zp, ms = b.autotune(steps=5)
    assert by >= 1 and 16 % zp == 0 and ms > 0 and b.solid_writes in (0, 1, 2)
    assert np.all(b.get_state() == 0)
    st, _, _ = b.run_to_residual(1e-7, 60000)
    r = b.results()
    assert st == "unstable"
    assert r["status"][1] == "unstable"
    assert r["status"][0] == "converged" and r["status"][2] == "converged"
    b.close()


def test_full_batch_configuration_sampled_cells(orc):
    """The full 256-cell batch of 64^3 cells (one sphere of D in [40, 60] at a
    random centre, tau in [0.55, 1], seed 4, as the batch study draws them),
    FP32 in 8 x 8 tiles (a state beyond 1 GiB), autotuned launch shape, 40
    steps from rest under per-cell pressure drops; sampled cells (first,
    middle, last) against the FP64 oracle run on that cell alone: velocity
    within 1e-5."""
    from paper_1508_02960_amd import batch_study

    draws, _ = batch_study.draw_cells(256, 4, 64)
    cells = [dict(spheres=c["spheres"], tau=c["tau"], magic=3 / 16,
                  delta_rho=1e-4 * (1 + (i % 7))) for i, c in enumerate(draws)]
    b = lbm.Batch((64, 64, 64), cells, wall="cli", storage="fp32")
    assert (b.info.tile_width, b.info.tile_height) == (8, 8)
    b.autotune(steps=3)
    b.init_equilibrium()
    b.step(40)
    _, u = b.macroscopic()
    b.close()
    for i in (0, 127, 255):
        c = cells[i]
        o = orc.Oracle((64, 64, 64), tau=c["tau"], magic=c["magic"], delta_rho=c["delta_rho"],
                       collision="trt", wall="cli", spheres=c["spheres"])
        o.init()
        o.step(40)
        _, uo = o.macroscopic()
        fluid = o.mask == 0
        err = np.max(np.abs(u[:, i][:, fluid] - uo[:, fluid])) / np.max(np.abs(uo[:, fluid]))
        assert err < 1e-5, (i, err)


def test_batch_speed_mode():
    """batch_study.speed (the timing run behind the batch step's profile):
    two cells of the study at a fixed launch shape, every cell running."""
    from paper_1508_02960_amd import batch_study

    r = batch_study.speed(n_cells=2, edge=64, seed=4, steps=4, shape=(4, 1, 2), log=lambda s: None)
    assert (r["waves_per_block"], r["z_planes_per_block"], r["solid_writes"]) == (4, 1, 2)
    assert r["n_fluid"] > 0 and r["ms_per_step"] > 0 and r["mflups"] > 0
    r = batch_study.speed(n_cells=1, edge=128, steps=2, shape=(2, 1, 2), packs=True,
                          log=lambda s: None)
    assert r["n_fluid"] > 0 and r["tile"] == [64, 1]  # one pack: 0.3 GB, rows of 64


def test_fp64_batch_in_large_tiles_matches_oracle(orc):
    """An FP64 batch beyond 1 GiB (16 cells of 64^3 of the batch study, so
    8 x 8 tiles and streaming stores), 20 steps from a random state under
    per-cell pressure drops: the first and last cells against the FP64
    oracle run on that cell alone, within 1e-12 of the largest population."""
    from paper_1508_02960_amd import batch_study

    draws, _ = batch_study.draw_cells(16, 4, 64)
    cells = [dict(spheres=c["spheres"], tau=c["tau"], magic=3 / 16,
                  delta_rho=1e-4 * (1 + (i % 5))) for i, c in enumerate(draws)]
    b = lbm.Batch((64, 64, 64), cells, wall="cli", storage="fp64")
    assert (b.info.tile_width, b.info.tile_height) == (8, 8)
    g0 = inputs.random_populations((16, 64, 64, 64), 1e-3, seed=70)
    b.set_state(g0)
    b.step(20)
    g = b.get_state()
    b.close()
    for i in (0, 15):
        c = cells[i]
        o = orc.Oracle((64, 64, 64), tau=c["tau"], magic=c["magic"], delta_rho=c["delta_rho"],
                       collision="trt", wall="cli", spheres=c["spheres"])
        o.set_state(np.ascontiguousarray(g0[:, i]))
        o.step(20)
        fluid = o.mask == 0
        err = np.max(np.abs(g[:, i][:, fluid] - o.g[:, fluid])) / np.max(np.abs(o.g[:, fluid]))
        assert err < 1e-12, (i, err)
