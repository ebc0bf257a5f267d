"""The learned warm start end to end at a small size: training fields from the
batch solver, a small U-Net trained by the library's kernels, and held-out
packs run to a 1e-8 residual from rest and from the network's prediction.
The warm start must need fewer steps and reach the same permeability."""
import numpy as np
import pytest

from paper_1508_02960_amd import inputs
from paper_1508_02960_amd import warmstart as W
from paper_1508_02960_amd import warmstart_study as S

pytestmark = pytest.mark.gpu

EDGE = 32


@pytest.fixture(scope="module")
def trained():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    packs = S.draw_packs(48, EDGE, 11, S.TRAIN_SPHERES)
    t, fluid, res = S.solve_stokes(packs, EDGE, tau=1.0, delta_rho=1e-5, tol=1e-6,
                                   max_steps=40000)
    ok = np.array([s == "converged" for s in res["status"]])
    assert ok.sum() >= 40, res["status"]
    net = W.UNet(widths=(16, 32, 32, 64), seed=1, device="cuda")
    f = torch.from_numpy(fluid[ok].astype(np.uint8)).cuda()
    tg = torch.from_numpy(t[ok]).cuda()
    hist = S.train(net, f, tg, epochs=20, minibatch=4, lr=3e-3, val_frac=0.1, log=print)
    return net, hist


def test_training_lowers_held_out_error(trained):
    _, hist = trained
    assert hist[-1]["val_rel_u"] < 0.5 * hist[0]["val_rel_u"] or hist[-1]["val_rel_u"] < 0.3
    assert hist[-1]["loss"] < hist[0]["loss"]


def _steps_to(traj, level, chunk):
    """Steps after which |U/U* - 1| stays below level, per cell."""
    out = []
    for col in np.asarray(traj).T:
        above = np.nonzero(col >= level)[0]
        out.append((above[-1] + 2 if len(above) else 1) * chunk)
    return np.array(out)


def test_warm_start_gains_over_rest(trained):
    net, _ = trained
    packs = S.draw_packs(8, EDGE, 12, S.TRAIN_SPHERES)
    res = S.evaluate(net, packs, EDGE, tau=0.8, delta_rho=1e-5, tol=1e-8, max_steps=100000,
                     log=print, chunk=100, n_chunks=40)
    for k in ("network_u", "converged_fields"):
        print(k, {q: res[k][q] for q in ("step_ratio_median", "total_step_ratio",
                                         "max_rel_K_diff")})
    print("network error u", np.median(res["network_rel_error_u"]), "U",
          np.abs(res["network_rel_error_U"]))
    rest = res["rest"]["trajectory_rel_error"]
    warm = res["network_u"]["trajectory_rel_error"]
    s_rest = _steps_to(rest, 1e-3, 100)
    s_warm = _steps_to(warm, 1e-3, 100)
    print("steps to 1e-3 of U*: rest", s_rest, "warm", s_warm)
    assert all(s == "converged" for s in res["rest"]["status"])
    assert all(s == "converged" for s in res["network_u"]["status"])
    # the plain iteration decides K: the same permeability from either start
    assert res["network_u"]["max_rel_K_diff"] <= 1e-3
    # the prediction starts much closer to the steady mean flow ...
    assert np.median(np.array(warm[0]) / np.array(rest[0])) < 0.3
    # ... and reaches 0.1 % of it in fewer steps
    assert np.median(s_warm / s_rest) < 1.0


def test_prolongate2_kernel_matches_host():
    """nn_prolongate2 (two batch entries, the first 4 of 8 channels, a channel
    scale) against warmstart.prolongate2, whose linear exactness and length
    scaling the host tests pin."""
    import torch

    lib = W._nn()
    ctx = W._Ctx("cuda")
    rng = np.random.default_rng(21)
    n, d, h, w, cx, c = 2, 4, 6, 8, 8, 4
    x = rng.standard_normal((n, d, h, w, cx)).astype(np.float32)
    xd = torch.from_numpy(x).to(ctx.dev)
    y = ctx.f32(n, 2 * d, 2 * h, 2 * w, c)
    scale = torch.tensor([4.0, 4.0, 4.0, 2.0], dtype=torch.float32, device=ctx.dev)
    assert lib.nn_prolongate2(W._p(xd), W._p(y), n, d, h, w, cx, c, W._p(scale), ctx.stream) == 0
    got = y.cpu().numpy()
    for b in range(n):
        want = W.prolongate2(x[b, ..., :c])
        assert np.max(np.abs(got[b] - want)) <= 1e-6 * np.max(np.abs(want))
    y1 = ctx.f32(n, 2 * d, 2 * h, 2 * w, 1)
    assert lib.nn_prolongate2(W._p(xd), W._p(y1), n, d, h, w, cx, 1, None, ctx.stream) == 0
    want1 = W.prolongate2(x[0, ..., :4])[..., 0] / 4.0
    assert np.max(np.abs(y1.cpu().numpy()[0, ..., 0] - want1)) <= 1e-6 * np.max(np.abs(want1))
    assert lib.nn_prolongate2(W._p(xd), W._p(y), n, d, h, w, cx, cx + 1, None, ctx.stream) != 0


def test_two_grid_prediction_on_the_device(trained):
    """predict_two_grid (network and prolongation on the device) equals the
    host composition prolongate2(predict(coarse_fluid)) to FP32 rounding."""
    net = trained[0] if isinstance(trained, tuple) else trained
    sp = S.draw_packs(1, 32, 9, (8, 12))[0][0]
    got = W.predict_two_grid(net, sp, 32)
    want = W.prolongate2(net.predict(W.coarse_fluid(sp, 32)))
    assert got.shape == want.shape == (32, 32, 32, 4)
    assert np.max(np.abs(got - want)) <= 1e-5 * np.max(np.abs(want))


def test_warm_start_fields_kernel_matches_host():
    """nn_warm_start_fields (two periodic packs, a ragged box, 4 target
    channels of which the velocity uses 3) against warmstart.warm_fields:
    the linear density on fluid nodes and the scaled predicted velocity away
    from the wall layer, bit for bit (the same FP64 products)."""
    import torch

    ctx = W._Ctx("cuda")
    rng = np.random.default_rng(23)
    shape = (2, 6, 9, 11)
    fluid = np.stack([inputs.random_mask(shape[1:], 0.05, seed=60 + i) == 0
                      for i in range(shape[0])])
    assert 0 < fluid.mean() < 1
    t = rng.standard_normal(shape + (4,)).astype(np.float32)
    delta_rho, tau = 3e-3, 0.8
    fields = W.warm_fields_device(ctx, torch.from_numpy(t).to(ctx.dev), fluid, delta_rho, tau)
    got = fields.cpu().numpy().reshape((4,) + shape)
    assert 0 < np.count_nonzero(got[1]) < fluid.sum()  # some nodes away from walls, not all
    for b in range(shape[0]):
        drho, u = W.warm_fields(t[b], delta_rho, tau, fluid[b])
        assert np.array_equal(got[0, b], drho)
        assert np.array_equal(got[1:, b], u)
    with pytest.raises(ValueError):
        W.warm_fields_device(ctx, torch.from_numpy(t[:1]).to(ctx.dev), fluid, delta_rho, tau)
