"""Warm-start network kernels (BF16 MFMA convolutions and the layers around
them) against the FP64 reference of oracle/nn_reference.py.

Inputs are BF16 values, so products are exact in FP32 and the kernels differ
from the FP64 reference only by FP32 accumulation: 1e-5 relative.  The whole
network's gradients are compared with a CPU twin that rounds to BF16 at the
same points (activations, upstream gradients): 2e-3 relative.
"""
import numpy as np
import pytest

from oracle import nn_reference as R
from paper_1508_02960_amd import warmstart as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return W._Ctx("cuda")


def rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-30))


def _bf_dev(ctx, a):
    t = ctx.torch
    return t.from_numpy(np.ascontiguousarray(a, np.float32)).to(ctx.dev).to(t.bfloat16)


def _f_dev(ctx, a):
    t = ctx.torch
    return t.from_numpy(np.ascontiguousarray(a, np.float32)).to(ctx.dev)


def _host(t):
    return t.float().cpu().numpy().astype(np.float64)


SHAPES = [((2, 6, 4, 8), 8, 8), ((1, 4, 6, 4), 16, 24), ((1, 4, 4, 4), 32, 80),
          ((1, 8, 8, 8), 8, 16),
          # spatially tiled forward path (4 x 8 x 8 tiles, 32-channel chunks):
          # two batch entries, 64 output channels, a ragged channel tile, and 8
          # outputs (16-column tile, as in the head)
          ((2, 16, 32, 32), 32, 32), ((1, 16, 32, 64), 64, 64), ((1, 8, 32, 64), 96, 96),
          ((2, 16, 32, 32), 32, 8),
          # spatially tiled weight gradient (at least 256 tiles): two input
          # channel chunks, two output channel tiles, and 16-channel tiles with
          # zero padding (8 inputs as in the first layer, 8 outputs as in the
          # head, 24 outputs)
          ((2, 16, 32, 64), 64, 32), ((1, 32, 32, 64), 32, 64), ((2, 16, 32, 64), 8, 32),
          ((2, 16, 32, 64), 32, 8), ((1, 32, 32, 64), 16, 24)]


@pytest.mark.parametrize("shape,ci,co", SHAPES)
def test_conv_forward_backward_match_reference(ctx, shape, ci, co):
    rng = np.random.default_rng(ci * 7 + co)
    x = R.bf16(rng.standard_normal(shape + (ci,)))
    w = R.bf16(rng.standard_normal((co, 27, ci)) * 0.2)
    b = rng.standard_normal(co).astype(np.float32).astype(np.float64)
    dy = R.bf16(rng.standard_normal(shape + (co,)))
    lib = W._nn()
    n, d, h, wd = shape
    xd, wb, bd = _bf_dev(ctx, x), _bf_dev(ctx, w), _f_dev(ctx, b)
    y = ctx.f32(n, d, h, wd, co)
    assert lib.nn_conv3d_forward(W._p(xd), W._p(wb), W._p(bd), W._p(y), n, d, h, wd, ci, co,
                                 ctx.stream) == 0
    assert rel(_host(y), R.conv3d(x, w, b)) < 1e-5
    # the fused activation equals the two-step form bit for bit
    for relu in (1, 0):
        a_ref = ctx.bf(n, d, h, wd, co)
        assert lib.nn_activation_forward(W._p(y), W._p(a_ref), y.numel(), relu, ctx.stream) == 0
        a = ctx.bf(n, d, h, wd, co)
        assert lib.nn_conv3d_forward_act(W._p(xd), W._p(wb), W._p(bd), W._p(a), n, d, h, wd, ci,
                                         co, relu, ctx.stream) == 0
        assert ctx.torch.equal(a.view(ctx.torch.int16), a_ref.view(ctx.torch.int16)), relu
    dx_ref, dw_ref, db_ref = R.conv3d_backward(x, w, dy)
    if co % 8 == 0:
        wt = ctx.bf(ci, 27, co)
        assert lib.nn_conv3d_flip_weights(W._p(wb), W._p(wt), ci, co, ctx.stream) == 0
        dx = ctx.f32(n, d, h, wd, ci)
        assert lib.nn_conv3d_backward_data(W._p(_bf_dev(ctx, dy)), W._p(wt), W._p(dx), n, d, h,
                                           wd, ci, co, ctx.stream) == 0
        assert rel(_host(dx), dx_ref) < 1e-5
        import ctypes as C
        nb = C.c_size_t()
        sp = C.c_int()
        assert lib.nn_conv3d_backward_weight_workspace(n, d, h, wd, ci, co, C.byref(nb),
                                                       C.byref(sp)) == 0
        ws = ctx.torch.empty(nb.value, dtype=ctx.torch.uint8, device=ctx.dev)
        dw = ctx.f32(co, 27, ci)
        assert lib.nn_conv3d_backward_weight(W._p(xd), W._p(_bf_dev(ctx, dy)), W._p(dw), W._p(ws),
                                             nb.value, n, d, h, wd, ci, co, ctx.stream) == 0
        assert rel(_host(dw), dw_ref) < 1e-5
        db = ctx.f32(co)
        bb = C.c_size_t()
        assert lib.nn_bias_grad_workspace(n * d * h * wd, co, C.byref(bb)) == 0
        bws = ctx.torch.empty(bb.value, dtype=ctx.torch.uint8, device=ctx.dev)
        assert lib.nn_bias_grad(W._p(_f_dev(ctx, dy)), W._p(db), W._p(bws), bb.value,
                                n * d * h * wd, co, ctx.stream) == 0
        assert rel(_host(db), db_ref) < 1e-5


@pytest.mark.parametrize("c", [8, 6])
def test_pool_up_concat_split_relu(ctx, c):
    """c = 8: the 16-byte granule kernels; c = 6: the element kernels."""
    rng = np.random.default_rng(3)
    lib = W._nn()
    s = ctx.stream
    x = R.bf16(rng.standard_normal((2, 4, 6, 8, c)))
    y = ctx.bf(2, 2, 3, 4, c)
    assert lib.nn_pool2_forward(W._p(_bf_dev(ctx, x)), W._p(y), 2, 4, 6, 8, c, s) == 0
    assert rel(_host(y), R.bf16(R.pool2(x))) < 1e-6
    dy = rng.standard_normal((2, 2, 3, 4, c))
    dx = ctx.f32(2, 4, 6, 8, c)
    assert lib.nn_pool2_backward(W._p(_f_dev(ctx, dy)), W._p(dx), 2, 4, 6, 8, c, s) == 0
    assert rel(_host(dx), R.pool2_backward(dy)) < 1e-6
    xc = R.bf16(rng.standard_normal((1, 2, 3, 2, c)))
    yf = ctx.bf(1, 4, 6, 4, c)
    assert lib.nn_upsample2_forward(W._p(_bf_dev(ctx, xc)), W._p(yf), 1, 2, 3, 2, c, s) == 0
    assert np.array_equal(_host(yf), R.up2(xc))
    dyf = rng.standard_normal((1, 4, 6, 4, c))
    dxc = ctx.f32(1, 2, 3, 2, c)
    assert lib.nn_upsample2_backward(W._p(_f_dev(ctx, dyf)), W._p(dxc), 1, 2, 3, 2, c, s) == 0
    assert rel(_host(dxc), R.up2_backward(dyf)) < 1e-6
    a = R.bf16(rng.standard_normal((5, c)))
    b = R.bf16(rng.standard_normal((5, 2 * c)))
    cat = ctx.bf(5, 3 * c)
    assert lib.nn_concat_channels(W._p(_bf_dev(ctx, a)), W._p(_bf_dev(ctx, b)), W._p(cat), 5, c,
                                  2 * c, s) == 0
    assert np.array_equal(_host(cat), np.concatenate([a, b], axis=1))
    g = rng.standard_normal((5, 3 * c))
    ga, gb = ctx.f32(5, c), ctx.f32(5, 2 * c)
    assert lib.nn_split_channels(W._p(_f_dev(ctx, g)), W._p(ga), W._p(gb), 5, c, 2 * c, s) == 0
    assert rel(_host(ga), g[:, :c]) < 1e-7 and rel(_host(gb), g[:, c:]) < 1e-7
    ne = 1000 if c == 8 else 1001  # four-element and element kernels
    z = rng.standard_normal(ne)
    act = ctx.bf(ne)
    assert lib.nn_activation_forward(W._p(_f_dev(ctx, z)), W._p(act), ne, 1, s) == 0
    assert np.array_equal(_host(act), R.bf16(np.maximum(z, 0)))
    cst = ctx.bf(ne)
    assert lib.nn_cast_bf16(W._p(_f_dev(ctx, z)), W._p(cst), ne, s) == 0
    assert np.array_equal(_host(cst), R.bf16(z.astype(np.float32).astype(np.float64)))
    da = rng.standard_normal(ne)
    dz = ctx.f32(ne)
    assert lib.nn_relu_backward(W._p(_f_dev(ctx, da)), W._p(act), W._p(dz), ne, s) == 0
    assert np.allclose(_host(dz), np.where(R.bf16(np.maximum(z, 0)) > 0,
                                           da.astype(np.float32), 0))


@pytest.mark.parametrize("m,c", [(3000, 32), (777, 6), (513, 300)])
def test_relu_backward_bias_fused(ctx, m, c):
    """nn_relu_backward_bias equals nn_relu_backward, nn_cast_bf16 and
    nn_bias_grad bit for bit (c = 300: the wide-channel branch), with and
    without the ReLU; db also against the FP64 sum."""
    import ctypes as C

    t = ctx.torch
    rng = np.random.default_rng(m + c)
    lib = W._nn()
    s = ctx.stream
    da = _f_dev(ctx, rng.standard_normal((m, c)))
    act = _bf_dev(ctx, np.maximum(rng.standard_normal((m, c)), 0))
    bb = C.c_size_t()
    assert lib.nn_bias_grad_workspace(m, c, C.byref(bb)) == 0
    ws = t.empty(bb.value, dtype=t.uint8, device=ctx.dev)
    for relu in (1, 0):
        dz32 = ctx.f32(m, c)
        if relu:
            assert lib.nn_relu_backward(W._p(da), W._p(act), W._p(dz32), m * c, s) == 0
        else:
            dz32.copy_(da)
        dz_ref, db_ref = ctx.bf(m, c), ctx.f32(c)
        assert lib.nn_cast_bf16(W._p(dz32), W._p(dz_ref), m * c, s) == 0
        assert lib.nn_bias_grad(W._p(dz32), W._p(db_ref), W._p(ws), bb.value, m, c, s) == 0
        dz, db = ctx.bf(m, c), ctx.f32(c)
        assert lib.nn_relu_backward_bias(W._p(da), W._p(act) if relu else None, W._p(dz),
                                         W._p(db), W._p(ws), bb.value, m, c, relu, s) == 0
        assert t.equal(dz.view(t.int16), dz_ref.view(t.int16)), relu
        assert t.equal(db, db_ref), relu
        assert rel(_host(db), _host(dz32).sum(axis=0)) < 1e-5
    assert lib.nn_relu_backward_bias(W._p(da), None, W._p(dz), W._p(db), W._p(ws), bb.value,
                                     m, c, 1, s) == 1  # ReLU without the activation


def test_bias_grad_vector_and_scalar_accesses_agree(ctx):
    """Four channels per thread: 16-byte FP32 and 8-byte BF16 accesses when
    the pointers allow them, element accesses in the same order when they do
    not (here: every pointer one element off alignment).  dz and db of the
    fused and plain bias gradients are bit for bit the same either way."""
    import ctypes as C

    t = ctx.torch
    m, c = 2000, 32
    rng = np.random.default_rng(9)
    lib = W._nn()
    s = ctx.stream
    da_h = rng.standard_normal((m, c)).astype(np.float32)
    act_bits = _bf_dev(ctx, np.maximum(rng.standard_normal((m, c)), 0)).reshape(-1)
    bb = C.c_size_t()
    assert lib.nn_bias_grad_workspace(m, c, C.byref(bb)) == 0
    ws = t.empty(bb.value, dtype=t.uint8, device=ctx.dev)
    outs = []
    for off in (0, 1):
        da = t.zeros(m * c + 4, dtype=t.float32, device=ctx.dev)
        da[off:off + m * c] = t.from_numpy(da_h.reshape(-1)).to(ctx.dev)
        act = t.zeros(m * c + 4, dtype=act_bits.dtype, device=ctx.dev)
        act[off:off + m * c] = act_bits
        dz = t.zeros(m * c + 4, dtype=act_bits.dtype, device=ctx.dev)
        db, db_plain = ctx.f32(c), ctx.f32(c)
        pa, pact, pdz = (W._p(x[off:]) for x in (da, act, dz))
        assert lib.nn_relu_backward_bias(pa, pact, pdz, W._p(db), W._p(ws), bb.value, m, c, 1,
                                         s) == 0
        assert lib.nn_bias_grad(pa, W._p(db_plain), W._p(ws), bb.value, m, c, s) == 0
        t.cuda.synchronize()
        outs.append((dz[off:off + m * c].clone(), db.clone(), db_plain.clone()))
    (dz0, db0, dp0), (dz1, db1, dp1) = outs
    assert t.equal(dz0.view(t.int16), dz1.view(t.int16))
    assert t.equal(db0, db1) and t.equal(dp0, dp1)
    assert rel(_host(dp0), da_h.astype(np.float64).sum(axis=0)) < 1e-5


def test_mse_and_adam(ctx):
    rng = np.random.default_rng(4)
    lib = W._nn()
    m = 300
    pred = rng.standard_normal((m, 8)).astype(np.float32)
    tgt = rng.standard_normal((m, 3)).astype(np.float32)
    wgt = (rng.uniform(size=m) > 0.3).astype(np.float32)
    norm = 3.0 * wgt.sum()
    grad = ctx.f32(m, 8)
    part = ctx.torch.empty(64, dtype=ctx.torch.float64, device=ctx.dev)
    assert lib.nn_masked_mse(W._p(_f_dev(ctx, pred)), W._p(_f_dev(ctx, tgt)),
                             W._p(_f_dev(ctx, wgt)), W._p(grad), W._p(part), 64, m, 8, 3, norm,
                             ctx.stream) == 0
    d = pred[:, :3].astype(np.float64) - tgt
    loss = float(np.sum(d ** 2 * wgt[:, None]) / norm)
    assert abs(float(part.sum().item()) - loss) < 1e-6 * loss
    g_ref = np.zeros((m, 8))
    g_ref[:, :3] = 2 * d * wgt[:, None] / norm
    assert rel(_host(grad), g_ref) < 1e-6
    # Adam, two steps against the textbook update
    w = rng.standard_normal(50)
    gs = [rng.standard_normal(50), rng.standard_normal(50)]
    wd, m1, m2 = _f_dev(ctx, w), ctx.zeros(50), ctx.zeros(50)
    ref, a, b = w.copy(), np.zeros(50), np.zeros(50)
    for t, g in enumerate(gs, start=1):
        assert lib.nn_adam(W._p(wd), W._p(_f_dev(ctx, g)), W._p(m1), W._p(m2), None, 50, 1e-2,
                           0.9, 0.999, 1e-8, t, ctx.stream) == 0
        a = 0.9 * a + 0.1 * g
        b = 0.999 * b + 0.001 * g * g
        ref = ref - 1e-2 * (a / (1 - 0.9 ** t)) / (np.sqrt(b / (1 - 0.999 ** t)) + 1e-8)
    assert rel(_host(wd), ref) < 1e-5


def _cpu_unet(net, x, target, weight, norm):
    """CPU twin of UNet forward/backward in FP64 with BF16 rounding where the
    GPU stores BF16 (weights, activations, concatenations, gradients fed to
    the convolution backward)."""
    def wts(conv):
        return (R.bf16(conv.w.cpu().numpy().astype(np.float64)),
                conv.b.cpu().numpy().astype(np.float64))

    e, ins = [], []
    inp = x
    for lvl, conv in enumerate(net.enc):
        if lvl > 0:
            inp = R.bf16(R.pool2(inp))
        ins.append(inp)
        w, b = wts(conv)
        e.append(R.bf16(np.maximum(R.conv3d(inp, w, b), 0)))
        inp = e[-1]
    cur, cats, ds = e[3], {}, {}
    for j, conv in enumerate(net.dec):
        lvl = 2 - j
        cat = np.concatenate([R.up2(cur), e[lvl]], axis=-1)
        cats[lvl] = cat
        w, b = wts(conv)
        cur = R.bf16(np.maximum(R.conv3d(cat, w, b), 0))
        ds[lvl] = cur
    wh, bh = wts(net.head)
    out = R.conv3d(ds[0], wh, bh)
    d = out[..., :3] - target
    loss = np.sum(d ** 2 * weight[..., None]) / norm
    dout = np.zeros_like(out)
    dout[..., :3] = 2 * d * weight[..., None] / norm
    grads = {}
    g, grads["head"], _ = R.conv3d_backward(ds[0], wh, R.bf16(dout))
    skip = {}
    for lvl in (0, 1, 2):
        conv = net.dec[2 - lvl]
        dz = np.where(ds[lvl] > 0, g, 0)
        w, _ = wts(conv)
        dcat, grads[f"dec{lvl}"], _ = R.conv3d_backward(cats[lvl], w, R.bf16(dz))
        cc = net.widths[lvl + 1]
        skip[lvl] = dcat[..., cc:]
        g = R.up2_backward(dcat[..., :cc])
    for lvl in (3, 2, 1, 0):
        if lvl < 3:
            g = g + skip[lvl]
        dz = np.where(e[lvl] > 0, g, 0)
        w, _ = wts(net.enc[lvl])
        dinp, grads[f"enc{lvl}"], _ = R.conv3d_backward(ins[lvl], w, R.bf16(dz))
        if lvl > 0:
            g = R.pool2_backward(dinp)
    return out, loss, grads


def test_unet_gradients_match_cpu_twin(ctx):
    net = W.UNet(widths=(8, 8, 16, 16), seed=7, device="cuda")
    rng = np.random.default_rng(8)
    shape = (1, 16, 16, 16)
    fluid = (rng.uniform(size=shape) > 0.3).astype(np.float32)
    x_np = np.zeros(shape + (8,))
    x_np[..., 0] = fluid
    target = rng.standard_normal(shape + (3,)).astype(np.float32)
    norm = 3.0 * fluid.sum()
    out = net.forward(W.network_input(net.ctx, fluid))
    loss, dout = net.loss(out, _f_dev(ctx, target), _f_dev(ctx, fluid), norm)
    net.backward(dout)
    out_ref, loss_ref, g_ref = _cpu_unet(net, x_np, target.astype(np.float64),
                                         fluid.astype(np.float64), norm)
    assert rel(_host(out), out_ref) < 2e-3
    assert abs(loss / loss_ref - 1) < 2e-3
    assert rel(_host(net.head.gw), g_ref["head"]) < 2e-3
    for lvl in range(3):
        assert rel(_host(net.dec[2 - lvl].gw), g_ref[f"dec{lvl}"]) < 2e-3, lvl
    for lvl in range(4):
        assert rel(_host(net.enc[lvl].gw), g_ref[f"enc{lvl}"]) < 2e-3, lvl


def test_unet_training_reduces_loss(ctx):
    """Adam steps on a learnable target lower the loss.  The network is
    translation-equivariant, so the target is a local function of the mask:
    the fluid fraction of each voxel's 3x3x3 neighbourhood, on fluid voxels."""
    from scipy import ndimage

    net = W.UNet(widths=(8, 16, 16, 32), seed=9, device="cuda")
    rng = np.random.default_rng(10)
    shape = (2, 16, 16, 16)
    fluid = (rng.uniform(size=shape) > 0.3).astype(np.float32)
    local = np.stack([ndimage.uniform_filter(f, size=3, mode="wrap") for f in fluid])
    target = (local * fluid)[..., None] * np.array([1.0, -0.5, 0.25])
    target = target.astype(np.float32)
    x = W.network_input(net.ctx, fluid)
    t, wgt = _f_dev(ctx, target), _f_dev(ctx, fluid)
    losses = []
    for _ in range(40):
        out = net.forward(x)
        loss, g = net.loss(out, t, wgt, 3.0 * fluid.sum())
        net.backward(g)
        net.adam_step(1e-2)
        losses.append(loss)
    assert losses[-1] < 0.3 * losses[0], losses
