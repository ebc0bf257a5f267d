"""Learned warm start for the lattice Boltzmann iteration.

A 3-D U-Net with periodic padding maps the fluid indicator of a periodic
sphere pack to the steady Stokes velocity, in the units t = u nu / G / scale
(G = |grad P| = delta_rho / (3 nx)): Stokes flow is linear in the forcing, so
t depends on the geometry only and one network serves every pressure drop
and viscosity.  A run then starts from the equilibrium of the predicted
velocity instead of rest; the plain iteration to the residual tolerance still
decides the result, so the prediction only changes how many steps it takes.

Every layer runs in the library's kernels (include/lbm_nn.h): BF16
convolutions on matrix cores with FP32 accumulation, FP32 master weights
updated by Adam.  PyTorch only provides device memory and the stream.

Architecture (widths w0..w3, default 32, 64, 128, 256): one 3x3x3 conv + ReLU
per level on the way down (2x2x2 average pooling between levels), and on the
way up nearest upsampling, concatenation with the skip, conv + ReLU; a linear
head conv gives 8 channels: the velocity (0..2) and the periodic part of the
density (3), both in the target units of fields_to_targets.  The forcing
is not an input: in the Stokes regime it only scales the output.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import inputs, lbm, observables

IN_CH = 8     # channel 0: fluid indicator, 1..7: zeros (conv inputs need multiples of 8)
OUT_CH = 8    # channels 0..2: velocity, 3: pressure fluctuation, 4..7: unused


def _nn():
    lib = lbm.library()
    if getattr(lib, "_nn_ready", False):
        return lib
    vp, i32, i64, f32, f64, sz = (C.c_void_p, C.c_int, C.c_longlong, C.c_float, C.c_double,
                                  C.c_size_t)
    sig = {
        "nn_conv3d_forward": [vp, vp, vp, vp, i32, i32, i32, i32, i32, i32, vp],
        "nn_conv3d_forward_act": [vp, vp, vp, vp, i32, i32, i32, i32, i32, i32, i32, vp],
        "nn_conv3d_flip_weights": [vp, vp, i32, i32, vp],
        "nn_conv3d_backward_data": [vp, vp, vp, i32, i32, i32, i32, i32, i32, vp],
        "nn_conv3d_backward_weight_workspace": [i32, i32, i32, i32, i32, i32, C.POINTER(sz),
                                                C.POINTER(i32)],
        "nn_conv3d_backward_weight": [vp, vp, vp, vp, sz, i32, i32, i32, i32, i32, i32, vp],
        "nn_bias_grad_workspace": [i64, i32, C.POINTER(sz)],
        "nn_bias_grad": [vp, vp, vp, sz, i64, i32, vp],
        "nn_activation_forward": [vp, vp, i64, i32, vp],
        "nn_relu_backward": [vp, vp, vp, i64, vp],
        "nn_relu_backward_bias": [vp, vp, vp, vp, vp, sz, i64, i32, i32, vp],
        "nn_cast_bf16": [vp, vp, i64, vp],
        "nn_pool2_forward": [vp, vp, i32, i32, i32, i32, i32, vp],
        "nn_pool2_backward": [vp, vp, i32, i32, i32, i32, i32, vp],
        "nn_upsample2_forward": [vp, vp, i32, i32, i32, i32, i32, vp],
        "nn_upsample2_backward": [vp, vp, i32, i32, i32, i32, i32, vp],
        "nn_concat_channels": [vp, vp, vp, i64, i32, i32, vp],
        "nn_split_channels": [vp, vp, vp, i64, i32, i32, vp],
        "nn_add": [vp, vp, i64, vp],
        "nn_prolongate2": [vp, vp, i32, i32, i32, i32, i32, i32, vp, vp],
        "nn_warm_start_fields": [vp, i32, vp, vp, i32, i32, i32, i32, f64, f64, vp],
        "nn_masked_mse": [vp, vp, vp, vp, vp, i32, i64, i32, i32, f64, vp],
        "nn_adam": [vp, vp, vp, vp, vp, i64, f32, f32, f32, f32, i32, vp],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = C.c_int
    lib._nn_ready = True
    return lib


NN_EXPORTS = (
    "nn_conv3d_forward", "nn_conv3d_forward_act", "nn_conv3d_flip_weights",
    "nn_conv3d_backward_data",
    "nn_conv3d_backward_weight_workspace", "nn_conv3d_backward_weight", "nn_bias_grad",
    "nn_bias_grad_workspace",
    "nn_activation_forward", "nn_relu_backward", "nn_relu_backward_bias", "nn_cast_bf16",
    "nn_pool2_forward",
    "nn_pool2_backward", "nn_upsample2_forward", "nn_upsample2_backward", "nn_concat_channels",
    "nn_split_channels", "nn_add", "nn_masked_mse", "nn_adam", "nn_prolongate2",
    "nn_warm_start_fields",
)


def _p(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _chk(st, what):
    if st != 0:
        raise lbm.LbmError(st, what)


class _Ctx:
    def __init__(self, device):
        import torch

        self.torch = torch
        self.dev = torch.device(device if device is not None else "cuda")
        self.stream = C.c_void_p(torch.cuda.current_stream(self.dev).cuda_stream)

    def f32(self, *shape):
        return self.torch.empty(shape, dtype=self.torch.float32, device=self.dev)

    def bf(self, *shape):
        return self.torch.empty(shape, dtype=self.torch.bfloat16, device=self.dev)

    def zeros(self, *shape):
        return self.torch.zeros(shape, dtype=self.torch.float32, device=self.dev)


class Conv:
    """3x3x3 periodic convolution ci -> co with bias; FP32 master weights,
    BF16 copies for the kernels, Adam moments."""

    def __init__(self, ctx: _Ctx, ci: int, co: int, rng: np.random.Generator):
        self.ctx, self.ci, self.co = ctx, ci, co
        std = np.sqrt(2.0 / (27 * ci))  # He initialisation for ReLU layers
        w = (rng.standard_normal((co, 27, ci)) * std).astype(np.float32)
        t = ctx.torch
        self.w = t.from_numpy(w).to(ctx.dev)
        self.b = ctx.zeros(co)
        self.wb = ctx.bf(co, 27, ci)
        self.wt = ctx.bf(ci, 27, co)
        self.gw = ctx.zeros(co, 27, ci)
        self.gb = ctx.zeros(co)
        self.mw, self.vw = ctx.zeros(co, 27, ci), ctx.zeros(co, 27, ci)
        self.mb, self.vb = ctx.zeros(co), ctx.zeros(co)
        self.refresh()

    def n_params(self) -> int:
        return self.co * 27 * self.ci + self.co

    def refresh(self):
        lib = _nn()
        _chk(lib.nn_cast_bf16(_p(self.w), _p(self.wb), self.w.numel(), self.ctx.stream), "cast")
        _chk(lib.nn_conv3d_flip_weights(_p(self.wb), _p(self.wt), self.ci, self.co,
                                        self.ctx.stream), "flip")

    def forward(self, x_bf, shape):
        n, d, h, w = shape
        y = self.ctx.f32(n, d, h, w, self.co)
        _chk(_nn().nn_conv3d_forward(_p(x_bf), _p(self.wb), _p(self.b), _p(y), n, d, h, w,
                                     self.ci, self.co, self.ctx.stream), "conv forward")
        return y

    def forward_act(self, x_bf, shape, relu=True):
        """bf16(relu(conv(x))): the convolution and the activation in one kernel."""
        n, d, h, w = shape
        a = self.ctx.bf(n, d, h, w, self.co)
        _chk(_nn().nn_conv3d_forward_act(_p(x_bf), _p(self.wb), _p(self.b), _p(a), n, d, h, w,
                                         self.ci, self.co, 1 if relu else 0, self.ctx.stream),
             "conv forward + activation")
        return a

    def backward(self, x_bf, dy32, shape, need_dx=True, act=None):
        """Weight and bias gradients (and the input gradient if need_dx) for
        the FP32 gradient dy32 of the layer's output; act is the stored BF16
        activation of a ReLU layer (its backward, the BF16 cast and the bias
        gradient are one kernel), None for a linear layer."""
        lib = _nn()
        n, d, h, w = shape
        m = n * d * h * w
        t = self.ctx.torch
        dy = self.ctx.bf(n, d, h, w, self.co)
        bb = C.c_size_t()
        _chk(lib.nn_bias_grad_workspace(m, self.co, C.byref(bb)), "bias ws")
        bws = t.empty(int(bb.value), dtype=t.uint8, device=self.ctx.dev)
        _chk(lib.nn_relu_backward_bias(_p(dy32), None if act is None else _p(act), _p(dy),
                                       _p(self.gb), _p(bws), bb.value, m, self.co,
                                       0 if act is None else 1, self.ctx.stream),
             "activation backward + bias grad")
        nbytes = C.c_size_t()
        sp = C.c_int()
        _chk(lib.nn_conv3d_backward_weight_workspace(n, d, h, w, self.ci, self.co,
                                                     C.byref(nbytes), C.byref(sp)), "ws")
        ws = t.empty(int(nbytes.value), dtype=t.uint8, device=self.ctx.dev)
        _chk(lib.nn_conv3d_backward_weight(_p(x_bf), _p(dy), _p(self.gw), _p(ws), nbytes.value,
                                           n, d, h, w, self.ci, self.co, self.ctx.stream),
             "conv backward weight")
        if not need_dx:
            return None
        dx = self.ctx.f32(n, d, h, w, self.ci)
        _chk(lib.nn_conv3d_backward_data(_p(dy), _p(self.wt), _p(dx), n, d, h, w, self.ci,
                                         self.co, self.ctx.stream), "conv backward data")
        return dx

    def adam(self, lr, step, b1=0.9, b2=0.999, eps=1e-8):
        lib = _nn()
        _chk(lib.nn_adam(_p(self.w), _p(self.gw), _p(self.mw), _p(self.vw), _p(self.wb),
                         self.w.numel(), lr, b1, b2, eps, step, self.ctx.stream), "adam")
        _chk(lib.nn_adam(_p(self.b), _p(self.gb), _p(self.mb), _p(self.vb), None, self.co, lr,
                         b1, b2, eps, step, self.ctx.stream), "adam")
        _chk(lib.nn_conv3d_flip_weights(_p(self.wb), _p(self.wt), self.ci, self.co,
                                        self.ctx.stream), "flip")


class UNet:
    def __init__(self, widths=(32, 64, 128, 256), seed: int = 0, device=None):
        self.ctx = _Ctx(device)
        rng = np.random.default_rng(seed)
        w0, w1, w2, w3 = widths
        self.widths = widths
        self.enc = [Conv(self.ctx, IN_CH, w0, rng), Conv(self.ctx, w0, w1, rng),
                    Conv(self.ctx, w1, w2, rng), Conv(self.ctx, w2, w3, rng)]
        self.dec = [Conv(self.ctx, w3 + w2, w2, rng), Conv(self.ctx, w2 + w1, w1, rng),
                    Conv(self.ctx, w1 + w0, w0, rng)]
        self.head = Conv(self.ctx, w0, OUT_CH, rng)
        # a linear head starts near zero output
        self.head.w.mul_(0.1)
        self.head.refresh()
        self.step_count = 0
        self.scale = 1.0  # target units per output unit

    def layers(self):
        return self.enc + self.dec + [self.head]

    def n_params(self) -> int:
        return sum(l.n_params() for l in self.layers())

    # -------------------------------------------------------------- passes
    def forward(self, x_bf):
        """x_bf: bf16 (n, d, h, w, 8), d, h, w divisible by 8.  Returns the
        FP32 output (n, d, h, w, 8) and keeps what the backward pass needs."""
        lib = _nn()
        s = self.ctx.stream
        n, d, h, w, _ = x_bf.shape
        shapes = [(n, d >> l, h >> l, w >> l) for l in range(4)]
        self.cache = dict(x=x_bf, shapes=shapes)
        e, inp = [], x_bf
        for lvl, conv in enumerate(self.enc):
            if lvl > 0:
                pn, pd, ph, pw = shapes[lvl - 1]
                p = self.ctx.bf(*shapes[lvl], conv.ci)
                _chk(lib.nn_pool2_forward(_p(inp), _p(p), pn, pd, ph, pw, conv.ci, s), "pool")
                inp = p
            self.cache[f"in{lvl}"] = inp
            e.append(conv.forward_act(inp, shapes[lvl]))
            inp = e[-1]
        cur = e[3]
        for j, conv in enumerate(self.dec):
            lvl = 2 - j
            ccur = self.widths[lvl + 1]
            up = self.ctx.bf(*shapes[lvl], ccur)
            qn, qd, qh, qw = shapes[lvl + 1]
            _chk(lib.nn_upsample2_forward(_p(cur), _p(up), qn, qd, qh, qw, ccur, s), "upsample")
            cat = self.ctx.bf(*shapes[lvl], conv.ci)
            m = int(np.prod(shapes[lvl]))
            _chk(lib.nn_concat_channels(_p(up), _p(e[lvl]), _p(cat), m, ccur, self.widths[lvl], s),
                 "concat")
            self.cache[f"cat{lvl}"] = cat
            cur = conv.forward_act(cat, shapes[lvl])
            self.cache[f"d{lvl}"] = cur
        self.cache["e"] = e
        out = self.head.forward(cur, shapes[0])
        return out

    def backward(self, dout):
        """Gradients of all weights for upstream gradient dout (n, d, h, w, 8)."""
        lib = _nn()
        s = self.ctx.stream
        c = self.cache
        shapes, e = c["shapes"], c["e"]
        # head (linear)
        g = self.head.backward(c["d0"], dout, shapes[0])
        skip_grads = [None] * 3
        for j, conv in enumerate(self.dec):
            lvl = j  # backward goes 0, 1, 2 through decoder levels
            conv = self.dec[2 - lvl]
            dcat = conv.backward(c[f"cat{lvl}"], g, shapes[lvl], act=c[f"d{lvl}"])
            ccur = self.widths[lvl + 1]
            m = int(np.prod(shapes[lvl]))
            dup = self.ctx.f32(*shapes[lvl], ccur)
            dskip = self.ctx.f32(*shapes[lvl], self.widths[lvl])
            _chk(lib.nn_split_channels(_p(dcat), _p(dup), _p(dskip), m, ccur, self.widths[lvl], s),
                 "split")
            skip_grads[lvl] = dskip
            g = self.ctx.f32(*shapes[lvl + 1], ccur)
            qn, qd, qh, qw = shapes[lvl + 1]
            _chk(lib.nn_upsample2_backward(_p(dup), _p(g), qn, qd, qh, qw, ccur, s), "up backward")
        # g: gradient of e[3]; down the encoder
        for lvl in (3, 2, 1, 0):
            conv = self.enc[lvl]
            if lvl < 3:
                _chk(lib.nn_add(_p(g), _p(skip_grads[lvl]), g.numel(), s), "add")
            dinp = conv.backward(c[f"in{lvl}"], g, shapes[lvl], need_dx=lvl > 0, act=e[lvl])
            if lvl > 0:
                g = self.ctx.f32(*shapes[lvl - 1], conv.ci)
                pn, pd, ph, pw = shapes[lvl - 1]
                _chk(lib.nn_pool2_backward(_p(dinp), _p(g), pn, pd, ph, pw, conv.ci, s),
                     "pool backward")

    def adam_step(self, lr: float):
        self.step_count += 1
        for l in self.layers():
            l.adam(lr, self.step_count)

    # --------------------------------------------------------------- loss
    def loss(self, out, target, weight, norm: float, sync: bool = True):
        """Weighted MSE of the first target.shape[-1] output channels against
        target; returns (loss, grad), the loss as a device scalar when
        sync is False."""
        lib = _nn()
        m = out.numel() // OUT_CH
        used = int(target.shape[-1])
        grad = self.ctx.f32(*out.shape)
        nb = 1024
        part = self.ctx.torch.empty(nb, dtype=self.ctx.torch.float64, device=self.ctx.dev)
        _chk(lib.nn_masked_mse(_p(out), _p(target), _p(weight), _p(grad), _p(part), nb, m,
                               OUT_CH, used, float(norm), self.ctx.stream), "mse")
        total = part.sum()
        return (float(total.item()) if sync else total), grad

    # ------------------------------------------------------ use and storage
    def predict(self, fluid: np.ndarray, used: int = 4) -> np.ndarray:
        """Targets (nz, ny, nx, used) for one fluid mask (edges multiples of
        8), in target units (the output times self.scale)."""
        out = self.forward(network_input(self.ctx, fluid[None].astype(np.uint8)))
        return out[0, ..., :used].float().cpu().numpy() * self.scale

    def save(self, path: str, bf16: bool = False) -> None:
        """FP32 master weights, or with bf16 the BF16 weights the kernels use
        (as raw 16-bit patterns, compressed): inference is unchanged."""
        arrays = {"widths": np.array(self.widths), "scale": np.array(self.scale),
                  "step_count": np.array(self.step_count)}
        for i, l in enumerate(self.layers()):
            w = l.w.cpu().numpy()
            arrays[f"w{i}"] = _to_bf16_bits(w) if bf16 else w
            arrays[f"b{i}"] = l.b.cpu().numpy()
        (np.savez_compressed if bf16 else np.savez)(path, **arrays)

    @classmethod
    def load(cls, path: str, device=None) -> "UNet":
        z = np.load(path)
        net = cls(widths=tuple(int(v) for v in z["widths"]), device=device)
        net.scale = float(z["scale"])
        net.step_count = int(z["step_count"])
        for i, l in enumerate(net.layers()):
            w = z[f"w{i}"]
            if w.dtype == np.uint16:
                w = (w.astype(np.uint32) << 16).view(np.float32)
            l.w.copy_(net.ctx.torch.from_numpy(np.ascontiguousarray(w)))
            l.b.copy_(net.ctx.torch.from_numpy(z[f"b{i}"]))
            l.refresh()
        return net


def _to_bf16_bits(a: np.ndarray) -> np.ndarray:
    """Round FP32 to the nearest BF16 (ties to even) as 16-bit patterns."""
    b = np.ascontiguousarray(a, np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) >> 16
    return b.astype(np.uint16)


# ------------------------------------------------------------------ data

def network_input(ctx: _Ctx, fluid):
    """bf16 input (n, d, h, w, 8) with the fluid indicator in channel 0, from
    a host array or a device tensor of shape (n, d, h, w)."""
    t = ctx.torch
    f = fluid if isinstance(fluid, t.Tensor) else t.from_numpy(np.ascontiguousarray(fluid))
    f = f.to(ctx.dev)
    x = t.zeros(tuple(f.shape) + (IN_CH,), dtype=t.bfloat16, device=ctx.dev)
    x[..., 0] = f.to(t.bfloat16)
    return x


def percolates_x(fluid: np.ndarray) -> bool:
    """True if fluid connects the plane x = 0 to x = nx - 1 through
    face-neighbours, with y and z periodic."""
    from scipy import ndimage

    lab, n = ndimage.label(fluid)
    if n == 0:
        return False
    parent = list(range(n + 1))

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    for ax in (0, 1):  # z and y faces wrap
        a = np.take(lab, 0, axis=ax)
        b = np.take(lab, -1, axis=ax)
        both = (a > 0) & (b > 0)
        for u, v in zip(a[both], b[both]):
            ru, rv = find(u), find(v)
            if ru != rv:
                parent[ru] = rv
    left = {find(v) for v in np.unique(lab[..., 0]) if v}
    right = {find(v) for v in np.unique(lab[..., -1]) if v}
    return bool(left & right)


# ------------------------------------------------------- target units
# Stokes flow is linear in the forcing, so the steady fields divided by the
# pressure gradient depend on the geometry alone.  With G = delta_rho / (3 nx)
# and the density written as the linear part -(delta_rho / nx)(x - (nx-1)/2)
# plus a periodic fluctuation rho', the targets are
#   t_u = u nu / G                      (length^2)
#   t_p = rho' nx / delta_rho           (length)
# and every target is further divided by the network's output scale.

def fields_to_targets(drho, u, delta_rho: float, tau: float, fluid):
    """(nz, ny, nx) density deviation and (3, nz, ny, nx) velocity of a
    steady run -> (nz, ny, nx, 4) targets; rho' has zero mean over fluid."""
    nz, ny, nx = drho.shape
    G = observables.pressure_gradient(delta_rho, nx)
    nu = observables.viscosity(tau)
    x = np.arange(nx) - (nx - 1) / 2.0
    tp = drho * (nx / delta_rho) + x[None, None, :]
    tp = np.where(fluid, tp - tp[fluid].mean(), 0.0)
    out = np.empty((nz, ny, nx, 4), np.float32)
    out[..., :3] = np.moveaxis(u, 0, -1) * (nu / G)
    out[..., 3] = tp
    return out


def targets_to_fields(t, delta_rho: float, tau: float, fluid):
    """Inverse of fields_to_targets: (drho, u) for lbm_init_equilibrium,
    zero on solid nodes."""
    nz, ny, nx, _ = t.shape
    G = observables.pressure_gradient(delta_rho, nx)
    nu = observables.viscosity(tau)
    x = np.arange(nx) - (nx - 1) / 2.0
    drho = (t[..., 3].astype(np.float64) - x[None, None, :]) * (delta_rho / nx)
    u = np.moveaxis(t[..., :3].astype(np.float64), -1, 0) * (G / nu)
    return np.where(fluid, drho, 0.0), np.where(fluid[None], u, 0.0)


def linear_density(shape, delta_rho: float, fluid):
    """The linear part of the steady density, -(delta_rho/nx)(x - (nx-1)/2),
    on fluid nodes."""
    nx = shape[-1]
    x = np.arange(nx) - (nx - 1) / 2.0
    return np.where(fluid, -(delta_rho / nx) * x, 0.0)


# ------------------------------------------------------ two-grid start
# A cell larger than the network's receptive field (about 54 nodes) is
# predicted on the grid of half the resolution instead: coarse node j sits at
# fine position 2j + 1/2, the centre of a 2 x 2 x 2 block of fine nodes, so
# the coarse pack is the same spheres in units of two fine cells.  The
# prediction is interpolated back to the fine nodes.

def coarse_fluid(spheres, edge: int) -> np.ndarray:
    """Fluid mask (edge/2)^3 of a periodic pack of spheres (rows cx, cy, cz,
    r in fine lattice units, box edge `edge`) on the coarse grid: a coarse
    node is solid iff its position lies strictly inside a sphere or one of its
    periodic images."""
    ec = edge // 2
    pos = 2.0 * np.arange(ec) + 0.5
    solid = np.zeros((ec, ec, ec), bool)
    for cx, cy, cz, r in np.reshape(spheres, (-1, 4)):
        per = []
        for v in (cz, cy, cx):
            a = np.abs(pos - v)
            per.append(np.minimum(a, edge - a) ** 2)
        solid |= per[0][:, None, None] + per[1][None, :, None] + per[2][None, None, :] < r * r
    return ~solid


def prolongate2(t: np.ndarray) -> np.ndarray:
    """Coarse targets (ec, ec, ec, C) -> fine (2ec, 2ec, 2ec, C): periodic
    trilinear interpolation at the fine nodes, which sit at coarse
    coordinates (i - 1/2)/2, so each fine node takes 3/4 of its nearer and
    1/4 of its farther coarse neighbour per axis.  Lengths double on the fine
    grid: velocity targets (length^2) are multiplied by 4, density targets
    (length) by 2."""
    out = np.asarray(t, np.float64)
    for ax in range(3):
        even = 0.75 * out + 0.25 * np.roll(out, 1, axis=ax)   # fine 2m: between m-1 and m
        odd = 0.75 * out + 0.25 * np.roll(out, -1, axis=ax)   # fine 2m+1: between m and m+1
        shape = list(out.shape)
        shape[ax] *= 2
        fine = np.empty(shape)
        sl_e = [slice(None)] * 4
        sl_o = [slice(None)] * 4
        sl_e[ax] = slice(0, None, 2)
        sl_o[ax] = slice(1, None, 2)
        fine[tuple(sl_e)] = even
        fine[tuple(sl_o)] = odd
        out = fine
    scale = np.ones(out.shape[-1])
    scale[:3] = 4.0
    scale[3:] = 2.0
    return (out * scale).astype(np.float32)


def predict_two_grid_device(net, spheres, edge: int, out=None, used: int = 4):
    """Two-grid prediction of a pack of edge^3 (edge a multiple of 16): the
    network on coarse_fluid's grid, then the prolongation of prolongate2 on
    the device (nn_prolongate2, with the network's output scale and the
    doubled lengths in the channel scale); target units, a device tensor
    (edge,)*3 + (used,), written into out if given."""
    lib = _nn()
    ctx = net.ctx
    t = ctx.torch
    ec = edge // 2
    y = net.forward(network_input(ctx, coarse_fluid(spheres, edge)[None].astype(np.uint8)))
    lengths = [4.0] * min(used, 3) + [2.0] * max(used - 3, 0)
    scale = t.tensor([net.scale * s for s in lengths], dtype=t.float32, device=ctx.dev)
    fine = out if out is not None else ctx.f32(edge, edge, edge, used)
    _chk(lib.nn_prolongate2(_p(y), _p(fine), 1, ec, ec, ec, int(y.shape[-1]), used, _p(scale),
                            ctx.stream), "prolongate2")
    return fine


def predict_two_grid(net, spheres, edge: int, used: int = 4) -> np.ndarray:
    """predict_two_grid_device on the host."""
    return predict_two_grid_device(net, spheres, edge, used=used).cpu().numpy()


def warm_fields_device(ctx, t, fluid, delta_rho: float, tau: float):
    """warm_fields on the device (nn_warm_start_fields): t the predicted
    targets (n, d, h, w, c) on the device, fluid the host masks (n, d, h, w);
    returns the (4, n d h w) float64 device fields of
    Batch.init_equilibrium_device (the linear density, the predicted velocity
    away from walls)."""
    lib = _nn()
    th = ctx.torch
    n, d, h, w = fluid.shape
    if (tuple(t.shape[:-1]) != (n, d, h, w) or t.shape[-1] < 3 or t.dtype != th.float32
            or not t.is_contiguous() or not t.is_cuda):
        raise ValueError(f"targets {tuple(t.shape)} do not match the masks {fluid.shape}")
    f = th.from_numpy(np.ascontiguousarray(fluid, np.uint8)).to(ctx.dev)
    fields = th.empty((4, n * d * h * w), dtype=th.float64, device=ctx.dev)
    factor = observables.pressure_gradient(delta_rho, w) / observables.viscosity(tau)
    _chk(lib.nn_warm_start_fields(_p(t), int(t.shape[-1]), _p(f), _p(fields), n, d, h, w,
                                  float(factor), float(delta_rho), ctx.stream), "warm fields")
    return fields


_D3Q19_NEIGHBOURS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)
                     if 0 < abs(dz) + abs(dy) + abs(dx) <= 2]


def wall_layer(fluid: np.ndarray) -> np.ndarray:
    """Fluid nodes with at least one solid node among their 18 lattice
    neighbours (periodic), over the last three axes."""
    solid_nb = np.zeros(fluid.shape, bool)
    for off in _D3Q19_NEIGHBOURS:
        solid_nb |= ~np.roll(fluid, off, axis=(-3, -2, -1))
    return fluid & solid_nb


def warm_fields(t, delta_rho: float, tau: float, fluid, use_density: bool = False):
    """Initial (drho, u) of a warm start from predicted targets t.  The
    predicted velocity is used away from walls only: on the wall layer an
    imposed velocity that differs from the wall-consistent one excites
    slowly decaying period-2 oscillations of the bounce-back links, so the
    wall layer starts at rest.  The density is the linear profile of the
    pressure drop, plus the predicted fluctuation if use_density."""
    drho, u = targets_to_fields(t, delta_rho, tau, fluid)
    u = np.where(wall_layer(fluid)[None], 0.0, u)
    if not use_density:
        drho = linear_density(fluid.shape, delta_rho, fluid)
    return drho, u
