"""Host-side checks of liblbm.so that need no GPU: exported symbols, argument
validation, and the host geometry against the oracle's own geometry."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1508_02960_amd import inputs, lbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions(header="lbm.h", prefix="lbm_"):
    src = open(os.path.join(ROOT, "include", header)).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(" + prefix + r"[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_header_function():
    lib = lbm.library()
    names = _header_functions()
    assert len(names) >= 19
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(lbm.EXPORTS)


def test_library_exports_every_network_function():
    from paper_1508_02960_amd import warmstart

    lib = warmstart._nn()
    names = _header_functions("lbm_nn.h", "nn_")
    assert len(names) == 23
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(warmstart.NN_EXPORTS)


def test_network_entry_points_validate_without_a_gpu():
    from paper_1508_02960_amd import warmstart

    lib = warmstart._nn()
    nb, sp = C.c_size_t(), C.c_int()
    # ci and co must be multiples of 8 for the weight gradient
    assert lib.nn_conv3d_backward_weight_workspace(1, 8, 8, 8, 12, 16, C.byref(nb),
                                                   C.byref(sp)) == 1
    assert lib.nn_conv3d_backward_weight_workspace(1, 8, 8, 8, 16, 16, C.byref(nb),
                                                   C.byref(sp)) == 0
    assert nb.value == sp.value * 16 * 27 * 16 * 4 and 1 <= sp.value <= 256
    assert lib.nn_conv3d_forward(None, None, None, None, 1, 4, 4, 4, 8, 8, None) == 1
    assert lib.nn_pool2_forward(C.c_void_p(16), C.c_void_p(16), 1, 3, 4, 4, 8, None) == 1


def _create(shape=(8, 9, 10), **kw):
    nz, ny, nx = shape
    p = lbm.Params(nx, ny, nz, kw.get("tau", 0.8), kw.get("magic", 3 / 16),
                   kw.get("delta_rho", 0.0), kw.get("collision", 1), kw.get("wall", 0),
                   kw.get("storage", 1), kw.get("check_interval", 100))
    mask = kw.get("mask", np.zeros(shape, np.uint8))
    h = C.c_void_p()
    st = lbm.library().lbm_create_domain(
        None if mask is None else mask.ctypes.data_as(C.c_void_p), kw.get("spheres"),
        kw.get("n_spheres", 0), C.byref(p), C.byref(h))
    return st, h


@pytest.mark.parametrize("kw", [
    dict(tau=0.5), dict(tau=0.3), dict(tau=float("nan")), dict(magic=0.0), dict(magic=0.8),
    dict(collision=3), dict(wall=6), dict(wall=-1), dict(storage=7), dict(check_interval=-1),
    dict(wall=2, storage=2), dict(wall=5, storage=3), dict(wall=4, tau=2.0),
    dict(delta_rho=float("inf")), dict(mask=None),
])
def test_invalid_arguments_are_rejected(kw):
    st, h = _create(**kw)
    assert st == 1 and not h.value
    assert lbm.library().lbm_last_error(None)


def test_invalid_dimensions_and_geometry():
    lib = lbm.library()
    for shape in [(0, 4, 4), (4, -1, 4)]:
        nz, ny, nx = shape
        p = lbm.Params(nx, ny, nz, 0.8, 0.1875, 0.0, 1, 0, 1, 0)
        h = C.c_void_p()
        assert lib.lbm_create_domain(None, None, 0, C.byref(p), C.byref(h)) == 1
    # all solid: no fluid cell
    st, h = _create(mask=np.ones((4, 4, 4), np.uint8), shape=(4, 4, 4))
    assert st == 1 and b"fluid" in lib.lbm_last_error(None)
    # both a mask and spheres
    sp = (lbm.Sphere * 1)(lbm.Sphere(2, 2, 2, 1.0))
    st, h = _create(mask=np.zeros((4, 4, 4), np.uint8), shape=(4, 4, 4), spheres=sp, n_spheres=1)
    assert st == 1
    # bad radius / centre
    for s in [lbm.Sphere(2, 2, 2, 0.0), lbm.Sphere(2, 2, 2, 4.0), lbm.Sphere(5, 2, 2, 1.0)]:
        sp = (lbm.Sphere * 1)(s)
        st, h = _create(mask=None, shape=(4, 4, 4), spheres=sp, n_spheres=1)
        assert st == 1


def test_unbound_domain_rejects_device_calls():
    st, h = _create()
    assert st == 0
    lib = lbm.library()
    try:
        assert lib.lbm_step(h, 1) == 6
        U = np.zeros(3)
        assert lib.lbm_mean_velocity(h, U.ctypes.data_as(C.c_void_p), None, None) == 6
        ws = C.c_void_p(0)
        assert lib.lbm_bind(h, ws, 0, None) == 2
    finally:
        lib.lbm_destroy(h)


def test_solid_write_mode_is_validated_without_a_gpu():
    """Solid writes are a batch option: a single domain accepts mode 0 only."""
    st, h = _create()
    assert st == 0
    lib = lbm.library()
    try:
        m = C.c_int32(-1)
        assert lib.lbm_get_solid_writes(h, C.byref(m)) == 0 and m.value == 0
        assert lib.lbm_set_solid_writes(h, 0) == 0
        assert lib.lbm_set_solid_writes(h, 2) == 6
        assert lib.lbm_set_solid_writes(h, 3) == 1
    finally:
        lib.lbm_destroy(h)
    b = lbm.Batch((8, 8, 8), [dict(tau=0.8, delta_rho=1e-4, mask=np.zeros((8, 8, 8), np.uint8))] * 2,
                  bind=False)
    for mode in (2, 1, 0):
        b.set_solid_writes(mode)
        assert b.solid_writes == mode
    with pytest.raises(lbm.LbmError):
        b.set_solid_writes(-1)
    b.close()


def test_info_and_workspace_size():
    shape = (16, 12, 20)
    d = lbm.Domain(shape, tau=0.8, spheres=inputs.centred_sphere(shape, 9.0), bind=False,
                   wall="cli")
    info = d.info
    assert info.n_cells == 16 * 12 * 20
    assert info.state_elems >= 19 * info.n_cells
    assert info.workspace_bytes >= 2 * info.state_elems * 4 + 4 * info.n_cells
    assert info.bytes_per_fluid_update == 152
    assert abs(info.nu - 0.1) < 1e-15 and abs(info.omega_plus - 1.25) < 1e-15
    d64 = lbm.Domain(shape, tau=0.8, spheres=inputs.centred_sphere(shape, 9.0), bind=False,
                     storage="fp64")
    assert d64.info.bytes_per_fluid_update == 304
    d.close()
    d64.close()


GEOMETRIES = [
    ("centred-32", (32, 32, 32), lambda s: inputs.centred_sphere(s, 24.0)),
    ("random", (13, 17, 21), lambda s: inputs.random_spheres(s, 5, (1.5, 4.5), seed=7)),
    ("random-dense", (12, 12, 12), lambda s: inputs.random_spheres(s, 9, (2.0, 3.5), seed=8)),
    ("sc-array", (24, 24, 24), lambda s: inputs.simple_cubic_array(2, 12, 9.0)),
]


@pytest.mark.parametrize("name,shape,make", GEOMETRIES, ids=[g[0] for g in GEOMETRIES])
def test_host_geometry_matches_oracle(orc, name, shape, make):
    """Mask bit-exact, same link set, q within 1e-14, same fallback links."""
    sp = make(shape)
    d = lbm.Domain(shape, tau=0.8, spheres=sp, wall="cli", bind=False)
    mask = d.mask()
    omask = orc.voxelise(shape, sp)
    assert np.array_equal(mask, omask)
    assert d.n_fluid == int((omask == 0).sum())
    cell, dirs, q, fb = d.links()
    Q = orc.wall_q(omask, sp)
    ncell = int(np.prod(shape))
    oj, oc = np.nonzero(Q.reshape(19, ncell) >= 0)
    order = np.lexsort((oj, oc))
    assert np.array_equal(cell, oc[order]) and np.array_equal(dirs, oj[order])
    assert np.max(np.abs(q - Q.reshape(19, ncell)[dirs, cell])) < 1e-14
    e, _, _ = orc.lattice()
    nz, ny, nx = shape
    x, y, z = cell % nx, (cell // nx) % ny, cell // (nx * ny)
    xb, yb, zb = (x - e[dirs, 0]) % nx, (y - e[dirs, 1]) % ny, (z - e[dirs, 2]) % nz
    assert np.array_equal(fb, omask[zb, yb, xb])
    assert d.info.n_fallback == int(fb.sum())
    d.close()


def test_mask_input_gives_half_distance():
    shape = (6, 7, 8)
    m = inputs.random_mask(shape, 0.3, seed=1)
    d = lbm.Domain(shape, tau=0.9, mask=m, wall="cli", bind=False)
    assert np.array_equal(d.mask(), m)
    _, _, q, _ = d.links()
    assert len(q) > 0 and np.all(q == 0.5)
    d.close()


def test_batch_creation_and_validation(orc):
    shape = (8, 9, 10)
    cells = [dict(spheres=inputs.random_spheres(shape, 2, (1.5, 3.0), seed=s), tau=0.7 + 0.1 * s,
                  delta_rho=1e-4) for s in range(3)]
    b = lbm.Batch(shape, cells, wall="cli", bind=False)
    m = b.mask()
    assert m.shape == (3,) + shape
    for i, c in enumerate(cells):
        assert np.array_equal(m[i], orc.voxelise(shape, c["spheres"]))
    assert b.info.n_fluid == int((m == 0).sum())
    # links of cell 1 are those of cell 1 alone, shifted by one cell
    cell, dirs, q, fb = b.links()
    ncell = int(np.prod(shape))
    sel = (cell >= ncell) & (cell < 2 * ncell)
    single = lbm.Domain(shape, tau=0.8, spheres=cells[1]["spheres"], wall="cli", bind=False)
    c1, d1, q1, f1 = single.links()
    assert np.array_equal(cell[sel] - ncell, c1) and np.array_equal(dirs[sel], d1)
    assert np.array_equal(q[sel], q1) and np.array_equal(fb[sel], f1)
    single.close()
    b.close()
    with pytest.raises(lbm.LbmError):
        lbm.Batch(shape, [dict(cells[0], tau=0.5)], bind=False)
    with pytest.raises(lbm.LbmError):
        lbm.Batch(shape, cells, storage="fp16", bind=False)
