"""Python binding of liblbm.so (include/lbm.h): argument marshalling only.

Every step of the hot path runs in the HIP library; PyTorch only provides the
device workspace (a uint8 tensor) and the stream.  There is no fallback: if
liblbm.so is missing or cannot be loaded, :func:`library` raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm.so")

COLLISIONS = {"srt": 0, "trt": 1, "mrt": 2}
WALLS = {"sbb": 0, "cli": 1, "libb": 2, "qibb": 3, "iebb": 4, "mr": 5}
STORAGES = {"fp64": 0, "fp32": 1, "fp16": 2, "bf16": 3, "fp16_rne": 4, "bf16_rne": 5}

STATUS = {0: "ok", 1: "invalid argument", 2: "workspace", 3: "device error", 4: "unstable",
          5: "not converged", 6: "invalid state"}

EXPORTS = (
    "lbm_create_domain", "lbm_get_info", "lbm_get_mask", "lbm_get_links", "lbm_bind",
    "lbm_init_equilibrium", "lbm_set_state", "lbm_get_state", "lbm_step",
    "lbm_run_to_residual", "lbm_macroscopic", "lbm_mean_velocity", "lbm_permeability",
    "lbm_drag", "lbm_set_delta_rho", "lbm_synchronize", "lbm_destroy", "lbm_status_string",
    "lbm_last_error", "lbm_create_batch", "lbm_batch_results", "lbm_batch_set_shape",
    "lbm_batch_autotune", "lbm_macroscopic_device", "lbm_init_equilibrium_device",
    "lbm_set_solid_writes", "lbm_get_solid_writes", "lbm_bandwidth_probe",
    "lbm_mean_velocity_static", "lbm_set_step_shape", "lbm_get_step_shape",
)

PROBES = {"read": 0, "write": 1, "copy": 2, "gather19": 3}


class LbmError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class Unstable(LbmError):
    pass


class NotConverged(LbmError):
    pass


class Params(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("tau", C.c_double), ("magic", C.c_double), ("delta_rho", C.c_double),
                ("collision", C.c_int32), ("wall", C.c_int32), ("storage", C.c_int32),
                ("check_interval", C.c_int32)]


class Sphere(C.Structure):
    _fields_ = [("cx", C.c_double), ("cy", C.c_double), ("cz", C.c_double), ("r", C.c_double)]


class CellParams(C.Structure):
    _fields_ = [("tau", C.c_double), ("magic", C.c_double), ("delta_rho", C.c_double)]


class Info(C.Structure):
    _fields_ = [("n_cells", C.c_int64), ("n_fluid", C.c_int64), ("n_links", C.c_int64),
                ("n_fallback", C.c_int64), ("workspace_bytes", C.c_int64),
                ("state_elems", C.c_int64), ("nu", C.c_double), ("omega_plus", C.c_double),
                ("omega_minus", C.c_double), ("bytes_per_fluid_update", C.c_int64),
                ("storage_scale", C.c_double), ("tile_width", C.c_int32),
                ("tile_height", C.c_int32)]


_lib = None


def library():
    """Load liblbm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    # torch ships its own HIP runtime; load it first so that liblbm.so binds
    # to the same libamdhip64 instead of a second copy that sees no device
    import torch  # noqa: F401
    lib = C.CDLL(LIB_PATH)
    vp, i32, i64, d = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    P = C.POINTER
    sig = {
        "lbm_create_domain": [vp, vp, i32, P(Params), P(vp)],
        "lbm_get_info": [vp, P(Info)],
        "lbm_get_mask": [vp, vp],
        "lbm_get_links": [vp, vp, vp, vp, vp],
        "lbm_bind": [vp, vp, C.c_size_t, vp],
        "lbm_init_equilibrium": [vp, vp, vp],
        "lbm_set_state": [vp, vp],
        "lbm_get_state": [vp, vp],
        "lbm_step": [vp, i64],
        "lbm_run_to_residual": [vp, d, i64, P(i64), P(d)],
        "lbm_macroscopic": [vp, vp, vp],
        "lbm_macroscopic_device": [vp, vp],
        "lbm_init_equilibrium_device": [vp, vp],
        "lbm_mean_velocity": [vp, vp, P(d), P(d)],
        "lbm_mean_velocity_static": [vp, vp, P(d), P(d)],
        "lbm_permeability": [vp, P(d), P(d), P(d)],
        "lbm_drag": [vp, vp],
        "lbm_set_delta_rho": [vp, d],
        "lbm_synchronize": [vp],
        "lbm_destroy": [vp],
        "lbm_create_batch": [i32, vp, vp, vp, vp, P(Params), P(vp)],
        "lbm_batch_results": [vp, vp, vp, vp, vp, vp],
        "lbm_batch_set_shape": [vp, i32, i32],
        "lbm_set_step_shape": [vp, i32, i32, i32],
        "lbm_get_step_shape": [vp, P(i32), P(i32), P(i32)],
        "lbm_batch_autotune": [vp, i32, P(i32), P(i32), P(d)],
        "lbm_set_solid_writes": [vp, i32],
        "lbm_get_solid_writes": [vp, P(i32)],
        "lbm_bandwidth_probe": [i32, vp, vp, i64, vp],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = C.c_int
    lib.lbm_status_string.argtypes = [C.c_int]
    lib.lbm_status_string.restype = C.c_char_p
    lib.lbm_last_error.argtypes = [vp]
    lib.lbm_last_error.restype = C.c_char_p
    _lib = lib
    return lib


def bandwidth_probe(kind: str, src, dst, n: int, stream) -> None:
    """Enqueue one attainable-bandwidth probe (lbm_bandwidth_probe) on a torch
    stream; src and dst are device tensors (dst only for "write")."""
    st = library().lbm_bandwidth_probe(PROBES[kind],
                                       C.c_void_p(src.data_ptr()) if src is not None else None,
                                       C.c_void_p(dst.data_ptr()), int(n),
                                       C.c_void_p(stream.cuda_stream))
    if st != 0:
        raise LbmError(st, f"bandwidth probe {kind} rejected")


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


class Domain:
    """A periodic D3Q19 domain on the GPU.

    ``shape`` is ``(nz, ny, nx)``.  Give either ``mask`` (uint8[nz, ny, nx],
    1 = solid) or ``spheres`` (rows cx, cy, cz, r).  ``bind=True`` allocates
    the workspace with torch on ``device`` and binds it to torch's current
    stream on that device.
    """

    def __init__(self, shape, *, tau: float, magic: float = 3 / 16, delta_rho: float = 0.0,
                 collision: str = "trt", wall: str = "sbb", storage: str = "fp32",
                 mask=None, spheres=None, check_interval: int = 100, device=None,
                 bind: bool = True):
        lib = library()
        self.shape = tuple(int(s) for s in shape)
        nz, ny, nx = self.shape
        self.params = Params(nx, ny, nz, float(tau), float(magic), float(delta_rho),
                             COLLISIONS[collision], WALLS[wall], STORAGES[storage],
                             int(check_interval))
        self.storage = storage
        m = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
        if m is not None and m.shape != self.shape:
            raise ValueError("mask shape must equal shape")
        sp = None
        nsp = 0
        if spheres is not None and len(spheres):
            arr = _f64(np.reshape(spheres, (-1, 4)))
            nsp = arr.shape[0]
            sp = (Sphere * nsp)(*[Sphere(*row) for row in arr])
        h = C.c_void_p()
        st = lib.lbm_create_domain(_ptr(m), sp, nsp, C.byref(self.params), C.byref(h))
        if st != 0:
            raise LbmError(st, lib.lbm_last_error(None).decode())
        self._h = h
        self._ws = None
        self._stream = None
        self.info = Info()
        self._check(lib.lbm_get_info(self._h, C.byref(self.info)))
        if bind:
            self.bind(device)

    # ------------------------------------------------------------ plumbing
    def _check(self, st: int) -> None:
        if st == 0:
            return
        msg = library().lbm_last_error(self._h).decode()
        if st == 4:
            raise Unstable(st, msg)
        if st == 5:
            raise NotConverged(st, msg)
        raise LbmError(st, msg)

    def close(self) -> None:
        if getattr(self, "_h", None):
            library().lbm_destroy(self._h)
            self._h = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def ncell(self) -> int:
        return int(self.info.n_cells)

    @property
    def n_fluid(self) -> int:
        return int(self.info.n_fluid)

    def bind(self, device=None) -> None:
        import torch

        dev = torch.device(device if device is not None else "cuda")
        if dev.type != "cuda":
            raise ValueError("the LBM library runs on a GPU device only")
        nbytes = int(self.info.workspace_bytes)
        self._ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        self._stream = torch.cuda.current_stream(dev)
        self._check(library().lbm_bind(self._h, C.c_void_p(self._ws.data_ptr()), nbytes,
                                       C.c_void_p(self._stream.cuda_stream)))

    @property
    def stream(self):
        return self._stream

    # ------------------------------------------------------------ geometry
    def mask(self) -> np.ndarray:
        m = np.zeros(self.shape, np.uint8)
        self._check(library().lbm_get_mask(self._h, _ptr(m)))
        return m

    def links(self):
        n = int(self.info.n_links)
        cell = np.zeros(n, np.int64)
        d = np.zeros(n, np.int32)
        q = np.zeros(n)
        fb = np.zeros(n, np.uint8)
        self._check(library().lbm_get_links(self._h, _ptr(cell), _ptr(d), _ptr(q), _ptr(fb)))
        return cell, d, q, fb

    # --------------------------------------------------------------- state
    def init_equilibrium(self, drho0=None, u0=None) -> None:
        d = None if drho0 is None else _f64(np.broadcast_to(drho0, self.shape))
        u = None if u0 is None else _f64(np.broadcast_to(u0, (3,) + self.shape))
        self._check(library().lbm_init_equilibrium(self._h, _ptr(d), _ptr(u)))

    def set_state(self, g) -> None:
        g = _f64(g).reshape((19,) + self.shape)
        self._check(library().lbm_set_state(self._h, _ptr(g)))

    def get_state(self) -> np.ndarray:
        g = np.zeros((19,) + self.shape)
        self._check(library().lbm_get_state(self._h, _ptr(g)))
        return g

    def refresh_info(self) -> Info:
        self._check(library().lbm_get_info(self._h, C.byref(self.info)))
        return self.info

    def step(self, n: int = 1) -> None:
        self._check(library().lbm_step(self._h, int(n)))

    def run_to_residual(self, tol: float, max_steps: int, raise_on_fail: bool = False):
        done = C.c_int64(0)
        res = C.c_double(0.0)
        st = library().lbm_run_to_residual(self._h, float(tol), int(max_steps),
                                           C.byref(done), C.byref(res))
        status = {0: "converged", 5: "not_converged", 4: "unstable"}.get(st)
        if status is None or (raise_on_fail and st != 0):
            self._check(st)
        return status, done.value, res.value

    def step_shape(self):
        """(wavefronts per workgroup, tile rows per workgroup, two cells per
        lane) of the step launch."""
        w, r, pr = C.c_int32(), C.c_int32(), C.c_int32()
        self._check(library().lbm_get_step_shape(self._h, C.byref(w), C.byref(r), C.byref(pr)))
        return w.value, r.value, bool(pr.value)

    def set_step_shape(self, waves: int, rows: int, pairs: bool) -> None:
        self._check(library().lbm_set_step_shape(self._h, int(waves), int(rows),
                                                 int(bool(pairs))))

    def set_delta_rho(self, delta_rho: float) -> None:
        self._check(library().lbm_set_delta_rho(self._h, float(delta_rho)))
        self.params.delta_rho = float(delta_rho)

    def synchronize(self) -> None:
        self._check(library().lbm_synchronize(self._h))

    @property
    def solid_writes(self) -> int:
        """Which solid cells a batch step writes (0, 1, 2; speed only, see lbm.h)."""
        m = C.c_int32()
        self._check(library().lbm_get_solid_writes(self._h, C.byref(m)))
        return m.value

    def set_solid_writes(self, mode: int) -> None:
        self._check(library().lbm_set_solid_writes(self._h, int(mode)))

    # --------------------------------------------------------- observables
    def macroscopic(self):
        drho = np.zeros(self.shape)
        u = np.zeros((3,) + self.shape)
        self._check(library().lbm_macroscopic(self._h, _ptr(drho), _ptr(u)))
        return drho, u

    def macroscopic_device(self):
        """(4, ncell) float64 tensor on the domain's device: drho, u_x, u_y,
        u_z in cell order (no host round trip)."""
        import torch

        out = torch.empty((4, self.ncell), dtype=torch.float64, device=self._ws.device)
        self._check(library().lbm_macroscopic_device(self._h, C.c_void_p(out.data_ptr())))
        return out

    def init_equilibrium_device(self, fields) -> None:
        """Equilibrium of device fields (4, ncell) float64 laid out as from
        macroscopic_device (FP32 and FP64 storage)."""
        if tuple(fields.shape) != (4, self.ncell) or not fields.is_contiguous():
            raise ValueError("fields must be a contiguous (4, ncell) tensor")
        self._check(library().lbm_init_equilibrium_device(self._h, C.c_void_p(fields.data_ptr())))

    def mean_velocity(self):
        U = np.zeros(3)
        vmax = C.c_double()
        tot = C.c_double()
        self._check(library().lbm_mean_velocity(self._h, _ptr(U), C.byref(vmax), C.byref(tot)))
        return U, vmax.value, tot.value

    def mean_velocity_static(self):
        """mean_velocity through the no-allocation entry point (scratch in a
        static device array of the library)."""
        U = np.zeros(3)
        vmax = C.c_double()
        tot = C.c_double()
        self._check(library().lbm_mean_velocity_static(self._h, _ptr(U), C.byref(vmax),
                                                       C.byref(tot)))
        return U, vmax.value, tot.value

    def permeability(self):
        """(K_D, U_x): Darcy permeability and superficial velocity."""
        K = C.c_double()
        U = C.c_double()
        self._check(library().lbm_permeability(self._h, C.byref(K), C.byref(U), None))
        return K.value, U.value

    def reynolds(self, diameter: float) -> float:
        """Pore Reynolds number U_x D / nu for the length scale D."""
        r = C.c_double()
        self._check(library().lbm_permeability(self._h, None, None, C.byref(r)))
        return r.value * float(diameter)

    def drag(self) -> np.ndarray:
        F = np.zeros(3)
        self._check(library().lbm_drag(self._h, _ptr(F)))
        return F


BATCH_STATUS = {0: "running", 1: "converged", 2: "unstable", 3: "step_limit"}


class Batch(Domain):
    """Independent periodic cells of one shape ``(nz, ny, nx)``, stepped together.

    ``cells`` is a list of dicts with ``tau``, ``delta_rho``, optional
    ``magic`` and either ``spheres`` (rows cx, cy, cz, r) or ``mask``.
    Arrays of the whole batch have shape ``(n_cells, nz, ny, nx)`` (per
    population or component in front).
    """

    def __init__(self, cell_shape, cells, *, collision: str = "trt", wall: str = "sbb",
                 storage: str = "fp32", check_interval: int = 100, device=None,
                 bind: bool = True):
        lib = library()
        self.cell_shape = tuple(int(v) for v in cell_shape)
        nz, ny, nx = self.cell_shape
        self.n_cells = len(cells)
        self.shape = (self.n_cells * nz, ny, nx)
        self.params = Params(nx, ny, nz, 0.0, 0.0, 0.0, COLLISIONS[collision], WALLS[wall],
                             STORAGES[storage], int(check_interval))
        self.storage = storage
        self.cells = [dict(c) for c in cells]
        cp = (CellParams * self.n_cells)(*[
            CellParams(float(c["tau"]), float(c.get("magic", 3 / 16)), float(c["delta_rho"]))
            for c in cells])
        masks = None
        sp = None
        counts = None
        if "mask" in cells[0]:
            masks = np.ascontiguousarray(np.stack([c["mask"] for c in cells]), dtype=np.uint8)
        else:
            rows = [np.reshape(np.asarray(c["spheres"], np.float64), (-1, 4)) for c in cells]
            allsp = np.concatenate(rows)
            sp = (Sphere * len(allsp))(*[Sphere(*r) for r in allsp])
            counts = np.array([len(r) for r in rows], np.int32)
        h = C.c_void_p()
        st = lib.lbm_create_batch(self.n_cells, _ptr(masks), sp, _ptr(counts), cp,
                                  C.byref(self.params), C.byref(h))
        if st != 0:
            raise LbmError(st, lib.lbm_last_error(None).decode())
        self._h = h
        self._ws = None
        self._stream = None
        self.info = Info()
        self._check(lib.lbm_get_info(self._h, C.byref(self.info)))
        if bind:
            self.bind(device)

    def _as_batch(self, a):
        return a.reshape(a.shape[:-3] + (self.n_cells,) + self.cell_shape)

    def mask(self) -> np.ndarray:
        return self._as_batch(super().mask())

    def get_state(self) -> np.ndarray:
        return self._as_batch(super().get_state())

    def macroscopic(self):
        drho, u = super().macroscopic()
        return self._as_batch(drho), self._as_batch(u)

    def init_equilibrium(self, drho0=None, u0=None) -> None:
        d = None if drho0 is None else np.reshape(drho0, self.shape)
        u = None if u0 is None else np.reshape(u0, (3,) + self.shape)
        super().init_equilibrium(d, u)

    def set_state(self, g) -> None:
        super().set_state(np.reshape(g, (19,) + self.shape))

    def set_shape(self, by: int, zper: int) -> None:
        self._check(library().lbm_batch_set_shape(self._h, int(by), int(zper)))

    def autotune(self, steps: int = 20):
        by = C.c_int32()
        zp = C.c_int32()
        ms = C.c_double()
        self._check(library().lbm_batch_autotune(self._h, int(steps), C.byref(by), C.byref(zp),
                                                 C.byref(ms)))
        return by.value, zp.value, ms.value

    def results(self):
        n = self.n_cells
        U = np.zeros((n, 3))
        K = np.zeros(n)
        steps = np.zeros(n, np.int64)
        res = np.zeros(n)
        status = np.zeros(n, np.int32)
        self._check(library().lbm_batch_results(self._h, _ptr(U), _ptr(K), _ptr(steps),
                                                _ptr(res), _ptr(status)))
        return dict(U=U, K_D=K, steps=steps, residual=res,
                    status=[BATCH_STATUS[int(v)] for v in status])

