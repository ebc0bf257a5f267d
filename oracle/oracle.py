"""ctypes wrapper around the plain-C FP64 oracle (``lbm_oracle.c``).

Test infrastructure only.  Array conventions follow ``lbm_oracle.h``:
populations are deviations ``g = f - w`` stored as ``g[k, z, y, x]``
(structure of arrays, x fastest), the mask is ``mask[z, y, x]`` with 1 = solid,
spheres are rows ``(cx, cy, cz, r)`` in lattice units.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_LIB = os.path.join(_HERE, "liblbm_oracle.so")

COLLISIONS = {"srt": 0, "trt": 1, "mrt": 2}
WALLS = {"sbb": 0, "cli": 1, "libb": 2, "qibb": 3, "iebb": 4, "mr": 5}


def library_path() -> str:
    return _LIB


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C, no contraction of a*b+c)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-Wall", "-shared", "-fPIC", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Params(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("tau", C.c_double), ("magic", C.c_double), ("drho", C.c_double),
                ("collision", C.c_int32), ("wall", C.c_int32)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = C.CDLL(_LIB)
        P = C.POINTER
        d, i32, i64 = C.c_double, C.c_int32, C.c_int64
        vp = C.c_void_p
        sigs = {
            "orc_lattice": (None, [vp, vp, vp]),
            "orc_mrt_matrix": (None, [vp, vp, vp]),
            "orc_mrt_rates": (None, [d, vp]),
            "orc_trt_omega_minus": (d, [d, d]),
            "orc_equilibrium": (None, [d, vp, vp]),
            "orc_collide": (None, [P(_Params), vp]),
            "orc_collide_mrt_rates": (None, [vp, vp]),
            "orc_voxelise": (i64, [i32, i32, i32, vp, i32, vp]),
            "orc_link_q": (d, [i32, i32, i32, vp, i32, i32, i32, i32, i32]),
            "orc_wall_q": (i64, [i32, i32, i32, vp, vp, i32, vp]),
            "orc_init": (None, [P(_Params), vp, vp, vp, vp]),
            "orc_step": (None, [P(_Params), vp, vp, vp, vp]),
            "orc_run": (None, [P(_Params), vp, vp, vp, vp, i64]),
            "orc_macroscopic": (None, [P(_Params), vp, vp, vp, vp]),
            "orc_mean_velocity": (None, [P(_Params), vp, vp, vp]),
            "orc_drag": (None, [P(_Params), vp, vp, vp, vp]),
            "orc_wall_value": (d, [P(_Params), vp, vp, vp, i32, i32, i32, i32]),
            "orc_permeability": (d, [P(_Params), d]),
            "orc_run_to_residual": (i32, [P(_Params), vp, vp, vp, vp, d, i64, i64,
                                          P(i64), P(d)]),
            "orc_set_threads": (None, [i32]),
        }
        for name, (res, args) in sigs.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def set_threads(n: int) -> None:
    """Threads of the oracle's time step (1 unless set; results do not
    depend on it)."""
    _load().orc_set_threads(int(n))


def _ptr(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def lattice():
    """(e[19,3] int32, w[19], opp[19] int32) as the oracle defines them."""
    lib = _load()
    e = np.zeros((19, 3), np.int32)
    w = np.zeros(19)
    opp = np.zeros(19, np.int32)
    lib.orc_lattice(_ptr(e), _ptr(w), _ptr(opp))
    return e, w, opp


def mrt_matrix():
    lib = _load()
    M = np.zeros((19, 19))
    Minv = np.zeros((19, 19))
    n2 = np.zeros(19)
    lib.orc_mrt_matrix(_ptr(M), _ptr(Minv), _ptr(n2))
    return M, Minv, n2


def mrt_rates(tau: float) -> np.ndarray:
    s = np.zeros(19)
    _load().orc_mrt_rates(float(tau), _ptr(s))
    return s


def trt_omega_minus(tau: float, magic: float) -> float:
    return _load().orc_trt_omega_minus(float(tau), float(magic))


def equilibrium(drho: float, u) -> np.ndarray:
    u = _f64(u)
    geq = np.zeros(19)
    _load().orc_equilibrium(float(drho), _ptr(u), _ptr(geq))
    return geq


def _params(shape, tau, magic, drho, collision, wall) -> _Params:
    nz, ny, nx = shape
    return _Params(nx, ny, nz, float(tau), float(magic), float(drho),
                   COLLISIONS[collision], WALLS[wall])


def collide(g, tau: float, collision: str = "trt", magic: float = 3 / 16) -> np.ndarray:
    g = _f64(g).copy()
    p = _params((1, 1, 1), tau, magic, 0.0, collision, "sbb")
    _load().orc_collide(C.byref(p), _ptr(g))
    return g


def collide_mrt_rates(g, s) -> np.ndarray:
    g = _f64(g).copy()
    s = _f64(s)
    _load().orc_collide_mrt_rates(_ptr(s), _ptr(g))
    return g


def voxelise(shape, spheres) -> np.ndarray:
    nz, ny, nx = shape
    sp = _f64(np.reshape(spheres, (-1, 4))) if len(spheres) else np.zeros((0, 4))
    mask = np.zeros(shape, np.uint8)
    _load().orc_voxelise(nx, ny, nz, _ptr(sp), sp.shape[0], _ptr(mask))
    return mask


def link_q(shape, spheres, x: int, y: int, z: int, j: int) -> float:
    nz, ny, nx = shape
    sp = _f64(np.reshape(spheres, (-1, 4)))
    return _load().orc_link_q(nx, ny, nz, _ptr(sp), sp.shape[0], x, y, z, j)


def wall_q(mask: np.ndarray, spheres=None) -> np.ndarray:
    """Dense q table Q[j, z, y, x] (-1 where (cell, j) is not a wall link)."""
    nz, ny, nx = mask.shape
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    sp = (_f64(np.reshape(spheres, (-1, 4))) if spheres is not None and len(spheres)
          else np.zeros((0, 4)))
    Q = np.zeros((19,) + mask.shape)
    _load().orc_wall_q(nx, ny, nz, _ptr(mask), _ptr(sp), sp.shape[0], _ptr(Q))
    return Q


class Oracle:
    """A periodic D3Q19 domain advanced by the oracle.

    Either ``mask`` (uint8[nz, ny, nx], 1 = solid; every wall link gets q = 1/2)
    or ``spheres`` (rows cx, cy, cz, r) defines the solid.
    """

    def __init__(self, shape, *, tau: float, magic: float = 3 / 16,
                 delta_rho: float = 0.0, collision: str = "trt", wall: str = "sbb",
                 mask: np.ndarray | None = None, spheres=None):
        self.shape = tuple(int(s) for s in shape)
        self.ncell = int(np.prod(self.shape))
        self.spheres = (np.zeros((0, 4)) if spheres is None
                        else _f64(np.reshape(spheres, (-1, 4))))
        if mask is None:
            mask = voxelise(self.shape, self.spheres)
        self.mask = np.ascontiguousarray(mask, dtype=np.uint8)
        assert self.mask.shape == self.shape
        self.p = _params(self.shape, tau, magic, delta_rho, collision, wall)
        self.Q = wall_q(self.mask, self.spheres)
        self.g = np.zeros((19,) + self.shape)
        self._work = np.zeros_like(self.g)
        self.steps = 0

    @property
    def tau(self):
        return self.p.tau

    def init(self, drho0=None, u0=None) -> None:
        d = None if drho0 is None else _f64(np.broadcast_to(drho0, self.shape))
        u = None if u0 is None else _f64(np.broadcast_to(u0, (3,) + self.shape))
        _load().orc_init(C.byref(self.p), _ptr(self.mask), _ptr(d), _ptr(u), _ptr(self.g))
        self.steps = 0

    def set_state(self, g) -> None:
        g = _f64(g).reshape((19,) + self.shape).copy()
        g[:, self.mask.astype(bool)] = 0.0
        self.g = g

    def step(self, n: int = 1) -> None:
        if n <= 0:
            return
        _load().orc_run(C.byref(self.p), _ptr(self.mask), _ptr(self.Q), _ptr(self.g),
                        _ptr(self._work), int(n))
        self.steps += n

    def macroscopic(self):
        drho = np.zeros(self.shape)
        u = np.zeros((3,) + self.shape)
        _load().orc_macroscopic(C.byref(self.p), _ptr(self.mask), _ptr(self.g),
                                _ptr(drho), _ptr(u))
        return drho, u

    def mean_velocity(self) -> np.ndarray:
        U = np.zeros(3)
        _load().orc_mean_velocity(C.byref(self.p), _ptr(self.mask), _ptr(self.g), _ptr(U))
        return U

    def wall_value(self, x: int, y: int, z: int, k: int) -> float:
        """Incoming value of direction k at fluid node (x, y, z) whose pull
        source is solid, from the current state by the wall rule."""
        return _load().orc_wall_value(C.byref(self.p), _ptr(self.mask), _ptr(self.Q),
                                      _ptr(self.g), x, y, z, k)

    def drag(self) -> np.ndarray:
        F = np.zeros(3)
        _load().orc_drag(C.byref(self.p), _ptr(self.mask), _ptr(self.Q), _ptr(self.g),
                         _ptr(F))
        return F

    def permeability(self, U: float | None = None) -> float:
        if U is None:
            U = self.mean_velocity()[0]
        return _load().orc_permeability(C.byref(self.p), float(U))

    def run_to_residual(self, tol: float, max_steps: int, interval: int = 100):
        done = C.c_int64(0)
        res = C.c_double(0.0)
        st = _load().orc_run_to_residual(C.byref(self.p), _ptr(self.mask), _ptr(self.Q),
                                         _ptr(self.g), _ptr(self._work), float(tol),
                                         int(max_steps), int(interval), C.byref(done),
                                         C.byref(res))
        self.steps += done.value
        return {0: "converged", 1: "not_converged", 2: "unstable"}[st], done.value, res.value
