"""ctypes wrapper of the FP64 CPU oracle (oracle/libdg2ref.so).

TEST INFRASTRUCTURE ONLY: the plain, slow reference for the uniform-grid DG2 step of
arXiv:2107.02750 (Sect. 2.1.1, 2.1.4), and for its FV1 counterpart (Sect. 2.1.2),
that the GPU library is checked against. Only the
test suite, the package smoke check and the benchmark's CPU-baseline leg may use it.

Inputs are passed as plain arrays (a scenario object from the seeded generators supplies
them); nothing here is shared with the GPU library or its binding.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdg2ref.so")

_dp = C.POINTER(C.c_double)


class _Config(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("dx", C.c_double), ("g", C.c_double),
                ("cfl", C.c_double), ("h_tol", C.c_double), ("dt_dry", C.c_double),
                ("t0", C.c_double), ("limiter", C.c_int32), ("edge_kind", C.c_int32 * 4),
                ("scheme", C.c_int32)]


class _Boundary(C.Structure):
    _fields_ = [("edge", C.c_int32), ("kind", C.c_int32), ("i0", C.c_int32), ("i1", C.c_int32),
                ("n_knots", C.c_int32), ("t_knots", _dp), ("q_knots", _dp),
                ("h_b", C.c_double), ("u_b", C.c_double), ("v_b", C.c_double)]


TALLY_LIB_PATH = os.path.join(HERE, "libdg2ref_tally.so")
TALLY_NAMES = ("add", "mul", "div", "sqrt", "cbrt", "minmax", "abs", "cmp")

_libs = {}


def load(path: str = LIB_PATH):
    """The oracle library (or, with TALLY_LIB_PATH, its operation-tally build)."""
    if path in _libs:
        return _libs[path]
    if not os.path.exists(path):
        from . import build as _b
        _b.build()
    lib = C.CDLL(path)
    vp = C.c_void_p
    lib.dg2ref_init.argtypes = [C.POINTER(_Config), _dp, _dp, C.c_double, C.c_int32, _dp,
                                C.c_double, C.POINTER(_Boundary), C.c_int32, C.POINTER(vp)]
    lib.dg2ref_step.argtypes = [vp, C.c_double, _dp]
    lib.dg2ref_run.argtypes = [vp, C.c_double, C.POINTER(C.c_int64)]
    lib.dg2ref_read.argtypes = [vp, C.c_int32, _dp]
    lib.dg2ref_get_scalars.argtypes = [vp, _dp, C.POINTER(C.c_int64), _dp, _dp, _dp, _dp]
    lib.dg2ref_next_dt.argtypes = [vp, _dp]
    lib.dg2ref_state_doubles.argtypes = [vp]
    lib.dg2ref_state_doubles.restype = C.c_int64
    lib.dg2ref_get_state.argtypes = [vp, _dp]
    lib.dg2ref_set_state.argtypes = [vp, _dp]
    lib.dg2ref_last_error.argtypes = [vp]
    lib.dg2ref_last_error.restype = C.c_char_p
    lib.dg2ref_init_error.argtypes = []
    lib.dg2ref_init_error.restype = C.c_char_p
    lib.dg2ref_destroy.argtypes = [vp]
    lib.dg2ref_destroy.restype = None
    lib.dg2ref_hll.argtypes = [C.c_double] * 7 + [_dp]
    lib.dg2ref_hll.restype = None
    lib.dg2ref_friction_point.argtypes = [C.c_double] * 7 + [_dp]
    lib.dg2ref_friction_point.restype = None
    lib.dg2ref_bed_coeffs.argtypes = [C.c_int32, C.c_int32, _dp, _dp, _dp, _dp]
    lib.dg2ref_bed_coeffs.restype = None
    lib.dg2ref_operator.argtypes = [vp, _dp, C.c_double, _dp, _dp, _dp]
    lib.dg2ref_threads.argtypes = []
    lib.dg2ref_threads.restype = C.c_int
    lib.dg2ref_set_threads.argtypes = [C.c_int]
    lib.dg2ref_set_threads.restype = None
    lib.dg2ref_limit.argtypes = [vp, _dp, _dp]
    lib.dg2ref_friction.argtypes = [vp, _dp, C.c_double, _dp]
    if path == TALLY_LIB_PATH:
        lib.dg2ref_tally_read.argtypes = [C.POINTER(C.c_longlong)]
        lib.dg2ref_tally_read.restype = None
        lib.dg2ref_tally_reset.argtypes = []
        lib.dg2ref_tally_reset.restype = None
    _libs[path] = lib
    return lib


def _ptr(a):
    return a.ctypes.data_as(_dp) if a is not None else None


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


class OracleError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"oracle error {code}: {msg}")
        self.code = code


class Oracle:
    """One FP64 CPU simulation built from a scenario (see the seeded generators)."""

    PLANES = ("h0", "h1x", "h1y", "qx0", "qx1x", "qx1y", "qy0", "qy1x", "qy1y")

    def __init__(self, sc, tallied: bool = False):
        """tallied: run on the operation-tally build (tally_reset / tally_read)."""
        lib = load(TALLY_LIB_PATH if tallied else LIB_PATH)
        self._lib = lib
        self.nx, self.ny = int(sc.nx), int(sc.ny)
        cfg = _Config(self.nx, self.ny, sc.dx, sc.g, sc.cfl, sc.h_tol, sc.dt_dry, sc.t0,
                      int(sc.limiter), (C.c_int32 * 4)(*sc.edge_kind),
                      int(getattr(sc, "scheme", 0)))
        self._keep = []
        zv = _f64(sc.zv)
        man = _f64(sc.manning)
        data = _f64(sc.init_data)
        self._keep += [zv, man, data]
        nb = len(sc.boundaries)
        arr = (_Boundary * max(nb, 1))()
        for k, b in enumerate(sc.boundaries):
            tk, qk = _f64(b.t_knots), _f64(b.q_knots)
            self._keep += [tk, qk]
            arr[k] = _Boundary(b.edge, b.kind, b.i0, b.i1, 0 if tk is None else len(tk),
                               _ptr(tk), _ptr(qk), b.h_b, b.u_b, b.v_b)
        h = C.c_void_p()
        rc = lib.dg2ref_init(C.byref(cfg), _ptr(zv), _ptr(man), float(sc.manning_scalar),
                             int(sc.init_mode), _ptr(data), float(sc.eta_level), arr, nb,
                             C.byref(h))
        if rc != 0:
            raise OracleError(rc, lib.dg2ref_init_error().decode())
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.dg2ref_destroy(h)
            self._h = None

    def _check(self, rc):
        if rc != 0:
            raise OracleError(rc, self._lib.dg2ref_last_error(self._h).decode())

    def step(self, dt_max: float = 0.0) -> float:
        dt = C.c_double()
        self._check(self._lib.dg2ref_step(self._h, dt_max, C.byref(dt)))
        return dt.value

    def run(self, t_end: float) -> int:
        k = C.c_int64()
        self._check(self._lib.dg2ref_run(self._h, t_end, C.byref(k)))
        return k.value

    def read(self, field: int) -> np.ndarray:
        out = np.empty((self.ny, self.nx))
        self._check(self._lib.dg2ref_read(self._h, field, _ptr(out)))
        return out

    def planes(self) -> np.ndarray:
        return np.stack([self.read(p) for p in range(9)])

    def scalars(self) -> dict:
        t, m, mi, mo, mc = (C.c_double() for _ in range(5))
        st = C.c_int64()
        self._check(self._lib.dg2ref_get_scalars(self._h, C.byref(t), C.byref(st), C.byref(m),
                                                 C.byref(mi), C.byref(mo), C.byref(mc)))
        return dict(t=t.value, step=st.value, mass=m.value, mass_in=mi.value,
                    mass_out=mo.value, mass_clip=mc.value)

    def next_dt(self) -> float:
        d = C.c_double()
        self._check(self._lib.dg2ref_next_dt(self._h, C.byref(d)))
        return d.value

    def get_state(self) -> np.ndarray:
        out = np.empty(self._lib.dg2ref_state_doubles(self._h))
        self._check(self._lib.dg2ref_get_state(self._h, _ptr(out)))
        return out

    def set_state(self, s: np.ndarray) -> None:
        s = _f64(s)
        self._check(self._lib.dg2ref_set_state(self._h, _ptr(s)))

    def operator(self, state: np.ndarray, t: float):
        """L of a 9-plane state at time t, with the boundary inflow/outflow rates."""
        st = _f64(state).reshape(9, self.ny, self.nx)
        L = np.empty_like(st)
        ri, ro = C.c_double(), C.c_double()
        self._check(self._lib.dg2ref_operator(self._h, _ptr(st), t, _ptr(L), C.byref(ri),
                                              C.byref(ro)))
        return L, ri.value, ro.value

    def limit(self, state: np.ndarray) -> np.ndarray:
        st = _f64(state).reshape(9, self.ny, self.nx)
        out = np.empty_like(st)
        self._check(self._lib.dg2ref_limit(self._h, _ptr(st), _ptr(out)))
        return out

    def friction(self, state: np.ndarray, dt: float) -> np.ndarray:
        """The friction update alone (centre and Gauss points) of a 9-plane state."""
        st = _f64(state).reshape(9, self.ny, self.nx)
        out = np.empty_like(st)
        self._check(self._lib.dg2ref_friction(self._h, _ptr(st), float(dt), _ptr(out)))
        return out

    def tally_reset(self) -> None:
        self._lib.dg2ref_tally_reset()

    def tally_read(self) -> dict:
        """Floating-point operations done since the last reset, by kind (tally build
        only): add (with subtract), mul, div, sqrt, cbrt, min/max, abs, compare."""
        out = (C.c_longlong * len(TALLY_NAMES))()
        self._lib.dg2ref_tally_read(out)
        return dict(zip(TALLY_NAMES, (int(v) for v in out)))


def hll(g, hL, unL, utL, hR, unR, utR) -> np.ndarray:
    out = np.empty(3)
    load().dg2ref_hll(g, hL, unL, utL, hR, unR, utR, _ptr(out))
    return out


def friction_point(g, n, h_tol, dt, h, qx, qy) -> np.ndarray:
    out = np.empty(2)
    load().dg2ref_friction_point(g, n, h_tol, dt, h, qx, qy, _ptr(out))
    return out


def bed_coeffs(zv: np.ndarray):
    zv = _f64(zv)
    ny, nx = zv.shape[0] - 1, zv.shape[1] - 1
    z0, z1x, z1y = (np.empty((ny, nx)) for _ in range(3))
    load().dg2ref_bed_coeffs(nx, ny, _ptr(zv), _ptr(z0), _ptr(z1x), _ptr(z1y))
    return z0, z1x, z1y


def threads() -> int:
    """OpenMP threads the oracle's passes run on."""
    return int(load().dg2ref_threads())


def set_threads(n: int) -> None:
    """Run the oracle's passes on n OpenMP threads (from the calling thread on)."""
    load().dg2ref_set_threads(int(n))
