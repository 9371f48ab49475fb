"""Thin ctypes binding of the gfx950 DG2 library (libdg2.so, interface in include/dg2.h).

Argument marshalling only: every step of the method runs in the library's kernels.
PyTorch provides the device workspace (a uint8 tensor) and the HIP stream (torch's
current stream at construction). If the library has not been built, loading fails with
an error; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdg2.so")

FP64, FP32 = 0, 1
SCHEME_DG2, SCHEME_FV1 = 0, 1
OK, E_ARG, E_DEVICE, E_NUMERIC, E_STATE, E_UNSUPPORTED = 0, -1, -2, -3, -4, -5
MAX_SEGMENTS, MAX_KNOTS = 64, 8192
SYMBOLS = ("dg2_workspace_size", "dg2_init", "dg2_step", "dg2_run", "dg2_read",
           "dg2_get_scalars", "dg2_next_dt", "dg2_state_bytes", "dg2_get_state",
           "dg2_set_state", "dg2_set_timing", "dg2_get_timing", "dg2_kernel_info",
           "dg2_bed_info", "dg2_plan_bed_datum", "dg2_tile_shapes", "dg2_tile_grid",
           "dg2_batch_create",
           "dg2_batch_step", "dg2_batch_run", "dg2_batch_last_error", "dg2_batch_destroy",
           "dg2_set_manning", "dg2_set_hydrograph", "dg2_knot_count", "dg2_tape_create",
           "dg2_tape_forward",
           "dg2_tape_backward", "dg2_tape_last_error", "dg2_tape_destroy",
           "dg2_step_noalloc", "dg2_noalloc_last_error",
           "dg2_last_error", "dg2_init_error", "dg2_destroy")

_dp = C.POINTER(C.c_double)


class Config(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("dx", C.c_double), ("g", C.c_double),
                ("cfl", C.c_double), ("h_tol", C.c_double), ("dt_dry", C.c_double),
                ("t0", C.c_double), ("precision", C.c_int32), ("limiter", C.c_int32),
                ("edge_kind", C.c_int32 * 4), ("bed_datum", C.c_int32), ("tile_x", C.c_int32),
                ("tile_y", C.c_int32), ("scheme", C.c_int32)]


class Boundary(C.Structure):
    _fields_ = [("edge", C.c_int32), ("kind", C.c_int32), ("i0", C.c_int32), ("i1", C.c_int32),
                ("n_knots", C.c_int32), ("t_knots", _dp), ("q_knots", _dp),
                ("h_b", C.c_double), ("u_b", C.c_double), ("v_b", C.c_double)]


class DG2Error(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"dg2 error {code}: {msg}")
        self.code = code


_lib = None


def load(path: str = LIB_PATH):
    """Load libdg2.so and declare its signatures (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run __graft_entry__.build() first")
    # torch first: the process then has one HIP runtime, the one torch brings up, and
    # the library's device pointers and streams are torch's own
    import torch  # noqa: F401
    lib = C.CDLL(path)
    vp, sz = C.c_void_p, C.c_size_t
    i32, i64 = C.c_int32, C.c_int64
    lib.dg2_workspace_size.argtypes = [C.POINTER(Config), C.POINTER(sz)]
    lib.dg2_init.argtypes = [C.POINTER(Config), _dp, _dp, C.c_double, i32, _dp, C.c_double,
                             C.POINTER(Boundary), i32, vp, sz, vp, C.POINTER(vp)]
    lib.dg2_step.argtypes = [vp, C.c_double, _dp]
    lib.dg2_run.argtypes = [vp, C.c_double, C.POINTER(i64)]
    lib.dg2_read.argtypes = [vp, i32, vp, i32]
    lib.dg2_get_scalars.argtypes = [vp, _dp, C.POINTER(i64), _dp, _dp, _dp, _dp]
    lib.dg2_next_dt.argtypes = [vp, _dp]
    lib.dg2_state_bytes.argtypes = [vp, C.POINTER(sz)]
    lib.dg2_get_state.argtypes = [vp, vp]
    lib.dg2_set_state.argtypes = [vp, vp]
    lib.dg2_set_timing.argtypes = [vp, i32]
    lib.dg2_get_timing.argtypes = [vp, C.POINTER(i64), _dp, _dp]
    lib.dg2_kernel_info.argtypes = [vp] + [C.POINTER(i32)] * 5
    lib.dg2_bed_info.argtypes = [vp, _dp, _dp]
    lib.dg2_plan_bed_datum.argtypes = [C.POINTER(Config), _dp, _dp, _dp, _dp, _dp]
    lib.dg2_tile_grid.argtypes = [C.POINTER(Config)] + [C.POINTER(i32)] * 4
    lib.dg2_tile_shapes.argtypes = [i32, C.POINTER(i32), i32, C.POINTER(i32)]
    lib.dg2_last_error.argtypes = [vp]
    lib.dg2_last_error.restype = C.c_char_p
    lib.dg2_init_error.argtypes = []
    lib.dg2_init_error.restype = C.c_char_p
    lib.dg2_destroy.argtypes = [vp]
    lib.dg2_destroy.restype = None
    lib.dg2_batch_create.argtypes = [C.POINTER(vp), i32, i32, C.POINTER(vp)]
    lib.dg2_batch_step.argtypes = [vp, i32]
    lib.dg2_batch_run.argtypes = [vp, C.c_double, C.POINTER(i64), C.POINTER(i64)]
    lib.dg2_batch_last_error.argtypes = [vp]
    lib.dg2_batch_last_error.restype = C.c_char_p
    lib.dg2_batch_destroy.argtypes = [vp]
    lib.dg2_batch_destroy.restype = None
    lib.dg2_set_manning.argtypes = [vp, vp, i32]
    lib.dg2_set_hydrograph.argtypes = [vp, i32, _dp]
    lib.dg2_knot_count.argtypes = [vp, i32, C.POINTER(i32)]
    lib.dg2_tape_create.argtypes = [vp, i32, _dp, C.POINTER(i32), i32, i32, C.POINTER(vp)]
    lib.dg2_tape_forward.argtypes = [vp, vp, i32]
    lib.dg2_tape_backward.argtypes = [vp, vp, vp, _dp, vp, i32]
    lib.dg2_tape_last_error.argtypes = [vp]
    lib.dg2_tape_last_error.restype = C.c_char_p
    lib.dg2_tape_destroy.argtypes = [vp]
    lib.dg2_tape_destroy.restype = None
    lib.dg2_step_noalloc.argtypes = [C.POINTER(Config), vp, vp, C.c_double, C.POINTER(Boundary),
                                     i32, vp, vp, C.c_double, C.c_double, C.c_double, _dp, vp]
    lib.dg2_noalloc_last_error.argtypes = []
    lib.dg2_noalloc_last_error.restype = C.c_char_p
    _lib = lib
    return lib


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _boundaries(sc):
    """The boundary segments of a scenario as a C array, their count, and the host
    arrays the C array points into (to be kept alive while it is used)."""
    keep = []
    nb = len(sc.boundaries)
    arr = (Boundary * max(nb, 1))()
    for k, b in enumerate(sc.boundaries):
        tk, qk = _f64(b.t_knots), _f64(b.q_knots)
        keep += [tk, qk]
        arr[k] = Boundary(b.edge, b.kind, b.i0, b.i1, 0 if tk is None else len(tk),
                          _ptr(tk), _ptr(qk), b.h_b, b.u_b, b.v_b)
    return arr, nb, keep


def _is_device_tensor(a) -> bool:
    return type(a).__module__.startswith("torch") and getattr(a, "is_cuda", False)


def _check_device_f64(t, count: int) -> None:
    import torch
    if t.dtype != torch.float64 or t.numel() != count:
        raise DG2Error(E_ARG, f"expected {count} float64 values, got {t.numel()} {t.dtype}")


def _ptr(a):
    return a.ctypes.data_as(_dp) if a is not None else None


def make_config(sc, precision: int, bed_datum: bool | None = None, tile=None) -> Config:
    """The C configuration of a scenario. bed_datum (FP32 only) defaults to on; tile is
    a (tile_x, tile_y) pair from tile_shapes(precision), or None for the default."""
    if bed_datum is None:
        bed_datum = precision == FP32
    tx, ty = (0, 0) if tile is None else (int(tile[0]), int(tile[1]))
    return Config(int(sc.nx), int(sc.ny), float(sc.dx), float(sc.g), float(sc.cfl),
                  float(sc.h_tol), float(sc.dt_dry), float(sc.t0), int(precision),
                  int(sc.limiter), (C.c_int32 * 4)(*[int(k) for k in sc.edge_kind]),
                  int(bool(bed_datum)), tx, ty, int(getattr(sc, "scheme", 0)))


def tile_shapes(precision: int) -> list:
    """The (tile_x, tile_y) shapes the stage kernels are built for; the first is the
    default."""
    lib = load()
    n = C.c_int32()
    rc = lib.dg2_tile_shapes(int(precision), None, 0, C.byref(n))
    if rc != 0:
        raise DG2Error(rc, "tile shapes")
    xy = (C.c_int32 * (2 * n.value))()
    lib.dg2_tile_shapes(int(precision), xy, n.value, C.byref(n))
    return [(xy[2 * k], xy[2 * k + 1]) for k in range(n.value)]


def workspace_bytes(sc, precision: int = FP64, bed_datum: bool | None = None, tile=None) -> int:
    lib = load()
    cfg = make_config(sc, precision, bed_datum, tile)
    out = C.c_size_t()
    rc = lib.dg2_workspace_size(C.byref(cfg), C.byref(out))
    if rc != 0:
        raise DG2Error(rc, "workspace size")
    return out.value


def tile_grid(sc, precision: int, tile=None) -> dict:
    """Tile shape and tile counts of the stage kernels (host only)."""
    lib = load()
    cfg = make_config(sc, precision, tile=tile)
    v = [C.c_int32() for _ in range(4)]
    rc = lib.dg2_tile_grid(C.byref(cfg), *[C.byref(x) for x in v])
    if rc != 0:
        raise DG2Error(rc, "bad configuration")
    return dict(zip(("tile_x", "tile_y", "tiles_x", "tiles_y"), [x.value for x in v]))


def plan_bed_datum(sc) -> dict:
    """The FP32 datum plan of a scenario's bed, as dg2_init builds it (host only):
    stored relative bed, per-tile datums (tiles_y x tiles_x), quantum, largest local
    elevation."""
    lib = load()
    cfg = make_config(sc, FP32, True)
    tg = tile_grid(sc, FP32)
    zv = _f64(sc.zv)
    zrel = np.empty_like(zv)
    datum = np.empty((tg["tiles_y"], tg["tiles_x"]))
    q, b = C.c_double(), C.c_double()
    rc = lib.dg2_plan_bed_datum(C.byref(cfg), _ptr(zv), _ptr(zrel), _ptr(datum), C.byref(q),
                                C.byref(b))
    if rc != 0:
        raise DG2Error(rc, "bed datum plan")
    return dict(zrel=zrel, datum=datum, quantum=q.value, max_local=b.value, **tg)


class DG2:
    """One simulation on the GPU, built from a scenario (see the seeded generators):
    attributes nx, ny, dx, g, cfl, h_tol, dt_dry, t0, limiter, edge_kind, zv, manning,
    manning_scalar, init_mode, init_data, eta_level, boundaries. FP32 stores the bed
    relative to per-tile datums unless bed_datum is False; tile picks one of
    tile_shapes(precision) (default: the first)."""

    PLANES = ("h0", "h1x", "h1y", "qx0", "qx1x", "qx1y", "qy0", "qy1x", "qy1y")

    def __init__(self, sc, precision: int = FP64, device: str = "cuda:0", stream=None,
                 bed_datum: bool | None = None, tile=None):
        import torch
        lib = load()
        self._lib = lib
        self.nx, self.ny = int(sc.nx), int(sc.ny)
        self.precision = precision
        self.dtype = np.float32 if precision == FP32 else np.float64
        self.torch_dtype = torch.float32 if precision == FP32 else torch.float64
        self.device = torch.device(device)
        cfg = make_config(sc, precision, bed_datum, tile)
        ws = C.c_size_t()
        rc = lib.dg2_workspace_size(C.byref(cfg), C.byref(ws))
        if rc != 0:
            raise DG2Error(rc, "bad configuration")
        self.workspace = torch.empty(ws.value, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        zv, man, data = _f64(sc.zv), _f64(sc.manning), _f64(sc.init_data)
        arr, nb, keep = _boundaries(sc)
        keep += [zv, man, data]
        h = C.c_void_p()
        rc = lib.dg2_init(C.byref(cfg), _ptr(zv), _ptr(man), float(sc.manning_scalar),
                          int(sc.init_mode), _ptr(data), float(sc.eta_level), arr, nb,
                          C.c_void_p(self.workspace.data_ptr()), ws.value,
                          C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if rc != 0:
            raise DG2Error(rc, lib.dg2_init_error().decode())
        self._h = h

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.dg2_destroy(h)
            self._h = None

    def __del__(self):
        self.close()

    def _check(self, rc):
        if rc != 0:
            raise DG2Error(rc, self._lib.dg2_last_error(self._h).decode())

    def step(self, dt_max: float = 0.0, sync: bool = True):
        """One RK2 step; returns the dt taken if sync, else None (nothing waits)."""
        if sync:
            dt = C.c_double()
            self._check(self._lib.dg2_step(self._h, dt_max, C.byref(dt)))
            return dt.value
        self._check(self._lib.dg2_step(self._h, dt_max, None))
        return None

    def run(self, t_end: float) -> int:
        k = C.c_int64()
        self._check(self._lib.dg2_run(self._h, t_end, C.byref(k)))
        return k.value

    def read(self, field: int) -> np.ndarray:
        out = np.empty((self.ny, self.nx), dtype=self.dtype)
        self._check(self._lib.dg2_read(self._h, field, out.ctypes.data_as(C.c_void_p), 0))
        return out

    def read_device(self, field: int):
        import torch
        out = torch.empty((self.ny, self.nx), dtype=self.torch_dtype, device=self.device)
        self._check(self._lib.dg2_read(self._h, field, C.c_void_p(out.data_ptr()), 1))
        return out

    def planes(self) -> np.ndarray:
        return np.stack([self.read(p) for p in range(9)])

    def scalars(self) -> dict:
        t, m, mi, mo, mc = (C.c_double() for _ in range(5))
        st = C.c_int64()
        self._check(self._lib.dg2_get_scalars(self._h, C.byref(t), C.byref(st), C.byref(m),
                                              C.byref(mi), C.byref(mo), C.byref(mc)))
        return dict(t=t.value, step=st.value, mass=m.value, mass_in=mi.value,
                    mass_out=mo.value, mass_clip=mc.value)

    def next_dt(self) -> float:
        d = C.c_double()
        self._check(self._lib.dg2_next_dt(self._h, C.byref(d)))
        return d.value

    def get_state(self) -> bytes:
        n = C.c_size_t()
        self._check(self._lib.dg2_state_bytes(self._h, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        self._check(self._lib.dg2_get_state(self._h, buf))
        return buf.raw

    def set_state(self, blob: bytes) -> None:
        buf = C.create_string_buffer(blob, len(blob))
        self._check(self._lib.dg2_set_state(self._h, buf))

    def set_timing(self, on, every: int = 1) -> None:
        """Time the stage kernels of every `every`-th step with HIP events (off: on=False)."""
        self._check(self._lib.dg2_set_timing(self._h, int(every) if on else 0))

    def timing(self) -> dict:
        s = C.c_int64()
        a, b = C.c_double(), C.c_double()
        self._check(self._lib.dg2_get_timing(self._h, C.byref(s), C.byref(a), C.byref(b)))
        return dict(steps=s.value, ms_stage1=a.value, ms_stage2=b.value)

    def set_manning(self, manning) -> None:
        """Replace the per-cell Manning plane: a host array, or a float64 torch tensor
        on this simulation's device (used in place, nothing goes through the host)."""
        if _is_device_tensor(manning):
            m = manning.detach().contiguous().reshape(-1)
            _check_device_f64(m, self.ny * self.nx)
            self._check(self._lib.dg2_set_manning(self._h, C.c_void_p(m.data_ptr()), 1))
            return
        m = _f64(manning).reshape(-1)
        self._check(self._lib.dg2_set_manning(self._h, m.ctypes.data_as(C.c_void_p), 0))

    def knot_count(self, seg: int = -1) -> int:
        """Hydrograph knots of boundary segment seg (-1: all segments together)."""
        k = C.c_int32()
        self._check(self._lib.dg2_knot_count(self._h, int(seg), C.byref(k)))
        return k.value

    def set_hydrograph(self, seg: int, q_knots: np.ndarray) -> None:
        q = _f64(q_knots).reshape(-1)
        self._check(self._lib.dg2_set_hydrograph(self._h, int(seg), _ptr(q)))

    def bed_info(self) -> dict:
        q, b = C.c_double(), C.c_double()
        self._check(self._lib.dg2_bed_info(self._h, C.byref(q), C.byref(b)))
        return dict(quantum=q.value, max_local=b.value)

    def kernel_info(self) -> dict:
        v = [C.c_int32() for _ in range(5)]
        self._check(self._lib.dg2_kernel_info(self._h, *[C.byref(x) for x in v]))
        return dict(zip(("tile_x", "tile_y", "threads", "blocks", "lds_bytes"),
                        [x.value for x in v]))


class Batch:
    """Several DG2 simulations of one precision, created on one (non-default) stream,
    advanced together by shared launches replayed from a HIP graph of graph_steps steps.
    While the batch exists its members can be read but not stepped alone."""

    def __init__(self, sims, graph_steps: int = 16):
        lib = load()
        self._lib = lib
        self.sims = list(sims)
        arr = (C.c_void_p * len(self.sims))(*[s._h.value for s in self.sims])
        h = C.c_void_p()
        rc = lib.dg2_batch_create(arr, len(self.sims), int(graph_steps), C.byref(h))
        if rc != 0:
            raise DG2Error(rc, lib.dg2_batch_last_error(None).decode())
        self._h = h

    def _check(self, rc):
        if rc != 0:
            raise DG2Error(rc, self._lib.dg2_batch_last_error(self._h).decode())

    def step(self, steps: int = 1) -> None:
        """steps steps of every member (no host wait)."""
        self._check(self._lib.dg2_batch_step(self._h, int(steps)))

    def run(self, t_end: float):
        """Run every member to t_end; returns (steps per member, launch pairs)."""
        ms = (C.c_int64 * len(self.sims))()
        lp = C.c_int64()
        self._check(self._lib.dg2_batch_run(self._h, float(t_end), ms, C.byref(lp)))
        return [int(x) for x in ms], lp.value

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.dg2_batch_destroy(h)
            self._h = None

    def __del__(self):
        self.close()


class Tape:
    """A recorded forward run of a DG2 simulation (FP64, limiter off, fully wet) with
    prescribed time steps, and the discrete adjoint of that run. checkpoint_every:
    0 for ceil(sqrt(n_steps)), k for every k steps (the backward pass recomputes each
    segment once), -1 to keep every step's stage states (no recomputation)."""

    def __init__(self, sim: DG2, dts, gauges, checkpoint_every: int = 0):
        lib = load()
        self._lib = lib
        self.sim = sim
        self.dts = _f64(dts).reshape(-1)
        self.gauges = np.ascontiguousarray(gauges, dtype=np.int32).reshape(-1)
        self.n_steps, self.ng = len(self.dts), len(self.gauges)
        h = C.c_void_p()
        rc = lib.dg2_tape_create(sim._h, self.n_steps, _ptr(self.dts),
                                 self.gauges.ctypes.data_as(C.POINTER(C.c_int32)), self.ng,
                                 int(checkpoint_every), C.byref(h))
        if rc != 0:
            raise DG2Error(rc, lib.dg2_tape_last_error(None).decode())
        self._h = h

    def _check(self, rc):
        if rc != 0:
            raise DG2Error(rc, self._lib.dg2_tape_last_error(self._h).decode())

    def forward(self, device: bool = False):
        """Run the schedule; returns the gauge depths, (n_steps + 1) x n_gauges (a numpy
        array, or with device=True a float64 tensor on the simulation's device)."""
        if device:
            import torch
            out = torch.empty((self.n_steps + 1, max(self.ng, 1)), dtype=torch.float64,
                              device=self.sim.device)
            self._check(self._lib.dg2_tape_forward(self._h, C.c_void_p(out.data_ptr()), 1))
            return out[:, :self.ng]
        out = np.empty((self.n_steps + 1, self.ng))
        self._check(self._lib.dg2_tape_forward(self._h, out.ctypes.data_as(C.c_void_p), 0))
        return out

    def backward(self, dj_dh, n_knots: int | None = None):
        """dJ/d(gauge depths) -> (dJ/dn per cell, dJ/dq per knot, dJ/dU0). dJ/dq covers
        every knot of every segment in segment order (the first n_knots if given).
        A float64 device tensor dj_dh keeps dJ/dn and dJ/dU0 on the device (tensors);
        a host array gives numpy arrays."""
        nq = self.sim.knot_count(-1)
        gq = np.zeros(max(nq, 1))
        ny, nx = self.sim.ny, self.sim.nx
        if _is_device_tensor(dj_dh):
            import torch
            dj = dj_dh.detach().to(torch.float64).contiguous().reshape(-1)
            _check_device_f64(dj, (self.n_steps + 1) * self.ng)
            gm = torch.empty(ny * nx, dtype=torch.float64, device=self.sim.device)
            gu = torch.empty(9 * ny * nx, dtype=torch.float64, device=self.sim.device)
            self._check(self._lib.dg2_tape_backward(self._h, C.c_void_p(dj.data_ptr()),
                                                    C.c_void_p(gm.data_ptr()), _ptr(gq),
                                                    C.c_void_p(gu.data_ptr()), 1))
        else:
            dj = _f64(dj_dh).reshape(self.n_steps + 1, self.ng)
            gm = np.empty(ny * nx)
            gu = np.empty(9 * ny * nx)
            self._check(self._lib.dg2_tape_backward(self._h, dj.ctypes.data_as(C.c_void_p),
                                                    _ptr(gm), _ptr(gq),
                                                    gu.ctypes.data_as(C.c_void_p), 0))
        gq = gq[:nq] if n_knots is None else gq[:n_knots]
        return gm.reshape(ny, nx), gq, gu.reshape(9, ny, nx)

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.dg2_tape_destroy(h)
            self._h = None

    def __del__(self):
        self.close()


def gauge_run_function():
    """A torch.autograd.Function: (manning per cell, knots of segment 0) -> gauge depths
    over a recorded run, differentiated by the library's adjoint. Call as
    f.apply(manning, q_knots, sim, dts, gauges, state0) with state0 the initial state
    blob (the simulation is reset to it before each forward)."""
    import torch

    class GaugeRun(torch.autograd.Function):
        @staticmethod
        def forward(ctx, manning, q_knots, sim, dts, gauges, state0):
            sim.set_state(state0)
            sim.set_manning(manning.detach().to(device=sim.device, dtype=torch.float64))
            sim.set_hydrograph(0, q_knots.detach().cpu().numpy())  # a few knots
            tape = Tape(sim, dts, gauges)
            gh = tape.forward(device=True)
            ctx.tape = tape
            ctx.n_knots = int(q_knots.numel())
            ctx.shapes = (manning.shape, manning.dtype, manning.device)
            return gh.to(dtype=manning.dtype, device=manning.device)

        @staticmethod
        def backward(ctx, g):
            gm, gq, _ = ctx.tape.backward(g.detach().to(device=ctx.tape.sim.device,
                                                          dtype=torch.float64), ctx.n_knots)
            ctx.tape.close()
            shape, dtype, dev = ctx.shapes
            return (gm.to(dtype=dtype, device=dev).reshape(shape),
                    torch.as_tensor(gq, dtype=dtype, device=dev), None, None, None, None)

    return GaugeRun


def step_noalloc(sc, zv, u_in, u_out, t: float, dt_max: float = 0.0,
                 t_end: float = float("inf"), manning=None, stream=None, sync: bool = True):
    """One FP64 DG2 step from the 9-plane state u_in to u_out through the entry point
    that allocates nothing (dg2_step_noalloc): zv ((ny+1) x (nx+1)), manning (ny x nx,
    or None for the scenario's scalar), u_in and u_out (9 x ny x nx) are float64 device
    tensors owned by the caller; the grid, edges and boundary segments come from the
    scenario. Returns the time step taken if sync, else None (nothing waits)."""
    import torch
    lib = load()
    cfg = make_config(sc, FP64)
    for a, count in ((zv, (sc.ny + 1) * (sc.nx + 1)), (u_in, 9 * sc.ny * sc.nx),
                     (u_out, 9 * sc.ny * sc.nx)) + (() if manning is None else ((manning, sc.ny * sc.nx),)):
        if not _is_device_tensor(a) or not a.is_contiguous():
            raise DG2Error(E_ARG, "device tensors (contiguous) expected")
        _check_device_f64(a, count)
    arr, nb, keep = _boundaries(sc)
    st = stream if stream is not None else torch.cuda.current_stream(u_in.device)
    dt = C.c_double()
    rc = lib.dg2_step_noalloc(C.byref(cfg), C.c_void_p(zv.data_ptr()),
                              C.c_void_p(manning.data_ptr()) if manning is not None else None,
                              float(sc.manning_scalar), arr, nb, C.c_void_p(u_in.data_ptr()),
                              C.c_void_p(u_out.data_ptr()), float(t), float(dt_max), float(t_end),
                              C.byref(dt) if sync else None, C.c_void_p(st.cuda_stream))
    del keep
    if rc != 0:
        raise DG2Error(rc, lib.dg2_noalloc_last_error().decode())
    return dt.value if sync else None
