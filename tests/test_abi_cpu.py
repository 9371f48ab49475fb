"""The GPU library loads, exports every symbol include/dg2.h declares, and rejects bad
arguments before it touches a device (no compute calls; runs without a GPU)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2107_02750_amd import dg2, scenarios as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "dg2.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dg2_[a-z_]+)\s*\(", text)))


def test_header_symbols_exported():
    lib = dg2.load()
    names = _declared()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(dg2.SYMBOLS) == names


def test_oracle_is_a_separate_library():
    # the product binding never loads the oracle, and they share no source
    src = open(os.path.join(ROOT, "paper_2107_02750_amd", "dg2.py")).read()
    assert "oracle" not in src.replace("no fallback", "")
    for f in os.listdir(os.path.join(ROOT, "paper_2107_02750_amd", "csrc")):
        body = open(os.path.join(ROOT, "paper_2107_02750_amd", "csrc", f)).read()
        assert "dg2ref" not in body


def test_workspace_size_scales_with_grid_and_precision():
    sc = S.dam_break(nx=100, ny=60)
    a = dg2.workspace_bytes(sc, dg2.FP64)
    b = dg2.workspace_bytes(sc, dg2.FP32)
    big = dg2.workspace_bytes(S.dam_break(nx=200, ny=60), dg2.FP64)
    assert a > b > 0 and big > a
    assert a >= 27 * 100 * 60 * 8   # three 9-plane FP64 buffers at least


def _init(sc, precision=dg2.FP64, ws=None, ws_bytes=0, **over):
    lib = dg2.load()
    cfg = dg2.make_config(sc, precision)
    for k, v in over.items():
        setattr(cfg, k, v)
    zv = np.ascontiguousarray(sc.zv, dtype=np.float64)
    data = None if sc.init_data is None else np.ascontiguousarray(sc.init_data, dtype=np.float64)
    bcs = (dg2.Boundary * max(len(sc.boundaries), 1))()
    keep = []
    for k, b in enumerate(sc.boundaries):
        tk = None if b.t_knots is None else np.ascontiguousarray(b.t_knots, dtype=np.float64)
        qk = None if b.q_knots is None else np.ascontiguousarray(b.q_knots, dtype=np.float64)
        keep += [tk, qk]
        bcs[k] = dg2.Boundary(b.edge, b.kind, b.i0, b.i1, 0 if tk is None else len(tk),
                              None if tk is None else tk.ctypes.data_as(C.POINTER(C.c_double)),
                              None if qk is None else qk.ctypes.data_as(C.POINTER(C.c_double)),
                              b.h_b, b.u_b, b.v_b)
    h = C.c_void_p()
    rc = lib.dg2_init(C.byref(cfg), zv.ctypes.data_as(C.POINTER(C.c_double)), None,
                      float(sc.manning_scalar), int(sc.init_mode),
                      None if data is None else data.ctypes.data_as(C.POINTER(C.c_double)),
                      float(sc.eta_level), bcs, len(sc.boundaries), ws, ws_bytes, None,
                      C.byref(h))
    return rc, lib.dg2_init_error().decode(), h


def test_bad_arguments_rejected_before_device_work():
    sc = S.dam_break(nx=20, ny=8)
    # a valid set-up without a workspace fails only at the workspace check
    rc, msg, h = _init(sc)
    assert rc == dg2.E_ARG and "workspace" in msg and not h.value
    assert _init(sc, nx=0)[0] == dg2.E_ARG
    assert _init(sc, precision=7)[0] == dg2.E_ARG
    assert _init(sc, dx=-1.0)[0] == dg2.E_ARG
    assert _init(sc, cfl=0.0)[0] == dg2.E_ARG
    neg = sc.init_data.copy()
    neg[0, 3, 3] = -0.1
    rc, msg, _ = _init(sc.replace(init_data=neg))
    assert rc == dg2.E_ARG and "negative" in msg
    nanz = sc.zv.copy()
    nanz[2, 2] = np.nan
    assert _init(sc.replace(zv=nanz))[0] == dg2.E_ARG
    t = np.array([0.0, 10.0, 5.0])
    q = np.array([1.0, 2.0, 3.0])
    rc, msg, _ = _init(sc.replace(boundaries=[S.Boundary(S.W, S.INFLOW, 0, 4, t, q)]))
    assert rc == dg2.E_ARG and "increasing" in msg
    rc, msg, _ = _init(sc.replace(boundaries=[S.Boundary(S.N, S.WALL, 0, 30)]))
    assert rc == dg2.E_ARG and "range" in msg
    both = [S.Boundary(S.W, S.WALL, 0, 4), S.Boundary(S.W, S.FIXED, 3, 6, h_b=1.0)]
    rc, msg, _ = _init(sc.replace(boundaries=both))
    assert rc == dg2.E_ARG and "overlap" in msg
    rc, msg, _ = _init(sc, edge_kind=(C.c_int32 * 4)(3, 0, 0, 0))
    assert rc == dg2.E_ARG


def test_tile_shapes_and_grid():
    for prec in (dg2.FP64, dg2.FP32):
        shapes = dg2.tile_shapes(prec)
        assert len(shapes) == 4 and len(set(shapes)) == 4
        for tx, ty in shapes:
            assert (tx * ty) % 64 == 0 and tx * ty <= 1024
            g = dg2.tile_grid(S.dam_break(nx=100, ny=37), prec, tile=(tx, ty))
            assert (g["tile_x"], g["tile_y"]) == (tx, ty)
            assert g["tiles_x"] == -(-100 // tx) and g["tiles_y"] == -(-37 // ty)
        assert dg2.tile_grid(S.dam_break(), prec)["tile_x"] == shapes[0][0]
    with pytest.raises(dg2.DG2Error) as e:
        dg2.workspace_bytes(S.dam_break(), dg2.FP64, tile=(24, 8))
    assert e.value.code == dg2.E_UNSUPPORTED


def test_grid_size_limit():
    """Up to 2^31 cells are accepted (32-bit cell indices) and sized in 64-bit byte
    counts; one more row is refused."""
    lib = dg2.load()
    for prec, rs in ((dg2.FP64, 8), (dg2.FP32, 4)):
        cfg = dg2.make_config(S.dam_break(nx=20, ny=8), prec)
        cfg.nx, cfg.ny = 65536, 32768
        out = C.c_size_t()
        assert lib.dg2_workspace_size(C.byref(cfg), C.byref(out)) == dg2.OK
        n = 65536 * 32768
        assert out.value >= 29 * n * rs and out.value < 29 * n * rs + (1 << 30)
        cfg.ny = 32769
        assert lib.dg2_workspace_size(C.byref(cfg), C.byref(out)) == dg2.E_UNSUPPORTED
