"""Parity of the gfx950 library (through its C interface) with the FP64 CPU oracle.

Tolerance (FP64): 1e-12 relative on the h and q fields. Each coefficient plane is
compared against its field's scale: the depth planes (h0, h1x, h1y) against
max|h0|, the discharge planes against max(max|qx0|, max|qy0|), each at least 1e-3
(m, m^2/s). In still water the exact discharge is zero and both sides hold round-off
noise of about 1e-15 m^2/s there, so those cases compare each side's discharge with
zero (1e-12 m^2/s) and the depth planes with each other. The GPU evaluates the same formulas in a different order
(fused multiply-adds, reciprocals instead of divisions), which accounts for
differences of a few ulp per step.
"""
import os

import numpy as np
import pytest

import closed_forms as CF
import urban_window as UW
from oracle import Oracle
from paper_2107_02750_amd import scenarios as S

pytestmark = pytest.mark.gpu

TOL = 1e-12
# the time step is Cr dx / max(|q/h| + sqrt(g h)), usually set by one thin, fast cell
# where |q/h| turns an absolute difference of round-off size in q into a relative one
# up to ~1e-11; it is checked less tightly than the fields it is computed from
DT_TOL = 1e-10
FLOOR = 1e-3
G = 9.80665


@pytest.fixture(scope="module")
def dg2():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2107_02750_amd import dg2 as mod
    mod.load()
    return mod


def field_scales(b):
    H = max(np.abs(b[0]).max(), FLOOR)
    Q = max(np.abs(b[3]).max(), np.abs(b[6]).max(), FLOOR)
    return [H] * 3 + [Q] * 6


def rel_errs(a, b):
    sc = field_scales(b)
    return np.array([np.abs(a[p] - b[p]).max() / sc[p] for p in range(9)])


def assert_close(gpu, ref, tol=TOL, what="", still=False):
    a, b = gpu.planes(), ref.planes()
    e = rel_errs(a, b)
    if still:
        # still water: the exact discharge is zero and both sides hold round-off noise
        # (about 1e-15 m^2/s); each is compared with zero instead of with the other
        assert np.abs(a[3:]).max() <= tol and np.abs(b[3:]).max() <= tol, what
        e = e[:3]
    assert e.max() <= tol, f"{what}: per-plane relative errors {e}"
    return e.max()


def run_pair(dg2, sc, steps, tol=TOL, every=1, still=False):
    gpu = dg2.DG2(sc, dg2.FP64)
    ref = Oracle(sc)
    assert abs(gpu.next_dt() - ref.next_dt()) <= DT_TOL * ref.next_dt()
    for k in range(steps):
        a, b = gpu.step(), ref.step()
        assert abs(a - b) <= DT_TOL * b, (k, a, b)
        if (k + 1) % every == 0 or k + 1 == steps:
            assert_close(gpu, ref, tol, f"{sc.name} step {k + 1}", still)
    return gpu, ref


def thacker(nx):
    dx = 4.0 / nx
    xv = np.arange(nx + 1) * dx
    X, Y = np.meshgrid(xv, xv)
    h, u, v, z, _ = CF.thacker_bowl(X, Y, 0.0, 1.0, 0.1, 0.8, G, 2.0, 2.0)
    return S.Scenario("thacker", nx, nx, dx, z, S.MODE_VERTEX, np.stack([h, h * u, h * v]),
                      h_tol=1e-4)


def sloped_plane_inflow(nx=70, ny=23, dx=4.0):
    """A plane tilted in x and y, wet to 0.6 m with a moving sheet of water, fed by an
    inflow hydrograph on part of the west edge, open on the other edges: the limiter's
    ghosts on a sloping bed at every edge, and an inflow face in sub- and
    supercritical flow."""
    xv, yv = np.meshgrid(np.arange(nx + 1) * dx, np.arange(ny + 1) * dx)
    zv = -0.004 * xv - 0.0015 * yv + 0.02 * np.sin(xv / 13.0) * np.cos(yv / 7.0)
    hv = np.full_like(zv, 0.6)
    vert = np.stack([hv, np.full_like(zv, 0.4), np.full_like(zv, 0.1)])
    t = np.array([0.0, 20.0, 50.0])
    q = np.array([3.0, 12.0, 5.0])
    return S.Scenario("sloped_plane_inflow", nx, ny, dx, zv, S.MODE_VERTEX, vert,
                      manning_scalar=0.03, boundaries=[S.Boundary(S.W, S.INFLOW, 5, 15, t, q)])


def small_cases():
    return [
        S.dam_break(),
        S.lake_at_rest(),
        S.partially_dry_lake(),
        thacker(64),
        S.fbm_channel(n=96, dx=5.0, amplitude=60.0, wavelength=300.0, q_peak=20.0),
        S.urban_wet(n=96, n_blocks=25),
        S.fbm_channel_wet(n=80),
        sloped_plane_inflow(),
    ]


@pytest.mark.parametrize("idx", range(8))
def test_steps_match_oracle(dg2, idx):
    sc = small_cases()[idx]
    print(f"case {sc.name} {sc.nx}x{sc.ny}", flush=True)
    run_pair(dg2, sc, steps=30, every=5, still=sc.name in ("lake_at_rest", "partially_dry_lake"))


@pytest.mark.parametrize("shape", [(1, 1), (1, 37), (37, 1), (33, 9), (31, 7), (65, 17), (100, 3)])
def test_ragged_and_degenerate_grids(dg2, shape):
    nx, ny = shape
    rng = np.random.default_rng(nx * 1000 + ny)
    zv = rng.uniform(0.0, 0.3, size=(ny + 1, nx + 1))
    hv = np.maximum(0.5 - zv + 0.2 * rng.normal(size=zv.shape), 0.0)
    qx = 0.2 * rng.normal(size=zv.shape) * (hv > 0)
    qy = 0.2 * rng.normal(size=zv.shape) * (hv > 0)
    sc = S.Scenario(f"ragged{nx}x{ny}", nx, ny, 0.8, zv, S.MODE_VERTEX, np.stack([hv, qx, qy]),
                    manning_scalar=0.03, edge_kind=(S.WALL, S.TRANSMISSIVE, S.TRANSMISSIVE, S.WALL))
    print(f"case {sc.name}", flush=True)
    run_pair(dg2, sc, steps=12, every=3)


def test_all_boundary_kinds(dg2):
    sc = S.fbm_channel(n=72, dx=5.0, amplitude=50.0, wavelength=250.0, q_peak=15.0)
    t = np.array([0.0, 30.0, 60.0])
    q = np.array([2.0, 8.0, 1.0])
    sc = sc.replace(boundaries=sc.boundaries + [
        S.Boundary(S.S, S.FIXED, 10, 30, h_b=0.4, u_b=0.1, v_b=0.5),
        S.Boundary(S.N, S.WALL, 0, 72),
        S.Boundary(S.E, S.INFLOW, 20, 26, t, q),
    ], edge_kind=(S.WALL, S.TRANSMISSIVE, S.TRANSMISSIVE, S.TRANSMISSIVE))
    print("case boundary kinds", flush=True)
    gpu, ref = run_pair(dg2, sc, steps=40, every=10)
    a, b = gpu.scalars(), ref.scalars()
    for k in ("mass", "mass_in", "mass_out", "mass_clip"):
        assert abs(a[k] - b[k]) <= 1e-12 * max(abs(b[k]), 1.0), (k, a[k], b[k])


def test_dam_break_and_lake_full_runs(dg2):
    for sc in (S.dam_break(), S.lake_at_rest()):
        print(f"case {sc.name} run to {sc.t_end}", flush=True)
        gpu = dg2.DG2(sc, dg2.FP64)
        ref = Oracle(sc)
        assert gpu.run(sc.t_end) == ref.run(sc.t_end)
        assert gpu.scalars()["t"] == sc.t_end
        assert_close(gpu, ref, what=sc.name, still=sc.name == "lake_at_rest")
    assert np.abs(gpu.read(3)).max() <= 1e-12 and np.abs(gpu.read(9) - 1.0).max() <= 1e-12


def test_full_size_channel_terrain_all_wet(dg2):
    # the 1024 x 1024 terrain at the benchmark's launch configuration
    sc = S.fbm_channel_wet(n=1024)
    print("case fbm_channel_wet 1024x1024, 3 steps", flush=True)
    run_pair(dg2, sc, steps=3, every=1)


def test_full_size_urban_window_wet(dg2):
    sc = S.window(S.urban_wet(n=2048), 2048, 512)
    print("case urban_wet 2048x512 window, 2 steps", flush=True)
    run_pair(dg2, sc, steps=2, every=1)


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_configured_channel_window_from_oracle_snapshot(dg2):
    """The 1024 x 1024 channel terrain as configured (dry start, trapezoid inflow):
    100 steps from the oracle's own state at t = 3600 s (stored by
    tests/golden/make_snapshots.py, which runs the oracle only), loaded into both
    sides, compared every 10 steps. Water lies in the channel and on its banks only;
    the rest of the grid is dry."""
    d = np.load(os.path.join(GOLDEN, "fbm_channel_1024_t3600.npz"))
    nx, ny = int(d["nx"]), int(d["ny"])
    P = np.zeros((9, nx * ny))
    P[:, d["idx"]] = d["vals"]
    sc = S.fbm_channel(n=nx).replace(init_mode=S.MODE_PLANES, init_data=P.reshape(9, ny, nx),
                                     t0=float(d["t"]))
    assert sc.ny == ny
    print(f"case fbm_channel 1024x1024 from t={float(d['t']):.0f} s, {d['idx'].size} wet cells, "
          "100 steps", flush=True)
    gpu, ref = run_pair(dg2, sc, steps=100, every=10)
    a, b = gpu.scalars(), ref.scalars()
    for k in ("mass", "mass_out", "mass_clip"):
        assert abs(a[k] - b[k]) <= 1e-12 * max(abs(b[k]), 1.0), (k, a[k], b[k])


def test_configured_urban_window_from_oracle_state(dg2):
    """100 steps from the oracle's state at t = 300 s, loaded into both sides (the GPU
    runs the whole 2048 x 512 window), compared every 10 steps; the GPU's columns the
    water has not reached stay exactly zero."""
    print("case urban_blocks 2048x512 window: oracle to t=300 s", flush=True)
    base, cut, P = UW.state_at_t0()
    cutc = UW.CUT
    full = np.zeros((9, base.ny, base.nx))
    full[:, :, :cutc] = P
    gsc = base.replace(init_mode=S.MODE_PLANES, init_data=full, t0=300.0)
    rsc = cut.replace(init_mode=S.MODE_PLANES, init_data=P, t0=300.0)
    gpu, ref = dg2.DG2(gsc, dg2.FP64), Oracle(rsc)
    print(f"case urban_blocks window from t=300 s, {(P[0] > 0).sum()} wet cells, 100 steps",
          flush=True)
    for k in range(100):
        a, b = gpu.step(), ref.step()
        assert abs(a - b) <= DT_TOL * b, (k, a, b)
        if (k + 1) % 10 == 0:
            g = gpu.planes()
            e = rel_errs(g[:, :, :cutc], ref.planes())
            assert e.max() <= TOL, f"urban window step {k + 1}: per-plane relative errors {e}"
            assert not g[:, :, cutc - 32:].any()
    a, b = gpu.scalars(), ref.scalars()
    for k in ("mass", "mass_in", "mass_out", "mass_clip"):
        assert abs(a[k] - b[k]) <= 1e-12 * max(abs(b[k]), 1.0), (k, a[k], b[k])


@pytest.mark.parametrize("idx", [4, 5, 7])
def test_non_default_tile_shape_matches_oracle(dg2, idx):
    """The second FP64 tile shape (another block shape, other edge/interior tiles)
    against the oracle directly."""
    sc = small_cases()[idx]
    shape = dg2.tile_shapes(dg2.FP64)[1]
    print(f"case {sc.name} tile {shape}", flush=True)
    gpu = dg2.DG2(sc, dg2.FP64, tile=shape)
    assert (gpu.kernel_info()["tile_x"], gpu.kernel_info()["tile_y"]) == tuple(shape)
    ref = Oracle(sc)
    for k in range(30):
        a, b = gpu.step(), ref.step()
        assert abs(a - b) <= DT_TOL * b, (k, a, b)
        if (k + 1) % 5 == 0:
            assert_close(gpu, ref, TOL, f"{sc.name} tile {shape} step {k + 1}")


def test_determinism_and_checkpoint_resume(dg2):
    sc = S.fbm_channel(n=96, dx=5.0, amplitude=60.0, wavelength=300.0, q_peak=20.0)
    a = dg2.DG2(sc, dg2.FP64)
    a.run(120.0)
    blob = a.get_state()
    a.run(240.0)
    b = dg2.DG2(sc, dg2.FP64)
    b.set_state(blob)
    b.run(240.0)
    assert a.get_state() == b.get_state()
    c = dg2.DG2(sc, dg2.FP64)
    c.run(120.0)
    c.run(240.0)
    assert a.get_state() == c.get_state()


def test_mass_ledger_closes(dg2):
    sc = S.fbm_channel(n=128, dx=5.0, amplitude=60.0, wavelength=300.0, q_peak=20.0)
    gpu = dg2.DG2(sc, dg2.FP64)
    m0 = gpu.scalars()["mass"]
    gpu.run(600.0)
    s = gpu.scalars()
    assert s["mass_in"] > 100.0
    bal = s["mass"] - m0 - s["mass_in"] + s["mass_out"] - s["mass_clip"]
    assert abs(bal) <= 1e-12 * max(s["mass"], s["mass_in"])


def test_fp32_error_against_fp64_oracle(dg2):
    sc = S.dam_break()
    gpu = dg2.DG2(sc, dg2.FP32)
    ref = Oracle(sc)
    gpu.run(sc.t_end)
    ref.run(sc.t_end)
    h32, h64 = gpu.read(0).astype(np.float64), ref.read(0)
    err = np.abs(h32 - h64).max()
    print(f"FP32 dam break max depth error {err:.3e} m", flush=True)
    assert err <= 1e-4
    lake = dg2.DG2(S.lake_at_rest(), dg2.FP32)
    lake.run(2.5)
    assert np.abs(lake.read(3)).max() <= 1e-5


@pytest.mark.parametrize("plane", [0, 3])
def test_numeric_error_reported(dg2, plane):
    sc = S.dam_break(nx=40, ny=8)
    gpu = dg2.DG2(sc, dg2.FP64)
    blob = bytearray(gpu.get_state())
    # blob: 8 int64 header words (word 4 = tile count), 3 doubles, 4 ledger doubles per
    # tile, then the planes; overwrite cell 5 of one plane with a NaN
    n_tiles = int(np.frombuffer(bytes(blob[32:40]), dtype=np.int64)[0])
    off = 8 * 8 + 3 * 8 + n_tiles * 32 + 8 * (plane * sc.nx * sc.ny + 5)
    blob[off:off + 8] = np.array([np.nan]).tobytes()
    gpu.set_state(bytes(blob))
    with pytest.raises(dg2.DG2Error) as e:
        gpu.run(1.0)
    assert e.value.code == dg2.E_NUMERIC
