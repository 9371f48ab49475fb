"""FP32 with the bed stored relative to per-tile datums, against the FP64 oracle.

The FP32 path uses the bed only through differences that are exact in its quantised,
datum-relative storage. Three consequences are checked here:
  - raising the whole bed (and a still-water level) by a whole number of metres leaves
    every FP32 result bitwise unchanged;
  - still water stays still to FP32 round-off of the depth, however high the bed lies;
  - the depth error against the FP64 oracle is that of FP32 arithmetic on the depth,
    not of float elevations (ulp(1000 m) = 6.1e-5 m): 1 m deep flow rounds each
    operation at 6e-8 m, and some ten roundings per step over 40 steps bound the
    error by about 2.4e-5 m.
Mass: the FP32 state is summed in FP64; its drift from the FP64 ledger is reported and
bounded by the per-step rounding of the mean depths.
"""
import numpy as np
import pytest

import urban_window as UW
from oracle import Oracle
from paper_2107_02750_amd import scenarios as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dg2():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2107_02750_amd import dg2 as mod
    mod.load()
    return mod


def quantised_fbm(n=96, q=2.0 ** -12):
    """fBm channel terrain rounded to a 2^-12 m grid, so that adding whole metres is
    exact in double as well."""
    sc = S.fbm_channel(n=n, dx=5.0, amplitude=60.0, wavelength=300.0, q_peak=20.0)
    return sc.replace(zv=np.round(sc.zv / q) * q)


def raised(sc, dz):
    return sc.replace(zv=sc.zv + dz, eta_level=sc.eta_level + dz)


def urban_small():
    return S.window(S.urban_wet(n=512, n_blocks=250), 200, 136)


def test_bed_info(dg2):
    sc = urban_small()
    a = dg2.DG2(sc, dg2.FP32).bed_info()
    assert a["quantum"] > 0 and a["max_local"] / a["quantum"] <= 2.0 ** 20
    b = dg2.DG2(sc, dg2.FP32, bed_datum=False).bed_info()
    assert b["quantum"] == 0 and b["max_local"] == 10.0
    assert dg2.DG2(sc, dg2.FP64).bed_info()["quantum"] == 0


@pytest.mark.parametrize("case", ["urban", "fbm_inflow", "lake_level"])
def test_fp32_datum_results_invariant_under_bed_shift(dg2, case):
    if case == "urban":
        sc, steps = urban_small(), 40
    elif case == "fbm_inflow":
        sc, steps = quantised_fbm(), 60
    else:
        base = S.lake_at_rest()
        sc, steps = base.replace(zv=np.round(base.zv * 4096) / 4096), 40
    print(f"case {case} {sc.nx}x{sc.ny}", flush=True)
    a = dg2.DG2(sc, dg2.FP32)
    b = dg2.DG2(raised(sc, 1000.0), dg2.FP32)
    for k in range(steps):
        assert a.step() == b.step(), k
    assert np.array_equal(a.planes(), b.planes())
    sa, sb = a.scalars(), b.scalars()
    for key in ("mass", "mass_in", "mass_out", "mass_clip"):
        assert sa[key] == sb[key], key
    # the free surface is reported in absolute elevation
    ea, eb = a.read(9).astype(np.float64), b.read(9).astype(np.float64)
    wet = a.read(0) > sc.h_tol
    assert np.abs((eb - ea)[wet] - 1000.0).max() <= 1e-4


@pytest.mark.parametrize("case", ["urban", "fbm_inflow"])
def test_fv1_fp32_datum_invariant_under_bed_shift(dg2, case):
    """FV1 (Sect. 2.1.2) in FP32 reads each cell's bed mean from a plane formed at set-up
    in the frame of the cell's own tile datum and moves halo cells into the reading
    tile's frame by whole metres: raising the bed by 1000 m changes no bit."""
    sc = (urban_small() if case == "urban" else quantised_fbm()).as_fv1()
    print(f"case fv1 {case} {sc.nx}x{sc.ny}", flush=True)
    a = dg2.DG2(sc, dg2.FP32)
    b = dg2.DG2(raised(sc, 1000.0), dg2.FP32)
    for k in range(60):
        assert a.step() == b.step(), k
    assert np.array_equal(a.planes(), b.planes())
    sa, sb = a.scalars(), b.scalars()
    for key in ("mass", "mass_in", "mass_out", "mass_clip"):
        assert sa[key] == sb[key], key


@pytest.mark.parametrize("dz", [0.0, 1000.0])
def test_fv1_fp32_datum_depth_error_vs_fp64_oracle(dg2, dz):
    """FV1 in FP32 with bed datums against the FP64 oracle's FV1 on the urban blocks
    (fronts at the block walls) and on a raised bed: the error is that of FP32 depth
    arithmetic, as for DG2."""
    sc = raised(urban_small(), dz).as_fv1()
    ref = Oracle(sc)
    gpu = dg2.DG2(sc, dg2.FP32)
    for _ in range(80):
        ref.step()
    t = ref.scalars()["t"]
    gpu.run(t)
    assert abs(gpu.scalars()["t"] - t) <= 1e-9
    err = np.abs(gpu.read(0).astype(np.float64) - ref.read(0))
    print(f"FV1 urban +{dz} m, t={t:.2f} s: FP32 datum max depth error {err.max():.2e} m, "
          f"rms {np.sqrt(np.mean(err ** 2)):.2e} m", flush=True)
    assert err.max() <= 5e-5
    assert np.sqrt(np.mean(err ** 2)) <= 2e-6


def test_fp32_datum_lake_at_rest_high_bed(dg2):
    base = S.lake_at_rest()
    for dz in (0.0, 1500.0):
        sc = raised(base, dz)
        gpu = dg2.DG2(sc, dg2.FP32)
        gpu.run(2.5)
        q = max(np.abs(gpu.read(3)).max(), np.abs(gpu.read(6)).max())
        print(f"lake at rest, bed +{dz} m: max |q| {q:.2e}", flush=True)
        assert q <= 1e-5


@pytest.mark.parametrize("dz", [0.0, 1000.0])
def test_fp32_datum_depth_error_vs_fp64_oracle(dg2, dz):
    sc = raised(urban_small(), dz)
    ref = Oracle(sc)
    gpu = dg2.DG2(sc, dg2.FP32)
    for _ in range(40):
        ref.step()
    t = ref.scalars()["t"]
    gpu.run(t)
    assert abs(gpu.scalars()["t"] - t) <= 1e-9
    err = np.abs(gpu.read(0).astype(np.float64) - ref.read(0))
    print(f"urban +{dz} m, t={t:.2f} s: FP32 datum max depth error {err.max():.2e} m, "
          f"rms {np.sqrt(np.mean(err ** 2)):.2e} m", flush=True)
    assert err.max() <= 5e-5
    assert np.sqrt(np.mean(err ** 2)) <= 2e-6


def test_fp32_mass_ledger_drift(dg2):
    sc = quantised_fbm(n=128)
    gpu = dg2.DG2(sc, dg2.FP32)
    m0 = gpu.scalars()["mass"]
    steps = gpu.run(600.0)
    s = gpu.scalars()
    bal = s["mass"] - m0 - s["mass_in"] + s["mass_out"] - s["mass_clip"]
    scale = max(s["mass"], s["mass_in"])
    print(f"FP32 datum mass drift {bal / scale:.2e} over {steps} steps", flush=True)
    # each step rounds every wet mean depth once per stage (<= 2^-24 relative)
    assert abs(bal) <= steps * 2 * 2.0 ** -24 * scale


def test_fp32_urban_window_error_against_oracle(dg2):
    """The precision form's terrain as configured: FP32 with bed datums and the FP64
    oracle, both from the oracle's state at t = 300 s on a 2048 x 512 window (fronts at
    every block wall), 100 steps each on their own time steps to the same end time;
    the errors are printed (and recorded in the design notes)."""
    base, cut, P = UW.state_at_t0()
    full = np.zeros((9, base.ny, base.nx))
    full[:, :, :UW.CUT] = P
    gpu = dg2.DG2(base.replace(init_mode=S.MODE_PLANES, init_data=full, t0=UW.T0), dg2.FP32)
    ref = Oracle(cut.replace(init_mode=S.MODE_PLANES, init_data=P, t0=UW.T0))
    for _ in range(100):
        ref.step()
    t = ref.scalars()["t"]
    gpu.run(t)
    h = gpu.read(0).astype(np.float64)
    assert not h[:, UW.CUT - 32:].any()
    href = ref.read(0)
    err = np.abs(h[:, :UW.CUT] - href)
    wet = (href > 0) | (h[:, :UW.CUT] > 0)
    rms = float(np.sqrt(np.mean(err[wet] ** 2)))
    print(f"urban window t={t:.1f} s: FP32 datum vs FP64 oracle max depth error "
          f"{err.max():.2e} m, RMS over wet cells {rms:.2e} m", flush=True)
    assert err.max() <= 5e-2 and rms <= 1e-3


def test_fp32_non_default_tile_against_oracle(dg2):
    """The second FP32 tile shape against the FP64 oracle directly (as the default
    shape in the test above)."""
    sc = urban_small()
    shape = dg2.tile_shapes(dg2.FP32)[1]
    gpu = dg2.DG2(sc, dg2.FP32, tile=shape)
    assert (gpu.kernel_info()["tile_x"], gpu.kernel_info()["tile_y"]) == tuple(shape)
    ref = Oracle(sc)
    for _ in range(40):
        ref.step()
    t = ref.scalars()["t"]
    gpu.run(t)
    err = np.abs(gpu.read(0).astype(np.float64) - ref.read(0))
    print(f"urban, FP32 tile {shape}: max depth error {err.max():.2e} m", flush=True)
    assert err.max() <= 5e-5
    assert np.sqrt(np.mean(err ** 2)) <= 2e-6
