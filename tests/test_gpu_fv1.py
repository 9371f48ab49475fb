"""Parity of the gfx950 FV1 kernel (through the C interface) with the FP64 oracle's FV1
scheme (arXiv:2107.02750 Sect. 2.1.2, eq 5-7).

Tolerance (FP64): 1e-12 relative on the mean planes against the field scales (as for
DG2: depth against max h0, discharge against the larger of max |q0| and the discharge
of a wave of that depth); time steps to 1e-10; slope planes exactly zero.
"""
import numpy as np
import pytest

from oracle import Oracle
from paper_2107_02750_amd import scenarios as S

pytestmark = pytest.mark.gpu

TOL = 1e-12
DT_TOL = 1e-10
G = 9.80665


@pytest.fixture(scope="module")
def dg2():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2107_02750_amd import dg2 as mod
    mod.load()
    return mod


def rel_err(gpu, ref, still=False):
    """Depth against max|h0|, discharges against max(max|qx0|, max|qy0|), each floored
    at 1e-3 (m, m^2/s); in still water (exact discharge zero, round-off noise of about
    1e-15 m^2/s on both sides) each side's discharge is compared with zero instead."""
    a, b = gpu.planes(), ref.planes()
    assert not a[[1, 2, 4, 5, 7, 8]].any(), "FV1 slope planes must stay zero"
    H = max(np.abs(b[0]).max(), 1e-3)
    if still:
        return max(np.abs(a[0] - b[0]).max() / H, np.abs(a[[3, 6]]).max(), np.abs(b[[3, 6]]).max())
    Q = max(np.abs(b[3]).max(), np.abs(b[6]).max(), 1e-3)
    return max(np.abs(a[0] - b[0]).max() / H, np.abs(a[3] - b[3]).max() / Q,
               np.abs(a[6] - b[6]).max() / Q)


def run_pair(dg2, sc, steps, every=5, still=False):
    gpu, ref = dg2.DG2(sc, dg2.FP64), Oracle(sc)
    assert abs(gpu.next_dt() - ref.next_dt()) <= DT_TOL * ref.next_dt()
    for k in range(steps):
        a, b = gpu.step(), ref.step()
        assert abs(a - b) <= DT_TOL * b, (k, a, b)
        if (k + 1) % every == 0 or k + 1 == steps:
            e = rel_err(gpu, ref, still)
            assert e <= TOL, (sc.name, k + 1, e)
    return gpu, ref


def cases():
    t = np.array([0.0, 30.0, 60.0])
    q = np.array([2.0, 8.0, 1.0])
    fb = S.fbm_channel(n=72, dx=5.0, amplitude=50.0, wavelength=250.0, q_peak=15.0)
    mixed = fb.replace(boundaries=fb.boundaries + [
        S.Boundary(S.S, S.FIXED, 10, 30, h_b=0.4, u_b=0.1, v_b=0.5),
        S.Boundary(S.N, S.WALL, 0, 72),
        S.Boundary(S.E, S.INFLOW, 20, 26, t, q),
    ], edge_kind=(S.WALL, S.TRANSMISSIVE, S.TRANSMISSIVE, S.TRANSMISSIVE))
    return [S.dam_break(), S.lake_at_rest(), S.partially_dry_lake(),
            S.fbm_channel(n=96, dx=5.0, amplitude=60.0, wavelength=300.0, q_peak=20.0),
            S.window(S.urban_wet(n=256, n_blocks=60), 131, 77), S.fbm_channel_wet(n=80), mixed]


@pytest.mark.parametrize("idx", range(7))
def test_fv1_steps_match_oracle(dg2, idx):
    sc = cases()[idx].as_fv1()
    print(f"case {sc.name} {sc.nx}x{sc.ny}", flush=True)
    gpu, ref = run_pair(dg2, sc, steps=30, still=idx in (1, 2))
    if idx == 6:
        a, b = gpu.scalars(), ref.scalars()
        for k in ("mass", "mass_in", "mass_out", "mass_clip"):
            assert abs(a[k] - b[k]) <= 1e-12 * max(abs(b[k]), 1.0), (k, a[k], b[k])


@pytest.mark.parametrize("shape", [(1, 1), (1, 37), (37, 1), (33, 9), (65, 17), (100, 3)])
def test_fv1_ragged_and_degenerate_grids(dg2, shape):
    nx, ny = shape
    rng = np.random.default_rng(nx * 1000 + ny + 7)
    zv = rng.uniform(0.0, 0.3, size=(ny + 1, nx + 1))
    hv = np.maximum(0.5 - zv + 0.2 * rng.normal(size=zv.shape), 0.0)
    qx = 0.2 * rng.normal(size=zv.shape) * (hv > 0)
    qy = 0.2 * rng.normal(size=zv.shape) * (hv > 0)
    sc = S.Scenario(f"ragged{nx}x{ny}", nx, ny, 0.8, zv, S.MODE_VERTEX, np.stack([hv, qx, qy]),
                    manning_scalar=0.03,
                    edge_kind=(S.WALL, S.TRANSMISSIVE, S.TRANSMISSIVE, S.WALL)).as_fv1()
    print(f"case {sc.name}", flush=True)
    run_pair(dg2, sc, steps=12, every=3)


def test_fv1_full_run_resume_and_tile_shapes(dg2):
    sc = S.dam_break().as_fv1()
    gpu, ref = dg2.DG2(sc, dg2.FP64), Oracle(sc)
    assert gpu.run(sc.t_end) == ref.run(sc.t_end)
    assert gpu.scalars()["t"] == sc.t_end
    assert rel_err(gpu, ref) <= TOL
    sc = S.fbm_channel(n=96, dx=5.0, amplitude=60.0, wavelength=300.0, q_peak=20.0).as_fv1()
    a = dg2.DG2(sc, dg2.FP64)
    a.run(120.0)
    blob = a.get_state()
    a.run(240.0)
    b = dg2.DG2(sc, dg2.FP64)
    b.set_state(blob)
    b.run(240.0)
    assert a.get_state() == b.get_state()
    for shape in dg2.tile_shapes(dg2.FP64)[1:]:
        c = dg2.DG2(sc, dg2.FP64, tile=shape)
        c.run(120.0)  # the same schedule as a
        c.run(240.0)
        P, Q = c.planes(), a.planes()
        H = max(np.abs(Q[0]).max(), 1e-3)
        assert np.abs(P[0] - Q[0]).max() <= 1e-13 * H, shape


def test_fv1_mass_ledger_closes(dg2):
    sc = S.fbm_channel(n=128, dx=5.0, amplitude=60.0, wavelength=300.0, q_peak=20.0).as_fv1()
    gpu = dg2.DG2(sc, dg2.FP64)
    m0 = gpu.scalars()["mass"]
    gpu.run(600.0)
    s = gpu.scalars()
    assert s["mass_in"] > 100.0
    bal = s["mass"] - m0 - s["mass_in"] + s["mass_out"] - s["mass_clip"]
    assert abs(bal) <= 1e-12 * max(s["mass"], s["mass_in"])


def test_fv1_fp32_against_fp64_oracle(dg2):
    sc = S.dam_break().as_fv1()
    gpu, ref = dg2.DG2(sc, dg2.FP32), Oracle(sc)
    gpu.run(sc.t_end)
    ref.run(sc.t_end)
    err = np.abs(gpu.read(0).astype(np.float64) - ref.read(0)).max()
    print(f"FV1 FP32 dam break max depth error {err:.2e} m", flush=True)
    assert err <= 1e-4


def test_fv1_not_batched_and_nan_reported(dg2):
    import torch
    st = torch.cuda.Stream()
    sims = [dg2.DG2(S.dam_break(nx=20, ny=4).as_fv1(), dg2.FP64, stream=st)]
    with pytest.raises(dg2.DG2Error) as e:
        dg2.Batch(sims)
    assert e.value.code == dg2.E_ARG
    sc = S.dam_break(nx=40, ny=8).as_fv1()
    gpu = dg2.DG2(sc, dg2.FP64)
    blob = bytearray(gpu.get_state())
    n_tiles = int(np.frombuffer(bytes(blob[32:40]), dtype=np.int64)[0])
    off = 8 * 8 + 3 * 8 + n_tiles * 32 + 8 * 5
    blob[off:off + 8] = np.array([np.nan]).tobytes()
    gpu.set_state(bytes(blob))
    with pytest.raises(dg2.DG2Error) as e:
        gpu.run(1.0)
    assert e.value.code == dg2.E_NUMERIC
