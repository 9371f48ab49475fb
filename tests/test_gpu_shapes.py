"""Every tile shape the stage kernels are built for gives the same cell values, to
round-off.

Each face is computed from the same inputs by the same formulas whichever tile owns it.
The compiler fuses multiplies and adds into FMAs differently in the interior-tile and
edge-tile code paths (and in the own-cell and halo copies of the face code), so cells
that one shape computes in an edge tile and another in an interior tile can differ in
the last bit; with contraction disabled the planes agree bit for bit (measured), at a
cost of 2 % (FP64) and 9 % (FP32) in speed. The check is therefore, for FP64, 1e-13
relative to the field scales (the parity tolerance is 1e-12) and 1e-12 on time steps
and ledgers; for FP32, 1e-5 on the fields and ledgers and 1e-6 on time steps (a float
ulp of the state moves the float CFL candidate by ~6e-8). The default shape is checked against the FP64 oracle by the parity tests; this
carries that check over to the other shapes. The autotuner returns one of the shapes.
"""
import numpy as np
import pytest

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


def cases():
    sc = S.fbm_channel(n=72, dx=5.0, amplitude=50.0, wavelength=250.0, q_peak=15.0)
    t = np.array([0.0, 30.0, 60.0])
    q = np.array([2.0, 8.0, 1.0])
    mixed = sc.replace(boundaries=sc.boundaries + [
        S.Boundary(S.S, S.FIXED, 10, 30, h_b=0.4, u_b=0.1, v_b=0.5),
        S.Boundary(S.N, S.WALL, 0, 72),
        S.Boundary(S.E, S.INFLOW, 20, 26, t, q),
    ], edge_kind=(S.WALL, S.TRANSMISSIVE, S.TRANSMISSIVE, S.TRANSMISSIVE))
    return [mixed, S.window(S.urban_wet(n=256, n_blocks=60), 131, 77), S.dam_break(nx=37, ny=3)]


@pytest.mark.parametrize("prec_name", ["FP64", "FP32"])
@pytest.mark.parametrize("idx", range(3))
def test_shapes_give_identical_planes(dg2, prec_name, idx):
    prec = getattr(dg2, prec_name)
    sc = cases()[idx]
    shapes = dg2.tile_shapes(prec)
    assert len(shapes) >= 2
    print(f"case {sc.name} {prec_name} shapes {shapes}", flush=True)
    ref = dg2.DG2(sc, prec, bed_datum=False)
    dts = [ref.step() for _ in range(25)]
    P = ref.planes().astype(np.float64)
    m = ref.scalars()
    H = max(np.abs(P[0]).max(), 1e-3)
    Q = max(np.abs(P[3]).max(), np.abs(P[6]).max(), 1e-3)
    scale = np.array([H] * 3 + [Q] * 6)[:, None, None]
    tol = 1e-13 if prec == dg2.FP64 else 1e-5
    for shape in shapes[1:]:
        sim = dg2.DG2(sc, prec, bed_datum=False, tile=shape)
        assert sim.kernel_info()["tile_x"] == shape[0]
        d = [sim.step() for _ in range(25)]
        assert np.allclose(d, dts, rtol=1e-12 if prec == dg2.FP64 else 1e-6, atol=0), shape
        err = (np.abs(sim.planes() - P) / scale).max()
        assert err <= tol, (shape, err)
        s = sim.scalars()
        for k in ("mass", "mass_in", "mass_out", "mass_clip"):
            assert abs(s[k] - m[k]) <= (1e-12 if prec == dg2.FP64 else 1e-5) * max(abs(m[k]), 1.0), (shape, k)


def test_unknown_shape_rejected(dg2):
    with pytest.raises(dg2.DG2Error) as e:
        dg2.DG2(S.dam_break(nx=20, ny=4), dg2.FP64, tile=(24, 8))
    assert e.value.code == dg2.E_UNSUPPORTED


def test_autotuner_picks_a_built_shape(dg2):
    from paper_2107_02750_amd import autotune
    r = autotune.tune_scenario(S.fbm_channel_wet(n=256), dg2.FP64, steps=10)
    print(f"autotuner: {r}", flush=True)
    assert r["best"] in dg2.tile_shapes(dg2.FP64)
    assert len(r["ms_per_step"]) == len(dg2.tile_shapes(dg2.FP64))
