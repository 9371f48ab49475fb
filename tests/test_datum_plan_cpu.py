"""Host logic of the FP32 bed datum (no GPU): the plan dg2_init builds is checked here
for the properties the FP32 kernels rely on, recomputed with numpy float32:
  - each tile's datum is a whole number of metres and every stored value is a float;
  - in every tile's frame (stored value + owner datum - tile datum, summed in float32)
    each bed elevation the tile reads is exact, as are the cell means (eq 8, summed in
    diagonal pairs), the face means and the differences of neighbouring cell means;
  - the stored bed moves by at most half a quantum;
  - raising the bed by whole metres raises every datum by the same amount and leaves
    the stored bed unchanged.
"""
import numpy as np
import pytest

from paper_2107_02750_amd import dg2, scenarios as S


def frames(sc, plan):
    """Yield, per tile, the float32 bed of the vertices it reads in its own frame and
    the exact (float64) values they must equal."""
    nx, ny = sc.nx, sc.ny
    tx, ty = plan["tile_x"], plan["tile_y"]
    d = plan["datum"]
    iv = np.minimum(np.arange(nx + 1), nx - 1) // tx
    jv = np.minimum(np.arange(ny + 1), ny - 1) // ty
    own = d[jv[:, None], iv[None, :]]
    absq = plan["zrel"] + own          # the quantised absolute bed (exact in float64)
    zr32 = plan["zrel"].astype(np.float32)
    own32 = own.astype(np.float32)
    for tj in range(d.shape[0]):
        for ti in range(d.shape[1]):
            a0, a1 = max(ti * tx - 2, 0), min(ti * tx + tx + 2, nx)
            b0, b1 = max(tj * ty - 2, 0), min(tj * ty + ty + 2, ny)
            box = np.s_[b0:b1 + 1, a0:a1 + 1]
            dT = d[tj, ti]
            z32 = zr32[box] + (own32[box] - np.float32(dT))
            yield z32, absq[box] - dT


def cell_means(z, f32):
    c = np.float32 if f32 else np.float64
    return c(0.25) * ((z[1:, 1:] + z[:-1, :-1]) + (z[1:, :-1] + z[:-1, 1:]))


@pytest.mark.parametrize("make", [
    lambda: S.fbm_channel_wet(n=200),
    lambda: S.urban_wet(n=256, n_blocks=60),
    lambda: S.lake_at_rest(),
    lambda: S.dam_break(nx=37, ny=5),
])
def test_plan_is_exact_in_every_tile_frame(make):
    sc = make()
    plan = dg2.plan_bed_datum(sc)
    q = plan["quantum"]
    assert np.all(plan["datum"] == np.round(plan["datum"]))
    assert np.all(plan["zrel"].astype(np.float32).astype(np.float64) == plan["zrel"])
    assert np.all(np.abs(plan["zrel"] / q - np.round(plan["zrel"] / q)) == 0)
    tg = dg2.tile_grid(sc, dg2.FP32)
    iv = np.minimum(np.arange(sc.nx + 1), sc.nx - 1) // tg["tile_x"]
    jv = np.minimum(np.arange(sc.ny + 1), sc.ny - 1) // tg["tile_y"]
    absq = plan["zrel"] + plan["datum"][jv[:, None], iv[None, :]]
    assert np.abs(absq - sc.zv).max() <= 0.5 * q + 1e-12 * max(1.0, np.abs(sc.zv).max())
    for z32, exact in frames(sc, plan):
        assert np.all(z32.astype(np.float64) == exact)
        assert np.abs(exact).max() <= plan["max_local"] + q
        m32, m64 = cell_means(z32, True), cell_means(exact, False)
        assert np.all(m32.astype(np.float64) == m64)
        fx32 = np.float32(0.5) * (z32[1:, :] + z32[:-1, :])   # W/E face beds
        assert np.all(fx32.astype(np.float64) == 0.5 * (exact[1:, :] + exact[:-1, :]))
        fy32 = np.float32(0.5) * (z32[:, 1:] + z32[:, :-1])   # S/N face beds
        assert np.all(fy32.astype(np.float64) == 0.5 * (exact[:, 1:] + exact[:, :-1]))
        if m32.shape[1] > 1:
            assert np.all(np.diff(m32, axis=1).astype(np.float64) == np.diff(m64, axis=1))
        if m32.shape[0] > 1:
            assert np.all(np.diff(m32, axis=0).astype(np.float64) == np.diff(m64, axis=0))


def test_plan_shifts_with_whole_metres():
    base = S.urban_wet(n=256, n_blocks=60)
    a = dg2.plan_bed_datum(base)
    b = dg2.plan_bed_datum(base.replace(zv=base.zv + 1234.0))
    assert np.array_equal(a["zrel"], b["zrel"])
    assert np.array_equal(b["datum"] - a["datum"], np.full_like(a["datum"], 1234.0))
    assert a["quantum"] == b["quantum"] and a["max_local"] == b["max_local"]


def test_plan_rejects_extreme_relief():
    sc = S.dam_break(nx=20, ny=4)
    zv = sc.zv.copy()
    zv[0, 0] = 3.0e6
    with pytest.raises(dg2.DG2Error) as e:
        dg2.plan_bed_datum(sc.replace(zv=zv))
    assert e.value.code == dg2.E_UNSUPPORTED
