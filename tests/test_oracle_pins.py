"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

Each test names the part of the method it pins (the paper's section or equation) and
checks it against something other than the oracle's own formulas: closed-form
solutions, exact discrete invariants, hand-worked fixtures, symmetries.
"""
import os

import numpy as np
import pytest
from scipy.optimize import brentq

import closed_forms as CF
import oracle
from oracle import Oracle
from paper_2107_02750_amd import scenarios as S

G = 9.80665
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    return np.loadtxt(os.path.join(GOLDEN, name), comments="#", ndmin=2)


# ------------------------------------------------------------------------------------
# eq 8 (Sect. 2.1.4): bed projection
# ------------------------------------------------------------------------------------

def test_eq8_worked_cell():
    ne, nw, se, sw, z0, z1x, z1y = _golden("eq8_worked_cell.txt")[0]
    zv = np.array([[sw, se], [nw, ne]])  # row j = 0 is the south vertex row
    a, b, c = oracle.bed_coeffs(zv)
    assert a[0, 0] == pytest.approx(z0, abs=1e-15)
    assert b[0, 0] == pytest.approx(z1x, abs=1e-15)
    assert c[0, 0] == pytest.approx(z1y, abs=1e-15)


def test_eq8_identities_and_planar_bed():
    rng = np.random.default_rng(7)
    zv = rng.normal(size=(9, 12))
    z0, z1x, z1y = oracle.bed_coeffs(zv)
    s3 = np.sqrt(3.0)
    zE = 0.5 * (zv[1:, 1:] + zv[:-1, 1:])
    zW = 0.5 * (zv[1:, :-1] + zv[:-1, :-1])
    zN = 0.5 * (zv[1:, :-1] + zv[1:, 1:])
    zS = 0.5 * (zv[:-1, :-1] + zv[:-1, 1:])
    # the three forms of eq 8a agree, and the face values are recovered from the planes
    np.testing.assert_allclose(z0, 0.5 * (zE + zW), atol=1e-15)
    np.testing.assert_allclose(z0, 0.5 * (zN + zS), atol=1e-15)
    np.testing.assert_allclose(z0 + s3 * z1x, zE, atol=4e-15)
    np.testing.assert_allclose(z0 - s3 * z1y, zS, atol=4e-15)
    # the 4-vertex forms of eq 8b-c
    np.testing.assert_allclose(
        z1x, (zv[1:, 1:] - zv[1:, :-1] + zv[:-1, 1:] - zv[:-1, :-1]) / (4 * s3), atol=1e-15)
    # a planar bed z = a + b x + c y is represented exactly: z0 = z(centre) and
    # z1x = b dx / (2 sqrt3) (the basis slope of eq 3 is 2 sqrt3 (x - xc) / R)
    dx = 2.5
    xv, yv = np.meshgrid(np.arange(13) * dx, np.arange(10) * dx)
    zp = 1.5 + 0.3 * xv - 0.7 * yv
    p0, p1x, p1y = oracle.bed_coeffs(zp)
    xc, yc = np.meshgrid((np.arange(12) + 0.5) * dx, (np.arange(9) + 0.5) * dx)
    np.testing.assert_allclose(p0, 1.5 + 0.3 * xc - 0.7 * yc, atol=1e-13)
    np.testing.assert_allclose(p1x, 0.3 * dx / (2 * s3), atol=1e-14)
    np.testing.assert_allclose(p1y, -0.7 * dx / (2 * s3), atol=1e-14)


# ------------------------------------------------------------------------------------
# HLL flux (Sect. 2.1.1)
# ------------------------------------------------------------------------------------

def _phys(h, un, ut):
    return np.array([h * un, h * un * un + 0.5 * G * h * h, h * un * ut])


def test_hll_consistency_symmetry_and_dry():
    rng = np.random.default_rng(3)
    for _ in range(200):
        h, un, ut = rng.uniform(0.01, 3.0), rng.normal(), rng.normal()
        np.testing.assert_allclose(oracle.hll(G, h, un, ut, h, un, ut), _phys(h, un, ut),
                                   rtol=1e-13, atol=1e-13)
        hl, ul, vl = rng.uniform(0, 3), rng.normal(), rng.normal()
        hr, ur, vr = rng.uniform(0, 3), rng.normal(), rng.normal()
        f = oracle.hll(G, hl, ul, vl, hr, ur, vr)
        m = oracle.hll(G, hr, -ur, vr, hl, -ul, vl)   # mirror image through the face
        np.testing.assert_allclose(m, [-f[0], f[1], -f[2]], rtol=1e-12, atol=1e-13)
    assert np.all(oracle.hll(G, 0.0, 1.0, 2.0, 0.0, -1.0, 3.0) == 0.0)
    # supersonic to the right: the upwind physical flux, exactly
    f = oracle.hll(G, 1.0, 10.0, 0.5, 0.5, 9.0, 0.0)
    assert np.array_equal(f, _phys(1.0, 10.0, 0.5))
    # still water against a dry bed at rest: the upwind side's pressure leaks out,
    # mass flows into the dry side
    f = oracle.hll(G, 1.0, 0.0, 0.0, 0.0, 0.0, 0.0)
    assert f[0] > 0.0


# ------------------------------------------------------------------------------------
# split-implicit Manning friction (Sect. 2.1.1, C_f of eq 1)
# ------------------------------------------------------------------------------------

def test_friction_point_1d_form_and_ode_convergence():
    n, h, q0 = 0.05, 0.4, 1.2
    # 1D: one Newton step of backward Euler reduces to q (1 + a) / (1 + 2 a),
    # a = dt C_f |u| / h (derived by hand from the update rule)
    for dt in (0.01, 0.5, 10.0, 1e4):
        a = dt * G * n * n / h ** (1.0 / 3.0) * abs(q0 / h) / h
        out = oracle.friction_point(G, n, 1e-3, dt, h, q0, 0.0)
        assert out[0] == pytest.approx(q0 * (1 + a) / (1 + 2 * a), rel=1e-14)
        assert 0.0 < out[0] < q0 and out[1] == 0.0    # decays, never flips sign
        neg = oracle.friction_point(G, n, 1e-3, dt, h, -q0, 0.0)
        assert neg[0] == pytest.approx(-out[0], rel=1e-15)
    # repeated steps converge at first order to the exact ODE solution
    T = 20.0
    errs = []
    for m in (20, 40, 80, 160):
        q = q0
        for _ in range(m):
            q = oracle.friction_point(G, n, 1e-3, T / m, h, q, 0.0)[0]
        errs.append(abs(q - CF.friction_ode(q0, h, n, G, T)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 0.9) and np.all(rates < 1.1), rates
    # dry, still or frictionless points are untouched
    assert list(oracle.friction_point(G, n, 1e-3, 1.0, 1e-4, 1.0, 1.0)) == [1.0, 1.0]
    assert list(oracle.friction_point(G, 0.0, 1e-3, 1.0, 1.0, 1.0, 1.0)) == [1.0, 1.0]
    assert list(oracle.friction_point(G, n, 1e-3, 1.0, 1.0, 0.0, 0.0)) == [0.0, 0.0]


# ------------------------------------------------------------------------------------
# well-balancedness (Sect. 2.1.1: revisions keep still water still)
# ------------------------------------------------------------------------------------

def test_lake_at_rest_round_off():
    o = Oracle(S.lake_at_rest(nx=100, ny=100, seed=1, eta=1.0))
    for _ in range(1000):
        o.step()
    assert np.abs(o.read(3)).max() <= 1e-12
    assert np.abs(o.read(6)).max() <= 1e-12
    assert np.abs(o.read(9) - 1.0).max() <= 1e-12


def test_partially_dry_lake_at_rest_round_off():
    sc = S.partially_dry_lake(nx=100, ny=100, seed=1, eta=0.2)
    o = Oracle(sc)
    h0 = o.read(0)
    assert (h0 == 0).sum() > 100 and (h0 > 0).sum() > 5000  # both dry and wet cells
    for _ in range(1000):
        o.step()
    h = o.read(0)
    assert np.abs(o.read(3)).max() <= 1e-12
    assert np.abs(o.read(6)).max() <= 1e-12
    wet = h > 0
    assert np.abs(o.read(9)[wet] - 0.2).max() <= 1e-12
    assert np.array_equal(h == 0, h0 == 0)       # no island gets wet


# ------------------------------------------------------------------------------------
# mass conservation (eq 1 is in conservative form)
# ------------------------------------------------------------------------------------

def test_mass_closed_box():
    sc = S.dam_break(nx=60, ny=40, dx=1.0, h_right=0.0, x_dam=30.0)
    sc = sc.replace(edge_kind=(S.WALL,) * 4)
    o = Oracle(sc)
    m0 = o.scalars()["mass"]
    o.run(20.0)
    s = o.scalars()
    assert abs(s["mass"] - m0 - s["mass_clip"]) <= 1e-13 * m0
    assert s["mass_in"] == 0.0 and s["mass_out"] == 0.0


def test_mass_ledger_open_domain_with_inflow_and_clipping():
    # a corner of the channel terrain with its inflow, plus outflow through open edges
    sc = S.fbm_channel(n=64, dx=5.0, seed=2, channel_width=30.0, amplitude=40.0,
                       wavelength=200.0, q_peak=20.0)
    o = Oracle(sc)
    m0 = o.scalars()["mass"]
    o.run(600.0)
    s = o.scalars()
    assert s["mass_in"] > 1000.0
    bal = s["mass"] - m0 - s["mass_in"] + s["mass_out"] - s["mass_clip"]
    assert abs(bal) <= 1e-12 * max(s["mass"], s["mass_in"])


# ------------------------------------------------------------------------------------
# closed-form dam breaks (flat bed, no friction): HLL + RK2 + limiter
# ------------------------------------------------------------------------------------

def test_stoker_closed_form_values():
    hm, um, xs, xa, xb = _golden("stoker_textbook.txt")[0]
    # the stored values against the relations that define them: the left rarefaction's
    # Riemann invariant, mass and momentum across the right shock, and the wave positions
    hl, hr, x0, t = 1.0, 0.5, 50.0, 2.5
    assert abs(um - 2.0 * (np.sqrt(G * hl) - np.sqrt(G * hm))) <= 2e-6
    s = hm * um / (hm - hr)
    assert abs(hm * um * um + 0.5 * G * (hm * hm - hr * hr) - s * hm * um) <= 1e-5
    assert abs(xs - (x0 + s * t)) <= 1e-4
    assert abs(xa - (x0 - np.sqrt(G * hl) * t)) <= 1e-4
    assert abs(xb - (x0 + (um - np.sqrt(G * hm)) * t)) <= 1e-4
    _, _, info = CF.stoker(np.array([0.0]), 2.5, 1.0, 0.5, 50.0, G)
    assert info["hm"] == pytest.approx(hm, abs=1e-7)
    assert info["um"] == pytest.approx(um, abs=1e-7)
    assert info["shock"] == pytest.approx(xs, abs=1e-4)
    assert info["rare_head"] == pytest.approx(xa, abs=1e-4)
    assert info["rare_tail"] == pytest.approx(xb, abs=1e-4)


def _front_1d(nx, h_right):
    dx = 100.0 / nx
    o = Oracle(S.dam_break(nx=nx, ny=2, dx=dx, h_right=h_right))
    o.run(2.5)
    h = o.read(0)
    assert np.array_equal(h[0], h[1])          # a y-uniform problem stays y-uniform
    return (np.arange(nx) + 0.5) * dx, h[0], o


def test_stoker_convergence_and_shock():
    errs = []
    for nx in (100, 200, 400):
        x, h, _ = _front_1d(nx, 0.5)
        he, _, info = CF.stoker(x, 2.5, 1.0, 0.5, 50.0, G)
        errs.append(np.abs(h - he).mean())
        mid = 0.5 * (info["hm"] + 0.5)
        k = np.nonzero((h[:-1] >= mid) & (h[1:] < mid))[0][-1]
        xs = x[k] + (h[k] - mid) / (h[k] - h[k + 1]) * (x[1] - x[0])
        assert abs(xs - info["shock"]) <= 1.5 * (x[1] - x[0])
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates >= 0.7), rates


def test_ritter_wet_dry_front():
    errs, lags = [], []
    for nx in (100, 200, 400):
        x, h, o = _front_1d(nx, 0.0)
        he, _, info = CF.ritter(x, 2.5, 1.0, 50.0, G)
        errs.append(np.abs(h - he).mean())
        # the wet edge (depth above h_tol) trails the point where the exact depth equals
        # the dry tolerance by a few cells at most, and closes in as the grid refines
        x_tol = info["front"] - 2.5 * np.sqrt(9.0 * G * 1e-3)
        lag = x_tol - x[h > 1e-3].max()
        dx = 100.0 / nx
        assert -dx <= lag <= 4 * dx
        lags.append(lag)
        assert np.all(h >= 0.0)
        assert o.scalars()["mass"] == pytest.approx(50.0 * 2 * (100.0 / nx), rel=1e-13)
    assert lags[0] > lags[1] > lags[2]
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates >= 0.7), rates


# ------------------------------------------------------------------------------------
# 2D wet/dry with bed source: Thacker's oscillation in a paraboloid bowl
# ------------------------------------------------------------------------------------

def _thacker(nx, h_tol=1e-4):
    a, h0, r0 = 1.0, 0.1, 0.8
    dx = 4.0 / nx
    xv = np.arange(nx + 1) * dx
    X, Y = np.meshgrid(xv, xv)
    h, u, v, z, info = CF.thacker_bowl(X, Y, 0.0, a, h0, r0, G, 2.0, 2.0)
    sc = S.Scenario("thacker", nx, nx, dx, z, S.MODE_VERTEX, np.stack([h, h * u, h * v]),
                    h_tol=h_tol)
    o = Oracle(sc)
    T = info["period"]
    o.run(T)
    xc = (np.arange(nx) + 0.5) * dx
    Xc, Yc = np.meshgrid(xc, xc)
    he, _, _, _, _ = CF.thacker_bowl(Xc, Yc, T, a, h0, r0, G, 2.0, 2.0)
    return np.abs(o.read(0) - he).mean(), o


def test_thacker_bowl_one_period():
    e50, _ = _thacker(50)
    e100, o = _thacker(100)
    assert e100 <= 4e-4
    assert np.log2(e50 / e100) >= 1.0
    s = o.scalars()
    assert np.isclose(s["t"], 2.0 * np.pi / (np.sqrt(8 * G * 0.1)), rtol=0, atol=1e-12)


# ------------------------------------------------------------------------------------
# friction + bed source + RK2: uniform flow on a tilted plane
# ------------------------------------------------------------------------------------

def test_manning_uniform_flow_equilibrium():
    """Uniform depth on a plane of slope S with transmissive edges stays uniform, and the
    discharge relaxes to the scheme's discrete equilibrium. For uniform flow the friction
    step maps q to q (1 + a)/(1 + 2 a) with a = dt g n^2 q / h^(7/3), and both RK2 stages
    add dt g h S (the bed source of eq 1), so equilibrium needs q a / (1 + 2 a) = dt g h S,
    with dt the CFL step dx / (q/h + sqrt(g h)) times the Courant number. As dt -> 0 this
    is Manning's normal flow q = h^(5/3) sqrt(S) / n."""
    q_n, n, sl = 1.0, 0.035, 1e-3
    hn = CF.manning_normal_depth(q_n, n, sl)
    nx, ny, dx = 12, 3, 5.0
    zv = np.tile(-sl * np.arange(nx + 1) * dx, (ny + 1, 1))
    vert = np.stack([np.full_like(zv, hn), np.full_like(zv, 0.5), np.zeros_like(zv)])
    sc = S.Scenario("manning", nx, ny, dx, zv, S.MODE_VERTEX, vert, manning_scalar=n,
                    limiter=0)
    o = Oracle(sc)
    for _ in range(8000):
        o.step()
    h, q = o.read(0), o.read(3)
    assert np.abs(h - hn).max() <= 1e-10          # depth moves by round-off only
    assert np.abs(q - q.mean()).max() <= 1e-10    # discharge stays uniform

    def resid(qq):
        dt = 0.33 * dx / (qq / hn + np.sqrt(G * hn))
        a = dt * G * n * n * qq / hn ** (7.0 / 3.0)
        return qq * a / (1 + 2 * a) - dt * G * hn * sl

    q_d = brentq(resid, 0.5, 2.0, xtol=1e-15)
    assert q.mean() == pytest.approx(q_d, rel=1e-9)
    assert q_d == pytest.approx(q_n, rel=5e-3)     # O(a) splitting error only


# ------------------------------------------------------------------------------------
# symmetry of the x and y code paths; determinism; checkpoint/resume
# ------------------------------------------------------------------------------------

def _transpose_planes(p):
    # (h0,h1x,h1y,qx0,qx1x,qx1y,qy0,qy1x,qy1y) -> transposed problem
    order = [0, 2, 1, 6, 8, 7, 3, 5, 4]
    return np.stack([p[k].T for k in order])


def test_transpose_symmetry_bitwise():
    rng = np.random.default_rng(11)
    nx, ny = 23, 17
    zv = rng.uniform(0, 0.5, size=(ny + 1, nx + 1))
    hv = np.maximum(0.6 - zv + 0.2 * rng.normal(size=zv.shape), 0.0)
    qx = 0.3 * rng.normal(size=zv.shape) * (hv > 0)
    qy = 0.3 * rng.normal(size=zv.shape) * (hv > 0)
    sc = S.Scenario("sym", nx, ny, 0.7, zv, S.MODE_VERTEX, np.stack([hv, qx, qy]),
                    manning_scalar=0.03, edge_kind=(S.WALL, S.TRANSMISSIVE, S.WALL, S.TRANSMISSIVE))
    sct = S.Scenario("symT", ny, nx, 0.7, zv.T.copy(), S.MODE_VERTEX,
                     np.stack([hv.T, qy.T, qx.T]).copy(), manning_scalar=0.03,
                     edge_kind=(S.WALL, S.TRANSMISSIVE, S.WALL, S.TRANSMISSIVE))
    a, b = Oracle(sc), Oracle(sct)
    for _ in range(15):
        da, db = a.step(), b.step()
        assert da == db
    assert np.array_equal(_transpose_planes(a.planes()), b.planes())


def test_determinism_and_checkpoint_resume():
    sc = S.fbm_channel(n=48, dx=5.0, seed=2, amplitude=30.0, wavelength=150.0, q_peak=10.0)
    a = Oracle(sc)
    a.run(300.0)
    snap = a.get_state()
    a.run(600.0)
    b = Oracle(sc)
    b.set_state(snap)
    b.run(600.0)
    assert np.array_equal(a.get_state(), b.get_state())
    c = Oracle(sc)          # same schedule (the run to 300 s lands exactly on it)
    c.run(300.0)
    c.run(600.0)
    assert np.array_equal(a.get_state(), c.get_state())


def test_run_lands_on_t_end_and_errors():
    o = Oracle(S.dam_break(nx=20, ny=4, dx=5.0))
    o.run(1.2345)
    assert o.scalars()["t"] == 1.2345
    with pytest.raises(oracle.OracleError):
        o.run(1.0)
    bad = S.dam_break(nx=20, ny=4, dx=5.0)
    with pytest.raises(oracle.OracleError):
        Oracle(bad.replace(dx=-1.0))
    with pytest.raises(oracle.OracleError):
        Oracle(bad.replace(nx=0))
    neg = bad.init_data.copy()
    neg[0, 0, 0] = -1.0
    with pytest.raises(oracle.OracleError):
        Oracle(bad.replace(init_data=neg))
    nanz = bad.zv.copy()
    nanz[1, 1] = np.nan
    with pytest.raises(oracle.OracleError):
        Oracle(bad.replace(zv=nanz))
    with pytest.raises(oracle.OracleError):
        Oracle(bad.replace(boundaries=[S.Boundary(S.W, S.INFLOW, 0, 2, np.array([0.0, 0.0]),
                                                  np.array([1.0, 2.0]))]))
    with pytest.raises(oracle.OracleError):
        Oracle(bad.replace(boundaries=[S.Boundary(S.N, S.WALL, 3, 30)]))
