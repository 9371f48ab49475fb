"""Pins of the oracle's limiter, boundary conditions and friction projection.

These parts of the step are readings (the paper names no limiter, gives no boundary
formulas and states friction only as a split implicit update, Sect. 2.1.1, 3.1-3.3),
so each is pinned against what the reading itself fixes, computed independently of the
oracle's code: hand-worked limiter values, a bound every limited state must satisfy,
steady uniform flow on a slope (Manning's normal flow up to the splitting error, with
the discrete equilibrium derived by hand), exact boundary mass fluxes, a Newton step
of backward Euler with a finite-difference Jacobian, and the L2 projection of the
friction update onto the slope basis by fine quadrature.
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
S3 = np.sqrt(3.0)
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------------------------------
# minmod limiter (reading R3; Sect. 2.1.1 names no limiter)
# ------------------------------------------------------------------------------------

def _row_case(var, b, a, a1, axis):
    """A 3-cell row (axis 0: along x, axis 1: along y) on the bed z = b * s (s the
    coordinate along the row, dx = 1 m) holding the means a of variable var and the
    slope a1 of the middle cell; every cell is wet. Returns the oracle and the state."""
    n_along = 3
    sv = np.arange(n_along + 1, dtype=np.float64)
    if axis == 0:
        nx, ny = 3, 1
        zv = np.tile(b * sv, (2, 1))
    else:
        nx, ny = 1, 3
        zv = np.tile((b * sv)[:, None], (1, 2))
    st = np.zeros((9, ny, nx))
    st[0] = 1.0                       # wet everywhere unless the case sets the depth
    plane = {0: 0, 1: 3, 2: 6}[var]
    if axis == 1 and var in (1, 2):
        plane = {1: 6, 2: 3}[var]     # the transposed row: qx <-> qy
    st[plane] = np.asarray(a, dtype=np.float64).reshape(ny, nx)
    slope = plane + (1 if axis == 0 else 2)
    mid = (0, 1) if axis == 0 else (1, 0)
    st[slope][mid] = a1
    sc = S.Scenario("row", nx, ny, 1.0, zv, S.MODE_PLANES, st)
    return Oracle(sc), st, slope, mid


@pytest.mark.parametrize("axis", [0, 1])
def test_minmod_worked_values(axis):
    rows = np.loadtxt(os.path.join(GOLDEN, "minmod_worked.txt"), comments="#", ndmin=2)
    for var, b, am, a0, ap, a1, expect in rows:
        o, st, slope, mid = _row_case(int(var), b, [am, a0, ap], a1, axis)
        out = o.limit(st)
        assert out[slope][mid] == pytest.approx(expect, abs=1e-15), (var, b, am, a0, ap, a1)


def test_minmod_face_values_stay_within_neighbour_means():
    """Every face value a0 +- sqrt3 a1 of a limited cell (free surface, qx, qy, each
    direction) lies between the smallest and largest mean of the cell and its two
    neighbours in that direction (the ghost beyond an edge: the edge cell's depth and
    discharge on its bed plane continued). Random wet states on a bumpy bed."""
    rng = np.random.default_rng(21)
    nx, ny, dx = 17, 13, 1.5
    zv = rng.uniform(0.0, 0.5, size=(ny + 1, nx + 1))
    st = np.zeros((9, ny, nx))
    st[0] = rng.uniform(0.8, 1.6, size=(ny, nx))
    st[[3, 6]] = rng.normal(0.0, 1.0, size=(2, ny, nx))
    st[[1, 2]] = rng.normal(0.0, 0.15, size=(2, ny, nx))
    st[[4, 5, 7, 8]] = rng.normal(0.0, 0.8, size=(4, ny, nx))
    sc = S.Scenario("bound", nx, ny, dx, zv, S.MODE_PLANES, st)
    out = Oracle(sc).limit(st)
    z0, z1x, z1y = oracle.bed_coeffs(zv)
    zfx = 0.5 * (zv[1:, :] + zv[:-1, :])   # x-face beds (ny, nx+1)
    zfy = 0.5 * (zv[:-1, :] + zv[1:, :].copy())  # placeholder, rebuilt below
    zfy = 0.5 * (zv[:, :-1] + zv[:, 1:])   # y-face beds (ny+1, nx)
    checked = 0
    for axis, s_off, z1 in ((1, 1, z1x), (0, 2, z1y)):
        for base, is_eta in ((0, True), (3, False), (6, False)):
            a0 = st[base] + (z0 if is_eta else 0.0)
            a1 = out[base + s_off] + (z1 if is_eta else 0.0)
            # ghost means beyond the two edges along this axis
            if is_eta:
                if axis == 1:
                    dz = zfx[:, 1:] - zfx[:, :-1]
                else:
                    dz = zfy[1:, :] - zfy[:-1, :]
            else:
                dz = np.zeros_like(a0)
            lo_g = np.take(a0, [0], axis=axis) - np.take(dz, [0], axis=axis)
            hi_g = np.take(a0, [-1], axis=axis) + np.take(dz, [-1], axis=axis)
            ext = np.concatenate([lo_g, a0, hi_g], axis=axis)
            am = np.take(ext, range(0, a0.shape[axis]), axis=axis)
            ap = np.take(ext, range(2, a0.shape[axis] + 2), axis=axis)
            lo = np.minimum(np.minimum(am, a0), ap)
            hi = np.maximum(np.maximum(am, a0), ap)
            for sgn in (1.0, -1.0):
                fv = a0 + sgn * S3 * a1
                assert np.all(fv >= lo - 1e-12) and np.all(fv <= hi + 1e-12)
            checked += a0.size
    assert checked == 6 * nx * ny
    # the bound binds: many slopes were cut
    assert np.sum(np.abs(out[[4, 5, 7, 8]]) < np.abs(st[[4, 5, 7, 8]])) > 100


def test_open_edges_pass_uniform_flow_on_a_slope():
    """Uniform flow down a tilted plane through open (transmissive) edges, limiter on:
    the depth stays uniform to round-off and the discharge relaxes to the discrete
    equilibrium of the split step (the edge cells' ghosts continue the bed plane, so
    the edge cells are not flattened into sills)."""
    q0, n, sl = 1.0, 0.035, 1e-3
    hn = CF.manning_normal_depth(q0, n, sl)
    nx, ny, dx = 40, 2, 10.0
    zv = np.tile(-sl * np.arange(nx + 1) * dx, (ny + 1, 1))
    vert = np.stack([np.full_like(zv, hn), np.full_like(zv, q0), np.zeros_like(zv)])
    sc = S.Scenario("plane", nx, ny, dx, zv, S.MODE_VERTEX, vert, manning_scalar=n)
    o = Oracle(sc)
    for _ in range(3000):
        dt = o.step()
    h, q = o.read(0), o.read(3)
    assert np.abs(h / hn - 1.0).max() <= 1e-12
    assert np.abs(q / q.mean() - 1.0).max() <= 1e-12

    def resid(qq):  # per step: friction removes q a/(1+2a), gravity adds dt g h S
        a = dt * G * n * n * qq / hn ** (7.0 / 3.0)
        return qq * a / (1 + 2 * a) - dt * G * hn * sl

    assert q.mean() == pytest.approx(brentq(resid, 0.5, 2.0, xtol=1e-15), rel=1e-9)


# ------------------------------------------------------------------------------------
# inflow hydrograph (reading R12; Sect. 3.1-3.3 impose a discharge hydrograph)
# ------------------------------------------------------------------------------------

def _discrete_normal_flow(q_n, n, sl, dt):
    """Uniform flow fed by a discharge q_n per unit width, by hand: with time step dt
    each step removes Q a/(1+2a) by friction (a = dt g n^2 Q / h^(7/3), the 1-D Newton
    step) and adds dt g h S in both RK2 stages; the stage-1 flux Q' = Q - Q a/(1+2a)
    and the stage-2 flux Q' + dt g h S average to q_n. So the stored discharge is
    Q = q_n + dt g h S / 2, and Q a/(1+2a) = dt g h S fixes h."""
    def parts(h):
        Q = q_n + 0.5 * dt * G * h * sl
        a = dt * G * n * n * Q / h ** (7.0 / 3.0)
        return Q * a / (1 + 2 * a) - dt * G * h * sl, Q, a

    h = brentq(lambda x: parts(x)[0], 0.5, 2.0, xtol=1e-15)
    return h, parts(h)[1], parts(h)[2]


def test_manning_normal_flow_fed_by_inflow():
    """Inflow of q = 1 m^2/s per unit width (an INFLOW segment over the whole west
    edge) down a plane of slope 1e-3 with n = 0.035 and an open outlet: the discharge
    entering is exactly q W t, and the flow settles to Manning's normal depth
    (q n / sqrt S)^(3/5) = 1.0627738 m up to the splitting error, at the discrete
    equilibrium derived by hand. The time step is the CFL step of the inflow state,
    which is the binding one here (read back from the run)."""
    q_n, n, sl = 1.0, 0.035, 1e-3
    hn = CF.manning_normal_depth(q_n, n, sl)
    assert hn == pytest.approx(1.0627738, abs=1e-7)
    nx, ny, dx = 200, 2, 10.0
    width = ny * dx
    zv = np.tile(-sl * np.arange(nx + 1) * dx, (ny + 1, 1))
    hc = (q_n * q_n / G) ** (1.0 / 3.0)
    dt = 0.33 * dx / (q_n / hc + np.sqrt(G * hc))     # inflow state's CFL step
    hd, Qd, a = _discrete_normal_flow(q_n, n, sl, dt)
    assert abs(hd / hn - 1.0) <= 2.0 * a                 # O(a) splitting error
    bc = S.Boundary(S.W, S.INFLOW, 0, ny, np.array([0.0]), np.array([q_n * width]))
    xv = np.arange(nx + 1) * dx
    for pert in (0.0, 0.02):
        hv = np.tile(hd * (1.0 + pert * np.sin(2 * np.pi * xv / (nx * dx))), (ny + 1, 1))
        vert = np.stack([hv, np.full_like(zv, Qd * (1.0 - pert)), np.zeros_like(zv)])
        sc = S.Scenario("p7", nx, ny, dx, zv, S.MODE_VERTEX, vert, manning_scalar=n,
                        boundaries=[bc])
        o = Oracle(sc)
        assert o.next_dt() == pytest.approx(dt, rel=1e-14)
        for _ in range(8000):
            o.step()
        s = o.scalars()
        assert s["mass_in"] == pytest.approx(q_n * width * s["t"], rel=1e-12)
        h, q = o.read(0)[:, 10:-10], o.read(3)[:, 10:-10]
        # the stored mean discharge is the transported q plus half a step of gravity
        assert np.abs(q / Qd - 1.0).max() <= 1e-5, np.abs(q / Qd - 1.0).max()
        if pert == 0.0:       # started at the discrete equilibrium: it stays there
            assert np.abs(h / hd - 1.0).max() <= 1e-8
        else:                 # any steady profile (the open outlet fixes no depth)
            assert np.abs(h / hn - 1.0).max() <= 2.0 * a
            assert np.abs(h[:, :30] / hd - 1.0).max() <= 1e-4   # upstream: normal


@pytest.mark.parametrize("edge", [S.W, S.E, S.S, S.N])
def test_hydrograph_enters_exactly(edge):
    """An inflow segment on part of one edge (walls elsewhere on it and on the sides,
    the far edge open) of a plane sloping away from that edge: the mass that enters is exactly the trapezoid-rule integral of
    the piecewise-linear hydrograph (held beyond its knots) over the stage times t^n and
    t^n + dt of every step, whatever the flow regime at the edge."""
    n_along, n_across, dx, sl = 30, 12, 2.5, 0.01
    i0, i1 = 3, 9
    s_across = np.arange(n_across + 1)
    s_along = np.arange(n_along + 1) * dx
    down = -sl * s_along if edge in (S.W, S.S) else -sl * s_along[::-1]
    if edge in (S.W, S.E):
        nx, ny = n_along, n_across
        zv = np.tile(down, (ny + 1, 1))
    else:
        nx, ny = n_across, n_along
        zv = np.tile(down[:, None], (1, nx + 1))
    assert zv.shape == (ny + 1, nx + 1) and s_across.size == n_across + 1
    tk = np.array([5.0, 20.0, 45.0, 80.0])
    qk = np.array([2.0, 9.0, 4.0, 6.0])
    kinds = [S.WALL] * 4     # open only downstream: no other face carries inflow
    kinds[{S.W: S.E, S.E: S.W, S.S: S.N, S.N: S.S}[edge]] = S.TRANSMISSIVE
    sc = S.Scenario("hydro", nx, ny, dx, zv, S.MODE_MEANS, np.zeros((3, ny, nx)),
                    manning_scalar=0.03, edge_kind=tuple(kinds),
                    boundaries=[S.Boundary(edge, S.INFLOW, i0, i1, tk, qk)])
    o = Oracle(sc)
    expect = 0.0
    for _ in range(400):
        t = o.scalars()["t"]
        dt = o.step()
        expect += 0.5 * dt * (np.interp(t, tk, qk) + np.interp(t + dt, tk, qk))
    s = o.scalars()
    assert s["t"] > 90.0
    assert s["mass_in"] == pytest.approx(expect, rel=1e-12)
    assert s["mass"] > 0.2 * expect


# ------------------------------------------------------------------------------------
# fixed-state boundary (reading R12)
# ------------------------------------------------------------------------------------

@pytest.mark.parametrize("edge", [S.W, S.E, S.S, S.N])
def test_supercritical_fixed_state_mass_flux(edge):
    """A supercritical fixed state (h_b = 0.5 m, 4 m/s inward, Froude 1.8) along a whole
    edge of a dry flat bed: while the flow stays supercritical at the edge the face
    flux is the upwind state's, so the mass in is exactly h_b u_b W t."""
    h_b, u_in = 0.5, 4.0
    n_along, n_across, dx = 40, 8, 2.0
    nx, ny = (n_along, n_across) if edge in (S.W, S.E) else (n_across, n_along)
    inward = 1.0 if edge in (S.W, S.S) else -1.0
    ub, vb = (inward * u_in, 0.0) if edge in (S.W, S.E) else (0.0, inward * u_in)
    kinds = [S.WALL] * 4
    kinds[{S.W: S.E, S.E: S.W, S.S: S.N, S.N: S.S}[edge]] = S.TRANSMISSIVE
    sc = S.Scenario("fixed", nx, ny, dx, np.zeros((ny + 1, nx + 1)), S.MODE_MEANS,
                    np.zeros((3, ny, nx)), edge_kind=tuple(kinds),
                    boundaries=[S.Boundary(edge, S.FIXED, 0, n_across, h_b=h_b, u_b=ub, v_b=vb)])
    o = Oracle(sc)
    first = {S.W: (slice(None), 0), S.E: (slice(None), -1), S.S: (0, slice(None)),
             S.N: (-1, slice(None))}[edge]
    vel_field = 10 if edge in (S.W, S.E) else 11
    for _ in range(60):
        o.step()
        h = o.read(0)[first]
        un = inward * o.read(vel_field)[first]
        wet = h > 1e-3
        assert wet.all() and np.all(un > np.sqrt(G * h))      # supercritical at the edge
    s = o.scalars()
    assert s["mass_in"] == pytest.approx(h_b * u_in * n_across * dx * s["t"], rel=1e-12)
    assert s["mass"] == pytest.approx(s["mass_in"] - s["mass_out"] + s["mass_clip"], rel=1e-12)


# ------------------------------------------------------------------------------------
# split-implicit friction (reading R9; C_f of eq 1)
# ------------------------------------------------------------------------------------

def _be_residual(qx2, qy2, qx, qy, h, n, dt):
    """Backward Euler residual of dq/dt = -C_f u |u| (eq 1, C_f = g n^2 / h^(1/3),
    u = q / h) for the new discharge (qx2, qy2)."""
    cf = G * n * n / h ** (1.0 / 3.0)
    sp = np.hypot(qx2, qy2) / h
    return (qx2 - qx + dt * cf * (qx2 / h) * sp, qy2 - qy + dt * cf * (qy2 / h) * sp)


def test_friction_point_is_one_newton_step_in_2d():
    """At oblique velocities the update equals one Newton step of backward Euler from
    q, with the diagonal of the Jacobian taken by central differences of the residual
    (independent of the oracle's closed form)."""
    rng = np.random.default_rng(9)
    for _ in range(200):
        h = rng.uniform(0.05, 3.0)
        qx, qy = rng.normal(0, 1.5, size=2)
        n = rng.uniform(0.01, 0.08)
        dt = 10.0 ** rng.uniform(-2, 1.5)
        rx, ry = _be_residual(qx, qy, qx, qy, h, n, dt)
        ex, ey = 1e-6 * max(abs(qx), 1e-3), 1e-6 * max(abs(qy), 1e-3)
        jxx = (_be_residual(qx + ex, qy, qx, qy, h, n, dt)[0]
               - _be_residual(qx - ex, qy, qx, qy, h, n, dt)[0]) / (2 * ex)
        jyy = (_be_residual(qx, qy + ey, qx, qy, h, n, dt)[1]
               - _be_residual(qx, qy - ey, qx, qy, h, n, dt)[1]) / (2 * ey)
        newton = np.array([qx - rx / jxx, qy - ry / jyy])
        got = oracle.friction_point(G, n, 1e-3, dt, h, qx, qy)
        np.testing.assert_allclose(got, newton, rtol=1e-7, atol=1e-9 * np.hypot(qx, qy))


def _friction_projection_gap(amp, d, seed=13):
    """Largest gap, over a 6x5 grid of random cells whose slopes (in direction d only)
    are amp times the means, between the oracle's slope after friction and the L2
    projection of the point update by a 64-point Gauss rule, relative to the size of
    the projection; also checks the means and the depth planes."""
    rng = np.random.default_rng(seed)
    nx, ny = 6, 5
    s = np.zeros((9, ny, nx))
    s[0] = rng.uniform(0.5, 2.0, size=(ny, nx))
    s[3], s[6] = rng.normal(0, 1.0, size=(2, ny, nx))
    s[d] = amp * s[0] * rng.uniform(-1, 1, size=(ny, nx))
    s[3 + d] = amp * np.abs(s[3]) * rng.uniform(-1, 1, size=(ny, nx))
    s[6 + d] = amp * np.abs(s[6]) * rng.uniform(-1, 1, size=(ny, nx))
    man = rng.uniform(0.02, 0.06, size=(ny, nx))
    sc = S.Scenario("fr", nx, ny, 1.0, np.zeros((ny + 1, nx + 1)), S.MODE_PLANES, s,
                    manning=man)
    dt = 5.0
    out = Oracle(sc).friction(s, dt)
    xi, w = np.polynomial.legendre.leggauss(64)
    gap = 0.0
    for j in range(ny):
        for i in range(nx):
            h = s[0, j, i] + S3 * xi * s[d, j, i]
            qx = s[3, j, i] + S3 * xi * s[3 + d, j, i]
            qy = s[6, j, i] + S3 * xi * s[6 + d, j, i]
            upd = np.array([oracle.friction_point(G, man[j, i], 1e-3, dt, h[k], qx[k], qy[k])
                            for k in range(xi.size)])
            for var, q in ((0, qx), (1, qy)):
                proj = 0.5 * np.sum(w * (upd[:, var] - q) * S3 * xi)
                want = s[3 + 3 * var + d, j, i] + proj
                got = out[3 + 3 * var + d, j, i]
                gap = max(gap, abs(got - want) / abs(proj))
    # the mean is the update at the centre; depth is untouched
    c = np.array([[oracle.friction_point(G, man[j, i], 1e-3, dt, s[0, j, i], s[3, j, i], s[6, j, i])
                   for i in range(nx)] for j in range(ny)])
    np.testing.assert_array_equal(out[3], c[..., 0])
    np.testing.assert_array_equal(out[6], c[..., 1])
    np.testing.assert_array_equal(out[:3], s[:3])
    return gap


@pytest.mark.parametrize("d", [1, 2])
def test_friction_slopes_are_the_gauss_projection_of_the_point_update(d):
    """The slope coefficients after friction are the L2 projection onto the slope
    basis (sqrt3 xi on [-1, 1], eq 2) of the point update applied along the cell (one
    direction at a time). The step's 2-point Gauss rule is compared with a 64-point
    rule: the gap is the rule's error, which shrinks with the square of the slopes
    relative to the projection (a wrong weight or sign would leave an O(1) gap)."""
    g1 = _friction_projection_gap(0.04, d)
    g2 = _friction_projection_gap(0.02, d)
    assert g1 <= 5e-3 and g2 <= 1.5e-3, (g1, g2)
    assert g1 / g2 >= 3.0, (g1, g2)
