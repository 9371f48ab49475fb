"""Pins of the oracle's CFL time step (reading R11 of Sect. 2.1.1: Cr = 0.33 times the
smallest cell crossing time at the fastest signal speed) against what the shallow
water equations fix, not against the oracle's own formula:

- the characteristic speeds of the SWE are u +- sqrt(g h) (and v +- sqrt(g h)), so on a
  uniform state the step is Cr dx / (max(|u|, |v|) + sqrt(g h));
- the minimum is over cells: one fast cell in still water sets the step alone;
- an inflow segment imposes its critical-depth state, where the Froude number is one
  (q = h_c sqrt(g h_c)): its speed is u + c = 2 sqrt(g h_c), with h_c = (q^2/g)^(1/3);
- a fixed state (h_b, u_b, v_b) bounds the step at its own characteristic speed;
- cells at or below h_tol take no part, and with nothing to bound it the step is
  dt_dry.
"""
import numpy as np
import pytest

from oracle import Oracle
from paper_2107_02750_amd import scenarios as S

G = 9.80665
CR = 0.33


def flat(nx, ny, h, qx, qy, dx=2.0, **kw):
    zv = np.zeros((ny + 1, nx + 1))
    means = np.stack([np.full((ny, nx), h), np.full((ny, nx), qx), np.full((ny, nx), qy)])
    return S.Scenario("flat", nx, ny, dx, zv, S.MODE_MEANS, means, **kw)


@pytest.mark.parametrize("h,qx,qy", [(1.0, 0.0, 0.0), (2.5, 3.0, -1.0), (0.4, -0.2, 1.1)])
def test_uniform_state_step_is_the_characteristic_speed(h, qx, qy):
    o = Oracle(flat(12, 9, h, qx, qy))
    speed = max(abs(qx), abs(qy)) / h + np.sqrt(G * h)
    assert o.next_dt() == pytest.approx(CR * 2.0 / speed, rel=1e-14)


def test_fastest_cell_sets_the_step():
    sc = flat(15, 11, 1.0, 0.0, 0.0)
    means = sc.init_data.copy()
    means[0, 4, 7] = 3.0   # one deep, fast cell
    means[2, 4, 7] = -6.0  # v = -2 m/s
    o = Oracle(sc.replace(init_data=means))
    assert o.next_dt() == pytest.approx(CR * 2.0 / (2.0 + np.sqrt(G * 3.0)), rel=1e-14)


@pytest.mark.parametrize("Q,faces", [(3.0, 4), (40.0, 10)])
def test_inflow_critical_state_bounds_the_step(Q, faces):
    dx = 2.0
    sc = flat(20, 16, 0.0, 0.0, 0.0, dx=dx)
    t = np.array([0.0, 100.0])
    sc = sc.replace(boundaries=[S.Boundary(S.W, S.INFLOW, 3, 3 + faces, t, np.array([Q, Q]))])
    q = Q / (faces * dx)
    hc = (q * q / G) ** (1.0 / 3.0)
    assert hc * np.sqrt(G * hc) == pytest.approx(q, rel=1e-14)  # Froude number one
    o = Oracle(sc)
    assert o.next_dt() == pytest.approx(CR * dx / (2.0 * np.sqrt(G * hc)), rel=1e-13)


def test_fixed_state_bounds_the_step():
    dx = 2.0
    sc = flat(20, 16, 0.0, 0.0, 0.0, dx=dx)
    sc = sc.replace(boundaries=[S.Boundary(S.S, S.FIXED, 2, 9, h_b=0.8, u_b=0.3, v_b=1.7)])
    o = Oracle(sc)
    assert o.next_dt() == pytest.approx(CR * dx / (1.7 + np.sqrt(G * 0.8)), rel=1e-14)


def test_dry_and_near_dry_cells_take_no_part():
    sc = flat(10, 10, 0.0, 0.0, 0.0, dt_dry=0.75)
    assert Oracle(sc).next_dt() == 0.75
    thin = sc.replace(init_data=np.stack([np.full((10, 10), sc.h_tol), np.zeros((10, 10)),
                                          np.zeros((10, 10))]))
    assert Oracle(thin).next_dt() == 0.75
    # one cell just above the tolerance: it alone sets the step
    means = thin.init_data.copy()
    means[0, 5, 5] = 2.0 * sc.h_tol
    o = Oracle(thin.replace(init_data=means))
    assert o.next_dt() == pytest.approx(CR * 2.0 / np.sqrt(G * 2.0 * sc.h_tol), rel=1e-14)


@pytest.mark.parametrize("h1x,h1y", [(0.12, 0.03), (-0.2, 0.15), (0.0, -0.25)])
def test_sloped_depth_takes_the_largest_depth_of_the_reconstruction(h1x, h1y):
    """Inside a cell the depth is the planar expansion of eq 2, h0 + sqrt(3) xi h1 for xi
    in [-1, 1] along each direction: the fastest signal in the cell runs at the mean
    velocity plus sqrt(g h) at the largest depth that expansion reaches, found here by
    sampling it."""
    nx, ny, h0, qx0, qy0 = 9, 7, 1.0, 0.5, -0.3
    P = np.zeros((9, ny, nx))
    P[0], P[1], P[2], P[3], P[6] = h0, h1x, h1y, qx0, qy0
    zv = np.zeros((ny + 1, nx + 1))
    o = Oracle(S.Scenario("sloped", nx, ny, 2.0, zv, S.MODE_PLANES, P))
    xi = np.linspace(-1.0, 1.0, 2001)
    speeds = [abs(q) / h0 + np.sqrt(G * (h0 + np.sqrt(3.0) * xi * h1).max())
              for q, h1 in ((qx0, h1x), (qy0, h1y))]
    assert o.next_dt() == pytest.approx(CR * 2.0 / max(speeds), rel=1e-14)
