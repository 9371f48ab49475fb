"""Closed-form shallow-water solutions used to pin the oracle.

Textbook results (not from the paper): Stoker's wet-wet and Ritter's wet-dry dam
breaks on a flat frictionless bed, Thacker's (1981) radially symmetric oscillation in a
paraboloidal bowl, Manning normal depth on a uniform slope, and the exact solution of
the friction-only ODE dq/dt = -g n^2 q|q| / h^(7/3).
"""
import numpy as np
from scipy.optimize import brentq


def stoker(x, t, h_l, h_r, x0, g):
    """Depth and velocity of the wet-wet dam break at time t > 0."""
    cl = np.sqrt(g * h_l)

    def f(hm):
        um_rare = 2.0 * (cl - np.sqrt(g * hm))
        um_shock = (hm - h_r) * np.sqrt(0.5 * g * (hm + h_r) / (hm * h_r))
        return um_rare - um_shock

    hm = brentq(f, h_r, h_l, xtol=1e-15, rtol=1e-15)
    um = 2.0 * (cl - np.sqrt(g * hm))
    s = hm * um / (hm - h_r)
    cm = np.sqrt(g * hm)
    xa = x0 - cl * t
    xb = x0 + (um - cm) * t
    xs = x0 + s * t
    x = np.asarray(x, dtype=float)
    h = np.empty_like(x)
    u = np.empty_like(x)
    a = x <= xa
    h[a], u[a] = h_l, 0.0
    r = (x > xa) & (x <= xb)
    xi = (x[r] - x0) / t
    h[r] = (2.0 * cl - xi) ** 2 / (9.0 * g)
    u[r] = 2.0 / 3.0 * (xi + cl)
    m = (x > xb) & (x <= xs)
    h[m], u[m] = hm, um
    b = x > xs
    h[b], u[b] = h_r, 0.0
    return h, u, dict(hm=hm, um=um, shock=xs, rare_head=xa, rare_tail=xb)


def ritter(x, t, h_l, x0, g):
    """Depth and velocity of the dam break onto a dry bed."""
    cl = np.sqrt(g * h_l)
    xa = x0 - cl * t
    xf = x0 + 2.0 * cl * t
    x = np.asarray(x, dtype=float)
    h = np.zeros_like(x)
    u = np.zeros_like(x)
    a = x <= xa
    h[a] = h_l
    r = (x > xa) & (x < xf)
    xi = (x[r] - x0) / t
    h[r] = (2.0 * cl - xi) ** 2 / (9.0 * g)
    u[r] = 2.0 / 3.0 * (xi + cl)
    return h, u, dict(front=xf, rare_head=xa)


def thacker_bowl(x, y, t, a, h0, r0, g, xc, yc):
    """Thacker's radially symmetric oscillation in the bowl z = -h0 (1 - r^2/a^2)
    (bed below the rim is negative). Returns depth, radial velocity components and the
    bed at (x, y)."""
    w = np.sqrt(8.0 * g * h0) / a
    A = (a * a - r0 * r0) / (a * a + r0 * r0)
    r2 = (x - xc) ** 2 + (y - yc) ** 2
    z = -h0 * (1.0 - r2 / (a * a))
    den = 1.0 - A * np.cos(w * t)
    eta = h0 * (np.sqrt(1.0 - A * A) / den - 1.0 - r2 / (a * a) * ((1.0 - A * A) / den ** 2 - 1.0))
    h = np.maximum(eta - z, 0.0)
    fac = 0.5 * w * A * np.sin(w * t) / den
    u = np.where(h > 0, fac * (x - xc), 0.0)
    v = np.where(h > 0, fac * (y - yc), 0.0)
    return h, u, v, z, dict(omega=w, period=2 * np.pi / w, A=A)


def manning_normal_depth(q, n, slope):
    return (q * n / np.sqrt(slope)) ** 0.6


def friction_ode(q0, h, n, g, t):
    """q(t) for dq/dt = -g n^2 q|q| / h^(7/3) with q0 > 0."""
    return q0 / (1.0 + g * n * n * abs(q0) * t / h ** (7.0 / 3.0))
