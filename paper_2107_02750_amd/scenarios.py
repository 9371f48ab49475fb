"""Seeded synthetic flood scenarios (inputs only).

This module builds the raw inputs a user would hand to the solver: a vertex-raster DEM,
Manning's n, an initial condition, boundary segments and inflow hydrographs. It holds
none of the DG2 method's arithmetic (no projection, limiting, fluxes or updates), so
both the GPU library's tests and the CPU oracle can be fed from it.

The paper's three case studies use Environment Agency DEMs that are not available
(arXiv:2107.02750, Data Availability Statement); the generators below stand in for
them with seeded terrain of the same kind: a rugged valley-like terrain with a channel
and an upstream inflow hydrograph (Sect. 3.1, 3.2), and an urban grid of building blocks
with an inflow along one edge (Sect. 3.3).
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

# boundary kinds and edges (the numbering is part of the C interface of both libraries)
TRANSMISSIVE, WALL, FIXED, INFLOW = 0, 1, 2, 3
W, E, S, N = 0, 1, 2, 3

# initial-condition modes
MODE_PLANES, MODE_MEANS, MODE_VERTEX, MODE_LEVEL = 0, 1, 2, 3

# schemes: DG2 (piecewise planar, RK2) and FV1 (piecewise constant, forward Euler)
SCHEME_DG2, SCHEME_FV1 = 0, 1

G_STD = 9.80665


@dataclass
class Boundary:
    """A run of boundary faces [i0, i1) on one edge with a non-default condition."""
    edge: int
    kind: int
    i0: int
    i1: int
    t_knots: Optional[np.ndarray] = None  # s
    q_knots: Optional[np.ndarray] = None  # m^3/s
    h_b: float = 0.0
    u_b: float = 0.0
    v_b: float = 0.0


@dataclass
class Scenario:
    name: str
    nx: int
    ny: int
    dx: float
    zv: np.ndarray                      # (ny+1, nx+1) vertex elevations, m
    init_mode: int
    init_data: Optional[np.ndarray] = None  # see MODE_*
    eta_level: float = 0.0
    manning: Optional[np.ndarray] = None    # (ny, nx) or None
    manning_scalar: float = 0.0
    boundaries: List[Boundary] = field(default_factory=list)
    edge_kind: tuple = (TRANSMISSIVE, TRANSMISSIVE, TRANSMISSIVE, TRANSMISSIVE)
    g: float = G_STD
    cfl: float = 0.33
    h_tol: float = 1e-3
    dt_dry: float = 1.0
    t0: float = 0.0
    limiter: int = 1
    t_end: float = 0.0
    scheme: int = SCHEME_DG2

    @property
    def cells(self) -> int:
        return self.nx * self.ny

    def replace(self, **kw) -> "Scenario":
        return dataclasses.replace(self, **kw)

    def as_fv1(self) -> "Scenario":
        """The same inputs for the FV1 scheme, with its Courant number of 0.5."""
        return dataclasses.replace(self, scheme=SCHEME_FV1, cfl=0.5,
                                   name=self.name + "_fv1")


def _flat_bed(nx: int, ny: int, z: float = 0.0) -> np.ndarray:
    return np.full((ny + 1, nx + 1), float(z))


# --------------------------------------------------------------------------------------
# small analytic set-ups
# --------------------------------------------------------------------------------------

def dam_break(nx: int = 100, ny: int = 100, dx: float = 1.0, h_left: float = 1.0,
              h_right: float = 0.5, x_dam: float = 50.0, t_end: float = 2.5) -> Scenario:
    """Wet-wet dam break on a flat frictionless bed, transmissive edges: cell-mean depth
    h_left west of x_dam and h_right east of it, at rest."""
    xc = (np.arange(nx) + 0.5) * dx
    h = np.where(xc < x_dam, h_left, h_right)
    means = np.zeros((3, ny, nx))
    means[0] = h[None, :]
    return Scenario("dam_break", nx, ny, dx, _flat_bed(nx, ny), MODE_MEANS, means, t_end=t_end)


def lake_at_rest(nx: int = 100, ny: int = 100, dx: float = 1.0, seed: int = 1,
                 bump_max: float = 0.4, eta: float = 1.0, t_end: float = 2.5) -> Scenario:
    """Still water at level eta over i.i.d. uniform random vertex bumps in [0, bump_max]."""
    rng = np.random.default_rng(seed)
    zv = rng.uniform(0.0, bump_max, size=(ny + 1, nx + 1))
    return Scenario("lake_at_rest", nx, ny, dx, zv, MODE_LEVEL, eta_level=eta, t_end=t_end)


def partially_dry_lake(nx: int = 100, ny: int = 100, dx: float = 1.0, seed: int = 1,
                       eta: float = 0.2, n_islands: int = 40, margin: float = 0.01,
                       spread: float = 0.09, t_end: float = 2.5) -> Scenario:
    """Still water at level eta with dry islands.

    Islands are rectangles of cells, at least two cells apart; all their vertices lie in
    [eta + margin, eta + margin + spread] and every other vertex in
    [0, eta - margin - spread]. A cell outside the islands then touches at most two
    island vertices, so its vertex mean is at most eta, while every island cell and every
    face on an island boundary lies above eta: a discrete still-water state with
    partially wet cells."""
    rng = np.random.default_rng(seed)
    low = rng.uniform(0.0, eta - margin - spread, size=(ny + 1, nx + 1))
    island = np.zeros((ny, nx), dtype=bool)
    taken = np.zeros((ny, nx), dtype=bool)  # islands plus a two-cell moat
    placed = 0
    tries = 0
    while placed < n_islands and tries < 100 * n_islands:
        tries += 1
        w = int(rng.integers(1, 7))
        h = int(rng.integers(1, 7))
        i0 = int(rng.integers(0, nx - w + 1))
        j0 = int(rng.integers(0, ny - h + 1))
        a, b = max(j0 - 2, 0), min(j0 + h + 2, ny)
        c, d = max(i0 - 2, 0), min(i0 + w + 2, nx)
        if taken[a:b, c:d].any():
            continue
        island[j0:j0 + h, i0:i0 + w] = True
        taken[a:b, c:d] = True
        placed += 1
    hv = np.zeros((ny + 1, nx + 1), dtype=bool)
    for jj, ii in zip(*np.nonzero(island)):
        hv[jj:jj + 2, ii:ii + 2] = True
    high = rng.uniform(eta + margin, eta + margin + spread, size=(ny + 1, nx + 1))
    zv = np.where(hv, high, low)
    return Scenario("partially_dry_lake", nx, ny, dx, zv, MODE_LEVEL, eta_level=eta,
                    t_end=t_end)


# --------------------------------------------------------------------------------------
# terrain
# --------------------------------------------------------------------------------------

def fbm_vertices(n_vert: int, seed: int, hurst: float = 0.8, relief: float = 20.0,
                 fft_n: Optional[int] = None) -> np.ndarray:
    """Spectral fractional-Brownian terrain on an (n_vert x n_vert) vertex raster:
    random phases, amplitude |k|^-(H+1) on an fft_n^2 periodic grid (default the next
    power of two at least twice n_vert), cropped and rescaled to [0, relief]."""
    if fft_n is None:
        fft_n = 1 << int(np.ceil(np.log2(2 * n_vert)))
    rng = np.random.default_rng(seed)
    kx = np.fft.fftfreq(fft_n)[None, :]
    ky = np.fft.fftfreq(fft_n)[:, None]
    k = np.sqrt(kx * kx + ky * ky)
    k[0, 0] = 1.0
    amp = k ** (-(hurst + 1.0))
    amp[0, 0] = 0.0
    phase = rng.uniform(0.0, 2.0 * np.pi, size=(fft_n, fft_n))
    field_ = np.fft.ifft2(amp * np.exp(1j * phase)).real[:n_vert, :n_vert]
    lo, hi = field_.min(), field_.max()
    return (field_ - lo) / (hi - lo) * relief


def trapezoid_hydrograph(q_peak: float, t_rise: float, t_hold_end: float,
                         t_fall_end: float) -> tuple:
    t = np.array([0.0, t_rise, t_hold_end, t_fall_end])
    q = np.array([0.0, q_peak, q_peak, 0.0])
    return t, q


def fbm_channel(n: int = 1024, dx: float = 5.0, seed: int = 2, hurst: float = 0.8,
                relief: float = 20.0, channel_width: float = 30.0,
                channel_depth: float = 3.0, amplitude: Optional[float] = None,
                wavelength: Optional[float] = None, q_peak: float = 50.0,
                manning: float = 0.035, t_end: float = 7200.0,
                fft_n: Optional[int] = None) -> Scenario:
    """Rugged terrain with a carved meandering channel, initially dry, fed at the west
    edge by a trapezoid hydrograph (0 -> q_peak over 900 s, held to 2700 s, back to 0
    at 3600 s); the other edges are transmissive.

    The channel centreline is y_c(x) = L/2 + amplitude sin(2 pi x / wavelength + phi);
    vertices within half the channel width of it are lowered to the running minimum
    (from the west) of the terrain along the centreline minus channel_depth, so the
    channel bed never rises downstream. By default the meander has amplitude 500 m and
    wavelength 2000 m on the 1024-cell, 5 m grid, and both scale with the domain length
    otherwise. fft_n: the spectral grid of the terrain (see fbm_vertices)."""
    if amplitude is None:
        amplitude = 500.0 * n * dx / 5120.0
    if wavelength is None:
        wavelength = 2000.0 * n * dx / 5120.0
    rng = np.random.default_rng(seed + 1000)
    zv = fbm_vertices(n + 1, seed, hurst, relief, fft_n)
    phi = rng.uniform(0.0, 2.0 * np.pi)
    xv = np.arange(n + 1) * dx
    yv = np.arange(n + 1) * dx
    ymid = 0.5 * n * dx
    yc = ymid + amplitude * np.sin(2.0 * np.pi * xv / wavelength + phi)
    jc = np.clip(np.rint(yc / dx).astype(int), 0, n)
    z_line = zv[jc, np.arange(n + 1)]
    z_bed = np.minimum.accumulate(z_line) - channel_depth
    inside = np.abs(yv[:, None] - yc[None, :]) <= 0.5 * channel_width
    zv = np.where(inside, np.minimum(zv, z_bed[None, :]), zv)
    # inflow faces on the west edge: rows whose face centre lies inside the channel
    yface = (np.arange(n) + 0.5) * dx
    rows = np.nonzero(np.abs(yface - yc[0]) <= 0.5 * channel_width)[0]
    t_k, q_k = trapezoid_hydrograph(q_peak, 900.0, 2700.0, 3600.0)
    bc = Boundary(W, INFLOW, int(rows.min()), int(rows.max()) + 1, t_k, q_k)
    zeros = np.zeros((3, n, n))
    return Scenario("fbm_channel", n, n, dx, zv, MODE_MEANS, zeros, manning_scalar=manning,
                    boundaries=[bc], t_end=t_end)


def fbm_channel_wet(n: int = 1024, dx: float = 5.0, seed: int = 2, eta: float = 25.0,
                    qx: float = 2.0, manning: float = 0.035) -> Scenario:
    """The fbm_channel terrain flooded everywhere: vertex depths eta - z and a uniform
    discharge qx at every vertex, transmissive edges. Every cell is wet and moving, so
    each one does the full wet-cell arithmetic (friction, wet-wet fluxes)."""
    base = fbm_channel(n, dx, seed, manning=manning)
    depth = eta - base.zv
    vert = np.stack([depth, np.full_like(depth, qx), np.zeros_like(depth)])
    return Scenario("fbm_channel_wet", n, n, dx, base.zv, MODE_VERTEX, vert,
                    manning_scalar=manning, t_end=600.0)


def batch_scenarios(count: int = 64, seed: int = 400, side_lo: int = 256, side_hi: int = 1024,
                    t_end: float = 1800.0) -> list:
    """Independent flood scenarios of uneven size for batched runs: scenario k has a
    square grid of side ~ U{side_lo..side_hi} cells, dx ~ U[2, 10] m, fBm channel
    terrain of seed seed + k, Manning n ~ U(0.015, 0.06) and a trapezoid inflow
    hydrograph peaking at ~ U(5, 100) m^3/s."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        n = int(rng.integers(side_lo, side_hi + 1))
        dx = float(rng.uniform(2.0, 10.0))
        man = float(rng.uniform(0.015, 0.06))
        qp = float(rng.uniform(5.0, 100.0))
        fft_n = 1 << int(np.ceil(np.log2(n + 1)))  # a period beyond the grid is enough
        sc = fbm_channel(n=n, dx=dx, seed=seed + k, manning=man, q_peak=qp, t_end=t_end,
                         fft_n=fft_n)
        out.append(dataclasses.replace(sc, name=f"batch{k}_{n}"))
    return out


def adjoint_case(n: int = 512, dx: float = 5.0, seed: int = 5, zones: int = 4,
                 n_knots: int = 48, t_span: float = 400.0, eta: float = 25.0,
                 band: float = 60.0) -> Scenario:
    """A fully wet, limiter-off flow for gradient studies: the fBm terrain (seed) under
    still water at level eta plus a weak uniform eastward discharge, Manning n constant
    on each of zones x zones rectangular blocks (n ~ U(0.02, 0.05)), and an inflow
    hydrograph of n_knots knots spread over t_span (Q ~ U(20, 120) m^3/s) through the
    west-edge faces of a central band; other edges transmissive."""
    rng = np.random.default_rng(seed + 5000)
    zv = fbm_vertices(n + 1, seed, 0.8, 20.0)
    depth = eta - zv
    vert = np.stack([depth, np.full_like(depth, 0.5), np.zeros_like(depth)])
    n_zone = rng.uniform(0.02, 0.05, size=(zones, zones))
    zi = np.minimum(np.arange(n) * zones // n, zones - 1)
    manning = n_zone[zi[:, None], zi[None, :]]
    rows = int(round(band / dx))
    j0 = n // 2 - rows // 2
    t_k = np.linspace(0.0, t_span, n_knots)
    q_k = rng.uniform(20.0, 120.0, size=n_knots)
    bc = Boundary(W, INFLOW, j0, j0 + rows, t_k, q_k)
    return Scenario("adjoint_case", n, n, dx, zv, MODE_VERTEX, vert, manning=manning,
                    boundaries=[bc], limiter=0, t_end=t_span)


def zone_index(n: int, zones: int = 4) -> np.ndarray:
    """Zone number (row-major over zones x zones blocks) of every cell of an n x n grid,
    as used by adjoint_case."""
    zi = np.minimum(np.arange(n) * zones // n, zones - 1)
    return zi[:, None] * zones + zi[None, :]


def urban_blocks(n: int = 2048, dx: float = 2.0, seed: int = 3, n_blocks: int = 4000,
                 side_min: float = 5.0, side_max: float = 30.0, height: float = 10.0,
                 h_in: float = 1.0, u_in: float = 2.0, manning: float = 0.02,
                 t_end: float = 600.0) -> Scenario:
    """Flat ground with seeded axis-aligned building blocks (vertices inside a block are
    raised by `height`), initially dry, with a fixed inflow state (depth h_in, velocity
    u_in eastward) imposed along the whole west edge."""
    rng = np.random.default_rng(seed)
    zv = np.zeros((n + 1, n + 1))
    ext = n * dx
    wx = rng.uniform(side_min, side_max, n_blocks)
    wy = rng.uniform(side_min, side_max, n_blocks)
    x0 = rng.uniform(0.0, ext, n_blocks)
    y0 = rng.uniform(0.0, ext, n_blocks)
    for k in range(n_blocks):
        a = int(np.ceil(x0[k] / dx)); b = int(np.floor((x0[k] + wx[k]) / dx))
        c = int(np.ceil(y0[k] / dx)); d = int(np.floor((y0[k] + wy[k]) / dx))
        zv[max(c, 0):min(d, n) + 1, max(a, 0):min(b, n) + 1] = height
    bc = Boundary(W, FIXED, 0, n, h_b=h_in, u_b=u_in, v_b=0.0)
    zeros = np.zeros((3, n, n))
    return Scenario("urban_blocks", n, n, dx, zv, MODE_MEANS, zeros, manning_scalar=manning,
                    boundaries=[bc], t_end=t_end)


def window(sc: Scenario, nx: int, ny: int, i0: int = 0, j0: int = 0) -> Scenario:
    """A sub-rectangle of a scenario's DEM (cells [i0, i0+nx) x [j0, j0+ny)), keeping
    its boundary segments clipped to the window where they lie on a kept edge."""
    zv = sc.zv[j0:j0 + ny + 1, i0:i0 + nx + 1].copy()
    data = sc.init_data
    if data is not None:
        if sc.init_mode in (MODE_PLANES, MODE_MEANS):
            data = data[:, j0:j0 + ny, i0:i0 + nx].copy()
        elif sc.init_mode == MODE_VERTEX:
            data = data[:, j0:j0 + ny + 1, i0:i0 + nx + 1].copy()
    man = None if sc.manning is None else sc.manning[j0:j0 + ny, i0:i0 + nx].copy()
    bcs = []
    for b in sc.boundaries:
        if b.edge == W and i0 == 0 or b.edge == E and i0 + nx == sc.nx:
            lo, hi = max(b.i0 - j0, 0), min(b.i1 - j0, ny)
        elif b.edge == S and j0 == 0 or b.edge == N and j0 + ny == sc.ny:
            lo, hi = max(b.i0 - i0, 0), min(b.i1 - i0, nx)
        else:
            continue
        if lo < hi:
            bcs.append(dataclasses.replace(b, i0=lo, i1=hi))
    return dataclasses.replace(sc, name=sc.name + f"_win{nx}x{ny}", nx=nx, ny=ny, zv=zv,
                               init_data=data, manning=man, boundaries=bcs)


def urban_wet(n: int = 2048, dx: float = 2.0, seed: int = 3, n_blocks: int = 4000,
              eta: float = 2.0, qx: float = 1.0, manning: float = 0.02) -> Scenario:
    """The urban_blocks terrain under water to level eta between the blocks (vertex
    depth eta - z where positive) with an eastward discharge qx where wet: flow around
    every block, wet/dry fronts at every block wall."""
    base = urban_blocks(n, dx, seed, n_blocks, manning=manning)
    depth = np.maximum(eta - base.zv, 0.0)
    vert = np.stack([depth, np.where(depth > 0, qx, 0.0), np.zeros_like(depth)])
    return Scenario("urban_wet", n, n, dx, base.zv, MODE_VERTEX, vert,
                    manning_scalar=manning, boundaries=base.boundaries, t_end=60.0)
