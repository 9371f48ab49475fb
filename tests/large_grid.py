"""Inputs of the large-grid test: still water 1 m deep on a flat bed, a moving mound
of water and a bed bump near the corner of the highest cell indices, both of compact
support; the oracle window is the last WIN x WIN cells. The mound centre sits 16
cells from the E and N edges (water leaves through them from the first step), the
bump 48 to 68 vertices from the E edge, so in STEPS steps (at most four cells each)
nothing within 20 cells of the window's cut edges moves."""
import numpy as np

from paper_2107_02750_amd import scenarios as S

WIN = 128
STEPS = 10


def add_bump(a, cy, cx, radius, height):
    """Adds height (1 - r^2/R^2)^2 around (cy, cx) of a 2-D array, R = radius in
    cells; exactly zero from R on. Returns the square it touched and the values."""
    y0, y1, x0, x1 = cy - radius, cy + radius + 1, cx - radius, cx + radius + 1
    y, x = np.ogrid[y0:y1, x0:x1]
    r2 = ((x - cx) ** 2 + (y - cy) ** 2) / float(radius * radius)
    add = height * np.maximum(1.0 - r2, 0.0) ** 2
    a[y0:y1, x0:x1] += add
    return (slice(y0, y1), slice(x0, x1)), add


def scenario(nx, ny):
    zv = np.zeros((ny + 1, nx + 1))
    add_bump(zv, ny - 50, nx - 58, 10, 0.15)
    means = np.zeros((3, ny, nx))
    means[0] = 1.0
    sq, mound = add_bump(means[0], ny - 16, nx - 16, 12, 0.3)
    means[1][sq] = 0.5 * mound
    means[2][sq] = -0.2 * mound
    return S.Scenario(f"large_grid{nx}x{ny}", nx, ny, 2.0, zv, S.MODE_MEANS, means,
                      manning_scalar=0.02)


def window(sc):
    return S.window(sc, WIN, WIN, sc.nx - WIN, sc.ny - WIN)
