"""The premise of the large-grid GPU test, checked with the oracle alone on a smaller
grid with the same corner: the oracle on the last 128 x 128 cells reproduces, for
every step of the test, the time step and those cells of the oracle on the whole
grid, and every other cell of the whole grid stays at rest (still water on a flat
bed stays still to the bit: both sides of every face are equal)."""
import numpy as np
import pytest

import large_grid as LG
from oracle import Oracle


@pytest.mark.parametrize("fv1", [False, True])
def test_window_reproduces_the_whole_grid(fv1):
    sc = LG.scenario(384, 256)
    if fv1:
        sc = sc.as_fv1()
    full, win = Oracle(sc), Oracle(LG.window(sc))
    W = LG.WIN
    for k in range(LG.STEPS):
        a, b = full.step(), win.step()
        assert a == b, (k, a, b)
    P, Q = full.planes(), win.planes()
    assert np.array_equal(P[:, -W:, -W:], Q)
    rest = P.copy()
    rest[:, -W:, -W:] = 0.0
    rest[0, -W:, -W:] = 1.0
    assert np.all(rest[0] == 1.0) and not rest[1:].any()
    # something moved, the outflow reached the E and N edges, and the window's cut
    # edges (W and S, 20 cells deep) are still
    assert np.abs(Q[0] - 1.0).max() > 1e-3
    assert full.scalars()["mass_out"] > 0.0
    assert np.all(Q[0, :, :20] == 1.0) and np.all(Q[0, :20, :] == 1.0)
    for key in ("mass_in", "mass_out", "mass_clip"):
        assert full.scalars()[key] == win.scalars()[key], key
