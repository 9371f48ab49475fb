"""A grid of 2^29 cells (32768 x 16384) on the GPU: every state plane past the first
starts beyond 4 GiB (FP64) and the state buffer spans 36 GiB, so any 32-bit offset in
the kernels or the library would show. Still water on a flat bed with a moving mound of
water and a bed bump in the corner of the highest cell indices (tests/large_grid.py);
the window around them is compared with the FP64 oracle run on that window alone, and
every cell outside it must stay at rest.

The window's results are those of the whole grid because nothing outside it moves: a
step reaches at most four cells (two stages, each a face neighbour and the limiter's
neighbour), the mound and the bump have compact support, and the time step is the
same on both sides (the background's CFL candidate is that of the window's still
cells; tests/test_large_grid_window_cpu.py checks all of this with the oracle on a
smaller grid). Host memory: about 17 GB of input arrays; device memory: up to 129 GB.
"""
import gc

import numpy as np
import pytest

import large_grid as LG
from oracle import Oracle

pytestmark = pytest.mark.gpu

NX, NY = 32768, 16384
WIN, STEPS = LG.WIN, LG.STEPS
TOL, DT_TOL, FLOOR = 1e-12, 1e-10, 1e-3


@pytest.fixture(scope="module")
def dg2():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2107_02750_amd import dg2 as mod
    mod.load()
    return mod


@pytest.fixture(scope="module")
def big():
    print(f"building the {NX}x{NY} inputs", flush=True)
    _free()
    return LG.scenario(NX, NY)


def _rel_errs(a, b):
    H = max(np.abs(b[0]).max(), FLOOR)
    Q = max(np.abs(b[3]).max(), np.abs(b[6]).max(), FLOOR)
    sc = [H] * 3 + [Q] * 6
    return np.array([np.abs(a[p] - b[p]).max() / sc[p] for p in range(9)])


def _window_and_rest(sim):
    """The window's planes (host) and the largest deviation from rest outside it,
    found on the device."""
    import torch
    win, dev = [], 0.0
    for p in range(9):
        t = sim.read_device(p)
        win.append(t[NY - WIN:, NX - WIN:].cpu().numpy().astype(np.float64))
        rest = 1.0 if p == 0 else 0.0
        t[NY - WIN:, NX - WIN:] = rest
        dev = max(dev, float((t - rest).abs().max()))
        del t
    torch.cuda.synchronize()
    return np.stack(win), dev


def _free(sim=None):
    """Destroys the simulation and returns its workspace (and whatever earlier tests
    left in torch's cache) to the device before the next large allocation."""
    import torch
    if sim is not None:
        sim.close()
        sim.workspace = None
    gc.collect()
    torch.cuda.empty_cache()


@pytest.mark.parametrize("scheme", ["dg2", "fv1"])
def test_large_grid_fp64_window_matches_oracle(dg2, big, scheme):
    sc = big if scheme == "dg2" else big.as_fv1()
    print(f"case {scheme} FP64 {NX}x{NY}: init", flush=True)
    sim = dg2.DG2(sc, dg2.FP64)
    ref = Oracle(LG.window(sc))
    try:
        print(f"case {scheme} FP64 {NX}x{NY}: {STEPS} steps", flush=True)
        for k in range(STEPS):
            a, b = sim.step(), ref.step()
            assert abs(a - b) <= DT_TOL * b, (k, a, b)
        win, dev = _window_and_rest(sim)
        e = _rel_errs(win, ref.planes())
        print(f"window errors {e.max():.2e}, deviation from rest outside {dev:.2e}", flush=True)
        assert e.max() <= TOL, e
        assert dev <= 1e-13
        # the disturbance stayed inside the window, away from its cut edges
        assert np.abs(win[0, :, :8] - 1.0).max() <= 1e-13 and np.abs(win[0, :8, :] - 1.0).max() <= 1e-13
        assert np.abs(win[0] - 1.0).max() > 1e-3
        ga, gb = sim.scalars(), ref.scalars()
        assert ga["t"] == pytest.approx(gb["t"], rel=1e-12)
        for key in ("mass_in", "mass_out", "mass_clip"):
            assert abs(ga[key] - gb[key]) <= 1e-12 * max(abs(gb[key]), 1.0), (key, ga[key], gb[key])
    finally:
        _free(sim)


def test_large_grid_fp32_window_against_fp64_oracle(dg2, big):
    print(f"case FP32 {NX}x{NY}: init", flush=True)
    sim = dg2.DG2(big, dg2.FP32)
    ref = Oracle(LG.window(big))
    try:
        for _ in range(STEPS):
            ref.step()
        t_end = ref.scalars()["t"]
        print(f"case FP32 {NX}x{NY}: run to t={t_end:.4f} s", flush=True)
        sim.run(t_end)
        assert sim.scalars()["t"] == t_end
        win, dev = _window_and_rest(sim)
        err = np.abs(win[0] - ref.read(0)).max()
        print(f"FP32 window depth error {err:.2e} m, deviation from rest outside {dev:.2e}",
              flush=True)
        assert err <= 1e-4
        assert dev <= 1e-6
    finally:
        _free(sim)
