"""Tile-shape autotuner for the stage kernels.

The library is built for a few tile shapes per precision (dg2.tile_shapes). Which one
is fastest depends on the grid (how tiles cover its edges, how many blocks a launch
has) and on the flow (dry tiles are cheap). The tuner runs a short timed window of the
actual scenario(s) with every shape and returns the fastest:
  - one scenario: the stage-kernel times from the library's HIP-event timing;
  - a batch: wall time of batched steps over a sample of the members, between device
    synchronisations.
Timing starts from the scenarios' current initial state, after a few warm-up steps.
"""
from __future__ import annotations

import time

from . import dg2


def tune_scenario(sc, precision: int, steps: int = 40, warmup: int = 5, stream=None) -> dict:
    """Fastest tile shape for one scenario: {'best': (tx, ty), 'ms_per_step': {...}}."""
    ms = {}
    for shape in dg2.tile_shapes(precision):
        sim = dg2.DG2(sc, precision, stream=stream, tile=shape)
        for _ in range(warmup):
            sim.step(sync=False)
        sim.set_timing(True)
        for _ in range(steps):
            sim.step(sync=False)
        tm = sim.timing()
        ms[shape] = tm["ms_stage1"] + tm["ms_stage2"]
        sim.close()
    best = min(ms, key=ms.get)
    return {"best": best, "ms_per_step": {f"{x}x{y}": v for (x, y), v in ms.items()}}


def tune_batch(scs, precision: int, stream, sample: int = 8, steps: int = 32,
               warmup: int = 4) -> dict:
    """Fastest tile shape for a batch of scenarios, timed on an evenly spaced sample of
    them (sorted by size): {'best': (tx, ty), 'ms_per_step': {...}}."""
    import torch
    order = sorted(range(len(scs)), key=lambda k: scs[k].nx * scs[k].ny)
    pick = [order[round(i * (len(order) - 1) / max(sample - 1, 1))] for i in range(min(sample, len(scs)))]
    ms = {}
    for shape in dg2.tile_shapes(precision):
        sims = [dg2.DG2(scs[k], precision, stream=stream, tile=shape) for k in pick]
        batch = dg2.Batch(sims, graph_steps=2)
        batch.step(warmup)
        stream.synchronize()
        t0 = time.perf_counter()
        batch.step(steps)
        stream.synchronize()
        ms[shape] = (time.perf_counter() - t0) * 1e3 / steps
        batch.close()
        for s in sims:
            s.close()
        torch.cuda.synchronize()
    best = min(ms, key=ms.get)
    return {"best": best, "ms_per_step": {f"{x}x{y}": v for (x, y), v in ms.items()}}
