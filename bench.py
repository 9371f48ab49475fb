"""Benchmark of the gfx950 DG2 step: cell-updates per second on one MI355X.

Workload: the 1024 x 1024 fractional-Brownian terrain with a carved meandering channel
(dx = 5 m, Manning n = 0.035; seeded, synthetic), flooded everywhere (vertex depth
25 m - z, uniform discharge 2 m^2/s) so that every cell does the full wet-cell work:
friction, limiting, wet-wet HLL fluxes. A step is one full RK2 time step (friction,
two stages, CFL time step) over every cell. The state is resident in HBM before the
timed region starts; after W warm-up steps, windows of exactly K steps are timed between
device synchronisations, with nothing recorded in between, until at least 1 s has been
timed, and the median window gives the rate. Further windows, each launch bracketed by
HIP events on the launch stream, give the kernel durations (an event record costs the
stream a few microseconds, about 9 % of a step with three per step, so the throughput
is taken without them).

Also reported, on the same line: the FP32 instantiation on the same workload with its
depth error against the FP64 path, the same terrain as configured (dry start, channel
inflow hydrograph) timed from a snapshot at t = 3600 s, the urban precision run (FP32
with per-tile bed datums against FP64: depth error, mass drift, also with the bed raised
by 1000 m), the batched run of 64 uneven scenarios against running them one at a
time, the adjoint leg (gradients of a gauge misfit on a 512x512 fully wet flow, 2000
steps, against finite differences; adjoint time over forward time), the stage-kernel
durations from HIP events recorded on the launch stream with the roofline of the
dominant kernel (algorithmic bytes of the method, see ALG_VALUES, over the kernel's
mean launch time; both kernels and the whole step are listed too), and the FP64 CPU
oracle timed on this host's cores on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, GB/s
# Algorithmic values per cell of each stage launch: what the method must move, halo
# re-reads excluded. Stage 1 reads U^n (9) and the bed (one vertex per cell) and
# writes U^int (9); stage 2 reads U^n (9, from which V^n is rebuilt), U^int (9) and the
# bed and writes U^{n+1} (9). 47 values = 376 B per cell-step in FP64.
ALG_VALUES = {"stage1": 19, "stage2": 28}
# What these kernels move by design: stage 1 also writes V^n (friction applied,
# limited), which stage 2 reads instead of rebuilding it from U^n on a halo.
IMPL_VALUES = {"stage1": 28, "stage2": 28}


def stage_bytes(stage, n_cells, real_bytes, table=ALG_VALUES):
    return table[stage] * real_bytes * n_cells


def kernel_source_hash():
    """sha256 of what the forward kernels are compiled from and launched by: their
    source, the host library that sets their launch geometry, and the build script
    that holds the compiler flags."""
    import hashlib
    h = hashlib.sha256()
    for f in (os.path.join(ROOT, "paper_2107_02750_amd", "csrc", "dg2_kernels.hpp"),
              os.path.join(ROOT, "paper_2107_02750_amd", "csrc", "dg2.hip"),
              os.path.join(ROOT, "paper_2107_02750_amd", "build.py")):
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(summary, kernel):
    """HBM bytes per launch of a kernel from a committed rocprofv3 counter summary
    (profiles/<summary>.json: FETCH_SIZE and WRITE_SIZE in KiB per dispatch, scaled by
    what they read for a plain copy of known size), or None when the kernel sources
    changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", summary + ".json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("kernel_source_sha256") != kernel_source_hash():
        return None
    k = rec["kib_per_dispatch"].get(kernel)
    if k is None:
        return None
    sc = rec["copy_scale"]
    return 1024.0 * (k["fetch"] * sc["fetch"] + k["write"] * sc["write"])


TIMING = {"min_seconds": 1.0, "event_seconds": 0.25}


def timed_steps(sim, steps, min_seconds=None, min_windows=5, event_seconds=None):
    """Throughput and kernel durations of a simulation.

    Throughput: windows of exactly `steps` steps, each between two device
    synchronisations with nothing recorded inside, repeated until at least min_seconds
    have been timed and at least min_windows windows run; returns the median window's
    wall time (robust to clock ramp-up and stray host delays) and the window count.
    Kernel durations: the mean stage-kernel times from HIP events on the launch stream
    over further windows with every launch bracketed (at least event_seconds; an event
    record costs the stream a few microseconds, which the throughput leaves out)."""
    import torch
    if min_seconds is None:
        min_seconds = TIMING["min_seconds"]
    if event_seconds is None:
        event_seconds = TIMING["event_seconds"]
    if min_seconds <= 0.0:
        min_windows = 1
    wins = []
    while sum(wins) < min_seconds or len(wins) < min_windows:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            sim.step(sync=False)
        torch.cuda.synchronize()
        wins.append(time.perf_counter() - t0)
    sim.set_timing(True)
    t_ev, first = 0.0, True
    while first or t_ev < event_seconds:
        first = False
        t0 = time.perf_counter()
        for _ in range(steps):
            sim.step(sync=False)
        torch.cuda.synchronize()
        t_ev += time.perf_counter() - t0
    tm = sim.timing()
    sim.set_timing(False)
    return float(np.median(wins)), tm, len(wins)


def copy_bandwidth(mib=1024, reps=20):
    """Measured device copy rate (GB/s, bytes read plus bytes written): the median of
    reps device-to-device copies of mib MiB, each timed with HIP events on the current
    stream. It is the practical ceiling that the kernels' traffic is held against
    beside the datasheet peak."""
    import torch
    a = torch.empty(mib << 20, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1) * 1e-3)
    del a, b
    return 2.0 * (mib << 20) / float(np.median(ts)) / 1e9


FP64_VECTOR_PEAK_TFLOPS = 78.6


def cpu_baseline(sc, budget_s, gpu_value=None, fv1_values=None):
    """The FP64 CPU oracle on this host, stepping the same workload until budget_s
    seconds have passed (at least one step) after two untimed steps, on all the
    threads OpenMP gives it; then the same on one thread for half that budget; then, on
    all threads for half the budget, the terrain as configured from the oracle's stored
    state at t = 3600 s (the GPU's as-configured leg times the same terrain). Last, the
    method's operations per cell and step from one step of the oracle's operation-tally
    build on the same workload (each face and cell computed once), and with the GPU's
    rate the algorithmic FP64 flop rate that implies; the same for one FV1 step, with the
    GPU's FV1 rates (FP64, FP32) when given."""
    import oracle

    def rate(o, budget):
        t1 = time.perf_counter()
        steps = 0
        while True:
            o.step()
            steps += 1
            secs = time.perf_counter() - t1
            if secs >= budget:
                return steps, secs

    o = oracle.Oracle(sc)
    o.step()  # the first two steps also start the threads and touch both state buffers
    o.step()
    cores = oracle.threads()
    steps, secs = rate(o, budget_s)
    oracle.set_threads(1)
    steps1, secs1 = rate(o, 0.5 * budget_s)
    oracle.set_threads(cores)
    out = dict(value=sc.nx * sc.ny * steps / secs, unit="cell-updates/s",
               cores=cores, kind="oracle",
               sample=f"{steps} FP64 oracle steps of the same {sc.nx}x{sc.ny} all-wet "
                      f"workload ({secs:.1f} s)",
               one_core={"value": sc.nx * sc.ny * steps1 / secs1, "cores": 1,
                         "sample": f"{steps1} further steps on one thread ({secs1:.1f} s)"})
    # the terrain as configured (dry start, inflow), from the oracle's own stored state
    # at t = 3600 s (written by tests/golden/make_snapshots.py, which runs the oracle only)
    snap = os.path.join(ROOT, "tests", "golden", f"fbm_channel_{sc.nx}_t3600.npz")
    if sc.nx == sc.ny and os.path.exists(snap):
        from paper_2107_02750_amd import scenarios as S
        d = np.load(snap)
        P = np.zeros((9, sc.nx * sc.ny))
        P[:, d["idx"]] = d["vals"]
        cs = S.fbm_channel(n=sc.nx).replace(init_mode=S.MODE_PLANES,
                                            init_data=P.reshape(9, sc.ny, sc.nx), t0=float(d["t"]))
        oc = oracle.Oracle(cs)
        oc.step()
        stc, sec = rate(oc, 0.5 * budget_s)
        out["as_configured"] = {"value": sc.nx * sc.ny * stc / sec, "cores": cores,
                                "sample": f"{stc} oracle steps of the terrain as configured from "
                                          f"its stored state at t=3600 s ({sec:.1f} s)"}
    ot = oracle.Oracle(sc, tallied=True)
    ot.tally_reset()
    ot.step()
    per = {k: v / (sc.nx * sc.ny) for k, v in ot.tally_read().items()}
    flops = per["add"] + per["mul"] + per["div"] + per["sqrt"] + per["cbrt"]
    out["op_tally"] = {"per_cell_step": per, "flops_per_cell_step": flops,
                       "counted": "add, subtract, multiply, divide, sqrt and cbrt one flop "
                                  "each; min/max, abs and compares listed apart",
                       "sample": f"one oracle step of the same {sc.nx}x{sc.ny} workload"}
    if gpu_value:
        tf = flops * gpu_value / 1e12
        out["op_tally"].update(gpu_algorithmic_tflops=tf,
                               frac_of_fp64_vector_peak=tf / FP64_VECTOR_PEAK_TFLOPS)
    of = oracle.Oracle(sc.as_fv1(), tallied=True)
    of.tally_reset()
    of.step()
    per = {k: v / (sc.nx * sc.ny) for k, v in of.tally_read().items()}
    flops = per["add"] + per["mul"] + per["div"] + per["sqrt"] + per["cbrt"]
    out["op_tally_fv1"] = {"per_cell_step": per, "flops_per_cell_step": flops,
                           "sample": f"one oracle FV1 step of the same {sc.nx}x{sc.ny} workload"}
    for prec, v in (fv1_values or {}).items():
        out["op_tally_fv1"][f"gpu_algorithmic_tflops_{prec}"] = flops * v / 1e12
    return out


def fp32_leg(dg2, S, n, steps, warmup, copy_gbs=None):
    """The DG2 step in FP32 with per-tile bed datums on the all-wet terrain: cell-updates/s,
    the stage kernels' HIP-event times and the step's fraction of the HBM roofline by
    the FP32 algorithmic bytes (188 B per cell-step), with the counter traffic where a
    record for the current kernel sources exists."""
    import torch
    sc = S.fbm_channel_wet(n=n)
    n_cells = sc.nx * sc.ny
    s32 = dg2.DG2(sc, dg2.FP32)
    for _ in range(warmup):
        s32.step(sync=False)
    torch.cuda.synchronize()
    el, tm, n_windows = timed_steps(s32, steps)
    ms = {"stage1": tm["ms_stage1"], "stage2": tm["ms_stage2"]}
    step_alg = stage_bytes("stage1", n_cells, 4) + stage_bytes("stage2", n_cells, 4)
    rate = step_alg / ((ms["stage1"] + ms["stage2"]) * 1e-3) / 1e9
    rec = f"traffic_stage_kernels_fbm_channel_wet_{n}_fp32"
    info = s32.kernel_info()
    out = {"value": n_cells * steps / el, "unit": "cell-updates/s", "windows": n_windows,
           "tile": [info["tile_x"], info["tile_y"]], "ms_per_launch": ms,
           "algorithmic_bytes_per_launch": {k: stage_bytes(k, n_cells, 4) for k in ms},
           "step_frac": rate / HBM_PEAK_GBS,
           "traffic": {k: measured_traffic(rec, k) for k in ms}}
    if copy_gbs:
        out["step_frac_of_copy"] = rate / copy_gbs
    return out


def fv1_leg(dg2, S, n, steps, warmup, copy_gbs=None):
    """The FV1 scheme (one launch per step) on the same all-wet terrain, FP64 and FP32:
    cell-updates/s and the fraction of the HBM roofline. Algorithmic bytes per cell and
    step: the three means and one bed vertex read, the three means written."""
    import torch
    sc = S.fbm_channel_wet(n=n).as_fv1()
    out = {"workload": f"FV1 (Courant number 0.5) on fbm+channel terrain {n}x{n}, every cell wet"}
    for prec, tag, rb in ((dg2.FP64, "fp64", 8), (dg2.FP32, "fp32", 4)):
        sim = dg2.DG2(sc, prec)
        for _ in range(warmup):
            sim.step(sync=False)
        torch.cuda.synchronize()
        el, tm, _ = timed_steps(sim, steps)
        ms = tm["ms_stage1"]
        bytes_ = 7 * rb * n * n
        out[tag] = {"value": n * n * steps / el, "unit": "cell-updates/s", "ms_per_launch": ms,
                    "algorithmic_bytes_per_launch": bytes_,
                    "roofline_frac": bytes_ / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                    "frac_of_copy": (bytes_ / (ms * 1e-3) / 1e9 / copy_gbs) if copy_gbs else None,
                    "traffic": measured_traffic(f"traffic_fv1_kernel_fbm_channel_wet_{n}", tag)}
    return out


def adjoint_leg(dg2, S, n, steps, n_gauges=32):
    """Gradients of a gauge misfit through the discrete adjoint: a fully wet, limiter-off
    flow on an n x n fBm terrain (dx 5 m) with Manning n in 16 zones and a 48-knot inflow
    hydrograph, `steps` RK2 steps on a replayed schedule (0.8 of the CFL steps of a plain
    run), misfit against a run with every zone value raised by 20 %. Times the plain
    forward, the recorded forward and the adjoint, and checks two zone and two knot
    gradients against central differences of the misfit (steps of 1e-4 relative)."""
    import torch
    sc = S.adjoint_case(n=n, dx=5.0, t_span=200.0, n_knots=48)
    rng = np.random.default_rng(5)
    gi = rng.choice(n * n, size=n_gauges, replace=False)
    probe = dg2.DG2(sc, dg2.FP64)
    dts = np.array([0.8 * probe.step() for _ in range(steps)])
    del probe
    zi = S.zone_index(n, 4)
    nz0 = np.array([sc.manning.reshape(-1)[zi.reshape(-1) == z][0] for z in range(16)])
    q0 = np.asarray(sc.boundaries[0].q_knots, dtype=np.float64)

    def run(manning=None, q=None, keep=False):
        sim = dg2.DG2(sc, dg2.FP64)
        if manning is not None:
            sim.set_manning(manning)
        if q is not None:
            sim.set_hydrograph(0, q)
        tape = dg2.Tape(sim, dts, gi, checkpoint_every=-1 if keep else 0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h = tape.forward()
        return sim, tape, h, time.perf_counter() - t0

    _, _, href, _ = run(manning=(nz0 * 1.2)[zi])
    # plain forward with the same schedule (no tape)
    plain = dg2.DG2(sc, dg2.FP64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for dt in dts:
        plain.step(dt_max=float(dt), sync=False)   # each step is capped at dts[k]
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    # the same schedule as the tape (the CFL step never fell below dts[k])
    assert abs(plain.scalars()["t"] - float(np.sum(dts))) <= 1e-9 * float(np.sum(dts))
    sim, tape, h, t_fwd = run()
    J = float(((h - href) ** 2).sum())
    t0 = time.perf_counter()
    gm, gq, _ = tape.backward(2.0 * (h - href), len(q0))
    t_bwd = time.perf_counter() - t0
    gz = np.array([gm.reshape(-1)[zi.reshape(-1) == z].sum() for z in range(16)])
    del tape, sim
    # the same gradient with every step's stage states kept by the forward run (three
    # states per step of HBM, no recomputation in the backward pass)
    simk, tapek, hk, t_fwd_k = run(keep=True)
    t0 = time.perf_counter()
    gmk, gqk, _ = tapek.backward(2.0 * (hk - href), len(q0))
    t_bwd_k = time.perf_counter() - t0
    same = bool(np.array_equal(gmk, gm) and np.array_equal(gqk, gq) and np.array_equal(hk, h))
    del tapek, simk

    def misfit(manning=None, q=None):
        return float(((run(manning=manning, q=q)[2] - href) ** 2).sum())

    checks = {}
    for z in (0, 5):
        e = 1e-4 * nz0[z]
        p_, m_ = nz0.copy(), nz0.copy()
        p_[z] += e
        m_[z] -= e
        fd = (misfit(manning=p_[zi]) - misfit(manning=m_[zi])) / (2 * e)
        checks[f"zone{z}"] = {"adjoint": float(gz[z]), "fd": fd}
    for k in (10, 30):
        e = 1e-4 * q0[k]
        p_, m_ = q0.copy(), q0.copy()
        p_[k] += e
        m_[k] -= e
        fd = (misfit(q=p_) - misfit(q=m_)) / (2 * e)
        checks[f"knot{k}"] = {"adjoint": float(gq[k]), "fd": fd}
    worst = max(abs(c["adjoint"] - c["fd"]) / max(abs(c["fd"]), 1e-300) for c in checks.values())
    return {"workload": f"fully wet fBm {n}x{n}, dx 5 m, 16 Manning zones, 48-knot inflow, "
                        f"{steps} steps, {n_gauges} gauges, FP64",
            "misfit": J, "checkpoint_every": int(np.ceil(np.sqrt(steps))),
            "seconds": {"forward_plain": t_plain, "forward_recorded": t_fwd, "adjoint": t_bwd},
            "adjoint_over_forward": t_bwd / t_plain,
            "gradient_over_forward": (t_fwd + t_bwd) / t_plain,
            "keep_every_step": {
                "seconds": {"forward_recorded": t_fwd_k, "adjoint": t_bwd_k},
                "adjoint_over_forward": t_bwd_k / t_plain,
                "gradient_over_forward": (t_fwd_k + t_bwd_k) / t_plain,
                "device_bytes": 3 * (len(dts) + 1) * 9 * n * n * 8,
                "bitwise_equal_to_checkpointed": same},
            "fd_checks": checks, "max_rel_diff_vs_fd": worst}


def precision_form(dg2, S, n, t_end):
    """FP32 with per-tile bed datums against FP64.

    Urban terrain (flat ground with building blocks, dry start, 1 m deep inflow at 2 m/s
    along the west edge), both precisions advanced side by side to checkpoints up to
    t_end: FP32 depth error against the FP64 run at each checkpoint, mass-balance
    drift at the end, cell-update rates. Then the all-wet channel terrain raised by
    1000 m, 60 s: FP32 with datums against FP32 storing absolute elevations."""
    import torch
    sc = S.urban_blocks(n=n)
    res = {"workload": f"urban blocks {n}x{n}, dx=2 m, 4000 blocks, 1 m at 2 m/s inflow on W, "
                       "n=0.02, dry start", "cells": n * n}
    sims = {"fp64": dg2.DG2(sc, dg2.FP64), "fp32_datum": dg2.DG2(sc, dg2.FP32)}
    secs = {k: 0.0 for k in sims}
    steps = {k: 0 for k in sims}
    errs = []
    for tc in (10.0, 60.0, t_end):
        for k, sim in sims.items():
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            steps[k] += sim.run(tc)
            secs[k] += time.perf_counter() - t0
        d = sims["fp32_datum"].read(0).astype(np.float64) - sims["fp64"].read(0)
        errs.append({"t": tc, "max_depth_error_m": float(np.abs(d).max()),
                     "rms_depth_error_m": float(np.sqrt(np.mean(d * d)))})
    for k, sim in sims.items():
        sc_ = sim.scalars()
        bal = sc_["mass"] - sc_["mass_in"] + sc_["mass_out"] - sc_["mass_clip"]  # dry start
        res[k] = {"value": n * n * steps[k] / secs[k], "unit": "cell-updates/s",
                  "steps": steps[k], "mass_balance_rel": bal / max(sc_["mass"], sc_["mass_in"]),
                  "bed_quantum_m": sim.bed_info()["quantum"]}
    res["fp32_datum"]["depth_error_vs_fp64"] = errs
    del sims

    hi = S.fbm_channel_wet(n=1024)
    hi = hi.replace(zv=hi.zv + 1000.0)  # initial depths are given, not levels
    ref = dg2.DG2(hi, dg2.FP64)
    ref.run(60.0)
    h64 = ref.read(0)
    elev = {"workload": "the all-wet channel terrain with the bed raised by 1000 m, t=60 s"}
    for key, datum in (("fp32_datum", True), ("fp32_absolute", False)):
        sim = dg2.DG2(hi, dg2.FP32, bed_datum=datum)
        sim.run(60.0)
        d = sim.read(0).astype(np.float64) - h64
        elev[key] = {"max_depth_error_m": float(np.abs(d).max()),
                     "rms_depth_error_m": float(np.sqrt(np.mean(d * d))),
                     "bed_quantum_m": sim.bed_info()["quantum"]}
    res["bed_plus_1000m"] = elev
    res["error_vs"] = ("the FP64 GPU run on the same bed; the parity tests hold that run to the "
                       "FP64 oracle at 1e-12 on a 2048x512 window of this terrain (100 steps from "
                       "the oracle's state at t=300 s) and check the FP32 path against the oracle "
                       "on it")
    return res


def batched(dg2, S, count, t_end):
    """count scenarios of uneven size (seeded; FP32 with bed datums, FP64 mass ledgers)
    run to t_end as one batch (shared launches from a HIP graph, tile shape from the
    autotuner), then the same scenarios one after another; aggregate cell-updates/s of
    both, and whether every member ends bitwise where it does alone."""
    import torch
    from paper_2107_02750_amd import autotune
    scs = S.batch_scenarios(count=count, t_end=t_end)
    cells = [sc.nx * sc.ny for sc in scs]
    stream = torch.cuda.Stream()
    tuned = autotune.tune_batch(scs, dg2.FP32, stream)
    tile = tuned["best"]
    sims = [dg2.DG2(sc, dg2.FP32, stream=stream, tile=tile) for sc in scs]
    batch = dg2.Batch(sims, graph_steps=32)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps, pairs = batch.run(t_end)
    el = time.perf_counter() - t0
    batch.close()
    work = sum(c * k for c, k in zip(cells, steps))
    drift = 0.0
    for sim in sims:
        s_ = sim.scalars()
        bal = s_["mass"] - s_["mass_in"] + s_["mass_out"] - s_["mass_clip"]  # dry start
        drift = max(drift, abs(bal) / max(s_["mass"], s_["mass_in"], 1e-300))
    seq_el = 0.0
    slowest = 0.0
    equal = True
    for sc, sim in zip(scs, sims):
        one = dg2.DG2(sc, dg2.FP32, stream=stream, tile=tile)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        one.run(t_end)
        el_one = time.perf_counter() - t0
        seq_el += el_one
        slowest = max(slowest, el_one)
        equal = equal and one.get_state() == sim.get_state()
        del one
    return {"workload": f"{count} fBm channel scenarios, sides U{{256..1024}} (total "
                        f"{sum(cells)} cells), dx U[2,10] m, n U(0.015,0.06), inflow peaks "
                        f"U(5,100) m^3/s, dry start, each run to t={t_end:.0f} s, FP32 with bed datums",
            "value": work / el, "unit": "cell-updates/s", "seconds": el,
            "member_steps": {"min": min(steps), "max": max(steps), "total": sum(steps)},
            "launch_pairs": pairs,
            "one_at_a_time": {"value": work / seq_el, "seconds": seq_el},
            "speedup": seq_el / el, "bitwise_equal_to_one_at_a_time": equal,
            "slowest_member_alone_s": slowest,
            "tile": list(tile), "autotuner_ms_per_step": tuned["ms_per_step"],
            "max_mass_balance_rel": drift}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--n", type=int, default=1024, help="grid side (default: the 1024 case)")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--n-urban", type=int, default=2048, help="grid side of the urban precision run")
    ap.add_argument("--t-urban", type=float, default=600.0, help="simulated seconds of the urban run")
    ap.add_argument("--batch-count", type=int, default=64, help="scenarios in the batched run")
    ap.add_argument("--batch-t-end", type=float, default=1800.0, help="simulated seconds per scenario")
    ap.add_argument("--adjoint-n", type=int, default=512, help="grid side of the adjoint leg")
    ap.add_argument("--adjoint-steps", type=int, default=2000, help="RK2 steps of the adjoint leg")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the FP64 timed region (for profiler runs)")
    ap.add_argument("--fv1-only", action="store_true",
                    help="only the FV1 leg, as its own JSON line (for profiler runs)")
    ap.add_argument("--fp32-only", action="store_true",
                    help="only the FP32 DG2 step on the all-wet terrain (profiler runs)")
    ap.add_argument("--batched-only", action="store_true",
                    help="only the batched-scenario leg (profiler runs)")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="only the adjoint leg, as its own JSON line (for profiler runs)")
    ap.add_argument("--min-seconds", type=float, default=1.0,
                    help="timed windows repeat until this much has been timed (profiler runs: 0)")
    ap.add_argument("--event-seconds", type=float, default=0.25,
                    help="evented windows repeat until this much has run (profiler runs: 0)")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="also run one device-to-device copy of this many MiB (counter scale)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the step would shard by 2D domain decomposition with halo exchange).",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2107_02750_amd import dg2, scenarios as S

    TIMING.update(min_seconds=args.min_seconds, event_seconds=args.event_seconds)
    if args.fv1_only:
        r = fv1_leg(dg2, S, args.n, args.steps, args.warmup, copy_bandwidth())
        if args.calibrate_copy_mib:
            a = torch.empty(args.calibrate_copy_mib << 20, dtype=torch.uint8, device="cuda")
            torch.empty_like(a).copy_(a)
            torch.cuda.synchronize()
        print(json.dumps({"metric": "FV1 cell-updates/s (forward-Euler step, FP64)",
                          "value": r["fp64"]["value"], "unit": "cell-updates/s", "fv1": r}),
              flush=True)
        return

    if args.fp32_only:
        r = fp32_leg(dg2, S, args.n, args.steps, args.warmup, copy_bandwidth())
        if args.calibrate_copy_mib:
            a = torch.empty(args.calibrate_copy_mib << 20, dtype=torch.uint8, device="cuda")
            torch.empty_like(a).copy_(a)
            torch.cuda.synchronize()
        print(json.dumps({"metric": "DG2 cell-updates/s (full RK2 step, FP32 with bed datums)",
                          "value": r["value"], "unit": "cell-updates/s", "fp32": r}), flush=True)
        return

    if args.batched_only:
        r = batched(dg2, S, args.batch_count, args.batch_t_end)
        print(json.dumps({"metric": "batched scenarios, aggregate cell-updates/s (FP32)",
                          "value": r["value"], "unit": "cell-updates/s", "batched": r}),
              flush=True)
        return

    if args.adjoint_only:
        r = adjoint_leg(dg2, S, args.adjoint_n, args.adjoint_steps)
        if args.calibrate_copy_mib:
            a = torch.empty(args.calibrate_copy_mib << 20, dtype=torch.uint8, device="cuda")
            torch.empty_like(a).copy_(a)
            torch.cuda.synchronize()
        print(json.dumps({"metric": "adjoint time over forward time (gauge misfit gradients)",
                          "value": r["adjoint_over_forward"], "unit": "ratio", "adjoint": r}),
              flush=True)
        return

    sc = S.fbm_channel_wet(n=args.n)
    n_cells = sc.nx * sc.ny
    print(f"[bench] workload {sc.name} {sc.nx}x{sc.ny}, FP64 warmup {args.warmup}, "
          f"steps {args.steps}", file=sys.stderr, flush=True)
    sim = dg2.DG2(sc, dg2.FP64)
    for _ in range(args.warmup):
        sim.step(sync=False)
    torch.cuda.synchronize()
    TIMING.update(min_seconds=args.min_seconds, event_seconds=args.event_seconds)
    el, tm, n_windows = timed_steps(sim, args.steps)
    value = n_cells * args.steps / el
    ms1, ms2 = tm["ms_stage1"], tm["ms_stage2"]
    dom, dom_ms = ("stage2", ms2) if ms2 >= ms1 else ("stage1", ms1)
    achieved = stage_bytes(dom, n_cells, 8) / (dom_ms * 1e-3) / 1e9
    frac_of = {k: stage_bytes(k, n_cells, 8) / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS
               for k, ms in (("stage1", ms1), ("stage2", ms2))}
    step_alg = stage_bytes("stage1", n_cells, 8) + stage_bytes("stage2", n_cells, 8)
    info = sim.kernel_info()
    copy_gbs = copy_bandwidth()
    print(f"[bench] FP64 {value:.4g} cell-updates/s, stage1 {ms1:.4f} ms, stage2 {ms2:.4f} ms, "
          f"device copy {copy_gbs:.0f} GB/s", file=sys.stderr, flush=True)

    if args.calibrate_copy_mib:
        a = torch.empty(args.calibrate_copy_mib << 20, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()

    out = {
        "metric": "DG2 cell-updates/s (full RK2 step, FP64)",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"fbm+channel terrain {sc.nx}x{sc.ny}, dx=5 m, n=0.035, "
                               "flooded to 25 m with qx=2 m^2/s (every cell wet)",
                   "cells": n_cells, "tile": [info["tile_x"], info["tile_y"]],
                   "blocks_per_launch": info["blocks"],
                   "timing": f"median of {n_windows} windows of {args.steps} steps "
                             f"(at least 1 s timed in all)", "windows": n_windows},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(
                         f"traffic_stage_kernels_fbm_channel_wet_{args.n}_fp64", dom),
                     "ms_per_launch": {"stage1": ms1, "stage2": ms2},
                     "algorithmic_bytes_per_launch": stage_bytes(dom, n_cells, 8),
                     "frac_per_kernel": frac_of,
                     "step_frac": step_alg / ((ms1 + ms2) * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "copy_gbs": copy_gbs,
                     "frac_of_copy": achieved / copy_gbs,
                     "step_frac_of_copy": step_alg / ((ms1 + ms2) * 1e-3) / 1e9 / copy_gbs,
                     "implementation_bytes_per_launch": {
                         k: stage_bytes(k, n_cells, 8, IMPL_VALUES) for k in ("stage1", "stage2")}},
    }
    if not args.no_extras:
        # FP32 instantiation, same workload, and its depth error against FP64 at t = 60 s
        out["fp32"] = fp32_leg(dg2, S, args.n, args.steps, args.warmup, copy_gbs)
        a64, a32 = dg2.DG2(sc, dg2.FP64), dg2.DG2(sc, dg2.FP32)
        a64.run(60.0)
        a32.run(60.0)
        h64 = a64.read(0)
        h32 = a32.read(0).astype(np.float64)
        d = h32 - h64
        out["fp32"].update({
            "max_depth_error_m": float(np.abs(d).max()),
            "rms_depth_error_m": float(np.sqrt(np.mean(d * d))),
            "error_at": "t=60 s vs the FP64 GPU path (held to the FP64 oracle at 1e-12 by the parity tests)"})
        print(f"[bench] FP32 {out['fp32']['value']:.4g} cell-updates/s, max depth err "
              f"{out['fp32']['max_depth_error_m']:.3g} m", file=sys.stderr, flush=True)
        # the terrain as configured: dry start, inflow hydrograph, snapshot at t = 3600 s
        dry = S.fbm_channel(n=args.n)
        sd = dg2.DG2(dry, dg2.FP64)
        t0 = time.perf_counter()
        spin = sd.run(3600.0)
        spin_s = time.perf_counter() - t0
        wet = float((sd.read(0) > dry.h_tol).mean())
        eld, _, _ = timed_steps(sd, args.steps)
        out["as_configured"] = {"workload": "same terrain, dry start, 50 m^3/s trapezoid inflow, "
                                            "timed from the state at t=3600 s",
                                "value": n_cells * args.steps / eld, "wet_fraction": wet,
                                "spin_up_steps": spin, "spin_up_s": spin_s}
        print(f"[bench] as configured {out['as_configured']['value']:.4g} cell-updates/s, "
              f"wet {wet:.4f}", file=sys.stderr, flush=True)
        out["fv1"] = fv1_leg(dg2, S, args.n, args.steps, args.warmup, copy_gbs)
        print(f"[bench] FV1 FP64 {out['fv1']['fp64']['value']:.4g} cell-updates/s "
              f"({out['fv1']['fp64']['roofline_frac']:.2f} of HBM roofline), FP32 "
              f"{out['fv1']['fp32']['value']:.4g}", file=sys.stderr, flush=True)
        out["precision_form"] = precision_form(dg2, S, args.n_urban, args.t_urban)
        pf = out["precision_form"]
        e = pf["fp32_datum"]["depth_error_vs_fp64"]
        print(f"[bench] urban {pf['cells']} cells: FP32 datum max/rms depth err "
              + ", ".join(f"t={x['t']:.0f} s {x['max_depth_error_m']:.2g}/{x['rms_depth_error_m']:.2g} m"
                          for x in e)
              + f"; bed +1000 m, t=60 s: datum {pf['bed_plus_1000m']['fp32_datum']['max_depth_error_m']:.2g} m, "
              f"absolute {pf['bed_plus_1000m']['fp32_absolute']['max_depth_error_m']:.2g} m",
              file=sys.stderr, flush=True)
        out["batched"] = batched(dg2, S, args.batch_count, args.batch_t_end)
        bt = out["batched"]
        print(f"[bench] batched {args.batch_count} scenarios: {bt['value']:.4g} cell-updates/s "
              f"({bt['seconds']:.1f} s), one at a time {bt['one_at_a_time']['value']:.4g} "
              f"({bt['one_at_a_time']['seconds']:.1f} s), bitwise equal: "
              f"{bt['bitwise_equal_to_one_at_a_time']}", file=sys.stderr, flush=True)
        out["adjoint"] = adjoint_leg(dg2, S, args.adjoint_n, args.adjoint_steps)
        ad = out["adjoint"]
        print(f"[bench] adjoint {args.adjoint_n}^2 x {args.adjoint_steps} steps: forward "
              f"{ad['seconds']['forward_plain']:.3f} s, adjoint {ad['seconds']['adjoint']:.3f} s "
              f"({ad['adjoint_over_forward']:.1f}x; gradient {ad['gradient_over_forward']:.2f}x, keeping "
              f"every step {ad['keep_every_step']['gradient_over_forward']:.2f}x), max rel diff vs FD "
              f"{ad['max_rel_diff_vs_fd']:.1e}",
              file=sys.stderr, flush=True)
        fv1_values = ({k: out["fv1"][k]["value"] for k in ("fp64", "fp32")}
                      if "fv1" in out else None)
        out["cpu_baseline"] = cpu_baseline(sc, args.cpu_budget, gpu_value=value,
                                           fv1_values=fv1_values)
        cb = out["cpu_baseline"]
        print(f"[bench] CPU oracle {cb['value']:.4g} cell-updates/s on {cb['cores']} threads, "
              f"{cb['one_core']['value']:.4g} on one"
              + (f"; as configured {cb['as_configured']['value']:.4g}" if "as_configured" in cb else "")
              + f"; {cb['op_tally']['flops_per_cell_step']:.0f} algorithmic flops per cell-step "
              f"({cb['op_tally']['gpu_algorithmic_tflops']:.2f} TFLOP/s on the GPU)",
              file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
