"""Batched scenarios: several contexts of uneven grid size advanced by shared launches
(one launch per stage over all their tiles, replayed from a HIP graph).

Each member keeps its own time step, so a batched step must leave every member
bitwise where a step of that member alone would: states, times, step counts and mass
ledgers are compared exactly against members stepped one at a time, after several
graph replays with host work (reads, synchronisations) between them, and one member
is also checked against the FP64 oracle.
"""
import numpy as np
import pytest

from oracle import Oracle
from paper_2107_02750_amd import scenarios as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2107_02750_amd import dg2 as mod
    mod.load()
    stream = torch.cuda.Stream()  # default priority; graphs cannot capture the null stream
    return mod, stream


def members():
    return [
        S.dam_break(nx=100, ny=40),
        S.window(S.urban_wet(n=256, n_blocks=60), 96, 72),
        S.fbm_channel(n=70, dx=5.0, amplitude=40.0, wavelength=250.0, q_peak=20.0),
        S.lake_at_rest(nx=33, ny=17),
        S.partially_dry_lake(),
    ]


def make(mod, stream, prec):
    return [mod.DG2(sc, prec, stream=stream) for sc in members()]


def same(a, b):
    return a.get_state() == b.get_state()


@pytest.mark.parametrize("prec_name", ["FP64", "FP32"])
def test_graph_replays_match_single_steps(env, prec_name):
    mod, stream = env
    prec = getattr(mod, prec_name)
    batched, alone = make(mod, stream, prec), make(mod, stream, prec)
    batch = mod.Batch(batched, graph_steps=8)
    done = 0
    for chunk in (8, 8, 5, 8, 3):  # replays, an odd tail, replays again
        batch.step(chunk)
        for s in alone:
            for _ in range(chunk):
                s.step(sync=False)
        done += chunk
        stream.synchronize()
        for k, (a, b) in enumerate(zip(batched, alone)):
            assert same(a, b), (prec_name, k, done)
            assert a.scalars() == b.scalars()
    print(f"{prec_name}: {len(batched)} members bitwise equal after {done} steps", flush=True)
    batch.close()


def test_batch_run_lands_on_t_end_per_member(env):
    mod, stream = env
    batched, alone = make(mod, stream, mod.FP64), make(mod, stream, mod.FP64)
    batch = mod.Batch(batched, graph_steps=16)
    steps, launches = batch.run(3.0)
    ref = [s.run(3.0) for s in alone]
    assert steps == ref
    assert launches >= max(ref)
    for a, b in zip(batched, alone):
        assert a.scalars()["t"] == 3.0
        assert same(a, b)
    # a second run continues from there; the oracle, run on the same schedule (to 3 s,
    # then to 5 s), agrees with a batched member
    batch.run(5.0)
    o = Oracle(members()[2])
    o.run(3.0)
    o.run(5.0)
    g = batched[2]
    P, Q = g.planes(), o.planes()
    H = max(np.abs(Q[0]).max(), 1e-3)
    Qs = max(np.abs(Q[3]).max(), np.abs(Q[6]).max(), 1e-3)
    scale = np.array([H] * 3 + [Qs] * 6)
    err = max(np.abs(P[p] - Q[p]).max() / scale[p] for p in range(9))
    print(f"batched member vs oracle at t=5 s: {err:.2e}", flush=True)
    assert err <= 1e-12
    batch.close()


def test_members_are_borrowed(env):
    mod, stream = env
    sims = make(mod, stream, mod.FP64)[:2]
    batch = mod.Batch(sims)
    with pytest.raises(mod.DG2Error) as e:
        sims[0].step()
    assert e.value.code == mod.E_STATE
    with pytest.raises(mod.DG2Error) as e:
        mod.Batch([sims[1]])          # already in a batch
    assert e.value.code == mod.E_ARG
    batch.close()
    sims[0].step()                    # free again
    mixed = [mod.DG2(S.dam_break(nx=20, ny=4), mod.FP64, stream=stream),
             mod.DG2(S.dam_break(nx=20, ny=4), mod.FP32, stream=stream)]
    with pytest.raises(mod.DG2Error) as e:
        mod.Batch(mixed)
    assert e.value.code == mod.E_ARG
    with pytest.raises(mod.DG2Error) as e:
        mod.Batch(sims, graph_steps=7)
    assert e.value.code == mod.E_ARG
