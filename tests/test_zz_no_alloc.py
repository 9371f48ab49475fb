"""The entry point that allocates nothing (dg2_step_noalloc, scratch in a static device
array) against a context's step (dg2_step): the same kernels on the same inputs, so
the same time step and bitwise the same planes. Two calls in a row, the second on a
smaller grid, so the second runs on what the first left in the shared scratch."""
import numpy as np
import pytest
import torch

from paper_2107_02750_amd import scenarios as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dg2():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2107_02750_amd import dg2 as mod
    mod.load()
    return mod


def planes_device(sim):
    return torch.stack([sim.read_device(p) for p in range(9)]).contiguous()


def one_step_both_ways(dg2, sc, manning_plane):
    print(f"case {sc.name} {sc.nx}x{sc.ny}", flush=True)
    sim = dg2.DG2(sc, dg2.FP64)
    u0 = planes_device(sim)
    t0 = sim.scalars()["t"]
    dt_ctx = sim.step()
    u1 = planes_device(sim)
    zv = torch.as_tensor(np.ascontiguousarray(sc.zv), dtype=torch.float64, device="cuda")
    man = (torch.as_tensor(np.ascontiguousarray(sc.manning), dtype=torch.float64, device="cuda")
           if manning_plane else None)
    out = torch.full_like(u0, float("nan"))
    dt = dg2.step_noalloc(sc, zv, u0, out, t0, manning=man)
    assert dt == dt_ctx
    assert torch.equal(out, u1)
    assert torch.equal(u0, planes_device(dg2.DG2(sc, dg2.FP64)))   # input untouched
    return dt


def test_no_alloc_step_matches_context_step(dg2):
    # a wet channel terrain with an inflow segment and per-cell Manning n (several
    # tiles, partial edge tiles), then a smaller urban window with a fixed inflow state
    big = S.adjoint_case(n=203, dx=5.0, t_span=10.0, n_knots=6).replace(limiter=1)
    one_step_both_ways(dg2, big, manning_plane=True)
    small = S.window(S.urban_wet(n=128, n_blocks=20), 75, 41)
    one_step_both_ways(dg2, small, manning_plane=False)


def test_no_alloc_rejects_what_it_cannot_do(dg2):
    sc = S.dam_break(nx=20, ny=4)
    u = torch.zeros((9, 4, 20), dtype=torch.float64, device="cuda")
    zv = torch.zeros((5, 21), dtype=torch.float64, device="cuda")
    with pytest.raises(dg2.DG2Error) as e:
        dg2.step_noalloc(sc, zv, u, u, 0.0)        # same buffer in and out
    assert e.value.code == dg2.E_ARG
    big = S.Scenario("big", 1024, 1024, 1.0, np.zeros((2, 2)), S.MODE_MEANS)
    ub = torch.zeros((9, 1024, 1024), dtype=torch.float64, device="cuda")
    zb = torch.zeros((1025, 1025), dtype=torch.float64, device="cuda")
    with pytest.raises(dg2.DG2Error) as e:
        dg2.step_noalloc(big, zb, ub, torch.empty_like(ub), 0.0)   # scratch too small
    assert e.value.code == dg2.E_ARG
    assert "scratch" in str(e.value)
