"""The library's discrete adjoint (through the C interface) against the differentiable
FP64 CPU reference (oracle/adjoint_ref.py, itself pinned to the C oracle and to finite
differences), on a fully wet, limiter-off flow with zoned Manning n and a knotted
inflow hydrograph, over a replayed time-step schedule.

Checked: the recorded gauge depths (1e-12 relative), the gradients of a gauge misfit
with respect to the per-cell Manning n (summed over zones) and the hydrograph knots
(1e-7 relative to the largest component) and the initial state (1e-6), also with wall
edges and a fixed-state segment, independence from the checkpoint spacing (bit for
bit), a grid whose last tile column and row are partial, the torch.autograd.Function
wrapper, and the regime check. Measured agreement on this case: 2e-9 (zones), 3e-9 (knots),
2.5e-8 (initial state, largest at boundary cells); over 5 to 40 steps it does not
grow. The gradients are sums over cells and steps with cancellation that the two
sides form in different orders on states that differ in the last bits; the larger
initial-state differences at boundary cells are not explained beyond that.
"""
import numpy as np
import pytest
import torch

from oracle import Oracle
from oracle.adjoint_ref import WetDG2
from paper_2107_02750_amd import scenarios as S

pytestmark = pytest.mark.gpu

N, STEPS = 40, 40


@pytest.fixture(scope="module")
def dg2():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2107_02750_amd import dg2 as mod
    mod.load()
    return mod


def case():
    return S.adjoint_case(n=N, dx=5.0, t_span=4.0, n_knots=8)


def schedule(sc, steps):
    o = Oracle(sc)
    dts = []
    for _ in range(steps):
        dts.append(0.9 * o.next_dt())
        o.step(dts[-1])
    return np.array(dts)


def gauges(n, k=16, seed=5):
    rng = np.random.default_rng(seed)
    far = rng.choice(n * n, size=k // 2, replace=False)
    near = [(n // 2 + int(rng.integers(-6, 7))) * n + int(rng.integers(0, 5)) for _ in range(k - k // 2)]
    return np.concatenate([far, near]).astype(np.int64)


def reference(sc, dts, gi, href):
    """misfit J and its gradients (zones, knots, U0) from the CPU reference"""
    ref = WetDG2(sc)
    zi = S.zone_index(sc.nx, 4)
    nz0 = np.array([sc.manning.reshape(-1)[zi.reshape(-1) == z][0] for z in range(16)])
    nz = torch.tensor(nz0, requires_grad=True)
    qk = torch.tensor(np.asarray(sc.boundaries[0].q_knots, dtype=np.float64), requires_grad=True)
    U0 = torch.tensor(Oracle(sc).planes(), requires_grad=True)
    n_cell = nz[torch.as_tensor(zi)]
    U, t, J = U0, 0.0, 0.0
    hs = [U0[0].reshape(-1)[torch.as_tensor(gi)].detach().numpy()]
    J = ((U0[0].reshape(-1)[torch.as_tensor(gi)] - torch.as_tensor(href[0])) ** 2).sum()
    for k, dt in enumerate(dts):
        U = ref.step(U, float(dt), t, n_cell, [qk])
        t += float(dt)
        hk = U[0].reshape(-1)[torch.as_tensor(gi)]
        hs.append(hk.detach().numpy())
        J = J + ((hk - torch.as_tensor(href[k + 1])) ** 2).sum()
    J.backward()
    return float(J.detach()), np.array(hs), nz.grad.numpy(), qk.grad.numpy(), U0.grad.numpy()


def href_of(sc, dts, gi):
    zi = S.zone_index(sc.nx, 4)
    nz0 = np.array([sc.manning.reshape(-1)[zi.reshape(-1) == z][0] for z in range(16)])
    o = Oracle(sc.replace(manning=(nz0 * 1.2)[zi]))
    out = [o.read(0).ravel()[gi]]
    for dt in dts:
        o.step(dt)
        out.append(o.read(0).ravel()[gi])
    return np.array(out)


def test_adjoint_matches_reference_gradient(dg2):
    sc = case()
    dts = schedule(sc, STEPS)
    gi = gauges(N)
    href = href_of(sc, dts, gi)
    J, hs_ref, gz_ref, gq_ref, gu_ref = reference(sc, dts, gi, href)
    sim = dg2.DG2(sc, dg2.FP64)
    tape = dg2.Tape(sim, dts, gi)
    hs = tape.forward()
    assert np.abs(hs - hs_ref).max() <= 1e-12 * np.abs(hs_ref).max()
    assert J > 0
    gm, gq, gu = tape.backward(2.0 * (hs - href), len(sc.boundaries[0].q_knots))
    zi = S.zone_index(N, 4)
    gz = np.array([gm.reshape(-1)[zi.reshape(-1) == z].sum() for z in range(16)])
    ez = np.abs(gz - gz_ref).max() / np.abs(gz_ref).max()
    eq = np.abs(gq - gq_ref).max() / np.abs(gq_ref).max()
    eu = np.abs(gu - gu_ref).max() / np.abs(gu_ref).max()
    print(f"adjoint vs reference: zones {ez:.2e}, knots {eq:.2e}, U0 {eu:.2e}", flush=True)
    assert ez <= 1e-7 and eq <= 1e-7 and eu <= 1e-6
    # the checkpoint spacing changes nothing
    sim2 = dg2.DG2(sc, dg2.FP64)
    tape2 = dg2.Tape(sim2, dts, gi, checkpoint_every=7)
    assert np.array_equal(tape2.forward(), hs)
    gm2, gq2, gu2 = tape2.backward(2.0 * (hs - href), len(sc.boundaries[0].q_knots))
    assert np.array_equal(gm2, gm) and np.array_equal(gq2, gq) and np.array_equal(gu2, gu)
    # nor does keeping every step's states (no recomputation in the backward pass); the
    # context ends where the checkpointed run left it and steps on from there alike
    sim3 = dg2.DG2(sc, dg2.FP64)
    tape3 = dg2.Tape(sim3, dts, gi, checkpoint_every=-1)
    assert np.array_equal(tape3.forward(), hs)
    gm3, gq3, gu3 = tape3.backward(2.0 * (hs - href), len(sc.boundaries[0].q_knots))
    assert np.array_equal(gm3, gm) and np.array_equal(gq3, gq) and np.array_equal(gu3, gu)
    assert sim3.get_state() == sim2.get_state()
    assert sim3.step() == sim2.step() and sim3.planes().tobytes() == sim2.planes().tobytes()


def test_adjoint_with_walls_and_a_fixed_segment(dg2):
    """Wall edges (reflected normal velocity) and a fixed-state segment (a constant
    ghost) besides the inflow: gradients of the zone values and of the initial state
    against the reference. The fixed state is close to the local one (2 cm deeper, the
    local mean velocity, a small tangential one): a state far from it drives face
    velocities past their cap next to the segment, which is outside the regime."""
    base = case()
    P = Oracle(base).planes()
    h_b = float(P[0][14:18, -1].mean()) + 0.02
    u_b = float((P[3] / P[0])[14:18, -1].mean())
    sc = base.replace(edge_kind=(S.TRANSMISSIVE, S.TRANSMISSIVE, S.WALL, S.WALL),
                      boundaries=base.boundaries + [S.Boundary(S.E, S.FIXED, 14, 18, h_b=h_b,
                                                               u_b=u_b, v_b=0.01)])
    dts = schedule(sc, 25)
    gi = gauges(N)
    href = href_of(sc, dts, gi)
    _, hs_ref, gz_ref, gq_ref, gu_ref = reference(sc, dts, gi, href)
    sim = dg2.DG2(sc, dg2.FP64)
    tape = dg2.Tape(sim, dts, gi)
    hs = tape.forward()
    assert np.abs(hs - hs_ref).max() <= 1e-12 * np.abs(hs_ref).max()
    gm, gq, gu = tape.backward(2.0 * (hs - href), len(sc.boundaries[0].q_knots))
    zi = S.zone_index(N, 4)
    gz = np.array([gm.reshape(-1)[zi.reshape(-1) == z].sum() for z in range(16)])
    ez = np.abs(gz - gz_ref).max() / np.abs(gz_ref).max()
    eq = np.abs(gq - gq_ref).max() / np.abs(gq_ref).max()
    eu = np.abs(gu - gu_ref).max() / np.abs(gu_ref).max()
    print(f"walls + fixed segment: zones {ez:.2e}, knots {eq:.2e}, U0 {eu:.2e}", flush=True)
    assert ez <= 1e-7 and eq <= 1e-7 and eu <= 1e-6


def test_adjoint_on_ragged_tiles(dg2):
    """A 37 x 37 grid: the last tile column (5 of 32 cells) and the last tile row (5 of
    8) are partial, so the faces on the east and north sides of the active cells of
    those tiles come from the threads that take the tile's extra faces, next to the
    domain's edges (transmissive east, wall north) and inside it. (A fixed-state
    segment on this grid's east edge drives face velocities past their cap in the CPU
    reference as well, outside the regime.)"""
    n = 37
    base = S.adjoint_case(n=n, dx=5.0, t_span=4.0, n_knots=8)
    sc = base.replace(edge_kind=(S.TRANSMISSIVE, S.TRANSMISSIVE, S.WALL, S.WALL))
    dts = schedule(sc, 20)
    gi = gauges(n)
    href = href_of(sc, dts, gi)
    _, hs_ref, gz_ref, gq_ref, gu_ref = reference(sc, dts, gi, href)
    sim = dg2.DG2(sc, dg2.FP64)
    tape = dg2.Tape(sim, dts, gi)
    hs = tape.forward()
    assert np.abs(hs - hs_ref).max() <= 1e-12 * np.abs(hs_ref).max()
    gm, gq, gu = tape.backward(2.0 * (hs - href), len(sc.boundaries[0].q_knots))
    zi = S.zone_index(n, 4)
    gz = np.array([gm.reshape(-1)[zi.reshape(-1) == z].sum() for z in range(16)])
    ez = np.abs(gz - gz_ref).max() / np.abs(gz_ref).max()
    eq = np.abs(gq - gq_ref).max() / np.abs(gq_ref).max()
    eu = np.abs(gu - gu_ref).max() / np.abs(gu_ref).max()
    print(f"ragged tiles: zones {ez:.2e}, knots {eq:.2e}, U0 {eu:.2e}", flush=True)
    assert ez <= 1e-7 and eq <= 1e-7 and eu <= 1e-6


def test_autograd_function(dg2):
    sc = case()
    dts = schedule(sc, 20)
    gi = gauges(N)
    href = href_of(sc, dts, gi)
    _, _, gz_ref, gq_ref, _ = reference(sc, dts, gi, href)
    sim = dg2.DG2(sc, dg2.FP64)
    state0 = sim.get_state()
    zi = torch.as_tensor(S.zone_index(N, 4), device="cuda")
    nz0 = np.array([sc.manning.reshape(-1)[S.zone_index(N, 4).reshape(-1) == z][0] for z in range(16)])
    nz = torch.tensor(nz0, device="cuda", requires_grad=True)
    qk = torch.tensor(np.asarray(sc.boundaries[0].q_knots, dtype=np.float64), device="cuda",
                      requires_grad=True)
    f = dg2.gauge_run_function()
    h = f.apply(nz[zi], qk, sim, dts, gi, state0)
    loss = ((h - torch.as_tensor(href, device="cuda")) ** 2).sum()
    loss.backward()
    ez = np.abs(nz.grad.cpu().numpy() - gz_ref).max() / np.abs(gz_ref).max()
    eq = np.abs(qk.grad.cpu().numpy() - gq_ref).max() / np.abs(gq_ref).max()
    print(f"autograd Function vs reference: zones {ez:.2e}, knots {eq:.2e}", flush=True)
    assert ez <= 1e-7 and eq <= 1e-7


def test_regime_and_argument_checks(dg2):
    sc = case()
    data = sc.init_data.copy()
    data[0, 10:13, 10:13] = 0.0    # a dry patch
    dry = sc.replace(init_data=data)
    sim = dg2.DG2(dry, dg2.FP64)
    dts = np.full(5, 0.01)
    tape = dg2.Tape(sim, dts, [0, 1])
    tape.forward()
    with pytest.raises(dg2.DG2Error) as e:
        tape.backward(np.ones((6, 2)), 8)
    assert e.value.code == dg2.E_UNSUPPORTED
    with pytest.raises(dg2.DG2Error) as e:
        dg2.Tape(dg2.DG2(sc, dg2.FP32), dts, [0])
    assert e.value.code == dg2.E_UNSUPPORTED
    with pytest.raises(dg2.DG2Error) as e:
        dg2.Tape(dg2.DG2(sc.replace(limiter=1), dg2.FP64), dts, [0])
    assert e.value.code == dg2.E_UNSUPPORTED
    with pytest.raises(dg2.DG2Error) as e:
        dg2.Tape(dg2.DG2(sc, dg2.FP64), dts, [N * N])
    assert e.value.code == dg2.E_ARG


def test_regime_flag_from_a_partial_tile_edge_face(dg2):
    """On a 37 x 37 grid a fixed-state face on the east edge at row 15 drives the face
    velocity of the last cell of that row past its cap (the CPU reference shows it
    there and nowhere else in the first steps). That face is one of its tile's extra
    faces, taken by a thread whose own cell lies outside the grid (the tile has 5
    active columns); its flag must still reach the regime check."""
    n = 37
    base = S.adjoint_case(n=n, dx=5.0, t_span=4.0, n_knots=8)
    P = Oracle(base).planes()
    h_b = float(P[0][15:16, -1].mean()) + 0.02
    u_b = float((P[3] / P[0])[15:16, -1].mean())
    sc = base.replace(edge_kind=(S.TRANSMISSIVE, S.TRANSMISSIVE, S.WALL, S.WALL),
                      boundaries=base.boundaries + [S.Boundary(S.E, S.FIXED, 15, 16, h_b=h_b,
                                                               u_b=u_b, v_b=0.01)])
    dts = schedule(sc, 4)
    tape = dg2.Tape(dg2.DG2(sc, dg2.FP64), dts, gauges(n))
    hs = tape.forward()
    with pytest.raises(dg2.DG2Error) as e:
        tape.backward(np.ones_like(hs), len(sc.boundaries[0].q_knots))
    assert e.value.code == dg2.E_UNSUPPORTED
    assert "velocity cap" in str(e.value)


def test_two_inflow_segments_give_every_knot_gradient(dg2):
    """A second inflow segment (south edge, 3 knots) besides the west one (8 knots):
    dJ/dq comes back for all 11 knots in segment order, each part against the CPU
    reference."""
    base = case()
    t2 = np.array([0.0, 2.0, 4.0])
    q2 = np.array([5.0, 15.0, 8.0])
    sc = base.replace(boundaries=base.boundaries + [S.Boundary(S.S, S.INFLOW, 14, 20, t2, q2)])
    dts = schedule(sc, 15)
    gi = gauges(N)
    href = href_of(sc, dts, gi)
    ref = WetDG2(sc)
    zi = S.zone_index(N, 4)
    n_cell = torch.as_tensor(sc.manning)
    qa = torch.tensor(np.asarray(sc.boundaries[0].q_knots, dtype=np.float64), requires_grad=True)
    qb = torch.tensor(q2, requires_grad=True)
    U = torch.tensor(Oracle(sc).planes())
    t, J = 0.0, 0.0
    for k, dt in enumerate(dts):
        U = ref.step(U, float(dt), t, n_cell, [qa, qb])
        t += float(dt)
        J = J + ((U[0].reshape(-1)[torch.as_tensor(gi)] - torch.as_tensor(href[k + 1])) ** 2).sum()
    J.backward()
    sim = dg2.DG2(sc, dg2.FP64)
    assert sim.knot_count(0) == 8 and sim.knot_count(1) == 3 and sim.knot_count(-1) == 11
    tape = dg2.Tape(sim, dts, gi)
    hs = tape.forward()
    dj = 2.0 * (hs - href)
    dj[0] = 0.0                       # the reference's misfit starts after step 1
    _, gq, _ = tape.backward(dj)
    assert gq.shape == (11,)
    want = np.concatenate([qa.grad.numpy(), qb.grad.numpy()])
    err = np.abs(gq - want).max() / np.abs(want).max()
    print(f"two inflow segments: knot gradients vs reference {err:.2e}", flush=True)
    assert err <= 1e-7
    assert np.abs(qb.grad.numpy()).max() > 0.0
    del zi


def test_backward_uses_the_parameters_it_was_recorded_with(dg2):
    """Two applies of the autograd Function with different Manning values on the same
    simulation, then the backward of the first only: its gradient is the one at the
    first values (the tape keeps the parameters of its own run)."""
    sc = case()
    dts = schedule(sc, 12)
    gi = gauges(N)
    href = href_of(sc, dts, gi)
    _, _, gz_ref, _, _ = reference(sc, dts, gi, href)
    sim = dg2.DG2(sc, dg2.FP64)
    state0 = sim.get_state()
    zi = torch.as_tensor(S.zone_index(N, 4), device="cuda")
    nz0 = np.array([sc.manning.reshape(-1)[S.zone_index(N, 4).reshape(-1) == z][0] for z in range(16)])
    nz = torch.tensor(nz0, device="cuda", requires_grad=True)
    other = torch.tensor(1.5 * nz0, device="cuda", requires_grad=True)
    qk = torch.tensor(np.asarray(sc.boundaries[0].q_knots, dtype=np.float64), device="cuda")
    f = dg2.gauge_run_function()
    h1 = f.apply(nz[zi], qk, sim, dts, gi, state0)
    h2 = f.apply(other[zi], qk, sim, dts, gi, state0)   # leaves the context at 1.5 n
    assert not torch.equal(h1, h2)
    ((h1 - torch.as_tensor(href, device="cuda")) ** 2).sum().backward()
    ez = np.abs(nz.grad.cpu().numpy() - gz_ref).max() / np.abs(gz_ref).max()
    print(f"backward after a second forward: zones {ez:.2e}", flush=True)
    assert ez <= 1e-7
    assert other.grad is None


@pytest.mark.parametrize("keep", [0, -1])
def test_recorded_gauge_depths_with_shared_cells(dg2, keep):
    """Gauges that share a cell (the stage-2 kernel follows each cell's chain of gauges)
    record the same depth, and every recorded row equals the state of a plain run after
    that many steps; in both recording modes."""
    sc = case()
    dts = schedule(sc, 6)
    c1, c2 = 7 * N + 3, (N // 2) * N + 1
    gi = np.array([c1, c2, c1, c1, c2], dtype=np.int64)
    sim = dg2.DG2(sc, dg2.FP64)
    hs = dg2.Tape(sim, dts, gi, checkpoint_every=keep).forward()
    assert hs.shape == (7, 5)
    assert np.array_equal(hs[:, 0], hs[:, 2]) and np.array_equal(hs[:, 0], hs[:, 3])
    assert np.array_equal(hs[:, 1], hs[:, 4])
    plain = dg2.DG2(sc, dg2.FP64)
    for k in range(7):
        h = plain.read(0).reshape(-1)
        assert hs[k, 0] == h[c1] and hs[k, 1] == h[c2], k
        if k < 6:
            plain.step(float(dts[k]))
