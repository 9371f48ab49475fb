"""Differentiable FP64 CPU reference of the DG2 step in its fully wet, limiter-off
regime (plain PyTorch CPU ops; torch.autograd supplies the reference gradient).

TEST INFRASTRUCTURE ONLY: the reference the GPU library's hand-written adjoint is
checked against. Only the test suite and the benchmark may use it.

It restates the step of arXiv:2107.02750 Sect. 2.1.1 (eq 2-4) with the same readings
as the C oracle, for states where every cell is wet (h0 > h_tol, so no cell is a
wet/dry front or flattened) and the limiter is off, so that the step is a smooth (or
piecewise smooth: min/max and the HLL branches) function of the state, the per-cell
Manning n and the inflow hydrograph knots:
  friction at the centre and the Gauss points (split implicit, one Newton step),
  face limits (eq 2), the temporary revision with the face bed (vertex mean), the
  face-velocity cap, boundary ghosts (transmissive, wall, fixed state, inflow Q(t)),
  HLL fluxes (an inflow face carries the inflow state's own flux), the operator L with 2-point Gauss fluxes and the bed source,
  RK2: U_int = V + dt L(V, t), U_next = (V + U_int + dt L(U_int, t + dt)) / 2.
The time steps are given (a replayed schedule), not differentiated. The regime is
checked on every stage input; a violation raises.
"""
from __future__ import annotations

import numpy as np
import torch

SQ3 = 3.0 ** 0.5
TRANSMISSIVE, WALL, FIXED, INFLOW = 0, 1, 2, 3
W, E, S, N = 0, 1, 2, 3


class RegimeError(RuntimeError):
    pass


def _t(a):
    return torch.as_tensor(np.asarray(a, dtype=np.float64))


class WetDG2:
    """Reference step for one scenario (see the seeded generators): grid, bed, edges
    and boundary segments are taken from it; Manning n (per cell) and the inflow knot
    discharges are arguments of step() so that gradients can flow to them."""

    def __init__(self, sc):
        if sc.limiter != 0:
            raise RegimeError("the reference covers the limiter-off step only")
        self.nx, self.ny, self.dx, self.g, self.ht = sc.nx, sc.ny, sc.dx, sc.g, sc.h_tol
        zv = np.asarray(sc.zv, dtype=np.float64)
        self.zfx = _t(0.5 * (zv[1:, :] + zv[:-1, :]))         # (ny, nx+1) x-face beds
        self.zfy = _t(0.5 * (zv[:, :-1] + zv[:, 1:]))         # (ny+1, nx) y-face beds
        # per boundary face: kind and segment (W/E along j, S/N along i)
        self.kind = {e: np.full(sc.ny if e < 2 else sc.nx, sc.edge_kind[e]) for e in range(4)}
        self.seg = {e: np.full(sc.ny if e < 2 else sc.nx, -1) for e in range(4)}
        self.segs = list(sc.boundaries)
        for s_, b in enumerate(self.segs):
            self.kind[b.edge][b.i0:b.i1] = b.kind
            self.seg[b.edge][b.i0:b.i1] = s_
        self.slack = float(np.sqrt(sc.g * sc.h_tol))

    # -- pieces -------------------------------------------------------------------
    def friction_point(self, h, qx, qy, n, dt):
        g, ht = self.g, self.ht
        act = (n > 0) & (h > ht)
        hs = torch.where(act, h, torch.ones_like(h))
        u, v = qx / hs, qy / hs
        s2 = u * u + v * v
        act = act & (s2 > 0)
        s = torch.sqrt(torch.where(act, s2, torch.ones_like(s2)))
        cf = g * n * n / torch.pow(hs, 1.0 / 3.0)
        dx_ = 1.0 + dt * cf * (2.0 * u * u + v * v) / (hs * s)
        dy_ = 1.0 + dt * cf * (u * u + 2.0 * v * v) / (hs * s)
        qx2 = qx - dt * cf * u * s / dx_
        qy2 = qy - dt * cf * v * s / dy_
        return torch.where(act, qx2, qx), torch.where(act, qy2, qy)

    def friction(self, U, n, dt):
        h0, h1x, h1y, qx0, qx1x, qx1y, qy0, qy1x, qy1y = U
        cx, cy = self.friction_point(h0, qx0, qy0, n, dt)
        out = [h0, h1x, h1y, cx, None, None, cy, None, None]
        for d, (h1, qx1, qy1) in ((1, (h1x, qx1x, qy1x)), (2, (h1y, qx1y, qy1y))):
            px, py = self.friction_point(h0 + h1, qx0 + qx1, qy0 + qy1, n, dt)
            mx, my = self.friction_point(h0 - h1, qx0 - qx1, qy0 - qy1, n, dt)
            out[3 + d] = qx1 + 0.5 * ((px - (qx0 + qx1)) - (mx - (qx0 - qx1)))
            out[6 + d] = qy1 + 0.5 * ((py - (qy0 + qy1)) - (my - (qy0 - qy1)))
        return torch.stack(out)

    def revise(self, h, qn, qt, zf):
        eta = h + zf
        hs = torch.clamp(eta - zf, min=0.0)
        wet = h > self.ht
        hh = torch.where(wet, h, torch.ones_like(h))
        un = torch.where(wet, qn / hh, torch.zeros_like(h))
        ut = torch.where(wet, qt / hh, torch.zeros_like(h))
        zz = torch.minimum(eta, zf)
        return hs, un, ut, zz

    def cap(self, x, a, b):
        m = torch.maximum(a.abs(), b.abs()) + self.slack
        return torch.minimum(torch.maximum(x, -m), m)

    def hll(self, hL, unL, utL, hR, unR, utR):
        g = self.g
        cL, cR = torch.sqrt(g * hL), torch.sqrt(g * hR)
        us = 0.5 * (unL + unR) + cL - cR
        cs = 0.5 * (cL + cR) + 0.25 * (unL - unR)
        sL = torch.minimum(unL - cL, us - cs)
        sR = torch.maximum(unR + cR, us + cs)
        FL = [hL * unL, hL * unL * unL + 0.5 * g * hL * hL, hL * unL * utL]
        FR = [hR * unR, hR * unR * unR + 0.5 * g * hR * hR, hR * unR * utR]
        UL = [hL, hL * unL, hL * utL]
        UR = [hR, hR * unR, hR * utR]
        out = []
        for m in range(3):
            mid = (sR * FL[m] - sL * FR[m] + sL * sR * (UR[m] - UL[m])) / (sR - sL)
            out.append(torch.where(sL >= 0, FL[m], torch.where(sR <= 0, FR[m], mid)))
        return out

    def qin(self, seg, t, qk):
        tk = np.asarray(seg.t_knots, dtype=np.float64)
        if t <= tk[0]:
            return qk[0]
        if t >= tk[-1]:
            return qk[-1]
        k = int(np.searchsorted(tk, t, side="right") - 1)
        a = (t - tk[k]) / (tk[k + 1] - tk[k])
        return qk[k] + a * (qk[k + 1] - qk[k])

    def ghost(self, edge, t, inward, h, un, ut, qknots):
        """Ghost states beyond every face of one edge, from the interior sides (h, un,
        ut) in the face's normal frame (1-D tensors along the edge)."""
        kind = torch.as_tensor(self.kind[edge])
        gh = torch.where(kind == WALL, h, h)
        gn = torch.where(kind == WALL, -un, un)
        gt = ut
        nx_ = edge < 2
        for s_, seg in enumerate(self.segs):
            if seg.edge != edge:
                continue
            m = torch.zeros(len(self.kind[edge]), dtype=torch.bool)
            m[seg.i0:seg.i1] = True
            if seg.kind == FIXED:
                hb = torch.full_like(h, seg.h_b)
                nb = torch.full_like(h, seg.u_b if nx_ else seg.v_b)
                tb = torch.full_like(h, seg.v_b if nx_ else seg.u_b)
                gh, gn, gt = torch.where(m, hb, gh), torch.where(m, nb, gn), torch.where(m, tb, gt)
            elif seg.kind == INFLOW:
                qn = self.qin(seg, t, qknots[s_]) / ((seg.i1 - seg.i0) * self.dx)
                hc = torch.pow(qn * qn / self.g, 1.0 / 3.0)
                hg = torch.maximum(h, hc * torch.ones_like(h))
                gh = torch.where(m, hg, gh)
                gn = torch.where(m, inward * (qn / hg), gn)
                gt = torch.where(m, torch.zeros_like(h), gt)
        return gh, gn, gt

    def check(self, V):
        h0 = V[0]
        if not bool((h0 > self.ht).all()):
            raise RegimeError("a cell is at or below the dry tolerance")
        if not bool(((h0 - SQ3 * V[1].abs()) >= 0).all() and ((h0 - SQ3 * V[2].abs()) >= 0).all()):
            raise RegimeError("a depth plane is negative at a face centre")

    def faces(self, h, qn, qt, h1, qn1, qt1, un_m, ut_m, zf, axis, t, qknots, edges):
        """Fluxes through every face along one axis (axis 1: x faces, normal frame
        (h, u, v); axis 0: y faces, (h, v, u)) and the cells' own revised sides at
        their high and low faces. Arrays are (ny, nx) cell planes; zf the face beds."""
        cat = lambda a, b: torch.cat([a, b], axis)
        first = (slice(None), slice(0, 1)) if axis == 1 else (slice(0, 1), slice(None))
        last = (slice(None), slice(-1, None)) if axis == 1 else (slice(-1, None), slice(None))
        hi_ = (slice(None), slice(1, None)) if axis == 1 else (slice(1, None), slice(None))
        lo_ = (slice(None), slice(None, -1)) if axis == 1 else (slice(None, -1), slice(None))
        # limits: high side of each cell (face i+1), low side (face i)
        pH = self.revise(h + SQ3 * h1, qn + SQ3 * qn1, qt + SQ3 * qt1, zf[hi_])
        pL = self.revise(h - SQ3 * h1, qn - SQ3 * qn1, qt - SQ3 * qt1, zf[lo_])
        # mean velocities on the two sides of each face (a boundary side copies the cell)
        una, unb = cat(un_m[first], un_m), cat(un_m, un_m[last])
        uta, utb = cat(ut_m[first], ut_m), cat(ut_m, ut_m[last])
        capH = lambda x, a, b: self.cap(x, a[hi_], b[hi_])
        capL = lambda x, a, b: self.cap(x, a[lo_], b[lo_])
        Hh, Hn, Ht, Hz = pH[0], capH(pH[1], una, unb), capH(pH[2], uta, utb), pH[3]
        Lh, Ln, Lt, Lz = pL[0], capL(pL[1], una, unb), capL(pL[2], uta, utb), pL[3]
        sq = lambda x: x.squeeze(axis)
        g0 = self.ghost(edges[0], t, 1.0, sq(Lh[first]), sq(Ln[first]), sq(Lt[first]), qknots)
        g1 = self.ghost(edges[1], t, -1.0, sq(Hh[last]), sq(Hn[last]), sq(Ht[last]), qknots)
        us = lambda x: x.unsqueeze(axis)
        # face arrays: left state = high side of the cell before, right = low side after
        fl = [cat(us(g0[k]), X) for k, X in enumerate((Hh, Hn, Ht))]
        fr = [cat(X, us(g1[k])) for k, X in enumerate((Lh, Ln, Lt))]
        F = self.hll(fl[0], fl[1], fl[2], fr[0], fr[1], fr[2])
        # an inflow face carries the inflow (ghost) state's own physical flux
        for e, gs, sl_ in ((edges[0], g0, first), (edges[1], g1, last)):
            m = torch.as_tensor(self.kind[e] == INFLOW)
            if not bool(m.any()):
                continue
            P = self.phys(*gs)
            F = [self._put(F[k], sl_, torch.where(us(m), us(P[k]), F[k][sl_]))
                 for k in range(3)]
        return F, (Hh, Hn, Ht, Hz), (Lh, Ln, Lt, Lz)

    @staticmethod
    def _put(a, sl_, v):
        b = a.clone()
        b[sl_] = v
        return b

    def phys(self, h, un, ut):
        return [h * un, h * un * un + 0.5 * self.g * h * h, h * un * ut]

    def operator(self, V, t, qknots):
        """L(V) for a stage input V (9, ny, nx) at stage time t."""
        self.check(V)
        dx, g, ht = self.dx, self.g, self.ht
        h0, h1x, h1y, qx0, qx1x, qx1y, qy0, qy1x, qy1y = V
        hm = torch.where(h0 > ht, h0, torch.ones_like(h0))
        um = torch.where(h0 > ht, qx0 / hm, torch.zeros_like(h0))
        vm = torch.where(h0 > ht, qy0 / hm, torch.zeros_like(h0))
        L = [None] * 9
        # x: normal frame (h, u, v); F = [mass, x-mom, y-mom]
        F, (hE, uE, vE, zE), (hW, uW, vW, zW) = self.faces(
            h0, qx0, qy0, h1x, qx1x, qy1x, um, vm, self.zfx, 1, t, qknots, (W, E))
        fe = [F[m][:, 1:] for m in range(3)]
        fw = [F[m][:, :-1] for m in range(3)]
        hb0, hb1 = 0.5 * (hE + hW), (hE - hW) / (2.0 * SQ3)
        qxE, qxW, qyE, qyW = hE * uE, hW * uW, hE * vE, hW * vW
        qb0, qb1 = 0.5 * (qxE + qxW), (qxE - qxW) / (2.0 * SQ3)
        rb0, rb1 = 0.5 * (qyE + qyW), (qyE - qyW) / (2.0 * SQ3)
        zb1 = (zE - zW) / (2.0 * SQ3)
        Fp = self.flux_n(hb0 + hb1, qb0 + qb1, rb0 + rb1)
        Fm = self.flux_n(hb0 - hb1, qb0 - qb1, rb0 - rb1)
        L[0] = -(fe[0] - fw[0]) / dx
        L[3] = -(fe[1] - fw[1]) / dx - 2.0 * SQ3 * g * hb0 * zb1 / dx
        L[6] = -(fe[2] - fw[2]) / dx
        L[1] = -(SQ3 / dx) * (fe[0] + fw[0] - Fp[0] - Fm[0])
        L[4] = -(SQ3 / dx) * (fe[1] + fw[1] - Fp[1] - Fm[1]) - 2.0 * SQ3 * g * hb1 * zb1 / dx
        L[7] = -(SQ3 / dx) * (fe[2] + fw[2] - Fp[2] - Fm[2])
        # y: normal frame (h, v, u); HLL gives [mass, y-mom, x-mom]
        G, (hN, vN, uN, zN), (hS, vS, uS, zS) = self.faces(
            h0, qy0, qx0, h1y, qy1y, qx1y, vm, um, self.zfy, 0, t, qknots, (S, N))
        fn = [G[m][1:, :] for m in (0, 2, 1)]
        fs = [G[m][:-1, :] for m in (0, 2, 1)]
        hb0, hb1 = 0.5 * (hN + hS), (hN - hS) / (2.0 * SQ3)
        qxN, qxS, qyN, qyS = hN * uN, hS * uS, hN * vN, hS * vS
        qb0, qb1 = 0.5 * (qxN + qxS), (qxN - qxS) / (2.0 * SQ3)
        rb0, rb1 = 0.5 * (qyN + qyS), (qyN - qyS) / (2.0 * SQ3)
        zb1 = (zN - zS) / (2.0 * SQ3)
        Gp = self.flux_n(hb0 + hb1, rb0 + rb1, qb0 + qb1)
        Gm = self.flux_n(hb0 - hb1, rb0 - rb1, qb0 - qb1)
        L[0] = L[0] - (fn[0] - fs[0]) / dx
        L[3] = L[3] - (fn[1] - fs[1]) / dx
        L[6] = L[6] - (fn[2] - fs[2]) / dx - 2.0 * SQ3 * g * hb0 * zb1 / dx
        L[2] = -(SQ3 / dx) * (fn[0] + fs[0] - Gp[0] - Gm[0])
        L[5] = -(SQ3 / dx) * (fn[1] + fs[1] - Gp[2] - Gm[2])
        L[8] = -(SQ3 / dx) * (fn[2] + fs[2] - Gp[1] - Gm[1]) - 2.0 * SQ3 * g * hb1 * zb1 / dx
        return torch.stack(L)

    def flux_n(self, h, qn, qt):
        wet = h > self.ht
        hh = torch.where(wet, h, torch.ones_like(h))
        un = torch.where(wet, qn / hh, torch.zeros_like(h))
        ut = torch.where(wet, qt / hh, torch.zeros_like(h))
        return [h * un, h * un * un + 0.5 * self.g * h * h, h * un * ut]

    def step(self, U, dt, t, n_cell, qknots):
        """One RK2 step of a (9, ny, nx) state with time step dt from time t."""
        V = self.friction(U, n_cell, dt)
        Ui = V + dt * self.operator(V, t, qknots)
        if not bool((Ui[0] > self.ht).all()):
            raise RegimeError("a depth fell to the dry tolerance in stage 1")
        Un = 0.5 * (V + Ui + dt * self.operator(Ui, t + dt, qknots))
        if not bool((Un[0] > self.ht).all()):
            raise RegimeError("a depth fell to the dry tolerance in stage 2")
        return Un
