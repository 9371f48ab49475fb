// dg2_adjoint.hpp -- gfx950 kernels of the discrete adjoint of the DG2 step (FP64),
// for flows that stay fully wet with the limiter off. Included by dg2.hip only.
//
// The forward step (Sect. 2.1.1) is F = friction(U^n); U^int = F + dt L(F, t);
// U^{n+1} = (F + U^int + dt L(U^int, t + dt)) / 2 with a prescribed dt. Its adjoint,
// for a cotangent lambda of U^{n+1}:
//   lam_int = lambda / 2 + (dL/dV)(U^int)^T (dt lambda / 2)
//   lam_F   = lambda / 2 + lam_int + (dL/dV)(F)^T (dt lam_int)
//   lam_U   = (dfriction/dU)^T lam_F
// plus the parameter terms: Manning n through friction, the inflow discharge Q(t)
// through the inflow ghost states of both stages.
//
// (dL/dV)^T mu: L of a cell depends on its own coefficients through its four face
// sides (Gauss fluxes, bed source, and the four face fluxes) and on a neighbour's only
// through the shared face flux. Each face therefore takes the cotangent of its flux
// (from mu of the two cells that share it) back through the same flux, ghost and
// revision formulas as the forward kernels (reverse mode written out per formula,
// recomputing the forward values) to the face limits of both cells; each cell adds
// the cotangents of its four face limits, its own Gauss and source terms and the
// friction, and maps them to its nine coefficients.
//
// The regime is checked while the adjoint runs: a cell at or below h_tol, a face
// depth not above zero, or an active face-velocity cap set a flag (the derivative
// would then need terms this adjoint leaves out).
#pragma once

namespace dg2k {

// ---------------------------------------------------------------------------------
// reverse-mode pieces: each takes the inputs of a forward formula and the cotangents
// of its outputs, recomputes what it needs, and returns the cotangents of the inputs
// ---------------------------------------------------------------------------------

// a face side in the normal frame: depth, normal and tangential velocity
struct NSide {
  double h, un, ut;
};

// HLL (the forward kernel's hll, same branches): cotangents fb of [mass, normal
// momentum, tangential momentum] -> cotangents of the two sides
__device__ __forceinline__ void hll_rev(double g, NSide L, NSide R, const double fb[3], NSide& Lb,
                                        NSide& Rb) {
  Lb = NSide{0.0, 0.0, 0.0};
  Rb = NSide{0.0, 0.0, 0.0};
  const bool wL = L.h > 0.0, wR = R.h > 0.0;
  if (!wL && !wR) return;  // both dry: zero flux
  const double cL = fsqrt(g * L.h), cR = fsqrt(g * R.h);
  const double us = 0.5 * (L.un + R.un) + cL - cR;
  const double cs = 0.5 * (cL + cR) + 0.25 * (L.un - R.un);
  const double a1 = L.un - cL, a2 = us - cs, b1 = R.un + cR, b2 = us + cs;
  const double sL = wL ? (wR ? (a1 <= a2 ? a1 : a2) : L.un - cL) : R.un - 2.0 * cR;
  const double sR = wL ? (wR ? (b1 >= b2 ? b1 : b2) : L.un + 2.0 * cL) : R.un + cR;
  const double qL = L.h * L.un, qR = R.h * R.un;
  const double FL[3] = {qL, qL * L.un + 0.5 * g * L.h * L.h, qL * L.ut};
  const double FR[3] = {qR, qR * R.un + 0.5 * g * R.h * R.h, qR * R.ut};
  const double UL[3] = {L.h, qL, L.h * L.ut};
  const double UR[3] = {R.h, qR, R.h * R.ut};
  double FLb[3] = {0.0, 0.0, 0.0}, FRb[3] = {0.0, 0.0, 0.0}, ULb[3] = {0.0, 0.0, 0.0},
         URb[3] = {0.0, 0.0, 0.0};
  double sLb = 0.0, sRb = 0.0;
  if (sL >= 0.0) {
#pragma unroll
    for (int m = 0; m < 3; ++m) FLb[m] = fb[m];
  } else if (sR <= 0.0) {
#pragma unroll
    for (int m = 0; m < 3; ++m) FRb[m] = fb[m];
  } else {
    // mid = (sR FL - sL FR + sL sR (UR - UL)) / (sR - sL)
    const double inv = frcp(sR - sL), ss = sL * sR;
    double invb = 0.0, ssb = 0.0;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      const double tm = sR * FL[m] - sL * FR[m] + ss * (UR[m] - UL[m]);
      invb += fb[m] * tm;
      const double tb = fb[m] * inv;
      sRb += tb * FL[m];
      FLb[m] = tb * sR;
      sLb -= tb * FR[m];
      FRb[m] = -tb * sL;
      ssb += tb * (UR[m] - UL[m]);
      URb[m] = tb * ss;
      ULb[m] = -tb * ss;
    }
    sLb += ssb * sR + invb * inv * inv;
    sRb += ssb * sL - invb * inv * inv;
  }
  // wave speeds
  double cLb = 0.0, cRb = 0.0, usb = 0.0, csb = 0.0;
  if (wL && wR) {
    if (a1 <= a2) { Lb.un += sLb; cLb -= sLb; } else { usb += sLb; csb -= sLb; }
    if (b1 >= b2) { Rb.un += sRb; cRb += sRb; } else { usb += sRb; csb += sRb; }
  } else if (wL) {
    Lb.un += sLb + sRb;
    cLb += 2.0 * sRb - sLb;
  } else {
    Rb.un += sLb + sRb;
    cRb += sRb - 2.0 * sLb;
  }
  Lb.un += 0.5 * usb + 0.25 * csb;
  Rb.un += 0.5 * usb - 0.25 * csb;
  cLb += usb + 0.5 * csb;
  cRb += 0.5 * csb - usb;
  // fluxes and states of each side: F = [q, q un + g h^2 / 2, q ut], U = [h, q, h ut]
  {
    const double qb = FLb[0] + FLb[1] * L.un + FLb[2] * L.ut + ULb[1];
    Lb.un += FLb[1] * qL + qb * L.h;
    Lb.ut += FLb[2] * qL + ULb[2] * L.h;
    Lb.h += FLb[1] * g * L.h + ULb[0] + ULb[2] * L.ut + qb * L.un;
    if (cL > 0.0) Lb.h += cLb * 0.5 * g * frcp(cL);
  }
  {
    const double qb = FRb[0] + FRb[1] * R.un + FRb[2] * R.ut + URb[1];
    Rb.un += FRb[1] * qR + qb * R.h;
    Rb.ut += FRb[2] * qR + URb[2] * R.h;
    Rb.h += FRb[1] * g * R.h + URb[0] + URb[2] * R.ut + qb * R.un;
    if (cR > 0.0) Rb.h += cRb * 0.5 * g * frcp(cR);
  }
}

// physical flux at a Gauss point (gauss_flux): cotangents fb -> (h, qn, qt)
__device__ __forceinline__ void gauss_rev(double g, double ht, double h, double qn, double qt, const double fb[3],
                                          double& hb, double& qnb, double& qtb) {
  const bool wet = h > ht;
  const double r = frcp(fmaxr(h, Tiny<double>::v));
  const double un = wet ? qn * r : 0.0, ut = wet ? qt * r : 0.0;
  const double q = h * un;
  // f0 = q, f1 = q un + g h^2 / 2, f2 = q ut
  const double qb = fb[0] + fb[1] * un + fb[2] * ut;
  const double unb = fb[1] * q + qb * h, utb = fb[2] * q;
  hb = fb[1] * g * h + qb * un;
  qnb = wet ? unb * r : 0.0;
  qtb = wet ? utb * r : 0.0;
  hb -= wet ? (unb * un + utb * ut) * r : 0.0;  // d(q/h)/dh = -(q/h)/h
}

// the split-implicit friction increment at one point (friction_inc): cotangents
// (cx, cy) of (dqx, dqy) -> (h, qx, qy) and gn2dt
__device__ __forceinline__ void friction_rev(double gn2dt, double ht, double h, double qx, double qy, double cx,
                                             double cy, double& hb, double& qxb, double& qyb, double& gb) {
  hb = qxb = qyb = gb = 0.0;
  if (!(h > ht)) return;
  const double y = finvcbrt(h);  // h^(-1/3)
  const double y3 = y * y * y;   // 1/h
  const double u = qx * y3, v = qy * y3;
  const double s2 = u * u + v * v;
  if (!(s2 > 0.0)) return;
  const double rs = frsq(s2);    // 1/|u|
  const double y4 = y3 * y;
  const double w = gn2dt * y4;
  const double a = w * u * u * rs, b = w * v * v * rs;
  const double ab = a + b;
  const double d1 = 1.0 + 2.0 * a + b, d2 = 1.0 + a + 2.0 * b;
  const double inv = frcp(d1 * d2);
  const double P = ab * inv;
  // dqx = -qx d2 P, dqy = -qy d1 P
  qxb = -cx * d2 * P;
  qyb = -cy * d1 * P;
  double d2b = -cx * qx * P, d1b = -cy * qy * P;
  const double Pb = -cx * qx * d2 - cy * qy * d1;
  const double abb = Pb * inv, invb = Pb * ab;
  const double Db = -invb * inv * inv;  // inv = 1 / (d1 d2)
  d1b += Db * d2;
  d2b += Db * d1;
  const double ab_ = abb + 2.0 * d1b + d2b, bb_ = abb + d1b + 2.0 * d2b;  // of a, b
  const double wb = (ab_ * u * u + bb_ * v * v) * rs;
  double ub = 2.0 * ab_ * w * u * rs, vb = 2.0 * bb_ * w * v * rs;
  const double rsb = ab_ * w * u * u + bb_ * w * v * v;
  const double s2b = -0.5 * rsb * rs * rs * rs;  // rs = s2^(-1/2)
  ub += 2.0 * u * s2b;
  vb += 2.0 * v * s2b;
  gb = wb * y4;
  qxb += ub * y3;
  qyb += vb * y3;
  const double y3b = ub * qx + vb * qy;
  const double yb = wb * gn2dt * 4.0 * y3 + y3b * 3.0 * y * y;  // w = gn2dt y^4, y3 = y^3
  hb = -0.33333333333333333333 * yb * y4;                         // dy/dh = -y^4 / 3
}

// ---------------------------------------------------------------------------------
// adjoint of the friction step at one cell: lam (the cotangent of F) becomes the
// cotangent of U, lam_U = (dF/dU)^T lam_F; returns dJ/dn of the cell
// ---------------------------------------------------------------------------------
__device__ __forceinline__ double adj_friction_cell(const Params<double>& p, const double u[9], double nm,
                                                    double dt, double lam[9]) {
  if (!(nm > 0.0)) return 0.0;
  double lf[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) lf[q] = lam[q];
  const double ht = p.h_tol;
  const double gdt = p.g * dt, gn2dt = gdt * (nm * nm);
  double gsum = 0.0;
  // points: 0 centre; 1, 2: x +/-; 3, 4: y +/-
#pragma unroll
  for (int pt = 0; pt < 5; ++pt) {
    const int d = pt == 0 ? 0 : (pt <= 2 ? 1 : 2);
    const double sg = pt == 0 ? 0.0 : ((pt == 1 || pt == 3) ? 1.0 : -1.0);
    const bool xd = d == 1, yd = d == 2;
    const double h1 = xd ? u[1] : (yd ? u[2] : 0.0);
    const double qx1 = xd ? u[4] : (yd ? u[5] : 0.0);
    const double qy1 = xd ? u[7] : (yd ? u[8] : 0.0);
    // cotangents of the increments: the centre feeds the means, a Gauss pair feeds
    // half the difference into the slopes of its direction
    const double cx = pt == 0 ? lf[3] : 0.5 * sg * (xd ? lf[4] : lf[5]);
    const double cy = pt == 0 ? lf[6] : 0.5 * sg * (xd ? lf[7] : lf[8]);
    double hb, qxb, qyb, gb;
    friction_rev(gn2dt, ht, u[0] + sg * h1, u[3] + sg * qx1, u[6] + sg * qy1, cx, cy, hb, qxb, qyb, gb);
    // the point's inputs are U0 + sg U1d
    lam[0] += hb;
    lam[3] += qxb;
    lam[6] += qyb;
    lam[1] += xd ? sg * hb : 0.0;
    lam[4] += xd ? sg * qxb : 0.0;
    lam[7] += xd ? sg * qyb : 0.0;
    lam[2] += yd ? sg * hb : 0.0;
    lam[5] += yd ? sg * qxb : 0.0;
    lam[8] += yd ? sg * qyb : 0.0;
    gsum += gb;
  }
  return gsum * 2.0 * gdt * nm;  // gn2dt = g dt n^2
}

// ---------------------------------------------------------------------------------
// adjoint of one stage: out = cl lam_c + (dL/dV)(V)^T (alpha lam) + extra, and dJ/dQ of
// each inflow boundary face; with U_fr the friction adjoint then maps out to the
// cotangent of U (and adds dJ/dn to gman)
// ---------------------------------------------------------------------------------
struct AdjArgs {
  const double* V;      // stage input, 9 planes
  const double* lam;    // cotangent of the stage output; mu = alpha * lam
  double alpha;
  double t;             // stage time (inflow discharge)
  const double* lam_c;  // combined into the output: cl * lam_c (own cell)
  double cl;
  const double* extra;  // added to the output (own cell), or nullptr
  const double* U_fr;   // friction adjoint of the step from state U_fr, or nullptr
  double dt_fr;
  double* gman;         // dJ/dn per cell (accumulated) with U_fr
  const int* gmap;      // with gmap: each cell's gauges (first gauge, then gnext per
  const int* gnext;     // gauge; -1 ends) add their seed[g] to the output's mean depth
  const double* seed;
  double* out;          // 9 planes; may be lam_c itself (each cell reads its own first)
  double* gqf;          // out: dJ/dQ of each inflow boundary face (slots as the face
                        // codes: W[ny], E[ny], S[nx], N[nx]), summed per segment later
  int* regime;          // out: |= violation bits
};

// the adjoint works on 32 x 8 tiles: the stage input and mu of the tile and a one-cell
// halo are staged in LDS, so the neighbour reads of the face terms are LDS reads; once
// every face is done, the same LDS holds each face's cotangents of its two face limits
constexpr int ADJ_TX = 32, ADJ_TY = 8, ADJ_RX = ADJ_TX + 2, ADJ_RB = ADJ_RX * (ADJ_TY + 2);
constexpr int ADJ_NFX = (ADJ_TX + 1) * ADJ_TY, ADJ_NFY = ADJ_TX * (ADJ_TY + 1);
union AdjSmem {
  struct {
    double v[9][ADJ_RB];  // stage input V
    double m[9][ADJ_RB];  // mu = alpha lam
  };
  struct {                // per face: (h, qx, qy) cotangents of the low cell's limit (0..2)
    double fx[6][ADJ_NFX];  // and of the high cell's (3..5); x face f of tile row b at
    double fy[6][ADJ_NFY];  // b * (TX + 1) + f, y face f of tile column a at f * TX + a
  };
};

// One face of the adjoint: the cotangent of the face's stored flux (from mu of the cells
// on both sides) goes back through the HLL flux (at an inflow face: the inflow state's
// own flux), the ghost state (boundary faces) and the revision to the face limits
// (h, qx, qy) of the cells on both sides: lo for the low cell (its high limit), hi for
// the high cell (its low limit). A boundary face has one cell; the ghost's cotangent is
// folded into it.
struct AdjFace {
  bool xdir;
  int posL, posR;     // box positions of the low and high cells
  bool realL, realR;  // in the domain (at most one is not: a boundary face)
  double zf;          // face bed: the mean of its two vertices
  int line;           // row (x face) or column (y face) of the face
};

__device__ __forceinline__ void adj_face(const Params<double>& p, const AdjArgs& a, const AdjSmem& sm,
                                         const AdjFace& F, double lo[3], double hi[3], int& bad) {
  const int nx = p.nx, ny = p.ny;
  const double g = p.g, ht = p.h_tol, s3 = K<double>::s3;
  const double idx = p.idx, cc = -s3 * idx;
  const double slack = dsqrt(p.gd * p.htd);
  const bool xdir = F.xdir;
  auto V = [&](int pos, int q) { return sm.v[q][pos]; };
  auto mu = [&](int pos, int q) { return sm.m[q][pos]; };
  auto umean = [&](int pos, bool xv) {
    const double h0 = V(pos, 0);
    return h0 > ht ? V(pos, xv ? 3 : 6) * frcp(h0) : 0.0;
  };
  const double zf = F.zf;
  // velocity caps: the larger mean-velocity magnitude of the face's cells plus the slack
  const int pL = F.realL ? F.posL : F.posR, pR = F.realR ? F.posR : F.posL;
  const double ucap = fmax(fabs(umean(pL, true)), fabs(umean(pR, true))) + slack;
  const double vcap_ = fmax(fabs(umean(pL, false)), fabs(umean(pR, false))) + slack;
  // a cell's face limit (sgn +1: its high side, -1: its low side) after the revision
  // (both sides share the face bed in this regime)
  double uL = 0.0, vL = 0.0, rL = 0.0, uR = 0.0, vR = 0.0, rR = 0.0;
  NSide sL{}, sR{};
  auto side = [&](int pos, double sgn, double& u, double& v, double& r) {
    const double c1 = xdir ? V(pos, 1) : V(pos, 2), c4 = xdir ? V(pos, 4) : V(pos, 5);
    const double c7 = xdir ? V(pos, 7) : V(pos, 8);
    const double h = V(pos, 0) + sgn * s3 * c1, qx = V(pos, 3) + sgn * s3 * c4, qy = V(pos, 6) + sgn * s3 * c7;
    r = frcp(h);
    const double hs = fmax0((h + zf) - zf);
    u = qx * r;
    v = qy * r;
    if (!(h > ht) || !(hs > 0.0)) bad |= 1;
    if (fabs(u) > ucap || fabs(v) > vcap_) bad |= 2;
    return NSide{hs, xdir ? u : v, xdir ? v : u};
  };
  if (F.realL) sL = side(F.posL, 1.0, uL, vL, rL);
  if (F.realR) sR = side(F.posR, -1.0, uR, vR, rR);
  // the ghost beyond a boundary face, from the cell's side in the normal frame
  int kind = -1, qslot = -1;
  double qn = 0.0, hc = 0.0, inward = 0.0, width = 1.0;
  if (!F.realL || !F.realR) {
    const bool high = !F.realR;  // the cell is the low one: an east or north boundary
    const NSide own = high ? sL : sR;
    const int code = xdir ? p.bface[(high ? ny : 0) + F.line] : p.bface[2 * ny + (high ? nx : 0) + F.line];
    kind = code & 255;
    inward = high ? -1.0 : 1.0;
    NSide nb = own;
    if (kind == 1) {
      nb.un = -own.un;
    } else if (kind == 2) {
      const Seg& sg = p.segs[(code >> 8) - 1];
      nb = NSide{sg.h_b, xdir ? sg.u_b : sg.v_b, xdir ? sg.v_b : sg.u_b};
    } else if (kind == 3) {
      const Seg& sg = p.segs[(code >> 8) - 1];
      qslot = xdir ? (high ? ny : 0) + F.line : 2 * ny + (high ? nx : 0) + F.line;
      width = sg.width;
      qn = hydrograph(sg, p.knots, p.knots + p.max_knots, a.t) / width;
      hc = dcbrt(qn * qn / g);
      const double hg = own.h > hc ? own.h : hc;
      nb = NSide{hg, hg > 0.0 ? inward * (qn / hg) : 0.0, 0.0};
    }
    if (high) sR = nb;
    else sL = nb;
  }
  // cotangent of each stored flux component [mass, x-mom, y-mom]: L0 of the low cell
  // gets -F/dx and of the high cell +F/dx, L1 (this direction) of both cc F
  double mt[3];
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    const double tL = F.realL ? -idx * mu(F.posL, 3 * m) + cc * (xdir ? mu(F.posL, 3 * m + 1) : mu(F.posL, 3 * m + 2)) : 0.0;
    const double tR = F.realR ? idx * mu(F.posR, 3 * m) + cc * (xdir ? mu(F.posR, 3 * m + 1) : mu(F.posR, 3 * m + 2)) : 0.0;
    mt[m] = tL + tR;
  }
  // in the normal frame: [mass, normal momentum, tangential momentum]
  const double fb[3] = {mt[0], xdir ? mt[1] : mt[2], xdir ? mt[2] : mt[1]};
  NSide Lb, Rb;
  if (kind == 3) {  // an inflow face carries the inflow state's own physical flux
    const bool high = !F.realR;
    const NSide gs = high ? sR : sL;
    const NSide gb{fb[0] * gs.un + fb[1] * (gs.un * gs.un + g * gs.h) + fb[2] * gs.un * gs.ut,
                   (fb[0] + 2.0 * fb[1] * gs.un + fb[2] * gs.ut) * gs.h, fb[2] * gs.h * gs.un};
    Lb = high ? NSide{0.0, 0.0, 0.0} : gb;
    Rb = high ? gb : NSide{0.0, 0.0, 0.0};
  } else {
    hll_rev(g, sL, sR, fb, Lb, Rb);
  }
  if (kind >= 0) {
    const bool high = !F.realR;
    NSide& ob = high ? Lb : Rb;        // the cell's cotangent
    const NSide gb = high ? Rb : Lb;   // the ghost's (it depends on the cell's side)
    if (kind == 0) {                   // transmissive: a copy
      ob.h += gb.h; ob.un += gb.un; ob.ut += gb.ut;
    } else if (kind == 1) {            // wall: the normal velocity reversed
      ob.h += gb.h; ob.un -= gb.un; ob.ut += gb.ut;
    } else if (kind == 3) {            // critical-depth inflow: depends on h and Q
      const NSide own = high ? sL : sR;
      const double hg = own.h > hc ? own.h : hc;
      double hgb = gb.h, qnb = 0.0;
      if (hg > 0.0) {
        const double r = frcp(hg);
        qnb += gb.un * inward * r;
        hgb -= gb.un * inward * qn * r * r;
      }
      if (own.h > hc) ob.h += hgb;
      else if (hc > 0.0 && qn != 0.0) qnb += hgb * 2.0 * hc / (3.0 * qn);  // hc = (qn^2 / g)^(1/3)
      a.gqf[qslot] = qnb / width;
    }
  }
  // back through the revision of each cell's side: u = qx / h, v = qy / h, h* = h
  auto back = [&](const NSide& ob, double u, double v, double r, double o[3]) {
    const double ub = xdir ? ob.un : ob.ut, vbk = xdir ? ob.ut : ob.un;
    o[0] = ob.h - (ub * u + vbk * v) * r;
    o[1] = ub * r;
    o[2] = vbk * r;
  };
  lo[0] = lo[1] = lo[2] = hi[0] = hi[1] = hi[2] = 0.0;
  if (F.realL) back(Lb, uL, vL, rL, lo);
  if (F.realR) back(Rb, uR, vR, rR, hi);
}

__global__ __launch_bounds__(ADJ_TX * ADJ_TY, 3) void adj_stage_kernel(Params<double> p, AdjArgs a) {
  __shared__ AdjSmem sm;
  const long long n = p.n;
  const int nx = p.nx, ny = p.ny;
  const int tiles_x = (nx + ADJ_TX - 1) / ADJ_TX;
  const int i0 = (int(blockIdx.x) % tiles_x) * ADJ_TX, j0 = (int(blockIdx.x) / tiles_x) * ADJ_TY;
  const int tid = threadIdx.x;
  const int ta = tid % ADJ_TX, tb = tid / ADJ_TX;
  const int i = i0 + ta, j = j0 + tb;
  const bool active = i < nx && j < ny;
  // box cells (clamped to the domain), two per thread at most, and the cell's four bed
  // vertices: all loads issued before any is waited on
  constexpr int NT = ADJ_TX * ADJ_TY, BIT = (ADJ_RB + NT - 1) / NT;
  static_assert(BIT == 2, "two box cells per thread");
  double bv[BIT][9], bm[BIT][9];
#pragma unroll
  for (int it = 0; it < BIT; ++it) {
    const int r = tid + it * NT;
    if (r < ADJ_RB) {
      int bi = i0 - 1 + r % ADJ_RX, bj = j0 - 1 + r / ADJ_RX;
      bi = bi < 0 ? 0 : (bi >= nx ? nx - 1 : bi);
      bj = bj < 0 ? 0 : (bj >= ny ? ny - 1 : bj);
      const long long k = (long long)bj * nx + bi;
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        bv[it][q] = a.V[q * n + k];
        bm[it][q] = a.lam[q * n + k];
      }
    }
  }
  double zsw = 0.0, zse = 0.0, znw = 0.0, zne = 0.0;  // the cell's vertices
  if (active) {
    const long long v0 = (long long)j * (nx + 1) + i;
    zsw = p.zv[v0];
    zse = p.zv[v0 + 1];
    znw = p.zv[v0 + nx + 1];
    zne = p.zv[v0 + nx + 2];
  }
  // the extra face of threads 0..TY+TX-1 (below): its two vertices
  const int iend = nx < i0 + ADJ_TX ? nx : i0 + ADJ_TX, jend = ny < j0 + ADJ_TY ? ny : j0 + ADJ_TY;
  const int ejr = j0 + tid, eic = i0 + tid - ADJ_TY;
  const bool ex = tid < ADJ_TY && ejr < ny, ey = tid >= ADJ_TY && tid < ADJ_TY + ADJ_TX && eic < nx;
  double ez0 = 0.0, ez1 = 0.0;
  if (ex) {
    const long long v0 = (long long)ejr * (nx + 1) + iend;
    ez0 = p.zv[v0];
    ez1 = p.zv[v0 + nx + 1];
  } else if (ey) {
    const long long v0 = (long long)jend * (nx + 1) + eic;
    ez0 = p.zv[v0];
    ez1 = p.zv[v0 + 1];
  }
#pragma unroll
  for (int it = 0; it < BIT; ++it) {
    const int r = tid + it * NT;
    if (r < ADJ_RB) {
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        sm.v[q][r] = bv[it][q];
        sm.m[q][r] = a.alpha * bm[it][q];
      }
    }
  }
  __syncthreads();
  const long long c = (long long)j * nx + i;
  const int cpos = (tb + 1) * ADJ_RX + ta + 1;
  const double g = p.g, ht = p.h_tol, s3 = K<double>::s3;
  const double idx = p.idx, cc = -s3 * idx, i2s3 = K<double>::inv_2s3;
  const double k2s3 = 2.0 * s3 * g * idx;
  int bad = 0;

  // local terms of the cell's own L (Gauss fluxes and bed source), per direction:
  // mu . L_local = -cc (mu_d gs0 + mu_{3+d} gs1 + mu_{6+d} gs2) - mu_qn0 s0 - mu_qn1 s1
  double nl[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) nl[q] = 0.0;
  if (active) {
    double vc[9], mc[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      vc[q] = sm.v[q][cpos];
      mc[q] = sm.m[q][cpos];
    }
    if (!(vc[0] > ht)) bad |= 1;
#pragma unroll
    for (int dir = 0; dir < 2; ++dir) {
      const bool xdir = dir == 0;
      const double c1 = xdir ? vc[1] : vc[2], c4 = xdir ? vc[4] : vc[5], c7 = xdir ? vc[7] : vc[8];
      const double hH = vc[0] + s3 * c1, qxH = vc[3] + s3 * c4, qyH = vc[6] + s3 * c7;
      const double hL = vc[0] - s3 * c1, qxL = vc[3] - s3 * c4, qyL = vc[6] - s3 * c7;
      double zH, zL;
      if (xdir) { zH = 0.5 * (zne + zse); zL = 0.5 * (znw + zsw); }
      else { zH = 0.5 * (znw + zne); zL = 0.5 * (zsw + zse); }
      // revised sides (the bed of each side is its own face bed)
      const double rH = frcp(hH), rL = frcp(hL);
      const double shH = fmax0((hH + zH) - zH), shL = fmax0((hL + zL) - zL);
      const double uH = qxH * rH, vH = qyH * rH, uL = qxL * rL, vL = qyL * rL;
      const double zb1 = (fminr(hH + zH, zH) - fminr(hL + zL, zL)) * i2s3;
      const double hb0 = 0.5 * (shH + shL), hb1 = (shH - shL) * i2s3;
      const double qxH2 = shH * uH, qxL2 = shL * uL, qyH2 = shH * vH, qyL2 = shL * vL;
      const double qb0 = 0.5 * (qxH2 + qxL2), qb1 = (qxH2 - qxL2) * i2s3;
      const double rb0 = 0.5 * (qyH2 + qyL2), rb1 = (qyH2 - qyL2) * i2s3;
      // cotangents of the stored Gauss sums and of the source terms
      const double gsb[3] = {-cc * (xdir ? mc[1] : mc[2]), -cc * (xdir ? mc[4] : mc[5]),
                             -cc * (xdir ? mc[7] : mc[8])};
      const double s0b = -(xdir ? mc[3] : mc[6]), s1b = -(xdir ? mc[4] : mc[8]);
      // Gauss flux cotangents in the normal frame (y faces: normal momentum is y)
      const double fbn[3] = {gsb[0], xdir ? gsb[1] : gsb[2], xdir ? gsb[2] : gsb[1]};
      const double qn0 = xdir ? qb0 : rb0, qn1 = xdir ? qb1 : rb1, qt0 = xdir ? rb0 : qb0, qt1 = xdir ? rb1 : qb1;
      double hpb, qnpb, qtpb, hmb, qnmb, qtmb;
      gauss_rev(g, ht, hb0 + hb1, qn0 + qn1, qt0 + qt1, fbn, hpb, qnpb, qtpb);
      gauss_rev(g, ht, hb0 - hb1, qn0 - qn1, qt0 - qt1, fbn, hmb, qnmb, qtmb);
      // s0 = k2s3 hb0 zb1, s1 = k2s3 hb1 zb1 (zb1 does not depend on the coefficients here)
      const double hb0b = hpb + hmb + s0b * k2s3 * zb1, hb1b = hpb - hmb + s1b * k2s3 * zb1;
      const double qn0b = qnpb + qnmb, qn1b = qnpb - qnmb, qt0b = qtpb + qtmb, qt1b = qtpb - qtmb;
      const double qb0b = xdir ? qn0b : qt0b, qb1b = xdir ? qn1b : qt1b;
      const double rb0b = xdir ? qt0b : qn0b, rb1b = xdir ? qt1b : qn1b;
      const double qxH2b = 0.5 * qb0b + i2s3 * qb1b, qxL2b = 0.5 * qb0b - i2s3 * qb1b;
      const double qyH2b = 0.5 * rb0b + i2s3 * rb1b, qyL2b = 0.5 * rb0b - i2s3 * rb1b;
      const double shHb = 0.5 * hb0b + i2s3 * hb1b + qxH2b * uH + qyH2b * vH;
      const double shLb = 0.5 * hb0b - i2s3 * hb1b + qxL2b * uL + qyL2b * vL;
      const double uHb = qxH2b * shH, vHb = qyH2b * shH, uLb = qxL2b * shL, vLb = qyL2b * shL;
      // through the revision of each side
      const double hHb = shHb - (uHb * uH + vHb * vH) * rH, qxHb = uHb * rH, qyHb = vHb * rH;
      const double hLb = shLb - (uLb * uL + vLb * vL) * rL, qxLb = uLb * rL, qyLb = vLb * rL;
      // high side: d/dU0 = 1, d/dU1d = sqrt(3); low side: 1, -sqrt(3)
      nl[0] += hHb + hLb;
      nl[3] += qxHb + qxLb;
      nl[6] += qyHb + qyLb;
      nl[1] += xdir ? s3 * (hHb - hLb) : 0.0;
      nl[4] += xdir ? s3 * (qxHb - qxLb) : 0.0;
      nl[7] += xdir ? s3 * (qyHb - qyLb) : 0.0;
      nl[2] += xdir ? 0.0 : s3 * (hHb - hLb);
      nl[5] += xdir ? 0.0 : s3 * (qxHb - qxLb);
      nl[8] += xdir ? 0.0 : s3 * (qyHb - qyLb);
    }
  }

  // every face once: each cell's west and south faces, and (threads 0..TY+TX-1) the east
  // faces of the tile's last column and the north faces of its last row
  double ow[6], os[6], oe[6];
  if (active) {
    const AdjFace fw{true, cpos - 1, cpos, i > 0, true, 0.5 * (zsw + znw), j};
    adj_face(p, a, sm, fw, ow, ow + 3, bad);
    const AdjFace fs{false, cpos - ADJ_RX, cpos, j > 0, true, 0.5 * (zsw + zse), i};
    adj_face(p, a, sm, fs, os, os + 3, bad);
  }
  int eslot = -1;  // 0..NFX-1: an x face, NFX + ...: a y face
  if (ex) {
    const int pos = (tid + 1) * ADJ_RX + (iend - i0);  // the low cell, column iend - 1
    const AdjFace fe{true, pos, pos + 1, true, iend < nx, 0.5 * (ez0 + ez1), ejr};
    adj_face(p, a, sm, fe, oe, oe + 3, bad);
    eslot = tid * (ADJ_TX + 1) + (iend - i0);
  } else if (ey) {
    const int pos = (jend - j0) * ADJ_RX + (eic - i0) + 1;  // the low cell, row jend - 1
    const AdjFace fn{false, pos, pos + ADJ_RX, true, jend < ny, 0.5 * (ez0 + ez1), eic};
    adj_face(p, a, sm, fn, oe, oe + 3, bad);
    eslot = ADJ_NFX + (jend - j0) * ADJ_TX + (eic - i0);
  }
  __syncthreads();  // the box is no longer read: its LDS takes the face cotangents
  if (active) {
    const int xr = tb * (ADJ_TX + 1) + ta, yr = tb * ADJ_TX + ta;
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      sm.fx[q][xr] = ow[q];
      sm.fy[q][yr] = os[q];
    }
  }
  if (eslot >= 0) {
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      if (eslot < ADJ_NFX) sm.fx[q][eslot] = oe[q];
      else sm.fy[q][eslot - ADJ_NFX] = oe[q];
    }
  }
  // the epilogue's global inputs of the cell, issued now so that they arrive while the
  // face cotangents are gathered
  double lcv[9], exv[9], ufr[9], nmf = 0.0, gm0 = 0.0;
  int g0 = -1;
  if (active) {
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      lcv[q] = a.lam_c[q * n + c];
      exv[q] = a.extra ? a.extra[q * n + c] : 0.0;
      ufr[q] = a.U_fr ? a.U_fr[q * n + c] : 0.0;
    }
    if (a.U_fr) nmf = p.manning ? p.manning[c] : p.n_scalar;
    if (a.U_fr && a.gman) gm0 = a.gman[c];
    if (a.gmap) g0 = a.gmap[c];
  }
  __syncthreads();
  if (!active) {  // no barrier follows; an extra face may still have set a flag
    if (bad) atomicOr(a.regime, bad);
    return;
  }

  // the cell's face-limit cotangents (W, E, S, N), chained to the coefficients as
  // d/dU0 = 1, d/dU1 = sgn sqrt(3) (sgn + for the high side of the cell)
  double nu[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) nu[q] = 0.0;
  const int xr = tb * (ADJ_TX + 1) + ta, yr = tb * ADJ_TX + ta;
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    const bool xdir = f < 2, high = (f & 1) != 0;
    const double sgn = high ? 1.0 : -1.0;
    const int o = high ? 0 : 3;  // the cell is the low side of its east and north faces
    double hb, qxb, qyb;
    if (xdir) {
      const int r = xr + (high ? 1 : 0);
      hb = sm.fx[o][r]; qxb = sm.fx[o + 1][r]; qyb = sm.fx[o + 2][r];
    } else {
      const int r = yr + (high ? ADJ_TX : 0);
      hb = sm.fy[o][r]; qxb = sm.fy[o + 1][r]; qyb = sm.fy[o + 2][r];
    }
    nu[0] += hb;
    nu[3] += qxb;
    nu[6] += qyb;
    nu[1] += xdir ? sgn * s3 * hb : 0.0;
    nu[4] += xdir ? sgn * s3 * qxb : 0.0;
    nu[7] += xdir ? sgn * s3 * qyb : 0.0;
    nu[2] += xdir ? 0.0 : sgn * s3 * hb;
    nu[5] += xdir ? 0.0 : sgn * s3 * qxb;
    nu[8] += xdir ? 0.0 : sgn * s3 * qyb;
  }

  // the local terms, the combination with the incoming cotangents, then the friction
  // adjoint
#pragma unroll
  for (int q = 0; q < 9; ++q) nu[q] += nl[q] + a.cl * lcv[q] + exv[q];
  if (a.U_fr) {
    const double gn = adj_friction_cell(p, ufr, nmf, a.dt_fr, nu);
    if (a.gman) a.gman[c] = gm0 + gn;
  }
  for (int gg = g0; gg >= 0; gg = a.gnext[gg]) nu[0] += a.seed[gg];
#pragma unroll
  for (int q = 0; q < 9; ++q) a.out[q * n + c] = nu[q];
  if (bad) atomicOr(a.regime, bad);
}

// a recomputation's control block takes the time of step k (one thread)
__global__ void set_time_kernel(Ctrl* ctrl, const double* __restrict__ t, int k) {
  if (threadIdx.x == 0 && blockIdx.x == 0) ctrl->t[0] = t[k];
}

// gauge depths of a state (plane 0) into out[g]
__global__ void gauge_read_kernel(const double* __restrict__ U, const int* __restrict__ gi, int ng,
                                  double* __restrict__ out) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g < ng) out[g] = U[gi[g]];
}

// lam[plane 0][gauge g] += seed[g]
__global__ void gauge_seed_kernel(double* __restrict__ lam, const int* __restrict__ gi, int ng,
                                  const double* __restrict__ seed) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g < ng) atomicAdd(&lam[gi[g]], seed[g]);
}

}  // namespace dg2k
