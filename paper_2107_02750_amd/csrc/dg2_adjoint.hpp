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
// (dL/dV)^T mu is gathered per cell: L of a cell depends on its own coefficients
// through its four face sides (Gauss fluxes, bed source, and the four face fluxes)
// and on a neighbour's only through the shared face flux. So each cell needs the
// cotangent of each of its face fluxes (collected from the cell and the neighbour)
// and the derivative of those fluxes and of its own local terms with respect to its
// own face limits. Those local derivatives come from forward-mode dual numbers run
// through the same face, flux and friction formulas as the forward kernels; the
// products with the cotangents and the chain to the nine coefficients are written out.
//
// The regime is checked while the adjoint runs: a cell at or below h_tol, a face
// depth not above zero, or an active face-velocity cap set a flag (the derivative
// would then need terms this adjoint leaves out).
#pragma once

namespace dg2k {

// value and N first derivatives
template <int N>
struct Dual {
  double v;
  double d[N];
};

template <int N>
__device__ __forceinline__ Dual<N> dconst(double v) {
  Dual<N> r;
  r.v = v;
#pragma unroll
  for (int k = 0; k < N; ++k) r.d[k] = 0.0;
  return r;
}
template <int N>
__device__ __forceinline__ Dual<N> dvar(double v, int k) {
  Dual<N> r = dconst<N>(v);
  r.d[k] = 1.0;
  return r;
}
template <int N>
__device__ __forceinline__ Dual<N> operator+(Dual<N> a, Dual<N> b) {
  Dual<N> r;
  r.v = a.v + b.v;
#pragma unroll
  for (int k = 0; k < N; ++k) r.d[k] = a.d[k] + b.d[k];
  return r;
}
template <int N>
__device__ __forceinline__ Dual<N> operator-(Dual<N> a, Dual<N> b) {
  Dual<N> r;
  r.v = a.v - b.v;
#pragma unroll
  for (int k = 0; k < N; ++k) r.d[k] = a.d[k] - b.d[k];
  return r;
}
template <int N>
__device__ __forceinline__ Dual<N> operator-(Dual<N> a) {
  Dual<N> r;
  r.v = -a.v;
#pragma unroll
  for (int k = 0; k < N; ++k) r.d[k] = -a.d[k];
  return r;
}
template <int N>
__device__ __forceinline__ Dual<N> operator*(Dual<N> a, Dual<N> b) {
  Dual<N> r;
  r.v = a.v * b.v;
#pragma unroll
  for (int k = 0; k < N; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k];
  return r;
}
template <int N>
__device__ __forceinline__ Dual<N> operator*(double a, Dual<N> b) {
  Dual<N> r;
  r.v = a * b.v;
#pragma unroll
  for (int k = 0; k < N; ++k) r.d[k] = a * b.d[k];
  return r;
}
template <int N>
__device__ __forceinline__ Dual<N> operator*(Dual<N> b, double a) { return a * b; }
template <int N>
__device__ __forceinline__ Dual<N> operator+(Dual<N> a, double b) {
  a.v += b;
  return a;
}
template <int N>
__device__ __forceinline__ Dual<N> operator+(double b, Dual<N> a) {
  a.v += b;
  return a;
}
template <int N>
__device__ __forceinline__ Dual<N> operator-(Dual<N> a, double b) {
  a.v -= b;
  return a;
}
template <int N>
__device__ __forceinline__ Dual<N> operator-(double b, Dual<N> a) {
  return dconst<N>(b) - a;
}
// 1/x: d(1/x) = -dx / x^2
template <int N>
__device__ __forceinline__ Dual<N> drcp(Dual<N> x) {
  const double r = frcp(x.v);
  Dual<N> o;
  o.v = r;
#pragma unroll
  for (int k = 0; k < N; ++k) o.d[k] = -r * r * x.d[k];
  return o;
}
template <int N>
__device__ __forceinline__ Dual<N> operator/(Dual<N> a, Dual<N> b) { return a * drcp(b); }
// sqrt(x) for x > 0 (0 with zero derivative otherwise)
template <int N>
__device__ __forceinline__ Dual<N> dsqrtd(Dual<N> x) {
  const double s = fsqrt(x.v);
  Dual<N> o;
  o.v = s;
  const double h = s > 0.0 ? 0.5 * frcp(s) : 0.0;
#pragma unroll
  for (int k = 0; k < N; ++k) o.d[k] = h * x.d[k];
  return o;
}
// x^(-1/2) for x > 0
template <int N>
__device__ __forceinline__ Dual<N> drsq(Dual<N> x) {
  const double y = frsq(x.v);
  Dual<N> o;
  o.v = y;
  const double f = -0.5 * y * y * y;  // -x^(-3/2) / 2
#pragma unroll
  for (int k = 0; k < N; ++k) o.d[k] = f * x.d[k];
  return o;
}
// x^(-1/3) for x > 0
template <int N>
__device__ __forceinline__ Dual<N> dinvcbrt(Dual<N> x) {
  const double y = finvcbrt(x.v);
  Dual<N> o;
  o.v = y;
  const double f = -0.33333333333333333333 * (y * y) * (y * y);  // -x^(-4/3) / 3
#pragma unroll
  for (int k = 0; k < N; ++k) o.d[k] = f * x.d[k];
  return o;
}
// x^(1/3) for x >= 0
template <int N>
__device__ __forceinline__ Dual<N> dcbrtd(Dual<N> x) {
  const double y = cbrt(x.v);
  Dual<N> o;
  o.v = y;
  const double f = y > 0.0 ? y / (3.0 * x.v) : 0.0;
#pragma unroll
  for (int k = 0; k < N; ++k) o.d[k] = f * x.d[k];
  return o;
}
template <int N>
__device__ __forceinline__ Dual<N> dsel(bool c, Dual<N> a, Dual<N> b) { return c ? a : b; }
template <int N>
__device__ __forceinline__ Dual<N> dmax(Dual<N> a, Dual<N> b) { return a.v >= b.v ? a : b; }
template <int N>
__device__ __forceinline__ Dual<N> dmin(Dual<N> a, Dual<N> b) { return a.v <= b.v ? a : b; }

// a face side after the revision, as in the forward kernel (FP64 eta form); *capped
// is set when the velocity cap bounds a component (outside the regime)
template <int N>
struct DSide {
  Dual<N> h, u, v, z;
};
template <int N>
__device__ __forceinline__ DSide<N> drevise(Dual<N> h, Dual<N> qx, Dual<N> qy, double zb, double zs,
                                            double ht, double ucap, double vcap_, int* bad) {
  DSide<N> s;
  const Dual<N> eta = h + zb;
  s.h = dmax(eta - zs, dconst<N>(0.0));
  s.z = dmin(eta, dconst<N>(zs));
  if (!(h.v > ht)) *bad |= 1;
  const Dual<N> r = drcp(h);
  s.u = qx * r;
  s.v = qy * r;
  if (fabs(s.u.v) > ucap || fabs(s.v.v) > vcap_) *bad |= 2;
  return s;
}

// the same revision of a side that carries no derivatives (a neighbour's), in plain
// arithmetic
template <int N>
__device__ __forceinline__ DSide<N> drevise_const(double h, double qx, double qy, double zb, double zs,
                                                  double ht, int* bad) {
  const double eta = h + zb;
  if (!(h > ht)) *bad |= 1;
  const double r = frcp(h);
  DSide<N> s;
  s.h = dconst<N>(fmax0(eta - zs));
  s.z = dconst<N>(fminr(eta, zs));
  s.u = dconst<N>(qx * r);
  s.v = dconst<N>(qy * r);
  return s;
}

// HLL in the normal frame, wet-wet or a dry side, as in the forward kernel
template <int N>
__device__ __forceinline__ void dhll(double g, DSide<N> L, DSide<N> R, bool xdir, Dual<N> f[3]) {
  // normal / tangential velocities of each side
  const Dual<N> unL = xdir ? L.u : L.v, utL = xdir ? L.v : L.u;
  const Dual<N> unR = xdir ? R.u : R.v, utR = xdir ? R.v : R.u;
  const Dual<N> hL = L.h, hR = R.h;
  const bool wL = hL.v > 0.0, wR = hR.v > 0.0;
  const Dual<N> cL = dsqrtd(g * hL), cR = dsqrtd(g * hR);
  const Dual<N> us = 0.5 * (unL + unR) + cL - cR;
  const Dual<N> cs = 0.5 * (cL + cR) + 0.25 * (unL - unR);
  const Dual<N> sLw = dmin(unL - cL, us - cs), sRw = dmax(unR + cR, us + cs);
  const Dual<N> sL = wL ? (wR ? sLw : unL - cL) : unR - 2.0 * cR;
  const Dual<N> sR = wL ? (wR ? sRw : unL + 2.0 * cL) : unR + cR;
  const Dual<N> qL = hL * unL, qR = hR * unR;
  const Dual<N> FL[3] = {qL, qL * unL + 0.5 * g * hL * hL, qL * utL};
  const Dual<N> FR[3] = {qR, qR * unR + 0.5 * g * hR * hR, qR * utR};
  const Dual<N> UL[3] = {hL, qL, hL * utL};
  const Dual<N> UR[3] = {hR, qR, hR * utR};
  const Dual<N> inv = drcp(sR - sL), ss = sL * sR;
  const bool up = sL.v >= 0.0, dn = sR.v <= 0.0, dry = !wL && !wR;
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    const Dual<N> mid = (sR * FL[m] - sL * FR[m] + ss * (UR[m] - UL[m])) * inv;
    f[m] = dry ? dconst<N>(0.0) : (up ? FL[m] : (dn ? FR[m] : mid));
  }
}

// physical flux along a normal at a Gauss point (velocities zero at or below h_tol)
template <int N>
__device__ __forceinline__ void dgauss(double g, double ht, Dual<N> h, Dual<N> qn, Dual<N> qt, Dual<N> f[3]) {
  const bool wet = h.v > ht;
  const Dual<N> r = drcp(dmax(h, dconst<N>(Tiny<double>::v)));
  const Dual<N> un = wet ? qn * r : dconst<N>(0.0), ut = wet ? qt * r : dconst<N>(0.0);
  const Dual<N> q = h * un;
  f[0] = q;
  f[1] = q * un + 0.5 * g * h * h;
  f[2] = q * ut;
}

// the split-implicit friction increment at one point, as friction_inc
template <int N>
__device__ __forceinline__ void dfriction(Dual<N> gn2dt, double ht, Dual<N> h, Dual<N> qx, Dual<N> qy,
                                          Dual<N>& dqx, Dual<N>& dqy) {
  const bool wet = h.v > ht;
  if (!wet) {
    dqx = dqy = dconst<N>(0.0);
    return;
  }
  const Dual<N> y = dinvcbrt(h);
  const Dual<N> y3 = y * y * y;
  const Dual<N> u = qx * y3, v = qy * y3;
  const Dual<N> s2 = u * u + v * v;
  if (!(s2.v > 0.0)) {
    dqx = dqy = dconst<N>(0.0);
    return;
  }
  const Dual<N> rs = drsq(s2);
  const Dual<N> w = gn2dt * (y3 * y);
  const Dual<N> a = w * u * u * rs, b = w * v * v * rs;
  const Dual<N> ab = a + b;
  const Dual<N> d1 = 1.0 + 2.0 * a + b, d2 = 1.0 + a + 2.0 * b;
  const Dual<N> inv = drcp(d1 * d2);
  dqx = -(qx * ab * d2 * inv);
  dqy = -(qy * ab * d1 * inv);
}

// ---------------------------------------------------------------------------------
// adjoint of the friction step at one cell: lam (the cotangent of F) becomes the
// cotangent of U, lam_U = (dF/dU)^T lam_F; returns dJ/dn of the cell
// ---------------------------------------------------------------------------------
__device__ __forceinline__ double adj_friction_cell(const Params<double>& p, const double* __restrict__ U,
                                                    long long c, double dt, double lam[9]) {
  const long long n = p.n;
  const double nm = p.manning ? p.manning[c] : p.n_scalar;
  if (!(nm > 0.0)) return 0.0;
  double u[9], lf[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    u[q] = U[q * n + c];
    lf[q] = lam[q];
  }
  const double ht = p.h_tol;
  const Dual<4> nn = dvar<4>(nm, 3);
  const Dual<4> gn2dt = (p.g * dt) * (nn * nn);
  double gn = 0.0;
  // points: 0 centre; 1, 2: x +/-; 3, 4: y +/-
#pragma unroll 1
  for (int pt = 0; pt < 5; ++pt) {
    const int d = pt == 0 ? 0 : (pt <= 2 ? 1 : 2);
    const double sg = pt == 0 ? 0.0 : ((pt == 1 || pt == 3) ? 1.0 : -1.0);
    const bool xd = d == 1, yd = d == 2;
    const double h1 = xd ? u[1] : (yd ? u[2] : 0.0);
    const double qx1 = xd ? u[4] : (yd ? u[5] : 0.0);
    const double qy1 = xd ? u[7] : (yd ? u[8] : 0.0);
    const Dual<4> h = dvar<4>(u[0] + sg * h1, 0);
    const Dual<4> qx = dvar<4>(u[3] + sg * qx1, 1);
    const Dual<4> qy = dvar<4>(u[6] + sg * qy1, 2);
    Dual<4> dqx, dqy;
    dfriction<4>(gn2dt, ht, h, qx, qy, dqx, dqy);
    // cotangents of the increments: the centre feeds the means, a Gauss pair feeds
    // half the difference into the slopes of its direction
    const double cx = pt == 0 ? lf[3] : 0.5 * sg * (xd ? lf[4] : lf[5]);
    const double cy = pt == 0 ? lf[6] : 0.5 * sg * (xd ? lf[7] : lf[8]);
    double gin[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) gin[k] = cx * dqx.d[k] + cy * dqy.d[k];
    // the point's inputs are U0 + sg U1d
    lam[0] += gin[0];
    lam[3] += gin[1];
    lam[6] += gin[2];
    lam[1] += xd ? sg * gin[0] : 0.0;
    lam[4] += xd ? sg * gin[1] : 0.0;
    lam[7] += xd ? sg * gin[2] : 0.0;
    lam[2] += yd ? sg * gin[0] : 0.0;
    lam[5] += yd ? sg * gin[1] : 0.0;
    lam[8] += yd ? sg * gin[2] : 0.0;
    gn += gin[3];
  }
  return gn;
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
  double* out;          // 9 planes; may be lam_c itself (each cell reads its own first)
  double* gqf;          // out: dJ/dQ of each inflow boundary face (slots as the face
                        // codes: W[ny], E[ny], S[nx], N[nx]), summed per segment later
  int* regime;          // out: |= violation bits
};

__global__ __launch_bounds__(256) void adj_stage_kernel(Params<double> p, AdjArgs a) {
  const long long n = p.n;
  const int nx = p.nx, ny = p.ny;
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const int i = int(c % nx), j = int(c / nx);
  const double g = p.g, ht = p.h_tol, s3 = K<double>::s3;
  const double idx = 1.0 / p.dx, cc = -s3 * idx, i2s3 = K<double>::inv_2s3;
  const double k2s3 = 2.0 * s3 * g * idx;
  const double slack = dsqrt(p.gd * p.htd);
  auto V = [&](long long k, int q) { return a.V[q * n + k]; };
  auto mu = [&](long long k, int q) { return a.alpha * a.lam[q * n + k]; };
  auto zvv = [&](int iv, int jv) { return p.zv[(long long)jv * (nx + 1) + iv]; };
  auto umean = [&](long long k, bool xv) {
    const double h0 = V(k, 0);
    return h0 > ht ? V(k, xv ? 3 : 6) * frcp(h0) : 0.0;
  };
  int bad = 0;
  if (!(V(c, 0) > ht)) bad |= 1;
  double nu[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) nu[q] = 0.0;

  // the four faces: 0 W, 1 E, 2 S, 3 N; sgn = side of the cell's limit (+ for E/N);
  // the gradient of each face's terms with respect to the cell's own face limit
  // (h, qx, qy) chains to the coefficients as d/dU0 = 1, d/dU1 = sgn sqrt(3)
#pragma unroll 1
  for (int f = 0; f < 4; ++f) {
    const bool xdir = f < 2;
    const bool high = (f & 1) != 0;
    const double sgn = high ? 1.0 : -1.0;
    // own face limit as Dual<4> (h, qx, qy, Q)
    const double c0 = V(c, 0), c3 = V(c, 3), c6 = V(c, 6);
    const double c1 = xdir ? V(c, 1) : V(c, 2), c4 = xdir ? V(c, 4) : V(c, 5), c7 = xdir ? V(c, 7) : V(c, 8);
    const Dual<4> h = dvar<4>(c0 + sgn * s3 * c1, 0);
    const Dual<4> qx = dvar<4>(c3 + sgn * s3 * c4, 1);
    const Dual<4> qy = dvar<4>(c6 + sgn * s3 * c7, 2);
    // face bed (vertex mean) and the neighbour across the face
    const int ni = xdir ? (high ? i + 1 : i - 1) : i, nj = xdir ? j : (high ? j + 1 : j - 1);
    const int va = xdir ? (high ? i + 1 : i) : i, vb = xdir ? j : (high ? j + 1 : j);  // first vertex
    const double zf = 0.5 * (zvv(va, vb) + (xdir ? zvv(va, vb + 1) : zvv(va + 1, vb)));
    const bool inside = ni >= 0 && ni < nx && nj >= 0 && nj < ny;
    const long long nk = inside ? (long long)nj * nx + ni : c;
    // the velocity cap bound of each component (a boundary side copies the cell)
    const double ucap = fmax(fabs(umean(c, true)), fabs(umean(nk, true))) + slack;
    const double vcap_ = fmax(fabs(umean(c, false)), fabs(umean(nk, false))) + slack;
    const DSide<4> own = drevise<4>(h, qx, qy, zf, zf, ht, ucap, vcap_, &bad);
    int qslot = -1;  // face slot of an inflow face
    if (!(own.h.v > 0.0)) bad |= 1;
    DSide<4> nb;
    if (inside) {
      const double ns = -sgn;  // the neighbour's limit on its opposite side
      const double n1 = xdir ? V(nk, 1) : V(nk, 2), n4 = xdir ? V(nk, 4) : V(nk, 5);
      const double n7 = xdir ? V(nk, 7) : V(nk, 8);
      int nbad = 0;
      nb = drevise_const<4>(V(nk, 0) + ns * s3 * n1, V(nk, 3) + ns * s3 * n4, V(nk, 6) + ns * s3 * n7, zf,
                            zf, ht, &nbad);
      bad |= nbad & 1;
      if (!(nb.h.v > 0.0)) bad |= 1;
    } else {
      // ghost beyond a boundary face, from the own side in the normal frame
      const int code = xdir ? p.bface[(high ? ny : 0) + j] : p.bface[2 * ny + (high ? nx : 0) + i];
      const int kind = code & 255;
      const double inward = high ? -1.0 : 1.0;
      Dual<4> un = xdir ? own.u : own.v, ut = xdir ? own.v : own.u;
      Dual<4> gh = own.h, gun = un, gut = ut;
      if (kind == 1) {
        gun = -un;
      } else if (kind == 2) {
        const Seg& sg = p.segs[(code >> 8) - 1];
        gh = dconst<4>(sg.h_b);
        gun = dconst<4>(xdir ? sg.u_b : sg.v_b);
        gut = dconst<4>(xdir ? sg.v_b : sg.u_b);
      } else if (kind == 3) {
        const Seg& sg = p.segs[(code >> 8) - 1];
        qslot = xdir ? (high ? ny : 0) + j : 2 * ny + (high ? nx : 0) + i;
        const Dual<4> Q = dvar<4>(hydrograph(sg, p.knots, p.knots + p.max_knots, a.t), 3);
        const Dual<4> qn = Q * (1.0 / sg.width);
        const Dual<4> hc = dcbrtd(qn * qn * (1.0 / g));
        const Dual<4> hg = own.h.v > hc.v ? own.h : hc;
        gh = hg;
        gun = hg.v > 0.0 ? inward * (qn / hg) : dconst<4>(0.0);
        gut = dconst<4>(0.0);
      }
      nb.h = gh;
      nb.u = xdir ? gun : gut;
      nb.v = xdir ? gut : gun;
      nb.z = dconst<4>(zf);
    }
    // flux through the face: left state = the W/S cell's side
    Dual<4> F[3];
    if (high) dhll<4>(g, own, nb, xdir, F);
    else dhll<4>(g, nb, own, xdir, F);
    // stored order [mass, x-mom, y-mom]: on y faces the HLL gives [mass, y-mom, x-mom]
    const Dual<4> Fs[3] = {F[0], xdir ? F[1] : F[2], xdir ? F[2] : F[1]};
    // cotangent of each stored flux component, from both cells sharing the face:
    // L0 gets -(F_high - F_low)/dx, L1 (this direction) gets cc (F_high + F_low)
    double mt[3];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      const double own0 = mu(c, 3 * m), own1 = xdir ? mu(c, 3 * m + 1) : mu(c, 3 * m + 2);
      // this face is the cell's high face (E/N): -idx; low face (W/S): +idx
      double v = (high ? -idx : idx) * own0 + cc * own1;
      if (inside) {
        const double nb0 = mu(nk, 3 * m), nb1 = xdir ? mu(nk, 3 * m + 1) : mu(nk, 3 * m + 2);
        v += (high ? idx : -idx) * nb0 + cc * nb1;
      }
      mt[m] = v;
    }
    const Dual<4> J = mt[0] * Fs[0] + mt[1] * Fs[1] + mt[2] * Fs[2];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double gk = J.d[k];
      nu[3 * k] += gk;
      nu[3 * k + 1] += xdir ? sgn * s3 * gk : 0.0;
      nu[3 * k + 2] += xdir ? 0.0 : sgn * s3 * gk;
    }
    if (qslot >= 0) a.gqf[qslot] = J.d[3];
  }

  // local terms of the cell's own L (Gauss fluxes and bed source), per direction
#pragma unroll
  for (int dir = 0; dir < 2; ++dir) {
    const bool xdir = dir == 0;
    const int d = xdir ? 1 : 2;
    // Dual<6>: the high-side limit (E/N: h, qx, qy) then the low-side limit (W/S)
    Dual<6> hH = dvar<6>(V(c, 0) + s3 * V(c, d), 0), qxH = dvar<6>(V(c, 3) + s3 * V(c, 3 + d), 1),
            qyH = dvar<6>(V(c, 6) + s3 * V(c, 6 + d), 2);
    Dual<6> hL = dvar<6>(V(c, 0) - s3 * V(c, d), 3), qxL = dvar<6>(V(c, 3) - s3 * V(c, 3 + d), 4),
            qyL = dvar<6>(V(c, 6) - s3 * V(c, 6 + d), 5);
    double zH, zL;
    if (xdir) { zH = 0.5 * (zvv(i + 1, j + 1) + zvv(i + 1, j)); zL = 0.5 * (zvv(i, j + 1) + zvv(i, j)); }
    else { zH = 0.5 * (zvv(i, j + 1) + zvv(i + 1, j + 1)); zL = 0.5 * (zvv(i, j) + zvv(i + 1, j)); }
    int dummy = 0;
    const DSide<6> sH = drevise<6>(hH, qxH, qyH, zH, zH, ht, 1e300, 1e300, &dummy);
    const DSide<6> sL = drevise<6>(hL, qxL, qyL, zL, zL, ht, 1e300, 1e300, &dummy);
    const Dual<6> hb0 = 0.5 * (sH.h + sL.h), hb1 = (sH.h - sL.h) * i2s3;
    const Dual<6> qxH2 = sH.h * sH.u, qxL2 = sL.h * sL.u, qyH2 = sH.h * sH.v, qyL2 = sL.h * sL.v;
    const Dual<6> qb0 = 0.5 * (qxH2 + qxL2), qb1 = (qxH2 - qxL2) * i2s3;
    const Dual<6> rb0 = 0.5 * (qyH2 + qyL2), rb1 = (qyH2 - qyL2) * i2s3;
    const Dual<6> zb1 = (sH.z - sL.z) * i2s3;
    Dual<6> Gp[3], Gm[3];
    if (xdir) {
      dgauss<6>(g, ht, hb0 + hb1, qb0 + qb1, rb0 + rb1, Gp);
      dgauss<6>(g, ht, hb0 - hb1, qb0 - qb1, rb0 - rb1, Gm);
    } else {
      dgauss<6>(g, ht, hb0 + hb1, rb0 + rb1, qb0 + qb1, Gp);
      dgauss<6>(g, ht, hb0 - hb1, rb0 - rb1, qb0 - qb1, Gm);
    }
    // sums in stored order [mass, x-mom, y-mom]
    const Dual<6> gs[3] = {Gp[0] + Gm[0], xdir ? Gp[1] + Gm[1] : Gp[2] + Gm[2],
                           xdir ? Gp[2] + Gm[2] : Gp[1] + Gm[1]};
    const Dual<6> s0 = k2s3 * hb0 * zb1, s1 = k2s3 * hb1 * zb1;
    // local part of mu . L: -cc * gs in L1 of this direction; -s0 in the momentum mean
    // of this direction's normal component, -s1 in its slope
    const int qn0 = xdir ? 3 : 6, qn1 = xdir ? 4 : 8;
    Dual<6> J = (-cc * mu(c, d)) * gs[0] + (-cc * mu(c, 3 + d)) * gs[1] + (-cc * mu(c, 6 + d)) * gs[2];
    J = J - mu(c, qn0) * s0 - mu(c, qn1) * s1;
    // high-side limit: d/dU0 = 1, d/dU1d = sqrt(3); low side: 1, -sqrt(3)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      nu[3 * k] += J.d[k] + J.d[3 + k];
      nu[3 * k + d] += s3 * (J.d[k] - J.d[3 + k]);
    }
  }

  // the combination with the incoming cotangents, then the friction adjoint
#pragma unroll
  for (int q = 0; q < 9; ++q) nu[q] += a.cl * a.lam_c[q * n + c] + (a.extra ? a.extra[q * n + c] : 0.0);
  if (a.U_fr) {
    const double gn = adj_friction_cell(p, a.U_fr, c, a.dt_fr, nu);
    if (a.gman) a.gman[c] += gn;
  }
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
