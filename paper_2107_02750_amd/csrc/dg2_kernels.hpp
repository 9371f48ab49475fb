// dg2_kernels.hpp -- gfx950 kernels of the uniform-grid DG2 step (arXiv:2107.02750,
// Sect. 2.1.1 and 2.1.4). Included by dg2.hip only.
//
// One time step is two launches of one stage kernel:
//   stage 1: U^n (with a 2-cell cross halo) -> friction -> limiter -> face revision ->
//            HLL -> L -> writes V^n (the limited, friction-applied U^n) and
//            U^int = V^n + dt L(V^n)
//   stage 2: U^int (with halo) -> limiter -> ... -> L, plus V^n of the cell itself ->
//            writes U^{n+1} = (V^n + V^int + dt L(V^int)) / 2 over V^n, and reduces the
//            next CFL time step (wave shuffles -> LDS -> one 64-bit atomic min per block)
// Each block owns a TX x TY tile. It stages the tile and its halo in LDS, computes
// every face of the tile once, and keeps each cell's own data in registers. Blocks are
// mapped to tiles so that the blocks one XCD receives cover a contiguous band of tiles
// (neighbouring tiles then share that XCD's L2).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace dg2k {

constexpr int TX = 32;            // tile width (cells, x fastest in memory)
constexpr int TY = 8;             // tile height
constexpr int NT = TX * TY;       // threads per block, one cell each
constexpr int RX = TX + 4;        // LDS box with a 2-cell halo
constexpr int RY = TY + 4;
constexpr int RB = RX * RY;
constexpr int NRING = 2 * (TX + TY);  // non-corner cells of the first halo ring
constexpr int NXCD = 8;

constexpr unsigned long long INF_BITS = 0x7FF0000000000000ull;

struct Seg {
  int kind, edge, i0, i1, k0, nk;
  double width, h_b, u_b, v_b;
};

// control block shared by the launches of a context; slot [p] belongs to the step that
// starts from state buffer p
struct Ctrl {
  double t[2];
  double dt_used[2];
  unsigned long long dtc[2];  // min over cells of dx / (|u| + c), as positive-double bits
  long long step[2];
  int health;                 // bit 0: NaN seen, bit 1: time step below 1e-12 s
  int pad;
};

template <typename R>
struct Params {
  const R* __restrict__ uin;   // U^n (the stage-1 input; stage 2 reads ui)
  R* __restrict__ vbuf;        // V^n out (stage 1); V^n in, U^{n+1} out (stage 2)
  R* __restrict__ ui;          // U^int out (stage 1)
  const R* __restrict__ zv;    // vertex bed
  const R* __restrict__ manning;  // per cell, or nullptr
  const int* __restrict__ bface;  // boundary faces: W[ny], E[ny], S[nx], N[nx]
  const Seg* __restrict__ segs;
  const double* __restrict__ knots;  // t[DG2_MAX_KNOTS] then q[DG2_MAX_KNOTS]
  Ctrl* ctrl;
  double* ledger;              // per tile: in, out, clip, unused
  long long n;                 // nx * ny
  int nx, ny, tiles_x, n_tiles, per_xcd, nsegs, max_knots, limiter, parity;
  R dx, g, h_tol, n_scalar;
  double dxd, gd, cfl, htd, dt_dry, dt_max, t_end;
};

template <typename R> struct K;
template <> struct K<double> {
  static constexpr double s3 = 1.7320508075688772935274463415059;
  static constexpr double inv_s3 = 0.57735026918962576450914878050196;
  static constexpr double inv_2s3 = 0.28867513459481288225457439025098;
};
template <> struct K<float> {
  static constexpr float s3 = 1.7320508075688772935f;
  static constexpr float inv_s3 = 0.57735026918962576451f;
  static constexpr float inv_2s3 = 0.28867513459481288225f;
};

__device__ __forceinline__ double dsqrt(double x) { return __builtin_sqrt(x); }
__device__ __forceinline__ float dsqrt(float x) { return __builtin_sqrtf(x); }
__device__ __forceinline__ double dcbrt(double x) { return cbrt(x); }
__device__ __forceinline__ float dcbrt(float x) { return cbrtf(x); }
__device__ __forceinline__ double dabs(double x) { return __builtin_fabs(x); }
__device__ __forceinline__ float dabs(float x) { return __builtin_fabsf(x); }

template <typename R>
__device__ __forceinline__ R minmod3(R a, R b, R c) {
  if (a > R(0) && b > R(0) && c > R(0)) return a < b ? (a < c ? a : c) : (b < c ? b : c);
  if (a < R(0) && b < R(0) && c < R(0)) return a > b ? (a > c ? a : c) : (b > c ? b : c);
  return R(0);
}

// Q(t) of an inflow segment: linear between knots, held outside them
__device__ inline double hydrograph(const Seg& s, const double* kt, const double* kq, double t) {
  const int n = s.nk, k0 = s.k0;
  if (t <= kt[k0]) return kq[k0];
  if (t >= kt[k0 + n - 1]) return kq[k0 + n - 1];
  int k = 0;
  while (k + 1 < n && kt[k0 + k + 1] <= t) ++k;
  const double a = (t - kt[k0 + k]) / (kt[k0 + k + 1] - kt[k0 + k]);
  return kq[k0 + k] + a * (kq[k0 + k + 1] - kq[k0 + k]);
}

// the step's time step, identical in every block of both stage launches
template <typename R>
__device__ __forceinline__ void step_time(const Params<R>& p, double& t, double& dt, double& t_next,
                                          double& dt_cfl) {
  t = p.ctrl->t[p.parity];
  const double m = __longlong_as_double((long long)p.ctrl->dtc[p.parity]);
  double d = (m == __longlong_as_double((long long)INF_BITS)) ? p.dt_dry : p.cfl * m;
  dt_cfl = d;
  if (p.dt_max > 0.0 && p.dt_max < d) d = p.dt_max;
  t_next = t + d;
  if (p.t_end - t <= d) {
    d = p.t_end - t;
    t_next = p.t_end;
  }
  dt = d;
}

// a face side after the wet/dry revision: depth, velocities, revised bed
template <typename R>
struct Side {
  R h, u, v, z;
};

template <typename R>
__device__ __forceinline__ Side<R> revise(R h, R qx, R qy, R zb, R zs, R ht) {
  Side<R> s;
  const R eta = h + zb;
  const R d = eta - zs;
  s.h = d > R(0) ? d : R(0);
  if (h > ht) {
    const R r = R(1) / h;
    s.u = qx * r;
    s.v = qy * r;
  } else {
    s.u = R(0);
    s.v = R(0);
  }
  s.z = eta < zs ? eta : zs;
  return s;
}

// HLL flux through a face, normal frame: (h, un, ut) on each side ->
// [mass, normal momentum, tangential momentum]
template <typename R>
__device__ __forceinline__ void hll(R g, R hL, R unL, R utL, R hR, R unR, R utR, R f[3]) {
  if (!(hL > R(0)) && !(hR > R(0))) {
    f[0] = f[1] = f[2] = R(0);
    return;
  }
  const R cL = dsqrt(g * hL), cR = dsqrt(g * hR);
  R sL, sR;
  if (!(hL > R(0))) {
    sL = unR - R(2) * cR;
    sR = unR + cR;
  } else if (!(hR > R(0))) {
    sL = unL - cL;
    sR = unL + R(2) * cL;
  } else {
    const R us = R(0.5) * (unL + unR) + cL - cR;
    const R cs = R(0.5) * (cL + cR) + R(0.25) * (unL - unR);
    const R a = unL - cL, b = us - cs, c = unR + cR, d = us + cs;
    sL = a < b ? a : b;
    sR = c > d ? c : d;
  }
  const R qL = hL * unL, qR = hR * unR;
  const R pL = R(0.5) * g * hL * hL, pR = R(0.5) * g * hR * hR;
  if (sL >= R(0)) {
    f[0] = qL;
    f[1] = qL * unL + pL;
    f[2] = qL * utL;
  } else if (sR <= R(0)) {
    f[0] = qR;
    f[1] = qR * unR + pR;
    f[2] = qR * utR;
  } else {
    const R inv = R(1) / (sR - sL);
    const R ss = sL * sR;
    f[0] = (sR * qL - sL * qR + ss * (hR - hL)) * inv;
    f[1] = (sR * (qL * unL + pL) - sL * (qR * unR + pR) + ss * (qR - qL)) * inv;
    f[2] = (sR * qL * utL - sL * qR * utR + ss * (hR * utR - hL * utL)) * inv;
  }
}

// physical flux along a normal at a Gauss point, velocities zero at or below h_tol
template <typename R>
__device__ __forceinline__ void gauss_flux(R g, R ht, R h, R qn, R qt, R f[3]) {
  R un = R(0), ut = R(0);
  if (h > ht) {
    const R r = R(1) / h;
    un = qn * r;
    ut = qt * r;
  }
  const R q = h * un;
  f[0] = q;
  f[1] = q * un + R(0.5) * g * h * h;
  f[2] = q * ut;
}

// Split-implicit Manning increment at one point: with w = dt g n^2 h^(-4/3) and
// s = |u|, the Newton step of backward Euler with the diagonal Jacobian gives
// dqx = -qx w s / (1 + w (2u^2 + v^2) / s), and likewise for qy.
template <typename R>
__device__ __forceinline__ void friction_inc(R gn2dt, R ht, R h, R qx, R qy, R& dqx, R& dqy) {
  dqx = R(0);
  dqy = R(0);
  if (!(h > ht)) return;
  const R r = R(1) / h;
  const R u = qx * r, v = qy * r;
  const R s2 = u * u + v * v;
  if (!(s2 > R(0))) return;
  const R rs = R(1) / dsqrt(s2);
  const R w = gn2dt * r / dcbrt(h);
  const R a = w * u * u * rs, b = w * v * v * rs;
  const R ab = a + b;
  dqx = -qx * ab / (R(1) + R(2) * a + b);
  dqy = -qy * ab / (R(1) + a + R(2) * b);
}

template <typename R>
__device__ __forceinline__ R zvat(const Params<R>& p, int iv, int jv) {
  return p.zv[(long long)jv * (p.nx + 1) + iv];
}

// bed mean and slopes of cell (i, j) (eq 8; mean summed in diagonal pairs)
template <typename R>
__device__ __forceinline__ void bed(const Params<R>& p, int i, int j, R& z0, R& z1x, R& z1y) {
  const R sw = zvat(p, i, j), se = zvat(p, i + 1, j);
  const R nw = zvat(p, i, j + 1), ne = zvat(p, i + 1, j + 1);
  z0 = R(0.25) * ((ne + sw) + (nw + se));
  z1x = (R(0.5) * (ne + se) - R(0.5) * (nw + sw)) * K<R>::inv_2s3;
  z1y = (R(0.5) * (nw + ne) - R(0.5) * (sw + se)) * K<R>::inv_2s3;
}

// ghost state beyond a boundary face, from the interior side's revised state in the
// face's normal frame (inward = +1 on W/S edges, -1 on E/N edges)
template <typename R>
__device__ __forceinline__ void ghost(const Params<R>& p, int code, double t, bool normal_x, R inward,
                                      R h, R un, R ut, R& gh, R& gun, R& gut) {
  const int kind = code & 255;
  gh = h;
  gun = un;
  gut = ut;
  if (kind == 1) {
    gun = -un;
  } else if (kind == 2) {
    const Seg& s = p.segs[(code >> 8) - 1];
    gh = R(s.h_b);
    gun = R(normal_x ? s.u_b : s.v_b);
    gut = R(normal_x ? s.v_b : s.u_b);
  } else if (kind == 3) {
    const Seg& s = p.segs[(code >> 8) - 1];
    const R qn = R(hydrograph(s, p.knots, p.knots + p.max_knots, t) / s.width);
    const R hc = dcbrt(qn * qn / p.g);
    const R hg = h > hc ? h : hc;
    gh = hg;
    gun = hg > R(0) ? inward * (qn / hg) : R(0);
    gut = R(0);
  }
}

// CFL candidate of one cell: min over directions of dx / (|u0| + sqrt(g hmax)) with
// hmax the largest of the mean and the two face limits in that direction; +inf if dry
template <typename R>
__device__ __forceinline__ double cell_dtc(const Params<R>& p, R h0, R h1x, R h1y, R qx0, R qy0) {
  if (!(h0 > p.h_tol)) return __longlong_as_double((long long)INF_BITS);
  const R u = qx0 / h0, v = qy0 / h0;
  const R a = p.dx / (dabs(u) + dsqrt(p.g * (h0 + K<R>::s3 * dabs(h1x))));
  const R b = p.dx / (dabs(v) + dsqrt(p.g * (h0 + K<R>::s3 * dabs(h1y))));
  return double(a < b ? a : b);
}

// magnitude cap of a face-limit velocity component: the larger neighbouring mean
// velocity magnitude plus the velocity scale of the dry tolerance
template <typename R>
__device__ __forceinline__ R vcap(R x, R a, R b, R slack) {
  const R m = (dabs(a) > dabs(b) ? dabs(a) : dabs(b)) + slack;
  return x > m ? m : (x < -m ? -m : x);
}

// CFL candidate of the boundary forcing at time t (critical-depth inflow, fixed state)
template <typename R>
__device__ inline double forcing_dtc(const Params<R>& p, double t) {
  double m = __longlong_as_double((long long)INF_BITS);
  for (int s = 0; s < p.nsegs; ++s) {
    const Seg& sg = p.segs[s];
    if (sg.kind == 3) {
      const R qn = R(hydrograph(sg, p.knots, p.knots + p.max_knots, t) / sg.width);
      if (qn > R(0)) {
        const R hc = dcbrt(qn * qn / p.g);
        if (hc > p.h_tol) {
          const double a = double(p.dx / (qn / hc + dsqrt(p.g * hc)));
          m = a < m ? a : m;
        }
      }
    } else if (sg.kind == 2 && R(sg.h_b) > p.h_tol) {
      const R hb = R(sg.h_b);
      const R c = dsqrt(p.g * hb);
      const R a = p.dx / (dabs(R(sg.u_b)) + c), b = p.dx / (dabs(R(sg.v_b)) + c);
      const double d = double(a < b ? a : b);
      m = d < m ? d : m;
    }
  }
  return m;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}
__device__ __forceinline__ double wave_min(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double y = __shfl_xor(x, o, 64);
    x = y < x ? y : x;
  }
  return x;
}

// ---------------------------------------------------------------------------------
// the stage kernel
// ---------------------------------------------------------------------------------
template <typename R, int STAGE>
__global__ __launch_bounds__(NT) void stage_kernel(Params<R> p) {
  const int b = blockIdx.x;
  const int tile = (b % NXCD) * p.per_xcd + b / NXCD;
  if (tile >= p.n_tiles) return;
  const int tid = threadIdx.x;
  const int i0 = (tile % p.tiles_x) * TX, j0 = (tile / p.tiles_x) * TY;
  const int nx = p.nx, ny = p.ny;
  const long long n = p.n;
  const R ht = p.h_tol;

  double t, dt, t_next, dt_cfl;
  step_time(p, t, dt, t_next, dt_cfl);

  // own cell
  const int ci = i0 + tid % TX, cj = j0 + tid / TX;
  const bool active = ci < nx && cj < ny;
  const long long ck = (long long)cj * nx + ci;

  if (!(dt > 0.0)) {  // the run has reached t_end: carry the state over unchanged
    if (STAGE == 1) {
      if (active)
        for (int q = 0; q < 9; ++q) p.vbuf[q * n + ck] = p.uin[q * n + ck];
      if (tile == 0 && tid == 0) {
        Ctrl* c = p.ctrl;
        const int a = p.parity, o = 1 - p.parity;
        c->t[o] = c->t[a];
        c->step[o] = c->step[a];
        c->dtc[o] = c->dtc[a];
        c->dt_used[a] = 0.0;
      }
    }
    return;
  }
  if (STAGE == 1 && tile == 0 && tid == 0) {
    Ctrl* c = p.ctrl;
    const int a = p.parity, o = 1 - p.parity;
    c->t[o] = t_next;
    c->step[o] = c->step[a] + 1;
    c->dtc[o] = INF_BITS;
    c->dt_used[a] = dt;
    if (dt_cfl < 1e-12) atomicOr(&c->health, 2);
  }

  __shared__ R s_c[9][RB];   // halo box coefficients; later face states and fluxes
  __shared__ R s_z0[RB];
  __shared__ R s_um[RB];  // mean velocities (zero at or below h_tol)
  __shared__ R s_vm[RB];
  __shared__ unsigned char s_flag[RB];
  __shared__ double s_red[NT / 64][4];

  // ---- phase 1: load the box (friction applied in stage 1) ----
  const R dtr = R(dt);
  for (int r = tid; r < RB; r += NT) {
    const int a = r % RX, bb = r / RX;
    const bool inx = a >= 2 && a < TX + 2, iny = bb >= 2 && bb < TY + 2;
    const bool corner = (a == 1 || a == TX + 2) && (bb == 1 || bb == TY + 2);
    if (!(inx || iny || corner)) continue;
    int i = i0 - 2 + a, j = j0 - 2 + bb;
    i = i < 0 ? 0 : (i >= nx ? nx - 1 : i);
    j = j < 0 ? 0 : (j >= ny ? ny - 1 : j);
    const long long k = (long long)j * nx + i;
    R c[9];
    const R* __restrict__ src = STAGE == 1 ? p.uin : p.ui;
#pragma unroll
    for (int q = 0; q < 9; ++q) c[q] = src[q * n + k];
    const R sw = zvat(p, i, j), se = zvat(p, i + 1, j);
    const R nw = zvat(p, i, j + 1), ne = zvat(p, i + 1, j + 1);
    s_z0[r] = R(0.25) * ((ne + sw) + (nw + se));
    if (STAGE == 1 && !corner) {
      const R nm = p.manning ? p.manning[k] : p.n_scalar;
      if (nm > R(0)) {
        const R gn2dt = p.g * nm * nm * dtr;
        R dx0, dy0;
        friction_inc(gn2dt, ht, c[0], c[3], c[6], dx0, dy0);
        const bool needx = iny && a >= 1 && a <= TX + 2;
        const bool needy = inx && bb >= 1 && bb <= TY + 2;
        if (needx) {
          R dxp, dyp, dxm, dym;
          friction_inc(gn2dt, ht, c[0] + c[1], c[3] + c[4], c[6] + c[7], dxp, dyp);
          friction_inc(gn2dt, ht, c[0] - c[1], c[3] - c[4], c[6] - c[7], dxm, dym);
          c[4] += R(0.5) * (dxp - dxm);
          c[7] += R(0.5) * (dyp - dym);
        }
        if (needy) {
          R dxp, dyp, dxm, dym;
          friction_inc(gn2dt, ht, c[0] + c[2], c[3] + c[5], c[6] + c[8], dxp, dyp);
          friction_inc(gn2dt, ht, c[0] - c[2], c[3] - c[5], c[6] - c[8], dxm, dym);
          c[5] += R(0.5) * (dxp - dxm);
          c[8] += R(0.5) * (dyp - dym);
        }
        c[3] += dx0;
        c[6] += dy0;
      }
    }
#pragma unroll
    for (int q = 0; q < 9; ++q) s_c[q][r] = c[q];
    R um = R(0), vm = R(0);
    if (c[0] > ht) {
      const R rh = R(1) / c[0];
      um = c[3] * rh;
      vm = c[6] * rh;
    }
    s_um[r] = um;
    s_vm[r] = vm;
  }
  __syncthreads();

  // ---- phase 2a: front flags and the limiter ----
  // item A: the own cell (both directions); item B: one first-ring cell (one direction)
  const int ca = tid % TX + 2, cb = tid / TX + 2;
  const int cpos = cb * RX + ca;
  const bool has_b = tid < NRING;
  int rb_a = 0, rb_b = 0, rb_dir = 0, rb_side = 0;  // side: 0 W, 1 E, 2 S, 3 N
  if (has_b) {
    if (tid < TY) { rb_a = 1; rb_b = tid + 2; rb_dir = 1; rb_side = 0; }
    else if (tid < 2 * TY) { rb_a = TX + 2; rb_b = tid - TY + 2; rb_dir = 1; rb_side = 1; }
    else if (tid < 2 * TY + TX) { rb_a = tid - 2 * TY + 2; rb_b = 1; rb_dir = 2; rb_side = 2; }
    else { rb_a = tid - 2 * TY - TX + 2; rb_b = TY + 2; rb_dir = 2; rb_side = 3; }
  }
  const int rpos = rb_b * RX + rb_a;
  const int ri = i0 - 2 + rb_a, rj = j0 - 2 + rb_b;
  const bool b_in = has_b && ri >= 0 && ri < nx && rj >= 0 && rj < ny;

  auto limit_cell = [&](int pos, int i, int j, int dirs, R v[9]) -> unsigned char {
#pragma unroll
    for (int q = 0; q < 9; ++q) v[q] = s_c[q][pos];
    const R h0 = v[0];
    if (!(h0 > R(0))) {
#pragma unroll
      for (int q = 0; q < 9; ++q) v[q] = R(0);
      return 1;
    }
    const bool front = !(h0 > ht) || !(s_c[0][pos - 1] > ht) || !(s_c[0][pos + 1] > ht) ||
                       !(s_c[0][pos - RX] > ht) || !(s_c[0][pos + RX] > ht);
    if (front) {
      v[1] = v[2] = v[4] = v[5] = v[7] = v[8] = R(0);
      return 1;
    }
    if (p.limiter) {
      R z0, z1x, z1y;
      bed(p, i, j, z0, z1x, z1y);
      const R e0 = h0 + s_z0[pos];
#pragma unroll
      for (int d = 1; d <= 2; ++d) {
        const int off = d == 1 ? 1 : RX;
        const R zs = d == 1 ? z1x : z1y;
        const R em = s_c[0][pos - off] + s_z0[pos - off];
        const R ep = s_c[0][pos + off] + s_z0[pos + off];
        const R e1 = v[d] + zs;
        const R le = minmod3(e1, (ep - e0) * K<R>::inv_s3, (e0 - em) * K<R>::inv_s3);
        if (le != e1) v[d] = le - zs;
        if (!(dirs & d)) continue;  // discharge slopes only where they are used
#pragma unroll
        for (int var = 1; var <= 2; ++var) {
          const int q0 = 3 * var;
          const R a0 = v[q0];
          const R am = s_c[q0][pos - off], ap = s_c[q0][pos + off];
          v[q0 + d] = minmod3(v[q0 + d], (ap - a0) * K<R>::inv_s3, (a0 - am) * K<R>::inv_s3);
        }
      }
    }
    // a depth plane negative at a face centre: a front inside the cell
    if (h0 - K<R>::s3 * dabs(v[1]) < R(0) || h0 - K<R>::s3 * dabs(v[2]) < R(0)) {
      v[1] = v[2] = v[4] = v[5] = v[7] = v[8] = R(0);
      return 1;
    }
    return 0;
  };

  R va[9];
  if (active && s_c[0][cpos] != s_c[0][cpos]) atomicOr(&p.ctrl->health, 1);  // NaN depth
  const unsigned char fa = limit_cell(cpos, active ? ci : 0, active ? cj : 0, 3, va);
  R vb[9];
  unsigned char fb = 1;
  if (b_in) fb = limit_cell(rpos, ri, rj, rb_dir, vb);
  s_flag[cpos] = fa;
  if (has_b) s_flag[rpos] = fb;
  __syncthreads();  // box reads are done and the flags are visible

  // ---- phase 2b: revised face states ----
  // own cell: W, E, S, N sides (kept); E and N sides published for the neighbours
  R* const s_side = &s_c[0][0];  // planes 0..2: east side (h, u, v); 3..5: north side
  Side<R> sw_, se_, ss_, sn_;
  const R s3 = K<R>::s3;
  const R slack = R(dsqrt(p.gd * p.htd));
  auto zside = [&](int pos, int i, int j, R zf) -> R {
    // bed of the side at position pos: flat at z0 for a first-order cell
    (void)i; (void)j;
    return s_flag[pos] ? s_z0[pos] : zf;
  };
  if (active) {
    const R zW = R(0.5) * (zvat(p, ci, cj + 1) + zvat(p, ci, cj));
    const R zE = R(0.5) * (zvat(p, ci + 1, cj + 1) + zvat(p, ci + 1, cj));
    const R zS = R(0.5) * (zvat(p, ci, cj) + zvat(p, ci + 1, cj));
    const R zN = R(0.5) * (zvat(p, ci, cj + 1) + zvat(p, ci + 1, cj + 1));
    const R own_w = fa ? s_z0[cpos] : zW, own_e = fa ? s_z0[cpos] : zE;
    const R own_s = fa ? s_z0[cpos] : zS, own_n = fa ? s_z0[cpos] : zN;
    const R nb_w = ci > 0 ? zside(cpos - 1, ci - 1, cj, zW) : own_w;
    const R nb_e = ci < nx - 1 ? zside(cpos + 1, ci + 1, cj, zE) : own_e;
    const R nb_s = cj > 0 ? zside(cpos - RX, ci, cj - 1, zS) : own_s;
    const R nb_n = cj < ny - 1 ? zside(cpos + RX, ci, cj + 1, zN) : own_n;
    sw_ = revise(va[0] - s3 * va[1], va[3] - s3 * va[4], va[6] - s3 * va[7], own_w,
                 own_w > nb_w ? own_w : nb_w, ht);
    se_ = revise(va[0] + s3 * va[1], va[3] + s3 * va[4], va[6] + s3 * va[7], own_e,
                 own_e > nb_e ? own_e : nb_e, ht);
    ss_ = revise(va[0] - s3 * va[2], va[3] - s3 * va[5], va[6] - s3 * va[8], own_s,
                 own_s > nb_s ? own_s : nb_s, ht);
    sn_ = revise(va[0] + s3 * va[2], va[3] + s3 * va[5], va[6] + s3 * va[8], own_n,
                 own_n > nb_n ? own_n : nb_n, ht);
    const R u0 = s_um[cpos], v0 = s_vm[cpos];
    const int pw = ci > 0 ? cpos - 1 : cpos, pe = ci < nx - 1 ? cpos + 1 : cpos;
    const int ps = cj > 0 ? cpos - RX : cpos, pn = cj < ny - 1 ? cpos + RX : cpos;
    sw_.u = vcap(sw_.u, u0, s_um[pw], slack); sw_.v = vcap(sw_.v, v0, s_vm[pw], slack);
    se_.u = vcap(se_.u, u0, s_um[pe], slack); se_.v = vcap(se_.v, v0, s_vm[pe], slack);
    ss_.u = vcap(ss_.u, u0, s_um[ps], slack); ss_.v = vcap(ss_.v, v0, s_vm[ps], slack);
    sn_.u = vcap(sn_.u, u0, s_um[pn], slack); sn_.v = vcap(sn_.v, v0, s_vm[pn], slack);
  }
  // ring item: W ring publishes its east side, S ring its north side; E and N ring
  // cells keep their west / south side for the tile's east / north faces
  Side<R> sb_;
  sb_.h = sb_.u = sb_.v = sb_.z = R(0);
  if (b_in) {
    const int oa = rb_side == 0 ? 1 : (rb_side == 1 ? -1 : 0);
    const int ob = rb_side == 2 ? 1 : (rb_side == 3 ? -1 : 0);
    const int npos = rpos + oa + ob * RX;  // the tile cell across the face
    const int ni = ri + oa, nj = rj + ob;
    R zf;
    if (rb_side == 0) zf = R(0.5) * (zvat(p, ri + 1, rj + 1) + zvat(p, ri + 1, rj));
    else if (rb_side == 1) zf = R(0.5) * (zvat(p, ri, rj + 1) + zvat(p, ri, rj));
    else if (rb_side == 2) zf = R(0.5) * (zvat(p, ri, rj + 1) + zvat(p, ri + 1, rj + 1));
    else zf = R(0.5) * (zvat(p, ri, rj) + zvat(p, ri + 1, rj));
    const R own = fb ? s_z0[rpos] : zf;
    const R nb = (ni >= 0 && ni < nx && nj >= 0 && nj < ny) ? zside(npos, ni, nj, zf) : own;
    const R zs = own > nb ? own : nb;
    const int d = rb_dir;
    const R sg = (rb_side == 0 || rb_side == 2) ? s3 : -s3;  // toward the tile
    sb_ = revise(vb[0] + sg * vb[d], vb[3] + sg * vb[3 + d], vb[6] + sg * vb[6 + d], own, zs, ht);
    sb_.u = vcap(sb_.u, s_um[rpos], s_um[npos], slack);
    sb_.v = vcap(sb_.v, s_vm[rpos], s_vm[npos], slack);
  }
  if (active) {  // s_c is no longer read: it now holds face data
    s_side[0 * RB + cpos] = se_.h;
    s_side[1 * RB + cpos] = se_.u;
    s_side[2 * RB + cpos] = se_.v;
    s_side[3 * RB + cpos] = sn_.h;
    s_side[4 * RB + cpos] = sn_.u;
    s_side[5 * RB + cpos] = sn_.v;
  }
  if (b_in && rb_side == 0) {
    s_side[0 * RB + rpos] = sb_.h;
    s_side[1 * RB + rpos] = sb_.u;
    s_side[2 * RB + rpos] = sb_.v;
  }
  if (b_in && rb_side == 2) {
    s_side[3 * RB + rpos] = sb_.h;
    s_side[4 * RB + rpos] = sb_.u;
    s_side[5 * RB + rpos] = sb_.v;
  }
  __syncthreads();

  // ---- phase 2c: HLL on the west and south face of each position ----
  const double t_stage = STAGE == 1 ? t : t_next;
  const R g = p.g;
  double led_in = 0.0, led_out = 0.0, led_clip = 0.0;
  const double wflux = 0.5 * dt * p.dxd;  // ledger weight: RK2 half step times face width
  R fw[3] = {R(0), R(0), R(0)}, fs[3] = {R(0), R(0), R(0)};
  // x-face at index f between cells f-1 and f on row j; pos is the box position of f
  auto xface = [&](int f, int j, int pos, const Side<R>& own_r, bool have_r, R out[3]) -> bool {
    if (j >= ny || f > nx) return false;
    R lh, lu, lv, rh, ru, rv;
    if (f > 0) {
      lh = s_side[0 * RB + pos - 1];
      lu = s_side[1 * RB + pos - 1];
      lv = s_side[2 * RB + pos - 1];
    }
    if (f < nx) {
      if (!have_r) return false;
      rh = own_r.h; ru = own_r.u; rv = own_r.v;
    }
    if (f == 0) {
      ghost(p, p.bface[j], t_stage, true, R(1), rh, ru, rv, lh, lu, lv);
    } else if (f == nx) {
      ghost(p, p.bface[ny + j], t_stage, true, R(-1), lh, lu, lv, rh, ru, rv);
    }
    hll(g, lh, lu, lv, rh, ru, rv, out);
    if (f == 0) {
      const double m = double(out[0]) * wflux;
      if (m > 0) led_in += m; else led_out -= m;
    } else if (f == nx) {
      const double m = -double(out[0]) * wflux;
      if (m > 0) led_in += m; else led_out -= m;
    }
    return true;
  };
  auto yface = [&](int i, int f, int pos, const Side<R>& own_r, bool have_r, R out[3]) -> bool {
    if (i >= nx || f > ny) return false;
    R lh, lu, lv, rh, ru, rv;  // (h, normal = v, tangential = u)
    if (f > 0) {
      lh = s_side[3 * RB + pos - RX];
      lu = s_side[5 * RB + pos - RX];  // normal: v
      lv = s_side[4 * RB + pos - RX];  // tangential: u
    }
    if (f < ny) {
      if (!have_r) return false;
      rh = own_r.h; ru = own_r.v; rv = own_r.u;
    }
    if (f == 0) {
      ghost(p, p.bface[2 * ny + i], t_stage, false, R(1), rh, ru, rv, lh, lu, lv);
    } else if (f == ny) {
      ghost(p, p.bface[2 * ny + nx + i], t_stage, false, R(-1), lh, lu, lv, rh, ru, rv);
    }
    R o[3];
    hll(g, lh, lu, lv, rh, ru, rv, o);
    out[0] = o[0];
    out[1] = o[2];  // x-momentum is tangential on a y-face
    out[2] = o[1];
    if (f == 0) {
      const double m = double(o[0]) * wflux;
      if (m > 0) led_in += m; else led_out -= m;
    } else if (f == ny) {
      const double m = -double(o[0]) * wflux;
      if (m > 0) led_in += m; else led_out -= m;
    }
    return true;
  };
  // own position (also the east / north boundary face when the cell is just outside)
  const bool hw = xface(ci, cj, cpos, sw_, active, fw);
  const bool hs = yface(ci, cj, cpos, ss_, active, fs);
  R fb3[3] = {R(0), R(0), R(0)};
  bool hb = false;
  if (has_b && rb_side == 1) hb = xface(ri, rj, rpos, sb_, b_in, fb3);
  if (has_b && rb_side == 3) hb = yface(ri, rj, rpos, sb_, b_in, fb3);
  __syncthreads();  // side reads done; the same slots now receive fluxes
  if (hw) { s_side[0 * RB + cpos] = fw[0]; s_side[1 * RB + cpos] = fw[1]; s_side[2 * RB + cpos] = fw[2]; }
  if (hs) { s_side[3 * RB + cpos] = fs[0]; s_side[4 * RB + cpos] = fs[1]; s_side[5 * RB + cpos] = fs[2]; }
  if (hb && rb_side == 1) { s_side[0 * RB + rpos] = fb3[0]; s_side[1 * RB + rpos] = fb3[1]; s_side[2 * RB + rpos] = fb3[2]; }
  if (hb && rb_side == 3) { s_side[3 * RB + rpos] = fb3[0]; s_side[4 * RB + rpos] = fb3[1]; s_side[5 * RB + rpos] = fb3[2]; }
  __syncthreads();

  // ---- phase 3: L, the stage update, and the per-block reductions ----
  double my_dtc = __longlong_as_double((long long)INF_BITS);
  if (active) {
    const R fe[3] = {s_side[0 * RB + cpos + 1], s_side[1 * RB + cpos + 1], s_side[2 * RB + cpos + 1]};
    const R fn[3] = {s_side[3 * RB + cpos + RX], s_side[4 * RB + cpos + RX], s_side[5 * RB + cpos + RX]};
    const R idx = R(1) / p.dx;
    const R k2s3 = R(2) * s3 * g * idx;
    R L[9];
    {  // x direction
      const R hb0 = R(0.5) * (se_.h + sw_.h), hb1 = (se_.h - sw_.h) * K<R>::inv_2s3;
      const R qxE = se_.h * se_.u, qxW = sw_.h * sw_.u, qyE = se_.h * se_.v, qyW = sw_.h * sw_.v;
      const R qb0 = R(0.5) * (qxE + qxW), qb1 = (qxE - qxW) * K<R>::inv_2s3;
      const R rb0 = R(0.5) * (qyE + qyW), rb1 = (qyE - qyW) * K<R>::inv_2s3;
      const R zb1 = (se_.z - sw_.z) * K<R>::inv_2s3;
      R Fp[3], Fm[3];
      gauss_flux(g, ht, hb0 + hb1, qb0 + qb1, rb0 + rb1, Fp);
      gauss_flux(g, ht, hb0 - hb1, qb0 - qb1, rb0 - rb1, Fm);
      L[0] = -(fe[0] - fw[0]) * idx;
      L[3] = -(fe[1] - fw[1]) * idx - k2s3 * hb0 * zb1;
      L[6] = -(fe[2] - fw[2]) * idx;
      const R c = -s3 * idx;
      L[1] = c * (fe[0] + fw[0] - Fp[0] - Fm[0]);
      L[4] = c * (fe[1] + fw[1] - Fp[1] - Fm[1]) - k2s3 * hb1 * zb1;
      L[7] = c * (fe[2] + fw[2] - Fp[2] - Fm[2]);
    }
    {  // y direction
      const R hb0 = R(0.5) * (sn_.h + ss_.h), hb1 = (sn_.h - ss_.h) * K<R>::inv_2s3;
      const R qxN = sn_.h * sn_.u, qxS = ss_.h * ss_.u, qyN = sn_.h * sn_.v, qyS = ss_.h * ss_.v;
      const R qb0 = R(0.5) * (qxN + qxS), qb1 = (qxN - qxS) * K<R>::inv_2s3;
      const R rb0 = R(0.5) * (qyN + qyS), rb1 = (qyN - qyS) * K<R>::inv_2s3;
      const R zb1 = (sn_.z - ss_.z) * K<R>::inv_2s3;
      R Gp[3], Gm[3];  // [mass, y-mom (normal), x-mom (tangential)]
      gauss_flux(g, ht, hb0 + hb1, rb0 + rb1, qb0 + qb1, Gp);
      gauss_flux(g, ht, hb0 - hb1, rb0 - rb1, qb0 - qb1, Gm);
      L[0] += -(fn[0] - fs[0]) * idx;
      L[3] += -(fn[1] - fs[1]) * idx;
      L[6] += -(fn[2] - fs[2]) * idx - k2s3 * hb0 * zb1;
      const R c = -s3 * idx;
      L[2] = c * (fn[0] + fs[0] - Gp[0] - Gm[0]);
      L[5] = c * (fn[1] + fs[1] - Gp[2] - Gm[2]);
      L[8] = c * (fn[2] + fs[2] - Gp[1] - Gm[1]) - k2s3 * hb1 * zb1;
    }
    R u[9];
    if (STAGE == 1) {
#pragma unroll
      for (int q = 0; q < 9; ++q) u[q] = va[q] + dtr * L[q];
    } else {
#pragma unroll
      for (int q = 0; q < 9; ++q) u[q] = R(0.5) * (p.vbuf[q * n + ck] + va[q] + dtr * L[q]);
    }
    // after each stage: clip a negative mean depth (booking the mass), then drop the
    // discharge of cells at or below the dry tolerance
    if (u[0] < R(0)) {
      led_clip += -double(u[0]) * p.dxd * p.dxd * (STAGE == 1 ? 0.5 : 1.0);
      u[0] = u[1] = u[2] = R(0);
    }
    if (!(u[0] > ht)) u[3] = u[4] = u[5] = u[6] = u[7] = u[8] = R(0);
    bool bad = false;
#pragma unroll
    for (int q = 0; q < 9; ++q) bad |= (u[q] != u[q]);
    if (bad) atomicOr(&p.ctrl->health, 1);
    if (STAGE == 1) {
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        p.vbuf[q * n + ck] = va[q];
        p.ui[q * n + ck] = u[q];
      }
    } else {
#pragma unroll
      for (int q = 0; q < 9; ++q) p.vbuf[q * n + ck] = u[q];
      my_dtc = cell_dtc(p, u[0], u[1], u[2], u[3], u[6]);
    }
  }

  // per-block reductions in a fixed order (deterministic)
  const int lane = tid & 63, wv = tid >> 6;
  double r_in = wave_sum(led_in), r_out = wave_sum(led_out), r_clip = wave_sum(led_clip);
  double r_dt = 0.0;
  if (STAGE == 2) r_dt = wave_min(my_dtc);
  if (lane == 0) {
    s_red[wv][0] = r_in;
    s_red[wv][1] = r_out;
    s_red[wv][2] = r_clip;
    s_red[wv][3] = r_dt;
  }
  __syncthreads();
  if (tid == 0) {
    double a = 0, bsum = 0, c = 0, m = __longlong_as_double((long long)INF_BITS);
    for (int w = 0; w < NT / 64; ++w) {
      a += s_red[w][0];
      bsum += s_red[w][1];
      c += s_red[w][2];
      if (STAGE == 2) m = s_red[w][3] < m ? s_red[w][3] : m;
    }
    if (a != 0.0 || bsum != 0.0 || c != 0.0) {
      double* led = p.ledger + 4 * (long long)tile;
      led[0] += a;
      led[1] += bsum;
      led[2] += c;
    }
    if (STAGE == 2) {
      if (tile == 0) {
        const double fm = forcing_dtc(p, t_next);
        m = fm < m ? fm : m;
      }
      if (m != __longlong_as_double((long long)INF_BITS))
        atomicMin(&p.ctrl->dtc[1 - p.parity], (unsigned long long)__double_as_longlong(m));
    }
  }
}

// ---------------------------------------------------------------------------------
// set-up and diagnostics kernels
// ---------------------------------------------------------------------------------
template <typename R>
__global__ void convert_kernel(const double* __restrict__ src, R* __restrict__ dst, long long count) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < count) dst[k] = R(src[k]);
}

// initial coefficients (Sect. 2.1.4) from the staged double input
template <typename R>
__global__ void init_kernel(Params<R> p, const double* __restrict__ src, int mode, double eta) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= p.n) return;
  const int i = int(k % p.nx), j = int(k / p.nx);
  const long long n = p.n;
  R c[9];
  for (int q = 0; q < 9; ++q) c[q] = R(0);
  if (mode == 0) {
    for (int q = 0; q < 9; ++q) c[q] = R(src[q * n + k]);
  } else if (mode == 1) {
    c[0] = R(src[k]);
    c[3] = R(src[n + k]);
    c[6] = R(src[2 * n + k]);
  } else if (mode == 2) {
    const long long nv = (long long)(p.nx + 1) * (p.ny + 1);
    for (int var = 0; var < 3; ++var) {
      const double* r = src + var * nv;
      const long long w = p.nx + 1;
      const R sw = R(r[j * w + i]), se = R(r[j * w + i + 1]);
      const R nw = R(r[(j + 1) * w + i]), ne = R(r[(j + 1) * w + i + 1]);
      c[3 * var] = R(0.25) * ((ne + sw) + (nw + se));
      c[3 * var + 1] = (R(0.5) * (ne + se) - R(0.5) * (nw + sw)) * K<R>::inv_2s3;
      c[3 * var + 2] = (R(0.5) * (nw + ne) - R(0.5) * (sw + se)) * K<R>::inv_2s3;
    }
  } else {
    R z0, z1x, z1y;
    bed(p, i, j, z0, z1x, z1y);
    const R h0 = R(eta) - z0;
    if (h0 > R(0)) {
      c[0] = h0;
      c[1] = -z1x;
      c[2] = -z1y;
    }
  }
  if (!(c[0] > p.h_tol))
    for (int q = 3; q < 9; ++q) c[q] = R(0);
  for (int q = 0; q < 9; ++q) p.vbuf[q * n + k] = c[q];
}

// CFL candidate of a whole state (set-up and resume): grid-stride min, one atomic per
// block, plus the forcing at time t from block 0
template <typename R>
__global__ void dtc_kernel(Params<R> p, const R* __restrict__ u, double t, int slot) {
  double m = __longlong_as_double((long long)INF_BITS);
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < p.n;
       k += (long long)gridDim.x * blockDim.x) {
    const double d = cell_dtc(p, u[k], u[p.n + k], u[2 * p.n + k], u[3 * p.n + k], u[6 * p.n + k]);
    m = d < m ? d : m;
  }
  m = wave_min(m);
  __shared__ double red[16];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = red[w] < m ? red[w] : m;
    m = red[0] < m ? red[0] : m;
    if (blockIdx.x == 0) {
      const double fm = forcing_dtc(p, t);
      m = fm < m ? fm : m;
    }
    if (m != __longlong_as_double((long long)INF_BITS))
      atomicMin(&p.ctrl->dtc[slot], (unsigned long long)__double_as_longlong(m));
  }
}

// mass and ledger totals in a fixed order (one block of 1024 threads)
template <typename R>
__global__ __launch_bounds__(1024) void totals_kernel(const R* __restrict__ h0, long long n,
                                                      const double* __restrict__ ledger,
                                                      int n_tiles, double area, double* out) {
  __shared__ double red[4][1024];
  double s[4] = {0, 0, 0, 0};
  for (long long k = threadIdx.x; k < n; k += 1024) s[0] += double(h0[k]);
  for (int k = threadIdx.x; k < n_tiles; k += 1024) {
    s[1] += ledger[4 * k];
    s[2] += ledger[4 * k + 1];
    s[3] += ledger[4 * k + 2];
  }
  for (int q = 0; q < 4; ++q) red[q][threadIdx.x] = s[q];
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int q = 0; q < 4; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = red[0][0] * area;
    out[1] = red[1][0];
    out[2] = red[2][0];
    out[3] = red[3][0];
  }
}

// derived fields: 9 eta0, 10 u0, 11 v0
template <typename R>
__global__ void field_kernel(Params<R> p, const R* __restrict__ u, int field, R* __restrict__ out) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= p.n) return;
  const R h0 = u[k];
  if (field == 9) {
    R z0, z1x, z1y;
    bed(p, int(k % p.nx), int(k / p.nx), z0, z1x, z1y);
    out[k] = h0 + z0;
  } else {
    const R q = u[(field == 10 ? 3 : 6) * p.n + k];
    out[k] = h0 > p.h_tol ? q / h0 : R(0);
  }
}

}  // namespace dg2k
