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

// Tile shapes (cells; x fastest in memory). A context picks one of the shapes listed
// per precision; index 0 is the default. One block of TX * TY threads owns a tile.
// B1 / B2: the blocks per CU that the stage-1 / stage-2 kernel is compiled to fit
// (a register budget: 4 blocks of 4 waves leave 128 VGPRs per lane).
template <int TX_, int TY_, int B1_ = 1, int B2_ = 1>
struct Shape {
  static constexpr int X = TX_, Y = TY_, B1 = B1_, B2 = B2_;
};
constexpr int N_SHAPES = 4;
// FP64: 16x16 (default), 32x8, 16x8, 64x4; FP32: 64x8 (default), 32x16, 32x8, 16x16;
// columns: TX, TY, B1, B2
constexpr int SHAPE64[N_SHAPES][4] = {{16, 16, 4, 4}, {32, 8, 4, 4}, {16, 8, 1, 1}, {64, 4, 1, 1}};
constexpr int SHAPE32[N_SHAPES][4] = {{64, 8, 1, 1}, {32, 16, 1, 1}, {32, 8, 1, 1}, {16, 16, 1, 1}};

// LDS geometry of a tile: the cell box has a 2-cell halo, the vertex box one more
template <typename S>
struct Geo {
  static constexpr int TX = S::X, TY = S::Y;
  static constexpr int NT = TX * TY;           // threads per block, one cell each
  static constexpr int RX = TX + 4, RY = TY + 4, RB = RX * RY;
  static constexpr int VX = TX + 5, VY = TY + 5, VB = VX * VY;
  static constexpr int NRING = 2 * (TX + TY);  // non-corner cells of the first halo ring
  static_assert(NT % 64 == 0 && NT <= 1024 && NRING <= NT,
                "tile must give whole waves and one ring cell per thread at most");
};
constexpr int NXCD = 8;

constexpr unsigned long long INF_BITS = 0x7FF0000000000000ull;

struct Seg {
  int kind, edge, i0, i1, k0, nk;
  double width, h_b, u_b, v_b;
};

// control block shared by the launches of a context; slot [p] belongs to the step that
// starts from state buffer p
// A CFL candidate (min over cells of dx / (|u| + c), as positive-double bits, which
// order like the values) is kept as NSLOT partial minima, each on its own 128-byte
// line: block b reduces into slot b % NSLOT, so the blocks of a launch do not all
// queue on one address, and a reader takes the min of the slots.
constexpr int NSLOT = 16, SLOT_STRIDE = 16;
struct Cand {
  unsigned long long s[NSLOT * SLOT_STRIDE];
};

struct Ctrl {
  double t[2];
  double dt_used[2];
  long long step[2];
  int health;                 // bit 0: NaN seen, bit 1: time step below 1e-12 s
  int pad;
  alignas(128) Cand dtc[2];   // DG2: the candidate of the state in buffer p
  // FV1 (one launch per step): the candidate of step k lives in dtr[k % 3]; step k
  // reads dtr[k % 3], reduces into dtr[(k + 1) % 3] and clears dtr[(k + 2) % 3], which
  // no block of step k touches and step k - 1 has finished reading
  Cand dtr[3];
};

// the candidate's value: min over its slots (every lane of the wave must take part)
__device__ __forceinline__ double cand_read(const Cand& c);
__device__ __forceinline__ double wave_min(double x);
// post a block's candidate / clear all slots (one thread)
__device__ __forceinline__ void cand_post(Cand& c, int block, double m) {
  atomicMin(&c.s[(block % NSLOT) * SLOT_STRIDE], (unsigned long long)__double_as_longlong(m));
}
__device__ __forceinline__ void cand_clear(Cand& c) {
  for (int k = 0; k < NSLOT; ++k) c.s[k * SLOT_STRIDE] = INF_BITS;
}

template <typename R>
struct Params {
  const R* __restrict__ uin;   // U^n (the stage-1 input; stage 2 reads ui)
  R* vbuf;                     // V^n out (stage 1); V^n in (stage 2)
  R* uout;                     // U^{n+1} out (stage 2): vbuf itself in a plain run, so
                               // neither pointer is restrict
  R* __restrict__ ui;          // U^int out (stage 1)
  const R* __restrict__ zv;    // vertex bed (relative to the owner tile's datum if datum)
  const R* __restrict__ zc;    // FV1: bed mean of each cell (eq 8) in its own tile's frame
  const R* __restrict__ datum; // per tile, whole metres (FP32 with a bed datum), or nullptr
  const R* __restrict__ manning;  // per cell, or nullptr
  const int* __restrict__ bface;  // boundary faces: W[ny], E[ny], S[nx], N[nx]
  const Seg* __restrict__ segs;
  const double* __restrict__ knots;  // t[DG2_MAX_KNOTS] then q[DG2_MAX_KNOTS]
  Ctrl* ctrl;
  double* ledger;              // per tile: in, out, clip, unused
  long long n;                 // nx * ny
  int nx, ny, tx, ty, tiles_x, n_tiles, per_xcd, nsegs, max_knots, limiter, parity, fv1;
  R dx, idx, g, h_tol, n_scalar;  // idx = 1 / dx (rounded once, on the host)
  double dxd, gd, cfl, htd, dt_dry, dt_max, t_end;
  double dt_fix;               // > 0: the step takes exactly this dt (a replayed schedule)
  // a recorded run (FP64 only): stage 2 writes the new mean depth of every gauge cell to
  // gauge_h[g] (gmap: a cell's first gauge or -1; gnext: the next gauge of that cell)
  double* gauge_h;
  const int* gmap;
  const int* gnext;
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

// Reciprocal, square root and h^(-1/3) for the inner loops: the hardware estimates
// (relative errors measured on gfx950: 2^-24.4 for the FP64 reciprocal, 2^-24.2 for
// the FP64 reciprocal square root, 2^-20 for the FP32-seeded cube root) refined to full
// FP64 precision (within a few ulp, not correctly rounded); FP32 uses the 1-ulp
// hardware results.
// 1/d: with e = 1 - d r, 1/d = r / (1 - e) = r (1 + e + e^2 + ...); one third-order
// step leaves an error of order e^3, far below an ulp
__device__ __forceinline__ double frcp(double d) {
  const double r = __builtin_amdgcn_rcp(d);
  const double e = __builtin_fma(-d, r, 1.0);
  return __builtin_fma(r, __builtin_fma(e, e, e), r);
}
__device__ __forceinline__ float frcp(float d) { return __builtin_amdgcn_rcpf(d); }

__device__ __forceinline__ double fsqrt(double x) {
  if (!(x > 0.0)) return 0.0;
  double y = __builtin_amdgcn_rsq(x);
  double h = 0.5 * y;
  double s = x * y;                       // sqrt estimate
  double r = __builtin_fma(-s, h, 0.5);   // Goldschmidt refinement
  s = __builtin_fma(s, r, s);
  h = __builtin_fma(h, r, h);
  r = __builtin_fma(-s, s, x);
  return __builtin_fma(r, h, s);
}
__device__ __forceinline__ float fsqrt(float x) { return x > 0.0f ? __builtin_amdgcn_sqrtf(x) : 0.0f; }

// 1/sqrt(x) for x > 0: with e = 1 - x y^2, x^(-1/2) = y (1 - e)^(-1/2)
// = y (1 + e/2 + 3e^2/8 + ...); one third-order step from the hardware estimate
__device__ __forceinline__ double frsq(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double e = __builtin_fma(-x * y, y, 1.0);
  return __builtin_fma(y * e, __builtin_fma(e, 0.375, 0.5), y);
}
__device__ __forceinline__ float frsq(float x) { return __builtin_amdgcn_rsqf(x); }

// y = h^(-1/3) for h > 0: a float log2/exp2 seed, then with e = 1 - h y^3,
// h^(-1/3) = y (1 - e)^(-1/3) = y (1 + e/3 + 2e^2/9 + ...); one third-order step
__device__ __forceinline__ double finvcbrt(double h) {
  if (!(h >= 1e-30)) return 1.0 / cbrt(h);
  const float hf = float(h);
  const double y = double(__builtin_amdgcn_exp2f(-0.333333343f * __builtin_amdgcn_logf(hf)));
  const double e = __builtin_fma(-h, y * y * y, 1.0);
  return __builtin_fma(y * e, __builtin_fma(e, 0.22222222222222222222, 0.33333333333333333333), y);
}
__device__ __forceinline__ float finvcbrt(float h) {
  if (!(h >= 1e-30f)) return 1.0f / cbrtf(h);
  float y = __builtin_amdgcn_exp2f(-0.333333343f * __builtin_amdgcn_logf(h));
  return y * (4.0f - h * (y * y * y)) * 0.333333343f;
}
__device__ __forceinline__ double dcbrt(double x) { return cbrt(x); }
__device__ __forceinline__ float dcbrt(float x) { return cbrtf(x); }
__device__ __forceinline__ double dabs(double x) { return __builtin_fabs(x); }
__device__ __forceinline__ float dabs(float x) { return __builtin_fabsf(x); }

// the larger of x and 0 / the smaller of two values, as single min/max instructions
template <typename R> __device__ __forceinline__ R fmax0(R x) { return __builtin_fmax(x, R(0)); }
__device__ __forceinline__ float fmax0(float x) { return __builtin_fmaxf(x, 0.0f); }
__device__ __forceinline__ double fminr(double a, double b) { return __builtin_fmin(a, b); }
__device__ __forceinline__ float fminr(float a, float b) { return __builtin_fminf(a, b); }
__device__ __forceinline__ double fmaxr(double a, double b) { return __builtin_fmax(a, b); }
__device__ __forceinline__ float fmaxr(float a, float b) { return __builtin_fmaxf(a, b); }

// a positive floor for reciprocals whose result is discarded when the argument is not
// positive (keeps the arithmetic finite without a branch)
template <typename R> struct Tiny;
template <> struct Tiny<double> { static constexpr double v = 1e-300; };
template <> struct Tiny<float> { static constexpr float v = 1e-30f; };

// minmod of three: the smallest magnitude if all three share a sign, else 0, as
// max(min(a,b,c),0) + min(max(a,b,c),0) (one term is always zero; the sum is exact)
template <typename R>
__device__ __forceinline__ R minmod3(R a, R b, R c) {
  const R lo = fminr(a, fminr(b, c)), hi = fmaxr(a, fmaxr(b, c));
  return fmaxr(lo, R(0)) + fminr(hi, R(0));
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

// a value that is the same in every lane, kept in scalar registers
__device__ __forceinline__ double uniform(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readfirstlane((int)b), hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ long long uniform(long long x) {
  const int lo = __builtin_amdgcn_readfirstlane((int)x), hi = __builtin_amdgcn_readfirstlane((int)(x >> 32));
  return ((long long)hi << 32) | (unsigned)lo;
}

// the step's time step, identical in every block of both stage launches, in two parts
// so that a kernel can put its own loads between them: the loads (the step's start
// time; lane k < NSLOT one CFL slot), then the arithmetic
// s_waitcnt operand for gfx9-family encodings: vmcnt 0 (bits 3:0 and 15:14), expcnt and
// lgkmcnt left at their maxima (no wait on them)
constexpr int kWaitVmem = 0x0F70;

struct StepLoads {
  double t, slot;
};
template <typename R>
__device__ __forceinline__ StepLoads step_loads(const Params<R>& p) {
  const int lane = threadIdx.x & 63;
  const Cand& c = p.ctrl->dtc[p.parity];
  return StepLoads{p.ctrl->t[p.parity], lane < NSLOT ? __longlong_as_double((long long)c.s[lane * SLOT_STRIDE])
                                                      : __longlong_as_double((long long)INF_BITS)};
}
template <typename R>
__device__ __forceinline__ void step_time(const Params<R>& p, const StepLoads& l, double& t, double& dt,
                                          double& t_next, double& dt_cfl) {
  t = uniform(l.t);
  const double m = wave_min(l.slot);
  double d = (m == __longlong_as_double((long long)INF_BITS)) ? p.dt_dry : p.cfl * m;
  dt_cfl = d;
  if (p.dt_fix > 0.0) {
    dt = p.dt_fix;
    t_next = t + dt;
    return;
  }
  if (p.dt_max > 0.0 && p.dt_max < d) d = p.dt_max;
  t_next = t + d;
  if (p.t_end - t <= d) {
    d = p.t_end - t;
    t_next = p.t_end;
  }
  dt = d;
}

// a face side after the wet/dry revision: depth, velocities, and the revised bed
// z** = z + m (FP64: z = z**, m = 0; FP32: z = z*, m = min(h + zb - z*, 0))
template <typename R>
struct Side {
  R h, u, v, z, m;
};

// revision of one side's limit (h, qx, qy) with this side's bed zb and the face's
// z* = zs: h* = max(0, eta - z*), velocities from the unrevised depth (zero at or
// below h_tol), z** = min(z*, eta). FP32 forms the same quantities from the bed
// difference zb - z* (exact there), never from an absolute eta, so that they do not
// depend on the elevation datum.
template <typename R>
__device__ __forceinline__ Side<R> revise(R h, R qx, R qy, R zb, R zs, R ht) {
  Side<R> s;
  if constexpr (sizeof(R) == 8) {
    const R eta = h + zb;
    s.h = fmax0(eta - zs);
    s.z = fminr(eta, zs);
    s.m = R(0);
  } else {
    const R d = h + (zb - zs);
    s.h = fmax0(d);
    s.z = zs;
    s.m = fminr(d, R(0));
  }
  const bool wet = h > ht;
  const R r = frcp(fmaxr(h, Tiny<R>::v));
  s.u = wet ? qx * r : R(0);
  s.v = wet ? qy * r : R(0);
  return s;
}

// HLL flux through a face, normal frame: (h, un, ut) on each side ->
// [mass, normal momentum, tangential momentum]; wave speeds of the two-rarefaction
// estimate, the dry-bed front speeds where a side is exactly dry
template <typename R>
__device__ __forceinline__ void hll(R g, R hL, R unL, R utL, R hR, R unR, R utR, R f[3]) {
  const bool wL = hL > R(0), wR = hR > R(0);
  const R cL = fsqrt(g * hL), cR = fsqrt(g * hR);
  const R us = R(0.5) * (unL + unR) + cL - cR;
  const R cs = R(0.5) * (cL + cR) + R(0.25) * (unL - unR);
  const R sLw = fminr(unL - cL, us - cs), sRw = fmaxr(unR + cR, us + cs);
  const R sL = wL ? (wR ? sLw : unL - cL) : unR - R(2) * cR;
  const R sR = wL ? (wR ? sRw : unL + R(2) * cL) : unR + cR;
  const R qL = hL * unL, qR = hR * unR;
  const R FL0 = qL, FL1 = qL * unL + R(0.5) * g * hL * hL, FL2 = qL * utL;
  const R FR0 = qR, FR1 = qR * unR + R(0.5) * g * hR * hR, FR2 = qR * utR;
  const R inv = frcp(fmaxr(sR - sL, Tiny<R>::v));
  const R ss = sL * sR;
  const R S0 = (sR * FL0 - sL * FR0 + ss * (hR - hL)) * inv;
  const R S1 = (sR * FL1 - sL * FR1 + ss * (qR - qL)) * inv;
  const R S2 = (sR * FL2 - sL * FR2 + ss * (hR * utR - hL * utL)) * inv;
  const bool up = sL >= R(0), dn = sR <= R(0), dry = !wL && !wR;
  f[0] = dry ? R(0) : (up ? FL0 : (dn ? FR0 : S0));
  f[1] = dry ? R(0) : (up ? FL1 : (dn ? FR1 : S1));
  f[2] = dry ? R(0) : (up ? FL2 : (dn ? FR2 : S2));
}

// physical flux of a state (h, un, ut) through a face with normal n:
// [h un, h un^2 + g h^2 / 2, h un ut]; an inflow face carries its inflow state's own
// flux (instead of HLL with the interior side), so the segment lets in exactly Q(t)
template <typename R>
__device__ __forceinline__ void phys_flux(R g, R h, R un, R ut, R f[3]) {
  const R q = h * un;
  f[0] = q;
  f[1] = q * un + R(0.5) * g * h * h;
  f[2] = q * ut;
}

// physical flux along a normal at a Gauss point, velocities zero at or below h_tol
template <typename R>
__device__ __forceinline__ void gauss_flux(R g, R ht, R h, R qn, R qt, R f[3]) {
  const bool wet = h > ht;
  const R r = frcp(fmaxr(h, Tiny<R>::v));
  const R un = wet ? qn * r : R(0), ut = wet ? qt * r : R(0);
  const R q = h * un;
  f[0] = q;
  f[1] = q * un + R(0.5) * g * h * h;
  f[2] = q * ut;
}

// Split-implicit Manning increment at one point: with w = dt g n^2 h^(-4/3) and
// s = |u|, the Newton step of backward Euler with the diagonal Jacobian gives
// dqx = -qx w s / (1 + w (2u^2 + v^2) / s), and likewise for qy. Zero where h <= h_tol
// or the water is still.
template <typename R>
__device__ __forceinline__ void friction_inc(R gn2dt, R ht, R h, R qx, R qy, R& dqx, R& dqy) {
  const bool wet = h > ht;
  const R y = finvcbrt(wet ? h : R(1));  // h^(-1/3)
  const R y3 = y * y * y;                // 1/h
  const R u = qx * y3, v = qy * y3;
  const R s2 = u * u + v * v;
  const bool act = wet && s2 > R(0);
  const R rs = frsq(fmaxr(s2, Tiny<R>::v));  // 1/|u|
  const R m = gn2dt * (y3 * y) * rs;     // dt g n^2 h^(-4/3) / |u|
  const R a = m * (u * u), b = m * (v * v);
  const R ab = a + b;                    // dt g n^2 h^(-4/3) |u|
  const R d1 = (R(1) + a) + ab, d2 = (R(1) + b) + ab;
  const R P = ab * frcp(d1 * d2);
  dqx = act ? -qx * d2 * P : R(0);
  dqy = act ? -qy * d1 * P : R(0);
}

// datum of the tile holding cell (i, j) (0 without a datum)
template <typename R>
__device__ __forceinline__ R tile_datum(const Params<R>& p, int i, int j) {
  if constexpr (sizeof(R) == 8) return R(0);  // FP64 stores absolute elevations
  return p.datum ? p.datum[(j / p.ty) * p.tiles_x + i / p.tx] : R(0);
}

// bed at vertex (iv, jv) in the frame of datum dT: the stored value is relative to the
// datum of the tile owning the vertex (the tile of cell (min(iv, nx-1), min(jv, ny-1)));
// datums are whole metres and the stored bed is quantised, so the shift is exact
template <typename R>
__device__ __forceinline__ R zvat(const Params<R>& p, int iv, int jv, R dT) {
  R z = p.zv[(long long)jv * (p.nx + 1) + iv];
  if (sizeof(R) == 4 && p.datum) {
    const int oi = iv < p.nx ? iv : p.nx - 1, oj = jv < p.ny ? jv : p.ny - 1;
    z += tile_datum(p, oi, oj) - dT;
  }
  return z;
}

// bed mean and slopes of cell (i, j) (eq 8; mean summed in diagonal pairs), in the frame
// of the cell's tile datum
template <typename R>
__device__ __forceinline__ void bed(const Params<R>& p, int i, int j, R& z0, R& z1x, R& z1y) {
  const R dT = tile_datum(p, i, j);
  const R sw = zvat(p, i, j, dT), se = zvat(p, i + 1, j, dT);
  const R nw = zvat(p, i, j + 1, dT), ne = zvat(p, i + 1, j + 1, dT);
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
__device__ __forceinline__ R cell_dtc_r(const Params<R>& p, R h0, R h1x, R h1y, R qx0, R qy0) {
  const R r = frcp(fmaxr(h0, Tiny<R>::v));
  const R u = qx0 * r, v = qy0 * r;
  const R a = p.dx * frcp(dabs(u) + fsqrt(p.g * (h0 + K<R>::s3 * dabs(h1x))));
  const R b = p.dx * frcp(dabs(v) + fsqrt(p.g * (h0 + K<R>::s3 * dabs(h1y))));
  return h0 > p.h_tol ? fminr(a, b) : R(__builtin_huge_val());
}
// the same as a double (the widening is exact and keeps the order, so a minimum taken in
// R and widened once equals the minimum of the widened candidates)
template <typename R>
__device__ __forceinline__ double cell_dtc(const Params<R>& p, R h0, R h1x, R h1y, R qx0, R qy0) {
  return double(cell_dtc_r(p, h0, h1x, h1y, qx0, qy0));
}

// magnitude cap of a face-limit velocity component: the larger neighbouring mean
// velocity magnitude plus the velocity scale of the dry tolerance
template <typename R>
__device__ __forceinline__ R vcap(R x, R a, R b, R slack) {
  const R m = fmaxr(dabs(a), dabs(b)) + slack;
  return fminr(fmaxr(x, -m), m);
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

// Wave-wide sum / min of a double, the same value in every lane, in a fixed order:
// an xor butterfly over the 32-lane halves by ds_swizzle (the lane pattern is an
// immediate, so no lane-address registers are held), then the two halves combined.
template <int XOR>
__device__ __forceinline__ double swizzle_xor(double x) {
  constexpr int pattern = (XOR << 10) | 0x1F;  // bit mode: and 0x1F, or 0, xor XOR
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_ds_swizzle((int)b, pattern);
  const int hi = __builtin_amdgcn_ds_swizzle((int)(b >> 32), pattern);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double lane_value(double x, int lane) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)b, lane), hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double wave_sum(double x) {
  x += swizzle_xor<1>(x);
  x += swizzle_xor<2>(x);
  x += swizzle_xor<4>(x);
  x += swizzle_xor<8>(x);
  x += swizzle_xor<16>(x);
  return lane_value(x, 0) + lane_value(x, 32);
}
// the same, skipped when every lane holds zero (the sum is then exactly zero): the
// ledger's clipped-mass and boundary terms are zero in most waves, and the swizzle chain
// is five dependent LDS round trips
__device__ __forceinline__ double wave_sum_sparse(double x) {
  return __builtin_amdgcn_ballot_w64(x != 0.0) ? wave_sum(x) : 0.0;
}
__device__ __forceinline__ double dmin2(double a, double b) { return b < a ? b : a; }
__device__ __forceinline__ double wave_min(double x) {
  x = dmin2(x, swizzle_xor<1>(x));
  x = dmin2(x, swizzle_xor<2>(x));
  x = dmin2(x, swizzle_xor<4>(x));
  x = dmin2(x, swizzle_xor<8>(x));
  x = dmin2(x, swizzle_xor<16>(x));
  return dmin2(lane_value(x, 0), lane_value(x, 32));
}
// FP32 kernels take their CFL minimum in float: one swizzle per step instead of two
template <int XOR>
__device__ __forceinline__ float swizzle_xor(float x) {
  constexpr int pattern = (XOR << 10) | 0x1F;
  return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(x), pattern));
}
__device__ __forceinline__ float fmin2(float a, float b) { return b < a ? b : a; }
__device__ __forceinline__ float wave_min(float x) {
  x = fmin2(x, swizzle_xor<1>(x));
  x = fmin2(x, swizzle_xor<2>(x));
  x = fmin2(x, swizzle_xor<4>(x));
  x = fmin2(x, swizzle_xor<8>(x));
  x = fmin2(x, swizzle_xor<16>(x));
  return fmin2(__int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 0)),
               __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 32)));
}

// lane k < NSLOT reads slot k (one memory round trip for all of them) and the wave
// takes the minimum with the swizzle reduction, which holds no lane-address registers
__device__ __forceinline__ double cand_read(const Cand& c) {
  const int lane = threadIdx.x & 63;
  const double v = lane < NSLOT ? __longlong_as_double((long long)c.s[lane * SLOT_STRIDE])
                                : __longlong_as_double((long long)INF_BITS);
  return wave_min(v);
}

// ---------------------------------------------------------------------------------
// the stage kernel
// ---------------------------------------------------------------------------------
template <typename R, typename S>
struct Smem {
  static constexpr int TX = Geo<S>::TX, TY = Geo<S>::TY;
  static constexpr int NFX = (TX + 1) * TY, NFY = TX * (TY + 1);  // x / y faces of the tile
  R c[6][Geo<S>::RB];   // planes 0-2: box means h0, qx0, qy0; later the face-side states
  union {
    struct {
      R zv[Geo<S>::VB];  // bed vertices of the box
      R z0[Geo<S>::RB];  // bed means of the box cells
      R um[Geo<S>::RB];  // mean velocities (zero at or below h_tol)
      R vm[Geo<S>::RB];
    };
    struct {             // once the face sides are formed: the tile's face fluxes
      R fx[3][NFX];      // x face f of tile row b at b * (TX + 1) + f
      R fy[3][NFY];      // y face f of tile column a at f * TX + a
    };
  };
  unsigned char flag[Geo<S>::RB];  // 1: first-order (front) cell
  double red[Geo<S>::NT / 64][4];
};

// One stage over one tile. EDGE is false for tiles whose halo box lies inside the
// domain: no clamping, no boundary faces, every cell active.
template <typename R, typename S, int STAGE, bool EDGE>
__device__ __forceinline__ void stage_body(const Params<R>& p, Smem<R, S>& sm, const int tile,
                                           const int i0, const int j0) {
  constexpr int TX = Geo<S>::TX, TY = Geo<S>::TY, NT = Geo<S>::NT;
  constexpr int RX = Geo<S>::RX, RB = Geo<S>::RB, VX = Geo<S>::VX, VB = Geo<S>::VB;
  constexpr int NRING = Geo<S>::NRING;
  const int tid = threadIdx.x;
  const int nx = p.nx, ny = p.ny;
  const long long n = p.n;
  const R ht = p.h_tol;
  const R s3 = K<R>::s3;

  const int ci = i0 + tid % TX, cj = j0 + tid / TX;
  const bool active = !EDGE || (ci < nx && cj < ny);
  // unsigned: a cell past the grid's last row (inactive) may lie beyond INT_MAX
  const unsigned ck = (unsigned)cj * (unsigned)nx + (unsigned)ci;

  // stage 2 needs V^n of the own cell only at the end; FP32 has the registers to
  // issue its loads now
  constexpr bool kPrefetch = sizeof(R) == 4;
  R vn[9];
  if (STAGE == 2 && kPrefetch && active) {
#pragma unroll
    for (int q = 0; q < 9; ++q) vn[q] = (p.vbuf + q * n)[ck];
  }

  // ---- phase 1: the box (friction applied in stage 1) and its bed vertices ----
  // Every global load of this phase is issued before any is waited on: the bed vertices
  // (VITER per thread), the own cell and the thread's first halo item. Issued one after
  // the other, they cost a memory round trip each.
  const R dT = (sizeof(R) == 4 && p.datum) ? p.datum[tile] : R(0);
  const R* __restrict__ src = STAGE == 1 ? p.uin : p.ui;
  // FP32: the wave issues its phase-1 loads at raised priority (measured 1.8 % faster
  // for both FP32 stages; no gain for FP64)
  if constexpr (sizeof(R) == 4) __builtin_amdgcn_s_setprio(3);
  const StepLoads sl = step_loads(p);  // in flight with the tile's loads below
  double t, dt, t_next, dt_cfl;        // the step's times, formed once those are issued
  R dtr;
  constexpr int VITER = (VB + NT - 1) / NT;
  constexpr int NHALO = 2 * NRING + 4;  // halo items: first ring, second ring, corners
  // vertex (iv, jv) sits at box position (iv - i0 + 2, jv - j0 + 2); a clamped halo
  // cell only uses vertices of in-domain cells, which lie in the box
  // (FP32 with datums: the owner tile's datum is loaded beside the vertex and the shift
  // to this tile's frame is applied only when the vertex goes to LDS, so that no load of
  // the phase waits for another)
  R zl[VITER], zd[VITER];
#pragma unroll
  for (int k = 0; k < VITER; ++k) {
    const int r = tid + k * NT;
    zl[k] = R(0);
    zd[k] = dT;
    if (r < VB) {
      int iv = i0 - 2 + r % VX, jv = j0 - 2 + r / VX;
      if (EDGE) {
        iv = iv < 0 ? 0 : (iv > nx ? nx : iv);
        jv = jv < 0 ? 0 : (jv > ny ? ny : jv);
      }
      // unsigned: a grid of 2^31 cells has more than INT_MAX vertices
      zl[k] = p.zv[(unsigned)jv * (unsigned)(nx + 1) + (unsigned)iv];
      if (sizeof(R) == 4 && p.datum) {  // 32-bit unsigned index arithmetic (oi, oj >= 0)
        const unsigned oi = iv < nx ? iv : nx - 1, oj = jv < ny ? jv : ny - 1;
        zd[k] = p.datum[(oj / TY) * (unsigned)p.tiles_x + oi / TX];
      }
    }
  }
  auto zb = [&](int iv, int jv) -> R { return sm.zv[(jv - j0 + 2) * VX + (iv - i0 + 2)]; };
  // cell index of box position (a, bb), clamped to the domain
  auto cell_of = [&](int a, int bb) -> unsigned {
    int i = i0 - 2 + a, j = j0 - 2 + bb;
    if (EDGE) {
      i = i < 0 ? 0 : (i >= nx ? nx - 1 : i);
      j = j < 0 ? 0 : (j >= ny ? ny - 1 : j);
    }
    return (unsigned)j * (unsigned)nx + (unsigned)i;
  };
  // halo item h: its box position and friction points (npair: 0 centre only, 1 one
  // Gauss pair whose slopes are picked by xdir, -1 none)
  auto halo_item = [&](int h, int& a, int& bb, int& np, bool& xd) {
    if (h < NRING) {  // same numbering as the ring items below
      if (h < TY) { a = 1; bb = h + 2; xd = true; }
      else if (h < 2 * TY) { a = TX + 2; bb = h - TY + 2; xd = true; }
      else if (h < 2 * TY + TX) { a = h - 2 * TY + 2; bb = 1; xd = false; }
      else { a = h - 2 * TY - TX + 2; bb = TY + 2; xd = false; }
      np = 1;
    } else if (h < 2 * NRING) {
      const int m = h - NRING;
      if (m < TY) { a = 0; bb = m + 2; }
      else if (m < 2 * TY) { a = TX + 3; bb = m - TY + 2; }
      else if (m < 2 * TY + TX) { a = m - 2 * TY + 2; bb = 0; }
      else { a = m - 2 * TY - TX + 2; bb = TY + 3; }
      np = 0;
      xd = true;
    } else {
      const int m = h - 2 * NRING;
      a = (m & 1) ? TX + 2 : 1;
      bb = (m & 2) ? TY + 2 : 1;
      np = -1;
      xd = true;
    }
  };
  auto load_raw = [&](unsigned k, R c[9], R& nm) {
#pragma unroll
    for (int q = 0; q < 9; ++q) c[q] = (src + q * n)[k];
    nm = (STAGE == 1) ? (p.manning ? p.manning[k] : p.n_scalar) : R(0);
  };
  // apply friction in stage 1 (npair as above; 2: both pairs) and publish box cell (a, bb)
  auto publish = [&](int a, int bb, int npair, bool xdir, R c[9], R nm) {
    const int r = bb * RX + a;
    if (STAGE == 1 && npair >= 0 && nm > R(0)) {
      const R gn2dt = p.g * nm * nm * dtr;
      R dx0, dy0;
      friction_inc(gn2dt, ht, c[0], c[3], c[6], dx0, dy0);
      if (npair == 2) {
#pragma unroll
        for (int d = 1; d <= 2; ++d) {
          R dxp, dyp, dxm, dym;
          friction_inc(gn2dt, ht, c[0] + c[d], c[3] + c[3 + d], c[6] + c[6 + d], dxp, dyp);
          friction_inc(gn2dt, ht, c[0] - c[d], c[3] - c[3 + d], c[6] - c[6 + d], dxm, dym);
          c[3 + d] += R(0.5) * (dxp - dxm);
          c[6 + d] += R(0.5) * (dyp - dym);
        }
      } else if (npair == 1) {  // one pair; slopes selected, not indexed
        const R h1 = xdir ? c[1] : c[2], qx1 = xdir ? c[4] : c[5], qy1 = xdir ? c[7] : c[8];
        R dxp, dyp, dxm, dym;
        friction_inc(gn2dt, ht, c[0] + h1, c[3] + qx1, c[6] + qy1, dxp, dyp);
        friction_inc(gn2dt, ht, c[0] - h1, c[3] - qx1, c[6] - qy1, dxm, dym);
        const R ex = R(0.5) * (dxp - dxm), ey = R(0.5) * (dyp - dym);
        c[4] += xdir ? ex : R(0);
        c[5] += xdir ? R(0) : ex;
        c[7] += xdir ? ey : R(0);
        c[8] += xdir ? R(0) : ey;
      }
      c[3] += dx0;
      c[6] += dy0;
    }
    sm.c[0][r] = c[0];  // means only: the slopes stay with the thread that owns the cell
    sm.c[1][r] = c[3];
    sm.c[2][r] = c[6];
    const bool wet = c[0] > ht;
    const R rh = frcp(fmaxr(c[0], Tiny<R>::v));
    sm.um[r] = wet ? c[3] * rh : R(0);
    sm.vm[r] = wet ? c[6] * rh : R(0);
  };
  // the own tile cell (both Gauss pairs, the same path in every lane) and the thread's
  // halo item: the first ring (one pair across the tile edge), the second ring (centre
  // only) or the four first-ring corners (depth only)
  R va[9], vb[9];  // the own cell and the thread's halo item (the ring items below)
  R nma, nmb = R(0);
  load_raw(cell_of(tid % TX + 2, tid / TX + 2), va, nma);
  int ha = 0, hbb = 0, hnp = -1;
  bool hxd = true;
  const bool has_item = tid < NHALO;
  if (has_item) {
    halo_item(tid, ha, hbb, hnp, hxd);
    load_raw(cell_of(ha, hbb), vb, nmb);
  }
  if constexpr (sizeof(R) == 4) __builtin_amdgcn_s_setprio(0);
  // the step's time and time step (the same in every block), read only now, with the
  // tile's loads already in flight
  step_time(p, sl, t, dt, t_next, dt_cfl);
  dtr = R(dt);
  if (!(dt > 0.0)) {  // the run has reached t_end: carry the state over unchanged
    if (STAGE == 1) {
      if (active) {
#pragma unroll
        for (int q = 0; q < 9; ++q) (p.vbuf + q * n)[ck] = va[q];  // U^n as loaded
      }
      if (tile == 0 && tid == 0) {
        Ctrl* c = p.ctrl;
        const int a = p.parity, o = 1 - p.parity;
        c->t[o] = c->t[a];
        c->step[o] = c->step[a];
        for (int q = 0; q < NSLOT; ++q) c->dtc[o].s[q * SLOT_STRIDE] = c->dtc[a].s[q * SLOT_STRIDE];
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
    cand_clear(c->dtc[o]);
    c->dt_used[a] = dt;
    if (dt_cfl < 1e-12) atomicOr(&c->health, 2);
  }
#pragma unroll
  for (int k = 0; k < VITER; ++k)
    if (tid + k * NT < VB) {
      if (sizeof(R) == 4 && p.datum) sm.zv[tid + k * NT] = zl[k] + (zd[k] - dT);  // this tile's frame
      else sm.zv[tid + k * NT] = zl[k];
    }
  publish(tid % TX + 2, tid / TX + 2, 2, true, va, nma);
  if (has_item) publish(ha, hbb, hnp, hxd, vb, nmb);
  for (int h = tid + NT; h < NHALO; h += NT) {  // shapes with more halo items than threads
    int a, bb, np;
    bool xd;
    halo_item(h, a, bb, np, xd);
    R tmp[9], nm;
    load_raw(cell_of(a, bb), tmp, nm);
    publish(a, bb, np, xd, tmp, nm);
  }
  __syncthreads();
  for (int r = tid; r < RB; r += NT) {  // bed means of the box cells (eq 8, diagonal pairs)
    const int iu = i0 - 2 + r % RX, ju = j0 - 2 + r / RX;
    int i = iu, j = ju;
    if (EDGE) {
      i = i < 0 ? 0 : (i >= nx ? nx - 1 : i);
      j = j < 0 ? 0 : (j >= ny ? ny - 1 : j);
    }
    R z = R(0.25) * ((zb(i + 1, j + 1) + zb(i, j)) + (zb(i, j + 1) + zb(i + 1, j)));
    if (EDGE) {  // beyond an edge (the limiter's ghost): the edge cell's bed plane
      if (iu != i) {  // continued one cell out; its depth is the edge cell's (clamped)
        const R dzx = R(0.5) * (zb(i + 1, j + 1) + zb(i + 1, j)) - R(0.5) * (zb(i, j + 1) + zb(i, j));
        z = iu < i ? z - dzx : z + dzx;
      }
      if (ju != j) {
        const R dzy = R(0.5) * (zb(i, j + 1) + zb(i + 1, j + 1)) - R(0.5) * (zb(i, j) + zb(i + 1, j));
        z = ju < j ? z - dzy : z + dzy;
      }
    }
    sm.z0[r] = z;
  }
  __syncthreads();

  // ---- phase 2a: front flags and the limiter ----
  // item A: the own cell (both directions); item B: one first-ring cell (its slope
  // across the tile edge; the depth slope in both directions for the front test)
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
  const bool b_in = has_b && (!EDGE || (ri >= 0 && ri < nx && rj >= 0 && rj < ny));

  auto limit_cell = [&](int pos, int i, int j, int dirs, R v[9]) -> unsigned char {
    const R h0 = v[0];
    if (!(h0 > R(0))) {
#pragma unroll
      for (int q = 0; q < 9; ++q) v[q] = R(0);
      return 1;
    }
    const bool front = !(h0 > ht) || !(sm.c[0][pos - 1] > ht) || !(sm.c[0][pos + 1] > ht) ||
                       !(sm.c[0][pos - RX] > ht) || !(sm.c[0][pos + RX] > ht);
    if (front) {
      v[1] = v[2] = v[4] = v[5] = v[7] = v[8] = R(0);
      return 1;
    }
    if (p.limiter) {
      const R sw = zb(i, j), se = zb(i + 1, j), nw = zb(i, j + 1), ne = zb(i + 1, j + 1);
      const R z1x = (R(0.5) * (ne + se) - R(0.5) * (nw + sw)) * K<R>::inv_2s3;
      const R z1y = (R(0.5) * (nw + ne) - R(0.5) * (sw + se)) * K<R>::inv_2s3;
      const R z0c = sm.z0[pos];
      const R e0 = h0 + z0c;
#pragma unroll
      for (int d = 1; d <= 2; ++d) {
        const int off = d == 1 ? 1 : RX;
        const R zs = d == 1 ? z1x : z1y;
        // forward and backward differences of the mean free surface; FP32 sums the
        // depth and bed differences (the latter exact), free of the datum
        R dp, dm;
        if constexpr (sizeof(R) == 8) {
          dp = (sm.c[0][pos + off] + sm.z0[pos + off]) - e0;
          dm = e0 - (sm.c[0][pos - off] + sm.z0[pos - off]);
        } else {
          dp = (sm.c[0][pos + off] - h0) + (sm.z0[pos + off] - z0c);
          dm = (h0 - sm.c[0][pos - off]) + (z0c - sm.z0[pos - off]);
        }
        const R e1 = v[d] + zs;
        const R le = minmod3(e1, dp * K<R>::inv_s3, dm * K<R>::inv_s3);
        v[d] = le != e1 ? le - zs : v[d];
        if (!(dirs & d)) continue;  // discharge slopes only where they are used
#pragma unroll
        for (int var = 1; var <= 2; ++var) {
          const int q0 = 3 * var;
          const R a0 = v[q0];
          const R am = sm.c[var][pos - off], ap = sm.c[var][pos + off];
          v[q0 + d] = minmod3(v[q0 + d], (ap - a0) * K<R>::inv_s3, (a0 - am) * K<R>::inv_s3);
        }
      }
    }
    // a depth plane negative at a face centre: a front inside the cell
    if (h0 - s3 * dabs(v[1]) < R(0) || h0 - s3 * dabs(v[2]) < R(0)) {
      v[1] = v[2] = v[4] = v[5] = v[7] = v[8] = R(0);
      return 1;
    }
    return 0;
  };

  if (active) {  // a NaN anywhere in the cell's input would otherwise be absorbed
    R sum = R(0);
#pragma unroll
    for (int q = 0; q < 9; ++q) sum += va[q];
    if (sum != sum) atomicOr(&p.ctrl->health, 1);
  }
  const unsigned char fa = limit_cell(cpos, active ? ci : i0, active ? cj : j0, 3, va);
  unsigned char fb = 1;
  if (b_in) fb = limit_cell(rpos, ri, rj, rb_dir, vb);
  sm.flag[cpos] = fa;
  if (has_b) sm.flag[rpos] = fb;
  __syncthreads();  // box reads are done and the flags are visible

  // ---- phase 2b: revised face states ----
  // own cell: W, E, S, N sides (kept); E and N sides published for the neighbours
  R* const s_side = &sm.c[0][0];  // planes 0..2: east side (h, u, v); 3..5: north side
  Side<R> sw_, se_, ss_, sn_;
  const R slack = R(dsqrt(p.gd * p.htd));
  auto zside = [&](int pos, R zf) -> R { return sm.flag[pos] ? sm.z0[pos] : zf; };
  // ring item: W ring publishes its east side, S ring its north side; E and N ring
  // cells keep their west / south side for the tile's east / north faces
  Side<R> sb_;
  sb_.h = sb_.u = sb_.v = sb_.z = sb_.m = R(0);
  if (b_in) {
    const int oa = rb_side == 0 ? 1 : (rb_side == 1 ? -1 : 0);
    const int ob = rb_side == 2 ? 1 : (rb_side == 3 ? -1 : 0);
    const int npos = rpos + oa + ob * RX;  // the tile cell across the face
    const int ni = ri + oa, nj = rj + ob;
    R zf;
    if (rb_side == 0) zf = R(0.5) * (zb(ri + 1, rj + 1) + zb(ri + 1, rj));
    else if (rb_side == 1) zf = R(0.5) * (zb(ri, rj + 1) + zb(ri, rj));
    else if (rb_side == 2) zf = R(0.5) * (zb(ri, rj + 1) + zb(ri + 1, rj + 1));
    else zf = R(0.5) * (zb(ri, rj) + zb(ri + 1, rj));
    const R own = fb ? sm.z0[rpos] : zf;
    const R nb = (!EDGE || (ni >= 0 && ni < nx && nj >= 0 && nj < ny)) ? zside(npos, zf) : own;
    const R zs = fmaxr(own, nb);
    const bool dx_ = rb_dir == 1;  // select, not index: keeps vb in registers
    const R h1 = dx_ ? vb[1] : vb[2], qx1 = dx_ ? vb[4] : vb[5], qy1 = dx_ ? vb[7] : vb[8];
    const R sg = (rb_side == 0 || rb_side == 2) ? s3 : -s3;  // toward the tile
    sb_ = revise(vb[0] + sg * h1, vb[3] + sg * qx1, vb[6] + sg * qy1, own, zs, ht);
    sb_.u = vcap(sb_.u, sm.um[rpos], sm.um[npos], slack);
    sb_.v = vcap(sb_.v, sm.vm[rpos], sm.vm[npos], slack);
  }
  if (active) {
    const R zW = R(0.5) * (zb(ci, cj + 1) + zb(ci, cj));
    const R zE = R(0.5) * (zb(ci + 1, cj + 1) + zb(ci + 1, cj));
    const R zS = R(0.5) * (zb(ci, cj) + zb(ci + 1, cj));
    const R zN = R(0.5) * (zb(ci, cj + 1) + zb(ci + 1, cj + 1));
    const R z0c = sm.z0[cpos];
    const R own_w = fa ? z0c : zW, own_e = fa ? z0c : zE;
    const R own_s = fa ? z0c : zS, own_n = fa ? z0c : zN;
    const R nb_w = (!EDGE || ci > 0) ? zside(cpos - 1, zW) : own_w;
    const R nb_e = (!EDGE || ci < nx - 1) ? zside(cpos + 1, zE) : own_e;
    const R nb_s = (!EDGE || cj > 0) ? zside(cpos - RX, zS) : own_s;
    const R nb_n = (!EDGE || cj < ny - 1) ? zside(cpos + RX, zN) : own_n;
    sw_ = revise(va[0] - s3 * va[1], va[3] - s3 * va[4], va[6] - s3 * va[7], own_w,
                 fmaxr(own_w, nb_w), ht);
    se_ = revise(va[0] + s3 * va[1], va[3] + s3 * va[4], va[6] + s3 * va[7], own_e,
                 fmaxr(own_e, nb_e), ht);
    ss_ = revise(va[0] - s3 * va[2], va[3] - s3 * va[5], va[6] - s3 * va[8], own_s,
                 fmaxr(own_s, nb_s), ht);
    sn_ = revise(va[0] + s3 * va[2], va[3] + s3 * va[5], va[6] + s3 * va[8], own_n,
                 fmaxr(own_n, nb_n), ht);
    const R u0 = sm.um[cpos], v0 = sm.vm[cpos];
    const int pw = (!EDGE || ci > 0) ? cpos - 1 : cpos, pe = (!EDGE || ci < nx - 1) ? cpos + 1 : cpos;
    const int ps = (!EDGE || cj > 0) ? cpos - RX : cpos, pn = (!EDGE || cj < ny - 1) ? cpos + RX : cpos;
    sw_.u = vcap(sw_.u, u0, sm.um[pw], slack); sw_.v = vcap(sw_.v, v0, sm.vm[pw], slack);
    se_.u = vcap(se_.u, u0, sm.um[pe], slack); se_.v = vcap(se_.v, v0, sm.vm[pe], slack);
    ss_.u = vcap(ss_.u, u0, sm.um[ps], slack); ss_.v = vcap(ss_.v, v0, sm.vm[ps], slack);
    sn_.u = vcap(sn_.u, u0, sm.um[pn], slack); sn_.v = vcap(sn_.v, v0, sm.vm[pn], slack);
  }
  // the parts of L that need only the cell's own face sides (2-point Gauss fluxes and
  // bed source), taken now so that the sides need not stay live past the face phase:
  // gx/gy: F(U+) + F(U-) per direction; sx/sy: the source terms of L0 and L1
  R gx[3] = {R(0), R(0), R(0)}, gy[3] = {R(0), R(0), R(0)};
  R sx0 = R(0), sx1 = R(0), sy0 = R(0), sy1 = R(0);
  const R g = p.g;
  if (active) {
    const R k2s3 = R(2) * s3 * g * p.idx;
    {  // x direction
      const R hb0 = R(0.5) * (se_.h + sw_.h), hb1 = (se_.h - sw_.h) * K<R>::inv_2s3;
      const R qxE = se_.h * se_.u, qxW = sw_.h * sw_.u, qyE = se_.h * se_.v, qyW = sw_.h * sw_.v;
      const R qb0 = R(0.5) * (qxE + qxW), qb1 = (qxE - qxW) * K<R>::inv_2s3;
      const R rb0 = R(0.5) * (qyE + qyW), rb1 = (qyE - qyW) * K<R>::inv_2s3;
      const R zb1 = ((se_.z - sw_.z) + (se_.m - sw_.m)) * K<R>::inv_2s3;
      R Fp[3], Fm[3];
      gauss_flux(g, ht, hb0 + hb1, qb0 + qb1, rb0 + rb1, Fp);
      gauss_flux(g, ht, hb0 - hb1, qb0 - qb1, rb0 - rb1, Fm);
#pragma unroll
      for (int q = 0; q < 3; ++q) gx[q] = Fp[q] + Fm[q];
      sx0 = k2s3 * hb0 * zb1;
      sx1 = k2s3 * hb1 * zb1;
    }
    {  // y direction: Gp/Gm are [mass, y-mom (normal), x-mom (tangential)]
      const R hb0 = R(0.5) * (sn_.h + ss_.h), hb1 = (sn_.h - ss_.h) * K<R>::inv_2s3;
      const R qxN = sn_.h * sn_.u, qxS = ss_.h * ss_.u, qyN = sn_.h * sn_.v, qyS = ss_.h * ss_.v;
      const R qb0 = R(0.5) * (qxN + qxS), qb1 = (qxN - qxS) * K<R>::inv_2s3;
      const R rb0 = R(0.5) * (qyN + qyS), rb1 = (qyN - qyS) * K<R>::inv_2s3;
      const R zb1 = ((sn_.z - ss_.z) + (sn_.m - ss_.m)) * K<R>::inv_2s3;
      R Gp[3], Gm[3];
      gauss_flux(g, ht, hb0 + hb1, rb0 + rb1, qb0 + qb1, Gp);
      gauss_flux(g, ht, hb0 - hb1, rb0 - rb1, qb0 - qb1, Gm);
      gy[0] = Gp[0] + Gm[0];
      gy[1] = Gp[2] + Gm[2];  // x-momentum
      gy[2] = Gp[1] + Gm[1];  // y-momentum
      sy0 = k2s3 * hb0 * zb1;
      sy1 = k2s3 * hb1 * zb1;
    }
  }
  // the own-cell parts of L go into the stage update now (w = va + dt Lg), so that
  // neither they nor va stay live through the face phase; stage 1 publishes V^n here
  R w[9];
  {
    const R c = -s3 * p.idx;
    const R Lg[9] = {R(0), -c * gx[0], -c * gy[0], -sx0, -c * gx[1] - sx1, -c * gy[1],
                     -sy0, -c * gx[2], -c * gy[2] - sy1};
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      w[q] = va[q] + dtr * Lg[q];
      asm volatile("" : "+v"(w[q]));  // formed here: the compiler would otherwise sink it
    }                                 // past the flux phase, keeping its inputs live
    if (STAGE == 1 && active) {
#pragma unroll
      for (int q = 0; q < 9; ++q) (p.vbuf + q * n)[ck] = va[q];
    }
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
  double led_in = 0.0, led_out = 0.0, led_clip = 0.0;
  const double wflux = 0.5 * dt * p.dxd;  // ledger weight: RK2 half step times face width
  // x-face at index f between cells f-1 and f on row j; pos is the box position of f;
  // slot is the face's place in the flux array
  auto xface = [&](int f, int j, int pos, const Side<R>& own_r, bool have_r, int slot) {
    if (EDGE && (j >= ny || f > nx)) return;
    R lh = R(0), lu = R(0), lv = R(0), rh = R(0), ru = R(0), rv = R(0);
    if (!EDGE || f > 0) {
      lh = s_side[0 * RB + pos - 1];
      lu = s_side[1 * RB + pos - 1];
      lv = s_side[2 * RB + pos - 1];
    }
    if (!EDGE || f < nx) {
      if (!have_r) return;
      rh = own_r.h; ru = own_r.u; rv = own_r.v;
    }
    int kind = -1;
    if (EDGE && f == 0) {
      kind = p.bface[j] & 255;
      ghost(p, p.bface[j], t_stage, true, R(1), rh, ru, rv, lh, lu, lv);
    } else if (EDGE && f == nx) {
      kind = p.bface[ny + j] & 255;
      ghost(p, p.bface[ny + j], t_stage, true, R(-1), lh, lu, lv, rh, ru, rv);
    }
    R out[3];
    if (EDGE && kind == 3) {
      if (f == 0) phys_flux(g, lh, lu, lv, out);
      else phys_flux(g, rh, ru, rv, out);
    } else {
      hll(g, lh, lu, lv, rh, ru, rv, out);
    }
    sm.fx[0][slot] = out[0];
    sm.fx[1][slot] = out[1];
    sm.fx[2][slot] = out[2];
    if (EDGE && f == 0) {
      const double m = double(out[0]) * wflux;
      if (m > 0) led_in += m; else led_out -= m;
    } else if (EDGE && f == nx) {
      const double m = -double(out[0]) * wflux;
      if (m > 0) led_in += m; else led_out -= m;
    }
  };
  auto yface = [&](int i, int f, int pos, const Side<R>& own_r, bool have_r, int slot) {
    if (EDGE && (i >= nx || f > ny)) return;
    R lh = R(0), lu = R(0), lv = R(0), rh = R(0), ru = R(0), rv = R(0);  // (h, normal v, tangential u)
    if (!EDGE || f > 0) {
      lh = s_side[3 * RB + pos - RX];
      lu = s_side[5 * RB + pos - RX];
      lv = s_side[4 * RB + pos - RX];
    }
    if (!EDGE || f < ny) {
      if (!have_r) return;
      rh = own_r.h; ru = own_r.v; rv = own_r.u;
    }
    int kind = -1;
    if (EDGE && f == 0) {
      kind = p.bface[2 * ny + i] & 255;
      ghost(p, p.bface[2 * ny + i], t_stage, false, R(1), rh, ru, rv, lh, lu, lv);
    } else if (EDGE && f == ny) {
      kind = p.bface[2 * ny + nx + i] & 255;
      ghost(p, p.bface[2 * ny + nx + i], t_stage, false, R(-1), lh, lu, lv, rh, ru, rv);
    }
    R o[3];
    if (EDGE && kind == 3) {
      if (f == 0) phys_flux(g, lh, lu, lv, o);
      else phys_flux(g, rh, ru, rv, o);
    } else {
      hll(g, lh, lu, lv, rh, ru, rv, o);
    }
    sm.fy[0][slot] = o[0];
    sm.fy[1][slot] = o[2];  // x-momentum is tangential on a y-face
    sm.fy[2][slot] = o[1];
    if (EDGE && f == 0) {
      const double m = double(o[0]) * wflux;
      if (m > 0) led_in += m; else led_out -= m;
    } else if (EDGE && f == ny) {
      const double m = -double(o[0]) * wflux;
      if (m > 0) led_in += m; else led_out -= m;
    }
  };
  // own position (also the east / north boundary face when the cell is just outside)
  const int ta = tid % TX, tb = tid / TX;  // the thread's tile position
  xface(ci, cj, cpos, sw_, active, tb * (TX + 1) + ta);
  yface(ci, cj, cpos, ss_, active, tb * TX + ta);
  if (has_b && rb_side == 1) xface(ri, rj, rpos, sb_, b_in, (rb_b - 2) * (TX + 1) + TX);
  if (has_b && rb_side == 3) yface(ri, rj, rpos, sb_, b_in, TY * TX + (rb_a - 2));
  if (STAGE == 2 && !kPrefetch && active) {  // V^n of the own cell: in flight across the barrier
#pragma unroll
    for (int q = 0; q < 9; ++q) vn[q] = (p.vbuf + q * n)[ck];
  }
  const int gfirst = (STAGE == 2 && p.gauge_h && active) ? p.gmap[ck] : -1;
  __syncthreads();

  // ---- phase 3: L, the stage update, and the per-block reductions ----
  R my_dtc = R(__builtin_huge_val());  // the cell's CFL candidate, reduced in R
  if (active) {
    const int xw = tb * (TX + 1) + ta, ys = tb * TX + ta;
    const R fw[3] = {sm.fx[0][xw], sm.fx[1][xw], sm.fx[2][xw]};
    const R fe[3] = {sm.fx[0][xw + 1], sm.fx[1][xw + 1], sm.fx[2][xw + 1]};
    const R fs[3] = {sm.fy[0][ys], sm.fy[1][ys], sm.fy[2][ys]};
    const R fn[3] = {sm.fy[0][ys + TX], sm.fy[1][ys + TX], sm.fy[2][ys + TX]};
    const R idx = p.idx;
    const R c = -s3 * idx;
    R L[9];
    L[0] = -(fe[0] - fw[0]) * idx + -(fn[0] - fs[0]) * idx;
    L[3] = -(fe[1] - fw[1]) * idx + -(fn[1] - fs[1]) * idx;
    L[6] = -(fe[2] - fw[2]) * idx + -(fn[2] - fs[2]) * idx;
    L[1] = c * (fe[0] + fw[0]);
    L[4] = c * (fe[1] + fw[1]);
    L[7] = c * (fe[2] + fw[2]);
    L[2] = c * (fn[0] + fs[0]);
    L[5] = c * (fn[1] + fs[1]);
    L[8] = c * (fn[2] + fs[2]);
    R u[9];
    if (STAGE == 1) {
#pragma unroll
      for (int q = 0; q < 9; ++q) u[q] = w[q] + dtr * L[q];
    } else {
#pragma unroll
      for (int q = 0; q < 9; ++q) u[q] = R(0.5) * (vn[q] + w[q] + dtr * L[q]);
    }
    // after each stage: clip a negative mean depth (booking the mass), then drop the
    // discharge of cells at or below the dry tolerance
    {  // branch-free: a branch here splits the update and costs registers
      const bool neg = u[0] < R(0);
      led_clip = neg ? -double(u[0]) * p.dxd * p.dxd * (STAGE == 1 ? 0.5 : 1.0) : 0.0;
      u[0] = neg ? R(0) : u[0];
      u[1] = neg ? R(0) : u[1];
      u[2] = neg ? R(0) : u[2];
    }
    const bool dry = !(u[0] > ht);
#pragma unroll
    for (int q = 3; q < 9; ++q) u[q] = dry ? R(0) : u[q];
    R sum = R(0);
#pragma unroll
    for (int q = 0; q < 9; ++q) sum += u[q];
    if (sum != sum) atomicOr(&p.ctrl->health, 1);
    if (STAGE == 1) {
#pragma unroll
      for (int q = 0; q < 9; ++q) (p.ui + q * n)[ck] = u[q];
    } else {
#pragma unroll
      for (int q = 0; q < 9; ++q) (p.uout + q * n)[ck] = u[q];
      for (int g = gfirst; g >= 0; g = p.gnext[g]) p.gauge_h[g] = double(u[0]);
      my_dtc = cell_dtc_r(p, u[0], u[1], u[2], u[3], u[6]);
    }
  }

  // per-block reductions in a fixed order (deterministic); boundary-flux ledger terms
  // exist only in edge tiles
  const int lane = tid & 63, wv = tid >> 6;
  const double r_clip = wave_sum_sparse(led_clip);
  double r_in = 0.0, r_out = 0.0;
  if (EDGE) {
    r_in = wave_sum_sparse(led_in);
    r_out = wave_sum_sparse(led_out);
  }
  if (lane == 0) {
    sm.red[wv][0] = r_in;
    sm.red[wv][1] = r_out;
    sm.red[wv][2] = r_clip;
  }
  if (STAGE == 2) {
    const double r_dt = double(wave_min(my_dtc));
    if (lane == 0) sm.red[wv][3] = r_dt;
  }
  __syncthreads();
  if (tid == 0) {
    double a = 0, bsum = 0, c = 0, m = __longlong_as_double((long long)INF_BITS);
    for (int k = 0; k < NT / 64; ++k) {
      a += sm.red[k][0];
      bsum += sm.red[k][1];
      c += sm.red[k][2];
      if (STAGE == 2) m = sm.red[k][3] < m ? sm.red[k][3] : m;
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
        cand_post(p.ctrl->dtc[1 - p.parity], tile, m);
    }
  }
}

// One stage over tile `tile` of the context described by p: the step's time step, the
// control-block update (stage 1, tile 0), then the tile's work (or, once the run has
// reached t_end, a copy of the state that keeps the buffer parity).
template <typename R, typename S, int STAGE>
__device__ __forceinline__ void stage_tile(const Params<R> p, const int tile) {
  constexpr int TX = Geo<S>::TX, TY = Geo<S>::TY;
  const int i0 = (tile % p.tiles_x) * TX, j0 = (tile / p.tiles_x) * TY;

  __shared__ Smem<R, S> sm;
  const bool interior = i0 >= 2 && j0 >= 2 && i0 + TX + 2 <= p.nx && j0 + TY + 2 <= p.ny;
  if (interior)
    stage_body<R, S, STAGE, false>(p, sm, tile, i0, j0);
  else
    stage_body<R, S, STAGE, true>(p, sm, tile, i0, j0);
}

// one context: one block per tile, blocks of an XCD on a contiguous band of tiles
template <typename R, typename S, int STAGE>
__global__ __launch_bounds__(Geo<S>::NT, STAGE == 1 ? S::B1 : S::B2) void stage_kernel(Params<R> p) {
  const int b = blockIdx.x;
  const int tile = (b % NXCD) * p.per_xcd + b / NXCD;
  if (tile >= p.n_tiles) return;
  stage_tile<R, S, STAGE>(p, tile);
}

// ---------------------------------------------------------------------------------
// batched scenarios: one launch per stage over the tiles of every scenario
// ---------------------------------------------------------------------------------
constexpr int MAX_BATCH = 256;

// the launch description in device memory: the work list is the scenarios' tiles in
// order (scenario k owns items start[k] .. start[k+1]-1), and each scenario has its
// parameters for both buffer phases (its parity flips every step)
template <typename R>
struct BatchTable {
  int n, total, per_xcd, pad;
  int start[MAX_BATCH + 1];
  Params<R> p[2][MAX_BATCH];
};

template <typename R, typename S, int STAGE>
__global__ __launch_bounds__(Geo<S>::NT, STAGE == 1 ? S::B1 : S::B2) void stage_kernel_batch(
    const BatchTable<R>* __restrict__ tab, int phase) {
  const int b = blockIdx.x;
  const int g = (b % NXCD) * tab->per_xcd + b / NXCD;
  if (g >= tab->total) return;
  int lo = 0, hi = tab->n;  // start[lo] <= g < start[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (tab->start[mid] <= g) lo = mid; else hi = mid;
  }
  const Params<R> p = tab->p[phase][lo];
  stage_tile<R, S, STAGE>(p, g - tab->start[lo]);
}

// time and health of every scenario of a batch (one thread each)
template <typename R>
__global__ void batch_status_kernel(const BatchTable<R>* __restrict__ tab, int phase,
                                    double* __restrict__ t_out, int* __restrict__ health_out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= tab->n) return;
  const Params<R>& p = tab->p[phase][k];
  t_out[k] = p.ctrl->t[p.parity];
  health_out[k] = p.ctrl->health;
}

// ---------------------------------------------------------------------------------
// FV1 (Sect. 2.1.2, eq 5-7): piecewise-constant h, qx, qy and bed (z0 of eq 8), one
// launch per time step: friction at the centre, HLL fluxes of the two cells' means
// at each face after the temporary revision, L0 with the bed source
// -g (hE* + hW*)/2 (zE** - zW**)/dx, and the forward-Euler update of eq 7. Only the
// mean planes (0, 3, 6) are read and written; the slope planes stay zero.
// ---------------------------------------------------------------------------------
template <typename R, typename S>
struct SmemFV1 {
  static constexpr int TX = S::X, TY = S::Y, NT = TX * TY;
  static constexpr int RX = TX + 2, RB = RX * (TY + 2);   // 1-cell cross halo
  R h[RB], u[RB], v[RB], z0[RB];  // box depths and velocities after friction; bed means
  R f[3][RB];                     // fluxes of one direction: the west (then south)
                                  // face of each position
  double red[NT / 64][4];
};

// revised depth and bed of one side of a face (FP64: eta form; FP32: bed differences)
template <typename R>
__device__ __forceinline__ void fv1_side(R h, R zb, R zs, R& hs, R& zss) {
  if constexpr (sizeof(R) == 8) {
    const R eta = h + zb;
    hs = fmax0(eta - zs);
    zss = fminr(eta, zs);
  } else {
    const R d = h + (zb - zs);
    hs = fmax0(d);
    zss = zs + fminr(d, R(0));
  }
}

// One FV1 step over one tile. EDGE is false for tiles whose halo lies inside the
// domain: no clamping, no boundary faces.
template <typename R, typename S, bool EDGE>
__device__ __forceinline__ void fv1_body(const Params<R>& p, SmemFV1<R, S>& sm, const int tile, const int i0,
                                         const int j0) {
  using SM = SmemFV1<R, S>;
  constexpr int TX = SM::TX, TY = SM::TY, NT = SM::NT, RX = SM::RX;
  constexpr int NRING = 2 * (TX + TY);
  Ctrl* ctl = p.ctrl;
  const int tid = threadIdx.x;
  const int nx = p.nx, ny = p.ny;
  const long long n = p.n;
  const int ci = i0 + tid % TX, cj = j0 + tid / TX;
  const bool active = !EDGE || (ci < nx && cj < ny);
  // unsigned: a cell past the grid's last row (inactive) may lie beyond INT_MAX
  const unsigned ck = (unsigned)cj * (unsigned)nx + (unsigned)ci;
  const R* __restrict__ hin = p.uin;
  const R* __restrict__ qxin = p.uin + 3 * n;
  const R* __restrict__ qyin = p.uin + 6 * n;
  const R ht = p.h_tol, g = p.g;
  const R dT = (sizeof(R) == 4 && p.datum) ? p.datum[tile] : R(0);

  // No vector memory operation is in flight when a tile body starts; the wait costs
  // nothing and keeps the wait-count analysis from carrying in the other body's loads.
  __builtin_amdgcn_s_waitcnt(kWaitVmem);

  // ---- phase 1: the step's time step; the box depths and velocities (friction
  // applied) and bed means ----
  // The step count and time, then the state, Manning coefficient and bed mean of the
  // own cell and of the thread's halo item are all issued before any is waited on; the
  // ring candidate, whose slot the count picks, follows while they are in flight. (The
  // other two rings are not read: one takes this step's atomic minima, the other is
  // being cleared, and reading them costs more than the extra round trip.)
  const int a = p.parity, o = 1 - p.parity;
  const long long k_ld = ctl->step[a];
  const double t_ld = ctl->t[a];
  struct Raw {
    R h, qx, qy, nm, z, zd;
  };
  // box position (ab, bb); a cell of another tile is moved into this tile's datum frame
  // (a whole number of metres: exact) when published, so that its datum load waits for
  // nothing here
  auto load_raw = [&](int ab, int bb, bool own, Raw& w) {
    int i = i0 - 1 + ab, j = j0 - 1 + bb;
    if (EDGE) {
      i = i < 0 ? 0 : (i >= nx ? nx - 1 : i);
      j = j < 0 ? 0 : (j >= ny ? ny - 1 : j);
    }
    const unsigned kk = (unsigned)j * (unsigned)nx + (unsigned)i;
    w.h = hin[kk];
    w.qx = qxin[kk];
    w.qy = qyin[kk];
    w.nm = p.manning ? p.manning[kk] : p.n_scalar;
    w.z = p.zc[kk];
    w.zd = dT;
    if (sizeof(R) == 4 && p.datum && !own)  // i, j >= 0 here
      w.zd = p.datum[(unsigned)j / TY * (unsigned)p.tiles_x + (unsigned)i / TX];
  };
  const int ca = tid % TX + 1, cb = tid / TX + 1, cpos = cb * RX + ca;
  Raw w0, w1;
  load_raw(ca, cb, true, w0);
  int hab = 0, hbb = 0;
  const bool has_item = tid < NRING;
  if (has_item) {
    if (tid < TY) { hab = 0; hbb = tid + 1; }
    else if (tid < 2 * TY) { hab = TX + 1; hbb = tid - TY + 1; }
    else if (tid < 2 * TY + TX) { hab = tid - 2 * TY + 1; hbb = 0; }
    else { hab = tid - 2 * TY - TX + 1; hbb = TY + 1; }
    load_raw(hab, hbb, false, w1);
  }

  // the step's time step from the ring slot of this step
  const long long k = uniform(k_ld);
  const double t = uniform(t_ld);
  const double mm = uniform(cand_read(ctl->dtr[k % 3]));
  double dt = (mm == __longlong_as_double((long long)INF_BITS)) ? p.dt_dry : p.cfl * mm;
  const double dt_cfl = dt;
  if (p.dt_max > 0.0 && p.dt_max < dt) dt = p.dt_max;
  double t_next = t + dt;
  if (p.t_end - t <= dt) {
    dt = p.t_end - t;
    t_next = p.t_end;
  }
  dt = uniform(dt);  // the same in every lane: held in scalar registers
  t_next = uniform(t_next);
  if (!(dt > 0.0)) {  // past t_end: carry the state over
    if (active) {
      p.vbuf[ck] = w0.h;
      (p.vbuf + 3 * n)[ck] = w0.qx;
      (p.vbuf + 6 * n)[ck] = w0.qy;
    }
    if (tile == 0 && tid == 0) {
      ctl->t[o] = t;
      ctl->step[o] = k;
      ctl->dt_used[a] = 0.0;
    }
    return;
  }
  if (tile == 0 && tid == 0) {
    ctl->t[o] = t_next;
    ctl->step[o] = k + 1;
    ctl->dt_used[a] = dt;
    cand_clear(ctl->dtr[(k + 2) % 3]);
    if (dt_cfl < 1e-12) atomicOr(&ctl->health, 2);
  }
  const R dtr = R(dt);

  // friction, then the box cell's depth, velocities and bed mean (eq 8, from the plane
  // set up at initialisation) to LDS; returns the cell's discharges after friction
  auto publish = [&](int ab, int bb, bool own, const Raw& w, R& qx, R& qy) {
    qx = w.qx;
    qy = w.qy;
    if (w.nm > R(0)) {
      R dqx, dqy;
      friction_inc(g * w.nm * w.nm * dtr, ht, w.h, qx, qy, dqx, dqy);
      qx += dqx;
      qy += dqy;
    }
    const int r = bb * RX + ab;
    const R rr = frcp(fmaxr(w.h, Tiny<R>::v));
    sm.h[r] = w.h;
    sm.u[r] = w.h > ht ? qx * rr : R(0);
    sm.v[r] = w.h > ht ? qy * rr : R(0);
    sm.z0[r] = (sizeof(R) == 4 && p.datum && !own) ? w.z + (w.zd - dT) : w.z;
  };
  R qx0, qy0;
  publish(ca, cb, true, w0, qx0, qy0);
  if (has_item) {
    R qxr, qyr;
    publish(hab, hbb, false, w1, qxr, qyr);
  }
  __syncthreads();

  double led_in = 0.0, led_out = 0.0;
  const double wflux = dt * p.dxd;
  // HLL through face f of a line (x: f between cells f-1 and f of row `line`; y: f
  // between rows f-1 and f of column `line`); r is the box position of cell f; the flux
  // goes to sm.f at r, in (mass, x-mom, y-mom)
  auto face = [&](bool xdir, int f, int line, int r) {
    const int nf = xdir ? nx : ny;
    if (EDGE && (line >= (xdir ? ny : nx) || f > nf)) return;
    const int st = xdir ? 1 : RX;
    const int rl = (!EDGE || f > 0) ? r - st : r, rr_ = (!EDGE || f < nf) ? r : r - st;
    const R zl = sm.z0[rl], zr = sm.z0[rr_];
    const R zs = fmaxr(zl, zr);
    R hl, zll, hr, zrr;
    fv1_side(sm.h[rl], zl, zs, hl, zll);
    fv1_side(sm.h[rr_], zr, zs, hr, zrr);
    // normal frame: x faces (h, u, v), y faces (h, v, u)
    R nl = xdir ? sm.u[rl] : sm.v[rl], tl = xdir ? sm.v[rl] : sm.u[rl];
    R nr = xdir ? sm.u[rr_] : sm.v[rr_], tr = xdir ? sm.v[rr_] : sm.u[rr_];
    const int eo = xdir ? 0 : 2 * ny;
    int kind = -1;
    if (EDGE && f == 0) {
      kind = p.bface[eo + line] & 255;
      ghost(p, p.bface[eo + line], t, xdir, R(1), hr, nr, tr, hl, nl, tl);
    } else if (EDGE && f == nf) {
      kind = p.bface[eo + (xdir ? ny : nx) + line] & 255;
      ghost(p, p.bface[eo + (xdir ? ny : nx) + line], t, xdir, R(-1), hl, nl, tl, hr, nr, tr);
    }
    R o3[3];
    if (EDGE && kind == 3) {
      if (f == 0) phys_flux(g, hl, nl, tl, o3);
      else phys_flux(g, hr, nr, tr, o3);
    } else {
      hll(g, hl, nl, tl, hr, nr, tr, o3);
    }
    sm.f[0][r] = o3[0];
    sm.f[1][r] = xdir ? o3[1] : o3[2];  // x-momentum is tangential on a y-face
    sm.f[2][r] = xdir ? o3[2] : o3[1];
    if (EDGE && f == 0) {
      const double m = double(o3[0]) * wflux;
      if (m > 0) led_in += m; else led_out -= m;
    } else if (EDGE && f == nf) {
      const double m = -double(o3[0]) * wflux;
      if (m > 0) led_in += m; else led_out -= m;
    }
  };
  // the cell's own state and its revised depth and bed at one face
  const R h = sm.h[cpos], z = sm.z0[cpos];
  auto side = [&](int nb, bool inside, R& hs, R& zss) {
    const R zs = inside ? fmaxr(z, sm.z0[nb]) : z;
    fv1_side(h, z, zs, hs, zss);
  };
  const R idx = p.idx;
  R L0 = R(0), L1 = R(0), L2 = R(0);

  // ---- phase 2: x faces (each west face once; the tile's east faces by halo items) ----
  if (active) face(true, ci, cj, cpos);
  if (tid < TY) {
    if (!EDGE || i0 + TX <= nx) face(true, i0 + TX, j0 + tid, (tid + 1) * RX + TX + 1);
  }
  if (EDGE && active && ci == nx - 1 && i0 + TX > nx) face(true, nx, cj, cpos + 1);  // cut tile
  __syncthreads();
  if (active) {
    R hE, zE, hW, zW;
    side(cpos + 1, !EDGE || ci < nx - 1, hE, zE);
    side(cpos - 1, !EDGE || ci > 0, hW, zW);
    L0 = -(sm.f[0][cpos + 1] - sm.f[0][cpos]) * idx;
    L1 = -(sm.f[1][cpos + 1] - sm.f[1][cpos]) * idx - g * R(0.5) * (hE + hW) * (zE - zW) * idx;
    L2 = -(sm.f[2][cpos + 1] - sm.f[2][cpos]) * idx;
  }
  __syncthreads();

  // ---- phase 3: y faces, then L0 and the forward-Euler update ----
  if (active) face(false, cj, ci, cpos);
  if (tid >= 64 && tid < 64 + TX) {
    if (!EDGE || j0 + TY <= ny) face(false, j0 + TY, i0 + tid - 64, (TY + 1) * RX + tid - 64 + 1);
  }
  if (EDGE && active && cj == ny - 1 && j0 + TY > ny) face(false, ny, ci, cpos + RX);  // cut tile
  __syncthreads();
  R my_dtc = R(__builtin_huge_val());  // the cell's CFL candidate, reduced in R
  double led_clip = 0.0;
  if (active) {
    R hN, zN, hS, zS;
    side(cpos + RX, !EDGE || cj < ny - 1, hN, zN);
    side(cpos - RX, !EDGE || cj > 0, hS, zS);
    L0 += -(sm.f[0][cpos + RX] - sm.f[0][cpos]) * idx;
    L1 += -(sm.f[1][cpos + RX] - sm.f[1][cpos]) * idx;
    L2 += -(sm.f[2][cpos + RX] - sm.f[2][cpos]) * idx - g * R(0.5) * (hN + hS) * (zN - zS) * idx;
    R u0 = h + dtr * L0, u1 = qx0 + dtr * L1, u2 = qy0 + dtr * L2;
    const bool neg = u0 < R(0);  // clip (booking the mass), branch-free
    led_clip = neg ? -double(u0) * p.dxd * p.dxd : 0.0;
    u0 = neg ? R(0) : u0;
    const bool dry = !(u0 > ht);
    u1 = dry ? R(0) : u1;
    u2 = dry ? R(0) : u2;
    if ((u0 + u1 + u2) != (u0 + u1 + u2)) atomicOr(&ctl->health, 1);
    p.vbuf[ck] = u0;
    (p.vbuf + 3 * n)[ck] = u1;
    (p.vbuf + 6 * n)[ck] = u2;
    my_dtc = cell_dtc_r(p, u0, R(0), R(0), u1, u2);
  }
  const int lane = tid & 63, wv = tid >> 6;
  // boundary-flux ledger terms exist only in edge tiles
  const double r_clip = wave_sum_sparse(led_clip);
  double r_in = 0.0, r_out = 0.0;
  if (EDGE) {
    r_in = wave_sum_sparse(led_in);
    r_out = wave_sum_sparse(led_out);
  }
  const double r_dt = double(wave_min(my_dtc));
  if (lane == 0) {
    sm.red[wv][0] = r_in;
    sm.red[wv][1] = r_out;
    sm.red[wv][2] = r_clip;
    sm.red[wv][3] = r_dt;
  }
  __syncthreads();
  if (tid == 0) {
    double ai = 0, ao = 0, ac = 0, m = __longlong_as_double((long long)INF_BITS);
    for (int w = 0; w < NT / 64; ++w) {
      ai += sm.red[w][0];
      ao += sm.red[w][1];
      ac += sm.red[w][2];
      m = sm.red[w][3] < m ? sm.red[w][3] : m;
    }
    if (ai != 0.0 || ao != 0.0 || ac != 0.0) {
      double* led = p.ledger + 4 * (long long)tile;
      led[0] += ai;
      led[1] += ao;
      led[2] += ac;
    }
    if (tile == 0) {
      const double fm = forcing_dtc(p, t_next);
      m = fm < m ? fm : m;
    }
    if (m != __longlong_as_double((long long)INF_BITS))
      cand_post(ctl->dtr[(k + 1) % 3], tile, m);
  }
}

// FP32 is built for 8 waves per SIMD (it needs about 50 VGPRs; without the bound its
// scalar registers alone would hold it to 7), FP64 for 7 (70 VGPRs)
template <typename R, typename S>
__global__ __launch_bounds__(S::X * S::Y, sizeof(R) == 4 ? 8 : 7) void fv1_kernel(Params<R> p) {
  using SM = SmemFV1<R, S>;
  constexpr int TX = SM::TX, TY = SM::TY, NT = SM::NT;
  constexpr int NRING = 2 * (TX + TY);
  static_assert(NT % 64 == 0 && NRING <= NT && TY <= 64 && 64 + TX <= NT,
                "tile must give whole waves and room for the halo items");
  __shared__ SM sm;
  const int b = blockIdx.x;
  const int tile = (b % NXCD) * p.per_xcd + b / NXCD;
  if (tile >= p.n_tiles) return;
  const int nx = p.nx, ny = p.ny;
  const int i0 = (tile % p.tiles_x) * TX, j0 = (tile / p.tiles_x) * TY;
  const bool interior = i0 >= 1 && j0 >= 1 && i0 + TX + 1 <= nx && j0 + TY + 1 <= ny;
  if (interior)
    fv1_body<R, S, false>(p, sm, tile, i0, j0);
  else
    fv1_body<R, S, true>(p, sm, tile, i0, j0);
}

// ---------------------------------------------------------------------------------
// set-up and diagnostics kernels
// ---------------------------------------------------------------------------------
// the bed mean of every cell (eq 8, as the stage kernels form it), in the frame of the
// datum of the cell's own tile: the FV1 kernel's piecewise-constant bed
template <typename R>
__global__ void bedmean_kernel(Params<R> p, R* __restrict__ zc) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= p.n) return;
  const int i = int(k % p.nx), j = int(k / p.nx);
  R z0, z1x, z1y;
  bed(p, i, j, z0, z1x, z1y);
  zc[k] = z0;
}

template <typename R>
__global__ void convert_kernel(const double* __restrict__ src, R* __restrict__ dst, long long count) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < count) dst[k] = R(src[k]);
}

// a control block for a step with no history, starting at time t: every CFL slot
// cleared, times and counters set, health cleared, and n_led ledger doubles zeroed
// (a kernel rather than memsets, so that the clearing is an ordinary launch)
__global__ void reset_ctrl_kernel(Ctrl* __restrict__ ctrl, double t, double* __restrict__ ledger,
                                  long long n_led) {
  const long long k0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long stride = (long long)gridDim.x * blockDim.x;
  if (k0 == 0) {
    ctrl->t[0] = ctrl->t[1] = t;
    ctrl->dt_used[0] = ctrl->dt_used[1] = 0.0;
    ctrl->step[0] = ctrl->step[1] = 0;
    ctrl->health = 0;
    ctrl->pad = 0;
  }
  constexpr long long NS = NSLOT * SLOT_STRIDE;
  for (long long k = k0; k < 5 * NS; k += stride) {
    Cand& c = k < 2 * NS ? ctrl->dtc[k / NS] : ctrl->dtr[(k - 2 * NS) / NS];
    c.s[k % NS] = INF_BITS;
  }
  for (long long k = k0; k < n_led; k += stride) ledger[k] = 0.0;
}

// sets *bad when any of count values is negative or not finite (Manning n given in
// device memory is checked before it replaces the plane)
__global__ void check_nonneg_kernel(const double* __restrict__ src, long long count, int* bad) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < count) {
    const double v = src[k];
    if (!(v >= 0.0) || !(v <= 1.7976931348623157e308)) atomicOr(bad, 1);
  }
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
    bed(p, i, j, z0, z1x, z1y);  // in the frame of the tile's datum
    const R h0 = R((eta - double(tile_datum(p, i, j))) - double(z0));
    if (h0 > R(0)) {
      c[0] = h0;
      c[1] = -z1x;
      c[2] = -z1y;
    }
  }
  if (p.fv1)  // piecewise constant (eq 5): the means only
    c[1] = c[2] = c[4] = c[5] = c[7] = c[8] = R(0);
  if (!(c[0] > p.h_tol))
    for (int q = 3; q < 9; ++q) c[q] = R(0);
  for (int q = 0; q < 9; ++q) p.vbuf[q * n + k] = c[q];
}

// CFL candidate of a whole state (set-up and resume): grid-stride min, one atomic per
// block, plus the forcing at time t from block 0
template <typename R>
__global__ void dtc_kernel(Params<R> p, const R* __restrict__ u, double t,
                           unsigned long long* __restrict__ slot) {
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
      atomicMin(slot, (unsigned long long)__double_as_longlong(m));
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
    const int i = int(k % p.nx), j = int(k / p.nx);
    bed(p, i, j, z0, z1x, z1y);
    out[k] = R(double(h0) + double(z0) + double(tile_datum(p, i, j)));
  } else {
    const R q = u[(field == 10 ? 3 : 6) * p.n + k];
    out[k] = h0 > p.h_tol ? q / h0 : R(0);
  }
}

}  // namespace dg2k
