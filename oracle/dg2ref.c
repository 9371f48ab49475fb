/*
 * dg2ref.c -- FP64 CPU oracle for the uniform-grid DG2 time step (Sharifian &
 * Kesserwani, arXiv:2107.02750, Sect. 2.1.1 and 2.1.4).
 *
 * TEST INFRASTRUCTURE ONLY: the plain, slow reference the GPU library is checked
 * against. Never called by the product path.
 *
 * The paper defers the operator details to earlier DG2 papers; the readings this code
 * implements are stated where they are used, and each is one of the numbered readings
 * listed in the design notes of the repository. The structure is deliberately plain:
 * one pass per step of the method over whole arrays, an explicit array of face states
 * and fluxes, scalar loops (OpenMP over rows only), no fusion.
 *
 * Built with -ffp-contract=off so every expression rounds as written.
 */
#include "dg2ref.h"

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define SQRT3 1.7320508075688772935274463415059

/* coefficient plane index (eq 2): var in {0 h, 1 qx, 2 qy}, k in {0 mean, 1 x-slope,
 * 2 y-slope} */
#define PL(var, k) (3 * (var) + (k))

/* one side of a face after the wet/dry revision */
typedef struct {
  double h;  /* revised depth h* >= 0 */
  double u;  /* x velocity (0 if the unrevised depth is <= h_tol) */
  double v;  /* y velocity */
  double z;  /* revised bed z** */
} side_t;

typedef struct {
  double flux[3]; /* [mass, x-momentum, y-momentum] through the face, per unit length */
  side_t lo;      /* the west (x-face) or south (y-face) side */
  side_t hi;      /* the east or north side */
} face_t;

typedef struct {
  int32_t kind, seg;
} bface_t;

typedef struct {
  int32_t edge, kind, i0, i1, n_knots;
  double *t_knots, *q_knots;
  double h_b, u_b, v_b;
} seg_t;

struct dg2ref_ctx {
  dg2ref_config cfg;
  int nx, ny;
  size_t n;
  double *zv;             /* (ny+1)*(nx+1) */
  double *z0, *z1x, *z1y; /* eq 8 */
  double *manning;        /* per cell */
  double *U;              /* 9 planes: the state U^n */
  double *F, *V, *Ui, *W, *L; /* work planes */
  unsigned char *flat;    /* per cell: 1 if the limited stage input is locally first order */
  double *rowsum;         /* per row: partial sums of a pass */
  face_t *xf;             /* (nx+1)*ny x-faces, face f of row j at j*(nx+1)+f */
  face_t *yf;             /* nx*(ny+1) y-faces, face f of column i at f*nx+i */
  bface_t *bw, *be, *bs, *bn; /* boundary face kinds */
  seg_t *segs;
  int n_segs;
  double t;
  int64_t step;
  double dt_next;          /* CFL time step of the current state (before caps) */
  double mass_in, mass_out, mass_clip;
  char err[256];
};

static int fail(dg2ref_ctx *c, int code, const char *fmt, ...) {
  if (c) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(c->err, sizeof c->err, fmt, ap);
    va_end(ap);
  }
  return code;
}

/* ------------------------------------------------------------------------------ */
/* eq 8: bed coefficients from the vertex raster.                                  */
/* Face values are vertex means (Sect. 2.1.4); the mean is the quarter sum of the  */
/* four vertices (reading of the garbled last form of eq 8a: it must equal the two */
/* forms before it).                                                               */
/* ------------------------------------------------------------------------------ */
static double vtx(const double *zv, int nx, int iv, int jv) { return zv[(size_t)jv * (nx + 1) + iv]; }

void dg2ref_bed_coeffs(int32_t nx, int32_t ny, const double *zv, double *z0, double *z1x,
                       double *z1y) {
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      double sw = vtx(zv, nx, i, j), se = vtx(zv, nx, i + 1, j);
      double nw = vtx(zv, nx, i, j + 1), ne = vtx(zv, nx, i + 1, j + 1);
      double zE = 0.5 * (ne + se), zW = 0.5 * (nw + sw);
      double zN = 0.5 * (nw + ne), zS = 0.5 * (sw + se);
      size_t k = (size_t)j * nx + i;
      /* diagonal pairs first: the sum is then the same for the transposed raster */
      z0[k] = 0.25 * ((ne + sw) + (nw + se));
      z1x[k] = (zE - zW) / (2.0 * SQRT3);
      z1y[k] = (zN - zS) / (2.0 * SQRT3);
    }
}

/* bed at the centre of an x-face (vertical face at vertex column f, row j) and of a
 * y-face (horizontal face at vertex row f, column i): the mean of its two vertices.
 * Both neighbouring cells see the same value, so z is continuous at face centres. */
static double zface_x(const dg2ref_ctx *c, int f, int j) {
  return 0.5 * (vtx(c->zv, c->nx, f, j + 1) + vtx(c->zv, c->nx, f, j));
}
static double zface_y(const dg2ref_ctx *c, int i, int f) {
  return 0.5 * (vtx(c->zv, c->nx, i, f) + vtx(c->zv, c->nx, i + 1, f));
}

/* ------------------------------------------------------------------------------ */
/* Split-implicit Manning friction at one point (Sect. 2.1.1: friction is kept out  */
/* of L and applied at the start of each step; C_f = g n^2 / h^(1/3) from eq 1).    */
/* Reading: one Newton step of backward Euler on dq/dt = -C_f u |u| with the        */
/* diagonal of the Jacobian.                                                        */
/* ------------------------------------------------------------------------------ */
void dg2ref_friction_point(double g, double n, double h_tol, double dt, double h,
                           double qx, double qy, double out[2]) {
  out[0] = qx;
  out[1] = qy;
  if (n <= 0.0 || h <= h_tol) return;
  double u = qx / h, v = qy / h;
  double s = sqrt(u * u + v * v);
  if (s <= 0.0) return;
  double cf = g * n * n / cbrt(h);
  double Dx = 1.0 + dt * cf * (2.0 * u * u + v * v) / (h * s);
  double Dy = 1.0 + dt * cf * (u * u + 2.0 * v * v) / (h * s);
  out[0] = qx - dt * cf * u * s / Dx;
  out[1] = qy - dt * cf * v * s / Dy;
}

/* friction on every cell: at the centre (means) and at the two Gauss points in x and
 * in y (slopes). The projected slope is the old slope plus half the difference of the
 * friction increments at its two Gauss points U0 +- U1 (2-point Gauss rule with the
 * scaled Legendre basis of eq 2). h is never touched. */
static void pass_friction(dg2ref_ctx *c, const double *U, double dt, double *F) {
  const int nx = c->nx, ny = c->ny;
  const size_t n = c->n;
  const double g = c->cfg.g, ht = c->cfg.h_tol;
  memcpy(F, U, 9 * n * sizeof(double));
#pragma omp parallel for schedule(static)
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      size_t k = (size_t)j * nx + i;
      double nm = c->manning[k];
      if (nm <= 0.0) continue;
      const double h0 = U[PL(0, 0) * n + k], qx0 = U[PL(1, 0) * n + k], qy0 = U[PL(2, 0) * n + k];
      double q[2];
      dg2ref_friction_point(g, nm, ht, dt, h0, qx0, qy0, q);
      F[PL(1, 0) * n + k] = q[0];
      F[PL(2, 0) * n + k] = q[1];
      for (int d = 1; d <= 2; ++d) { /* d = 1: x Gauss points, d = 2: y Gauss points */
        const double h1 = U[PL(0, d) * n + k], qx1 = U[PL(1, d) * n + k], qy1 = U[PL(2, d) * n + k];
        double hp = h0 + h1, qxp = qx0 + qx1, qyp = qy0 + qy1;
        double hm = h0 - h1, qxm = qx0 - qx1, qym = qy0 - qy1;
        double qp[2], qm[2];
        dg2ref_friction_point(g, nm, ht, dt, hp, qxp, qyp, qp);
        dg2ref_friction_point(g, nm, ht, dt, hm, qxm, qym, qm);
        double dxp = qp[0] - qxp, dyp = qp[1] - qyp;
        double dxm = qm[0] - qxm, dym = qm[1] - qym;
        F[PL(1, d) * n + k] = qx1 + 0.5 * (dxp - dxm);
        F[PL(2, d) * n + k] = qy1 + 0.5 * (dyp - dym);
      }
    }
}

/* ------------------------------------------------------------------------------ */
/* Slope limiter and wet/dry fronts. The paper names no limiter; reading: minmod    */
/* (Cockburn-Shu form for the scaled basis) on the free-surface elevation           */
/* eta = h + z and on qx, qy, one direction at a time. Beyond a domain edge the     */
/* ghost cell copies the edge cell's depth and discharges and continues its bed     */
/* plane, so uniform flow down a sloping bed passes an open edge unlimited.         */
/* Limiting eta rather than h keeps still water still. A cell with h0 <= 0 is dry   */
/* and all its coefficients become zero.                                            */
/* Reading for wet/dry fronts: a cell whose mean depth is at most h_tol, or which   */
/* has such a neighbour across one of its four faces, is made locally first order:  */
/* its slopes become zero and the face revision sees its bed as flat at z0.         */
/* ------------------------------------------------------------------------------ */
static double minmod3(double a, double b, double c) {
  if (a > 0.0 && b > 0.0 && c > 0.0) return fmin(a, fmin(b, c));
  if (a < 0.0 && b < 0.0 && c < 0.0) return fmax(a, fmax(b, c));
  return 0.0;
}

static void pass_limit(dg2ref_ctx *c, const double *S, double *out) {
  const int nx = c->nx, ny = c->ny;
  const size_t n = c->n;
  const double ht = c->cfg.h_tol;
  memcpy(out, S, 9 * n * sizeof(double));
#pragma omp parallel for schedule(static)
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      size_t k = (size_t)j * nx + i;
      c->flat[k] = 0;
      if (S[PL(0, 0) * n + k] <= 0.0) {
        for (int p = 0; p < 9; ++p) out[p * n + k] = 0.0;
        c->flat[k] = 1;
        continue;
      }
      int front = S[PL(0, 0) * n + k] <= ht;
      if (i > 0 && S[PL(0, 0) * n + k - 1] <= ht) front = 1;
      if (i < nx - 1 && S[PL(0, 0) * n + k + 1] <= ht) front = 1;
      if (j > 0 && S[PL(0, 0) * n + k - nx] <= ht) front = 1;
      if (j < ny - 1 && S[PL(0, 0) * n + k + nx] <= ht) front = 1;
      if (front) {
        for (int var = 0; var < 3; ++var) {
          out[PL(var, 1) * n + k] = 0.0;
          out[PL(var, 2) * n + k] = 0.0;
        }
        c->flat[k] = 1;
        continue;
      }
      if (c->cfg.limiter)
      for (int d = 1; d <= 2; ++d) {
        size_t km, kp; /* neighbours in direction d, the cell itself at an edge */
        int at_lo, at_hi;
        double zlo, zhi; /* the cell's bed at its low and high faces in direction d */
        if (d == 1) {
          km = (size_t)j * nx + (i > 0 ? i - 1 : i);
          kp = (size_t)j * nx + (i < nx - 1 ? i + 1 : i);
          at_lo = i == 0;
          at_hi = i == nx - 1;
          zlo = zface_x(c, i, j);
          zhi = zface_x(c, i + 1, j);
        } else {
          km = (size_t)(j > 0 ? j - 1 : j) * nx + i;
          kp = (size_t)(j < ny - 1 ? j + 1 : j) * nx + i;
          at_lo = j == 0;
          at_hi = j == ny - 1;
          zlo = zface_y(c, i, j);
          zhi = zface_y(c, i, j + 1);
        }
        const double *zs = (d == 1) ? c->z1x : c->z1y;
        /* eta; beyond an edge the ghost cell has the edge cell's depth on the edge
           cell's bed plane continued one cell out (its centre lies zhi - zlo above or
           below z0), so a free surface parallel to a sloping bed stays unlimited */
        double e0 = S[PL(0, 0) * n + k] + c->z0[k];
        double em = at_lo ? S[PL(0, 0) * n + k] + (c->z0[k] - (zhi - zlo))
                          : S[PL(0, 0) * n + km] + c->z0[km];
        double ep = at_hi ? S[PL(0, 0) * n + k] + (c->z0[k] + (zhi - zlo))
                          : S[PL(0, 0) * n + kp] + c->z0[kp];
        double e1 = S[PL(0, d) * n + k] + zs[k];
        double le = minmod3(e1, (ep - e0) / SQRT3, (e0 - em) / SQRT3);
        if (le != e1) out[PL(0, d) * n + k] = le - zs[k];
        /* discharges */
        for (int var = 1; var <= 2; ++var) {
          double a0 = S[PL(var, 0) * n + k];
          double am = S[PL(var, 0) * n + km], ap = S[PL(var, 0) * n + kp];
          out[PL(var, d) * n + k] = minmod3(S[PL(var, d) * n + k], (ap - a0) / SQRT3, (a0 - am) / SQRT3);
        }
      }
      /* a depth plane that is negative at a face centre marks a wet/dry front inside
         the cell: it is made first order like the front cells above */
      {
        const double h0 = out[PL(0, 0) * n + k];
        const double ax = SQRT3 * fabs(out[PL(0, 1) * n + k]), ay = SQRT3 * fabs(out[PL(0, 2) * n + k]);
        if (h0 - ax < 0.0 || h0 - ay < 0.0) {
          for (int var = 0; var < 3; ++var) {
            out[PL(var, 1) * n + k] = 0.0;
            out[PL(var, 2) * n + k] = 0.0;
          }
          c->flat[k] = 1;
        }
      }
    }
}

int dg2ref_limit(dg2ref_ctx *c, const double *state, double *out) {
  pass_limit(c, state, out);
  return DG2REF_OK;
}

int dg2ref_friction(dg2ref_ctx *c, const double *state, double dt, double *out) {
  if (!c || !state || !out || !(dt >= 0.0)) return DG2REF_E_ARG;
  pass_friction(c, state, dt, out);
  return DG2REF_OK;
}

/* ------------------------------------------------------------------------------ */
/* Face states, wet/dry revision and HLL flux.                                      */
/* ------------------------------------------------------------------------------ */

/* Revision of one side's limit (h, qx, qy) at a face (Sect. 2.1.1: temporary
 * revisions for well-balancedness and non-negative depth). zb is this side's bed at
 * the face (the vertex mean of eq 8, or z0 for a first-order front cell) and zs = z*
 * the larger of the two sides' values. Reading: h* = max(0, eta - z*); velocities
 * from the unrevised depth, zero at or below h_tol; the revised bed seen from this
 * side is z** = min(z*, eta), so h* + z** = eta on every side. */
static side_t revise(double h, double qx, double qy, double zb, double zs, double h_tol) {
  side_t s;
  double eta = h + zb;
  double d = eta - zs;
  s.h = d > 0.0 ? d : 0.0;
  s.u = h > h_tol ? qx / h : 0.0;
  s.v = h > h_tol ? qy / h : 0.0;
  s.z = eta < zs ? eta : zs;
  return s;
}

/* HLL flux with the wave-speed estimates of Toro's textbook (two-rarefaction speeds
 * for wet-wet faces, the dry-bed front speeds when one side is dry). The paper names
 * only the HLL solver. */
void dg2ref_hll(double g, double hL, double unL, double utL, double hR, double unR,
                double utR, double out[3]) {
  if (hL <= 0.0 && hR <= 0.0) {
    out[0] = out[1] = out[2] = 0.0;
    return;
  }
  double cL = sqrt(g * hL), cR = sqrt(g * hR);
  double sL, sR;
  if (hL <= 0.0) {
    sL = unR - 2.0 * cR;
    sR = unR + cR;
  } else if (hR <= 0.0) {
    sL = unL - cL;
    sR = unL + 2.0 * cL;
  } else {
    double us = 0.5 * (unL + unR) + cL - cR;
    double cs = 0.5 * (cL + cR) + 0.25 * (unL - unR);
    sL = fmin(unL - cL, us - cs);
    sR = fmax(unR + cR, us + cs);
  }
  double FL[3] = {hL * unL, hL * unL * unL + 0.5 * g * hL * hL, hL * unL * utL};
  double FR[3] = {hR * unR, hR * unR * unR + 0.5 * g * hR * hR, hR * unR * utR};
  if (sL >= 0.0) {
    memcpy(out, FL, sizeof FL);
    return;
  }
  if (sR <= 0.0) {
    memcpy(out, FR, sizeof FR);
    return;
  }
  double UL[3] = {hL, hL * unL, hL * utL};
  double UR[3] = {hR, hR * unR, hR * utR};
  for (int m = 0; m < 3; ++m)
    out[m] = (sR * FL[m] - sL * FR[m] + sL * sR * (UR[m] - UL[m])) / (sR - sL);
}

/* physical flux of a state (h, un, ut) through a face with normal n:
 * [h un, h un^2 + g h^2 / 2, h un ut] */
static void phys_flux(double g, double h, double un, double ut, double o[3]) {
  o[0] = h * un;
  o[1] = h * un * un + 0.5 * g * h * h;
  o[2] = h * un * ut;
}

/* mean velocity of a cell, zero at or below h_tol */
static double mean_vel(const double *S, size_t n, size_t k, int var, double ht) {
  double h0 = S[PL(0, 0) * n + k];
  return h0 > ht ? S[PL(var, 0) * n + k] / h0 : 0.0;
}

static double capd(double x, double a, double b, double slack) {
  double m = (fabs(a) > fabs(b) ? fabs(a) : fabs(b)) + slack;
  return x > m ? m : (x < -m ? -m : x);
}

/* Reading: each velocity component of a face limit is capped in magnitude by the
 * larger magnitude of that component's mean velocity in the two cells sharing the
 * face (a cell across a boundary face counts as a copy of the interior cell), plus
 * sqrt(g h_tol), the velocity scale of the dry tolerance. Depth and discharge planes
 * are limited separately, so where the depth plane nears zero at a face their ratio
 * is otherwise unbounded. */
static void clamp_side(side_t *s, double ua, double va, double ub, double vb, double slack) {
  s->u = capd(s->u, ua, ub, slack);
  s->v = capd(s->v, va, vb, slack);
}

/* inflow hydrograph Q(t): piecewise linear between knots, held beyond the ends */
static double hydro(const seg_t *s, double t) {
  int n = s->n_knots;
  if (n <= 0) return 0.0;
  if (t <= s->t_knots[0]) return s->q_knots[0];
  if (t >= s->t_knots[n - 1]) return s->q_knots[n - 1];
  int k = 0;
  while (k + 1 < n && s->t_knots[k + 1] <= t) ++k;
  double a = (t - s->t_knots[k]) / (s->t_knots[k + 1] - s->t_knots[k]);
  return s->q_knots[k] + a * (s->q_knots[k + 1] - s->q_knots[k]);
}

/* Ghost state outside a boundary face, from the interior side's revised state
 * (h, un, ut) written in the face's normal frame with the normal along +x or +y.
 * inward = +1 on the W and S edges, -1 on the E and N edges. Reading of the
 * unspecified boundary treatment: transmissive copies, a wall reflects the normal
 * velocity, a fixed state is imposed, and an inflow of Q(t) spread over the segment
 * enters at the larger of the interior depth and the critical depth of that
 * discharge. The face flux is the HLL flux between the ghost and the interior side,
 * except at an inflow face, which carries the inflow state's own physical flux: the
 * hydrograph is then imposed exactly (mass flux Q(t) / width through every face of
 * the segment) with the interior depth in the pressure term. */
static void ghost(const dg2ref_ctx *c, const bface_t *b, double t, int normal_is_x,
                  double inward, double h, double un, double ut, double *gh, double *gun,
                  double *gut) {
  *gh = h;
  *gun = un;
  *gut = ut;
  if (b->kind == DG2REF_BC_WALL) {
    *gun = -un;
  } else if (b->kind == DG2REF_BC_FIXED) {
    const seg_t *s = &c->segs[b->seg];
    *gh = s->h_b;
    *gun = normal_is_x ? s->u_b : s->v_b;
    *gut = normal_is_x ? s->v_b : s->u_b;
  } else if (b->kind == DG2REF_BC_INFLOW) {
    const seg_t *s = &c->segs[b->seg];
    double width = (double)(s->i1 - s->i0) * c->cfg.dx;
    double qn = hydro(s, t) / width;
    double hc = cbrt(qn * qn / c->cfg.g);
    double hg = h > hc ? h : hc;
    *gh = hg;
    *gun = hg > 0.0 ? inward * (qn / hg) : 0.0;
    *gut = 0.0;
  }
}

/* all face states and fluxes of a (limited) coefficient state at stage time t;
 * returns the boundary inflow and outflow rates (m^3/s) */
static void pass_faces(dg2ref_ctx *c, const double *S, double t, double *in_rate,
                       double *out_rate) {
  const int nx = c->nx, ny = c->ny;
  const size_t n = c->n;
  const double g = c->cfg.g, ht = c->cfg.h_tol;
  const double slack = sqrt(g * ht);
#pragma omp parallel for schedule(static)
  for (int j = 0; j < ny; ++j)
    for (int f = 0; f <= nx; ++f) {
      face_t *fc = &c->xf[(size_t)j * (nx + 1) + f];
      double zf = zface_x(c, f, j);
      size_t kl = (size_t)j * nx + (f - 1), kr = (size_t)j * nx + f;
      double zl = f > 0 ? (c->flat[kl] ? c->z0[kl] : zf) : zf;
      double zr = f < nx ? (c->flat[kr] ? c->z0[kr] : zf) : zf;
      if (f == 0) zl = zr;
      if (f == nx) zr = zl;
      double zs = zl > zr ? zl : zr;
      if (f > 0) { /* east limit of cell f-1 */
        size_t k = kl;
        double h = S[PL(0, 0) * n + k] + SQRT3 * S[PL(0, 1) * n + k];
        double qx = S[PL(1, 0) * n + k] + SQRT3 * S[PL(1, 1) * n + k];
        double qy = S[PL(2, 0) * n + k] + SQRT3 * S[PL(2, 1) * n + k];
        fc->lo = revise(h, qx, qy, zl, zs, ht);
      }
      if (f < nx) { /* west limit of cell f */
        size_t k = kr;
        double h = S[PL(0, 0) * n + k] - SQRT3 * S[PL(0, 1) * n + k];
        double qx = S[PL(1, 0) * n + k] - SQRT3 * S[PL(1, 1) * n + k];
        double qy = S[PL(2, 0) * n + k] - SQRT3 * S[PL(2, 1) * n + k];
        fc->hi = revise(h, qx, qy, zr, zs, ht);
      }
      {
        size_t ka = f > 0 ? kl : kr, kb = f < nx ? kr : kl;
        double ua = mean_vel(S, n, ka, 1, ht), va = mean_vel(S, n, ka, 2, ht);
        double ub = mean_vel(S, n, kb, 1, ht), vb = mean_vel(S, n, kb, 2, ht);
        if (f > 0) clamp_side(&fc->lo, ua, va, ub, vb, slack);
        if (f < nx) clamp_side(&fc->hi, ua, va, ub, vb, slack);
      }
      double gh, gu, gv;
      if (f == 0) {
        ghost(c, &c->bw[j], t, 1, 1.0, fc->hi.h, fc->hi.u, fc->hi.v, &gh, &gu, &gv);
        fc->lo.h = gh; fc->lo.u = gu; fc->lo.v = gv; fc->lo.z = zs;
      } else if (f == nx) {
        ghost(c, &c->be[j], t, 1, -1.0, fc->lo.h, fc->lo.u, fc->lo.v, &gh, &gu, &gv);
        fc->hi.h = gh; fc->hi.u = gu; fc->hi.v = gv; fc->hi.z = zs;
      }
      /* normal = x: (h, u, v); an inflow face carries the inflow state's own flux */
      if (f == 0 && c->bw[j].kind == DG2REF_BC_INFLOW)
        phys_flux(g, fc->lo.h, fc->lo.u, fc->lo.v, fc->flux);
      else if (f == nx && c->be[j].kind == DG2REF_BC_INFLOW)
        phys_flux(g, fc->hi.h, fc->hi.u, fc->hi.v, fc->flux);
      else
        dg2ref_hll(g, fc->lo.h, fc->lo.u, fc->lo.v, fc->hi.h, fc->hi.u, fc->hi.v, fc->flux);
    }
#pragma omp parallel for schedule(static)
  for (int f = 0; f <= ny; ++f)
    for (int i = 0; i < nx; ++i) {
      face_t *fc = &c->yf[(size_t)f * nx + i];
      double zf = zface_y(c, i, f);
      size_t kl = (size_t)(f - 1) * nx + i, kr = (size_t)f * nx + i;
      double zl = f > 0 ? (c->flat[kl] ? c->z0[kl] : zf) : zf;
      double zr = f < ny ? (c->flat[kr] ? c->z0[kr] : zf) : zf;
      if (f == 0) zl = zr;
      if (f == ny) zr = zl;
      double zs = zl > zr ? zl : zr;
      if (f > 0) { /* north limit of cell (i, f-1) */
        size_t k = kl;
        double h = S[PL(0, 0) * n + k] + SQRT3 * S[PL(0, 2) * n + k];
        double qx = S[PL(1, 0) * n + k] + SQRT3 * S[PL(1, 2) * n + k];
        double qy = S[PL(2, 0) * n + k] + SQRT3 * S[PL(2, 2) * n + k];
        fc->lo = revise(h, qx, qy, zl, zs, ht);
      }
      if (f < ny) { /* south limit of cell (i, f) */
        size_t k = kr;
        double h = S[PL(0, 0) * n + k] - SQRT3 * S[PL(0, 2) * n + k];
        double qx = S[PL(1, 0) * n + k] - SQRT3 * S[PL(1, 2) * n + k];
        double qy = S[PL(2, 0) * n + k] - SQRT3 * S[PL(2, 2) * n + k];
        fc->hi = revise(h, qx, qy, zr, zs, ht);
      }
      {
        size_t ka = f > 0 ? kl : kr, kb = f < ny ? kr : kl;
        double ua = mean_vel(S, n, ka, 1, ht), va = mean_vel(S, n, ka, 2, ht);
        double ub = mean_vel(S, n, kb, 1, ht), vb = mean_vel(S, n, kb, 2, ht);
        if (f > 0) clamp_side(&fc->lo, ua, va, ub, vb, slack);
        if (f < ny) clamp_side(&fc->hi, ua, va, ub, vb, slack);
      }
      double gh, gn, gt;
      if (f == 0) {
        ghost(c, &c->bs[i], t, 0, 1.0, fc->hi.h, fc->hi.v, fc->hi.u, &gh, &gn, &gt);
        fc->lo.h = gh; fc->lo.v = gn; fc->lo.u = gt; fc->lo.z = zs;
      } else if (f == ny) {
        ghost(c, &c->bn[i], t, 0, -1.0, fc->lo.h, fc->lo.v, fc->lo.u, &gh, &gn, &gt);
        fc->hi.h = gh; fc->hi.v = gn; fc->hi.u = gt; fc->hi.z = zs;
      }
      /* normal = y: the normal velocity is v, the tangential one u */
      double o[3];
      if (f == 0 && c->bs[i].kind == DG2REF_BC_INFLOW)
        phys_flux(g, fc->lo.h, fc->lo.v, fc->lo.u, o);
      else if (f == ny && c->bn[i].kind == DG2REF_BC_INFLOW)
        phys_flux(g, fc->hi.h, fc->hi.v, fc->hi.u, o);
      else
        dg2ref_hll(g, fc->lo.h, fc->lo.v, fc->lo.u, fc->hi.h, fc->hi.v, fc->hi.u, o);
      fc->flux[0] = o[0];
      fc->flux[1] = o[2]; /* x-momentum is tangential here */
      fc->flux[2] = o[1];
    }
  /* boundary mass rates, summed in a fixed order */
  double rin = 0.0, rout = 0.0;
  const double dx = c->cfg.dx;
  for (int j = 0; j < ny; ++j) {
    double fw = c->xf[(size_t)j * (nx + 1) + 0].flux[0] * dx;  /* into the domain if > 0 */
    double fe = -c->xf[(size_t)j * (nx + 1) + nx].flux[0] * dx; /* into the domain if > 0 */
    if (fw > 0) rin += fw; else rout -= fw;
    if (fe > 0) rin += fe; else rout -= fe;
  }
  for (int i = 0; i < nx; ++i) {
    double fs = c->yf[(size_t)0 * nx + i].flux[0] * dx;
    double fn = -c->yf[(size_t)ny * nx + i].flux[0] * dx;
    if (fs > 0) rin += fs; else rout -= fs;
    if (fn > 0) rin += fn; else rout -= fn;
  }
  *in_rate = rin;
  *out_rate = rout;
}

/* physical flux along a normal at a Gauss point, velocities desingularised at h_tol:
 * [h un, h un^2 + g h^2 / 2, h un ut] */
static void flux_n(double g, double ht, double h, double qn, double qt, double o[3]) {
  double un = h > ht ? qn / h : 0.0;
  double ut = h > ht ? qt / h : 0.0;
  o[0] = h * un;
  o[1] = h * un * un + 0.5 * g * h * h;
  o[2] = h * un * ut;
}

/* ------------------------------------------------------------------------------ */
/* Spatial operator L = [L0, L1x, L1y] (eq 4; Sect. 2.1.1). Reading: the DG weak    */
/* form with the scaled Legendre basis of eq 2, the HLL flux at the face centres and */
/* a 2-point Gauss rule for the volume flux, slope-decoupled (L1x has only x terms,  */
/* L1y only y terms), evaluated on the cell coefficients rebuilt from the revised    */
/* face values: Ubar0 = (U_E* + U_W*)/2, Ubar1x = (U_E* - U_W*)/(2 sqrt3), and the   */
/* bed slope zbar1x = (z_E** - z_W**)/(2 sqrt3). The bed source is -g h dz/dx        */
/* projected on the basis: -2 sqrt3 g hbar zbar1 / dx.                               */
/* ------------------------------------------------------------------------------ */
static void pass_operator(dg2ref_ctx *c, double *L) {
  const int nx = c->nx, ny = c->ny;
  const size_t n = c->n;
  const double g = c->cfg.g, ht = c->cfg.h_tol, dx = c->cfg.dx;
#pragma omp parallel for schedule(static)
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      size_t k = (size_t)j * nx + i;
      double l[9] = {0};
      /* x direction: own side of the west face is its 'hi', of the east face its 'lo' */
      {
        const face_t *fw = &c->xf[(size_t)j * (nx + 1) + i];
        const face_t *fe = &c->xf[(size_t)j * (nx + 1) + i + 1];
        const side_t *W = &fw->hi, *E = &fe->lo;
        double hb0 = 0.5 * (E->h + W->h), hb1 = (E->h - W->h) / (2.0 * SQRT3);
        double qxE = E->h * E->u, qxW = W->h * W->u, qyE = E->h * E->v, qyW = W->h * W->v;
        double qb0 = 0.5 * (qxE + qxW), qb1 = (qxE - qxW) / (2.0 * SQRT3);
        double rb0 = 0.5 * (qyE + qyW), rb1 = (qyE - qyW) / (2.0 * SQRT3);
        double zb1 = (E->z - W->z) / (2.0 * SQRT3);
        double Fp[3], Fm[3];
        flux_n(g, ht, hb0 + hb1, qb0 + qb1, rb0 + rb1, Fp);
        flux_n(g, ht, hb0 - hb1, qb0 - qb1, rb0 - rb1, Fm);
        /* Fp/Fm are [mass, x-mom, y-mom] since the normal is x */
        l[PL(0, 0)] += -(fe->flux[0] - fw->flux[0]) / dx;
        l[PL(1, 0)] += -(fe->flux[1] - fw->flux[1]) / dx - 2.0 * SQRT3 * g * hb0 * zb1 / dx;
        l[PL(2, 0)] += -(fe->flux[2] - fw->flux[2]) / dx;
        l[PL(0, 1)] = -(SQRT3 / dx) * (fe->flux[0] + fw->flux[0] - Fp[0] - Fm[0]);
        l[PL(1, 1)] = -(SQRT3 / dx) * (fe->flux[1] + fw->flux[1] - Fp[1] - Fm[1]) -
                      2.0 * SQRT3 * g * hb1 * zb1 / dx;
        l[PL(2, 1)] = -(SQRT3 / dx) * (fe->flux[2] + fw->flux[2] - Fp[2] - Fm[2]);
      }
      /* y direction */
      {
        const face_t *fs = &c->yf[(size_t)j * nx + i];
        const face_t *fn = &c->yf[(size_t)(j + 1) * nx + i];
        const side_t *S = &fs->hi, *N = &fn->lo;
        double hb0 = 0.5 * (N->h + S->h), hb1 = (N->h - S->h) / (2.0 * SQRT3);
        double qxN = N->h * N->u, qxS = S->h * S->u, qyN = N->h * N->v, qyS = S->h * S->v;
        double qb0 = 0.5 * (qxN + qxS), qb1 = (qxN - qxS) / (2.0 * SQRT3);
        double rb0 = 0.5 * (qyN + qyS), rb1 = (qyN - qyS) / (2.0 * SQRT3);
        double zb1 = (N->z - S->z) / (2.0 * SQRT3);
        double Gp[3], Gm[3]; /* [mass, y-mom (normal), x-mom (tangential)] */
        flux_n(g, ht, hb0 + hb1, rb0 + rb1, qb0 + qb1, Gp);
        flux_n(g, ht, hb0 - hb1, rb0 - rb1, qb0 - qb1, Gm);
        l[PL(0, 0)] += -(fn->flux[0] - fs->flux[0]) / dx;
        l[PL(1, 0)] += -(fn->flux[1] - fs->flux[1]) / dx;
        l[PL(2, 0)] += -(fn->flux[2] - fs->flux[2]) / dx - 2.0 * SQRT3 * g * hb0 * zb1 / dx;
        l[PL(0, 2)] = -(SQRT3 / dx) * (fn->flux[0] + fs->flux[0] - Gp[0] - Gm[0]);
        l[PL(1, 2)] = -(SQRT3 / dx) * (fn->flux[1] + fs->flux[1] - Gp[2] - Gm[2]);
        l[PL(2, 2)] = -(SQRT3 / dx) * (fn->flux[2] + fs->flux[2] - Gp[1] - Gm[1]) -
                      2.0 * SQRT3 * g * hb1 * zb1 / dx;
      }
      for (int p = 0; p < 9; ++p) L[p * n + k] = l[p];
    }
}

int dg2ref_operator(dg2ref_ctx *c, const double *state, double t, double *L,
                    double *inflow_rate, double *outflow_rate) {
  double ri, ro;
  pass_limit(c, state, c->W); /* only for the front flags of this state */
  pass_faces(c, state, t, &ri, &ro);
  pass_operator(c, L);
  if (inflow_rate) *inflow_rate = ri;
  if (outflow_rate) *outflow_rate = ro;
  return DG2REF_OK;
}

/* After each stage: a negative mean depth is set to zero with its slopes (the mass
 * added is booked as clip mass), and a cell with h0 <= h_tol loses its discharge. */
static double pass_cleanup(dg2ref_ctx *c, double *S, int *bad) {
  const size_t n = c->n;
  const int nx = c->nx, ny = c->ny;
  const double area = c->cfg.dx * c->cfg.dx, ht = c->cfg.h_tol;
  int nan_seen = 0;
#pragma omp parallel for schedule(static) reduction(| : nan_seen)
  for (int j = 0; j < ny; ++j) {
    double clip = 0.0; /* the clipped mass of row j, summed along the row */
    for (int i = 0; i < nx; ++i) {
      size_t k = (size_t)j * nx + i;
      for (int p = 0; p < 9; ++p)
        if (isnan(S[p * n + k])) nan_seen |= 1;
      double h0 = S[PL(0, 0) * n + k];
      if (h0 < 0.0) {
        clip += -h0 * area;
        S[PL(0, 0) * n + k] = 0.0;
        S[PL(0, 1) * n + k] = 0.0;
        S[PL(0, 2) * n + k] = 0.0;
        h0 = 0.0;
      }
      if (h0 <= ht)
        for (int p = 3; p < 9; ++p) S[p * n + k] = 0.0;
    }
    c->rowsum[j] = clip;
  }
  double clip = 0.0; /* rows in order: the same sum on any number of threads */
  for (int j = 0; j < ny; ++j) clip += c->rowsum[j];
  *bad = nan_seen;
  return clip;
}

/* ------------------------------------------------------------------------------ */
/* CFL time step (Sect. 2.1.1, Courant number 0.33). Reading: over cells with       */
/* h0 > h_tol, dx / (|u0| + sqrt(g h)) per direction with the mean velocity u0 and  */
/* the largest depth among the mean and the two face-centre limits in that          */
/* direction (face velocities never exceed the neighbouring mean velocities, see    */
/* the revision); boundary forcing (the critical-depth inflow state, a fixed state) */
/* also bounds it; dt_dry if nothing does.                                          */
/* ------------------------------------------------------------------------------ */
static double cfl_dt(const dg2ref_ctx *c, const double *S, double t) {
  const size_t n = c->n;
  const double g = c->cfg.g, ht = c->cfg.h_tol, dx = c->cfg.dx;
  double m = INFINITY;
#pragma omp parallel for schedule(static) reduction(min : m)
  for (size_t k = 0; k < n; ++k) {
    double h0 = S[PL(0, 0) * n + k];
    if (!(h0 > ht)) continue;
    for (int d = 1; d <= 2; ++d) { /* d = 1: x (velocity qx0/h0), d = 2: y (qy0/h0) */
      double h1 = SQRT3 * fabs(S[PL(0, d) * n + k]);
      double hmax = h0 + h1;
      double u = S[PL(d, 0) * n + k] / h0;
      double a = dx / (fabs(u) + sqrt(g * hmax));
      if (a < m) m = a;
    }
  }
  for (int s = 0; s < c->n_segs; ++s) {
    const seg_t *sg = &c->segs[s];
    if (sg->kind == DG2REF_BC_INFLOW) {
      double qn = hydro(sg, t) / ((double)(sg->i1 - sg->i0) * dx);
      if (qn > 0.0) {
        double hc = cbrt(qn * qn / g);
        if (hc > ht) {
          double a = dx / (qn / hc + sqrt(g * hc));
          if (a < m) m = a;
        }
      }
    } else if (sg->kind == DG2REF_BC_FIXED && sg->h_b > ht) {
      double cw = sqrt(g * sg->h_b);
      double a = dx / (fabs(sg->u_b) + cw), b = dx / (fabs(sg->v_b) + cw);
      if (a < m) m = a;
      if (b < m) m = b;
    }
  }
  if (m == INFINITY) return c->cfg.dt_dry;
  return c->cfg.cfl * m;
}

/* ------------------------------------------------------------------------------ */
/* One step: friction at the start of the step, then the two RK2 stages of eq 4.    */
/* Reading: every stage input is limited first (U^n after friction gives V^n, U^int */
/* gives V^int), and the stage-2 combination uses the limited values (the           */
/* Cockburn-Shu form): U^int = V^n + dt L(V^n), U^{n+1} = (V^n + V^int +            */
/* dt L(V^int)) / 2.                                                                */
/* ------------------------------------------------------------------------------ */
static int do_step(dg2ref_ctx *c, double dt_max, double t_end, double *dt_used) {
  const size_t n = c->n;
  double dt = c->dt_next;
  if (dt_max > 0.0 && dt_max < dt) dt = dt_max;
  double t_next = c->t + dt;
  if (t_end - c->t <= dt) {
    dt = t_end - c->t;
    t_next = t_end;
  }
  if (!(dt > 0.0)) return fail(c, DG2REF_E_NUMERIC, "non-positive time step %g at t=%g", dt, c->t);
  pass_friction(c, c->U, dt, c->F);
  pass_limit(c, c->F, c->V);
  double in1, out1, in2, out2;
  int bad1 = 0, bad2 = 0;
  pass_faces(c, c->V, c->t, &in1, &out1);
  pass_operator(c, c->L);
#pragma omp parallel for schedule(static)
  for (size_t m = 0; m < 9 * n; ++m) c->Ui[m] = c->V[m] + dt * c->L[m];
  double clip1 = pass_cleanup(c, c->Ui, &bad1);
  pass_limit(c, c->Ui, c->W);
  pass_faces(c, c->W, t_next, &in2, &out2);
  pass_operator(c, c->L);
#pragma omp parallel for schedule(static)
  for (size_t m = 0; m < 9 * n; ++m) c->U[m] = 0.5 * (c->V[m] + c->W[m] + dt * c->L[m]);
  double clip2 = pass_cleanup(c, c->U, &bad2);
  c->mass_in += 0.5 * dt * (in1 + in2);
  c->mass_out += 0.5 * dt * (out1 + out2);
  c->mass_clip += 0.5 * clip1 + clip2;
  c->t = t_next;
  c->step += 1;
  c->dt_next = cfl_dt(c, c->U, c->t);
  if (dt_used) *dt_used = dt;
  if (bad1 || bad2) return fail(c, DG2REF_E_NUMERIC, "NaN in state at step %lld", (long long)c->step);
  return DG2REF_OK;
}

/* ------------------------------------------------------------------------------ */
/* FV1 (Sect. 2.1.2, eq 5-7): h, qx, qy and the bed are constant per cell (the      */
/* means; the bed is z0 of eq 8). The operator keeps only L0, built from the HLL     */
/* fluxes of the two cell means at each face, and eq 7 advances the means by one     */
/* forward-Euler step with Courant number 0.5. Friction is applied first, at the    */
/* cell centre, as in DG2. Reading: the faces get the same temporary revision as    */
/* DG2 (here with the two cells' own flat beds: z* = max, h* = max(0, eta - z*),    */
/* per-side z** = min(z*, eta)) and the bed source of L0 in its FV1 form,           */
/* -g (hE* + hW*)/2 (zE** - zW**)/dx, which keeps still water still exactly.        */
/* ------------------------------------------------------------------------------ */
static void fv1_faces(dg2ref_ctx *c, const double *S, double t, double *in_rate,
                      double *out_rate) {
  const int nx = c->nx, ny = c->ny;
  const size_t n = c->n;
  const double g = c->cfg.g, ht = c->cfg.h_tol;
  const double *h = S + PL(0, 0) * n, *qx = S + PL(1, 0) * n, *qy = S + PL(2, 0) * n;
#pragma omp parallel for schedule(static)
  for (int j = 0; j < ny; ++j)
    for (int f = 0; f <= nx; ++f) {
      face_t *fc = &c->xf[(size_t)j * (nx + 1) + f];
      size_t kl = (size_t)j * nx + (f - 1), kr = (size_t)j * nx + f;
      double zl = f > 0 ? c->z0[kl] : c->z0[kr];
      double zr = f < nx ? c->z0[kr] : c->z0[kl];
      double zs = zl > zr ? zl : zr;
      if (f > 0) fc->lo = revise(h[kl], qx[kl], qy[kl], zl, zs, ht);
      if (f < nx) fc->hi = revise(h[kr], qx[kr], qy[kr], zr, zs, ht);
      double gh, gu, gv;
      if (f == 0) {
        ghost(c, &c->bw[j], t, 1, 1.0, fc->hi.h, fc->hi.u, fc->hi.v, &gh, &gu, &gv);
        fc->lo.h = gh; fc->lo.u = gu; fc->lo.v = gv; fc->lo.z = zs;
      } else if (f == nx) {
        ghost(c, &c->be[j], t, 1, -1.0, fc->lo.h, fc->lo.u, fc->lo.v, &gh, &gu, &gv);
        fc->hi.h = gh; fc->hi.u = gu; fc->hi.v = gv; fc->hi.z = zs;
      }
      if (f == 0 && c->bw[j].kind == DG2REF_BC_INFLOW)
        phys_flux(g, fc->lo.h, fc->lo.u, fc->lo.v, fc->flux);
      else if (f == nx && c->be[j].kind == DG2REF_BC_INFLOW)
        phys_flux(g, fc->hi.h, fc->hi.u, fc->hi.v, fc->flux);
      else
        dg2ref_hll(g, fc->lo.h, fc->lo.u, fc->lo.v, fc->hi.h, fc->hi.u, fc->hi.v, fc->flux);
    }
#pragma omp parallel for schedule(static)
  for (int f = 0; f <= ny; ++f)
    for (int i = 0; i < nx; ++i) {
      face_t *fc = &c->yf[(size_t)f * nx + i];
      size_t kl = (size_t)(f - 1) * nx + i, kr = (size_t)f * nx + i;
      double zl = f > 0 ? c->z0[kl] : c->z0[kr];
      double zr = f < ny ? c->z0[kr] : c->z0[kl];
      double zs = zl > zr ? zl : zr;
      if (f > 0) fc->lo = revise(h[kl], qx[kl], qy[kl], zl, zs, ht);
      if (f < ny) fc->hi = revise(h[kr], qx[kr], qy[kr], zr, zs, ht);
      double gh, gn, gt;
      if (f == 0) {
        ghost(c, &c->bs[i], t, 0, 1.0, fc->hi.h, fc->hi.v, fc->hi.u, &gh, &gn, &gt);
        fc->lo.h = gh; fc->lo.v = gn; fc->lo.u = gt; fc->lo.z = zs;
      } else if (f == ny) {
        ghost(c, &c->bn[i], t, 0, -1.0, fc->lo.h, fc->lo.v, fc->lo.u, &gh, &gn, &gt);
        fc->hi.h = gh; fc->hi.v = gn; fc->hi.u = gt; fc->hi.z = zs;
      }
      double o[3];
      if (f == 0 && c->bs[i].kind == DG2REF_BC_INFLOW)
        phys_flux(g, fc->lo.h, fc->lo.v, fc->lo.u, o);
      else if (f == ny && c->bn[i].kind == DG2REF_BC_INFLOW)
        phys_flux(g, fc->hi.h, fc->hi.v, fc->hi.u, o);
      else
        dg2ref_hll(g, fc->lo.h, fc->lo.v, fc->lo.u, fc->hi.h, fc->hi.v, fc->hi.u, o);
      fc->flux[0] = o[0];
      fc->flux[1] = o[2];
      fc->flux[2] = o[1];
    }
  double rin = 0.0, rout = 0.0;
  const double dx = c->cfg.dx;
  for (int j = 0; j < ny; ++j) {
    double fw = c->xf[(size_t)j * (nx + 1) + 0].flux[0] * dx;
    double fe = -c->xf[(size_t)j * (nx + 1) + nx].flux[0] * dx;
    if (fw > 0) rin += fw; else rout -= fw;
    if (fe > 0) rin += fe; else rout -= fe;
  }
  for (int i = 0; i < nx; ++i) {
    double fs = c->yf[(size_t)0 * nx + i].flux[0] * dx;
    double fn = -c->yf[(size_t)ny * nx + i].flux[0] * dx;
    if (fs > 0) rin += fs; else rout -= fs;
    if (fn > 0) rin += fn; else rout -= fn;
  }
  *in_rate = rin;
  *out_rate = rout;
}

static int do_step_fv1(dg2ref_ctx *c, double dt_max, double t_end, double *dt_used) {
  const size_t n = c->n;
  const int nx = c->nx, ny = c->ny;
  const double g = c->cfg.g, ht = c->cfg.h_tol, dx = c->cfg.dx;
  double dt = c->dt_next;
  if (dt_max > 0.0 && dt_max < dt) dt = dt_max;
  double t_next = c->t + dt;
  if (t_end - c->t <= dt) {
    dt = t_end - c->t;
    t_next = t_end;
  }
  if (!(dt > 0.0)) return fail(c, DG2REF_E_NUMERIC, "non-positive time step %g at t=%g", dt, c->t);
  /* friction at the centre: F = U with q replaced by the friction update */
  memcpy(c->F, c->U, 9 * n * sizeof(double));
#pragma omp parallel for schedule(static)
  for (size_t k = 0; k < n; ++k) {
    double q[2];
    dg2ref_friction_point(g, c->manning[k], ht, dt, c->U[PL(0, 0) * n + k],
                          c->U[PL(1, 0) * n + k], c->U[PL(2, 0) * n + k], q);
    c->F[PL(1, 0) * n + k] = q[0];
    c->F[PL(2, 0) * n + k] = q[1];
  }
  double in, out;
  fv1_faces(c, c->F, c->t, &in, &out);
  /* eq 7 with L0: flux differences and the bed source of each direction */
#pragma omp parallel for schedule(static)
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      size_t k = (size_t)j * nx + i;
      const face_t *fw = &c->xf[(size_t)j * (nx + 1) + i], *fe = &c->xf[(size_t)j * (nx + 1) + i + 1];
      const face_t *fs = &c->yf[(size_t)j * nx + i], *fn = &c->yf[(size_t)(j + 1) * nx + i];
      const side_t *W = &fw->hi, *E = &fe->lo, *Sd = &fs->hi, *N = &fn->lo;
      double l0 = -(fe->flux[0] - fw->flux[0]) / dx - (fn->flux[0] - fs->flux[0]) / dx;
      double l1 = -(fe->flux[1] - fw->flux[1]) / dx - (fn->flux[1] - fs->flux[1]) / dx -
                  g * 0.5 * (E->h + W->h) * (E->z - W->z) / dx;
      double l2 = -(fe->flux[2] - fw->flux[2]) / dx - (fn->flux[2] - fs->flux[2]) / dx -
                  g * 0.5 * (N->h + Sd->h) * (N->z - Sd->z) / dx;
      c->U[PL(0, 0) * n + k] = c->F[PL(0, 0) * n + k] + dt * l0;
      c->U[PL(1, 0) * n + k] = c->F[PL(1, 0) * n + k] + dt * l1;
      c->U[PL(2, 0) * n + k] = c->F[PL(2, 0) * n + k] + dt * l2;
    }
  int bad = 0;
  double clip = pass_cleanup(c, c->U, &bad);
  c->mass_in += dt * in;
  c->mass_out += dt * out;
  c->mass_clip += clip;
  c->t = t_next;
  c->step += 1;
  c->dt_next = cfl_dt(c, c->U, c->t);
  if (dt_used) *dt_used = dt;
  if (bad) return fail(c, DG2REF_E_NUMERIC, "NaN in state at step %lld", (long long)c->step);
  return DG2REF_OK;
}

static int any_step(dg2ref_ctx *c, double dt_max, double t_end, double *dt_used) {
  return c->cfg.scheme == DG2REF_SCHEME_FV1 ? do_step_fv1(c, dt_max, t_end, dt_used)
                                            : do_step(c, dt_max, t_end, dt_used);
}

int dg2ref_step(dg2ref_ctx *c, double dt_max, double *dt_used) {
  if (!c) return DG2REF_E_ARG;
  return any_step(c, dt_max, INFINITY, dt_used);
}

int dg2ref_run(dg2ref_ctx *c, double t_end, int64_t *steps_taken) {
  if (!c) return DG2REF_E_ARG;
  if (!(t_end >= c->t)) return fail(c, DG2REF_E_ARG, "t_end %g is before t %g", t_end, c->t);
  int64_t k = 0;
  while (c->t < t_end) {
    int rc = any_step(c, 0.0, t_end, NULL);
    ++k;
    if (rc) {
      if (steps_taken) *steps_taken = k;
      return rc;
    }
  }
  if (steps_taken) *steps_taken = k;
  return DG2REF_OK;
}

/* ------------------------------------------------------------------------------ */
/* set-up                                                                           */
/* ------------------------------------------------------------------------------ */
static int edge_len(const dg2ref_ctx *c, int edge) { return edge <= DG2REF_E ? c->ny : c->nx; }

void dg2ref_destroy(dg2ref_ctx *c) {
  if (!c) return;
  free(c->zv); free(c->z0); free(c->z1x); free(c->z1y); free(c->manning);
  free(c->U); free(c->F); free(c->V); free(c->Ui); free(c->W); free(c->L); free(c->flat); free(c->rowsum);
  free(c->xf); free(c->yf); free(c->bw); free(c->be); free(c->bs); free(c->bn);
  if (c->segs)
    for (int s = 0; s < c->n_segs; ++s) { free(c->segs[s].t_knots); free(c->segs[s].q_knots); }
  free(c->segs);
  free(c);
}

static int finite_all(const double *a, size_t n) {
  for (size_t k = 0; k < n; ++k)
    if (!isfinite(a[k])) return 0;
  return 1;
}

static char init_err[256];
const char *dg2ref_init_error(void) { return init_err; }

int dg2ref_init(const dg2ref_config *cfg, const double *zv, const double *manning,
                double manning_scalar, int32_t init_mode, const double *init_data,
                double eta_level, const dg2ref_boundary *bcs, int32_t n_bcs,
                dg2ref_ctx **out) {
  init_err[0] = 0;
  if (!out) return DG2REF_E_ARG;
  *out = NULL;
  if (!cfg || !zv) return DG2REF_E_ARG;
  dg2ref_ctx *c = (dg2ref_ctx *)calloc(1, sizeof *c);
  if (!c) return DG2REF_E_ARG;
  c->cfg = *cfg;
  int rc = DG2REF_OK;
#define BAD(...) do { rc = fail(c, DG2REF_E_ARG, __VA_ARGS__); goto done; } while (0)
  if (cfg->nx < 1 || cfg->ny < 1) BAD("grid %d x %d", cfg->nx, cfg->ny);
  if (!(cfg->dx > 0.0) || !(cfg->g > 0.0) || !(cfg->cfl > 0.0) || !(cfg->h_tol >= 0.0) ||
      !(cfg->dt_dry > 0.0) || !isfinite(cfg->t0))
    BAD("bad scalar parameter");
  for (int e = 0; e < 4; ++e)
    if (cfg->edge_kind[e] != DG2REF_BC_TRANSMISSIVE && cfg->edge_kind[e] != DG2REF_BC_WALL)
      BAD("edge default kind must be transmissive or wall");
  c->nx = cfg->nx;
  c->ny = cfg->ny;
  c->n = (size_t)cfg->nx * cfg->ny;
  size_t n, nv;  /* assigned, not initialised: the earlier errors jump past them */
  n = c->n;
  nv = (size_t)(cfg->nx + 1) * (cfg->ny + 1);
  if (!finite_all(zv, nv)) BAD("non-finite bed elevation");
  c->zv = malloc(nv * sizeof(double));
  c->z0 = malloc(n * sizeof(double));
  c->z1x = malloc(n * sizeof(double));
  c->z1y = malloc(n * sizeof(double));
  c->manning = malloc(n * sizeof(double));
  c->U = calloc(9 * n, sizeof(double));
  c->F = calloc(9 * n, sizeof(double));
  c->V = calloc(9 * n, sizeof(double));
  c->Ui = calloc(9 * n, sizeof(double));
  c->W = calloc(9 * n, sizeof(double));
  c->L = calloc(9 * n, sizeof(double));
  c->flat = calloc(n, 1);
  c->rowsum = calloc(cfg->ny, sizeof(double));
  c->xf = calloc((size_t)(cfg->nx + 1) * cfg->ny, sizeof(face_t));
  c->yf = calloc((size_t)cfg->nx * (cfg->ny + 1), sizeof(face_t));
  c->bw = calloc(cfg->ny, sizeof(bface_t));
  c->be = calloc(cfg->ny, sizeof(bface_t));
  c->bs = calloc(cfg->nx, sizeof(bface_t));
  c->bn = calloc(cfg->nx, sizeof(bface_t));
  c->segs = calloc(n_bcs > 0 ? n_bcs : 1, sizeof(seg_t));
  if (!c->zv || !c->z0 || !c->z1x || !c->z1y || !c->manning || !c->U || !c->F || !c->V ||
      !c->Ui || !c->W || !c->L || !c->flat || !c->rowsum || !c->xf || !c->yf || !c->bw || !c->be || !c->bs || !c->bn ||
      !c->segs)
    BAD("out of host memory");
  memcpy(c->zv, zv, nv * sizeof(double));
  dg2ref_bed_coeffs(c->nx, c->ny, c->zv, c->z0, c->z1x, c->z1y);
  if (manning) {
    for (size_t k = 0; k < n; ++k) {
      if (!(manning[k] >= 0.0) || !isfinite(manning[k])) BAD("bad Manning n at cell %zu", k);
      c->manning[k] = manning[k];
    }
  } else {
    if (!(manning_scalar >= 0.0) || !isfinite(manning_scalar)) BAD("bad Manning n");
    for (size_t k = 0; k < n; ++k) c->manning[k] = manning_scalar;
  }
  /* boundaries */
  bface_t *edges[4];  /* assigned, not initialised: the set-up errors jump past it */
  edges[0] = c->bw; edges[1] = c->be; edges[2] = c->bs; edges[3] = c->bn;
  for (int e = 0; e < 4; ++e)
    for (int f = 0; f < edge_len(c, e); ++f) { edges[e][f].kind = cfg->edge_kind[e]; edges[e][f].seg = -1; }
  if (n_bcs < 0 || (n_bcs > 0 && !bcs)) BAD("bad boundary list");
  for (int s = 0; s < n_bcs; ++s) {
    const dg2ref_boundary *b = &bcs[s];
    if (b->edge < 0 || b->edge > 3) BAD("boundary %d: bad edge", s);
    if (b->kind < 0 || b->kind > 3) BAD("boundary %d: bad kind", s);
    if (b->i0 < 0 || b->i1 > edge_len(c, b->edge) || b->i0 >= b->i1) BAD("boundary %d: bad range", s);
    seg_t *sg = &c->segs[s];
    sg->edge = b->edge; sg->kind = b->kind; sg->i0 = b->i0; sg->i1 = b->i1;
    sg->h_b = b->h_b; sg->u_b = b->u_b; sg->v_b = b->v_b;
    if (b->kind == DG2REF_BC_FIXED &&
        (!(b->h_b >= 0.0) || !isfinite(b->h_b) || !isfinite(b->u_b) || !isfinite(b->v_b)))
      BAD("boundary %d: bad fixed state", s);
    if (b->kind == DG2REF_BC_INFLOW) {
      if (b->n_knots < 1 || !b->t_knots || !b->q_knots) BAD("boundary %d: no hydrograph", s);
      sg->n_knots = b->n_knots;
      sg->t_knots = malloc(b->n_knots * sizeof(double));
      sg->q_knots = malloc(b->n_knots * sizeof(double));
      if (!sg->t_knots || !sg->q_knots) BAD("out of host memory");
      for (int k = 0; k < b->n_knots; ++k) {
        if (!isfinite(b->t_knots[k]) || !isfinite(b->q_knots[k]) || b->q_knots[k] < 0.0)
          BAD("boundary %d: bad knot %d", s, k);
        if (k > 0 && !(b->t_knots[k] > b->t_knots[k - 1])) BAD("boundary %d: knots not increasing", s);
        sg->t_knots[k] = b->t_knots[k];
        sg->q_knots[k] = b->q_knots[k];
      }
    }
    c->n_segs = s + 1;
    for (int f = b->i0; f < b->i1; ++f) {
      edges[b->edge][f].kind = b->kind;
      edges[b->edge][f].seg = s;
    }
  }
  /* initial state (Sect. 2.1.4: flow coefficients are projected like the bed) */
  double *U;
  U = c->U;
  if (init_mode == 0) {
    if (!init_data || !finite_all(init_data, 9 * n)) BAD("bad initial planes");
    memcpy(U, init_data, 9 * n * sizeof(double));
  } else if (init_mode == 1) {
    if (!init_data || !finite_all(init_data, 3 * n)) BAD("bad initial means");
    for (int var = 0; var < 3; ++var)
      memcpy(U + PL(var, 0) * n, init_data + (size_t)var * n, n * sizeof(double));
  } else if (init_mode == 2) {
    if (!init_data || !finite_all(init_data, 3 * nv)) BAD("bad initial vertex rasters");
    for (size_t k = 0; k < nv; ++k)
      if (init_data[k] < 0.0) BAD("negative vertex depth");
    for (int var = 0; var < 3; ++var)
      dg2ref_bed_coeffs(c->nx, c->ny, init_data + (size_t)var * nv, U + PL(var, 0) * n,
                        U + PL(var, 1) * n, U + PL(var, 2) * n);
  } else if (init_mode == 3) {
    if (!isfinite(eta_level)) BAD("bad still-water level");
    for (size_t k = 0; k < n; ++k) {
      double h0 = eta_level - c->z0[k];
      if (h0 > 0.0) {
        U[PL(0, 0) * n + k] = h0;
        U[PL(0, 1) * n + k] = -c->z1x[k];
        U[PL(0, 2) * n + k] = -c->z1y[k];
      }
    }
  } else {
    BAD("bad init mode %d", init_mode);
  }
  if (cfg->scheme != DG2REF_SCHEME_DG2 && cfg->scheme != DG2REF_SCHEME_FV1) BAD("bad scheme");
  if (cfg->scheme == DG2REF_SCHEME_FV1) /* piecewise constant: the means only (eq 5) */
    for (int var = 0; var < 3; ++var)
      for (int d = 1; d <= 2; ++d) memset(U + PL(var, d) * n, 0, n * sizeof(double));
  for (size_t k = 0; k < n; ++k) {
    if (U[PL(0, 0) * n + k] < 0.0) BAD("negative mean depth at cell %zu", k);
    if (U[PL(0, 0) * n + k] <= cfg->h_tol)
      for (int p = 3; p < 9; ++p) U[p * n + k] = 0.0;
  }
  c->t = cfg->t0;
  c->step = 0;
  c->dt_next = cfl_dt(c, c->U, c->t);
done:
#undef BAD
  if (rc != DG2REF_OK) {
    memcpy(init_err, c->err, sizeof init_err);
    dg2ref_destroy(c);
    return rc;
  }
  *out = c;
  return DG2REF_OK;
}

int dg2ref_read(const dg2ref_ctx *c, int32_t field, double *dst) {
  if (!c || !dst) return DG2REF_E_ARG;
  const size_t n = c->n;
  if (field >= 0 && field < 9) {
    memcpy(dst, c->U + (size_t)field * n, n * sizeof(double));
    return DG2REF_OK;
  }
  for (size_t k = 0; k < n; ++k) {
    double h0 = c->U[k];
    if (field == 9) dst[k] = h0 + c->z0[k];
    else if (field == 10) dst[k] = h0 > c->cfg.h_tol ? c->U[PL(1, 0) * n + k] / h0 : 0.0;
    else if (field == 11) dst[k] = h0 > c->cfg.h_tol ? c->U[PL(2, 0) * n + k] / h0 : 0.0;
    else return DG2REF_E_ARG;
  }
  return DG2REF_OK;
}

int dg2ref_get_scalars(const dg2ref_ctx *c, double *t, int64_t *step, double *mass,
                       double *mass_in, double *mass_out, double *mass_clip) {
  if (!c) return DG2REF_E_ARG;
  if (t) *t = c->t;
  if (step) *step = c->step;
  if (mass) {
    double m = 0.0;
    for (size_t k = 0; k < c->n; ++k) m += c->U[k];
    *mass = m * c->cfg.dx * c->cfg.dx;
  }
  if (mass_in) *mass_in = c->mass_in;
  if (mass_out) *mass_out = c->mass_out;
  if (mass_clip) *mass_clip = c->mass_clip;
  return DG2REF_OK;
}

int dg2ref_next_dt(const dg2ref_ctx *c, double *dt) {
  if (!c || !dt) return DG2REF_E_ARG;
  *dt = c->dt_next;
  return DG2REF_OK;
}

int64_t dg2ref_state_doubles(const dg2ref_ctx *c) { return c ? (int64_t)(9 * c->n + 6) : 0; }

int dg2ref_get_state(const dg2ref_ctx *c, double *dst) {
  if (!c || !dst) return DG2REF_E_ARG;
  memcpy(dst, c->U, 9 * c->n * sizeof(double));
  double *s = dst + 9 * c->n;
  s[0] = c->t; s[1] = (double)c->step; s[2] = c->mass_in; s[3] = c->mass_out;
  s[4] = c->mass_clip; s[5] = c->dt_next;
  return DG2REF_OK;
}

int dg2ref_set_state(dg2ref_ctx *c, const double *src) {
  if (!c || !src) return DG2REF_E_ARG;
  if (!finite_all(src, 9 * c->n)) return fail(c, DG2REF_E_ARG, "non-finite state");
  memcpy(c->U, src, 9 * c->n * sizeof(double));
  const double *s = src + 9 * c->n;
  c->t = s[0]; c->step = (int64_t)s[1]; c->mass_in = s[2]; c->mass_out = s[3];
  c->mass_clip = s[4]; c->dt_next = s[5];
  return DG2REF_OK;
}

const char *dg2ref_last_error(const dg2ref_ctx *c) { return c ? c->err : "no context"; }

#ifdef _OPENMP
#include <omp.h>
#endif
int dg2ref_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void dg2ref_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}
