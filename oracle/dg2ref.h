/*
 * dg2ref.h -- FP64 CPU oracle for the uniform-grid DG2 time step of the 2D shallow
 * water equations (Sharifian & Kesserwani, arXiv:2107.02750, Sect. 2.1.1, eq 1-4, and
 * Sect. 2.1.4, eq 8).
 *
 * TEST INFRASTRUCTURE ONLY. This is the plain, slow reference that the GPU library is
 * checked against. Only the test suite, the package smoke check and the CPU-baseline
 * leg of the benchmark may load it; the product path never does. It shares no source,
 * header, table or helper with the GPU library.
 *
 * Everything is FP64 and lives in host memory. Calls return 0 on success and a
 * negative code on failure; dg2ref_last_error() then holds a message.
 *
 * Coefficient planes (eq 2): index = 3*var + k with var in {h, qx, qy} and
 * k in {0 (mean), 1x (x-slope), 1y (y-slope)}:
 *   0 h0, 1 h1x, 2 h1y, 3 qx0, 4 qx1x, 5 qx1y, 6 qy0, 7 qy1x, 8 qy1y.
 * Each plane is nx*ny doubles, row-major, cell (i, j) at j*nx + i, i west->east,
 * j south->north.
 */
#ifndef DG2REF_H
#define DG2REF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { DG2REF_OK = 0, DG2REF_E_ARG = -1, DG2REF_E_NUMERIC = -3, DG2REF_E_STATE = -4 };

/* schemes: DG2 (Sect. 2.1.1) or FV1 (Sect. 2.1.2: piecewise-constant h, qx, qy and
 * bed, one forward-Euler step of L0 per time step) */
enum { DG2REF_SCHEME_DG2 = 0, DG2REF_SCHEME_FV1 = 1 };

/* boundary kinds */
enum { DG2REF_BC_TRANSMISSIVE = 0, DG2REF_BC_WALL = 1, DG2REF_BC_FIXED = 2, DG2REF_BC_INFLOW = 3 };
/* edges */
enum { DG2REF_W = 0, DG2REF_E = 1, DG2REF_S = 2, DG2REF_N = 3 };

typedef struct {
  int32_t nx, ny;
  double dx;       /* R = dx = dy (m) */
  double g;        /* gravity (m/s^2) */
  double cfl;      /* Courant number (0.33 for DG2 with RK2) */
  double h_tol;    /* dry tolerance (m) */
  double dt_dry;   /* time step when no wet cell and no forcing bounds it (s) */
  double t0;       /* initial time (s) */
  int32_t limiter; /* 1 = minmod on eta, qx, qy; 0 = off */
  int32_t edge_kind[4]; /* default kind per edge W, E, S, N (transmissive or wall) */
  int32_t scheme;  /* DG2REF_SCHEME_*; FV1 keeps every slope plane zero and ignores the
                      limiter; its Courant number is 0.5 */
} dg2ref_config;

typedef struct {
  int32_t edge;     /* DG2REF_W .. DG2REF_N */
  int32_t kind;     /* DG2REF_BC_* */
  int32_t i0, i1;   /* faces [i0, i1) along the edge (j for W/E, i for S/N) */
  int32_t n_knots;  /* inflow hydrograph Q(t), piecewise linear, held beyond the ends */
  const double *t_knots, *q_knots; /* s, m^3/s */
  double h_b, u_b, v_b;            /* fixed state */
} dg2ref_boundary;

typedef struct dg2ref_ctx dg2ref_ctx;

/* zv: (ny+1)*(nx+1) vertex elevations, row-major. manning: nx*ny or NULL (then the
 * scalar is used). init_mode 0: init_data = 9 planes; 1: 3 planes (h, qx, qy) of cell
 * means; 2: 3 vertex rasters (h, qx, qy) projected like eq 8; 3: still water at level
 * eta_level. */
int dg2ref_init(const dg2ref_config *cfg, const double *zv, const double *manning,
                double manning_scalar, int32_t init_mode, const double *init_data,
                double eta_level, const dg2ref_boundary *bcs, int32_t n_bcs,
                dg2ref_ctx **out);
/* one time step (DG2: two RK2 stages; FV1: one forward-Euler step);
 * dt = min(CFL dt, dt_max if > 0) */
int dg2ref_step(dg2ref_ctx *c, double dt_max, double *dt_used);
/* steps until t == t_end exactly */
int dg2ref_run(dg2ref_ctx *c, double t_end, int64_t *steps_taken);
/* field 0..8 planes, 9 eta0 = h0 + z0, 10 u0, 11 v0; dst holds nx*ny doubles */
int dg2ref_read(const dg2ref_ctx *c, int32_t field, double *dst);
int dg2ref_get_scalars(const dg2ref_ctx *c, double *t, int64_t *step, double *mass,
                       double *mass_in, double *mass_out, double *mass_clip);
/* the CFL time step the next dg2ref_step would take with no cap */
int dg2ref_next_dt(const dg2ref_ctx *c, double *dt);
int64_t dg2ref_state_doubles(const dg2ref_ctx *c);
int dg2ref_get_state(const dg2ref_ctx *c, double *dst);
int dg2ref_set_state(dg2ref_ctx *c, const double *src);
const char *dg2ref_last_error(const dg2ref_ctx *c);
/* message of the last failed dg2ref_init */
const char *dg2ref_init_error(void);
void dg2ref_destroy(dg2ref_ctx *c);
/* number of OpenMP threads the passes use; set it (n > 0) for the calling thread */
int dg2ref_threads(void);
void dg2ref_set_threads(int n);

/* ---- pieces exposed for unit pins ---- */
/* HLL flux across a face with normal n: states (h, u_n, u_t) left and right;
 * out = [mass, normal momentum, tangential momentum] */
void dg2ref_hll(double g, double hL, double unL, double utL, double hR, double unR,
                double utR, double out[3]);
/* split-implicit Manning update of (qx, qy) at one point; out = new (qx, qy) */
void dg2ref_friction_point(double g, double n, double h_tol, double dt, double h,
                           double qx, double qy, double out[2]);
/* eq 8: bed coefficients of every cell from the vertex raster */
void dg2ref_bed_coeffs(int32_t nx, int32_t ny, const double *zv, double *z0, double *z1x,
                       double *z1y);
/* spatial operator L (9 planes) of a given coefficient state at time t, without
 * friction, limiting or update (front cells are those the limiter would flag for this
 * state); also the boundary inflow/outflow rates (m^3/s) */
int dg2ref_operator(dg2ref_ctx *c, const double *state, double t, double *L,
                    double *inflow_rate, double *outflow_rate);
/* the limiter alone applied to a state (9 planes), written to out */
int dg2ref_limit(dg2ref_ctx *c, const double *state, double *out);
/* the friction update alone (centre and Gauss points, time step dt) applied to a
 * state (9 planes) with the context's Manning n, written to out */
int dg2ref_friction(dg2ref_ctx *c, const double *state, double dt, double *out);

#ifdef __cplusplus
}
#endif
#endif
