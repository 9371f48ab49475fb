/*
 * dg2.h -- C interface of the MI355X (gfx950) library for the uniform-grid DG2 time
 * step of the 2D shallow water equations (Sharifian & Kesserwani, arXiv:2107.02750).
 *
 * The operation: the flood-model statement of Sect. 2.1 -- a raster DEM at resolution
 * R = dx = dy, Manning's n, an initial condition given as a raster, inflow hydrographs
 * at the boundary -- advanced by the second-order discontinuous Galerkin (DG2) scheme
 * of Sect. 2.1.1: piecewise-planar coefficients of h, qx, qy (eq 2) over a
 * piecewise-planar bed projected from the DEM vertices (eq 3, eq 8), a two-stage RK2
 * update (eq 4) of the spatial operator L with HLL fluxes at the four face centres
 * after wet/dry and well-balancing revisions, split-implicit Manning friction at the
 * start of each step, and a global CFL time step with Courant number 0.33.
 *
 * Conventions
 *  - All calls return int: DG2_OK (0) or a negative DG2_E_* code. No C++ exception
 *    crosses this interface. After an error on a context, dg2_last_error() describes
 *    it; after a failed dg2_init, dg2_init_error() does.
 *  - Grid: cells (i, j), i = 0..nx-1 west to east, j = 0..ny-1 south to north.
 *    Cell rasters are nx*ny values, row-major, cell (i, j) at index j*nx + i.
 *    Vertex rasters are (nx+1)*(ny+1) values, vertex (i, j) at j*(nx+1) + i; cell
 *    (i, j) has SW = (i, j), SE = (i+1, j), NW = (i, j+1), NE = (i+1, j+1).
 *  - Coefficient planes (eq 2), in this order: h0, h1x, h1y, qx0, qx1x, qx1y, qy0,
 *    qy1x, qy1y (index 3*var + k, var = h, qx, qy; k = mean, x-slope, y-slope).
 *  - Precision: DG2_FP64 computes and stores everything in double; DG2_FP32 computes
 *    and stores the coefficients and the bed in float, while time, the time step and
 *    the mass ledger stay in double. "real" below is the context's precision.
 *  - Bed datum (DG2_FP32 with bed_datum = 1): each tile of the stage kernels gets a
 *    datum, a whole number of metres near the middle of the bed range around the tile,
 *    and the bed is stored in float relative to the datum of the tile that owns each
 *    vertex, rounded to a power-of-two quantum (dg2_bed_info) chosen so that every
 *    elevation a tile sees in its own frame, and every mean and difference of them
 *    the scheme forms, is exact in float. The FP32 arithmetic uses the bed only
 *    through such differences, so a tile's results do not depend on its datum, and
 *    raising the whole bed (and any still-water level) by a whole number of metres
 *    leaves every result bitwise unchanged. Depth precision is then set by the local relief, not by the absolute
 *    elevation. The quantum is the bed's only change (at most half a quantum per
 *    vertex).
 *  - Memory: the caller owns every input; host inputs are copied during dg2_init and
 *    may be freed afterwards. The caller allocates the device workspace (its size from
 *    dg2_workspace_size) and keeps it alive, untouched, until dg2_destroy. The library
 *    owns the context. The HIP stream is borrowed: every kernel and copy of a context
 *    is issued on it, in order. A context is not thread-safe; use one per stream.
 *  - Units: metres, seconds, m^3/s for hydrographs.
 */
#ifndef DG2_H
#define DG2_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  DG2_OK = 0,
  DG2_E_ARG = -1,        /* bad argument; nothing was changed */
  DG2_E_DEVICE = -2,     /* a HIP call failed (message names it) */
  DG2_E_NUMERIC = -3,    /* NaN in the state, or the time step fell below 1e-12 s */
  DG2_E_STATE = -4,      /* state blob of the wrong size, precision or grid */
  DG2_E_UNSUPPORTED = -5 /* valid request the library does not support */
};

enum { DG2_FP64 = 0, DG2_FP32 = 1 };

/* boundary kinds. Transmissive: the ghost state copies the interior face state. Wall:
 * the normal velocity is reflected. Fixed: (h_b, u_b, v_b) is imposed. Inflow: a
 * hydrograph Q(t) spread evenly over the segment's faces enters at the larger of the
 * interior depth and the critical depth of that unit discharge (Sect. 3.1-3.3: inflow
 * hydrographs imposed near the domain edge; the paper gives no formula). */
enum { DG2_BC_TRANSMISSIVE = 0, DG2_BC_WALL = 1, DG2_BC_FIXED = 2, DG2_BC_INFLOW = 3 };
enum { DG2_EDGE_W = 0, DG2_EDGE_E = 1, DG2_EDGE_S = 2, DG2_EDGE_N = 3 };

/* initial-condition modes (Sect. 2.1.4: flow coefficients are initialised from a
 * raster in the same way as the bed) */
enum {
  DG2_INIT_PLANES = 0, /* init_data: 9 coefficient planes, nx*ny doubles each */
  DG2_INIT_MEANS = 1,  /* init_data: 3 cell rasters h, qx, qy (means; zero slopes) */
  DG2_INIT_VERTEX = 2, /* init_data: 3 vertex rasters h, qx, qy, projected as eq 8 */
  DG2_INIT_LEVEL = 3   /* still water at eta_level: h0 = eta - z0, h1 = -z1 where
                          h0 > 0, dry elsewhere; init_data unused */
};

/* schemes */
enum { DG2_SCHEME_DG2 = 0, DG2_SCHEME_FV1 = 1 };

/* limits of the boundary table */
#define DG2_MAX_SEGMENTS 64
#define DG2_MAX_KNOTS 8192 /* total over all inflow segments */

typedef struct {
  int32_t nx, ny;          /* cells, >= 1 each */
  double dx;               /* R = dx = dy, > 0 */
  double g;                /* gravity, > 0 (9.80665) */
  double cfl;              /* Courant number, > 0 (0.33, Sect. 2.1.1) */
  double h_tol;            /* dry tolerance, >= 0 (1e-3) */
  double dt_dry;           /* time step when no wet cell and no forcing bounds it, > 0 */
  double t0;               /* initial time */
  int32_t precision;       /* DG2_FP64 or DG2_FP32 */
  int32_t limiter;         /* 1: minmod on eta, qx, qy; 0: off (fronts stay first order) */
  int32_t edge_kind[4];    /* default kind of each edge W, E, S, N: transmissive or wall */
  int32_t bed_datum;       /* DG2_FP32 only (ignored for FP64): 1 stores the bed relative
                              to a per-tile datum, 0 stores absolute elevations; see
                              dg2_bed_info */
  int32_t tile_x, tile_y;  /* tile of the stage kernels in cells: 0, 0 for the
                              precision's default, else one of dg2_tile_shapes */
  int32_t scheme;          /* DG2_SCHEME_DG2, or DG2_SCHEME_FV1 (Sect. 2.1.2, eq 5-7):
                              piecewise-constant h, qx, qy and bed (the means; every
                              slope plane stays zero), L0 only, one forward-Euler step
                              per time step, Courant number cfl (the paper uses 0.5);
                              the limiter is not used */
} dg2_config;

typedef struct {
  int32_t edge;            /* DG2_EDGE_* */
  int32_t kind;            /* DG2_BC_* */
  int32_t i0, i1;          /* faces [i0, i1) along the edge: j for W/E, i for S/N */
  int32_t n_knots;         /* inflow: number of hydrograph knots (>= 1) */
  const double *t_knots;   /* inflow: strictly increasing times (host memory) */
  const double *q_knots;   /* inflow: Q >= 0 at the knots; linear between, held
                              constant before the first and after the last */
  double h_b, u_b, v_b;    /* fixed: imposed depth (>= 0) and velocity */
} dg2_boundary;

typedef struct dg2_ctx dg2_ctx;

/* Device workspace bytes a context with this configuration needs (256-byte aligned
 * base required): 29 planes of nx*ny values (three 9-plane states, the bed vertices,
 * Manning n; FV1 one more, its bed means) plus per-tile and fixed-size tables.
 * Errors: DG2_E_ARG for a NULL pointer, a grid below 1x1 or an unknown precision;
 * DG2_E_UNSUPPORTED for a grid of more than 2^31 cells (cell indices are 32-bit) or a
 * tile shape that is not built. */
int dg2_workspace_size(const dg2_config *cfg, size_t *bytes);

/* Create a context: validate the inputs on the host, copy them to the workspace on
 * `hip_stream` (a hipStream_t; NULL = the default stream), project the bed (eq 8) and
 * the initial state on the GPU, and compute the first CFL time step. An FV1 context
 * also forms every cell's bed mean (eq 8) once, into its workspace, as its
 * piecewise-constant bed (Sect. 2.1.2).
 *  z_vertices: (nx+1)*(ny+1) host doubles, finite.
 *  manning: nx*ny host doubles >= 0, or NULL to use manning_scalar everywhere.
 *  init_mode / init_data / eta_level: see DG2_INIT_*; depths must be >= 0. Discharge
 *    in cells whose mean depth is <= h_tol is set to zero.
 *  bcs / n_bcs: up to DG2_MAX_SEGMENTS segments; faces not covered use the edge default.
 *  d_workspace / ws_bytes: device memory of at least dg2_workspace_size bytes.
 * On success *out is the new context; on failure *out is NULL and nothing is kept.
 * Errors: DG2_E_ARG (bad sizes, non-finite or negative values, overlapping or
 * out-of-range segments, unsorted knots, small workspace); DG2_E_UNSUPPORTED (as for
 * dg2_workspace_size, or an FP32 bed whose relief around some tile reaches 2^20 m);
 * DG2_E_DEVICE (a HIP call failed, including the temporary device buffer of up to
 * 9*nx*ny doubles that stages the host inputs). */
int dg2_init(const dg2_config *cfg, const double *z_vertices, const double *manning,
             double manning_scalar, int32_t init_mode, const double *init_data,
             double eta_level, const dg2_boundary *bcs, int32_t n_bcs, void *d_workspace,
             size_t ws_bytes, void *hip_stream, dg2_ctx **out);

/* Enqueue one time step (friction, then the two RK2 stages of eq 4) with
 * dt = min(CFL dt, dt_max) (dt_max <= 0: no cap). The step's dt is found on the GPU;
 * with dt_used == NULL the call does not wait for the GPU. With dt_used != NULL it
 * waits and returns the dt taken, and reports DG2_E_NUMERIC if the health flag is set.
 */
int dg2_step(dg2_ctx *c, double dt_max, double *dt_used);

/* Run the simulation to a simulated end time, as the paper's case studies run each
 * scenario over a stated duration (Sect. 3.1-3.3): step until t == t_end exactly (the
 * last step is shortened). Waits for the GPU.
 * *steps_taken (may be NULL) receives the number of steps. Errors: DG2_E_ARG if
 * t_end is before the current time, DG2_E_NUMERIC (state left at the failing step). */
int dg2_run(dg2_ctx *c, double t_end, int64_t *steps_taken);

/* Copy one field of the current state to dst (nx*ny values of the context's real type):
 * 0..8 the coefficient planes of eq 2 (mean, x-slope and y-slope coefficients of h, qx
 * and qy), and the outputs the paper reports (Sect. 3: depth, velocity, water level):
 * 9 eta0 = h0 + z0, 10 u0 = qx0/h0, 11 v0 = qy0/h0 (0
 * where h0 <= h_tol). dst is device memory if dst_is_device, else host memory. Waits
 * for the GPU. */
int dg2_read(dg2_ctx *c, int32_t field, void *dst, int32_t dst_is_device);

/* Time, step count, stored mass sum(h0) dx^2 (computed now, FP64) and the FP64 mass
 * ledger that the conservative form of eq 1 closes: boundary inflow, boundary outflow
 * and mass added by clipping negative mean depths, so that
 * mass - mass(t0) == mass_in - mass_out + mass_clip up to round-off.
 * Any pointer may be NULL. Waits for the GPU. */
int dg2_get_scalars(dg2_ctx *c, double *t, int64_t *step, double *mass, double *mass_in,
                    double *mass_out, double *mass_clip);

/* The CFL time step (before any cap) that the next step would take. Waits. */
int dg2_next_dt(dg2_ctx *c, double *dt);

/* Checkpoint / resume: an opaque host blob with the coefficient planes, time, step,
 * next time step and ledger. dg2_set_state accepts only a blob from a context of the
 * same grid, precision and tile layout (else DG2_E_STATE). Both wait. */
int dg2_state_bytes(const dg2_ctx *c, size_t *bytes);
int dg2_get_state(dg2_ctx *c, void *host_dst);
int dg2_set_state(dg2_ctx *c, const void *host_src);

/* Per-kernel timing with HIP events on the context's stream. on = 0 disables it; with
 * on = k > 0 the stage kernel launches of every k-th step (the first, the (k+1)-th, ...)
 * are bracketed by events (each event record costs the stream a few microseconds, so a
 * throughput measurement samples); on < 0 is DG2_E_ARG. dg2_get_timing waits and
 * returns the number of timed steps and the mean milliseconds per launch of the
 * stage-1 and stage-2 kernels (FV1: its one kernel as stage 1) over those steps since
 * timing was (re)enabled. */
int dg2_set_timing(dg2_ctx *c, int32_t on);
int dg2_get_timing(dg2_ctx *c, int64_t *steps, double *ms_stage1, double *ms_stage2);

/* Launch geometry of the stage kernels (for the roofline accounting): tile width and
 * height in cells, threads per block, blocks per launch, LDS bytes per block. */
int dg2_kernel_info(const dg2_ctx *c, int32_t *tile_x, int32_t *tile_y, int32_t *threads,
                    int32_t *blocks, int32_t *lds_bytes);

/* The bed representation of a context: the quantum (m) the stored bed was rounded to
 * (0 when the bed is stored unrounded: FP64, or FP32 without a datum) and the largest
 * |z - datum| over the vertices any tile reads (the absolute elevation when there is
 * no datum). */
int dg2_bed_info(const dg2_ctx *c, double *quantum, double *max_local);

/* Host-only (no device needed): the per-tile datums and the stored bed that dg2_init
 * builds for an FP32 configuration with bed_datum = 1. zv: (nx+1)*(ny+1) vertex bed
 * (host). zrel (host, (nx+1)*(ny+1) doubles, may be NULL): the stored bed, relative to
 * the datum of each vertex's owner tile (the tile of cell (min(i, nx-1),
 * min(j, ny-1))) and rounded to the quantum; every value is a float. datum (host,
 * n_tiles doubles, may be NULL): tile (ti, tj) at tj*tiles_x + ti, tiles as reported
 * by dg2_tile_grid. DG2_E_UNSUPPORTED if the relief around some tile reaches 2^20 m. */
int dg2_plan_bed_datum(const dg2_config *cfg, const double *zv, double *zrel, double *datum,
                       double *quantum, double *max_local);

/* Host-only: the tile shapes the stage kernels are built for, for a precision:
 * *count shapes, written as (tile_x, tile_y) pairs into xy (room for cap pairs; xy may
 * be NULL to query the count). The first is the default. */
int dg2_tile_shapes(int32_t precision, int32_t *xy, int32_t cap, int32_t *count);

/* Host-only: the tile grid of the stage kernels for a configuration (tile width and
 * height in cells, tiles along x and y). */
int dg2_tile_grid(const dg2_config *cfg, int32_t *tile_x, int32_t *tile_y, int32_t *tiles_x,
                  int32_t *tiles_y);

/* ---- Batched scenarios --------------------------------------------------------
 * A batch advances many independent contexts (flood scenarios of any grid size) with
 * shared launches: each step launches the two stage kernels once over the tiles of
 * every member, and every member keeps its own time, CFL time step, state, mass
 * ledger and health word. For each member a batch step is bitwise the same as a
 * dg2_step of that member alone (no dt_max). Steps are issued by replaying a HIP graph
 * of graph_steps steps (an even number, 2..256) captured on the members' stream.
 *  - members: n (1..DG2_MAX_BATCH) distinct DG2-scheme contexts of one precision and
 *    tile shape, all created on the same stream. The batch borrows them: they must outlive it, and while it
 *    exists they may be read and queried but not stepped, run or restored alone.
 *  - The batch allocates its launch table and status buffers (a few hundred KB of
 *    device memory and a little pinned host memory); dg2_batch_destroy frees them.
 *  - Errors: DG2_E_ARG (bad list, mixed precision, tile shape or streams, a repeated
 *    member, an FV1 member),
 *    DG2_E_DEVICE, DG2_E_NUMERIC (a member's health word tripped; the message names
 *    it). */
#define DG2_MAX_BATCH 256
typedef struct dg2_batch dg2_batch;
int dg2_batch_create(dg2_ctx *const *members, int32_t n, int32_t graph_steps, dg2_batch **out);
/* 'steps' steps of every member, issued without waiting for the device */
int dg2_batch_step(dg2_batch *b, int32_t steps);
/* Run every member to t_end (each lands exactly on it, as dg2_run does); members that
 * reach it leave the launches. member_steps (n int64, may be NULL) receives the steps
 * each member took; launches (may be NULL) the stage-kernel launch pairs issued. */
int dg2_batch_run(dg2_batch *b, double t_end, int64_t *member_steps, int64_t *launches);
const char *dg2_batch_last_error(const dg2_batch *b);
void dg2_batch_destroy(dg2_batch *b);

/* ---- Parameters for gradient studies ------------------------------------------
 * dg2_set_manning: replace the per-cell Manning plane (nx*ny doubles, >= 0 and finite,
 * in host memory, or in device memory of the context's GPU if src_is_device; device
 * values are checked on the device before they replace the plane); the context must
 * have been created with one (else DG2_E_STATE); DG2_E_ARG for bad values.
 * dg2_set_hydrograph: replace the discharges of boundary segment seg's hydrograph
 * knots (host, as many values as it was created with, >= 0; knot times unchanged). */
int dg2_set_manning(dg2_ctx *c, const double *manning, int32_t src_is_device);
int dg2_set_hydrograph(dg2_ctx *c, int32_t seg, const double *q_knots);
/* dg2_knot_count: the hydrograph knots of boundary segment seg (0 unless it is an
 * inflow segment), or with seg = -1 of all segments together: the length of the
 * dJ/dq array that dg2_tape_backward fills. DG2_E_ARG for a bad segment or pointer. */
int dg2_knot_count(const dg2_ctx *c, int32_t seg, int32_t *n_knots);

/* ---- Discrete adjoint (FP64, DG2, limiter off, fully wet flows) ------------------
 * The adjoint of the step of Sect. 2.1.1 (eq 4, friction and L) for gradient studies;
 * the paper has no adjoint, this is an extension. A tape records a forward run of
 * n_steps steps of a context with prescribed time steps dts[k] (the replayed
 * schedule: each step takes exactly dts[k]; choose them within the CFL bound, e.g.
 * from a previous run), keeping the state every checkpoint_every steps
 * (0: ceil(sqrt(n_steps)); -1: every step's stage states, V^n, U^int and U^{n+1},
 * so that the backward pass recomputes nothing, at 3 states per step of device memory)
 * and the depth h0 of n_gauges gauge cells (indices j*nx + i)
 * at every step, initial state included: dg2_tape_forward writes them to gauge_h,
 * (n_steps+1) x n_gauges doubles, host memory or device memory if dst_is_device. The
 * Manning plane and the hydrograph knots in effect at dg2_tape_forward are copied into
 * the tape, and the backward pass uses those, whatever the context holds by then.
 * dg2_tape_backward then propagates dJ/dh ((n_steps+1) x n_gauges, row k = after k
 * steps) back through the recorded run, recomputing each segment between checkpoints,
 * and returns (each may be NULL): dJ/dn for every cell (nx*ny), dJ/dq for every
 * hydrograph knot of every boundary segment in segment order (their total count, see
 * dg2_knot_count; always host memory), and dJ/dU0 for the initial state (9 planes).
 * With device_ptrs, dj_dh, grad_manning and grad_u0 are device memory of the
 * context's GPU, else host memory. It is the exact derivative of the recorded
 * discrete run while every cell stays wet (h0 > h_tol), face depths stay positive and
 * no face-velocity cap binds; if the run leaves that regime the call fails with
 * DG2_E_UNSUPPORTED. The forward call advances the context like dg2_step; the tape
 * allocates its checkpoints and work buffers (device memory, about
 * (n_steps / checkpoint_every + 3 checkpoint_every + 8) x 9 x nx x ny doubles, or
 * (3 n_steps + 9) x 9 x nx x ny with every step kept) and frees
 * them in dg2_tape_destroy. Errors: DG2_E_ARG (bad arguments), DG2_E_UNSUPPORTED (not
 * FP64, not DG2, limiter on, or outside the regime), DG2_E_DEVICE, DG2_E_NUMERIC. */
typedef struct dg2_tape dg2_tape;
int dg2_tape_create(dg2_ctx *c, int32_t n_steps, const double *dts, const int32_t *gauges,
                    int32_t n_gauges, int32_t checkpoint_every, dg2_tape **out);
int dg2_tape_forward(dg2_tape *tp, double *gauge_h, int32_t dst_is_device);
int dg2_tape_backward(dg2_tape *tp, const double *dj_dh, double *grad_manning, double *grad_q,
                      double *grad_u0, int32_t device_ptrs);
const char *dg2_tape_last_error(const dg2_tape *tp);
void dg2_tape_destroy(dg2_tape *tp);

/* ---- One step that allocates nothing ----------------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): one DG2 step (the step of dg2_step,
 * same kernels) from the 9-plane FP64 state u_in to u_out, with no context and no
 * workspace. The scratch it needs (V^n and U^int, 18 planes, the control block, the
 * ledger and the boundary tables) lives in a static device array of
 * DG2_NOALLOC_SCRATCH_BYTES bytes that each GPU the library runs on holds until the
 * process ends; grids whose scratch does not fit (about 460,000 cells) are rejected
 * with DG2_E_ARG. It calls no hipMalloc or hipFree.
 * cfg: as for dg2_init (precision must be DG2_FP64, scheme DG2; bed_datum ignored).
 * zv: device, (ny+1)*(nx+1) vertex elevations; manning: device, nx*ny values, or NULL
 * to use manning_scalar; bcs, n_bcs: boundary segments (host), as for dg2_init.
 * u_in, u_out: device, 9 planes of nx*ny doubles each (layout of dg2_read), distinct
 * buffers, both owned by the caller; u_in is not modified. t: the time of u_in; the
 * step takes the CFL step of u_in, capped at dt_max (if > 0) and at t_end - t (pass
 * INFINITY for no end). dt_used (host, may be NULL): with it the call waits for the
 * step and reports the time step taken, and DG2_E_NUMERIC if the state holds a NaN or
 * the time step fell below 1e-12 s; without it the call returns once the work is
 * queued on hip_stream (a hipStream_t, borrowed). Every call on one GPU shares that
 * GPU's scratch array, which keeps the last call's contents: calls that overlap in
 * time on one GPU (other streams, other host threads) race and must be serialised by
 * the caller. Errors: DG2_E_ARG, DG2_E_UNSUPPORTED, DG2_E_DEVICE, DG2_E_NUMERIC;
 * dg2_noalloc_last_error() holds the message (per host thread). */
#define DG2_NOALLOC_SCRATCH_BYTES (64u << 20)
int dg2_step_noalloc(const dg2_config *cfg, const double *zv, const double *manning,
                     double manning_scalar, const dg2_boundary *bcs, int32_t n_bcs,
                     const double *u_in, double *u_out, double t, double dt_max, double t_end,
                     double *dt_used, void *hip_stream);
const char *dg2_noalloc_last_error(void);

const char *dg2_last_error(const dg2_ctx *c);
const char *dg2_init_error(void);

/* Release the context (waits for its stream). The workspace is the caller's. */
void dg2_destroy(dg2_ctx *c);

#ifdef __cplusplus
}
#endif
#endif /* DG2_H */
