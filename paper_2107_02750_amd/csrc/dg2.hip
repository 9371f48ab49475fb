// dg2.hip -- host side of the C interface declared in include/dg2.h: argument checks,
// workspace layout, launches on the borrowed stream, and state transfer. The kernels
// are in dg2_kernels.hpp.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "dg2.h"
#include "dg2_kernels.hpp"
#include "dg2_adjoint.hpp"

using dg2k::Ctrl;
using dg2k::Params;
using dg2k::Seg;

namespace {

constexpr size_t ALIGN = 256;
size_t up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

struct Layout {
  size_t u0, u1, ui, zv, zc, datum, man, bface, segs, knots, ctrl, ledger, scal, total;
  int shape, tx, ty, threads, tiles_x, tiles_y, n_tiles, per_xcd, grid;
};

const int (*shape_table(int precision))[4] {
  return precision == DG2_FP32 ? dg2k::SHAPE32 : dg2k::SHAPE64;
}

// index of the configured tile shape, or -1 if it is not one of the built shapes
int shape_index(const dg2_config& c) {
  if (c.tile_x == 0 && c.tile_y == 0) return 0;
  const int (*t)[4] = shape_table(c.precision);
  for (int k = 0; k < dg2k::N_SHAPES; ++k)
    if (t[k][0] == c.tile_x && t[k][1] == c.tile_y) return k;
  return -1;
}

// the K-th tile shape of precision R
template <typename R, int K> struct ShapeOf;
template <int K> struct ShapeOf<double, K> {
  using type = dg2k::Shape<dg2k::SHAPE64[K][0], dg2k::SHAPE64[K][1], dg2k::SHAPE64[K][2],
                           dg2k::SHAPE64[K][3]>;
};
template <int K> struct ShapeOf<float, K> {
  using type = dg2k::Shape<dg2k::SHAPE32[K][0], dg2k::SHAPE32[K][1], dg2k::SHAPE32[K][2],
                           dg2k::SHAPE32[K][3]>;
};

// call F<R, shape>::run(args...) for the shape with index k
template <typename R, template <typename, typename> class F, typename... A>
int with_shape(int k, A... a) {
  switch (k) {
    case 0: return F<R, typename ShapeOf<R, 0>::type>::run(a...);
    case 1: return F<R, typename ShapeOf<R, 1>::type>::run(a...);
    case 2: return F<R, typename ShapeOf<R, 2>::type>::run(a...);
    default: return F<R, typename ShapeOf<R, 3>::type>::run(a...);
  }
}
static_assert(dg2k::N_SHAPES == 4, "with_shape lists every shape");

Layout layout(const dg2_config& c) {
  Layout L{};
  const size_t n = (size_t)c.nx * c.ny;
  const size_t rs = c.precision == DG2_FP32 ? 4 : 8;
  L.shape = shape_index(c);
  L.tx = shape_table(c.precision)[L.shape][0];
  L.ty = shape_table(c.precision)[L.shape][1];
  L.threads = L.tx * L.ty;
  L.tiles_x = (c.nx + L.tx - 1) / L.tx;
  L.tiles_y = (c.ny + L.ty - 1) / L.ty;
  L.n_tiles = L.tiles_x * L.tiles_y;
  L.per_xcd = (L.n_tiles + dg2k::NXCD - 1) / dg2k::NXCD;
  L.grid = L.per_xcd * dg2k::NXCD;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = up(off + bytes);
    return o;
  };
  L.u0 = take(9 * n * rs);
  L.u1 = take(9 * n * rs);
  L.ui = take(9 * n * rs);
  L.zv = take((size_t)(c.nx + 1) * (c.ny + 1) * rs);
  L.zc = take(c.scheme == DG2_SCHEME_FV1 ? n * rs : 0);  // FV1: the cell bed means
  L.datum = take((size_t)L.n_tiles * rs);
  L.man = take(n * rs);
  L.bface = take((size_t)2 * (c.nx + c.ny) * sizeof(int));
  L.segs = take(DG2_MAX_SEGMENTS * sizeof(Seg));
  L.knots = take(2 * DG2_MAX_KNOTS * sizeof(double));
  L.ctrl = take(sizeof(Ctrl));
  L.ledger = take((size_t)L.n_tiles * 4 * sizeof(double));
  L.scal = take(8 * sizeof(double));
  L.total = off;
  return L;
}

thread_local std::string g_init_err;

}  // namespace

struct dg2_ctx {
  dg2_config cfg;
  hipStream_t stream;
  Layout L;
  char* ws;
  size_t n;
  bool fp32;
  bool fv1;            // FV1 scheme: one launch per step, mean planes only
  bool datum;          // FP32 bed stored relative to per-tile datums
  double bed_q;        // quantum of the stored bed (0: unrounded)
  double bed_max;      // largest |z - datum| a tile reads (absolute |z| without datums)
  bool has_manning;
  double manning_scalar;
  // set by a tape around each recorded step: gauge depths written by stage 2
  double* gauge_h = nullptr;
  const int* gmap = nullptr;
  const int* gnext = nullptr;
  int nsegs;
  int parity;          // state buffer holding the current U^n
  Ctrl* h_ctrl;        // pinned mirror of the control block
  double* h_scal;      // pinned totals
  bool timing;
  int timing_every;         // with timing: bracket every timing_every-th step
  long long timing_count;   // steps launched since timing was (re)enabled
  std::vector<hipEvent_t> ev;  // 3 events per timed step
  size_t ev_used;
  int64_t t_steps;
  double t_ms1, t_ms2;
  bool in_batch;       // borrowed by a batch: not stepped alone
  double dt_fix;       // > 0: the next steps take exactly this dt (a tape's schedule)
  std::vector<int> knot_count;  // hydrograph knots of each boundary segment
  std::vector<int> seg_edge, seg_i0, seg_i1;  // each boundary segment's faces
  std::string err;
};

struct dg2_batch {
  std::vector<dg2_ctx*> members;
  std::vector<int> active;   // member indices in the current launch table
  hipStream_t stream;
  bool fp32;
  int graph_steps;
  void* d_table;             // dg2k::BatchTable<R>
  size_t table_bytes;
  double* d_t;               // status: time and health of each table entry
  int* d_health;
  double* h_t;               // pinned mirrors
  int* h_health;
  int grid;                  // blocks per launch of the current table
  double t_end;              // t_end of the current table
  hipGraph_t graph;
  hipGraphExec_t exec;
  bool graph_ok;
  std::string err;
};

namespace {

int fail(dg2_ctx* c, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return code;
}

#define HIPC(ctx, call)                                                                    \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess) return fail(ctx, DG2_E_DEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

template <typename R>
Params<R> params(const dg2_ctx* c) {
  Params<R> p{};
  const Layout& L = c->L;
  p.uin = reinterpret_cast<const R*>(c->ws + (c->parity ? L.u1 : L.u0));
  p.vbuf = reinterpret_cast<R*>(c->ws + (c->parity ? L.u0 : L.u1));
  p.uout = p.vbuf;
  p.ui = reinterpret_cast<R*>(c->ws + L.ui);
  p.zv = reinterpret_cast<const R*>(c->ws + L.zv);
  p.zc = c->fv1 ? reinterpret_cast<const R*>(c->ws + L.zc) : nullptr;
  p.datum = c->datum ? reinterpret_cast<const R*>(c->ws + L.datum) : nullptr;
  p.manning = c->has_manning ? reinterpret_cast<const R*>(c->ws + L.man) : nullptr;
  p.bface = reinterpret_cast<const int*>(c->ws + L.bface);
  p.segs = reinterpret_cast<const Seg*>(c->ws + L.segs);
  p.knots = reinterpret_cast<const double*>(c->ws + L.knots);
  p.ctrl = reinterpret_cast<Ctrl*>(c->ws + L.ctrl);
  p.ledger = reinterpret_cast<double*>(c->ws + L.ledger);
  p.n = (long long)c->n;
  p.nx = c->cfg.nx;
  p.ny = c->cfg.ny;
  p.tx = L.tx;
  p.ty = L.ty;
  p.tiles_x = L.tiles_x;
  p.n_tiles = L.n_tiles;
  p.per_xcd = L.per_xcd;
  p.nsegs = c->nsegs;
  p.max_knots = DG2_MAX_KNOTS;
  p.limiter = c->cfg.limiter;
  p.parity = c->parity;
  p.fv1 = c->fv1 ? 1 : 0;
  p.dx = R(c->cfg.dx);
  p.idx = R(1) / p.dx;
  p.g = R(c->cfg.g);
  p.h_tol = R(c->cfg.h_tol);
  p.n_scalar = R(c->manning_scalar);
  p.dxd = c->cfg.dx;
  p.gd = c->cfg.g;
  p.cfl = c->cfg.cfl;
  p.htd = c->cfg.h_tol;
  p.dt_dry = c->cfg.dt_dry;
  p.dt_max = 0.0;
  p.t_end = INFINITY;
  p.dt_fix = c->dt_fix;
  if constexpr (sizeof(R) == 8) {
    p.gauge_h = c->gauge_h;
    p.gmap = c->gmap;
    p.gnext = c->gnext;
  }
  return p;
}

template <typename R, typename S>
struct SmemBytes {
  static int run(bool fv1) { return fv1 ? (int)sizeof(dg2k::SmemFV1<R, S>) : (int)sizeof(dg2k::Smem<R, S>); }
};

template <typename R, typename S>
struct LaunchStep {
  static int run(dg2_ctx* c, double dt_max, double t_end) {
  Params<R> p = params<R>(c);
  if (c->fv1) return run_fv1(c, p, dt_max, t_end);
  p.dt_max = dt_max;
  p.t_end = t_end;
  const dim3 grid(c->L.grid), block(c->L.threads);
  hipEvent_t* e = nullptr;
  if (c->timing && c->timing_count++ % c->timing_every == 0) {
    if (c->ev_used + 3 > c->ev.size()) {
      const size_t old = c->ev.size();
      c->ev.resize(old + 3 * 1024);
      for (size_t k = old; k < c->ev.size(); ++k) HIPC(c, hipEventCreate(&c->ev[k]));
    }
    e = &c->ev[c->ev_used];
    c->ev_used += 3;
    HIPC(c, hipEventRecord(e[0], c->stream));
  }
  hipLaunchKernelGGL((dg2k::stage_kernel<R, S, 1>), grid, block, 0, c->stream, p);
  HIPC(c, hipGetLastError());
  if (e) HIPC(c, hipEventRecord(e[1], c->stream));
  hipLaunchKernelGGL((dg2k::stage_kernel<R, S, 2>), grid, block, 0, c->stream, p);
  HIPC(c, hipGetLastError());
  if (e) HIPC(c, hipEventRecord(e[2], c->stream));
  c->parity ^= 1;
  return DG2_OK;
  }

  static int run_fv1(dg2_ctx* c, Params<R> p, double dt_max, double t_end) {
    p.dt_max = dt_max;
    p.t_end = t_end;
    const dim3 grid(c->L.grid), block(c->L.threads);
    hipEvent_t* e = nullptr;
    if (c->timing && c->timing_count++ % c->timing_every == 0) {
      if (c->ev_used + 3 > c->ev.size()) {
        const size_t old = c->ev.size();
        c->ev.resize(old + 3 * 1024);
        for (size_t k = old; k < c->ev.size(); ++k) HIPC(c, hipEventCreate(&c->ev[k]));
      }
      e = &c->ev[c->ev_used];
      c->ev_used += 3;
      HIPC(c, hipEventRecord(e[0], c->stream));
    }
    hipLaunchKernelGGL((dg2k::fv1_kernel<R, S>), grid, block, 0, c->stream, p);
    HIPC(c, hipGetLastError());
    if (e) {
      HIPC(c, hipEventRecord(e[1], c->stream));
      HIPC(c, hipEventRecord(e[2], c->stream));
    }
    c->parity ^= 1;
    return DG2_OK;
  }
};

template <typename R>
int launch_step(dg2_ctx* c, double dt_max, double t_end) {
  return with_shape<R, LaunchStep>(c->L.shape, c, dt_max, t_end);
}

int step_any(dg2_ctx* c, double dt_max, double t_end) {
  return c->fp32 ? launch_step<float>(c, dt_max, t_end) : launch_step<double>(c, dt_max, t_end);
}

int pull_ctrl(dg2_ctx* c) {
  HIPC(c, hipMemcpyAsync(c->h_ctrl, c->ws + c->L.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost,
                         c->stream));
  HIPC(c, hipStreamSynchronize(c->stream));
  return DG2_OK;
}

void set_cands_inf(Ctrl& c) {
  for (auto* cd : {&c.dtc[0], &c.dtc[1], &c.dtr[0], &c.dtr[1], &c.dtr[2]})
    for (auto& v : cd->s) v = dg2k::INF_BITS;
}

// the CFL candidate of the current state, as pulled into h_ctrl
unsigned long long dtc_bits(const dg2_ctx* c) {
  const Ctrl& h = *c->h_ctrl;
  const dg2k::Cand& cd = c->fv1 ? h.dtr[h.step[c->parity] % 3] : h.dtc[c->parity];
  unsigned long long m = dg2k::INF_BITS;
  for (int k = 0; k < dg2k::NSLOT; ++k) m = std::min(m, cd.s[k * dg2k::SLOT_STRIDE]);
  return m;
}

int check_health(dg2_ctx* c) {
  const int h = c->h_ctrl->health;
  if (h & 1) return fail(c, DG2_E_NUMERIC, "NaN in the state by step %lld", (long long)c->h_ctrl->step[c->parity]);
  if (h & 2) return fail(c, DG2_E_NUMERIC, "CFL time step below 1e-12 s by step %lld", (long long)c->h_ctrl->step[c->parity]);
  return DG2_OK;
}

template <typename R>
int launch_dtc(dg2_ctx* c, double t) {
  Params<R> p = params<R>(c);
  const R* u = reinterpret_cast<const R*>(c->ws + (c->parity ? c->L.u1 : c->L.u0));
  long long blocks = ((long long)c->n + 255) / 256;
  if (blocks > 2048) blocks = 2048;
  Ctrl* ctl = reinterpret_cast<Ctrl*>(c->ws + c->L.ctrl);
  unsigned long long* slot = c->fv1 ? &ctl->dtr[0].s[0] : &ctl->dtc[c->parity].s[0];  // step 0
  hipLaunchKernelGGL((dg2k::dtc_kernel<R>), dim3((unsigned)blocks), dim3(256), 0, c->stream, p, u, t,
                     slot);
  HIPC(c, hipGetLastError());
  return DG2_OK;
}

bool finite_all(const double* a, size_t n) {
  for (size_t k = 0; k < n; ++k)
    if (!std::isfinite(a[k])) return false;
  return true;
}

int edge_len(const dg2_config& c, int edge) { return edge <= DG2_EDGE_E ? c.ny : c.nx; }

int why_fail(std::string& why, const char* fmt, ...) {
  char buf[256];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  why = buf;
  return 1;
}

// the boundary tables of a configuration: per boundary face its kind and segment
// (W[ny], E[ny], S[nx], N[nx]), the segment table and the hydrograph knot table
// (t[DG2_MAX_KNOTS] then q[DG2_MAX_KNOTS]); returns non-zero with a reason if a
// segment is invalid
int build_tables(const dg2_config& c, const dg2_boundary* bcs, int n_bcs, std::vector<int>& bface,
                 std::vector<Seg>& segs, std::vector<double>& knots, std::string& why) {
  if (n_bcs < 0 || n_bcs > DG2_MAX_SEGMENTS || (n_bcs > 0 && !bcs)) return why_fail(why, "bad boundary list");
  bface.assign(2 * (size_t)(c.nx + c.ny), 0);
  const size_t eoff[4] = {0, (size_t)c.ny, 2 * (size_t)c.ny, 2 * (size_t)c.ny + c.nx};
  for (int e = 0; e < 4; ++e)
    for (int f = 0; f < edge_len(c, e); ++f) bface[eoff[e] + f] = c.edge_kind[e];
  segs.assign(DG2_MAX_SEGMENTS, Seg{});
  knots.assign(2 * DG2_MAX_KNOTS, 0.0);
  std::vector<char> covered(bface.size(), 0);
  int kused = 0;
  for (int s = 0; s < n_bcs; ++s) {
    const dg2_boundary& b = bcs[s];
    if (b.edge < 0 || b.edge > 3) return why_fail(why, "boundary %d: bad edge", s);
    if (b.kind < 0 || b.kind > 3) return why_fail(why, "boundary %d: bad kind", s);
    if (b.i0 < 0 || b.i1 > edge_len(c, b.edge) || b.i0 >= b.i1) return why_fail(why, "boundary %d: bad range", s);
    Seg& g = segs[s];
    g.kind = b.kind; g.edge = b.edge; g.i0 = b.i0; g.i1 = b.i1; g.k0 = 0; g.nk = 0;
    g.width = (double)(b.i1 - b.i0) * c.dx;
    g.h_b = b.h_b; g.u_b = b.u_b; g.v_b = b.v_b;
    if (b.kind == DG2_BC_FIXED && (!(b.h_b >= 0) || !std::isfinite(b.h_b) || !std::isfinite(b.u_b) || !std::isfinite(b.v_b)))
      return why_fail(why, "boundary %d: bad fixed state", s);
    if (b.kind == DG2_BC_INFLOW) {
      if (b.n_knots < 1 || !b.t_knots || !b.q_knots) return why_fail(why, "boundary %d: no hydrograph", s);
      if (kused + b.n_knots > DG2_MAX_KNOTS) return why_fail(why, "too many hydrograph knots");
      for (int k = 0; k < b.n_knots; ++k) {
        if (!std::isfinite(b.t_knots[k]) || !std::isfinite(b.q_knots[k]) || b.q_knots[k] < 0)
          return why_fail(why, "boundary %d: bad knot %d", s, k);
        if (k > 0 && !(b.t_knots[k] > b.t_knots[k - 1])) return why_fail(why, "boundary %d: knots not increasing", s);
        knots[kused + k] = b.t_knots[k];
        knots[DG2_MAX_KNOTS + kused + k] = b.q_knots[k];
      }
      g.k0 = kused;
      g.nk = b.n_knots;
      kused += b.n_knots;
    }
    for (int f = b.i0; f < b.i1; ++f) {
      if (covered[eoff[b.edge] + f]) return why_fail(why, "boundary %d overlaps another", s);
      covered[eoff[b.edge] + f] = 1;
      bface[eoff[b.edge] + f] = b.kind | ((s + 1) << 8);
    }
  }
  return 0;
}

int check_config(const dg2_config* cfg) {
  if (!cfg) return fail(nullptr, DG2_E_ARG, "null config");
  if (cfg->nx < 1 || cfg->ny < 1) return DG2_E_ARG;
  if ((long long)cfg->nx * cfg->ny > (1LL << 31)) return DG2_E_UNSUPPORTED;
  if (cfg->precision != DG2_FP64 && cfg->precision != DG2_FP32) return DG2_E_ARG;
  if (cfg->bed_datum != 0 && cfg->bed_datum != 1) return DG2_E_ARG;
  if (shape_index(*cfg) < 0) return DG2_E_UNSUPPORTED;
  if (cfg->scheme != DG2_SCHEME_DG2 && cfg->scheme != DG2_SCHEME_FV1) return DG2_E_ARG;
  return DG2_OK;
}

// Per-tile datums and the quantised relative bed (FP32 with a bed datum). Each tile's
// datum is the whole number of metres nearest the middle of the bed range over the
// vertices its stage kernels read (the tile's vertices and a 2-cell halo). With B the
// largest |z - datum| over those reads, the bed is rounded to the quantum
// q = 2^-(20 - ceil(log2 B)), so |z| / q <= 2^20 in every tile's frame: the shifts
// between frames (whole metres, multiples of q), the face means (q/2), the cell means
// (q/4) and the differences of any two of them stay below 2^24 units of their
// quantum, i.e. exact in float.
bool plan_datum(const dg2_config& cfg, const Layout& L, const double* zv, std::vector<double>& zrel,
                std::vector<double>& datum, double& q, double& bmax) {
  const int nx = cfg.nx, ny = cfg.ny, tx = L.tx, ty = L.ty;
  const size_t w = (size_t)nx + 1;
  datum.assign(L.n_tiles, 0.0);
  bmax = 0.0;
  for (int tj = 0; tj < L.tiles_y; ++tj)
    for (int ti = 0; ti < L.tiles_x; ++ti) {
      const int a0 = std::max(ti * tx - 2, 0), a1 = std::min(ti * tx + tx + 2, nx);
      const int b0 = std::max(tj * ty - 2, 0), b1 = std::min(tj * ty + ty + 2, ny);
      double lo = INFINITY, hi = -INFINITY;
      for (int jv = b0; jv <= b1; ++jv)
        for (int iv = a0; iv <= a1; ++iv) {
          const double z = zv[jv * w + iv];
          lo = std::min(lo, z);
          hi = std::max(hi, z);
        }
      const double d = std::floor(0.5 * (lo + hi) + 0.5);
      datum[(size_t)tj * L.tiles_x + ti] = d;
      bmax = std::max(bmax, std::max(hi - d, d - lo));
    }
  if (!(bmax < 1048576.0)) return false;  // relief beyond 2^20 m: no useful quantum
  const int e = bmax > 0x1p-20 ? (int)std::ceil(std::log2(bmax)) : -20;
  q = std::ldexp(1.0, e - 20);
  zrel.resize(w * (ny + 1));
  for (int jv = 0; jv <= ny; ++jv)
    for (int iv = 0; iv <= nx; ++iv) {
      const int oi = std::min(iv, nx - 1), oj = std::min(jv, ny - 1);
      const double d = datum[(size_t)(oj / ty) * L.tiles_x + oi / tx];
      zrel[jv * w + iv] = q * std::nearbyint((zv[jv * w + iv] - d) / q);
    }
  return true;
}

template <typename R>
int init_device(dg2_ctx* c, const double* zv, const double* man, int mode, const double* data,
                double eta) {
  const size_t n = c->n, nv = (size_t)(c->cfg.nx + 1) * (c->cfg.ny + 1);
  size_t staged = nv;
  if (man) staged = std::max(staged, n);
  if (mode == DG2_INIT_PLANES) staged = std::max(staged, 9 * n);
  if (mode == DG2_INIT_MEANS) staged = std::max(staged, 3 * n);
  if (mode == DG2_INIT_VERTEX) staged = std::max(staged, 3 * nv);
  double* st = nullptr;
  HIPC(c, hipMalloc(&st, staged * sizeof(double)));
  int rc = DG2_OK;
  auto conv = [&](const double* src, size_t cnt, size_t dst_off) -> int {
    HIPC(c, hipMemcpyAsync(st, src, cnt * sizeof(double), hipMemcpyHostToDevice, c->stream));
    const unsigned blocks = (unsigned)((cnt + 255) / 256);
    hipLaunchKernelGGL((dg2k::convert_kernel<R>), dim3(blocks), dim3(256), 0, c->stream, st,
                       reinterpret_cast<R*>(c->ws + dst_off), (long long)cnt);
    HIPC(c, hipGetLastError());
    HIPC(c, hipStreamSynchronize(c->stream));
    return DG2_OK;
  };
  do {
    if (c->datum) {
      std::vector<double> zrel, datum;
      if (!plan_datum(c->cfg, c->L, zv, zrel, datum, c->bed_q, c->bed_max)) {
        rc = fail(c, DG2_E_UNSUPPORTED, "bed relief too large for a float datum");
        break;
      }
      if ((rc = conv(zrel.data(), nv, c->L.zv))) break;
      if ((rc = conv(datum.data(), datum.size(), c->L.datum))) break;
    } else {
      c->bed_q = 0.0;
      c->bed_max = 0.0;
      for (size_t k = 0; k < nv; ++k) c->bed_max = std::max(c->bed_max, std::fabs(zv[k]));
      if ((rc = conv(zv, nv, c->L.zv))) break;
    }
    if (man && (rc = conv(man, n, c->L.man))) break;
    if (c->fv1) {  // FV1 reads each cell's bed mean, fixed for the run, from its own plane
      const Params<R> pb = params<R>(c);
      hipLaunchKernelGGL((dg2k::bedmean_kernel<R>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                         c->stream, pb, reinterpret_cast<R*>(c->ws + c->L.zc));
    }
    if (mode != DG2_INIT_LEVEL) {
      size_t cnt = mode == DG2_INIT_PLANES ? 9 * n : (mode == DG2_INIT_MEANS ? 3 * n : 3 * nv);
      hipError_t e = hipMemcpyAsync(st, data, cnt * sizeof(double), hipMemcpyHostToDevice, c->stream);
      if (e != hipSuccess) { rc = fail(c, DG2_E_DEVICE, "staging copy: %s", hipGetErrorString(e)); break; }
    }
    Params<R> p = params<R>(c);
    p.vbuf = p.uout = reinterpret_cast<R*>(c->ws + c->L.u0);
    const unsigned blocks = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL((dg2k::init_kernel<R>), dim3(blocks), dim3(256), 0, c->stream, p, st, mode, eta);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) { rc = fail(c, DG2_E_DEVICE, "init kernel: %s", hipGetErrorString(e)); break; }
  } while (false);
  (void)hipFree(st);
  return rc;
}

int bfail(dg2_batch* b, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  b->err = buf;
  return code;
}

#define BHIPC(b, call)                                                                     \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess) return bfail(b, DG2_E_DEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

// launch table of the active members: phase 0 uses each member's current parity
template <typename R>
int batch_table(dg2_batch* b) {
  std::vector<char> buf(sizeof(dg2k::BatchTable<R>), 0);
  auto* tab = reinterpret_cast<dg2k::BatchTable<R>*>(buf.data());
  tab->n = (int)b->active.size();
  int total = 0;
  for (int k = 0; k < tab->n; ++k) {
    dg2_ctx* c = b->members[b->active[k]];
    tab->start[k] = total;
    total += c->L.n_tiles;
    for (int ph = 0; ph < 2; ++ph) {
      const int keep = c->parity;
      c->parity = keep ^ ph;
      Params<R> p = params<R>(c);
      c->parity = keep;
      p.dt_max = 0.0;
      p.t_end = b->t_end;
      tab->p[ph][k] = p;
    }
  }
  tab->start[tab->n] = total;
  tab->total = total;
  tab->per_xcd = (total + dg2k::NXCD - 1) / dg2k::NXCD;
  b->grid = tab->per_xcd * dg2k::NXCD;
  BHIPC(b, hipMemcpyAsync(b->d_table, buf.data(), buf.size(), hipMemcpyHostToDevice, b->stream));
  BHIPC(b, hipStreamSynchronize(b->stream));
  return DG2_OK;
}

template <typename R, typename S>
struct BatchLaunch {
  static int run(dg2_batch* b, int phase) {
    const auto* tab = reinterpret_cast<const dg2k::BatchTable<R>*>(b->d_table);
    const dim3 grid(b->grid), block(dg2k::Geo<S>::NT);
    hipLaunchKernelGGL((dg2k::stage_kernel_batch<R, S, 1>), grid, block, 0, b->stream, tab, phase);
    BHIPC(b, hipGetLastError());
    hipLaunchKernelGGL((dg2k::stage_kernel_batch<R, S, 2>), grid, block, 0, b->stream, tab, phase);
    BHIPC(b, hipGetLastError());
    return DG2_OK;
  }
};

template <typename R>
int batch_launch_step(dg2_batch* b, int phase) {
  return with_shape<R, BatchLaunch>(b->members[0]->L.shape, b, phase);
}

void batch_drop_graph(dg2_batch* b) {
  if (b->graph_ok) {
    (void)hipGraphExecDestroy(b->exec);
    (void)hipGraphDestroy(b->graph);
    b->graph_ok = false;
  }
}

// (re)build the table for the active members and capture graph_steps steps of it
int batch_prepare(dg2_batch* b, double t_end) {
  batch_drop_graph(b);
  b->t_end = t_end;
  int rc = b->fp32 ? batch_table<float>(b) : batch_table<double>(b);
  if (rc) return rc;
  if (b->active.empty()) return DG2_OK;
  BHIPC(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
  for (int s = 0; s < b->graph_steps && rc == DG2_OK; ++s)
    rc = b->fp32 ? batch_launch_step<float>(b, s & 1) : batch_launch_step<double>(b, s & 1);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(b->stream, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return bfail(b, DG2_E_DEVICE, "graph capture: %s", hipGetErrorString(e));
  e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    return bfail(b, DG2_E_DEVICE, "graph instantiation: %s", hipGetErrorString(e));
  }
  b->graph = g;
  b->graph_ok = true;
  return DG2_OK;
}

// issue 'steps' steps of the active members (graph replays, then single steps)
int batch_issue(dg2_batch* b, long long steps) {
  if (b->active.empty() || steps <= 0) return DG2_OK;
  const long long reps = steps / b->graph_steps, rest = steps % b->graph_steps;
  for (long long r = 0; r < reps; ++r) BHIPC(b, hipGraphLaunch(b->exec, b->stream));
  int rc = DG2_OK;
  for (long long s = 0; s < rest && rc == DG2_OK; ++s)
    rc = b->fp32 ? batch_launch_step<float>(b, (int)(s & 1)) : batch_launch_step<double>(b, (int)(s & 1));
  if (rc) return rc;
  if (steps & 1)
    for (int k : b->active) b->members[k]->parity ^= 1;
  if (rest & 1) return batch_prepare(b, b->t_end);  // phase 0 must match the parities again
  return DG2_OK;
}

// time and health of the active members (waits)
int batch_status(dg2_batch* b) {
  const int n = (int)b->active.size();
  if (n == 0) return DG2_OK;
  const unsigned blocks = (unsigned)((n + 63) / 64);
  if (b->fp32)
    hipLaunchKernelGGL((dg2k::batch_status_kernel<float>), dim3(blocks), dim3(64), 0, b->stream,
                       reinterpret_cast<const dg2k::BatchTable<float>*>(b->d_table), 0, b->d_t, b->d_health);
  else
    hipLaunchKernelGGL((dg2k::batch_status_kernel<double>), dim3(blocks), dim3(64), 0, b->stream,
                       reinterpret_cast<const dg2k::BatchTable<double>*>(b->d_table), 0, b->d_t, b->d_health);
  BHIPC(b, hipGetLastError());
  BHIPC(b, hipMemcpyAsync(b->h_t, b->d_t, n * sizeof(double), hipMemcpyDeviceToHost, b->stream));
  BHIPC(b, hipMemcpyAsync(b->h_health, b->d_health, n * sizeof(int), hipMemcpyDeviceToHost, b->stream));
  BHIPC(b, hipStreamSynchronize(b->stream));
  for (int k = 0; k < n; ++k) {
    const int h = b->h_health[k];
    if (h & 1) return bfail(b, DG2_E_NUMERIC, "member %d: NaN in the state", b->active[k]);
    if (h & 2) return bfail(b, DG2_E_NUMERIC, "member %d: CFL time step below 1e-12 s", b->active[k]);
  }
  return DG2_OK;
}

}  // namespace

extern "C" {

int dg2_batch_create(dg2_ctx* const* members, int32_t n, int32_t graph_steps, dg2_batch** out) {
  g_init_err.clear();
  if (!out) return DG2_E_ARG;
  *out = nullptr;
  if (!members || n < 1 || n > DG2_MAX_BATCH || n > dg2k::MAX_BATCH) {
    g_init_err = "bad member list";
    return DG2_E_ARG;
  }
  if (graph_steps < 2 || graph_steps > 256 || (graph_steps & 1)) {
    g_init_err = "graph_steps must be even, 2..256";
    return DG2_E_ARG;
  }
  for (int k = 0; k < n; ++k) {
    const dg2_ctx* c = members[k];
    if (!c || c->in_batch || c->fv1 || c->fp32 != members[0]->fp32 || c->stream != members[0]->stream ||
        c->L.shape != members[0]->L.shape) {
      g_init_err = "members must be distinct free contexts of one precision and tile shape on one stream";
      return DG2_E_ARG;
    }
    for (int j = 0; j < k; ++j)
      if (members[j] == c) {
        g_init_err = "repeated member";
        return DG2_E_ARG;
      }
  }
  if (!members[0]->stream) {
    g_init_err = "a batch is captured into a HIP graph: its stream must not be the null stream";
    return DG2_E_ARG;
  }
  dg2_batch* b = new (std::nothrow) dg2_batch();
  if (!b) return DG2_E_ARG;
  b->members.assign(members, members + n);
  b->stream = members[0]->stream;
  b->fp32 = members[0]->fp32;
  b->graph_steps = graph_steps;
  b->table_bytes = b->fp32 ? sizeof(dg2k::BatchTable<float>) : sizeof(dg2k::BatchTable<double>);
  b->t_end = INFINITY;
  b->graph_ok = false;
  hipError_t e = hipMalloc(&b->d_table, b->table_bytes);
  if (e == hipSuccess) e = hipMalloc((void**)&b->d_t, n * sizeof(double));
  if (e == hipSuccess) e = hipMalloc((void**)&b->d_health, n * sizeof(int));
  if (e == hipSuccess) e = hipHostMalloc((void**)&b->h_t, n * sizeof(double));
  if (e == hipSuccess) e = hipHostMalloc((void**)&b->h_health, n * sizeof(int));
  if (e != hipSuccess) {
    g_init_err = std::string("batch buffers: ") + hipGetErrorString(e);
    dg2_batch_destroy(b);
    return DG2_E_DEVICE;
  }
  for (int k = 0; k < n; ++k) {
    b->active.push_back(k);
    members[k]->in_batch = true;
  }
  int rc = batch_prepare(b, INFINITY);
  if (rc) {
    g_init_err = b->err;
    dg2_batch_destroy(b);
    return rc;
  }
  *out = b;
  return DG2_OK;
}

int dg2_batch_step(dg2_batch* b, int32_t steps) {
  if (!b || steps < 0) return DG2_E_ARG;
  if (b->active.size() != b->members.size() || !std::isinf(b->t_end)) {
    b->active.clear();
    for (int k = 0; k < (int)b->members.size(); ++k) b->active.push_back(k);
    int rc = batch_prepare(b, INFINITY);
    if (rc) return rc;
  }
  return batch_issue(b, steps);
}

int dg2_batch_run(dg2_batch* b, double t_end, int64_t* member_steps, int64_t* launches) {
  if (!b || std::isnan(t_end)) return DG2_E_ARG;
  const int n = (int)b->members.size();
  std::vector<long long> s0(n);
  for (int k = 0; k < n; ++k) {
    dg2_ctx* c = b->members[k];
    int rc = pull_ctrl(c);
    if (rc) return bfail(b, rc, "member %d: %s", k, c->err.c_str());
    if (!(t_end >= c->h_ctrl->t[c->parity]))
      return bfail(b, DG2_E_ARG, "member %d: t_end %g is before t %g", k, t_end, c->h_ctrl->t[c->parity]);
    s0[k] = c->h_ctrl->step[c->parity];
  }
  b->active.clear();
  for (int k = 0; k < n; ++k)
    if (b->members[k]->h_ctrl->t[b->members[k]->parity] < t_end) b->active.push_back(k);
  int rc = batch_prepare(b, t_end);
  long long pairs = 0;
  while (rc == DG2_OK && !b->active.empty()) {
    if ((rc = batch_issue(b, b->graph_steps))) break;
    pairs += b->graph_steps;
    if ((rc = batch_status(b))) break;
    std::vector<int> keep;
    for (int k = 0; k < (int)b->active.size(); ++k)
      if (b->h_t[k] < t_end) keep.push_back(b->active[k]);
    if (keep.size() != b->active.size()) {
      b->active = keep;
      rc = batch_prepare(b, t_end);
    }
  }
  if (launches) *launches = pairs;
  if (member_steps) {
    for (int k = 0; k < n; ++k) {
      dg2_ctx* c = b->members[k];
      if (pull_ctrl(c) == DG2_OK) member_steps[k] = c->h_ctrl->step[c->parity] - s0[k];
    }
  }
  return rc;
}

const char* dg2_batch_last_error(const dg2_batch* b) { return b ? b->err.c_str() : g_init_err.c_str(); }

void dg2_batch_destroy(dg2_batch* b) {
  if (!b) return;
  (void)hipStreamSynchronize(b->stream);
  batch_drop_graph(b);
  for (dg2_ctx* c : b->members) c->in_batch = false;
  if (b->d_table) (void)hipFree(b->d_table);
  if (b->d_t) (void)hipFree(b->d_t);
  if (b->d_health) (void)hipFree(b->d_health);
  if (b->h_t) (void)hipHostFree(b->h_t);
  if (b->h_health) (void)hipHostFree(b->h_health);
  delete b;
}


int dg2_workspace_size(const dg2_config* cfg, size_t* bytes) {
  if (!bytes) return DG2_E_ARG;
  const int rc = check_config(cfg);
  if (rc) return rc;
  *bytes = layout(*cfg).total;
  return DG2_OK;
}

const char* dg2_init_error(void) { return g_init_err.c_str(); }

int dg2_init(const dg2_config* cfg, const double* zv, const double* manning, double manning_scalar,
             int32_t init_mode, const double* init_data, double eta_level, const dg2_boundary* bcs,
             int32_t n_bcs, void* d_workspace, size_t ws_bytes, void* hip_stream, dg2_ctx** out) {
  g_init_err.clear();
  auto bad = [](int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_init_err = buf;
    return code;
  };
  if (!out) return bad(DG2_E_ARG, "null output pointer");
  *out = nullptr;
  int rc = check_config(cfg);
  if (rc) return bad(rc, "bad grid size or precision");
  const dg2_config& c = *cfg;
  if (!(c.dx > 0) || !(c.g > 0) || !(c.cfl > 0) || !(c.h_tol >= 0) || !(c.dt_dry > 0) ||
      !std::isfinite(c.t0) || !std::isfinite(c.dx) || !std::isfinite(c.g))
    return bad(DG2_E_ARG, "bad scalar parameter");
  for (int e = 0; e < 4; ++e)
    if (c.edge_kind[e] != DG2_BC_TRANSMISSIVE && c.edge_kind[e] != DG2_BC_WALL)
      return bad(DG2_E_ARG, "edge default must be transmissive or wall");
  if (!zv) return bad(DG2_E_ARG, "null bed");
  const size_t n = (size_t)c.nx * c.ny, nv = (size_t)(c.nx + 1) * (c.ny + 1);
  if (!finite_all(zv, nv)) return bad(DG2_E_ARG, "non-finite bed elevation");
  if (manning) {
    for (size_t k = 0; k < n; ++k)
      if (!(manning[k] >= 0) || !std::isfinite(manning[k])) return bad(DG2_E_ARG, "bad Manning n at cell %zu", k);
  } else if (!(manning_scalar >= 0) || !std::isfinite(manning_scalar)) {
    return bad(DG2_E_ARG, "bad Manning n");
  }
  if (init_mode == DG2_INIT_PLANES || init_mode == DG2_INIT_MEANS) {
    const size_t cnt = (init_mode == DG2_INIT_PLANES ? 9 : 3) * n;
    if (!init_data || !finite_all(init_data, cnt)) return bad(DG2_E_ARG, "bad initial data");
    for (size_t k = 0; k < n; ++k)
      if (init_data[k] < 0) return bad(DG2_E_ARG, "negative mean depth at cell %zu", k);
  } else if (init_mode == DG2_INIT_VERTEX) {
    if (!init_data || !finite_all(init_data, 3 * nv)) return bad(DG2_E_ARG, "bad initial vertex data");
    for (size_t k = 0; k < nv; ++k)
      if (init_data[k] < 0) return bad(DG2_E_ARG, "negative vertex depth");
  } else if (init_mode == DG2_INIT_LEVEL) {
    if (!std::isfinite(eta_level)) return bad(DG2_E_ARG, "bad still-water level");
  } else {
    return bad(DG2_E_ARG, "bad init mode %d", init_mode);
  }
  // boundary table
  std::vector<int> bface;
  std::vector<Seg> segs;
  std::vector<double> knots;
  {
    std::string why;
    if (build_tables(c, bcs, n_bcs, bface, segs, knots, why)) return bad(DG2_E_ARG, "%s", why.c_str());
  }
  const Layout L = layout(c);
  if (!d_workspace || ws_bytes < L.total) return bad(DG2_E_ARG, "workspace needs %zu bytes", L.total);
  if (reinterpret_cast<uintptr_t>(d_workspace) % ALIGN) return bad(DG2_E_ARG, "workspace not 256-byte aligned");

  dg2_ctx* x = new (std::nothrow) dg2_ctx();
  if (!x) return bad(DG2_E_ARG, "out of host memory");
  x->cfg = c;
  x->stream = reinterpret_cast<hipStream_t>(hip_stream);
  x->L = L;
  x->ws = reinterpret_cast<char*>(d_workspace);
  x->n = n;
  x->fp32 = c.precision == DG2_FP32;
  x->fv1 = c.scheme == DG2_SCHEME_FV1;
  x->datum = x->fp32 && c.bed_datum == 1;
  x->has_manning = manning != nullptr;
  x->manning_scalar = manning_scalar;
  x->nsegs = n_bcs;
  x->parity = 0;
  x->timing = false;
  x->timing_every = 1;
  x->timing_count = 0;
  x->ev_used = 0;
  x->t_steps = 0;
  x->t_ms1 = x->t_ms2 = 0;
  x->in_batch = false;
  x->dt_fix = 0.0;
  for (int s = 0; s < n_bcs; ++s) {
    x->knot_count.push_back(bcs[s].kind == DG2_BC_INFLOW ? bcs[s].n_knots : 0);
    x->seg_edge.push_back(bcs[s].edge);
    x->seg_i0.push_back(bcs[s].i0);
    x->seg_i1.push_back(bcs[s].i1);
  }
  auto dev = [&](hipError_t e, const char* what) {
    if (e == hipSuccess) return false;
    g_init_err = std::string(what) + ": " + hipGetErrorString(e);
    return true;
  };
  bool err = dev(hipHostMalloc((void**)&x->h_ctrl, sizeof(Ctrl)), "pinned control block") ||
             dev(hipHostMalloc((void**)&x->h_scal, 8 * sizeof(double)), "pinned totals");
  if (!err) {
    Ctrl ctrl{};
    ctrl.t[0] = ctrl.t[1] = c.t0;
    set_cands_inf(ctrl);
    err = dev(hipMemcpyAsync(x->ws + L.ctrl, &ctrl, sizeof ctrl, hipMemcpyHostToDevice, x->stream), "control block") ||
          dev(hipMemsetAsync(x->ws + L.ledger, 0, (size_t)L.n_tiles * 4 * sizeof(double), x->stream), "ledger") ||
          dev(hipMemsetAsync(x->ws + L.u1, 0, 9 * n * (x->fp32 ? 4 : 8), x->stream), "state buffer") ||
          dev(hipMemcpyAsync(x->ws + L.bface, bface.data(), bface.size() * sizeof(int), hipMemcpyHostToDevice, x->stream), "boundary faces") ||
          dev(hipMemcpyAsync(x->ws + L.segs, segs.data(), segs.size() * sizeof(Seg), hipMemcpyHostToDevice, x->stream), "segments") ||
          dev(hipMemcpyAsync(x->ws + L.knots, knots.data(), knots.size() * sizeof(double), hipMemcpyHostToDevice, x->stream), "knots") ||
          dev(hipStreamSynchronize(x->stream), "set-up copies");
  }
  if (!err) {
    rc = x->fp32 ? init_device<float>(x, zv, manning, init_mode, init_data, eta_level)
                 : init_device<double>(x, zv, manning, init_mode, init_data, eta_level);
    if (rc) { g_init_err = x->err; err = true; }
  }
  if (!err) {
    rc = x->fp32 ? launch_dtc<float>(x, c.t0) : launch_dtc<double>(x, c.t0);
    if (rc || pull_ctrl(x)) { g_init_err = x->err; err = true; }
  }
  if (err) {
    dg2_destroy(x);
    return DG2_E_DEVICE;
  }
  *out = x;
  return DG2_OK;
}

int dg2_step(dg2_ctx* c, double dt_max, double* dt_used) {
  if (!c) return DG2_E_ARG;
  if (c->in_batch) return fail(c, DG2_E_STATE, "context belongs to a batch");
  const int p = c->parity;
  int rc = step_any(c, dt_max, INFINITY);
  if (rc) return rc;
  if (dt_used) {
    if ((rc = pull_ctrl(c))) return rc;
    *dt_used = c->h_ctrl->dt_used[p];
    return check_health(c);
  }
  return DG2_OK;
}

int dg2_run(dg2_ctx* c, double t_end, int64_t* steps_taken) {
  if (!c) return DG2_E_ARG;
  if (c->in_batch) return fail(c, DG2_E_STATE, "context belongs to a batch");
  int rc = pull_ctrl(c);
  if (rc) return rc;
  const double t_start = c->h_ctrl->t[c->parity];
  const long long s_start = c->h_ctrl->step[c->parity];
  if (!(t_end >= t_start)) return fail(c, DG2_E_ARG, "t_end %g is before t %g", t_end, t_start);
  long long batch = 1;
  while (true) {
    const Ctrl& h = *c->h_ctrl;
    const double t = h.t[c->parity];
    if (steps_taken) *steps_taken = h.step[c->parity] - s_start;
    if ((rc = check_health(c))) return rc;
    if (t >= t_end) return DG2_OK;
    // size the next batch from the current time step; steps issued past t_end are
    // no-ops that only carry the state over
    const double m = __builtin_bit_cast(double, dtc_bits(c));
    double dt = std::isinf(m) ? c->cfg.dt_dry : c->cfg.cfl * m;
    double est = (t_end - t) / dt;
    batch = est < 1 ? 1 : (long long)std::ceil(est);
    if (batch > 256) batch = 256;
    for (long long k = 0; k < batch; ++k)
      if ((rc = step_any(c, 0.0, t_end))) return rc;
    if ((rc = pull_ctrl(c))) return rc;
  }
}

int dg2_read(dg2_ctx* c, int32_t field, void* dst, int32_t dst_is_device) {
  if (!c || !dst || field < 0 || field > 11) return fail(c, DG2_E_ARG, "bad field or destination");
  const size_t rs = c->fp32 ? 4 : 8;
  const char* cur = c->ws + (c->parity ? c->L.u1 : c->L.u0);
  const char* src = cur + (size_t)(field < 9 ? field : 0) * c->n * rs;
  if (field >= 9) {
    char* tmp = c->ws + c->L.ui;  // stage scratch, free between steps
    const unsigned blocks = (unsigned)((c->n + 255) / 256);
    if (c->fp32) {
      Params<float> p = params<float>(c);
      hipLaunchKernelGGL((dg2k::field_kernel<float>), dim3(blocks), dim3(256), 0, c->stream, p,
                         reinterpret_cast<const float*>(cur), field, reinterpret_cast<float*>(tmp));
    } else {
      Params<double> p = params<double>(c);
      hipLaunchKernelGGL((dg2k::field_kernel<double>), dim3(blocks), dim3(256), 0, c->stream, p,
                         reinterpret_cast<const double*>(cur), field, reinterpret_cast<double*>(tmp));
    }
    HIPC(c, hipGetLastError());
    src = tmp;
  }
  HIPC(c, hipMemcpyAsync(dst, src, c->n * rs, dst_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                         c->stream));
  HIPC(c, hipStreamSynchronize(c->stream));
  return DG2_OK;
}

int dg2_get_scalars(dg2_ctx* c, double* t, int64_t* step, double* mass, double* mass_in, double* mass_out,
                    double* mass_clip) {
  if (!c) return DG2_E_ARG;
  const char* cur = c->ws + (c->parity ? c->L.u1 : c->L.u0);
  double* dout = reinterpret_cast<double*>(c->ws + c->L.scal);
  const double area = c->cfg.dx * c->cfg.dx;
  const double* led = reinterpret_cast<const double*>(c->ws + c->L.ledger);
  if (c->fp32)
    hipLaunchKernelGGL((dg2k::totals_kernel<float>), dim3(1), dim3(1024), 0, c->stream,
                       reinterpret_cast<const float*>(cur), (long long)c->n, led, c->L.n_tiles, area, dout);
  else
    hipLaunchKernelGGL((dg2k::totals_kernel<double>), dim3(1), dim3(1024), 0, c->stream,
                       reinterpret_cast<const double*>(cur), (long long)c->n, led, c->L.n_tiles, area, dout);
  HIPC(c, hipGetLastError());
  HIPC(c, hipMemcpyAsync(c->h_scal, dout, 4 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  int rc = pull_ctrl(c);
  if (rc) return rc;
  if (t) *t = c->h_ctrl->t[c->parity];
  if (step) *step = c->h_ctrl->step[c->parity];
  if (mass) *mass = c->h_scal[0];
  if (mass_in) *mass_in = c->h_scal[1];
  if (mass_out) *mass_out = c->h_scal[2];
  if (mass_clip) *mass_clip = c->h_scal[3];
  return DG2_OK;
}

int dg2_next_dt(dg2_ctx* c, double* dt) {
  if (!c || !dt) return DG2_E_ARG;
  const int rc = pull_ctrl(c);
  if (rc) return rc;
  const double m = __builtin_bit_cast(double, dtc_bits(c));
  *dt = std::isinf(m) ? c->cfg.dt_dry : c->cfg.cfl * m;
  return DG2_OK;
}

// blob: header (8 x int64), t, step, dtc bits, ledger (n_tiles x 4 doubles), planes
namespace {
constexpr int64_t MAGIC = 0x4447325354415445LL;  // "DG2STATE"
size_t blob_bytes(const dg2_ctx* c) {
  return 8 * 8 + 3 * 8 + (size_t)c->L.n_tiles * 4 * 8 + 9 * c->n * (c->fp32 ? 4 : 8);
}
}  // namespace

int dg2_state_bytes(const dg2_ctx* c, size_t* bytes) {
  if (!c || !bytes) return DG2_E_ARG;
  *bytes = blob_bytes(c);
  return DG2_OK;
}

int dg2_get_state(dg2_ctx* c, void* host_dst) {
  if (!c || !host_dst) return DG2_E_ARG;
  int rc = pull_ctrl(c);
  if (rc) return rc;
  char* b = reinterpret_cast<char*>(host_dst);
  int64_t hdr[8] = {MAGIC, c->fp32 ? 1 : 0, c->cfg.nx, c->cfg.ny, c->L.n_tiles, c->L.tx, c->L.ty, 0};
  std::memcpy(b, hdr, sizeof hdr);
  double* s = reinterpret_cast<double*>(b + sizeof hdr);
  s[0] = c->h_ctrl->t[c->parity];
  s[1] = (double)c->h_ctrl->step[c->parity];
  const unsigned long long bits = dtc_bits(c);
  std::memcpy(&s[2], &bits, 8);
  char* led = b + sizeof hdr + 24;
  HIPC(c, hipMemcpyAsync(led, c->ws + c->L.ledger, (size_t)c->L.n_tiles * 32, hipMemcpyDeviceToHost, c->stream));
  char* pl = led + (size_t)c->L.n_tiles * 32;
  HIPC(c, hipMemcpyAsync(pl, c->ws + (c->parity ? c->L.u1 : c->L.u0), 9 * c->n * (c->fp32 ? 4 : 8),
                         hipMemcpyDeviceToHost, c->stream));
  HIPC(c, hipStreamSynchronize(c->stream));
  return DG2_OK;
}

int dg2_set_state(dg2_ctx* c, const void* host_src) {
  if (!c || !host_src) return DG2_E_ARG;
  if (c->in_batch) return fail(c, DG2_E_STATE, "context belongs to a batch");
  const char* b = reinterpret_cast<const char*>(host_src);
  int64_t hdr[8];
  std::memcpy(hdr, b, sizeof hdr);
  if (hdr[0] != MAGIC || hdr[1] != (c->fp32 ? 1 : 0) || hdr[2] != c->cfg.nx || hdr[3] != c->cfg.ny ||
      hdr[4] != c->L.n_tiles || hdr[5] != c->L.tx || hdr[6] != c->L.ty)
    return fail(c, DG2_E_STATE, "state blob does not match this context");
  int rc = pull_ctrl(c);
  if (rc) return rc;
  const double* s = reinterpret_cast<const double*>(b + sizeof hdr);
  Ctrl ctrl = *c->h_ctrl;
  ctrl.t[c->parity] = s[0];
  ctrl.step[c->parity] = (long long)s[1];
  set_cands_inf(ctrl);
  std::memcpy(&ctrl.dtc[c->parity].s[0], &s[2], 8);
  std::memcpy(&ctrl.dtr[ctrl.step[c->parity] % 3].s[0], &s[2], 8);
  ctrl.health = 0;
  HIPC(c, hipMemcpyAsync(c->ws + c->L.ctrl, &ctrl, sizeof ctrl, hipMemcpyHostToDevice, c->stream));
  const char* led = b + sizeof hdr + 24;
  HIPC(c, hipMemcpyAsync(c->ws + c->L.ledger, led, (size_t)c->L.n_tiles * 32, hipMemcpyHostToDevice, c->stream));
  const char* pl = led + (size_t)c->L.n_tiles * 32;
  HIPC(c, hipMemcpyAsync(c->ws + (c->parity ? c->L.u1 : c->L.u0), pl, 9 * c->n * (c->fp32 ? 4 : 8),
                         hipMemcpyHostToDevice, c->stream));
  HIPC(c, hipStreamSynchronize(c->stream));
  return DG2_OK;
}

int dg2_set_timing(dg2_ctx* c, int32_t on) {
  if (!c) return DG2_E_ARG;
  HIPC(c, hipStreamSynchronize(c->stream));
  if (on < 0) return DG2_E_ARG;
  c->timing = on != 0;
  c->timing_every = on > 0 ? on : 1;
  c->timing_count = 0;
  c->ev_used = 0;
  c->t_steps = 0;
  c->t_ms1 = c->t_ms2 = 0;
  return DG2_OK;
}

int dg2_get_timing(dg2_ctx* c, int64_t* steps, double* ms1, double* ms2) {
  if (!c) return DG2_E_ARG;
  HIPC(c, hipStreamSynchronize(c->stream));
  for (size_t k = 0; k + 3 <= c->ev_used; k += 3) {
    float a = 0, b = 0;
    HIPC(c, hipEventElapsedTime(&a, c->ev[k], c->ev[k + 1]));
    HIPC(c, hipEventElapsedTime(&b, c->ev[k + 1], c->ev[k + 2]));
    c->t_ms1 += a;
    c->t_ms2 += b;
    c->t_steps += 1;
  }
  c->ev_used = 0;
  if (steps) *steps = c->t_steps;
  if (ms1) *ms1 = c->t_steps ? c->t_ms1 / c->t_steps : 0.0;
  if (ms2) *ms2 = c->t_steps ? c->t_ms2 / c->t_steps : 0.0;
  return DG2_OK;
}

int dg2_tile_shapes(int32_t precision, int32_t* xy, int32_t cap, int32_t* count) {
  if (precision != DG2_FP64 && precision != DG2_FP32) return DG2_E_ARG;
  const int (*t)[4] = shape_table(precision);
  if (count) *count = dg2k::N_SHAPES;
  for (int k = 0; xy && k < dg2k::N_SHAPES && k < cap; ++k) {
    xy[2 * k] = t[k][0];
    xy[2 * k + 1] = t[k][1];
  }
  return DG2_OK;
}

int dg2_kernel_info(const dg2_ctx* c, int32_t* tile_x, int32_t* tile_y, int32_t* threads, int32_t* blocks,
                    int32_t* lds_bytes) {
  if (!c) return DG2_E_ARG;
  if (tile_x) *tile_x = c->L.tx;
  if (tile_y) *tile_y = c->L.ty;
  if (threads) *threads = c->L.threads;
  if (blocks) *blocks = c->L.grid;
  if (lds_bytes) *lds_bytes = c->fp32 ? with_shape<float, SmemBytes>(c->L.shape, c->fv1)
                                      : with_shape<double, SmemBytes>(c->L.shape, c->fv1);
  return DG2_OK;
}

int dg2_plan_bed_datum(const dg2_config* cfg, const double* zv, double* zrel, double* datum,
                       double* quantum, double* max_local) {
  const int rc = check_config(cfg);
  if (rc) return rc;
  if (!zv) return DG2_E_ARG;
  const Layout L = layout(*cfg);
  std::vector<double> zr, d;
  double q = 0.0, b = 0.0;
  if (!plan_datum(*cfg, L, zv, zr, d, q, b)) return DG2_E_UNSUPPORTED;
  if (zrel) std::memcpy(zrel, zr.data(), zr.size() * sizeof(double));
  if (datum) std::memcpy(datum, d.data(), d.size() * sizeof(double));
  if (quantum) *quantum = q;
  if (max_local) *max_local = b;
  return DG2_OK;
}

int dg2_tile_grid(const dg2_config* cfg, int32_t* tile_x, int32_t* tile_y, int32_t* tiles_x,
                  int32_t* tiles_y) {
  const int rc = check_config(cfg);
  if (rc) return rc;
  const Layout L = layout(*cfg);
  if (tile_x) *tile_x = L.tx;
  if (tile_y) *tile_y = L.ty;
  if (tiles_x) *tiles_x = L.tiles_x;
  if (tiles_y) *tiles_y = L.tiles_y;
  return DG2_OK;
}

int dg2_set_manning(dg2_ctx* c, const double* manning, int32_t src_is_device) {
  if (!c || !manning) return DG2_E_ARG;
  if (!c->has_manning) return fail(c, DG2_E_STATE, "context has no per-cell Manning plane");
  const unsigned blocks = (unsigned)((c->n + 255) / 256);
  const double* src = manning;
  void* tmp = nullptr;  // host input: a staging copy; device input: the check flag
  hipError_t e = hipSuccess;
  if (!src_is_device) {
    for (size_t k = 0; k < c->n; ++k)
      if (!(manning[k] >= 0) || !std::isfinite(manning[k])) return fail(c, DG2_E_ARG, "bad Manning n at cell %zu", k);
    HIPC(c, hipMalloc(&tmp, c->n * sizeof(double)));
    e = hipMemcpyAsync(tmp, manning, c->n * sizeof(double), hipMemcpyHostToDevice, c->stream);
    src = static_cast<const double*>(tmp);
  } else {
    HIPC(c, hipMalloc(&tmp, sizeof(int)));
    int bad = 0;
    e = hipMemsetAsync(tmp, 0, sizeof(int), c->stream);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(dg2k::check_nonneg_kernel, dim3(blocks), dim3(256), 0, c->stream, manning,
                         (long long)c->n, static_cast<int*>(tmp));
      e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(&bad, tmp, sizeof(int), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess && bad) {
      (void)hipFree(tmp);
      return fail(c, DG2_E_ARG, "bad Manning n (negative or not finite)");
    }
  }
  if (e == hipSuccess) {
    if (c->fp32)
      hipLaunchKernelGGL((dg2k::convert_kernel<float>), dim3(blocks), dim3(256), 0, c->stream, src,
                         reinterpret_cast<float*>(c->ws + c->L.man), (long long)c->n);
    else
      hipLaunchKernelGGL((dg2k::convert_kernel<double>), dim3(blocks), dim3(256), 0, c->stream, src,
                         reinterpret_cast<double*>(c->ws + c->L.man), (long long)c->n);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  (void)hipFree(tmp);
  if (e != hipSuccess) return fail(c, DG2_E_DEVICE, "set Manning: %s", hipGetErrorString(e));
  return DG2_OK;
}

int dg2_knot_count(const dg2_ctx* c, int32_t seg, int32_t* n_knots) {
  if (!c || !n_knots || seg < -1 || seg >= (int)c->knot_count.size()) return DG2_E_ARG;
  int total = 0;
  for (int s2 = 0; s2 < (int)c->knot_count.size(); ++s2)
    if (seg < 0 || s2 == seg) total += c->knot_count[s2];
  *n_knots = total;
  return DG2_OK;
}

int dg2_set_hydrograph(dg2_ctx* c, int32_t seg, const double* q_knots) {
  if (!c || !q_knots || seg < 0 || seg >= (int)c->knot_count.size()) return DG2_E_ARG;
  const int nk = c->knot_count[seg];
  if (nk <= 0) return fail(c, DG2_E_ARG, "segment %d has no hydrograph", seg);
  int k0 = 0;
  for (int s2 = 0; s2 < seg; ++s2) k0 += c->knot_count[s2];
  for (int k = 0; k < nk; ++k)
    if (!(q_knots[k] >= 0) || !std::isfinite(q_knots[k])) return fail(c, DG2_E_ARG, "bad knot %d", k);
  double* kq = reinterpret_cast<double*>(c->ws + c->L.knots) + DG2_MAX_KNOTS + k0;
  HIPC(c, hipMemcpyAsync(kq, q_knots, nk * sizeof(double), hipMemcpyHostToDevice, c->stream));
  HIPC(c, hipStreamSynchronize(c->stream));
  return DG2_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------------
// tape: recorded forward run and its discrete adjoint
// ---------------------------------------------------------------------------------
struct dg2_tape {
  dg2_ctx* c;
  int n_steps, K, n_ckpt, ng;
  bool keep_all;               // every step's states kept by the forward run (no recomputation)
  std::vector<double> dts, t;  // t[k]: time at the start of step k
  double* ckpt;                // n_ckpt states (9n each)
  double* seg;                 // K states U^n of the segment being reversed
  double* segV;                // and for each of its steps V^n (friction applied)
  double* segI;                // and U^int
  double* lam;                 // cotangent of the current state
  double* nu2;                 // cotangent of U^int
  double* gman;                // dJ/dn per cell
  double* gq;                  // dJ/dQ(t) per (step, stage, boundary face slot)
  double* gh;                  // gauge depths (n_steps + 1) x ng
  double* dj;                  // dJ/dh on the device
  int* gidx;
  int* gmap;                   // per cell: its first gauge, or -1
  int* gnext;                  // per gauge: the next gauge on the same cell, or -1
  int* regime;
  dg2k::Ctrl* ctrl;            // the tape's own control block for recomputation
  double* ledger;
  double* d_t;                 // the step start times on the device
  double* man;                 // Manning n per cell as recorded (contexts with a plane)
  double* knots;               // hydrograph knot table as recorded
  bool recorded;
  std::string err;
};

namespace {

int tfail(dg2_tape* tp, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  tp->err = buf;
  return code;
}

#define THIPC(tp, call)                                                                    \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess) return tfail(tp, DG2_E_DEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

template <typename R, typename S>
struct TapeStage {
  static int run(dg2_tape* tp, Params<R> p, int stage) {
    const dim3 grid(tp->c->L.grid), block(tp->c->L.threads);
    if (stage == 1)
      hipLaunchKernelGGL((dg2k::stage_kernel<R, S, 1>), grid, block, 0, tp->c->stream, p);
    else
      hipLaunchKernelGGL((dg2k::stage_kernel<R, S, 2>), grid, block, 0, tp->c->stream, p);
    THIPC(tp, hipGetLastError());
    return DG2_OK;
  }
};

// parameters of the recomputed step k of the current segment (its r-th step): from
// seg[r] into segV[r], segI[r] and seg[r + 1]; the parity alternates along the segment,
// so the stage kernels carry the time from step to step
Params<double> tape_params(dg2_tape* tp, int r, int k) {
  dg2_ctx* c = tp->c;
  const size_t m9 = 9 * c->n;
  Params<double> p = params<double>(c);
  p.uin = tp->seg + r * m9;
  p.vbuf = tp->segV + r * m9;
  p.ui = tp->segI + r * m9;
  // seg holds K states (K + 1 when every step is kept: the run's final state too)
  p.uout = r + 1 < tp->K + (tp->keep_all ? 1 : 0) ? tp->seg + (r + 1) * m9 : nullptr;
  p.ctrl = tp->ctrl;
  p.ledger = tp->ledger;
  if (p.manning) p.manning = tp->man;  // the parameters the run was recorded with
  p.knots = tp->knots;
  p.parity = r & 1;
  p.dt_fix = tp->dts[k];
  p.dt_max = 0.0;
  p.t_end = INFINITY;
  return p;
}

// set the tape's control block to time t[k] (stream ordered)
int tape_set_time(dg2_tape* tp, int k) {
  hipLaunchKernelGGL(dg2k::set_time_kernel, dim3(1), dim3(64), 0, tp->c->stream, tp->ctrl, tp->d_t, k);
  THIPC(tp, hipGetLastError());
  return DG2_OK;
}

// recompute the r-th step (step k) of the current segment; U^{n+1} too if both
int tape_step(dg2_tape* tp, int r, int k, bool both) {
  Params<double> p = tape_params(tp, r, k);
  int rc = with_shape<double, TapeStage>(tp->c->L.shape, tp, p, 1);
  if (rc == DG2_OK && both) rc = with_shape<double, TapeStage>(tp->c->L.shape, tp, p, 2);
  return rc;
}

}  // namespace

extern "C" {

int dg2_tape_create(dg2_ctx* c, int32_t n_steps, const double* dts, const int32_t* gauges,
                    int32_t n_gauges, int32_t checkpoint_every, dg2_tape** out) {
  g_init_err.clear();
  if (!out) return DG2_E_ARG;
  *out = nullptr;
  if (!c || n_steps < 1 || !dts || n_gauges < 0 || (n_gauges > 0 && !gauges) || checkpoint_every < -1) {
    g_init_err = "bad tape arguments";
    return DG2_E_ARG;
  }
  if (c->fp32 || c->fv1 || c->cfg.limiter != 0 || c->in_batch) {
    g_init_err = "the adjoint covers FP64 DG2 contexts with the limiter off";
    return DG2_E_UNSUPPORTED;
  }
  for (int k = 0; k < n_steps; ++k)
    if (!(dts[k] > 0) || !std::isfinite(dts[k])) {
      g_init_err = "time steps must be positive";
      return DG2_E_ARG;
    }
  for (int g = 0; g < n_gauges; ++g)
    if (gauges[g] < 0 || (size_t)gauges[g] >= c->n) {
      g_init_err = "gauge outside the grid";
      return DG2_E_ARG;
    }
  dg2_tape* tp = new (std::nothrow) dg2_tape();
  if (!tp) return DG2_E_ARG;
  tp->c = c;
  tp->n_steps = n_steps;
  tp->keep_all = checkpoint_every == -1;
  tp->K = tp->keep_all ? n_steps
                       : checkpoint_every > 0 ? checkpoint_every : (int)std::ceil(std::sqrt((double)n_steps));
  tp->n_ckpt = (n_steps + tp->K - 1) / tp->K;
  tp->ng = n_gauges;
  tp->dts.assign(dts, dts + n_steps);
  tp->recorded = false;
  const size_t st = 9 * c->n * sizeof(double);
  const size_t nfs = 2 * ((size_t)c->cfg.nx + c->cfg.ny);  // boundary face slots
  hipError_t e = hipMalloc((void**)&tp->ckpt, st * tp->n_ckpt);
  for (double** b : {&tp->seg, &tp->segV, &tp->segI})
    if (e == hipSuccess) e = hipMalloc((void**)b, st * (tp->K + (tp->keep_all && b == &tp->seg ? 1 : 0)));
  for (double** b : {&tp->lam, &tp->nu2})
    if (e == hipSuccess) e = hipMalloc((void**)b, st);
  if (e == hipSuccess) e = hipMalloc((void**)&tp->gman, c->n * sizeof(double));
  if (e == hipSuccess) e = hipMalloc((void**)&tp->gq, (size_t)n_steps * 2 * nfs * sizeof(double));
  if (e == hipSuccess) e = hipMalloc((void**)&tp->gh, (size_t)(n_steps + 1) * std::max(n_gauges, 1) * sizeof(double));
  if (e == hipSuccess) e = hipMalloc((void**)&tp->dj, (size_t)(n_steps + 1) * std::max(n_gauges, 1) * sizeof(double));
  if (e == hipSuccess) e = hipMalloc((void**)&tp->gidx, std::max(n_gauges, 1) * sizeof(int));
  if (e == hipSuccess) e = hipMalloc((void**)&tp->gmap, c->n * sizeof(int));
  if (e == hipSuccess) e = hipMalloc((void**)&tp->gnext, std::max(n_gauges, 1) * sizeof(int));
  if (e == hipSuccess) e = hipMalloc((void**)&tp->regime, sizeof(int));
  if (e == hipSuccess) e = hipMalloc((void**)&tp->ctrl, sizeof(dg2k::Ctrl));
  if (e == hipSuccess) e = hipMalloc((void**)&tp->ledger, (size_t)c->L.n_tiles * 4 * sizeof(double));
  if (e == hipSuccess) e = hipMalloc((void**)&tp->d_t, (size_t)(n_steps + 1) * sizeof(double));
  if (e == hipSuccess && c->has_manning) e = hipMalloc((void**)&tp->man, c->n * sizeof(double));
  if (e == hipSuccess) e = hipMalloc((void**)&tp->knots, 2 * DG2_MAX_KNOTS * sizeof(double));
  if (e == hipSuccess && n_gauges > 0)
    e = hipMemcpyAsync(tp->gidx, gauges, n_gauges * sizeof(int), hipMemcpyHostToDevice, c->stream);
  // the gauges of each cell as a chain in gauge order (the adjoint adds their seeds)
  std::vector<int> gmap(c->n, -1), gnext(std::max(n_gauges, 1), -1);
  for (int g = n_gauges - 1; g >= 0; --g) {
    gnext[g] = gmap[gauges[g]];
    gmap[gauges[g]] = g;
  }
  if (e == hipSuccess) e = hipMemcpyAsync(tp->gmap, gmap.data(), c->n * sizeof(int), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(tp->gnext, gnext.data(), gnext.size() * sizeof(int), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    g_init_err = std::string("tape buffers: ") + hipGetErrorString(e);
    dg2_tape_destroy(tp);
    return DG2_E_DEVICE;
  }
  *out = tp;
  return DG2_OK;
}

int dg2_tape_forward(dg2_tape* tp, double* gauge_h, int32_t dst_is_device) {
  if (!tp) return DG2_E_ARG;
  dg2_ctx* c = tp->c;
  const size_t st = 9 * c->n * sizeof(double);
  int rc = pull_ctrl(c);
  if (rc) return tfail(tp, rc, "%s", c->err.c_str());
  tp->t.assign(tp->n_steps + 1, 0.0);
  tp->t[0] = c->h_ctrl->t[c->parity];
  for (int k = 0; k < tp->n_steps; ++k) tp->t[k + 1] = tp->t[k] + tp->dts[k];
  THIPC(tp, hipMemcpyAsync(tp->d_t, tp->t.data(), tp->t.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
  // the parameters of this run: the backward pass recomputes and reverses with these,
  // whatever the context holds by then
  if (tp->man)
    THIPC(tp, hipMemcpyAsync(tp->man, c->ws + c->L.man, c->n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  THIPC(tp, hipMemcpyAsync(tp->knots, c->ws + c->L.knots, 2 * DG2_MAX_KNOTS * sizeof(double),
                           hipMemcpyDeviceToDevice, c->stream));
  const unsigned gb = (unsigned)((tp->ng + 63) / 64);
  auto cur = [&]() { return reinterpret_cast<double*>(c->ws + (c->parity ? c->L.u1 : c->L.u0)); };
  if (tp->ng > 0) hipLaunchKernelGGL(dg2k::gauge_read_kernel, dim3(gb), dim3(64), 0, c->stream, cur(), tp->gidx, tp->ng, tp->gh);
  if (tp->keep_all) {
    // the stage kernels write each step's V^n, U^int and U^{n+1} into the tape's own
    // buffers (as the recomputation of the checkpointed mode does), with the tape's
    // control block carrying the time and the context's ledger the boundary mass; the
    // final state and time go back to the context afterwards
    const size_t m9 = 9 * c->n;
    {
      dg2k::Ctrl ctrl{};
      set_cands_inf(ctrl);
      ctrl.step[0] = ctrl.step[1] = 0;
      THIPC(tp, hipMemcpyAsync(tp->ctrl, &ctrl, sizeof ctrl, hipMemcpyHostToDevice, c->stream));
      THIPC(tp, hipStreamSynchronize(c->stream));
    }
    THIPC(tp, hipMemcpyAsync(tp->seg, cur(), st, hipMemcpyDeviceToDevice, c->stream));
    if ((rc = tape_set_time(tp, 0))) return rc;
    for (int k = 0; k < tp->n_steps && rc == DG2_OK; ++k) {
      Params<double> p = tape_params(tp, k, k);
      p.ledger = reinterpret_cast<double*>(c->ws + c->L.ledger);
      if (tp->ng > 0) {  // stage 2 writes the gauge depths after the step
        p.gauge_h = tp->gh + (size_t)(k + 1) * tp->ng;
        p.gmap = tp->gmap;
        p.gnext = tp->gnext;
      }
      rc = with_shape<double, TapeStage>(c->L.shape, tp, p, 1);
      if (rc == DG2_OK) rc = with_shape<double, TapeStage>(c->L.shape, tp, p, 2);
    }
    if (rc) return rc;
    THIPC(tp, hipGetLastError());
    THIPC(tp, hipMemcpyAsync(cur(), tp->seg + (size_t)tp->n_steps * m9, st, hipMemcpyDeviceToDevice, c->stream));
    int health = 0;
    THIPC(tp, hipMemcpyAsync(&health, &tp->ctrl->health, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    if ((rc = pull_ctrl(c))) return tfail(tp, rc, "%s", c->err.c_str());
    if (health & 1) return tfail(tp, DG2_E_NUMERIC, "NaN in the state");
    Ctrl ctrl = *c->h_ctrl;  // the context moves to the end of the run
    ctrl.t[c->parity] = tp->t[tp->n_steps];
    ctrl.step[c->parity] += tp->n_steps;
    set_cands_inf(ctrl);
    THIPC(tp, hipMemcpyAsync(c->ws + c->L.ctrl, &ctrl, sizeof ctrl, hipMemcpyHostToDevice, c->stream));
    if ((rc = launch_dtc<double>(c, tp->t[tp->n_steps]))) return tfail(tp, rc, "%s", c->err.c_str());
  } else {
    for (int k = 0; k < tp->n_steps; ++k) {
      if (k % tp->K == 0)
        THIPC(tp, hipMemcpyAsync(tp->ckpt + (size_t)(k / tp->K) * 9 * c->n, cur(), st, hipMemcpyDeviceToDevice, c->stream));
      c->dt_fix = tp->dts[k];
      if (tp->ng > 0) {  // stage 2 writes the gauge depths after the step
        c->gauge_h = tp->gh + (size_t)(k + 1) * tp->ng;
        c->gmap = tp->gmap;
        c->gnext = tp->gnext;
      }
      rc = step_any(c, 0.0, INFINITY);
      c->dt_fix = 0.0;
      c->gauge_h = nullptr;
      c->gmap = c->gnext = nullptr;
      if (rc) return tfail(tp, rc, "%s", c->err.c_str());
    }
    THIPC(tp, hipGetLastError());
  }
  if ((rc = pull_ctrl(c))) return tfail(tp, rc, "%s", c->err.c_str());
  if ((rc = check_health(c))) return tfail(tp, rc, "%s", c->err.c_str());
  if (gauge_h && tp->ng > 0) {
    THIPC(tp, hipMemcpyAsync(gauge_h, tp->gh, (size_t)(tp->n_steps + 1) * tp->ng * sizeof(double),
                             dst_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream));
    THIPC(tp, hipStreamSynchronize(c->stream));
  }
  tp->recorded = true;
  return DG2_OK;
}

int dg2_tape_backward(dg2_tape* tp, const double* dj_dh, double* grad_manning, double* grad_q,
                      double* grad_u0, int32_t device_ptrs) {
  if (!tp || (tp->ng > 0 && !dj_dh)) return DG2_E_ARG;
  if (!tp->recorded) return tfail(tp, DG2_E_STATE, "no forward run recorded");
  dg2_ctx* c = tp->c;
  hipStream_t sm = c->stream;
  const long long n = (long long)c->n, m9 = 9 * n;
  const size_t st = 9 * c->n * sizeof(double);
  const int nseg = (int)c->knot_count.size();
  const size_t nfs = 2 * ((size_t)c->cfg.nx + c->cfg.ny);
  // the adjoint kernel's 32 x 8 tiles
  const unsigned cb = (unsigned)(((c->cfg.nx + dg2k::ADJ_TX - 1) / dg2k::ADJ_TX) *
                                 ((c->cfg.ny + dg2k::ADJ_TY - 1) / dg2k::ADJ_TY));
  const unsigned gb = (unsigned)((tp->ng + 63) / 64);
  // reset
  {
    dg2k::Ctrl ctrl{};
    set_cands_inf(ctrl);
    ctrl.step[0] = ctrl.step[1] = 0;
    THIPC(tp, hipMemcpyAsync(tp->ctrl, &ctrl, sizeof ctrl, hipMemcpyHostToDevice, sm));
    THIPC(tp, hipStreamSynchronize(sm));
  }
  THIPC(tp, hipMemsetAsync(tp->lam, 0, st, sm));
  THIPC(tp, hipMemsetAsync(tp->gman, 0, c->n * sizeof(double), sm));
  THIPC(tp, hipMemsetAsync(tp->gq, 0, (size_t)tp->n_steps * 2 * nfs * sizeof(double), sm));
  THIPC(tp, hipMemsetAsync(tp->regime, 0, sizeof(int), sm));
  if (tp->ng > 0) {
    THIPC(tp, hipMemcpyAsync(tp->dj, dj_dh, (size_t)(tp->n_steps + 1) * tp->ng * sizeof(double),
                             device_ptrs ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, sm));
    hipLaunchKernelGGL(dg2k::gauge_seed_kernel, dim3(gb), dim3(64), 0, sm, tp->lam, tp->gidx, tp->ng,
                       tp->dj + (size_t)tp->n_steps * tp->ng);
  }
  int rc = DG2_OK;
  for (int sgi = tp->n_ckpt - 1; sgi >= 0 && rc == DG2_OK; --sgi) {
    const int s0 = sgi * tp->K, s1 = std::min(tp->n_steps, s0 + tp->K);
    // recompute the segment from its checkpoint, keeping each step's V^n and U^int
    // (with every step kept, the forward run left them in place)
    if (!tp->keep_all) {
      THIPC(tp, hipMemcpyAsync(tp->seg, tp->ckpt + (size_t)sgi * m9, st, hipMemcpyDeviceToDevice, sm));
      if ((rc = tape_set_time(tp, s0))) break;
      for (int k = s0; k < s1 && rc == DG2_OK; ++k) rc = tape_step(tp, k - s0, k, k + 1 < s1);
    }
    for (int k = s1 - 1; k >= s0 && rc == DG2_OK; --k) {
      const size_t r = (size_t)(k - s0) * m9;
      const double dt = tp->dts[k];
      Params<double> p = params<double>(c);
      if (p.manning) p.manning = tp->man;  // the recorded parameters
      p.knots = tp->knots;
      // stage 2: nu2 = lam / 2 + (dL/dV)(U^int)^T (dt lam / 2)
      dg2k::AdjArgs a2{tp->segI + r, tp->lam, 0.5 * dt, tp->t[k] + dt, tp->lam, 0.5, nullptr,
                       nullptr, 0.0, nullptr, nullptr, nullptr, nullptr,
                       tp->nu2, tp->gq + ((size_t)k * 2 + 1) * nfs, tp->regime};
      hipLaunchKernelGGL(dg2k::adj_stage_kernel, dim3(cb), dim3(dg2k::ADJ_TX * dg2k::ADJ_TY), 0, sm, p, a2);
      // stage 1 and friction: lam <- (dF/dU)^T (lam / 2 + nu2 + (dL/dV)(V^n)^T (dt nu2)),
      // then the misfit's seeds of the gauges at step k
      dg2k::AdjArgs a1{tp->segV + r, tp->nu2, dt, tp->t[k], tp->lam, 0.5, tp->nu2,
                       tp->seg + r, dt, tp->gman,
                       tp->ng > 0 ? tp->gmap : nullptr, tp->gnext, tp->dj + (size_t)k * tp->ng,
                       tp->lam, tp->gq + ((size_t)k * 2) * nfs, tp->regime};
      hipLaunchKernelGGL(dg2k::adj_stage_kernel, dim3(cb), dim3(dg2k::ADJ_TX * dg2k::ADJ_TY), 0, sm, p, a1);
      THIPC(tp, hipGetLastError());
    }
  }
  if (rc) return rc;
  int regime = 0, health = 0;
  THIPC(tp, hipMemcpyAsync(&regime, tp->regime, sizeof(int), hipMemcpyDeviceToHost, sm));
  THIPC(tp, hipMemcpyAsync(&health, &tp->ctrl->health, sizeof(int), hipMemcpyDeviceToHost, sm));
  THIPC(tp, hipStreamSynchronize(sm));
  if (health & 1) return tfail(tp, DG2_E_NUMERIC, "NaN in a recomputed state");
  if (regime)
    return tfail(tp, DG2_E_UNSUPPORTED, "the run leaves the adjoint's regime (%s%s)",
                 (regime & 1) ? "a dry cell or face" : "", (regime & 2) ? " a binding velocity cap" : "");
  const hipMemcpyKind out_kind = device_ptrs ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if (grad_manning) THIPC(tp, hipMemcpyAsync(grad_manning, tp->gman, c->n * sizeof(double), out_kind, sm));
  if (grad_u0) THIPC(tp, hipMemcpyAsync(grad_u0, tp->lam, st, out_kind, sm));
  THIPC(tp, hipStreamSynchronize(sm));
  if (grad_q && nseg > 0) {
    std::vector<double> gqf((size_t)tp->n_steps * 2 * nfs);
    THIPC(tp, hipMemcpy(gqf.data(), tp->gq, gqf.size() * sizeof(double), hipMemcpyDeviceToHost));
    // per (step, stage, segment): the segment's faces summed in order
    const size_t eoff[4] = {0, (size_t)c->cfg.ny, 2 * (size_t)c->cfg.ny, 2 * (size_t)c->cfg.ny + c->cfg.nx};
    std::vector<double> gq((size_t)tp->n_steps * 2 * nseg, 0.0);
    for (size_t ks = 0; ks < (size_t)tp->n_steps * 2; ++ks)
      for (int sg = 0; sg < nseg; ++sg) {
        double v = 0.0;
        for (int f = c->seg_i0[sg]; f < c->seg_i1[sg]; ++f) v += gqf[ks * nfs + eoff[c->seg_edge[sg]] + f];
        gq[ks * nseg + sg] = v;
      }
    // knots of every inflow segment (host copy of the device table)
    std::vector<double> kn(2 * DG2_MAX_KNOTS);
    THIPC(tp, hipMemcpy(kn.data(), tp->knots, kn.size() * sizeof(double), hipMemcpyDeviceToHost));
    int k0 = 0, out0 = 0;
    for (int sg = 0; sg < nseg; ++sg) {
      const int nk = c->knot_count[sg];
      for (int q = 0; q < nk; ++q) grad_q[out0 + q] = 0.0;
      const double* kt = kn.data() + k0;
      for (int k = 0; k < tp->n_steps && nk > 0; ++k)
        for (int stg = 0; stg < 2; ++stg) {
          const double tq = stg == 0 ? tp->t[k] : tp->t[k] + tp->dts[k];
          const double gv = gq[((size_t)k * 2 + stg) * nseg + sg];
          if (gv == 0.0) continue;
          // Q(t) is linear between knots and held outside them (as in the kernels)
          if (tq <= kt[0]) { grad_q[out0] += gv; continue; }
          if (tq >= kt[nk - 1]) { grad_q[out0 + nk - 1] += gv; continue; }
          int j = 0;
          while (j + 1 < nk && kt[j + 1] <= tq) ++j;
          const double w = (tq - kt[j]) / (kt[j + 1] - kt[j]);
          grad_q[out0 + j] += (1.0 - w) * gv;
          grad_q[out0 + j + 1] += w * gv;
        }
      k0 += nk;
      out0 += nk;
    }
  }
  return DG2_OK;
}

const char* dg2_tape_last_error(const dg2_tape* tp) { return tp ? tp->err.c_str() : g_init_err.c_str(); }

void dg2_tape_destroy(dg2_tape* tp) {
  if (!tp) return;
  (void)hipStreamSynchronize(tp->c->stream);
  for (void* b : {(void*)tp->ckpt, (void*)tp->seg, (void*)tp->segV, (void*)tp->segI, (void*)tp->lam,
                  (void*)tp->nu2, (void*)tp->gman, (void*)tp->gq, (void*)tp->gh, (void*)tp->dj, (void*)tp->gidx, (void*)tp->gmap, (void*)tp->gnext,
                  (void*)tp->regime, (void*)tp->ctrl, (void*)tp->ledger, (void*)tp->d_t,
                  (void*)tp->man, (void*)tp->knots})
    if (b) (void)hipFree(b);
  delete tp;
}

int dg2_bed_info(const dg2_ctx* c, double* quantum, double* max_local) {
  if (!c) return DG2_E_ARG;
  if (quantum) *quantum = c->bed_q;
  if (max_local) *max_local = c->bed_max;
  return DG2_OK;
}

const char* dg2_last_error(const dg2_ctx* c) { return c ? c->err.c_str() : "null context"; }

void dg2_destroy(dg2_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
  if (c->h_ctrl) (void)hipHostFree(c->h_ctrl);
  if (c->h_scal) (void)hipHostFree(c->h_scal);
  delete c;
}

}  // extern "C"

// ---------------------------------------------------------------------------------
// one step that allocates nothing: its scratch (V^n, U^int, control block, ledger,
// boundary tables) lives in a static device array, one copy per GPU for the process
// ---------------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[DG2_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
void* g_scratch_ptr[kMaxDevices];  // the array's device address on each GPU
std::mutex g_scratch_mu;
thread_local std::string g_noalloc_err;

int noalloc_fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_noalloc_err = buf;
  return code;
}

// the scratch array's address on the current device (looked up once per device, with
// that device current; host code never passes the array's own name to a kernel)
int scratch_on_current_device(char** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return noalloc_fail(DG2_E_DEVICE, "hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return noalloc_fail(DG2_E_DEVICE, "device %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return noalloc_fail(DG2_E_DEVICE, "scratch address: %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = static_cast<char*>(g_scratch_ptr[dev]);
  return DG2_OK;
}

template <typename R, typename S>
struct NoAllocStages {
  static int run(Params<R> p, dim3 grid, dim3 block, hipStream_t st) {
    hipLaunchKernelGGL((dg2k::stage_kernel<R, S, 1>), grid, block, 0, st, p);
    hipLaunchKernelGGL((dg2k::stage_kernel<R, S, 2>), grid, block, 0, st, p);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? DG2_OK : noalloc_fail(DG2_E_DEVICE, "stage launch: %s", hipGetErrorString(e));
  }
};

}  // namespace

extern "C" {

int dg2_step_noalloc(const dg2_config* cfg, const double* zv, const double* manning,
                     double manning_scalar, const dg2_boundary* bcs, int32_t n_bcs,
                     const double* u_in, double* u_out, double t, double dt_max, double t_end,
                     double* dt_used, void* hip_stream) {
  g_noalloc_err.clear();
  if (check_config(cfg)) return noalloc_fail(DG2_E_ARG, "bad grid size or tile shape");
  const dg2_config& c = *cfg;
  if (c.precision != DG2_FP64 || c.scheme != DG2_SCHEME_DG2)
    return noalloc_fail(DG2_E_UNSUPPORTED, "the no-allocation step covers FP64 DG2 only");
  if (!(c.dx > 0) || !(c.g > 0) || !(c.cfl > 0) || !(c.h_tol >= 0) || !(c.dt_dry > 0) ||
      !std::isfinite(c.dx) || !std::isfinite(c.g) || !std::isfinite(t) || !(t_end > t))
    return noalloc_fail(DG2_E_ARG, "bad scalar parameter or time");
  for (int e = 0; e < 4; ++e)
    if (c.edge_kind[e] != DG2_BC_TRANSMISSIVE && c.edge_kind[e] != DG2_BC_WALL)
      return noalloc_fail(DG2_E_ARG, "edge default must be transmissive or wall");
  if (!zv || !u_in || !u_out) return noalloc_fail(DG2_E_ARG, "null bed or state pointer");
  if (u_in == u_out) return noalloc_fail(DG2_E_ARG, "u_in and u_out must not overlap");
  if (!manning && !(manning_scalar >= 0 && std::isfinite(manning_scalar)))
    return noalloc_fail(DG2_E_ARG, "bad Manning n");
  std::vector<int> bface;
  std::vector<Seg> segs;
  std::vector<double> knots;
  std::string why;
  if (build_tables(c, bcs, n_bcs, bface, segs, knots, why)) return noalloc_fail(DG2_E_ARG, "%s", why.c_str());
  const Layout L = layout(c);
  const size_t n = (size_t)c.nx * c.ny;
  // scratch layout (256-byte aligned sections)
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = up(off + bytes);
    return o;
  };
  const size_t o_v = take(9 * n * sizeof(double)), o_ui = take(9 * n * sizeof(double));
  const size_t o_ctrl = take(sizeof(Ctrl)), o_led = take((size_t)L.n_tiles * 4 * sizeof(double));
  const size_t o_bf = take(bface.size() * sizeof(int)), o_seg = take(segs.size() * sizeof(Seg));
  const size_t o_kn = take(knots.size() * sizeof(double));
  if (off > (size_t)DG2_NOALLOC_SCRATCH_BYTES)
    return noalloc_fail(DG2_E_ARG, "grid of %zu cells needs %zu bytes of scratch; the no-allocation step has %zu",
                        n, off, (size_t)DG2_NOALLOC_SCRATCH_BYTES);
  char* base = nullptr;
  int rc = scratch_on_current_device(&base);
  if (rc) return rc;
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  Ctrl* ctrl = reinterpret_cast<Ctrl*>(base + o_ctrl);
  double* ledger = reinterpret_cast<double*>(base + o_led);
  hipError_t e = hipMemcpyAsync(base + o_bf, bface.data(), bface.size() * sizeof(int), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(base + o_seg, segs.data(), segs.size() * sizeof(Seg), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(base + o_kn, knots.data(), knots.size() * sizeof(double), hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return noalloc_fail(DG2_E_DEVICE, "boundary tables: %s", hipGetErrorString(e));
  hipLaunchKernelGGL(dg2k::reset_ctrl_kernel, dim3(64), dim3(256), 0, st, ctrl, t, ledger, (long long)L.n_tiles * 4);
  Params<double> p{};
  p.uin = u_in;
  p.vbuf = reinterpret_cast<double*>(base + o_v);
  p.uout = u_out;
  p.ui = reinterpret_cast<double*>(base + o_ui);
  p.zv = zv;
  p.datum = nullptr;
  p.manning = manning;
  p.bface = reinterpret_cast<const int*>(base + o_bf);
  p.segs = reinterpret_cast<const Seg*>(base + o_seg);
  p.knots = reinterpret_cast<const double*>(base + o_kn);
  p.ctrl = ctrl;
  p.ledger = ledger;
  p.n = (long long)n;
  p.nx = c.nx;
  p.ny = c.ny;
  p.tx = L.tx;
  p.ty = L.ty;
  p.tiles_x = L.tiles_x;
  p.n_tiles = L.n_tiles;
  p.per_xcd = L.per_xcd;
  p.nsegs = n_bcs;
  p.max_knots = DG2_MAX_KNOTS;
  p.limiter = c.limiter;
  p.parity = 0;
  p.fv1 = 0;
  p.dx = c.dx;
  p.idx = 1.0 / c.dx;
  p.g = c.g;
  p.h_tol = c.h_tol;
  p.n_scalar = manning_scalar;
  p.dxd = c.dx;
  p.gd = c.g;
  p.cfl = c.cfl;
  p.htd = c.h_tol;
  p.dt_dry = c.dt_dry;
  p.dt_max = dt_max;
  p.t_end = t_end;
  p.dt_fix = 0.0;
  // the CFL candidate of U^n (as a context's first step takes it), then the two stages
  {
    long long blocks = ((long long)n + 255) / 256;
    if (blocks > 2048) blocks = 2048;
    hipLaunchKernelGGL((dg2k::dtc_kernel<double>), dim3((unsigned)blocks), dim3(256), 0, st, p, u_in, t,
                       &ctrl->dtc[0].s[0]);
  }
  e = hipGetLastError();
  if (e != hipSuccess) return noalloc_fail(DG2_E_DEVICE, "launch: %s", hipGetErrorString(e));
  rc = with_shape<double, NoAllocStages>(L.shape, p, dim3(L.grid), dim3(L.threads), st);
  if (rc) return rc;
  if (dt_used) {
    struct Head {
      double t[2], dt_used[2];
      long long step[2];
      int health;
    } h{};
    static_assert(offsetof(Ctrl, health) == offsetof(Head, health), "control block head");
    e = hipMemcpyAsync(&h, ctrl, sizeof h, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return noalloc_fail(DG2_E_DEVICE, "read back: %s", hipGetErrorString(e));
    if (h.health & 1) return noalloc_fail(DG2_E_NUMERIC, "NaN in the state");
    if (h.health & 2) return noalloc_fail(DG2_E_NUMERIC, "CFL time step below 1e-12 s");
    *dt_used = h.dt_used[0];
  }
  return DG2_OK;
}

const char* dg2_noalloc_last_error(void) { return g_noalloc_err.c_str(); }

}  // extern "C"
