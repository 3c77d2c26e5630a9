// C-ABI of libdg.so (declared in include/dg.h): configuration checks,
// workspace layout, the SSP-RK3 step sequence and its HIP-graph replay.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <limits>
#include <mutex>
#include <new>
#include <vector>

#include "dg_internal.h"

using dg::DevScalars;
using dg::LaunchCtx;

// Event-bracketed kernel timing for dg_profile_*.
struct Profiler {
  static constexpr int kEvents = 512;
  bool enabled = false;
  hipEvent_t ev[kEvents] = {};
  int kind[kEvents / 2] = {};
  int used = 0;  // events recorded since the last harvest
  double ms[DG_PROF_KINDS] = {};
  int64_t n[DG_PROF_KINDS] = {};
};

struct dg_problem {
  dg_config cfg;
  LaunchCtx ctx;
  Profiler prof;
  size_t ws_bytes;
  size_t state_elems;
  int device;
  hipStream_t user_stream;
  hipStream_t capture_stream;
  hipGraphExec_t graph;
  const double *graph_state;
  int graph_cfl;
};

// ---------------------------------------------------------------------------
// Helpers shared with the batched API.
// ---------------------------------------------------------------------------
namespace dg {

int num_vars(const dg_config *c) { return c->equation == DG_EQ_BURGERS ? 1 : c->dim + 2; }
int num_modes(const dg_config *c) { return c->dim == 1 ? c->order + 1 : (c->order + 1) * (c->order + 1); }

int validate_config(const dg_config *c) {
  if (!c) return DG_ERR_INVALID_ARG;
  if (c->abi_version != DG_ABI_VERSION || c->pad != 0) return DG_ERR_INVALID_ARG;
  if (c->dim != 1 && c->dim != 2) return DG_ERR_UNSUPPORTED;
  if (c->equation != DG_EQ_BURGERS && c->equation != DG_EQ_EULER) return DG_ERR_UNSUPPORTED;
  if (c->order < 1 || c->order > dg::kMaxN) return DG_ERR_UNSUPPORTED;
  if (c->nx < 1 || c->ny < 1 || (c->dim == 1 && c->ny != 1)) return DG_ERR_INVALID_ARG;
  const int sides = c->dim == 1 ? 2 : 4;
  for (int k = 0; k < sides; ++k) {
    const int kind = c->bc[k], beyond = c->bc_beyond[k];
    if (kind < DG_BC_PERIODIC || kind > DG_BC_INFLOW) return DG_ERR_INVALID_ARG;
    if (beyond != -1) {
      if (k < 2 || kind == DG_BC_PERIODIC || beyond < DG_BC_TRANSMISSIVE || beyond > DG_BC_INFLOW)
        return DG_ERR_INVALID_ARG;
      if (!std::isfinite(c->bc_switch[k][0]) || !std::isfinite(c->bc_switch[k][1])) return DG_ERR_INVALID_ARG;
    }
    for (int part = 0; part < 2; ++part) {
      const int kk = part == 0 ? kind : beyond;
      if (kk == DG_BC_REFLECTIVE && c->equation != DG_EQ_EULER) return DG_ERR_UNSUPPORTED;
      if (kk == DG_BC_INFLOW) {  // an admissible state
        const double *w = c->bc_state[k][part];
        const int nv = num_vars(c);
        for (int v = 0; v < nv; ++v)
          if (!std::isfinite(w[v])) return DG_ERR_INVALID_ARG;
        if (c->equation == DG_EQ_EULER) {
          double ke = 0.0;
          for (int d = 1; d <= c->dim; ++d) ke += w[d] * w[d];
          if (!(w[0] > 0.0) || !(w[nv - 1] - 0.5 * ke / w[0] > 0.0)) return DG_ERR_INVALID_ARG;
        }
      }
    }
  }
  for (int k = sides; k < 4; ++k)
    if (c->bc_beyond[k] != -1) return DG_ERR_INVALID_ARG;
  if ((c->bc[0] == DG_BC_PERIODIC) != (c->bc[1] == DG_BC_PERIODIC)) return DG_ERR_INVALID_ARG;
  if (c->dim == 2 && (c->bc[2] == DG_BC_PERIODIC) != (c->bc[3] == DG_BC_PERIODIC)) return DG_ERR_INVALID_ARG;
  if (c->positivity != 0 && c->positivity != 1) return DG_ERR_INVALID_ARG;
  if (c->x_nodes || c->y_nodes) {  // non-uniform tensor-product mesh
    if (!c->x_nodes || (c->dim == 2) != (c->y_nodes != nullptr)) return DG_ERR_INVALID_ARG;
    for (int i = 0; i <= c->nx; ++i)
      if (!std::isfinite(c->x_nodes[i]) || (i > 0 && !(c->x_nodes[i] > c->x_nodes[i - 1]))) return DG_ERR_INVALID_ARG;
    if (c->dim == 2)
      for (int j = 0; j <= c->ny; ++j)
        if (!std::isfinite(c->y_nodes[j]) || (j > 0 && !(c->y_nodes[j] > c->y_nodes[j - 1]))) return DG_ERR_INVALID_ARG;
    if (c->indicator == DG_IND_LEARNED || c->bc_beyond[2] >= 0 || c->bc_beyond[3] >= 0) return DG_ERR_UNSUPPORTED;
  }
  if (c->positivity && c->equation != DG_EQ_EULER) return DG_ERR_UNSUPPORTED;
  if (c->limiter != DG_LIM_NONE && c->limiter != DG_LIM_CSWENO && c->limiter != DG_LIM_CSWENO_CHAR)
    return DG_ERR_INVALID_ARG;
  if (c->indicator != DG_IND_TVB && c->indicator != DG_IND_ALL && c->indicator != DG_IND_LEARNED &&
      c->indicator != DG_IND_KXRCF)
    return DG_ERR_UNSUPPORTED;
  if (c->indicator == DG_IND_LEARNED && (c->dim != 2 || c->equation != DG_EQ_EULER)) return DG_ERR_UNSUPPORTED;
  // the network's features see ghost cells by periodic wrap or even reflection
  // only (the sides it was trained on): no walls, inflow or switching sides
  if (c->indicator == DG_IND_LEARNED)
    for (int k = 0; k < 4; ++k)
      if (c->bc[k] == DG_BC_REFLECTIVE || c->bc[k] == DG_BC_INFLOW || c->bc_beyond[k] != -1)
        return DG_ERR_UNSUPPORTED;
  if (c->negw_mode != DG_NEGW_SPLIT && c->negw_mode != DG_NEGW_RAW) return DG_ERR_INVALID_ARG;
  if (!(c->x1 > c->x0) || (c->dim == 2 && !(c->y1 > c->y0))) return DG_ERR_INVALID_ARG;
  if (c->equation == DG_EQ_EULER && !(c->gamma > 1.0)) return DG_ERR_INVALID_ARG;
  if (!(c->tvb_M >= 0.0) || !(c->weno_eps > 0.0) || !(c->cfl > 0.0)) return DG_ERR_INVALID_ARG;
  const long long cells = (long long)c->nx * c->ny;
  if (cells > (1ll << 31) - 1) return DG_ERR_UNSUPPORTED;  // cell index stored as int32
  return DG_OK;
}

bool g_tables_ready[64];
std::mutex g_tables_mu;

int ensure_tables(int device) {
  std::lock_guard<std::mutex> lk(g_tables_mu);
  if (device < 0 || device >= 64) return DG_ERR_HIP;
  if (g_tables_ready[device]) return DG_OK;
  dg::OrderTables tabs[dg::kMaxN + 1];
  std::memset(tabs, 0, sizeof(tabs));
  for (int N = 1; N <= dg::kMaxN; ++N) {
    int rc = dg::build_order_tables(N, &tabs[N]);
    if (rc) return rc;
  }
  int rc = dg::upload_tables_part0(tabs);
  if (!rc) rc = dg::upload_tables_part1(tabs);
  if (!rc) rc = dg::upload_tables_part2(tabs);
  if (!rc) rc = dg::upload_tables_part3(tabs);
  if (!rc) rc = dg::upload_tables_part4(tabs);
  if (!rc) rc = dg::upload_tables_part5(tabs);
  if (rc) return rc;
  g_tables_ready[device] = true;
  return DG_OK;
}

bool special_bc(const Geometry &g) {
  if (g.hxa) return true;  // non-uniform mesh
  for (int k = 0; k < 4; ++k)
    if (g.bc[k] == DG_BC_REFLECTIVE || g.bc[k] == DG_BC_INFLOW || g.bcb[k] >= 0) return true;
  return false;
}

void fill_geometry(const dg_config *cfg, Geometry *g) {
  g->nx = cfg->nx;
  g->ny = cfg->ny;
  for (int k = 0; k < 4; ++k) g->bc[k] = cfg->bc[k];
  if (cfg->dim == 1) {  // the y-direction of a 1D problem is a single periodic row
    g->bc[2] = g->bc[3] = DG_BC_PERIODIC;
  }
  g->hx = (cfg->x1 - cfg->x0) / cfg->nx;
  g->hy = cfg->dim == 2 ? (cfg->y1 - cfg->y0) / cfg->ny : 1.0;
  g->rhx = 2.0 / g->hx;
  g->rhy = 2.0 / g->hy;
  g->gamma = cfg->gamma;
  g->tvb_Mx = cfg->tvb_M * g->hx * g->hx;
  g->tvb_My = cfg->tvb_M * g->hy * g->hy;
  g->eps = cfg->weno_eps;
  g->negw_raw = cfg->negw_mode == DG_NEGW_RAW ? 1 : 0;
  g->pad = 0;
  const double rad = cfg->dim == 1 ? 0.5 * g->hx : 0.5 * std::sqrt(g->hx * g->hx + g->hy * g->hy);
  g->kx_scale = 1.0 / std::pow(rad, 0.5 * (cfg->order + 1));
  g->x0 = cfg->x0;
  // an inflow ghost holds only the lowest mode: mean / psi_0^dim, psi_0 = 1/sqrt(2)
  const double p0 = std::sqrt(0.5), k0 = cfg->dim == 1 ? p0 : p0 * p0;
  for (int k = 0; k < 4; ++k) {
    g->bcb[k] = cfg->dim == 1 && k >= 2 ? -1 : cfg->bc_beyond[k];
    g->bsw[k][0] = cfg->bc_switch[k][0];
    g->bsw[k][1] = cfg->bc_switch[k][1];
    for (int part = 0; part < 2; ++part)
      for (int v = 0; v < 4; ++v) g->bst[2 * k + part][v] = cfg->bc_state[k][part][v] / k0;
  }
  g->tb = nullptr;
  g->tvb_M = cfg->tvb_M;
  g->hxa = g->hya = g->rhxa = g->rhya = g->mhx = g->mhy = nullptr;
  g->wtx = g->wty = nullptr;
}

}  // namespace dg

using dg::num_modes;
using dg::num_vars;

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Layout {
  size_t scalars, bufA, bufB, flags, margin, list, mesh, total;
};

Layout layout(const dg_config *c) {
  Layout L;
  const size_t cells = (size_t)c->nx * c->ny;
  const size_t state = cells * num_vars(c) * num_modes(c) * sizeof(double);
  size_t off = 0;
  L.scalars = off;
  off += align_up(sizeof(DevScalars));
  L.bufA = off;
  off += align_up(state);
  L.bufB = off;
  off += align_up(state);
  L.flags = off;
  off += align_up(cells);
  L.margin = off;
  off += align_up(cells * sizeof(double));
  L.list = off;
  off += align_up(cells * sizeof(int32_t));
  L.mesh = off;  // non-uniform meshes: 3 arrays and the tables per column and per row
  if (c->x_nodes) {
    const size_t lines = (size_t)c->nx + (c->dim == 2 ? c->ny : 0);
    off += align_up(3 * lines * sizeof(double)) + align_up(lines * sizeof(dg::WenoCoef));
  }
  L.total = off;
  return L;
}

// Width of column i of nodes e[0..n] with the ghost rule of the boundary
// sides lo/hi: the periodic image or the mirrored adjacent cell.
double line_width(const double *e, int n, int i, int bc_lo, int bc_hi) {
  if (i < 0) i = bc_lo == DG_BC_PERIODIC ? i + n : -1 - i;
  else if (i >= n) i = bc_hi == DG_BC_PERIODIC ? i - n : 2 * n - 1 - i;
  return e[i + 1] - e[i];
}

// Uploads widths, 2/width, M width^2 and the CSWENO tables of every column
// (and row) into the workspace and points the geometry at them.
int upload_mesh(const dg_config *c, char *ws, const Layout &L, hipStream_t st, dg::Geometry *g) {
  const int lines_x = c->nx, lines_y = c->dim == 2 ? c->ny : 0, lines = lines_x + lines_y;
  std::vector<double> arr(3 * (size_t)lines);
  std::vector<dg::WenoCoef> tab(lines);
  for (int d = 0; d < (c->dim == 2 ? 2 : 1); ++d) {
    const double *e = d == 0 ? c->x_nodes : c->y_nodes;
    const int n = d == 0 ? c->nx : c->ny, off = d == 0 ? 0 : lines_x;
    const int lo = c->bc[2 * d], hi = c->bc[2 * d + 1];
    for (int i = 0; i < n; ++i) {
      const double h = e[i + 1] - e[i];
      arr[off + i] = h;
      arr[lines + off + i] = 2.0 / h;
      arr[2 * lines + off + i] = c->tvb_M * h * h;
      int rc = dg::build_weno_coef(c->order, line_width(e, n, i - 1, lo, hi) / h, line_width(e, n, i + 1, lo, hi) / h,
                                   &tab[off + i]);
      if (rc) return rc;
    }
  }
  double *dv = (double *)(ws + L.mesh);
  dg::WenoCoef *dt = (dg::WenoCoef *)(ws + L.mesh + align_up(3 * (size_t)lines * sizeof(double)));
  if (hipMemcpyAsync(dv, arr.data(), arr.size() * sizeof(double), hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(dt, tab.data(), tab.size() * sizeof(dg::WenoCoef), hipMemcpyHostToDevice, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return DG_ERR_HIP;
  g->hxa = dv;
  g->rhxa = dv + lines;
  g->mhx = dv + 2 * lines;
  g->wtx = dt;
  if (lines_y) {
    g->hya = dv + lines_x;
    g->rhya = dv + lines + lines_x;
    g->mhy = dv + 2 * lines + lines_x;
    g->wty = dt + lines_x;
  }
  return DG_OK;
}

int hip_ok(hipError_t e) { return e == hipSuccess ? DG_OK : DG_ERR_HIP; }

int sync_status(dg_problem *p, DevScalars *host) {
  DevScalars tmp;
  DevScalars *h = host ? host : &tmp;
  if (hipMemcpyAsync(h, p->ctx.sc, sizeof(DevScalars), hipMemcpyDeviceToHost, p->user_stream) != hipSuccess)
    return DG_ERR_HIP;
  if (hipStreamSynchronize(p->user_stream) != hipSuccess) return DG_ERR_HIP;
  return h->status ? DG_ERR_NONPHYSICAL : DG_OK;
}

// Brackets one launch (or a group of launches) with events when profiling.
struct Timed {
  dg_problem *p;
  int slot;
  Timed(dg_problem *p_, int kind) : p(p_), slot(-1) {
    Profiler &f = p->prof;
    if (!f.enabled || f.used + 2 > Profiler::kEvents) return;
    slot = f.used;
    f.kind[slot / 2] = kind;
    f.used += 2;
    (void)hipEventRecord(f.ev[slot], (hipStream_t)p->ctx.stream);
  }
  ~Timed() {
    if (slot >= 0) (void)hipEventRecord(p->prof.ev[slot + 1], (hipStream_t)p->ctx.stream);
  }
};

// Adds the recorded intervals to the accumulators (stream must be idle).
void harvest(dg_problem *p) {
  Profiler &f = p->prof;
  for (int k = 0; k + 1 < f.used; k += 2) {
    float t = 0.0f;
    if (hipEventElapsedTime(&t, f.ev[k], f.ev[k + 1]) == hipSuccess) {
      f.ms[f.kind[k / 2]] += t;
      f.n[f.kind[k / 2]] += 1;
    }
  }
  f.used = 0;
}

// One SSP-RK3 step with the limiter after every stage (enqueue only).
// Boundary data of a stage stand for the time its input approximates: t^n
// for the first residual (decide_dt sets it), t^n + dt for the limiter after
// stage 1 and the second residual, t^n + dt/2 for the limiter after stage 2
// and the third residual, t^n + dt after stage 3.
int enqueue_step(dg_problem *p, double *state, bool cfl_mode) {
  LaunchCtx &c = p->ctx;
  const bool lim = p->cfg.limiter != DG_LIM_NONE, pos = p->cfg.positivity != 0, timed = c.timed_bc != 0;
  int rc;
  auto limit = [&](double *u, double *side, int slot, double frac) {
    int r = DG_OK;
    if (timed) r = dg::launch_set_tb(c, frac, 0.0);
    if (!r && lim) { Timed t(p, DG_PROF_LIMITER); r = dg::launch_limit(c, u, side, slot, c.flags, nullptr, nullptr); }
    if (!r && pos) { Timed t(p, DG_PROF_LIMITER); r = dg::launch_positivity(c, u, 1); }
    return r;
  };
  { Timed t(p, DG_PROF_DT); rc = dg::launch_dt_finalize(c); }
  if (!rc) { Timed t(p, DG_PROF_STAGE1); rc = dg::launch_stage(c, 1, state, nullptr, c.bufA, false); }
  if (!rc) rc = limit(c.bufA, c.bufB, 0, 1.0);
  if (!rc) { Timed t(p, DG_PROF_STAGE23); rc = dg::launch_stage(c, 2, c.bufA, state, c.bufB, false); }
  if (!rc) rc = limit(c.bufB, c.bufA, 1, 0.5);
  if (!rc) { Timed t(p, DG_PROF_STAGE23); rc = dg::launch_stage(c, 3, c.bufB, state, state, cfl_mode); }
  if (!rc) rc = limit(state, c.bufA, 2, 1.0);
  return rc;
}

int build_graph(dg_problem *p, double *state, bool cfl_mode) {
  if (p->graph) {
    (void)hipGraphExecDestroy(p->graph);
    p->graph = nullptr;
  }
  if (!p->capture_stream && hipStreamCreateWithFlags(&p->capture_stream, hipStreamNonBlocking) != hipSuccess)
    return DG_ERR_HIP;
  void *saved = p->ctx.stream;
  p->ctx.stream = p->capture_stream;
  if (hipStreamBeginCapture(p->capture_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    p->ctx.stream = saved;
    return DG_ERR_HIP;
  }
  int rc = enqueue_step(p, state, cfl_mode);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(p->capture_stream, &g);
  p->ctx.stream = saved;
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return DG_ERR_HIP;
  e = hipGraphInstantiate(&p->graph, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    p->graph = nullptr;
    return DG_ERR_HIP;
  }
  p->graph_state = state;
  p->graph_cfl = cfl_mode ? 1 : 0;
  return DG_OK;
}

// Launch context of a configuration on a uniform mesh: geometry, modes and
// the scalar block sc; the state-sized buffers, flags, margins and list are
// left null for the caller to point at its memory.
void fill_ctx(const dg_config *cfg, void *stream, DevScalars *sc, LaunchCtx *out) {
  LaunchCtx &c = *out;
  c = LaunchCtx{};
  c.dim = cfg->dim;
  c.eq = cfg->equation;
  c.N = cfg->order;
  c.nv = dg::num_vars(cfg);
  c.nm = dg::num_modes(cfg);
  dg::fill_geometry(cfg, &c.geo);
  c.stream = stream;
  c.sc = sc;
  c.cfl = cfg->cfl;
  c.limiter = cfg->limiter;
  c.indicator = cfg->indicator;
  c.positivity = cfg->positivity;
  c.timed_bc = 0;
  for (int k = 2; k < 4; ++k)
    if (c.geo.bcb[k] >= 0 && c.geo.bsw[k][1] != 0.0) c.timed_bc = 1;
  c.special_bc = dg::special_bc(c.geo);
  c.geo.tb = &sc->tb;
  c.grid_cap = 2048;
  c.use_march = 1;
  c.rows = 0;
  c.mlp_w = nullptr;
  c.mlp_m = nullptr;
  c.mlp_prob = nullptr;
  c.band_lo = 0.2;
  c.band_hi = 0.8;
}

}  // namespace

extern "C" {

int dg_workspace_bytes(const dg_config *cfg, size_t *bytes) {
  if (!bytes) return DG_ERR_INVALID_ARG;
  int rc = dg::validate_config(cfg);
  if (rc) return rc;
  *bytes = layout(cfg).total;
  return DG_OK;
}

int dg_init(const dg_config *cfg, void *workspace, size_t workspace_bytes, void *stream, dg_problem **out) {
  if (!out) return DG_ERR_INVALID_ARG;
  *out = nullptr;
  int rc = dg::validate_config(cfg);
  if (rc) return rc;
  Layout L = layout(cfg);
  if (!workspace || workspace_bytes < L.total || ((uintptr_t)workspace % kAlign) != 0) return DG_ERR_WORKSPACE;
  int device = 0;
  if (hipGetDevice(&device) != hipSuccess) return DG_ERR_HIP;
  rc = dg::ensure_tables(device);
  if (rc) return rc;
  dg_problem *p = new (std::nothrow) dg_problem();
  if (!p) return DG_ERR_INVALID_ARG;
  p->cfg = *cfg;
  p->cfg.x_nodes = p->cfg.y_nodes = nullptr;  // caller memory: read here only
  p->device = device;
  p->user_stream = (hipStream_t)stream;
  p->ws_bytes = workspace_bytes;
  p->state_elems = (size_t)cfg->nx * cfg->ny * num_vars(cfg) * num_modes(cfg);
  char *ws = (char *)workspace;
  LaunchCtx &c = p->ctx;
  fill_ctx(cfg, stream, (DevScalars *)(ws + L.scalars), &c);
  c.bufA = (double *)(ws + L.bufA);
  c.bufB = (double *)(ws + L.bufB);
  c.flags = (uint8_t *)(ws + L.flags);
  c.margin = (double *)(ws + L.margin);
  c.list = (int32_t *)(ws + L.list);
  if (cfg->x_nodes) {
    rc = upload_mesh(cfg, ws, L, p->user_stream, &c.geo);
    if (rc) {
      delete p;
      return rc;
    }
    c.special_bc = dg::special_bc(c.geo);
  }
  if (hipMemsetAsync(c.sc, 0, sizeof(DevScalars), p->user_stream) != hipSuccess ||
      hipStreamSynchronize(p->user_stream) != hipSuccess) {
    delete p;
    return DG_ERR_HIP;
  }
  *out = p;
  return DG_OK;
}

int dg_destroy(dg_problem *p) {
  if (!p) return DG_OK;
  for (int k = 0; k < Profiler::kEvents; ++k)
    if (p->prof.ev[k]) (void)hipEventDestroy(p->prof.ev[k]);
  if (p->graph) (void)hipGraphExecDestroy(p->graph);
  if (p->capture_stream) (void)hipStreamDestroy(p->capture_stream);
  delete p;
  return DG_OK;
}

int dg_proj_nodes(const dg_problem *p, double *r_nodes, double *weights, int32_t *nq) {
  if (!p || !nq) return DG_ERR_INVALID_ARG;
  dg::OrderTables t;
  int rc = dg::build_order_tables(p->cfg.order, &t);
  if (rc) return rc;
  *nq = t.npq;
  for (int k = 0; k < t.npq; ++k) {
    if (r_nodes) r_nodes[k] = t.rpq[k];
    if (weights) weights[k] = t.wpq[k];
  }
  return DG_OK;
}

int dg_project(dg_problem *p, const double *point_values, int32_t j0, int32_t nrows, double *state) {
  if (!p || !point_values || !state || nrows < 1 || j0 < 0 || j0 + nrows > p->cfg.ny) return DG_ERR_INVALID_ARG;
  int rc = dg::launch_project(p->ctx, point_values, j0, nrows, state);
  if (rc) return rc;
  return hip_ok(hipStreamSynchronize(p->user_stream));
}

int dg_residual(dg_problem *p, const double *state, double *out) {
  if (!p || !state || !out || state == out) return DG_ERR_INVALID_ARG;
  int rc = dg::launch_residual(p->ctx, state, out);
  if (rc) return rc;
  return sync_status(p, nullptr);
}

int dg_limit(dg_problem *p, double *state, uint8_t *flags, double *margin, const uint8_t *flags_override,
             int32_t *n_troubled) {
  if (!p || !state) return DG_ERR_INVALID_ARG;
  if (p->cfg.indicator == DG_IND_LEARNED && !p->ctx.mlp_w && !flags_override) return DG_ERR_INVALID_ARG;
  int rc = dg::launch_reset_counts(p->ctx);
  if (rc) return rc;
  const LaunchCtx &c = p->ctx;  // with DG_LIM_NONE only the indicator runs
  rc = dg::launch_limit(c, state, c.bufA, 3, flags, margin, flags_override);
  if (!rc && p->cfg.positivity) rc = dg::launch_positivity(c, state, 0);
  if (rc) return rc;
  DevScalars h;
  rc = sync_status(p, &h);
  if (n_troubled) *n_troubled = h.count[3];
  return rc;
}

int dg_limit_noalloc(const dg_config *cfg, double *state, uint8_t *flags, double *margin,
                     const uint8_t *flags_override, double t, int32_t *n_troubled, void *stream) {
  if (!state || !std::isfinite(t)) return DG_ERR_INVALID_ARG;
  int rc = dg::validate_config(cfg);
  if (rc) return rc;
  if (cfg->indicator == DG_IND_LEARNED || cfg->x_nodes || cfg->y_nodes) return DG_ERR_UNSUPPORTED;
  const size_t cells = (size_t)cfg->nx * cfg->ny;
  const size_t side_off = dg::kStaticListOffset + align_up(cells * sizeof(int32_t));
  const size_t state_bytes = cells * dg::num_vars(cfg) * dg::num_modes(cfg) * sizeof(double);
  if (side_off + state_bytes > dg::kStaticScratchBytes) return DG_ERR_WORKSPACE;
  int device = 0;
  if (hipGetDevice(&device) != hipSuccess) return DG_ERR_HIP;
  if ((rc = dg::ensure_tables(device))) return rc;
  void *scratch = nullptr;
  if ((rc = dg::static_scratch(device, &scratch))) return rc;
  char *base = (char *)scratch;
  LaunchCtx c;
  fill_ctx(cfg, stream, (DevScalars *)base, &c);
  c.list = (int32_t *)(base + dg::kStaticListOffset);
  c.bufA = (double *)(base + side_off);
  if ((rc = dg::launch_scratch_init(c, t))) return rc;
  rc = dg::launch_limit(c, state, c.bufA, 3, flags, margin, flags_override);
  if (!rc && cfg->positivity) rc = dg::launch_positivity(c, state, 0);
  if (rc) return rc;
  DevScalars h;
  if (hipMemcpyAsync(&h, c.sc, sizeof(DevScalars), hipMemcpyDeviceToHost, (hipStream_t)stream) != hipSuccess ||
      hipStreamSynchronize((hipStream_t)stream) != hipSuccess)
    return DG_ERR_HIP;
  if (n_troubled) *n_troubled = h.count[3];
  return h.status ? DG_ERR_NONPHYSICAL : DG_OK;
}

int dg_set_time(dg_problem *p, double t) {
  if (!p || !std::isfinite(t)) return DG_ERR_INVALID_ARG;
  return dg::launch_set_tb(p->ctx, -1.0, t);
}

int dg_cfl_dt(dg_problem *p, const double *state, double *dt) {
  if (!p || !state || !dt) return DG_ERR_INVALID_ARG;
  int rc = dg::launch_speed(p->ctx, state);
  if (rc) return rc;
  DevScalars h;
  rc = sync_status(p, &h);
  double sx, sy;
  std::memcpy(&sx, &h.smax[0], sizeof(double));
  std::memcpy(&sy, &h.smax[1], sizeof(double));
  const double inf = std::numeric_limits<double>::infinity();
  const bool nu = p->ctx.geo.hxa != nullptr;  // speeds are already per width
  const double hx = nu ? 1.0 : p->ctx.geo.hx, hy = nu ? 1.0 : p->ctx.geo.hy;
  if (p->cfg.dim == 1) {
    *dt = sx > 0.0 ? p->cfg.cfl * hx / sx : inf;
  } else {
    double den = sx / hx + sy / hy;
    *dt = den > 0.0 ? p->cfg.cfl / den : inf;
  }
  return rc;
}

int dg_step(dg_problem *p, double *state, double *t, double t_end, double dt, int32_t max_steps,
            int32_t *steps_taken) {
  if (!p || !state || !t || max_steps < 0) return DG_ERR_INVALID_ARG;
  if (p->cfg.indicator == DG_IND_LEARNED && !p->ctx.mlp_w) return DG_ERR_INVALID_ARG;
  if (steps_taken) *steps_taken = 0;
  if (max_steps == 0 || !(*t < t_end)) return DG_OK;
  const bool cfl_mode = !(dt > 0.0);
  // device scalars for this call
  DevScalars h;
  int rc = sync_status(p, &h);
  if (rc == DG_ERR_HIP) return rc;
  // A non-physical state met before this call is reported by the return
  // value; the step loop starts with a clear status word and ends after the
  // step in which a kernel meets one (the time-step kernel marks the run done).
  const int32_t entry_status = h.status;
  h.status = 0;
  h.t = *t;
  h.t_end = t_end;
  h.dt_fixed = cfl_mode ? 0.0 : dt;
  h.dt = 0.0;
  h.steps = 0;
  h.max_steps = max_steps;
  h.done = 0;
  h.smax[0] = h.smax[1] = 0ull;
  for (int k = 0; k < 4; ++k) h.count[k] = 0;
  if (hipMemcpyAsync(p->ctx.sc, &h, sizeof(DevScalars), hipMemcpyHostToDevice, p->user_stream) != hipSuccess ||
      hipStreamSynchronize(p->user_stream) != hipSuccess)
    return DG_ERR_HIP;
  // the first step's speed; later steps take it from the stage-3 kernel
  if (cfl_mode && (rc = dg::launch_speed(p->ctx, state)) != DG_OK) return rc;
  const bool prof = p->prof.enabled;
  if (!prof && (!p->graph || p->graph_state != state || p->graph_cfl != (cfl_mode ? 1 : 0))) {
    rc = build_graph(p, state, cfl_mode);
    if (rc) return rc;
  }
  long remaining = max_steps;
  long chunk = 8;
  if (!cfl_mode) {
    double n = std::ceil((t_end - *t) / dt) + 1.0;
    if (n < (double)remaining) remaining = (long)n;
    chunk = remaining;
  }
  long launched = 0;
  while (launched < remaining) {
    long k = chunk < remaining - launched ? chunk : remaining - launched;
    if (prof && k > 16) k = 16;  // bounded by the event pool
    for (long s = 0; s < k; ++s) {
      if (prof) {
        rc = enqueue_step(p, state, cfl_mode);
        if (rc) return rc;
      } else if (hipGraphLaunch(p->graph, p->user_stream) != hipSuccess) {
        return DG_ERR_HIP;
      }
    }
    launched += k;
    rc = sync_status(p, &h);
    if (rc == DG_ERR_HIP) return rc;
    if (prof) harvest(p);
    if (h.done) break;
    if (chunk < 256) chunk *= 2;
  }
  if (!h.done) {
    // one more finalize pass decides whether t_end or max_steps was reached
    rc = sync_status(p, &h);
    if (rc == DG_ERR_HIP) return rc;
  }
  *t = h.t;
  if (steps_taken) *steps_taken = h.steps;
  if (entry_status && !h.status) {  // the status word stays set until dg_status reads it
    const int32_t one = 1;
    if (hipMemcpyAsync(&p->ctx.sc->status, &one, sizeof(one), hipMemcpyHostToDevice, p->user_stream) != hipSuccess ||
        hipStreamSynchronize(p->user_stream) != hipSuccess)
      return DG_ERR_HIP;
  }
  return (h.status || entry_status) ? DG_ERR_NONPHYSICAL : DG_OK;
}

int dg_autotune(dg_problem *p, const double *state, int32_t *rows, float *ms) {
  if (!p || !state) return DG_ERR_INVALID_ARG;
  if (rows) *rows = 0;
  if (ms) *ms = 0.f;
  if (p->cfg.dim != 2) return DG_OK;
  static const int kChoices[] = {4, 8, 16, 32, 64};
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return DG_ERR_HIP;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return DG_ERR_HIP;
  }
  int rc = DG_OK, best_rows = 0;
  float best = 1e30f;
  for (int r : kChoices) {
    p->ctx.rows = r;
    if ((rc = dg::launch_residual(p->ctx, state, p->ctx.bufA))) break;  // warm-up
    constexpr int reps = 3;
    (void)hipEventRecord(e0, p->user_stream);
    for (int k = 0; k < reps && !rc; ++k) rc = dg::launch_residual(p->ctx, state, p->ctx.bufA);
    (void)hipEventRecord(e1, p->user_stream);
    if (rc || (rc = hip_ok(hipEventSynchronize(e1)))) break;
    float t = 0.f;
    if ((rc = hip_ok(hipEventElapsedTime(&t, e0, e1)))) break;
    if (t / reps < best) {
      best = t / reps;
      best_rows = r;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  p->ctx.rows = rc ? 0 : best_rows;
  if (p->graph) {  // the captured step holds the old grid
    (void)hipGraphExecDestroy(p->graph);
    p->graph = nullptr;
  }
  if (rc) return rc;
  if (rows) *rows = best_rows;
  if (ms) *ms = best;
  return sync_status(p, nullptr) == DG_ERR_HIP ? DG_ERR_HIP : DG_OK;
}

int dg_status(dg_problem *p) {
  if (!p) return DG_ERR_INVALID_ARG;
  DevScalars h;
  int rc = sync_status(p, &h);
  if (rc == DG_ERR_HIP) return rc;
  if (h.status) {
    int32_t zero = 0;
    if (hipMemcpyAsync(&p->ctx.sc->status, &zero, sizeof(zero), hipMemcpyHostToDevice, p->user_stream) !=
            hipSuccess ||
        hipStreamSynchronize(p->user_stream) != hipSuccess)
      return DG_ERR_HIP;
  }
  return rc;
}

int dg_profile_enable(dg_problem *p, int enable) {
  if (!p) return DG_ERR_INVALID_ARG;
  if (enable && !p->prof.ev[0]) {
    for (int k = 0; k < Profiler::kEvents; ++k)
      if (hipEventCreate(&p->prof.ev[k]) != hipSuccess) return DG_ERR_HIP;
  }
  p->prof.enabled = enable != 0;
  p->prof.used = 0;
  return DG_OK;
}

int dg_profile_read(dg_problem *p, double *ms, int64_t *launches, int64_t *troubled, int reset) {
  if (!p) return DG_ERR_INVALID_ARG;
  DevScalars h;
  int rc = sync_status(p, &h);
  if (rc == DG_ERR_HIP) return rc;
  harvest(p);
  for (int k = 0; k < DG_PROF_KINDS; ++k) {
    if (ms) ms[k] = p->prof.ms[k];
    if (launches) launches[k] = p->prof.n[k];
  }
  if (troubled) *troubled = (int64_t)h.troubled_total;
  if (reset) {
    for (int k = 0; k < DG_PROF_KINDS; ++k) {
      p->prof.ms[k] = 0.0;
      p->prof.n[k] = 0;
    }
    unsigned long long zero = 0;
    if (hipMemcpyAsync(&p->ctx.sc->troubled_total, &zero, sizeof(zero), hipMemcpyHostToDevice, p->user_stream) !=
            hipSuccess ||
        hipStreamSynchronize(p->user_stream) != hipSuccess)
      return DG_ERR_HIP;
  }
  return DG_OK;
}

int dg_mlp_layout(int32_t features, int32_t *padded, int64_t *n_master, int64_t *n_bf16) {
  int kp;
  long nm, nb;
  int rc = dg::mlp_layout(features, &kp, &nm, &nb);
  if (rc) return rc;
  if (padded) *padded = kp;
  if (n_master) *n_master = nm;
  if (n_bf16) *n_bf16 = nb;
  return DG_OK;
}

int dg_mlp_features(dg_problem *p, const double *state, float *f32, uint16_t *bf16) {
  if (!p || !state || (!f32 && !bf16) || p->cfg.dim != 2) return DG_ERR_INVALID_ARG;
  const int F = 5 * p->ctx.nm * p->ctx.nv;
  int kp;
  int rc = dg::mlp_layout(F, &kp, nullptr, nullptr);
  if (!rc) rc = dg::launch_mlp_features(p->ctx, state, f32, bf16, kp);
  if (rc) return rc;
  return hip_ok(hipStreamSynchronize(p->user_stream));
}

int dg_mlp_forward(const uint16_t *x, int32_t n, int32_t features, const uint16_t *w_bf16, const float *master,
                   float *prob, void *stream) {
  if (!x || !w_bf16 || !master || !prob || n < 0) return DG_ERR_INVALID_ARG;
  int rc = dg::launch_mlp_forward(x, n, features, w_bf16, master, prob, stream);
  if (rc) return rc;
  return hip_ok(hipStreamSynchronize((hipStream_t)stream));
}

int dg_mlp_gradient(const uint16_t *x, const float *y, const float *wgt, int32_t n, int32_t features,
                    const uint16_t *w_bf16, const float *master, float *grad, uint16_t *dh1, float *loss,
                    void *stream) {
  if (!x || !y || !wgt || !w_bf16 || !master || !grad || !dh1 || !loss || n < 0) return DG_ERR_INVALID_ARG;
  int rc = dg::launch_mlp_gradient(x, y, wgt, n, features, w_bf16, master, grad, dh1, loss, stream);
  if (rc) return rc;
  return hip_ok(hipStreamSynchronize((hipStream_t)stream));
}

int dg_mlp_adam(float *master, float *adam_m, float *adam_v, float *grad, uint16_t *w_bf16, int32_t features,
                float lr, int32_t step, void *stream) {
  if (!master || !w_bf16 || step < 0 || (step > 0 && (!adam_m || !adam_v || !grad))) return DG_ERR_INVALID_ARG;
  int rc = dg::launch_mlp_adam(master, adam_m, adam_v, grad, w_bf16, features, lr, step, stream);
  if (rc) return rc;
  return hip_ok(hipStreamSynchronize((hipStream_t)stream));
}

int dg_set_learned(dg_problem *p, const uint16_t *w_bf16, const float *master, double band_lo, double band_hi,
                   float *prob) {
  if (!p || !w_bf16 || !master || !(band_lo <= band_hi) || p->cfg.dim != 2) return DG_ERR_INVALID_ARG;
  p->ctx.mlp_w = w_bf16;
  p->ctx.mlp_m = master;
  p->ctx.band_lo = band_lo;
  p->ctx.band_hi = band_hi;
  p->ctx.mlp_prob = prob;
  if (p->graph) {  // the captured step holds the old arguments
    (void)hipGraphExecDestroy(p->graph);
    p->graph = nullptr;
  }
  return DG_OK;
}

const char *dg_strerror(int code) {
  switch (code) {
    case DG_OK: return "ok";
    case DG_ERR_INVALID_ARG: return "invalid argument";
    case DG_ERR_UNSUPPORTED: return "unsupported configuration";
    case DG_ERR_WORKSPACE: return "workspace too small or misaligned";
    case DG_ERR_HIP: return "HIP runtime error";
    case DG_ERR_NONPHYSICAL: return "non-physical state (density or pressure <= 0, or NaN)";
    default: return "unknown error";
  }
}

}  // extern "C"
