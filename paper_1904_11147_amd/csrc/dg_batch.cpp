// C-ABI of the batched execution (declared in include/dg.h): workspace
// layout, instance descriptors, the captured batch step and the tile-shape
// autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

#include "dg_internal.h"

using dg::BatchCtx;
using dg::BatchInst;
using dg::BatchQueue;
using dg::DevScalars;
using dg::kMaxN;

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

constexpr int kRowChoices[] = {4, 8, 16, 32, 64};
// columns per stage tile (the stage kernel's strip width: two lanes per cell
// for Q1, Q2, four for Q3)
constexpr int strip_cols(int order) { return order == 3 ? 14 : 30; }

struct BatchLayout {
  size_t active, scalars, inst, queue, list[kMaxN + 1], bufs, total;
  std::vector<size_t> state_bytes;
};

size_t cells_of(const dg_config &c) { return (size_t)c.nx * c.ny; }

int validate_batch(const dg_config *cfgs, int32_t n) {
  if (!cfgs || n < 1 || n > dg::kBatchMax) return DG_ERR_INVALID_ARG;
  long long cells = 0;
  for (int i = 0; i < n; ++i) {
    int rc = dg::validate_config(&cfgs[i]);
    if (rc) return rc;
    if (cfgs[i].dim != 2 || cfgs[i].equation != DG_EQ_EULER) return DG_ERR_UNSUPPORTED;
    if (cfgs[i].limiter != cfgs[0].limiter || cfgs[i].indicator != cfgs[0].indicator) return DG_ERR_INVALID_ARG;
    // walls, inflow and switching sides and non-uniform meshes run on single meshes only
    for (int k = 0; k < 4; ++k)
      if (cfgs[i].bc[k] != DG_BC_PERIODIC && cfgs[i].bc[k] != DG_BC_TRANSMISSIVE) return DG_ERR_UNSUPPORTED;
    if (cfgs[i].positivity != cfgs[0].positivity) return DG_ERR_INVALID_ARG;
    if (cfgs[i].bc_beyond[2] >= 0 || cfgs[i].bc_beyond[3] >= 0 || cfgs[i].x_nodes) return DG_ERR_UNSUPPORTED;
    // the batched stage kernel addresses an instance's state with 32-bit byte offsets
    const long long n_i = (long long)cfgs[i].nx * cfgs[i].ny;
    if (32ll * (cfgs[i].order + 1) * (cfgs[i].order + 1) * n_i > (1ll << 32)) return DG_ERR_UNSUPPORTED;
    cells += n_i;
  }
  if (cells > (1ll << 31) - 1) return DG_ERR_UNSUPPORTED;
  return DG_OK;
}

BatchLayout batch_layout(const dg_config *cfgs, int32_t n) {
  BatchLayout L;
  size_t off = 0;
  L.active = off;
  off += align_up(sizeof(int32_t));
  L.scalars = off;
  off += align_up(n * sizeof(DevScalars));
  L.inst = off;
  off += align_up(n * sizeof(BatchInst));
  L.queue = off;
  off += align_up((kMaxN + 1) * sizeof(BatchQueue));
  size_t cells_by_order[kMaxN + 1] = {};
  for (int i = 0; i < n; ++i) cells_by_order[cfgs[i].order] += cells_of(cfgs[i]);
  for (int o = 0; o <= kMaxN; ++o) {
    L.list[o] = off;
    off += align_up(cells_by_order[o] * sizeof(long long));
  }
  L.bufs = off;
  L.state_bytes.resize(n);
  for (int i = 0; i < n; ++i) {
    L.state_bytes[i] = cells_of(cfgs[i]) * dg::num_vars(&cfgs[i]) * dg::num_modes(&cfgs[i]) * sizeof(double);
    off += 2 * align_up(L.state_bytes[i]);
  }
  L.total = off;
  return L;
}

int hip_ok(hipError_t e) { return e == hipSuccess ? DG_OK : DG_ERR_HIP; }

}  // namespace

struct dg_batch {
  int n = 0, device = 0, cus = 256;
  std::vector<dg_config> cfg;
  std::vector<BatchInst> inst;  // host copy of the descriptors
  std::vector<size_t> state_elems;
  BatchCtx ctx{};
  DevScalars *sc = nullptr;  // device [n]
  hipStream_t user_stream = nullptr, capture_stream = nullptr;
  // per-order branches of the captured step (orders after the first present
  // one run on their own stream between a fork and a join event)
  hipStream_t branch[kMaxN + 1] = {};
  hipEvent_t fork = nullptr, join[kMaxN + 1] = {};
  hipGraphExec_t graph = nullptr;
  int present[kMaxN + 1] = {};
  int rows[kMaxN + 1] = {};
  int grid[kMaxN + 1] = {};
  const double *states = nullptr;  // buffer the descriptors point into
  std::vector<int64_t> offsets;
};

namespace {

void drop_graph(dg_batch *b) {
  if (b->graph) (void)hipGraphExecDestroy(b->graph);
  b->graph = nullptr;
}

// Tile height of one order; the stage grid of that order is its full tile count.
void set_rows(dg_batch *b, int order, int rows) {
  b->rows[order] = rows;
  long tiles = 0;
  for (int i = 0; i < b->n; ++i) {
    BatchInst &I = b->inst[i];
    if (I.order != order) continue;
    I.rows = rows;
    I.tiles_y = (I.geo.ny + rows - 1) / rows;
    tiles += (long)I.tiles_x * I.tiles_y;
  }
  b->grid[order] = (int)tiles;
}

int upload_inst(dg_batch *b) {
  if (hipMemcpyAsync(b->ctx.inst, b->inst.data(), b->n * sizeof(BatchInst), hipMemcpyHostToDevice,
                     b->user_stream) != hipSuccess)
    return DG_ERR_HIP;
  return hip_ok(hipStreamSynchronize(b->user_stream));
}

// Learned-indicator probability outputs of the instances, at the states' offsets.
void set_prob_pointers(dg_batch *b) {
  for (int i = 0; i < b->n; ++i) {
    float *base = b->ctx.learned[b->inst[i].order].prob;
    b->inst[i].prob = (base && b->states) ? base + b->offsets[i] : nullptr;
  }
}

// Points the descriptors at the caller's states (uploaded when they change).
int set_states(dg_batch *b, double *states, const int64_t *offsets) {
  if (!states || !offsets) return DG_ERR_INVALID_ARG;
  std::vector<int> order(b->n);
  std::iota(order.begin(), order.end(), 0);
  for (int i = 0; i < b->n; ++i)
    if (offsets[i] < 0 || offsets[i] % 32 != 0) return DG_ERR_INVALID_ARG;
  std::sort(order.begin(), order.end(), [&](int x, int y) { return offsets[x] < offsets[y]; });
  for (int k = 0; k + 1 < b->n; ++k)
    if (offsets[order[k]] + (int64_t)b->state_elems[order[k]] > offsets[order[k + 1]]) return DG_ERR_INVALID_ARG;
  bool same = b->states == states;
  for (int i = 0; same && i < b->n; ++i) same = b->offsets[i] == offsets[i];
  if (same) return DG_OK;
  for (int i = 0; i < b->n; ++i) {
    b->inst[i].u = states + offsets[i];
    b->offsets[i] = offsets[i];
  }
  b->states = states;
  set_prob_pointers(b);
  return upload_inst(b);
}

// Writes every instance's scalars for a call.
int write_scalars(dg_batch *b, const double *t, const double *t_end, int32_t max_steps) {
  std::vector<DevScalars> h(b->n);
  for (int i = 0; i < b->n; ++i) {
    DevScalars &s = h[i];
    std::memset(&s, 0, sizeof(s));
    s.t = t ? t[i] : 0.0;
    s.t_end = t_end ? t_end[i] : 1.0;
    s.max_steps = max_steps;
    s.done = (max_steps == 0 || !(s.t < s.t_end)) ? 1 : 0;
  }
  if (hipMemcpyAsync(b->sc, h.data(), b->n * sizeof(DevScalars), hipMemcpyHostToDevice, b->user_stream) !=
      hipSuccess)
    return DG_ERR_HIP;
  return hip_ok(hipStreamSynchronize(b->user_stream));
}

// One batched SSP-RK3 step (enqueue only): time-step decisions and queues,
// then the three stages, each followed by its limiter pass.  The orders
// touch disjoint instances, queues and lists, so their chains are
// independent.  With the learned indicator (whose passes leave most of the
// GPU idle: few blocks, each holding a network in LDS) the first present
// order runs on the step's stream and each other one on a branch stream
// forked after the decision and joined at the end (parallel branches of the
// captured graph, which the GPU may run at once).  Otherwise one stream runs
// each stage of all orders, then their limiter passes (concurrent stage
// kernels, each sized to fill the GPU, only contend).
int enqueue_batch_step(dg_batch *b) {
  int rc = dg::batch_launch_decide(b->ctx, 1);
  const bool limit = b->ctx.limiter != DG_LIM_NONE || b->ctx.positivity;
  if (b->ctx.indicator != DG_IND_LEARNED) {
    for (int stage = 1; stage <= 3 && !rc; ++stage) {
      for (int o = 1; o <= kMaxN && !rc; ++o)
        if (b->present[o]) rc = dg::batch_launch_stage(b->ctx, o, stage, b->grid[o]);
      if (!limit) continue;
      for (int o = 1; o <= kMaxN && !rc; ++o)
        if (b->present[o]) rc = dg::batch_launch_limit(b->ctx, o, stage - 1);
    }
    return rc;
  }
  if (rc) return rc;
  const hipStream_t st0 = (hipStream_t)b->ctx.stream;
  int first = 0;
  for (int o = 1; o <= kMaxN && !first; ++o)
    if (b->present[o]) first = o;
  if (hipEventRecord(b->fork, st0) != hipSuccess) return DG_ERR_HIP;
  for (int o = 1; o <= kMaxN && !rc; ++o) {
    if (!b->present[o]) continue;
    dg::BatchCtx c = b->ctx;
    if (o != first) {
      if (hipStreamWaitEvent(b->branch[o], b->fork, 0) != hipSuccess) return DG_ERR_HIP;
      c.stream = b->branch[o];
    }
    for (int stage = 1; stage <= 3 && !rc; ++stage) {
      rc = dg::batch_launch_stage(c, o, stage, b->grid[o]);
      if (!rc && limit) rc = dg::batch_launch_limit(c, o, stage - 1);
    }
    if (!rc && o != first) {
      if (hipEventRecord(b->join[o], b->branch[o]) != hipSuccess || hipStreamWaitEvent(st0, b->join[o], 0) != hipSuccess)
        return DG_ERR_HIP;
    }
  }
  return rc;
}

// Streams and events of the per-order branches (created once, default priority).
int make_branches(dg_batch *b) {
  if (!b->fork && hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess) return DG_ERR_HIP;
  for (int o = 1; o <= kMaxN; ++o) {
    if (!b->branch[o] && hipStreamCreateWithFlags(&b->branch[o], hipStreamNonBlocking) != hipSuccess) return DG_ERR_HIP;
    if (!b->join[o] && hipEventCreateWithFlags(&b->join[o], hipEventDisableTiming) != hipSuccess) return DG_ERR_HIP;
  }
  return DG_OK;
}

int build_batch_graph(dg_batch *b) {
  drop_graph(b);
  if (!b->capture_stream && hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking) != hipSuccess)
    return DG_ERR_HIP;
  if (b->ctx.indicator == DG_IND_LEARNED)
    if (int r = make_branches(b)) return r;
  void *saved = b->ctx.stream;
  b->ctx.stream = b->capture_stream;
  if (hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    b->ctx.stream = saved;
    return DG_ERR_HIP;
  }
  int rc = enqueue_batch_step(b);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(b->capture_stream, &g);
  b->ctx.stream = saved;
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return DG_ERR_HIP;
  e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    b->graph = nullptr;
    return DG_ERR_HIP;
  }
  return DG_OK;
}

int read_active(dg_batch *b, int32_t *active) {
  if (hipMemcpyAsync(active, b->ctx.active, sizeof(int32_t), hipMemcpyDeviceToHost, b->user_stream) != hipSuccess)
    return DG_ERR_HIP;
  return hip_ok(hipStreamSynchronize(b->user_stream));
}

}  // namespace

extern "C" {

int dg_batch_workspace_bytes(const dg_config *cfgs, int32_t n, size_t *bytes) {
  if (!bytes) return DG_ERR_INVALID_ARG;
  int rc = validate_batch(cfgs, n);
  if (rc) return rc;
  *bytes = batch_layout(cfgs, n).total;
  return DG_OK;
}

int dg_batch_init(const dg_config *cfgs, int32_t n, void *workspace, size_t workspace_bytes, void *stream,
                  dg_batch **out) {
  if (!out) return DG_ERR_INVALID_ARG;
  *out = nullptr;
  int rc = validate_batch(cfgs, n);
  if (rc) return rc;
  BatchLayout L = batch_layout(cfgs, n);
  if (!workspace || workspace_bytes < L.total || ((uintptr_t)workspace % kAlign) != 0) return DG_ERR_WORKSPACE;
  int device = 0;
  if (hipGetDevice(&device) != hipSuccess) return DG_ERR_HIP;
  rc = dg::ensure_tables(device);
  if (rc) return rc;
  dg_batch *b = new (std::nothrow) dg_batch();
  if (!b) return DG_ERR_INVALID_ARG;
  b->n = n;
  b->device = device;
  if (hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || b->cus < 1)
    b->cus = 256;
  b->user_stream = (hipStream_t)stream;
  b->cfg.assign(cfgs, cfgs + n);
  b->offsets.assign(n, -1);
  b->state_elems.resize(n);
  char *ws = (char *)workspace;
  BatchCtx &c = b->ctx;
  c.n = n;
  c.inst = (BatchInst *)(ws + L.inst);
  c.queue = (BatchQueue *)(ws + L.queue);
  c.active = (int32_t *)(ws + L.active);
  c.stream = stream;
  c.limiter = cfgs[0].limiter;
  c.indicator = cfgs[0].indicator;
  c.positivity = cfgs[0].positivity;
  c.grid_cap = 2048;
  b->sc = (DevScalars *)(ws + L.scalars);
  b->inst.resize(n);
  size_t off = L.bufs;
  for (int i = 0; i < n; ++i) {
    const dg_config &cf = cfgs[i];
    BatchInst &I = b->inst[i];
    std::memset(&I, 0, sizeof(I));
    dg::fill_geometry(&cf, &I.geo);
    I.u = nullptr;
    I.A = (double *)(ws + off);
    off += align_up(L.state_bytes[i]);
    I.B = (double *)(ws + off);
    off += align_up(L.state_bytes[i]);
    I.sc = b->sc + i;
    I.order = cf.order;
    I.tiles_x = (cf.nx + strip_cols(cf.order) - 1) / strip_cols(cf.order);
    I.segs = (cf.nx + 63) / 64 * cf.ny;
    I.ltiles = ((cf.nx + dg::kLmStrip - 1) / dg::kLmStrip + dg::lm_waves(cf.order) - 1) / dg::lm_waves(cf.order) *
               ((cf.ny + dg::kLmRows - 1) / dg::kLmRows);
    I.indicator = cf.indicator;
    I.cfl = cf.cfl;
    b->state_elems[i] = L.state_bytes[i] / sizeof(double);
    b->present[cf.order] = 1;
  }
  for (int o = 0; o <= kMaxN; ++o) c.list[o] = (long long *)(ws + L.list[o]);
  for (int o = 1; o <= kMaxN; ++o) set_rows(b, o, 16);
  if (hipMemsetAsync(ws, 0, L.bufs, b->user_stream) != hipSuccess || upload_inst(b) != DG_OK) {
    delete b;
    return DG_ERR_HIP;
  }
  *out = b;
  return DG_OK;
}

int dg_batch_destroy(dg_batch *b) {
  if (!b) return DG_OK;
  drop_graph(b);
  if (b->capture_stream) (void)hipStreamDestroy(b->capture_stream);
  for (int o = 1; o <= kMaxN; ++o) {
    if (b->branch[o]) (void)hipStreamDestroy(b->branch[o]);
    if (b->join[o]) (void)hipEventDestroy(b->join[o]);
  }
  if (b->fork) (void)hipEventDestroy(b->fork);
  delete b;
  return DG_OK;
}

int dg_batch_set_tiles(dg_batch *b, int32_t order, int32_t rows) {
  if (!b || order < 1 || order > kMaxN || rows < 1) return DG_ERR_INVALID_ARG;
  set_rows(b, order, rows);
  drop_graph(b);
  return upload_inst(b);
}

int dg_batch_autotune(dg_batch *b, double *states, const int64_t *offsets, int32_t *rows, int32_t *tiles,
                      float *ms) {
  if (!b) return DG_ERR_INVALID_ARG;
  int rc = set_states(b, states, offsets);
  if (rc) return rc;
  rc = write_scalars(b, nullptr, nullptr, 1);  // every instance queued
  if (rc) return rc;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return DG_ERR_HIP;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return DG_ERR_HIP;
  }
  for (int o = 1; o <= kMaxN && !rc; ++o) {
    if (rows) rows[o] = 0;
    if (tiles) tiles[o] = 0;
    if (ms) ms[o] = 0.f;
    if (!b->present[o]) continue;
    float best = 1e30f;
    int best_rows = b->rows[o];
    for (int r : kRowChoices) {
      set_rows(b, o, r);
      if ((rc = upload_inst(b)) || (rc = dg::batch_launch_decide(b->ctx, 0))) break;
      if ((rc = dg::batch_launch_stage(b->ctx, o, 0, b->grid[o]))) break;  // warm-up
      constexpr int reps = 3;
      (void)hipEventRecord(e0, b->user_stream);
      for (int k = 0; k < reps && !rc; ++k) rc = dg::batch_launch_stage(b->ctx, o, 0, b->grid[o]);
      (void)hipEventRecord(e1, b->user_stream);
      if (rc || (rc = hip_ok(hipEventSynchronize(e1)))) break;
      float t = 0.f;
      if ((rc = hip_ok(hipEventElapsedTime(&t, e0, e1)))) break;
      t /= reps;
      if (t < best) {
        best = t;
        best_rows = r;
      }
    }
    set_rows(b, o, best_rows);
    if (rows) rows[o] = best_rows;
    if (tiles) tiles[o] = b->grid[o];
    if (ms) ms[o] = best;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  drop_graph(b);
  int rc2 = upload_inst(b);
  return rc ? rc : rc2;
}

int dg_batch_set_learned(dg_batch *b, int32_t order, const uint16_t *w_bf16, const float *master, double band_lo,
                         double band_hi, float *prob) {
  if (!b || order < 1 || order > kMaxN || !w_bf16 || !master || !(band_lo <= band_hi)) return DG_ERR_INVALID_ARG;
  b->ctx.learned[order] = dg::BatchLearned{w_bf16, master, (float)band_lo, (float)band_hi, prob};
  drop_graph(b);
  set_prob_pointers(b);
  return b->states ? upload_inst(b) : DG_OK;
}

int dg_batch_step(dg_batch *b, double *states, const int64_t *offsets, double *t, const double *t_end,
                  int32_t max_steps, int32_t *steps, int32_t *status, int64_t *troubled) {
  if (!b || !t || !t_end || max_steps < 0) return DG_ERR_INVALID_ARG;
  if (b->ctx.indicator == DG_IND_LEARNED)
    for (int o = 1; o <= kMaxN; ++o)
      if (b->present[o] && !b->ctx.learned[o].W) return DG_ERR_INVALID_ARG;
  int rc = set_states(b, states, offsets);
  if (rc) return rc;
  if ((rc = write_scalars(b, t, t_end, max_steps))) return rc;
  // queues of the instances that start, and their first CFL speeds
  if ((rc = dg::batch_launch_decide(b->ctx, 0))) return rc;
  for (int o = 1; o <= kMaxN && !rc; ++o)
    if (b->present[o]) rc = dg::batch_launch_speed(b->ctx, o);
  if (rc) return rc;
  if (!b->graph && (rc = build_batch_graph(b))) return rc;
  int32_t active = 0;
  if ((rc = read_active(b, &active))) return rc;
  long chunk = 8;
  while (active > 0) {
    for (long k = 0; k < chunk; ++k)
      if (hipGraphLaunch(b->graph, b->user_stream) != hipSuccess) return DG_ERR_HIP;
    if ((rc = read_active(b, &active))) return rc;
    if (chunk < 256) chunk *= 2;
  }
  std::vector<DevScalars> h(b->n);
  if (hipMemcpyAsync(h.data(), b->sc, b->n * sizeof(DevScalars), hipMemcpyDeviceToHost, b->user_stream) !=
          hipSuccess ||
      hipStreamSynchronize(b->user_stream) != hipSuccess)
    return DG_ERR_HIP;
  int any_bad = 0;
  int64_t tr = 0;
  for (int i = 0; i < b->n; ++i) {
    t[i] = h[i].t;
    if (steps) steps[i] = h[i].steps;
    if (status) status[i] = h[i].status ? DG_ERR_NONPHYSICAL : DG_OK;
    any_bad |= h[i].status ? 1 : 0;
    tr += (int64_t)h[i].troubled_total;
  }
  if (troubled) *troubled = tr;
  return any_bad ? DG_ERR_NONPHYSICAL : DG_OK;
}

}  // extern "C"
