// Internal declarations shared by the host side of libdg (tables, C-ABI) and
// the HIP kernel translation unit.  Not part of the public ABI.
#pragma once

#include <cstddef>
#include <cstdint>

#include "../../include/dg.h"

namespace dg {

constexpr int kMaxN = 3;
constexpr int kMaxP = kMaxN + 1;  // N+1
constexpr int kMaxG = 4;          // reconstruction points per direction
constexpr int kMaxPQ = 10;        // projection nodes per direction

// Coefficients of one order N, in double, as the kernels read them.
struct OrderTables {
  int32_t N, ng, npq, pad;
  double wq[kMaxP];           // (N+1)-point Gauss weights on [-1,1]
  double bq[kMaxP][kMaxP];    // psi_n(r_q)            [n][q]
  double dbq[kMaxP][kMaxP];   // psi_n'(r_q)           [n][q]
  double bm[kMaxP], bp[kMaxP], b0[kMaxP];  // psi_n(-1), psi_n(+1), psi_n(0)
  double wg[kMaxG];           // reconstruction-rule weights (sum 2)
  double bg[kMaxP][kMaxG];    // psi_n(r_G)            [n][G]
  double T[kMaxG][kMaxP][kMaxP];  // p_i(x_G) = sum_k T[G][i][k] a[i+k]
  double gam[kMaxG][kMaxP];       // linear weights
  int32_t split[kMaxG];           // point has a negative linear weight
  double gpn[kMaxG][kMaxP], gmn[kMaxG][kMaxP];  // split groups, normalised
  double sp[kMaxG], sm[kMaxG];                  // split group sums
  double B[kMaxP][kMaxP][kMaxP];  // beta_i = sum_kl B[i][k][l] a[i+k] a[i+l]
  double sub[kMaxP][kMaxP];       // mean of psi_n over subcell k of [-1,1]  [k][n]
  double rpq[kMaxPQ], wpq[kMaxPQ];
  double bpq[kMaxP][kMaxPQ];      // psi_n at the projection nodes
};

// Builds the tables of order N (1..3) on the host.  Returns 0 or a DG_ERR code.
int build_order_tables(int N, OrderTables *out);

// The stencil-dependent part of the tables (members named as in
// OrderTables) for a troubled cell whose left and right neighbours are rl and
// rr times as wide as itself: non-uniform meshes keep one per column (x
// sweeps) and one per row (y sweeps).
struct WenoCoef {
  double T[kMaxG][kMaxP][kMaxP];
  double gam[kMaxG][kMaxP];
  int32_t split[kMaxG];
  double gpn[kMaxG][kMaxP], gmn[kMaxG][kMaxP];
  double sp[kMaxG], sm[kMaxG];
  double B[kMaxP][kMaxP][kMaxP];
};
int build_weno_coef(int N, double rl, double rr, WenoCoef *out);

// Uploads tables of all orders to the current device, one call per part of
// the kernel code (each part is its own code object with its own copy).
constexpr int kKernelParts = 6;
int upload_tables_part0(const OrderTables *tabs /* [kMaxN+1], index N */);
int upload_tables_part1(const OrderTables *tabs);
int upload_tables_part2(const OrderTables *tabs);
int upload_tables_part3(const OrderTables *tabs);
int upload_tables_part4(const OrderTables *tabs);
int upload_tables_part5(const OrderTables *tabs);

// Device scalars at the head of the workspace.
struct DevScalars {
  unsigned long long smax[2];  // max spectral radius (bits of a positive double), x and y
  double dt;
  double t;
  double t_end;
  double dt_fixed;
  int32_t steps;
  int32_t max_steps;
  int32_t done;
  int32_t status;
  int32_t count[4];  // troubled-cell counts: stage 1..3, standalone limiter
  unsigned long long troubled_total;  // all troubled cells flagged since the last reset
  int32_t count_scratch;  // the learned pass's own list (rebuilt in row order after it)
  int32_t pad[3];
  double tn;  // start time of the current step
  double tb;  // time of the boundary data of the kernels running now
};

struct Geometry {
  int32_t nx, ny;
  int32_t bc[4];
  double hx, hy;     // cell widths
  double rhx, rhy;   // 2/hx, 2/hy
  double gamma;
  double tvb_Mx, tvb_My;  // M hx^2, M hy^2
  double eps;
  int32_t negw_raw;
  int32_t pad;
  double kx_scale;  // KXRCF: 1 / h^((N+1)/2), h the cell's circumscribed radius
  double tvb_M;
  // non-uniform tensor-product meshes (device, null on uniform meshes): per
  // column / row width, 2 / width, M width^2 and the stencil tables
  const double *hxa, *hya, *rhxa, *rhya, *mhx, *mhy;
  const WenoCoef *wtx, *wty;
  double x0;        // west end of the mesh
  int32_t bcb[4];   // south/north: kind beyond the switch point, -1 none
  double bsw[4][2]; // switch at bsw[s][0] + bsw[s][1] * t (x along the side)
  double bst[8][4]; // inflow ghost modes: [2 side + part][variable], the lowest mode only
  const double *tb; // device: time of the boundary data (DevScalars::tb)
};

struct Kernels;  // launch helpers live in the kernel TU

// Work of one call, described to the kernel TU.
struct LaunchCtx {
  int dim, eq, N, nv, nm;
  Geometry geo;
  void *stream;
  DevScalars *sc;        // device
  double *bufA, *bufB;   // device, state-sized
  uint8_t *flags;        // device [cells]
  double *margin;        // device [cells]
  int32_t *list;         // device [cells]
  double cfl;
  int limiter, indicator;
  int positivity;        // Zhang-Shu scaling after every limiter pass
  int timed_bc;          // a side switches at a moving point: keep DevScalars::tb current
  int special_bc;        // a wall, inflow or switching side (else periodic / transmissive only)
  int grid_cap;          // blocks for list-driven kernels
  int use_march;         // 2D: marching stage kernel where registers allow
  int rows;              // 2D marching kernels: rows per tile (0: a rule from the mesh size)
  const uint16_t *mlp_w; // learned indicator: bf16 weights (caller-owned)
  const float *mlp_m;    // fp32 master parameters (biases read from here)
  float *mlp_prob;       // optional per-cell probability output
  double band_lo, band_hi;
};

// Work layout of the learned indicator kernels: blocks of lm_waves(N)
// wavefronts, each marching kLmRows rows of a kLmStrip-column strip.
constexpr int kLmStrip = 14, kLmRows = 16;
constexpr int lm_waves(int order) { return order == 3 ? 8 : 4; }  // constexpr: usable in device code too
constexpr int lm_occupancy(int order) { return order == 3 ? 2 : 3; }  // wavefronts per SIMD the kernels are built for

// ---------------------------------------------------------------------------
// Batched execution: many independent 2D Euler meshes of any size and order,
// each with its own time step, advanced together.
// ---------------------------------------------------------------------------
constexpr int kBatchMax = 4096;  // instances per batch

// One instance, in device memory.
struct BatchInst {
  Geometry geo;
  double *u;           // state (caller-owned, inside the batch's states buffer)
  double *A, *B;       // stage buffers (workspace)
  DevScalars *sc;      // this instance's scalars (workspace)
  int32_t order;       // N
  int32_t rows;        // rows per stage-kernel tile
  int32_t tiles_x, tiles_y;
  int32_t segs;        // 64-cell row segments (indicator work items)
  int32_t ltiles;      // learned-indicator blocks (lm_waves strips x kLmRows rows)
  int32_t indicator;   // DG_IND_*
  int32_t pad;
  double cfl;
  float *prob;         // learned indicator: p of every cell at each pass (optional, caller memory)
};

// Work queue of the instances of one order, rebuilt on the device after every
// time-step decision.  Entries are the active instances in index order with
// inclusive prefix sums of their stage tiles and indicator segments.
struct BatchQueue {
  int32_t n_active, total_tiles, total_segs, total_ltiles;
  int32_t count[4];  // troubled-list length of the limiter pass after stage 1, 2, 3
  int32_t inst[kBatchMax];
  int32_t tile_end[kBatchMax];
  int32_t seg_end[kBatchMax];
  int32_t ltile_end[kBatchMax];
};

struct BatchLearned {  // learned indicator of one order (null weights: not set)
  const uint16_t *W;
  const float *M;
  float band_lo, band_hi;
  float *prob;  // optional: p of instance i's cell c at prob[offsets[i] + c]
};

// Work of one batched call, described to the kernel TU.
struct BatchCtx {
  int n;                 // instances
  BatchInst *inst;       // device [n]
  BatchQueue *queue;     // device [kMaxN + 1], indexed by order
  int32_t *active;       // device: instances still advancing after the last decision
  long long *list[kMaxN + 1];  // device, per order: troubled entries (instance << 32 | cell)
  void *stream;
  int limiter, indicator;  // one of each for the whole batch
  int positivity;          // Zhang-Shu scaling after every limiter pass (all instances)
  int grid_cap;          // blocks of list-driven and indicator kernels
  BatchLearned learned[kMaxN + 1];
};

// Host helpers of the C-ABI (dg_api.cpp).
int validate_config(const dg_config *c);
int ensure_tables(int device);
void fill_geometry(const dg_config *cfg, Geometry *g);
bool special_bc(const Geometry &g);  // a wall, inflow or switching side
int num_vars(const dg_config *c);
int num_modes(const dg_config *c);

// Kernel-TU entry points (host functions, enqueue only).
int launch_residual(const LaunchCtx &c, const double *u, double *out);
int launch_stage(const LaunchCtx &c, int stage, const double *u, const double *un, double *out, bool want_speed);
// The stage launches of one order (stage 0: residual of u into out).
int launch_stage_order1(const LaunchCtx &c, int stage, const double *u, const double *un, double *out, bool want_speed);
int launch_stage_order2(const LaunchCtx &c, int stage, const double *u, const double *un, double *out, bool want_speed);
int launch_stage_order3(const LaunchCtx &c, int stage, const double *u, const double *un, double *out, bool want_speed);
int launch_limit(const LaunchCtx &c, double *u, double *side, int count_slot, uint8_t *flags, double *margin,
                 const uint8_t *flags_override);
// Allocation-free limiter call: the device address of this device's static
// scratch array (kStaticScratchBytes; looked up once per device), and a
// kernel that clears its count and status words and sets the boundary time.
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
constexpr size_t kStaticListOffset = 256;
int static_scratch(int device, void **ptr);
int launch_scratch_init(const LaunchCtx &c, double tb);
int launch_speed(const LaunchCtx &c, const double *u);
int launch_dt_finalize(const LaunchCtx &c);
// Positivity scaling of every cell of u (Euler); check_done: skip once the
// step loop is done (calls inside dg_step).
int launch_positivity(const LaunchCtx &c, double *u, int check_done);
// DevScalars::tb = tn + frac * dt (frac < 0: = value).
int launch_set_tb(const LaunchCtx &c, double frac, double value);
int launch_reset_counts(const LaunchCtx &c);
int launch_project(const LaunchCtx &c, const double *pv, int j0, int nrows, double *u);
int launch_mlp_features(const LaunchCtx &c, const double *u, float *f32, uint16_t *bf, int KP);
int mlp_layout(int F, int *KP, long *nmaster, long *nbf16);
int launch_mlp_forward(const uint16_t *x, int n, int F, const uint16_t *W, const float *M, float *p, void *stream);
int launch_mlp_gradient(const uint16_t *x, const float *y, const float *w, int n, int F, const uint16_t *W,
                        const float *M, float *G, uint16_t *dh1, float *loss, void *stream);
int launch_mlp_adam(float *M, float *m1, float *m2, float *G, uint16_t *W, int F, float lr, int step, void *stream);

// Batched execution.  finalize = 0: rebuild the queues only (call start).
int batch_launch_decide(const BatchCtx &b, int finalize);
int batch_launch_speed(const BatchCtx &b, int order);
// stage 0: residual of u into A (used to time tile shapes); 1..3: SSP-RK3 stages
int batch_launch_stage(const BatchCtx &b, int order, int stage, int grid);
int batch_launch_limit(const BatchCtx &b, int order, int slot);

}  // namespace dg
