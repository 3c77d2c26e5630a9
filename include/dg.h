/*
 * dg.h -- C-ABI of libdg.so: the explicit SSP-RK3 Runge-Kutta discontinuous
 * Galerkin step on uniform Cartesian meshes with the compact subcell WENO
 * (CSWENO) limiter of Kochi & Ramakrishna, "A compact subcell WENO limiting
 * strategy using immediate neighbors for Runge-Kutta Discontinuous Galerkin
 * Methods" (arXiv 1904.11147), running in HIP kernels on gfx950 (MI355X).
 *
 * Conventions shared by every call
 * --------------------------------
 * Problem (Section 2, first equation and its 2D form in Section 4):
 *   u_t + f(u)_x (+ g(u)_y) = 0 on [x0,x1] (x [y0,y1]) split into nx (x ny)
 *   equal cells; Burgers f = g = u^2/2, or the ideal-gas Euler equations with
 *   conserved variables (rho, rho u, E) in 1D and (rho, rho u, rho v, E) in 2D
 *   (Examples 7 and 3 of Section 4).
 * Basis (Section 2, orthonormalised Legendre polynomials and the affine map):
 *   psi_n(r) = sqrt((2n+1)/2) P_n(r) on r in [-1,1]; in 2D the tensor product
 *   psi_m(r) psi_n(s) with m, n <= N (Q^N).  A cell mean is U_0 / sqrt(2) in 1D
 *   and U_00 / 2 in 2D.
 * State layout ("state" arguments): FP64, structure of arrays
 *   state[v][q][j][i], i fastest, v < nv (1 Burgers, 3 Euler 1D, 4 Euler 2D),
 *   q = m + (N+1) n < (N+1)^dim (m the x-degree), j < ny (1 in 1D), i < nx.
 * Pointers: every pointer named "state", "out", "point_values", "flags",
 *   "margin" or "flags_override" is DEVICE memory on the device that was
 *   current when dg_init ran; every other pointer is HOST memory.  The caller
 *   owns all memory, including the workspace given to dg_init; the library
 *   allocates no device memory.  Device buffers are only borrowed for the
 *   duration of a call.
 * Streams: every call enqueues its work on the stream given to dg_init and
 *   returns after that stream has finished it, unless stated otherwise.
 * Errors: every call returns DG_OK (0) or a negative DG_ERR_* code; no
 *   exception crosses the ABI.  DG_ERR_NONPHYSICAL means a kernel met a
 *   non-positive density or pressure, or a NaN, since the previous check; the
 *   results of that call are still written.  dg_strerror names a code.
 * Threads: a dg_problem may be used by one host thread at a time; distinct
 *   problems are independent.
 */
#ifndef DG_H
#define DG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DG_ABI_VERSION 3

enum {
  DG_OK = 0,
  DG_ERR_INVALID_ARG = -1,
  DG_ERR_UNSUPPORTED = -2,
  DG_ERR_WORKSPACE = -3,
  DG_ERR_HIP = -4,
  DG_ERR_NONPHYSICAL = -5
};

enum { DG_EQ_BURGERS = 0, DG_EQ_EULER = 1 };
enum { DG_BC_PERIODIC = 0, DG_BC_TRANSMISSIVE = 1, DG_BC_REFLECTIVE = 2, DG_BC_INFLOW = 3 };
enum { DG_LIM_NONE = 0, DG_LIM_CSWENO = 1, DG_LIM_CSWENO_CHAR = 2 };
enum { DG_IND_TVB = 0, DG_IND_ALL = 1, DG_IND_LEARNED = 2, DG_IND_KXRCF = 3 };
enum { DG_NEGW_SPLIT = 0, DG_NEGW_RAW = 1 };

typedef struct dg_config {
  int32_t abi_version; /* DG_ABI_VERSION */
  int32_t dim;         /* 1 or 2 */
  int32_t equation;    /* DG_EQ_BURGERS or DG_EQ_EULER */
  int32_t order;       /* N in 1..3: P^N in 1D, Q^N in 2D */
  int32_t nx, ny;      /* cells per direction; ny must be 1 in 1D */
  int32_t bc[4];       /* west, east, south, north; the ghost cell beyond a side is:
                          DG_BC_PERIODIC   the periodic image (sides come in pairs);
                          DG_BC_TRANSMISSIVE the even reflection of the adjacent cell
                                           (odd modes in the normal direction change sign);
                          DG_BC_REFLECTIVE that reflection with the normal momentum
                                           negated as well (a wall; Euler only);
                          DG_BC_INFLOW     the constant state bc_state[side][0].
                          A corner ghost beyond an inflow west/east side is that
                          inflow state; otherwise the south/north rule applies to the
                          column the west/east rule mapped to. */
  int32_t limiter;     /* DG_LIM_NONE, DG_LIM_CSWENO (componentwise), or DG_LIM_CSWENO_CHAR
                          (Euler: each WENO sweep in the local characteristic fields of its
                          direction, eigenvectors of the flux Jacobian at the troubled
                          cell's mean state, end of Sec. 3; Burgers: as DG_LIM_CSWENO) */
  int32_t indicator;   /* DG_IND_TVB (TVB-modified minmod), DG_IND_ALL (every cell),
                          DG_IND_LEARNED (2D Euler with periodic or transmissive sides
                          only: the MLP of dg_set_learned with the TVB decision in its
                          uncertain band), or DG_IND_KXRCF (the
                          inflow-jump indicator of Krivodonova et al. that Sec. 3, step 1
                          cites: |integral of the trace jump over the inflow boundary| /
                          (h^((N+1)/2) |inflow boundary| max_q |u|) > 1, h the cell's
                          circumscribed radius, inflow from the cell-average velocity,
                          variables u or density and energy; margin min(|I-1|, |v_x|, |v_y|)) */
  int32_t negw_mode;   /* P3 points with a negative linear weight: DG_NEGW_SPLIT
                          (positive/negative split, theta = 3) or DG_NEGW_RAW */
  int32_t positivity;  /* 1: positivity-preserving scaling of Zhang and Shu after the
                          limiter of every stage (Example 11 adds it; Euler only): per
                          cell the density, then the whole state, scaled towards the
                          cell mean by the largest factors that keep density and
                          pressure >= eps = min(1e-10, mean density, mean pressure) at
                          the tensor points of the face Gauss rule with the 3-point
                          (Q1: 2-point) Gauss-Lobatto rule in both orders and at the
                          volume Gauss points.  0: off */
  double gamma;        /* ratio of specific heats (Euler), 1.4 */
  double x0, x1, y0, y1;
  double tvb_M;        /* TVB constant M; threshold M h^2 per direction */
  double weno_eps;     /* epsilon of the nonlinear weights (Section 3, Step 5), 1e-6 */
  double cfl;          /* CFL number used when dg_step is given dt <= 0 */
  /* A south or north side may switch kind along x: kind bc[s] for ghost
   * cells whose centre x < bc_switch[s][0] + bc_switch[s][1] t, kind
   * bc_beyond[s] (DG_BC_TRANSMISSIVE, DG_BC_REFLECTIVE or DG_BC_INFLOW with
   * state bc_state[s][1]) from there on; -1: no switch.  West and east sides
   * never switch (-1).  t is the time the data of a stage stand for: dg_step
   * takes t^n for the first residual, t^n + dt for the limiter after the
   * first stage and the second residual, t^n + dt/2 for the limiter after the
   * second stage and the third residual, t^n + dt after the last stage;
   * dg_residual and dg_limit take the time of dg_set_time (0 initially). */
  int32_t bc_beyond[4];
  int32_t pad;              /* must be 0 */
  double bc_switch[4][2];
  double bc_state[4][2][4]; /* conserved inflow states [side][before, beyond][variable] */
  /* Non-uniform tensor-product meshes (the accuracy tests of Sec. 4 move every
   * node of the uniform mesh): host arrays of nx+1 (x_nodes) and ny+1
   * (y_nodes, 2D) strictly increasing node coordinates, or NULL for the
   * uniform mesh on [x0,x1] x [y0,y1].  Cells stay rectangles; each column
   * and row has its own width, TVB threshold M h^2, KXRCF radius and CSWENO
   * tables (Steps 2-4 on the stencil of the cell and its two neighbours; a
   * ghost column has the width of the cell it images); the CFL rule becomes
   * dt = cfl / (max S_x/h_x + max S_y/h_y) over the cells.  Read by
   * dg_workspace_bytes and dg_init only (dg_init copies what it needs into the
   * workspace).  Not with DG_IND_LEARNED, switching sides or batches. */
  const double *x_nodes;
  const double *y_nodes;
} dg_config;

typedef struct dg_problem dg_problem;

/* Size in bytes of the device workspace dg_init needs for this configuration
 * (two stage buffers of the state's size plus indicator arrays).  Returns
 * DG_ERR_INVALID_ARG / DG_ERR_UNSUPPORTED for a bad configuration.  Host only:
 * touches no device. */
int dg_workspace_bytes(const dg_config *cfg, size_t *bytes);

/* Creates a problem.  cfg is copied.  workspace: device memory of at least
 * dg_workspace_bytes bytes, 256-byte aligned, kept by the caller until
 * dg_destroy.  stream: a hipStream_t (NULL = the null stream).  Uploads the
 * method's coefficient tables (Section 3, Steps 1-3) to the current device. */
int dg_init(const dg_config *cfg, void *workspace, size_t workspace_bytes, void *stream, dg_problem **out);

/* Frees the host-side handle (and any captured graph).  NULL is accepted. */
int dg_destroy(dg_problem *p);

/* Nodes and weights of the rule dg_project integrates with, on the reference
 * cell [-1,1]: two panels [-1,0] and [0,1], each with an (N+2)-point Gauss
 * rule, so a jump at a cell face or centre is integrated piecewise.  r_nodes
 * and weights receive *nq values each (at most 10); either may be NULL. */
int dg_proj_nodes(const dg_problem *p, double *r_nodes, double *weights, int32_t *nq);

/* L2 projection of initial data onto the modal basis (Section 2, modal form),
 * for the cell rows j0 .. j0+nrows-1 (1D: j0 = 0, nrows = 1).
 * point_values: device, [nv][nq][nq][nrows][nx] in 2D ([nv][nq][1][nx] in 1D),
 * the value at the physical point of reference coordinates
 * (r_nodes[a], r_nodes[b]) of cell (i, j0+jr) stored at [v][b][a][jr][i].
 * Writes those rows of state.  Does not limit: call dg_limit afterwards. */
int dg_project(dg_problem *p, const double *point_values, int32_t j0, int32_t nrows, double *state);

/* Spatial operator L(U) of the semi-discrete scheme (Section 2, eq.
 * weakFormScheme, modal form with a local Lax-Friedrichs flux evaluated
 * pointwise at the (N+1)-point Gauss nodes of each face, and the volume term
 * by (N+1)^dim-point Gauss quadrature).  out has the layout of state and must
 * not alias it. */
int dg_residual(dg_problem *p, const double *state, double *out);

/* One application of the limiter (Section 3): troubled-cell indicator, then
 * CSWENO reconstruction of every troubled cell (compact subcell stencil,
 * WENO values at the Step-1 points, projection of moments 1..N; the cell mean
 * is kept bit for bit).  Jacobi semantics: every decision and reconstruction
 * reads state as it was on entry.  In place on state.
 * flags (device uint8[ny][nx]) and margin (device double[ny][nx]) receive the
 * indicator and, for DG_IND_TVB, a lower bound on the change of the tested
 * quantities that would alter the decision; either may be NULL.
 * flags_override (device uint8[ny][nx], non-zero = troubled) replaces the
 * indicator when not NULL.  n_troubled (host) receives the count; may be NULL.
 * With positivity on, every cell is then scaled as dg_config.positivity says. */
int dg_limit(dg_problem *p, double *state, uint8_t *flags, double *margin, const uint8_t *flags_override,
             int32_t *n_troubled);

/* Time step of the CFL rule on cell means: 1D dt = cfl h / S, 2D
 * dt = cfl / (S_x/h_x + S_y/h_y), S the largest spectral radius of the mean
 * states (|u| for Burgers, |u_n| + c for Euler).  *dt is a host double;
 * infinity when S = 0. */
int dg_cfl_dt(dg_problem *p, const double *state, double *dt);

/* Advances state from *t towards t_end by third-order TVD Runge-Kutta steps
 * with the limiter after every stage (Section 3, last paragraph), at most
 * max_steps steps.  dt > 0: fixed step; dt <= 0: the CFL rule of dg_cfl_dt,
 * recomputed each step on the device.  The last step is clipped so that t
 * lands on t_end.  *t (host) is updated; *steps_taken (host, may be NULL)
 * receives the number of steps.  A step in which a kernel meets a
 * non-physical state is the last one: the call returns DG_ERR_NONPHYSICAL
 * with *t and *steps_taken after that step (also returned, without ending
 * the run early, for a non-physical state met before the call and not yet
 * read by dg_status).  The step sequence is captured once in a HIP graph per
 * state pointer and replayed. */
int dg_step(dg_problem *p, double *state, double *t, double t_end, double dt, int32_t max_steps,
            int32_t *steps_taken);

/* dg_limit for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): no
 * problem handle and no workspace.  The configuration is passed directly
 * (validated as by dg_workspace_bytes; uniform meshes, any indicator but
 * DG_IND_LEARNED), t is the time of time-dependent boundary data, stream a
 * hipStream_t (NULL = null stream); state, flags, margin, flags_override and
 * n_troubled mean what they mean for dg_limit.  The limiter's scratch (scalar
 * words, troubled-cell list, Jacobi side buffer) lives in a static device
 * array of 64 MiB that each device holds from the first call until the
 * process ends: a problem needs 256 + 4 cells (rounded up to 256 bytes) +
 * the state's bytes, e.g. up to 229,000 cells of 2D Euler Q2; larger ones
 * return DG_ERR_WORKSPACE.  The call allocates nothing, enqueues its work on
 * stream and returns after the stream has finished it.  Every call on a
 * device shares that device's array: calls that overlap on one device
 * (several host threads or streams) race and must be serialised by the
 * caller. */
int dg_limit_noalloc(const dg_config *cfg, double *state, uint8_t *flags, double *margin,
                     const uint8_t *flags_override, double t, int32_t *n_troubled, void *stream);

/* Time at which dg_residual and dg_limit evaluate time-dependent boundary
 * data (switching sides).  Enqueued on the problem's stream. */
int dg_set_time(dg_problem *p, double t);

/* Status word of the problem: DG_OK or DG_ERR_NONPHYSICAL (sticky until read;
 * reading clears it).  Synchronises the stream. */
int dg_status(dg_problem *p);

/* Static string naming a status code. */
const char *dg_strerror(int code);

/* Profiling (measurement only; not part of the method).  While enabled,
 * dg_step launches its kernels one by one instead of replaying the graph and
 * brackets every launch with HIP events on the problem's stream.
 * dg_profile_read returns, per kind, the summed event time in milliseconds
 * (ms[DG_PROF_KINDS], host) and the number of launches (launches[], host),
 * plus the number of troubled cells flagged by all limiter passes
 * (*troubled, host; may be NULL); reset != 0 clears the accumulators. */
enum { DG_PROF_STAGE1 = 0, DG_PROF_STAGE23 = 1, DG_PROF_LIMITER = 2, DG_PROF_DT = 3, DG_PROF_KINDS = 4 };
int dg_profile_enable(dg_problem *p, int enable);
int dg_profile_read(dg_problem *p, double *ms, int64_t *launches, int64_t *troubled, int reset);

/* ---- Learned troubled-cell indicator (not in the paper: its indicator is
 * KXRCF, Sec. 3; the workload asks for a small MLP trained on the flags and
 * limited/unlimited pairs of the plain method, with TVB as the fallback).
 *
 * Features of a cell, per conserved variable v, in the order of the cells
 * C, W, E, S, N and their (N+1)^2 modes: the five mode-0 entries minus the
 * centre's mode 0, all divided by max(max |entry|, M hx^2).  F = 5 (N+1)^2 nv
 * features (180 for 2D Euler Q2), zero-padded to KP = 16 ceil(F/16) in the
 * bf16 layout.  Network: 64 ReLU units, 64 ReLU units, one sigmoid output;
 * bf16 weights, fp32 biases and accumulation (BF16 MFMA).
 * Master parameters (fp32, host or device order W1 [64][F] | W2 [64][64] |
 * w3 [64] | b1 [64] | b2 [64] | b3); bf16 weight buffer W1 [64][KP] |
 * W2 [64][64] | W2^T [64][64] | w3 [64].  All buffers below are DEVICE memory
 * owned by the caller; "stream" is a hipStream_t. */

/* Tile-shape autotuner of one problem (2D; 1D problems return rows 0 and
 * change nothing): times the stage kernel (a residual evaluation of state
 * into the workspace; state is not changed) for each tile height (rows
 * marched per wavefront: 4, 8, 16, 32, 64) and keeps the fastest for later
 * calls; rows and ms (host, may be NULL) receive the choice and its time.
 * Results do not depend on the tile height. */
int dg_autotune(dg_problem *p, const double *state, int32_t *rows, float *ms);

/* Sizes for F features: padded width, master and bf16 element counts (host). */
int dg_mlp_layout(int32_t features, int32_t *padded, int64_t *n_master, int64_t *n_bf16);

/* Features of every cell of a 2D state: f32 [cells][F] and/or bf16 [cells][KP]
 * (either may be NULL). */
int dg_mlp_features(dg_problem *p, const double *state, float *f32, uint16_t *bf16);

/* prob[i] = sigmoid(network(x[i])) for n rows of x (bf16 [n][KP]). */
int dg_mlp_forward(const uint16_t *x, int32_t n, int32_t features, const uint16_t *w_bf16, const float *master,
                   float *prob, void *stream);

/* Adds to grad (fp32, master order, zeroed by the caller or by dg_mlp_adam)
 * the gradient of the mean weighted binary cross-entropy
 * (1/n) sum_i wgt[i] (log(1 + e^z_i) - y[i] z_i) and adds that loss to *loss
 * (device float).  dh1: bf16 scratch of n*64 elements. */
int dg_mlp_gradient(const uint16_t *x, const float *y, const float *wgt, int32_t n, int32_t features,
                    const uint16_t *w_bf16, const float *master, float *grad, uint16_t *dh1, float *loss,
                    void *stream);

/* One Adam step (beta 0.9, 0.999, eps 1e-8, bias-corrected with step >= 1) on
 * master from grad, then grad := 0 and the bf16 buffer refreshed; step = 0
 * only refreshes the bf16 buffer from master. */
int dg_mlp_adam(float *master, float *adam_m, float *adam_v, float *grad, uint16_t *w_bf16, int32_t features,
                float lr, int32_t step, void *stream);

/* Weights for DG_IND_LEARNED on this problem (kept as pointers until
 * replaced): a cell is troubled when p > band_hi, untroubled when p < band_lo,
 * and decided by TVB in between.  prob (device float [cells], may be NULL)
 * receives p at every indicator pass. */
int dg_set_learned(dg_problem *p, const uint16_t *w_bf16, const float *master, double band_lo, double band_hi,
                   float *prob);

/* ------------------------------------------------------------------------
 * Batched execution: n independent 2D Euler problems (any sizes, orders
 * 1..3, boundary conditions and CFL numbers; one limiter and one indicator
 * mode for all) advanced together, each with its own CFL time step
 * (Section 2's scheme and Section 3's limiter applied to every instance as
 * dg_step applies them to one).  A step of the batch is one SSP-RK3 step of
 * every instance still short of its end time: per RK stage one kernel per
 * order whose wavefronts take the (instance, tile) work items of a
 * device-side queue (a grid of the order's full tile count; wavefronts past
 * the live count exit at once), followed by the limiter pass of that stage;
 * finished instances leave the queue on the device.  The step is one
 * captured graph; with the learned indicator each order's chain is its own
 * branch of it.  Each instance's results are identical, bit for bit, to
 * dg_step on the same problem.
 *
 * Memory: the caller owns one device buffer `states` holding every
 * instance's state (layout of dg_project, FP64) at element offsets
 * offsets[i] (host int64 array, multiples of 32), and one workspace of
 * dg_batch_workspace_bytes (256-byte aligned) that holds per-instance stage
 * buffers (two state volumes each), scalars, descriptors, the work queues and
 * the troubled-cell lists.  The library allocates no device memory; it
 * creates a capture stream (with the learned indicator also one stream and
 * event per order), released by dg_batch_destroy.
 * ------------------------------------------------------------------------ */
typedef struct dg_batch dg_batch;

/* Workspace bytes for the n configurations cfgs[0..n-1] (n <= 4096; all 2D
 * Euler; equal limiter, indicator and positivity flag; periodic or
 * transmissive sides on uniform meshes (else DG_ERR_UNSUPPORTED); at most
 * 2^31 - 1 cells in total, and at most 2^27 / (N+1)^2 cells per instance,
 * e.g. 14.9 million at N = 2, as the batched stage kernel addresses an
 * instance's state with 32-bit byte offsets (else DG_ERR_UNSUPPORTED)). */
int dg_batch_workspace_bytes(const dg_config *cfgs, int32_t n, size_t *bytes);

/* Creates the batch on the current device and the given stream (NULL =
 * default stream).  The workspace must stay valid until dg_batch_destroy. */
int dg_batch_init(const dg_config *cfgs, int32_t n, void *workspace, size_t workspace_bytes, void *stream,
                  dg_batch **out);

int dg_batch_destroy(dg_batch *b);

/* Times the stage kernel of every order present for each candidate tile
 * height (rows marched per work item: 4, 8, 16, 32, 64; a tile is 30 columns
 * wide) on the given states (a residual evaluation into the workspace; the
 * states are not changed) and keeps the fastest per order for later
 * dg_batch_step calls.  rows, tiles (host int32 [4], indexed by order: the
 * tile height and the resulting tile count) and ms (host float [4], the best
 * stage time) receive the choices and may be NULL.  Default height: 16. */
int dg_batch_autotune(dg_batch *b, double *states, const int64_t *offsets, int32_t *rows, int32_t *tiles,
                      float *ms);

/* Sets the tile height of one order by hand. */
int dg_batch_set_tiles(dg_batch *b, int32_t order, int32_t rows);

/* Advances every instance i from t[i] (host double [n], updated) towards
 * t_end[i] (host double [n]) by CFL time steps, at most max_steps steps each;
 * steps (host int32 [n], may be NULL) receives the steps taken and status
 * (host int32 [n], may be NULL) DG_OK or DG_ERR_NONPHYSICAL per instance (an
 * instance that meets a non-physical state stops there).  troubled (host,
 * may be NULL) receives the number of troubled cells flagged over all
 * instances and limiter passes of the call.  Returns DG_ERR_NONPHYSICAL if
 * any instance stopped that way. */
int dg_batch_step(dg_batch *b, double *states, const int64_t *offsets, double *t, const double *t_end,
                  int32_t max_steps, int32_t *steps, int32_t *status, int64_t *troubled);

/* Weights of the learned indicator for the instances of one order (required
 * for each order present when the batch uses DG_IND_LEARNED); as
 * dg_set_learned.  prob (device float, may be NULL; kept as a pointer like
 * the weights) receives, at every indicator pass, p of cell c of instance i
 * of this order at prob[offsets[i] + c] (offsets as given to dg_batch_step,
 * so a buffer with as many elements as the states buffer serves every
 * order). */
int dg_batch_set_learned(dg_batch *b, int32_t order, const uint16_t *w_bf16, const float *master, double band_lo,
                         double band_hi, float *prob);

#ifdef __cplusplus
}
#endif
#endif /* DG_H */
