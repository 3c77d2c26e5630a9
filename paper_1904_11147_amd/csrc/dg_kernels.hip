// HIP kernels for gfx950 of the RKDG step with the compact subcell WENO
// limiter (Kochi & Ramakrishna, arXiv 1904.11147).
//
// Data layout: state[v][q][j][i], FP64, i fastest.  One thread owns one cell;
// consecutive lanes of a 64-wide wavefront own consecutive cells of a row, so
// every per-mode load and store is a coalesced 512-byte access.
//
// Kernels:
//   k_stage      Section 2 residual (volume term by sum-factorised Gauss
//                quadrature, local Lax-Friedrichs flux at the face Gauss points,
//                lift) fused with the SSP-RK3 stage combination; stage 3 also
//                reduces the largest spectral radius of the new cell means for
//                the next time step.
//   k_indicator  TVB-modified minmod on face-midpoint traces (Cockburn-Shu),
//                with decision margins and a wave-aggregated compaction of the
//                troubled cells into a list.
//   k_csweno     Section 3 Steps 1-6 for one (troubled cell, variable): subcell
//                means of the immediate neighbours, WENO values at the Step-1
//                points (2D: x-sweeps on every y-interval, then y-sweeps),
//                projection of moments >= 1 into a side buffer (Jacobi).
//   k_scatter    copies the side buffer back into the state for listed cells.
//   k_speed, k_dt_finalize, k_reset, k_project: time step and set-up.
#include <hip/hip_runtime.h>

#include <algorithm>

#include <cmath>
#include <mutex>
#include <type_traits>

#include "dg_internal.h"

// The file is compiled kKernelParts times, with DG_PART = 0 .. kKernelParts-1,
// so that the kernel families build in parallel: parts 0, 4, 5 the stage
// kernels of orders 1, 2, 3 (part 0 also the time-step and set-up kernels),
// part 1 the limiter, part 2 the network, part 3 the batched launches.  Each
// part is its own code object with its own copy of the coefficient tables.
#ifndef DG_PART
#error "compile with -DDG_PART=0..5"
#endif
#define DG_CAT2(a, b) a##b
#define DG_CAT(a, b) DG_CAT2(a, b)

#if DG_PART == 1
// Scratch of dg_limit_noalloc (each device holds its own copy until the
// process ends).  Host code never passes this name to a kernel: it takes the
// device address from hipGetSymbolAddress (static_scratch below).
static __device__ __align__(256) unsigned char scratch[dg::kStaticScratchBytes];
#endif

namespace dg {

namespace {
__constant__ OrderTables c_tab[kMaxN + 1];  // this part's copy (internal linkage)
}  // namespace

int DG_CAT(upload_tables_part, DG_PART)(const OrderTables *tabs) {
  hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(c_tab), tabs, sizeof(OrderTables) * (kMaxN + 1), 0,
                                   hipMemcpyHostToDevice);
  return e == hipSuccess ? DG_OK : DG_ERR_HIP;
}

namespace {

constexpr int kBlock = 256;

template <int N> constexpr int num_points() { return N == 1 ? 2 : 4; }

// ---------------------------------------------------------------------------
// Physics: Burgers (f = g = u^2/2) and ideal-gas Euler in 1D / 2D.
// ---------------------------------------------------------------------------
template <int EQ, int DIM> struct Phys;

template <int DIM> struct Phys<0, DIM> {
  static constexpr int NV = 1;
  template <int DIR>
  __device__ static inline void flux(const double *u, double *f, double, bool &) { f[0] = 0.5 * u[0] * u[0]; }
  template <int DIR>
  __device__ static inline double speed(const double *u, double, bool &) { return fabs(u[0]); }
};

template <> struct Phys<1, 1> {
  static constexpr int NV = 3;
  template <int DIR>
  __device__ static inline void flux(const double *u, double *f, double g, bool &bad) {
    double rho = u[0], vx = u[1] / rho;
    double p = (g - 1.0) * (u[2] - 0.5 * rho * vx * vx);
    bad |= !(rho > 0.0 && p > 0.0);
    f[0] = u[1];
    f[1] = u[1] * vx + p;
    f[2] = (u[2] + p) * vx;
  }
  template <int DIR>
  __device__ static inline double speed(const double *u, double g, bool &bad) {
    double rho = u[0], vx = u[1] / rho;
    double p = (g - 1.0) * (u[2] - 0.5 * rho * vx * vx);
    bad |= !(rho > 0.0 && p > 0.0);
    return fabs(vx) + sqrt(g * p / rho);
  }
};

template <> struct Phys<1, 2> {
  static constexpr int NV = 4;
  template <int DIR>
  __device__ static inline void flux(const double *u, double *f, double g, bool &bad) {
    double rho = u[0], ir = 1.0 / rho, vx = u[1] * ir, vy = u[2] * ir;
    double p = (g - 1.0) * (u[3] - 0.5 * rho * (vx * vx + vy * vy));
    bad |= !(rho > 0.0 && p > 0.0);
    double vn = DIR == 0 ? vx : vy;
    f[0] = DIR == 0 ? u[1] : u[2];
    f[1] = u[1] * vn + (DIR == 0 ? p : 0.0);
    f[2] = u[2] * vn + (DIR == 1 ? p : 0.0);
    f[3] = (u[3] + p) * vn;
  }
  template <int DIR>
  __device__ static inline double speed(const double *u, double g, bool &bad) {
    double rho = u[0], ir = 1.0 / rho, vx = u[1] * ir, vy = u[2] * ir;
    double p = (g - 1.0) * (u[3] - 0.5 * rho * (vx * vx + vy * vy));
    bad |= !(rho > 0.0 && p > 0.0);
    return fabs(DIR == 0 ? vx : vy) + sqrt(g * p * ir);
  }
};

// Local Lax-Friedrichs flux between the left/lower trace a and the
// right/upper trace b, dissipation from the two traces at this point.
template <int EQ, int DIM, int DIR>
__device__ inline void llf(const double *a, const double *b, double *F, double g, bool &bad) {
  using P = Phys<EQ, DIM>;
  double fa[P::NV], fb[P::NV];
  P::template flux<DIR>(a, fa, g, bad);
  P::template flux<DIR>(b, fb, g, bad);
  double al = fmax(P::template speed<DIR>(a, g, bad), P::template speed<DIR>(b, g, bad));
#pragma unroll
  for (int v = 0; v < P::NV; ++v) F[v] = 0.5 * (fa[v] + fb[v]) - 0.5 * al * (b[v] - a[v]);
}

// ---------------------------------------------------------------------------
// Cell access with boundary conditions.  Beyond a side the ghost cell is the
// periodic image, the even reflection of the adjacent cell (odd modes in the
// normal direction change sign), that reflection with the normal momentum
// negated (wall), or a constant inflow state.  The west/east rule is applied
// first; a corner beyond an inflow west/east side is that inflow state.
// South/north sides may switch kind at x = a + b t (t: DevScalars::tb).
// ---------------------------------------------------------------------------
struct CellIdx {
  long idx;      // a cell inside the mesh (also for inflow ghosts, so loads stay in bounds)
  bool fx, fy;   // odd modes in x / y change sign
  uint8_t neg;   // bit v: variable v changes sign
  int8_t gs;     // >= 0: inflow ghost with lowest mode Geometry::bst[gs]
};

// BND = false: only periodic and transmissive sides can occur (the launch
// checked), which keeps the hot stage kernel free of the other cases.
template <bool BND = true>
__device__ inline CellIdx map_cell(const Geometry &g, int i, int j) {
  CellIdx c;
  c.fx = c.fy = false;
  c.neg = 0;
  c.gs = -1;
  if constexpr (!BND) {
    if (i < 0) {
      if (g.bc[0] == DG_BC_PERIODIC) i += g.nx; else { i = 0; c.fx = true; }
    } else if (i >= g.nx) {
      if (g.bc[1] == DG_BC_PERIODIC) i -= g.nx; else { i = g.nx - 1; c.fx = true; }
    }
    if (j < 0) {
      if (g.bc[2] == DG_BC_PERIODIC) j += g.ny; else { j = 0; c.fy = true; }
    } else if (j >= g.ny) {
      if (g.bc[3] == DG_BC_PERIODIC) j -= g.ny; else { j = g.ny - 1; c.fy = true; }
    }
    c.idx = (long)j * g.nx + i;
    return c;
  }
  if (i < 0 || i >= g.nx) {
    const int s = i < 0 ? 0 : 1, k = g.bc[s];
    if (k == DG_BC_PERIODIC) {
      i += s ? -g.nx : g.nx;
    } else {
      i = s ? g.nx - 1 : 0;
      c.fx = true;
      if (k == DG_BC_REFLECTIVE) c.neg = 2;
      if (k == DG_BC_INFLOW) c.gs = (int8_t)(2 * s);
    }
  }
  if (j < 0 || j >= g.ny) {
    const int s = j < 0 ? 2 : 3;
    int k = g.bc[s], part = 0;
    if (g.bcb[s] >= 0) {  // rounded like a plain product and sum, without contraction
      const double xc = __dadd_rn(g.x0, __dmul_rn(i + 0.5, g.hx));
      if (!(xc < __dadd_rn(g.bsw[s][0], __dmul_rn(g.bsw[s][1], *g.tb)))) {
        part = 1;
        k = g.bcb[s];
      }
    }
    if (k == DG_BC_PERIODIC) {
      j += s == 3 ? -g.ny : g.ny;
    } else {
      j = s == 3 ? g.ny - 1 : 0;
      if (c.gs < 0) {
        c.fy = true;
        if (k == DG_BC_REFLECTIVE) c.neg |= 4;
        if (k == DG_BC_INFLOW) c.gs = (int8_t)(2 * s + part);
      }
    }
  }
  c.idx = (long)j * g.nx + i;
  return c;
}

// Mode q (= m + NP n) of variable v of the cell or ghost c.
template <int NP, int NM, int DIM>
__device__ __forceinline__ double cell_mode(const double *__restrict__ u, long plane, const Geometry &g,
                                            const CellIdx &c, int v, int q) {
  const int m = q % NP, n = q / NP;
  double s = u[(long)(v * NM + q) * plane + c.idx];
  const bool flip = ((c.fx && (m & 1)) != (DIM == 2 && c.fy && (n & 1))) != (((c.neg >> v) & 1) != 0);
  s = flip ? -s : s;
  if (c.gs >= 0) s = q == 0 ? g.bst[c.gs][v] : 0.0;
  return s;
}

template <int NP, int NM, int NV, int DIM>
__device__ inline void load_cell(const double *__restrict__ u, long plane, const Geometry &g, const CellIdx &c,
                                 double C[NV][NM]) {
#pragma unroll
  for (int v = 0; v < NV; ++v)
#pragma unroll
    for (int q = 0; q < NM; ++q) C[v][q] = cell_mode<NP, NM, DIM>(u, plane, g, c, v, q);
}

// Per-column / per-row geometry of non-uniform meshes (uniform: the scalars).
__device__ inline double rh_x(const Geometry &g, int i) {
  return g.rhxa ? g.rhxa[min(max(i, 0), g.nx - 1)] : g.rhx;
}
__device__ inline double rh_y(const Geometry &g, int j) {
  return g.rhya ? g.rhya[min(max(j, 0), g.ny - 1)] : g.rhy;
}
// A spectral radius over the cell width on non-uniform meshes, whose CFL rule
// then takes unit widths; unchanged on uniform meshes.
__device__ inline double per_wx(const Geometry &g, int i, double s) { return g.hxa ? s / g.hxa[i] : s; }
__device__ inline double per_wy(const Geometry &g, int j, double s) { return g.hya ? s / g.hya[j] : s; }

// ---------------------------------------------------------------------------
// Residual + SSP-RK3 stage.  STAGE 0: out = L(u).  1: u + dt L.  2: 3/4 un +
// 1/4 (u + dt L).  3: 1/3 un + 2/3 (u + dt L).
// ---------------------------------------------------------------------------
// Last SSP-RK3 stage, 1/3 un + 2/3 v: products with the rounded constants
// (within an ulp of the quotients, and no division sequence per value).
__device__ __forceinline__ double rk3_last(double un, double v) {
  constexpr double third = 1.0 / 3.0, two_thirds = 2.0 / 3.0;
  return un * third + v * two_thirds;
}

struct StageArgs {
  const double *u;
  const double *un;
  double *out;
  DevScalars *sc;
  Geometry geo;
  int want_speed;
};

template <int N, int EQ, int STAGE>
__global__ __launch_bounds__(kBlock) void k_stage_1d(StageArgs a) {
  constexpr int NP = N + 1, NV = Phys<EQ, 1>::NV;
  using P = Phys<EQ, 1>;
  const OrderTables &T = c_tab[N];
  const Geometry &g = a.geo;
  if (STAGE != 0 && a.sc->done) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const long plane = g.nx;
  bool bad = false;
  double spd = 0.0;
  if (i < g.nx) {
    const double rx = rh_x(g, i);
    double C[NV][NP], Nb[NV][NP], L[NV][NP];
    load_cell<NP, NP, NV, 1>(a.u, plane, g, map_cell(g, i, 0), C);
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int n = 0; n < NP; ++n) L[v][n] = 0.0;
    // volume term
#pragma unroll
    for (int q = 0; q < NP; ++q) {
      double uq[NV], f[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        double s = 0.0;
#pragma unroll
        for (int n = 0; n < NP; ++n) s += C[v][n] * T.bq[n][q];
        uq[v] = s;
      }
      P::template flux<0>(uq, f, g.gamma, bad);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        double fw = rx * T.wq[q] * f[v];
#pragma unroll
        for (int n = 0; n < NP; ++n) L[v][n] += fw * T.dbq[n][q];
      }
    }
    // faces
    double a_[NV], b_[NV], F[NV];
    load_cell<NP, NP, NV, 1>(a.u, plane, g, map_cell(g, i + 1, 0), Nb);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      double s0 = 0.0, s1 = 0.0;
#pragma unroll
      for (int n = 0; n < NP; ++n) {
        s0 += C[v][n] * T.bp[n];
        s1 += Nb[v][n] * T.bm[n];
      }
      a_[v] = s0;
      b_[v] = s1;
    }
    llf<EQ, 1, 0>(a_, b_, F, g.gamma, bad);
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int n = 0; n < NP; ++n) L[v][n] -= rx * F[v] * T.bp[n];
    load_cell<NP, NP, NV, 1>(a.u, plane, g, map_cell(g, i - 1, 0), Nb);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      double s0 = 0.0, s1 = 0.0;
#pragma unroll
      for (int n = 0; n < NP; ++n) {
        s0 += Nb[v][n] * T.bp[n];
        s1 += C[v][n] * T.bm[n];
      }
      a_[v] = s0;
      b_[v] = s1;
    }
    llf<EQ, 1, 0>(a_, b_, F, g.gamma, bad);
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int n = 0; n < NP; ++n) L[v][n] += rx * F[v] * T.bm[n];

    const double dt = STAGE == 0 ? 0.0 : a.sc->dt;
    double mean[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int n = 0; n < NP; ++n) {
        long k = (long)(v * NP + n) * plane + i;
        double r;
        if (STAGE == 0) r = L[v][n];
        else if (STAGE == 1) r = C[v][n] + dt * L[v][n];
        else if (STAGE == 2) r = 0.75 * a.un[k] + 0.25 * (C[v][n] + dt * L[v][n]);
        else r = rk3_last(a.un[k], C[v][n] + dt * L[v][n]);
        a.out[k] = r;
        if (n == 0) mean[v] = r * T.b0[0];
      }
    if (STAGE == 3 && a.want_speed) spd = per_wx(g, i, P::template speed<0>(mean, g.gamma, bad));
  }
  if (bad) atomicOr(&a.sc->status, 1);
  if (STAGE == 3 && a.want_speed) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) spd = fmax(spd, __shfl_xor(spd, o));
    if (__lane_id() == 0) atomicMax(&a.sc->smax[0], (unsigned long long)__double_as_longlong(spd));
  }
}

template <int N, int EQ, int STAGE>
__global__ __launch_bounds__(kBlock) void k_stage_2d(StageArgs a) {
  constexpr int NP = N + 1, NM = NP * NP, NV = Phys<EQ, 2>::NV;
  using P = Phys<EQ, 2>;
  const OrderTables &T = c_tab[N];
  const Geometry &g = a.geo;
  if (STAGE != 0 && a.sc->done) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  const long plane = (long)g.nx * g.ny;
  bool bad = false;
  double spx = 0.0, spy = 0.0;
  if (i < g.nx && j < g.ny) {
    double C[NV][NM], L[NV][NM];
    load_cell<NP, NM, NV, 2>(a.u, plane, g, map_cell(g, i, j), C);
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int q = 0; q < NM; ++q) L[v][q] = 0.0;

    // volume term, sum-factorised: row sums t[v][n][qx] first
    double t[NV][NP][NP];
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int n = 0; n < NP; ++n)
#pragma unroll
        for (int qx = 0; qx < NP; ++qx) {
          double s = 0.0;
#pragma unroll
          for (int m = 0; m < NP; ++m) s += C[v][m + NP * n] * T.bq[m][qx];
          t[v][n][qx] = s;
        }
#pragma unroll
    for (int qy = 0; qy < NP; ++qy) {
      double Fx[NV][NP], Gy[NV][NP];
#pragma unroll
      for (int qx = 0; qx < NP; ++qx) {
        double uq[NV], f[NV], gg[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          double s = 0.0;
#pragma unroll
          for (int n = 0; n < NP; ++n) s += t[v][n][qx] * T.bq[n][qy];
          uq[v] = s;
        }
        P::template flux<0>(uq, f, g.gamma, bad);
        P::template flux<1>(uq, gg, g.gamma, bad);
        double w = T.wq[qx] * T.wq[qy];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          Fx[v][qx] = w * rh_x(g, i) * f[v];
          Gy[v][qx] = w * rh_y(g, j) * gg[v];
        }
      }
#pragma unroll
      for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int m = 0; m < NP; ++m) {
          double sa = 0.0, sb = 0.0;
#pragma unroll
          for (int qx = 0; qx < NP; ++qx) {
            sa += Fx[v][qx] * T.dbq[m][qx];
            sb += Gy[v][qx] * T.bq[m][qx];
          }
#pragma unroll
          for (int n = 0; n < NP; ++n) L[v][m + NP * n] += sa * T.bq[n][qy] + sb * T.dbq[n][qy];
        }
    }

    // faces: x-direction (east, west), then y-direction (north, south)
#pragma unroll
    for (int face = 0; face < 4; ++face) {
      const int di = face == 0 ? 1 : (face == 1 ? -1 : 0);
      const int dj = face == 2 ? 1 : (face == 3 ? -1 : 0);
      double Nb[NV][NM];
      load_cell<NP, NM, NV, 2>(a.u, plane, g, map_cell(g, i + di, j + dj), Nb);
      // own and neighbour 1D trace coefficients along the face: c[v][k]
      double co[NV][NP], cn[NV][NP];
      const double *bo = (face == 0 || face == 2) ? T.bp : T.bm;  // own side
      const double *bn = (face == 0 || face == 2) ? T.bm : T.bp;  // neighbour side
#pragma unroll
      for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int k = 0; k < NP; ++k) {
          double so = 0.0, sn = 0.0;
#pragma unroll
          for (int l = 0; l < NP; ++l) {
            int q = face < 2 ? (l + NP * k) : (k + NP * l);  // x-face: sum over m; y-face: sum over n
            so += C[v][q] * bo[l];
            sn += Nb[v][q] * bn[l];
          }
          co[v][k] = so;
          cn[v][k] = sn;
        }
      double phi[NV][NP];
#pragma unroll
      for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int k = 0; k < NP; ++k) phi[v][k] = 0.0;
#pragma unroll
      for (int e = 0; e < NP; ++e) {
        double uo[NV], un_[NV], F[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          double so = 0.0, sn = 0.0;
#pragma unroll
          for (int k = 0; k < NP; ++k) {
            so += co[v][k] * T.bq[k][e];
            sn += cn[v][k] * T.bq[k][e];
          }
          uo[v] = so;
          un_[v] = sn;
        }
        if (face == 0) llf<EQ, 2, 0>(uo, un_, F, g.gamma, bad);
        else if (face == 1) llf<EQ, 2, 0>(un_, uo, F, g.gamma, bad);
        else if (face == 2) llf<EQ, 2, 1>(uo, un_, F, g.gamma, bad);
        else llf<EQ, 2, 1>(un_, uo, F, g.gamma, bad);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          double fw = T.wq[e] * F[v];
#pragma unroll
          for (int k = 0; k < NP; ++k) phi[v][k] += fw * T.bq[k][e];
        }
      }
      // lift: east/north subtract F psi(+1), west/south add F psi(-1)
      const double sc = face < 2 ? rh_x(g, i) : rh_y(g, j);
#pragma unroll
      for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int l = 0; l < NP; ++l)
#pragma unroll
          for (int k = 0; k < NP; ++k) {
            int q = face < 2 ? (l + NP * k) : (k + NP * l);
            double contrib = sc * bo[l] * phi[v][k];
            if (face == 0 || face == 2) L[v][q] -= contrib;
            else L[v][q] += contrib;
          }
    }

    const double dt = STAGE == 0 ? 0.0 : a.sc->dt;
    const long cell = (long)j * g.nx + i;
    double mean[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int q = 0; q < NM; ++q) {
        long k = (long)(v * NM + q) * plane + cell;
        double r;
        if (STAGE == 0) r = L[v][q];
        else if (STAGE == 1) r = C[v][q] + dt * L[v][q];
        else if (STAGE == 2) r = 0.75 * a.un[k] + 0.25 * (C[v][q] + dt * L[v][q]);
        else r = rk3_last(a.un[k], C[v][q] + dt * L[v][q]);
        a.out[k] = r;
        if (q == 0) mean[v] = r * (T.b0[0] * T.b0[0]);
      }
    if (STAGE == 3 && a.want_speed) {
      spx = per_wx(g, i, P::template speed<0>(mean, g.gamma, bad));
      spy = per_wy(g, j, P::template speed<1>(mean, g.gamma, bad));
    }
  }
  if (bad) atomicOr(&a.sc->status, 1);
  if (STAGE == 3 && a.want_speed) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      spx = fmax(spx, __shfl_xor(spx, o));
      spy = fmax(spy, __shfl_xor(spy, o));
    }
    if (__lane_id() == 0) {
      atomicMax(&a.sc->smax[0], (unsigned long long)__double_as_longlong(spx));
      atomicMax(&a.sc->smax[1], (unsigned long long)__double_as_longlong(spy));
    }
  }
}

// ---------------------------------------------------------------------------
// Residual + SSP-RK3 stage in 2D, marching form.  One 64-lane wavefront owns a
// strip of 62 columns (lanes 1..62; lanes 0 and 63 are the strip's x-halo)
// and walks up a chunk of rows.  Each lane loads its cell's modes once per
// row (coalesced, 512 B per mode plane); the east trace of the western
// neighbour and the western face flux of the eastern neighbour move between
// lanes by shuffles, so every x-face flux is computed once; the flux on the
// south face of a row is the north-face flux of the row below, carried in
// registers, so rows are not re-read except one halo row per chunk.
// ---------------------------------------------------------------------------
constexpr int kStrip = 62;

// Trace of the cell polynomial on the face x = +-1 (SIDE = +1 / -1) at the N+1
// edge Gauss points s_e:  sum_n (sum_m U_mn psi_m(+-1)) psi_n(s_e).
template <int N, int NV, int SIDE>
__device__ inline void trace_x(const OrderTables &T, const double (&U)[NV][(N + 1) * (N + 1)], double (&out)[NV][N + 1]) {
  constexpr int NP = N + 1;
  const double *b = SIDE > 0 ? T.bp : T.bm;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    double c[NP];
#pragma unroll
    for (int n = 0; n < NP; ++n) {
      double s = 0.0;
#pragma unroll
      for (int m = 0; m < NP; ++m) s += U[v][m + NP * n] * b[m];
      c[n] = s;
    }
#pragma unroll
    for (int e = 0; e < NP; ++e) {
      double s = 0.0;
#pragma unroll
      for (int n = 0; n < NP; ++n) s += c[n] * T.bq[n][e];
      out[v][e] = s;
    }
  }
}

// Trace on the face y = +-1 at the edge Gauss points r_e.
template <int N, int NV, int SIDE>
__device__ inline void trace_y(const OrderTables &T, const double (&U)[NV][(N + 1) * (N + 1)], double (&out)[NV][N + 1]) {
  constexpr int NP = N + 1;
  const double *b = SIDE > 0 ? T.bp : T.bm;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    double c[NP];
#pragma unroll
    for (int m = 0; m < NP; ++m) {
      double s = 0.0;
#pragma unroll
      for (int n = 0; n < NP; ++n) s += U[v][m + NP * n] * b[n];
      c[m] = s;
    }
#pragma unroll
    for (int e = 0; e < NP; ++e) {
      double s = 0.0;
#pragma unroll
      for (int m = 0; m < NP; ++m) s += c[m] * T.bq[m][e];
      out[v][e] = s;
    }
  }
}

// LLF fluxes at the N+1 points of a face from the lower/left traces a and the
// upper/right traces b.
template <int EQ, int N, int NV, int DIR>
__device__ inline void face_flux(const double (&a)[NV][N + 1], const double (&b)[NV][N + 1], double (&F)[NV][N + 1],
                                 double g, bool &bad) {
#pragma unroll
  for (int e = 0; e < N + 1; ++e) {
    double ua[NV], ub[NV], f[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      ua[v] = a[v][e];
      ub[v] = b[v][e];
    }
    llf<EQ, 2, DIR>(ua, ub, f, g, bad);
#pragma unroll
    for (int v = 0; v < NV; ++v) F[v][e] = f[v];
  }
}

// Lift of a face flux into the residual: L -= sgn * scale * psi_normal(+-1) *
// sum_e w_e F_e psi_tangential(e)  (DIR 0: x-face, normal degree m).
template <int N, int NV, int DIR, int SIDE>
__device__ inline void lift(const OrderTables &T, const double (&F)[NV][N + 1], double scale,
                            double (&L)[NV][(N + 1) * (N + 1)]) {
  constexpr int NP = N + 1;
  const double *b = SIDE > 0 ? T.bp : T.bm;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    double phi[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      double s = 0.0;
#pragma unroll
      for (int e = 0; e < NP; ++e) s += T.wq[e] * F[v][e] * T.bq[k][e];
      phi[k] = s * scale;
    }
#pragma unroll
    for (int l = 0; l < NP; ++l)
#pragma unroll
      for (int k = 0; k < NP; ++k) {
        const int q = DIR == 0 ? (l + NP * k) : (k + NP * l);
        if (SIDE > 0) L[v][q] -= b[l] * phi[k];
        else L[v][q] += b[l] * phi[k];
      }
  }
}

// South trace (y = -1) of the cell of row j+1 at the edge points, streamed one
// variable at a time so that no full cell state stays live.
template <int N, int NV>
__device__ inline void south_trace_streamed(const OrderTables &T, const double *__restrict__ u, long plane,
                                            const Geometry &g, const CellIdx &c, double (&ts)[NV][N + 1]) {
  constexpr int NP = N + 1, NM = NP * NP;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    double m9[NM];
#pragma unroll
    for (int q = 0; q < NM; ++q) m9[q] = cell_mode<NP, NM, 2>(u, plane, g, c, v, q);
#pragma unroll
    for (int e = 0; e < NP; ++e) {
      double acc = 0.0;
#pragma unroll
      for (int m = 0; m < NP; ++m) {
        double cm = 0.0;
#pragma unroll
        for (int n = 0; n < NP; ++n) cm += m9[m + NP * n] * T.bm[n];
        acc += cm * T.bq[m][e];
      }
      ts[v][e] = acc;
    }
  }
}

template <int N, int EQ, int STAGE>
__global__ __launch_bounds__(64) void k_stage_2d_march(StageArgs a, int rows_per_block) {
  constexpr int NP = N + 1, NM = NP * NP, NV = Phys<EQ, 2>::NV;
  using P = Phys<EQ, 2>;
  const OrderTables &T = c_tab[N];
  const Geometry &g = a.geo;
  if (STAGE != 0 && a.sc->done) return;
  const int lane = threadIdx.x;
  int col = blockIdx.x * kStrip + lane - 1;
  if (col > g.nx) col = g.nx;  // lanes past the east ghost column duplicate it
  const bool owner = lane >= 1 && lane <= kStrip && col < g.nx;
  const int j0 = blockIdx.y * rows_per_block;
  const int j1 = min(j0 + rows_per_block, g.ny);
  const long plane = (long)g.nx * g.ny;
  const double dt = STAGE == 0 ? 0.0 : a.sc->dt;
  bool bad = false;
  double spx = 0.0, spy = 0.0;
  const double rx = rh_x(g, col);

  // flux on the south face of row j0 from the halo row below
  double FS[NV][NP];
  {
    double Ub[NV][NM], tn[NV][NP], ts[NV][NP];
    load_cell<NP, NM, NV, 2>(a.u, plane, g, map_cell(g, col, j0 - 1), Ub);
    trace_y<N, NV, +1>(T, Ub, tn);
    south_trace_streamed<N, NV>(T, a.u, plane, g, map_cell(g, col, j0), ts);
    face_flux<EQ, N, NV, 1>(tn, ts, FS, g.gamma, bad);
  }
  for (int j = j0; j < j1; ++j) {
    // Re-derive the table reference every row: the empty asm makes the
    // pointer opaque, so table values are re-read from the scalar cache
    // instead of being hoisted out of the loop into registers.
    const OrderTables *Tp = &c_tab[N];
    asm volatile("" : "+s"(Tp));
    const OrderTables &T = *Tp;
    const CellIdx me = map_cell(g, col, j);
    double L[NV][NM];
    double tn[NV][NP];
    {
      double U[NV][NM];
      load_cell<NP, NM, NV, 2>(a.u, plane, g, me, U);
#pragma unroll
      for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int q = 0; q < NM; ++q) L[v][q] = 0.0;
      // x-faces first: this lane's west face uses the east trace of lane-1
      {
        double te[NV][NP], tl[NV][NP];
        trace_x<N, NV, +1>(T, U, te);
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
          for (int e = 0; e < NP; ++e) tl[v][e] = __shfl_up(te[v][e], 1);
        double tw[NV][NP], FW[NV][NP];
        trace_x<N, NV, -1>(T, U, tw);
        face_flux<EQ, N, NV, 0>(tl, tw, FW, g.gamma, bad);
        lift<N, NV, 0, -1>(T, FW, rx, L);
        double FE[NV][NP];
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
          for (int e = 0; e < NP; ++e) FE[v][e] = __shfl_down(FW[v][e], 1);
        lift<N, NV, 0, +1>(T, FE, rx, L);
      }
      __builtin_amdgcn_sched_barrier(0);
      // volume term, one quadrature row qy at a time (not unrolled: keeps
      // one row of point values and fluxes live)
#pragma unroll 1
      for (int qy = 0; qy < NP; ++qy) {
        double Fx[NV][NP], Gy[NV][NP];
#pragma unroll
        for (int qx = 0; qx < NP; ++qx) {
          double uq[NV], f[NV], gg[NV];
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            double s = 0.0;
#pragma unroll
            for (int n = 0; n < NP; ++n) {
              double t = 0.0;
#pragma unroll
              for (int m = 0; m < NP; ++m) t += U[v][m + NP * n] * T.bq[m][qx];
              s += t * T.bq[n][qy];
            }
            uq[v] = s;
          }
          P::template flux<0>(uq, f, g.gamma, bad);
          P::template flux<1>(uq, gg, g.gamma, bad);
          const double w = T.wq[qx] * T.wq[qy];
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            Fx[v][qx] = w * rx * f[v];
            Gy[v][qx] = w * rh_y(g, j) * gg[v];
          }
        }
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
          for (int m = 0; m < NP; ++m) {
            double sa = 0.0, sb = 0.0;
#pragma unroll
            for (int qx = 0; qx < NP; ++qx) {
              sa += Fx[v][qx] * T.dbq[m][qx];
              sb += Gy[v][qx] * T.bq[m][qx];
            }
#pragma unroll
            for (int n = 0; n < NP; ++n) L[v][m + NP * n] += sa * T.bq[n][qy] + sb * T.dbq[n][qy];
          }
      }
      trace_y<N, NV, +1>(T, U, tn);
    }
    __builtin_amdgcn_sched_barrier(0);
    // y-faces: south flux carried from the row below; north flux from this
    // row's north trace and the next row's south trace
    {
      double ts[NV][NP], FN[NV][NP];
      south_trace_streamed<N, NV>(T, a.u, plane, g, map_cell(g, col, j + 1), ts);
      face_flux<EQ, N, NV, 1>(tn, ts, FN, g.gamma, bad);
      lift<N, NV, 1, -1>(T, FS, rh_y(g, j), L);
      lift<N, NV, 1, +1>(T, FN, rh_y(g, j), L);
#pragma unroll
      for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int e = 0; e < NP; ++e) FS[v][e] = FN[v][e];
    }
    __builtin_amdgcn_sched_barrier(0);
    if (owner) {
      const long cell = (long)j * g.nx + col;
      double mean[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int q = 0; q < NM; ++q) {
          const long k = (long)(v * NM + q) * plane + cell;
          double r;
          if (STAGE == 0) r = L[v][q];
          else if (STAGE == 1) r = a.u[k] + dt * L[v][q];
          else if (STAGE == 2) r = 0.75 * a.un[k] + 0.25 * (a.u[k] + dt * L[v][q]);
          else r = rk3_last(a.un[k], a.u[k] + dt * L[v][q]);
          a.out[k] = r;
          if (q == 0) mean[v] = r * (T.b0[0] * T.b0[0]);
        }
      }
      if (STAGE == 3 && a.want_speed) {
        spx = fmax(spx, per_wx(g, col, P::template speed<0>(mean, g.gamma, bad)));
        spy = fmax(spy, per_wy(g, j, P::template speed<1>(mean, g.gamma, bad)));
      }
    }
  }
  if (bad) atomicOr(&a.sc->status, 1);
  if (STAGE == 3 && a.want_speed) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      spx = fmax(spx, __shfl_xor(spx, o));
      spy = fmax(spy, __shfl_xor(spy, o));
    }
    if (lane == 0) {
      atomicMax(&a.sc->smax[0], (unsigned long long)__double_as_longlong(spx));
      atomicMax(&a.sc->smax[1], (unsigned long long)__double_as_longlong(spy));
    }
  }
}

// ---------------------------------------------------------------------------
// 2D Euler stage kernel with two lanes per cell.  Lane 2s+h of a wavefront
// owns conserved variables 2h and 2h+1 of the cell in slot s, i.e.
// (rho, rho u) for h = 0 and (rho v, E) for h = 1, and the matching modes of
// the residual, which halves the per-lane state.  Every linear step (traces,
// quadrature values, contractions, lifts) works on the lane's own two
// variables; at each flux point the two lanes swap their point values
// (shfl_xor 1), both form the primitive variables, and each evaluates only
// its own flux components.  The wavefront marches up a chunk of rows over a
// strip of 30 columns (slots 1..30; slots 0 and 31 are the x-halo).
// ---------------------------------------------------------------------------

struct EulerPrim {
  double ir, vx, vy, p;
};

// 1/x from the hardware estimate refined by two Newton steps (about 1 ulp for
// normal x; the density is checked separately).
__device__ inline double fast_rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// sqrt(a) for a > 0 from the reciprocal square-root estimate and Newton
// (Goldschmidt) refinement, about 1 ulp; a <= 0 or NaN gives NaN.
__device__ inline double fast_sqrt(double a) {
  double y = __builtin_amdgcn_rsq(a);
  double gq = a * y, h = 0.5 * y;
  double r = fma(-gq, h, 0.5);
  gq = fma(gq, r, gq);
  h = fma(h, r, h);
  r = fma(-gq, h, 0.5);
  gq = fma(gq, r, gq);
  h = fma(h, r, h);
  const double d = fma(-gq, gq, a);
  gq = fma(d, h, gq);
  return a > 0.0 ? gq : (a == 0.0 ? 0.0 : __builtin_nan(""));
}

template <int DIR>
__device__ inline double euler_speed(const EulerPrim &s, double rho, double g) {
  return fabs(DIR == 0 ? s.vx : s.vy) + fast_sqrt(g * s.p * s.ir);
}

// Lanes of one cell: VPL = 2 variables per lane (lanes 2s, 2s+1 hold
// variables {0,1}, {2,3}; Q1, Q2) or VPL = 1 (lanes 4s+v hold variable v;
// Q3, whose modes would not fit two variables per lane).  `part` is the
// lane's index within its cell.

// Lane P_{l} of each aligned group of four lanes, for lane l of the group, by
// a DPP quad permutation: a register move with no LDS round trip (the cell's
// lanes are one such group or half of one).  Every lane of the wavefront is
// active where it is called.
template <int P0, int P1, int P2, int P3>
__device__ __forceinline__ double quad_perm(double v) {
  constexpr int ctrl = P0 | (P1 << 2) | (P2 << 4) | (P3 << 6);
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)b, ctrl, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), ctrl, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// The full state (rho, mx, my, E) at a point from the cell's lanes, each
// component broadcast from the lane that holds it (no selects).
template <int VPL>
__device__ inline void gather_state(const double (&a)[VPL], int part, double (&w)[4]) {
  (void)part;
  if constexpr (VPL == 2) {  // variables 0, 1 in the even lane of the pair, 2, 3 in the odd one
    w[0] = quad_perm<0, 0, 2, 2>(a[0]);
    w[1] = quad_perm<0, 0, 2, 2>(a[1]);
    w[2] = quad_perm<1, 1, 3, 3>(a[0]);
    w[3] = quad_perm<1, 1, 3, 3>(a[1]);
  } else {  // variable v in lane v of the four
    w[0] = quad_perm<0, 0, 0, 0>(a[0]);
    w[1] = quad_perm<1, 1, 1, 1>(a[0]);
    w[2] = quad_perm<2, 2, 2, 2>(a[0]);
    w[3] = quad_perm<3, 3, 3, 3>(a[0]);
  }
}

__device__ inline EulerPrim prim_of(const double (&w)[4], double g, bool &bad) {
  EulerPrim s;
  s.ir = fast_rcp(w[0]);
  s.vx = w[1] * s.ir;
  s.vy = w[2] * s.ir;
  s.p = (g - 1.0) * (w[3] - 0.5 * w[0] * (s.vx * s.vx + s.vy * s.vy));
  bad |= !(w[0] > 0.0 && s.p > 0.0);
  return s;
}

// Flux component of variable var (the lane's own value a) in direction DIR:
// f = w vx + (0, p, 0, p vx), g = w vy + (0, 0, p, p vy).
template <int DIR>
__device__ inline double flux_comp(const EulerPrim &s, double a, int var) {
  const double vn = DIR == 0 ? s.vx : s.vy;
  if (DIR == 0) return (var & 1) ? a * vn + (var == 3 ? s.p * vn : s.p) : a * vn;
  return a * vn + (var == 2 ? s.p : (var == 3 ? s.p * vn : 0.0));
}

// LLF flux at one face point for the lane's variables: left/lower trace l,
// right/upper trace r (the lane's own components).
template <int DIR, int VPL>
__device__ inline void llf_lane(const double (&l)[VPL], const double (&r)[VPL], int part, double g,
                                double (&F)[VPL], bool &bad) {
  double wl[4], wr[4];
  gather_state<VPL>(l, part, wl);
  gather_state<VPL>(r, part, wr);
  const EulerPrim sl = prim_of(wl, g, bad);
  const EulerPrim sr = prim_of(wr, g, bad);
  const double al = fmax(euler_speed<DIR>(sl, 0.0, g), euler_speed<DIR>(sr, 0.0, g));
#pragma unroll
  for (int k = 0; k < VPL; ++k) {
    const double fl = flux_comp<DIR>(sl, l[k], VPL * part + k), fr = flux_comp<DIR>(sr, r[k], VPL * part + k);
    F[k] = 0.5 * (fl + fr) - 0.5 * al * (r[k] - l[k]);
  }
}

__host__ __device__ constexpr int euler_vpl(int N) { return N == 3 ? 1 : 2; }
// columns owned by one wavefront's tile (the other two cell slots are the x-halo)
__host__ __device__ constexpr int euler_strip(int N) { return 64 * euler_vpl(N) / 4 - 2; }

// One tile: columns [bx*STRIP, +STRIP) of rows [by*rows, +rows), marched
// row by row by one wavefront.  `row` is the wavefront's LDS staging area of
// VPL (N+1)^2 64 doubles (the current row's modes of each lane's variables,
// [k*NM+q][lane]).
// OFF32: every byte offset into the state arrays is below 2^32 (the host
// checks 32 (N+1)^2 nx ny <= 2^32).  Each access is then the array's address
// (a scalar) plus a 32-bit per-lane offset, and the plane offsets are 32-bit
// scalars: far fewer scalar registers than one 64-bit address per plane.
__host__ __device__ constexpr bool euler_off32_fits(int N, long long cells) {
  return 32ll * (N + 1) * (N + 1) * cells <= (1ll << 32);
}

template <int N, int STAGE, bool BND, bool OFF32>
__device__ __forceinline__ void euler_tile(const StageArgs &a, int bx, int by, int rows_per_block,
                                           double *__restrict__ row) {
  constexpr int NP = N + 1, NM = NP * NP, VPL = euler_vpl(N), LPC = 4 / VPL, STRIP = euler_strip(N);
  const OrderTables &T = c_tab[N];
  const Geometry &g = a.geo;
  if (STAGE != 0 && a.sc->done) return;
  const int lane = threadIdx.x, slot = lane / LPC, part = lane % LPC;
  int col = bx * STRIP + slot - 1;
  if (col > g.nx) col = g.nx;
  const bool owner = slot >= 1 && slot <= STRIP && col < g.nx;
  const int j0 = by * rows_per_block;
  // 2 / width of the lane's column (per column on non-uniform meshes)
  const double rhx = BND ? rh_x(g, col) : g.rhx;
  const int j1 = min(j0 + rows_per_block, g.ny);
  const long plane = (long)g.nx * g.ny;
  const double dt = STAGE == 0 ? 0.0 : a.sc->dt;
  const int v0 = VPL * part;  // first owned variable
  bool bad = false;
  double spx = 0.0, spy = 0.0;

  // address in arr of mode q of the lane's variable k (variable v0 + k) of
  // the cell at index idx
  const unsigned plane8 = (unsigned)plane * 8u, lane8 = (unsigned)(v0 * NM) * plane8;
  auto at = [&](auto *arr, int k, int q, unsigned idx) {
    if constexpr (OFF32) {
      using B = std::conditional_t<std::is_const<std::remove_pointer_t<decltype(arr)>>::value, const char, char>;
      return reinterpret_cast<decltype(arr)>(reinterpret_cast<B *>(arr) +
                                             (lane8 + idx * 8u + (unsigned)(k * NM + q) * plane8));
    } else {
      return arr + (size_t)(v0 * NM) * plane + ((size_t)(k * NM + q) * plane + idx);
    }
  };
  auto load2 = [&](const CellIdx &c, double (&U)[VPL][NM]) {
    const unsigned idx = (unsigned)c.idx;
    const unsigned long long sx = c.fx ? 0x8000000000000000ull : 0ull, sy = c.fy ? 0x8000000000000000ull : 0ull;
#pragma unroll
    for (int k = 0; k < VPL; ++k)
#pragma unroll
      for (int q = 0; q < NM; ++q) {
        const int m = q % NP, n = q / NP;
        double s = *at(a.u, k, q, idx);
        if ((m & 1) || (n & 1)) {
          const unsigned long long msk = ((m & 1) ? sx : 0ull) ^ ((n & 1) ? sy : 0ull);
          s = __longlong_as_double(__double_as_longlong(s) ^ (long long)msk);
        }
        U[k][q] = s;
      }
    if (BND && (c.neg != 0 || c.gs >= 0)) {  // wall and inflow ghosts: boundary cells only
#pragma unroll
      for (int k = 0; k < VPL; ++k) {
        const int v = v0 + k;
#pragma unroll
        for (int q = 0; q < NM; ++q) {
          double s = ((c.neg >> v) & 1) ? -U[k][q] : U[k][q];
          if (c.gs >= 0) s = q == 0 ? g.bst[c.gs][v] : 0.0;
          U[k][q] = s;
        }
      }
    }
  };
  auto rd = [&](int k, int q) -> double { return row[(k * NM + q) * 64 + lane]; };
  // trace of the two own variables on a face (dirf 0: x-face, 1: y-face)
  // from modes given by a getter
  auto trace2 = [&](auto get, const double *b, int dirf, double (&out)[VPL][NP]) {
#pragma unroll
    for (int k = 0; k < VPL; ++k) {
      double c[NP];
#pragma unroll
      for (int t = 0; t < NP; ++t) {
        double s = 0.0;
#pragma unroll
        for (int l = 0; l < NP; ++l) s += get(k, dirf == 0 ? (l + NP * t) : (t + NP * l)) * b[l];
        c[t] = s;
      }
#pragma unroll
      for (int e = 0; e < NP; ++e) {
        double s = 0.0;
#pragma unroll
        for (int t = 0; t < NP; ++t) s += c[t] * T.bq[t][e];
        out[k][e] = s;
      }
    }
  };
  auto lift2 = [&](const double (&F)[VPL][NP], const double *b, int dirf, int side, double scale, double (&L)[VPL][NM]) {
#pragma unroll
    for (int k = 0; k < VPL; ++k) {
      double phi[NP];
#pragma unroll
      for (int t = 0; t < NP; ++t) {
        double s = 0.0;
#pragma unroll
        for (int e = 0; e < NP; ++e) s += T.wq[e] * F[k][e] * T.bq[t][e];
        phi[t] = s * scale;
      }
#pragma unroll
      for (int l = 0; l < NP; ++l)
#pragma unroll
        for (int t = 0; t < NP; ++t) {
          const int q = dirf == 0 ? (l + NP * t) : (t + NP * l);
          if (side > 0) L[k][q] -= b[l] * phi[t];
          else L[k][q] += b[l] * phi[t];
        }
    }
  };

  // south-face flux of row j0 from the halo row below; row j0 into LDS
  double FS[VPL][NP];
  {
    double P[VPL][NM], tn[VPL][NP], ts[VPL][NP];
    load2(map_cell<BND>(g, col, j0 - 1), P);
    trace2([&](int k, int q) { return P[k][q]; }, T.bp, 1, tn);
    load2(map_cell<BND>(g, col, j0), P);
    trace2([&](int k, int q) { return P[k][q]; }, T.bm, 1, ts);
#pragma unroll
    for (int e = 0; e < NP; ++e) {
      double l[VPL], r[VPL], F[VPL];
#pragma unroll
      for (int k = 0; k < VPL; ++k) {
        l[k] = tn[k][e];
        r[k] = ts[k][e];
      }
      llf_lane<1, VPL>(l, r, part, g.gamma, F, bad);
#pragma unroll
      for (int k = 0; k < VPL; ++k) FS[k][e] = F[k];
    }
#pragma unroll
    for (int k = 0; k < VPL; ++k)
#pragma unroll
      for (int q = 0; q < NM; ++q) row[(k * NM + q) * 64 + lane] = P[k][q];
  }
  for (int j = j0; j < j1; ++j) {
    const double rhy = BND ? rh_y(g, j) : g.rhy;
    // next row in flight while this row is computed
    double P[VPL][NM];
    load2(map_cell<BND>(g, col, j + 1), P);
    const long cellj = (long)j * g.nx + col;
    double L[VPL][NM];
#pragma unroll
    for (int k = 0; k < VPL; ++k)
#pragma unroll
      for (int q = 0; q < NM; ++q) L[k][q] = 0.0;
    // x-faces: west face from slot-1's east trace; east flux from slot+1
    {
      double te[VPL][NP], tw[VPL][NP], FW[VPL][NP], FE[VPL][NP];
      trace2(rd, T.bp, 0, te);
      trace2(rd, T.bm, 0, tw);
#pragma unroll
      for (int e = 0; e < NP; ++e) {
        double l[VPL], r[VPL], F[VPL];
#pragma unroll
        for (int k = 0; k < VPL; ++k) {
          l[k] = __shfl_up(te[k][e], LPC);
          r[k] = tw[k][e];
        }
        llf_lane<0, VPL>(l, r, part, g.gamma, F, bad);
#pragma unroll
        for (int k = 0; k < VPL; ++k) FW[k][e] = F[k];
      }
#pragma unroll
      for (int k = 0; k < VPL; ++k)
#pragma unroll
        for (int e = 0; e < NP; ++e) FE[k][e] = __shfl_down(FW[k][e], LPC);
      lift2(FW, T.bm, 0, -1, rhx, L);
      lift2(FE, T.bp, 0, +1, rhx, L);
    }
    // volume term
#pragma unroll 1
    for (int qy = 0; qy < NP; ++qy) {
      double Fx[VPL][NP], Gy[VPL][NP];
#pragma unroll
      for (int qx = 0; qx < NP; ++qx) {
        double uq[VPL];
#pragma unroll
        for (int k = 0; k < VPL; ++k) {
          double s = 0.0;
#pragma unroll
          for (int n = 0; n < NP; ++n) {
            double t = 0.0;
#pragma unroll
            for (int m = 0; m < NP; ++m) t += rd(k, m + NP * n) * T.bq[m][qx];
            s += t * T.bq[n][qy];
          }
          uq[k] = s;
        }
        double wst[4];
        gather_state<VPL>(uq, part, wst);
        const EulerPrim st = prim_of(wst, g.gamma, bad);
        const double w = T.wq[qx] * T.wq[qy];
#pragma unroll
        for (int k = 0; k < VPL; ++k) {
          Fx[k][qx] = w * rhx * flux_comp<0>(st, uq[k], v0 + k);
          Gy[k][qx] = w * rhy * flux_comp<1>(st, uq[k], v0 + k);
        }
      }
#pragma unroll
      for (int k = 0; k < VPL; ++k)
#pragma unroll
        for (int m = 0; m < NP; ++m) {
          double sa = 0.0, sb = 0.0;
#pragma unroll
          for (int qx = 0; qx < NP; ++qx) {
            sa += Fx[k][qx] * T.dbq[m][qx];
            sb += Gy[k][qx] * T.bq[m][qx];
          }
#pragma unroll
          for (int n = 0; n < NP; ++n) L[k][m + NP * n] += sa * T.bq[n][qy] + sb * T.dbq[n][qy];
        }
    }
    // this row's u^n, in flight during the y-face work (Q3: loaded after it,
    // as its registers are needed there)
    double Un[VPL][NM];
    auto load_un = [&]() {
      __builtin_amdgcn_sched_barrier(0);
      const unsigned idx = (unsigned)(owner ? cellj : 0);
#pragma unroll
      for (int k = 0; k < VPL; ++k)
#pragma unroll
        for (int q = 0; q < NM; ++q) Un[k][q] = *at(a.un, k, q, idx);
    };
    if (STAGE >= 2 && N <= 2) load_un();
    // y-faces: carried south flux, north flux from the next row's south trace
    {
      double tn[VPL][NP], ts[VPL][NP], FN[VPL][NP];
      trace2(rd, T.bp, 1, tn);
      trace2([&](int k, int q) { return P[k][q]; }, T.bm, 1, ts);
#pragma unroll
      for (int e = 0; e < NP; ++e) {
        double l[VPL], r[VPL], F[VPL];
#pragma unroll
        for (int k = 0; k < VPL; ++k) {
          l[k] = tn[k][e];
          r[k] = ts[k][e];
        }
        llf_lane<1, VPL>(l, r, part, g.gamma, F, bad);
#pragma unroll
        for (int k = 0; k < VPL; ++k) FN[k][e] = F[k];
      }
      lift2(FS, T.bm, 1, -1, rhy, L);
      lift2(FN, T.bp, 1, +1, rhy, L);
#pragma unroll
      for (int k = 0; k < VPL; ++k)
#pragma unroll
        for (int e = 0; e < NP; ++e) FS[k][e] = FN[k][e];
    }
    if (STAGE >= 2 && N > 2) load_un();
    // RK stage combination (u^(s) of this row from LDS)
    double mm[VPL];
    {
#pragma unroll
      for (int k = 0; k < VPL; ++k)
#pragma unroll
        for (int q = 0; q < NM; ++q) {

          double r = 0.0;
          if (owner) {
            const double uo = rd(k, q);
            if (STAGE == 0) r = L[k][q];
            else if (STAGE == 1) r = uo + dt * L[k][q];
            else if (STAGE == 2) r = 0.75 * Un[k][q] + 0.25 * (uo + dt * L[k][q]);
            else r = rk3_last(Un[k][q], uo + dt * L[k][q]);
            *at(a.out, k, q, (unsigned)cellj) = r;
          }
          if (q == 0) mm[k] = r * (T.b0[0] * T.b0[0]);
        }
    }
    if (STAGE == 3 && a.want_speed) {
      double wm[4];
      gather_state<VPL>(mm, part, wm);
      if (owner) {
        const EulerPrim s = prim_of(wm, g.gamma, bad);
        if (BND) {
          spx = fmax(spx, per_wx(g, col, euler_speed<0>(s, 0.0, g.gamma)));
          spy = fmax(spy, per_wy(g, j, euler_speed<1>(s, 0.0, g.gamma)));
        } else {
          spx = fmax(spx, euler_speed<0>(s, 0.0, g.gamma));
          spy = fmax(spy, euler_speed<1>(s, 0.0, g.gamma));
        }
      }
    }
    // the next row becomes the current one (each lane touches only its own slots)
#pragma unroll
    for (int k = 0; k < VPL; ++k)
#pragma unroll
      for (int q = 0; q < NM; ++q) row[(k * NM + q) * 64 + lane] = P[k][q];
  }
  if (bad) atomicOr(&a.sc->status, 1);
  if (STAGE == 3 && a.want_speed) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      spx = fmax(spx, __shfl_xor(spx, o));
      spy = fmax(spy, __shfl_xor(spy, o));
    }
    if (lane == 0) {
      atomicMax(&a.sc->smax[0], (unsigned long long)__double_as_longlong(spx));
      atomicMax(&a.sc->smax[1], (unsigned long long)__double_as_longlong(spy));
    }
  }
}

// Workgroups are dealt to the 8 XCDs (each with its own L2) round-robin by
// dispatch index L.  This maps L to a tile index so that every XCD receives
// one contiguous range of tiles: x-neighbouring tiles, which read the same
// halo cache lines, then run on the same L2.  A bijection on [0, total).
__device__ inline int xcd_tile(int L, int total) {
  constexpr int kXcd = 8;
  const int q = total / kXcd, r = total % kXcd, x = L % kXcd;
  return x * q + min(x, r) + L / kXcd;
}

template <int N, int STAGE, bool BND, bool OFF32>
__global__ __launch_bounds__(64, 2) void k_stage_2d_euler(StageArgs a, int rows_per_block) {
  __shared__ double row[euler_vpl(N) * (N + 1) * (N + 1) * 64];
  const int tiles_x = gridDim.x;
  const int w = xcd_tile(blockIdx.x + blockIdx.y * tiles_x, tiles_x * gridDim.y);
  euler_tile<N, STAGE, BND, OFF32>(a, w % tiles_x, w / tiles_x, rows_per_block, row);
}

// ---------------------------------------------------------------------------
// Spectral radius of cell means (first step of a dg_step call, dg_cfl_dt).
// ---------------------------------------------------------------------------
template <int N, int EQ, int DIM>
__global__ __launch_bounds__(kBlock) void k_speed(const double *__restrict__ u, DevScalars *sc, Geometry g) {
  constexpr int NP = N + 1, NM = DIM == 1 ? NP : NP * NP, NV = Phys<EQ, DIM>::NV;
  using P = Phys<EQ, DIM>;
  const OrderTables &T = c_tab[N];
  const long plane = (long)g.nx * g.ny;
  const double k0 = DIM == 1 ? T.b0[0] : T.b0[0] * T.b0[0];
  double sx = 0.0, sy = 0.0;
  bool bad = false;
  for (long cell = (long)blockIdx.x * blockDim.x + threadIdx.x; cell < plane; cell += (long)gridDim.x * blockDim.x) {
    double m[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) m[v] = u[(long)(v * NM) * plane + cell] * k0;
    sx = fmax(sx, per_wx(g, (int)(cell % g.nx), P::template speed<0>(m, g.gamma, bad)));
    if (DIM == 2) sy = fmax(sy, per_wy(g, (int)(cell / g.nx), P::template speed<1>(m, g.gamma, bad)));
  }
  if (bad) atomicOr(&sc->status, 1);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    sx = fmax(sx, __shfl_xor(sx, o));
    sy = fmax(sy, __shfl_xor(sy, o));
  }
  // one atomic per block (a maximum: the order does not matter)
  __shared__ double red[2][kBlock / 64];
  const int wave = threadIdx.x >> 6;
  if (__lane_id() == 0) {
    red[0][wave] = sx;
    red[1][wave] = sy;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int w = 1; w < kBlock / 64; ++w) {
      sx = fmax(sx, red[0][w]);
      sy = fmax(sy, red[1][w]);
    }
    atomicMax(&sc->smax[0], (unsigned long long)__double_as_longlong(sx));
    if (DIM == 2) atomicMax(&sc->smax[1], (unsigned long long)__double_as_longlong(sy));
  }
}

// One thread: time step of the CFL rule (or the fixed one), clipped at
// t_end; marks the run done; clears the per-step accumulators.
__device__ inline void decide_dt(DevScalars *sc, int dim, double cfl, double hx, double hy) {
  if (sc->done) return;
  if (sc->steps >= sc->max_steps || !(sc->t < sc->t_end)) {
    sc->done = 1;
    sc->dt = 0.0;
    return;
  }
  double dt;
  if (sc->dt_fixed > 0.0) {
    dt = sc->dt_fixed;
  } else {
    double sx = __longlong_as_double((long long)sc->smax[0]);
    double sy = __longlong_as_double((long long)sc->smax[1]);
    if (dim == 1) {
      dt = sx > 0.0 ? cfl * hx / sx : INFINITY;
    } else {
      double den = sx / hx + sy / hy;
      dt = den > 0.0 ? cfl / den : INFINITY;
    }
  }
  bool last = false;
  if (sc->t + dt >= sc->t_end) {
    dt = sc->t_end - sc->t;
    last = true;
  }
  sc->dt = dt;
  sc->tn = sc->t;
  sc->tb = sc->t;
  sc->t = last ? sc->t_end : sc->t + dt;
  sc->steps += 1;
  sc->smax[0] = 0ull;
  sc->smax[1] = 0ull;
  sc->count[0] = sc->count[1] = sc->count[2] = 0;
}

__global__ void k_dt_finalize(DevScalars *sc, int dim, double cfl, double hx, double hy) {
  if (threadIdx.x == 0) {
    if (sc->status) sc->done = 1;  // a non-physical state ends the run after the step that met it
    decide_dt(sc, dim, cfl, hx, hy);
  }
}

// Time of the boundary data: tn + frac dt during a step (frac >= 0), or the
// given value (frac < 0).  Nothing once the run is done.
__global__ void k_set_tb(DevScalars *sc, double frac, double value) {
  if (threadIdx.x != 0) return;
  if (frac < 0.0) sc->tb = value;
  else if (!sc->done) sc->tb = sc->tn + frac * sc->dt;
}

__global__ void k_reset(DevScalars *sc, int what) {
  if (threadIdx.x != 0) return;
  if (what == 0) {  // standalone limiter count
    sc->count[3] = 0;
  } else if (what == 2) {  // the learned pass's own list
    sc->count_scratch = 0;
  } else {  // speed accumulators
    sc->smax[0] = 0ull;
    sc->smax[1] = 0ull;
  }
}

// ---------------------------------------------------------------------------
// Positivity-preserving scaling of Zhang and Shu on every cell (Euler), one
// thread per cell.  Points: the face Gauss rule G (the residual's N+1 nodes)
// crossed with the Gauss-Lobatto rule S (end points, and the centre for
// N >= 2) in both orders, and the volume points G x G; 1D: S and G.  Density
// is scaled towards the mean by theta1 so that it is >= eps at every point,
// then the whole state by theta2 so that the pressure is, eps = min(1e-10,
// mean density, mean pressure).  A cell that needs neither keeps its modes
// untouched; a cell whose mean is not admissible sets the status word.
// ---------------------------------------------------------------------------
constexpr double kPosEps = 1e-10;

template <int DIM>
__device__ inline double pos_pressure(const double *w, double gam) {
  double ke = w[1] * w[1];
  if (DIM == 2) ke += w[2] * w[2];
  return (gam - 1.0) * (w[DIM + 1] - 0.5 * ke / w[0]);
}

// The t in [0,1] where the pressure along wb + t (wq - wb) reaches eps, for
// p(wb) >= eps > p(wq): the decreasing root of rho (p - eps) / (gamma - 1),
// a quadratic A t^2 + B t + C, in the form without cancellation.
template <int DIM>
__device__ inline double pos_root(const double *wb, const double *wq, double eps, double gam) {
  constexpr int E = DIM + 1;
  const double ee = eps / (gam - 1.0);
  const double dr = wq[0] - wb[0], dE = wq[E] - wb[E];
  double mm = 0.0, md = 0.0, dd = 0.0;
#pragma unroll
  for (int d = 1; d <= DIM; ++d) {
    const double dm = wq[d] - wb[d];
    mm += wb[d] * wb[d];
    md += wb[d] * dm;
    dd += dm * dm;
  }
  const double A = dE * dr - 0.5 * dd;
  const double B = wb[E] * dr + wb[0] * dE - md - ee * dr;
  const double C = wb[E] * wb[0] - 0.5 * mm - ee * wb[0];
  if (!(C > 0.0)) return 0.0;
  double D = B * B - 4.0 * A * C;
  if (D < 0.0) D = 0.0;
  const double t = B <= 0.0 ? 2.0 * C / (sqrt(D) - B) : (-B - sqrt(D)) / (2.0 * A);
  return fmin(fmax(t, 0.0), 1.0);
}

// One cell of a state with `plane` cells per mode plane; returns true when
// the cell's mean itself is not admissible (the cell is then left as it is).
template <int N, int DIM>
__device__ inline bool positivity_cell(double *__restrict__ u, long plane, long cell, const Geometry &g) {
  constexpr int NP = N + 1, NM = DIM == 1 ? NP : NP * NP, NV = DIM + 2, NL = N == 1 ? 2 : 3;
  const OrderTables &T = c_tab[N];
  const double k0 = DIM == 1 ? T.b0[0] : T.b0[0] * T.b0[0];
  // basis rows of the Gauss-Lobatto points
  auto lob = [&](int a, int n) { return a == 0 ? T.bm[n] : (a == NL - 1 ? T.bp[n] : T.b0[n]); };

  double C[NV][NM], wb[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
#pragma unroll
    for (int q = 0; q < NM; ++q) C[v][q] = u[(long)(v * NM + q) * plane + cell];
    wb[v] = C[v][0] * k0;
  }
  const double pb = pos_pressure<DIM>(wb, g.gamma);
  if (!(wb[0] > 0.0 && pb > 0.0)) return true;
  const double eps = fmin(kPosEps, fmin(wb[0], pb));
  // visit(f): f(point values of the requested variables) at every point
  auto visit = [&](auto nvars, auto f) {
    constexpr int K = decltype(nvars)::value;
    if (DIM == 1) {
      for (int a = 0; a < NL + NP; ++a) {
        double w[NV];
#pragma unroll
        for (int v = 0; v < K; ++v) {
          double acc = 0.0;
#pragma unroll
          for (int m = 0; m < NP; ++m) acc += C[v][m] * (a < NL ? lob(a, m) : T.bq[m][a - NL]);
          w[v] = acc;
        }
        f(w);
      }
    } else {
      // rows s: Gauss-Lobatto rows take the Gauss columns, Gauss rows take both
      for (int b = 0; b < NL + NP; ++b) {
        double cr[K][NP];  // partial sums over the y-degree at this row
#pragma unroll
        for (int v = 0; v < K; ++v)
#pragma unroll
          for (int m = 0; m < NP; ++m) {
            double acc = 0.0;
#pragma unroll
            for (int n = 0; n < NP; ++n) acc += C[v][m + NP * n] * (b < NL ? lob(b, n) : T.bq[n][b - NL]);
            cr[v][m] = acc;
          }
        const int a0 = b < NL ? NL : 0;
        for (int a = a0; a < NL + NP; ++a) {
          double w[NV];
#pragma unroll
          for (int v = 0; v < K; ++v) {
            double acc = 0.0;
#pragma unroll
            for (int m = 0; m < NP; ++m) acc += cr[v][m] * (a < NL ? lob(a, m) : T.bq[m][a - NL]);
            w[v] = acc;
          }
          f(w);
        }
      }
    }
  };
  double rmin = INFINITY;
  visit(std::integral_constant<int, 1>{}, [&](const double *w) { rmin = fmin(rmin, w[0]); });
  double th1 = 1.0, th2 = 1.0;
  if (rmin < eps) {
    th1 = (wb[0] - eps) / (wb[0] - rmin);
#pragma unroll
    for (int q = 1; q < NM; ++q) C[0][q] *= th1;
  }
  visit(std::integral_constant<int, NV>{}, [&](const double *w) {
    if (pos_pressure<DIM>(w, g.gamma) < eps) th2 = fmin(th2, pos_root<DIM>(wb, w, eps, g.gamma));
  });
  if (th1 < 1.0 || th2 < 1.0) {
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int q = 1; q < NM; ++q) u[(long)(v * NM + q) * plane + cell] = th2 < 1.0 ? C[v][q] * th2 : C[v][q];
  }
  return false;
}

template <int N, int DIM>
__global__ __launch_bounds__(kBlock) void k_positivity(double *__restrict__ u, DevScalars *sc, Geometry g,
                                                       int check_done) {
  if (check_done && sc->done) return;
  const long plane = (long)g.nx * g.ny;
  bool bad = false;
  for (long cell = blockIdx.x * (long)blockDim.x + threadIdx.x; cell < plane; cell += (long)gridDim.x * blockDim.x)
    bad |= positivity_cell<N, DIM>(u, plane, cell, g);
  if (bad) atomicOr(&sc->status, 1);
}

// ---------------------------------------------------------------------------
// TVB-modified minmod indicator (Cockburn and Shu), per cell, with the list
// of troubled cells built by one atomic per wavefront.
// ---------------------------------------------------------------------------
__device__ inline double minmod3(double a, double b, double c) {
  if (a > 0.0 && b > 0.0 && c > 0.0) return fmin(a, fmin(b, c));
  if (a < 0.0 && b < 0.0 && c < 0.0) return fmax(a, fmax(b, c));
  return 0.0;
}

__device__ inline bool tvb_test(double a, double dp, double dm, double Mh2, double &margin) {
  double aa = fabs(a);
  if (aa <= Mh2) {
    margin = fmin(margin, Mh2 - aa);
    return false;
  }
  margin = fmin(margin, fmin(aa - Mh2, fmin(fabs(aa - fabs(dp)), fabs(aa - fabs(dm)))));
  return minmod3(a, dp, dm) != a;
}

struct LimitArgs {
  const double *u;      // pre-limit state (read only)
  double *side;         // side buffer, state layout
  DevScalars *sc;
  int32_t *count;       // device counter
  int32_t *list;
  uint8_t *flags;       // may be null
  double *margin;       // may be null
  const uint8_t *ovr;   // may be null
  Geometry geo;
  int mode;             // DG_IND_TVB / DG_IND_ALL
  int check_done;
};

// TVB-modified minmod decision of cell (i, j) from the state u; mg receives
// the decision margin.
template <int N, int EQ, int DIM, bool BND = true>
__device__ inline bool tvb_cell(const double *__restrict__ u, const Geometry &g, int i, int j, double &mg) {
  constexpr int NP = N + 1, NM = DIM == 1 ? NP : NP * NP, NV = Phys<EQ, DIM>::NV;
  const OrderTables &T = c_tab[N];
  const long plane = (long)g.nx * g.ny;
  const double k0 = DIM == 1 ? T.b0[0] : T.b0[0] * T.b0[0];
  bool flag = false;
  const CellIdx me = map_cell<BND>(g, i, j);
  CellIdx cp[DIM], cm[DIM];
  double Mh2[DIM];
#pragma unroll
  for (int dir = 0; dir < DIM; ++dir) {
    Mh2[dir] = dir == 0 ? g.tvb_Mx : g.tvb_My;
    if (BND && g.mhx) Mh2[dir] = dir == 0 ? g.mhx[i] : g.mhy[j];  // per column / row
    cp[dir] = map_cell<BND>(g, i + (dir == 0), j + (dir == 1));
    cm[dir] = map_cell<BND>(g, i - (dir == 0), j - (dir == 1));
  }
  // variable by variable: each variable's modes are dead once its tests are
  // done (decisions and margins combine by or / min, in any order)
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    double C[NM];
#pragma unroll
    for (int q = 0; q < NM; ++q) C[q] = cell_mode<NP, NM, DIM>(u, plane, g, me, v, q);
    const double mean = C[0] * k0;
#pragma unroll
    for (int dir = 0; dir < DIM; ++dir) {
      const double mp = cell_mode<NP, NM, DIM>(u, plane, g, cp[dir], v, 0) * k0;
      const double mm = cell_mode<NP, NM, DIM>(u, plane, g, cm[dir], v, 0) * k0;
      double up = 0.0, um = 0.0;
#pragma unroll
      for (int q = 0; q < NM; ++q) {
        int m = q % NP, n = q / NP;
        // odd Legendre polynomials vanish at the centre, psi_n(0) = 0: a
        // mode odd in the tangential direction adds nothing to a
        // face-midpoint trace, and one odd in both (never loaded) to none
        if (DIM == 2 && (dir == 0 ? (n & 1) : (m & 1))) continue;
        double bu, bd;
        if (DIM == 1) {
          bu = T.bp[m];
          bd = T.bm[m];
        } else if (dir == 0) {
          bu = T.bp[m] * T.b0[n];
          bd = T.bm[m] * T.b0[n];
        } else {
          bu = T.b0[m] * T.bp[n];
          bd = T.b0[m] * T.bm[n];
        }
        up += C[q] * bu;
        um += C[q] * bd;
      }
      const double dp = mp - mean, dm = mean - mm;
      flag |= tvb_test(up - mean, dp, dm, Mh2[dir], mg);
      flag |= tvb_test(mean - um, dp, dm, Mh2[dir], mg);
    }
  }
  return flag;
}

// KXRCF decision of cell (i, j) (Krivodonova et al., cited by Sec. 3 step 1):
// for each indicator variable (u; Euler: density and energy) the integral of
// the trace jump over the inflow faces (cell-average velocity pointing in),
// divided by h^((N+1)/2) (g.kx_scale), the inflow boundary's measure and the
// maximum of |u| over the volume quadrature points; troubled above 1.  mg
// receives min(|I - 1|, |v_x|, |v_y|).
template <int N, int EQ, int DIM, bool BND = true>
__device__ inline bool kxrcf_cell(const double *__restrict__ u, const Geometry &g, int i, int j, double &mg) {
  constexpr int NP = N + 1, NM = DIM == 1 ? NP : NP * NP, NV = Phys<EQ, DIM>::NV;
  constexpr int NVAR = EQ == 0 ? 1 : 2;
  const OrderTables &T = c_tab[N];
  const long plane = (long)g.nx * g.ny;
  const double k0 = DIM == 1 ? T.b0[0] : T.b0[0] * T.b0[0];
  double C[NV][NM];
  load_cell<NP, NM, NV, DIM>(u, plane, g, map_cell<BND>(g, i, j), C);
  double vel[2] = {0.0, 0.0};
  if (EQ == 0) {
    vel[0] = vel[1] = C[0][0] * k0;
  } else {
    const double rho = C[0][0] * k0;
    vel[0] = C[1][0] * k0 / rho;
    if (DIM == 2) vel[1] = C[2][0] * k0 / rho;
  }
  mg = fabs(vel[0]);
  if (DIM == 2) mg = fmin(mg, fabs(vel[1]));
  double kxs = g.kx_scale;
  if (BND && g.hxa) {  // non-uniform mesh: this cell's circumscribed radius
    const double hx = g.hxa[i], hy = DIM == 2 ? g.hya[j] : 0.0;
    const double rad = DIM == 1 ? 0.5 * hx : 0.5 * sqrt(hx * hx + hy * hy);
    kxs = 1.0 / pow(rad, 0.5 * (N + 1));
  }
  double J[NVAR], len = 0.0;
#pragma unroll
  for (int k = 0; k < NVAR; ++k) J[k] = 0.0;
#pragma unroll
  for (int dir = 0; dir < DIM; ++dir) {
    if (vel[dir] == 0.0) continue;
    const bool minus = vel[dir] > 0.0;  // inflow through the west / south face
    const int d = minus ? -1 : 1;
    const CellIdx cn = map_cell<BND>(g, i + (dir == 0 ? d : 0), j + (dir == 1 ? d : 0));
    const double *own = minus ? T.bm : T.bp, *nbr = minus ? T.bp : T.bm;
    const double flen = DIM == 1 ? 1.0 : (dir == 0 ? (BND && g.hya ? g.hya[j] : g.hy) : (BND && g.hxa ? g.hxa[i] : g.hx));
#pragma unroll
    for (int k = 0; k < NVAR; ++k) {
      const int v = k == 0 ? 0 : DIM + 1;
      double Nb[NM];
#pragma unroll
      for (int q = 0; q < NM; ++q) Nb[q] = cell_mode<NP, NM, DIM>(u, plane, g, cn, v, q);
      if (DIM == 1) {
        double a = 0.0, b = 0.0;
#pragma unroll
        for (int m = 0; m < NP; ++m) {
          a += C[v][m] * own[m];
          b += Nb[m] * nbr[m];
        }
        J[k] += a - b;
      } else {
        double integral = 0.0;
#pragma unroll
        for (int e = 0; e < NP; ++e) {
          double a = 0.0, b = 0.0;
#pragma unroll
          for (int q = 0; q < NM; ++q) {
            const int m = q % NP, n = q / NP;
            const double bb = dir == 0 ? own[m] * T.bq[n][e] : T.bq[m][e] * own[n];
            const double bn = dir == 0 ? nbr[m] * T.bq[n][e] : T.bq[m][e] * nbr[n];
            a += C[v][q] * bb;
            b += Nb[q] * bn;
          }
          integral += T.wq[e] * (a - b);
        }
        J[k] += 0.5 * flen * integral;
      }
    }
    len += flen;
  }
  bool flag = false;
#pragma unroll
  for (int k = 0; k < NVAR; ++k) {
    const int v = k == 0 ? 0 : DIM + 1;
    double norm = 0.0;
#pragma unroll
    for (int qy = 0; qy < (DIM == 2 ? NP : 1); ++qy)
#pragma unroll
      for (int qx = 0; qx < NP; ++qx) {
        double a = 0.0;
#pragma unroll
        for (int q = 0; q < NM; ++q) {
          const int m = q % NP, n = q / NP;
          a += C[v][q] * (DIM == 2 ? T.bq[m][qx] * T.bq[n][qy] : T.bq[m][qx]);
        }
        norm = fmax(norm, fabs(a));
      }
    const double I = (len > 0.0 && norm > 0.0) ? fabs(J[k]) * kxs / (len * norm) : 0.0;
    flag |= I > 1.0;
    mg = fmin(mg, fabs(I - 1.0));
  }
  return flag;
}

// Appends the flagged cells of a block to the troubled list (every thread of
// the block calls it): one atomic per block, since one per wavefront contends
// for the counter once most wavefronts flag a cell.  total: also add them to
// the run's count of troubled cells.
__device__ inline void append_troubled_block(const LimitArgs &a, bool flag, long cell, bool total = true) {
  __shared__ int s_cnt[kBlock / 64];
  __shared__ int s_base;
  const unsigned long long ballot = __ballot(flag);
  const int lane = __lane_id();
  const int wave = (threadIdx.x + threadIdx.y * blockDim.x) >> 6, waves = (blockDim.x * blockDim.y) >> 6;
  if (lane == 0) s_cnt[wave] = __popcll(ballot);
  __syncthreads();
  if (wave == 0 && lane == 0) {
    int n = 0;
    for (int w = 0; w < waves; ++w) n += s_cnt[w];
    s_base = n ? atomicAdd(a.count, n) : 0;
    if (n && total) atomicAdd(&a.sc->troubled_total, (unsigned long long)n);
  }
  __syncthreads();
  if (flag) {
    int base = s_base;
    for (int w = 0; w < wave; ++w) base += s_cnt[w];
    a.list[base + __popcll(ballot & ((1ull << lane) - 1ull))] = (int32_t)cell;
  }
}

// KX: the KXRCF indicator (an instantiation of its own, so that the TVB one
// keeps only one variable's modes live)
template <int N, int EQ, int DIM, bool BND, bool KX>
__global__ __launch_bounds__(kBlock) void k_indicator(LimitArgs a) {
  const Geometry &g = a.geo;
  if (a.check_done && a.sc->done) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = DIM == 1 ? 0 : blockIdx.y * blockDim.y + threadIdx.y;
  const bool active = i < g.nx && j < g.ny;
  const long cell = (long)j * g.nx + i;
  bool flag = false;
  double mg = INFINITY;
  if (active) {
    if (a.ovr) {
      flag = a.ovr[cell] != 0;
    } else if (a.mode == DG_IND_ALL) {
      flag = true;
    } else if (KX) {
      flag = kxrcf_cell<N, EQ, DIM, BND>(a.u, g, i, j, mg);
    } else {
      flag = tvb_cell<N, EQ, DIM, BND>(a.u, g, i, j, mg);
    }
    if (a.flags) a.flags[cell] = flag ? 1 : 0;
    if (a.margin) a.margin[cell] = mg;
  }
  append_troubled_block(a, flag, cell);
}

// ---------------------------------------------------------------------------
// CSWENO (Section 3).  One thread per (troubled cell, variable).
// ---------------------------------------------------------------------------

// WENO values at the Step-1 points of one row of 2N+1 stencil means.  The
// row is taken relative to the troubled cell's mean a[N] (the smoothness
// indicators only see derivatives and the normalised weights sum to one), so
// the quadratic forms do not cancel O(1) means.  The normalised weights
// (gamma_i / (eps + beta_i)^2) / sum_k (...) equal gamma_i d_i / sum_k gamma_k d_k
// with d_i = prod_{k != i} (eps + beta_k)^2 (numerator and denominator times
// the product of all (eps + beta_k)^2), which leaves one reciprocal per point.
template <int N, typename Tab>
__device__ inline void weno_row(const Tab &T, const double *a_in, double *out, double eps, bool raw) {
  constexpr int NP = N + 1, NG = num_points<N>(), NS = 2 * N + 1;
  const double a0 = a_in[N];
  double a[NS];
#pragma unroll
  for (int k = 0; k < NS; ++k) a[k] = a_in[k] - a0;
  double e2[NP];
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    double beta = 0.0;
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      double s = 0.0;
#pragma unroll
      for (int l = 0; l < NP; ++l) s += T.B[i][k][l] * a[i + l];
      beta += a[i + k] * s;
    }
    const double e = eps + beta;
    e2[i] = e * e;
  }
  double d[NP];  // products of the other stencils' (eps + beta)^2
  {
    double pre[NP], suf[NP];
    pre[0] = 1.0;
#pragma unroll
    for (int i = 1; i < NP; ++i) pre[i] = pre[i - 1] * e2[i - 1];
    suf[NP - 1] = 1.0;
#pragma unroll
    for (int i = NP - 2; i >= 0; --i) suf[i] = suf[i + 1] * e2[i + 1];
#pragma unroll
    for (int i = 0; i < NP; ++i) d[i] = pre[i] * suf[i];
  }
#pragma unroll
  for (int G = 0; G < NG; ++G) {
    double p[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < NP; ++k) s += T.T[G][i][k] * a[i + k];
      p[i] = s;
    }
    if (N == 3 && T.split[G] && !raw) {
      double wp = 0.0, up = 0.0, wm = 0.0, um = 0.0;
#pragma unroll
      for (int i = 0; i < NP; ++i) {
        double x = T.gpn[G][i] * d[i], y = T.gmn[G][i] * d[i];
        wp += x;
        up += x * p[i];
        wm += y;
        um += y * p[i];
      }
      out[G] = a0 + (T.sp[G] * (up * fast_rcp(wp)) - T.sm[G] * (um * fast_rcp(wm)));
    } else {
      double ws = 0.0, us = 0.0;
#pragma unroll
      for (int i = 0; i < NP; ++i) {
        double x = T.gam[G][i] * d[i];
        ws += x;
        us += x * p[i];
      }
      out[G] = a0 + us * fast_rcp(ws);
    }
  }
}

// The uniform-mesh tables of order N through a pointer the compiler cannot
// see through, produced after `dep` is computed.  Coefficients read through
// it are loaded into scalar registers at that point of the program: a phase
// of the limiter loads only its own coefficients once the previous phase's
// result exists.  (Read through c_tab directly, every coefficient the kernel
// uses is loaded once at its start; they overflow the scalar register file
// and are read back from vector-register lanes at every use.)
typedef const __attribute__((address_space(4))) OrderTables *tab_sptr;
template <int N>
__device__ __forceinline__ tab_sptr tab_after(double dep) {
  tab_sptr p = (tab_sptr)&c_tab[N];
  asm volatile("" : "+s"(p) : "v"(dep));
  return p;
}

// weno_row on rows F .. F+R-1 of src (row r: 2N+1 stencil means) with the
// uniform-mesh tables, out[G][r] = the WENO value at point G.  The same
// arithmetic, grouped by coefficient: one phase per stencil's smoothness
// matrix, then one per point, each over all R rows.
template <int N, int F, int R, int NR>
__device__ inline double weno_rows(const double (&src)[NR][2 * N + 1], double (&out)[num_points<N>()][NR], double eps,
                                   bool raw, double dep) {
  constexpr int NP = N + 1, NG = num_points<N>(), NS = 2 * N + 1;
  double a[R][NS], a0[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    a0[r] = src[F + r][N];
#pragma unroll
    for (int k = 0; k < NS; ++k) a[r][k] = src[F + r][k] - a0[r];
  }
  double e2[R][NP];
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    const tab_sptr T = tab_after<N>(dep);
    double B[NP][NP];
#pragma unroll
    for (int k = 0; k < NP; ++k)
#pragma unroll
      for (int l = 0; l < NP; ++l) B[k][l] = T->B[i][k][l];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      double beta = 0.0;
#pragma unroll
      for (int k = 0; k < NP; ++k) {
        double s = 0.0;
#pragma unroll
        for (int l = 0; l < NP; ++l) s += B[k][l] * a[r][i + l];
        beta += a[r][i + k] * s;
      }
      const double e = eps + beta;
      e2[r][i] = e * e;
    }
    dep = e2[0][i];
  }
  double d[R][NP];  // products of the other stencils' (eps + beta)^2
#pragma unroll
  for (int r = 0; r < R; ++r) {
    double pre[NP], suf[NP];
    pre[0] = 1.0;
#pragma unroll
    for (int i = 1; i < NP; ++i) pre[i] = pre[i - 1] * e2[r][i - 1];
    suf[NP - 1] = 1.0;
#pragma unroll
    for (int i = NP - 2; i >= 0; --i) suf[i] = suf[i + 1] * e2[r][i + 1];
#pragma unroll
    for (int i = 0; i < NP; ++i) d[r][i] = pre[i] * suf[i];
  }
#pragma unroll
  for (int G = 0; G < NG; ++G) {
    // the stencils' polynomials at x_G (one phase), then their weights (another)
    double p[R][NP];
    {
      const tab_sptr T = tab_after<N>(dep);
      double Tg[NP][NP];
#pragma unroll
      for (int i = 0; i < NP; ++i)
#pragma unroll
        for (int k = 0; k < NP; ++k) Tg[i][k] = T->T[G][i][k];
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int i = 0; i < NP; ++i) {
          double s = 0.0;
#pragma unroll
          for (int k = 0; k < NP; ++k) s += Tg[i][k] * a[r][i + k];
          p[r][i] = s;
        }
      dep = p[0][0];
    }
    const tab_sptr T = tab_after<N>(dep);
    const bool split = N == 3 && T->split[G] && !raw;
    double c1[NP], c2[NP], s1 = 0.0, s2 = 0.0;
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      c1[i] = split ? T->gpn[G][i] : T->gam[G][i];
      c2[i] = split ? T->gmn[G][i] : 0.0;
    }
    if (split) {
      s1 = T->sp[G];
      s2 = T->sm[G];
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (split) {
        double wp = 0.0, up = 0.0, wm = 0.0, um = 0.0;
#pragma unroll
        for (int i = 0; i < NP; ++i) {
          const double x = c1[i] * d[r][i], y = c2[i] * d[r][i];
          wp += x;
          up += x * p[r][i];
          wm += y;
          um += y * p[r][i];
        }
        out[G][F + r] = a0[r] + (s1 * (up * fast_rcp(wp)) - s2 * (um * fast_rcp(wm)));
      } else {
        double ws = 0.0, us = 0.0;
#pragma unroll
        for (int i = 0; i < NP; ++i) {
          const double x = c1[i] * d[r][i];
          ws += x;
          us += x * p[r][i];
        }
        out[G][F + r] = a0[r] + us * fast_rcp(ws);
      }
    }
    dep = out[G][F];
  }
  return dep;
}

// mean of psi_n over stencil interval k (0..2N) of the compact stencil
template <int N>
__device__ inline double interval_mean(const OrderTables &T, int k, int n) {
  if (k == N) return n == 0 ? T.b0[0] : 0.0;
  return T.sub[k < N ? k : k - N - 1][n];
}

// Reconstruction of variable v of the troubled cell `cell` from the
// pre-limit state u; the non-mean modes are written to `side`.
template <int N, int EQ, int DIM, bool BND = true>
__device__ inline void csweno_cell(const double *__restrict__ u, double *__restrict__ side, const Geometry &g,
                                   long cell, int v) {
  constexpr int NP = N + 1, NM = DIM == 1 ? NP : NP * NP;
  constexpr int NS = 2 * N + 1, NG = num_points<N>();
  const OrderTables &T = c_tab[N];
  const long plane = (long)g.nx * g.ny;
  const bool raw = g.negw_raw != 0;
  const int i = (int)(cell % g.nx), j = (int)(cell / g.nx);
  if (DIM == 1) {
    double st[NS];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      CellIdx ci = map_cell<BND>(g, i + c - 1, 0);
      double md[NP];
#pragma unroll
      for (int n = 0; n < NP; ++n) md[n] = cell_mode<NP, NM, 1>(u, plane, g, ci, v, n);
      const int k0 = c == 0 ? 0 : (c == 1 ? N : N + 1), k1 = c == 0 ? N : (c == 1 ? N + 1 : NS);
#pragma unroll
      for (int k = 0; k < NS; ++k) {
        if (k < k0 || k >= k1) continue;
        double s = 0.0;
#pragma unroll
        for (int n = 0; n < NP; ++n) s += md[n] * interval_mean<N>(T, k, n);
        st[k] = s;
      }
    }
    double uG[NG];
    if (BND && g.wtx) weno_row<N>(g.wtx[i], st, uG, g.eps, raw);  // this column's stencil
    else weno_row<N>(T, st, uG, g.eps, raw);
#pragma unroll
    for (int n = 1; n < NP; ++n) {
      double s = 0.0;
#pragma unroll
      for (int G = 0; G < NG; ++G) s += T.wg[G] * uG[G] * T.bg[n][G];
      side[(long)(v * NM + n) * plane + cell] = s;
    }
  } else {
    // (2N+1)^2 sub-rectangle means of the 3x3 block, [iy][ix]; im(k, n) is
    // interval_mean
    double st[NS][NS];
    auto fill_st = [&](auto im) {
#pragma unroll
      for (int cy = 0; cy < 3; ++cy)
#pragma unroll
        for (int cx = 0; cx < 3; ++cx) {
          CellIdx ci = map_cell<BND>(g, i + cx - 1, j + cy - 1);
          double md[NM];
#pragma unroll
          for (int q = 0; q < NM; ++q) md[q] = cell_mode<NP, NM, 2>(u, plane, g, ci, v, q);
          const int x0 = cx == 0 ? 0 : (cx == 1 ? N : N + 1), x1 = cx == 0 ? N : (cx == 1 ? N + 1 : NS);
          const int y0 = cy == 0 ? 0 : (cy == 1 ? N : N + 1), y1 = cy == 0 ? N : (cy == 1 ? N + 1 : NS);
#pragma unroll
          for (int ix = 0; ix < NS; ++ix) {
            if (ix < x0 || ix >= x1) continue;
            double tn[NP];
#pragma unroll
            for (int n = 0; n < NP; ++n) {
              double s = 0.0;
#pragma unroll
              for (int m = 0; m < NP; ++m) s += md[m + NP * n] * im(ix, m);
              tn[n] = s;
            }
#pragma unroll
            for (int iy = 0; iy < NS; ++iy) {
              if (iy < y0 || iy >= y1) continue;
              double s = 0.0;
#pragma unroll
              for (int n = 0; n < NP; ++n) s += tn[n] * im(iy, n);
              st[iy][ix] = s;
            }
          }
        }
    };
    if constexpr (!BND) {
      // the periodic/transmissive kernels (the hot ones): interval means and
      // then each WENO phase's coefficients loaded when needed (tab_after), the
      // rows of each sweep batched
      const tab_sptr Ts = tab_after<N>((double)(int)cell);
      double sb[N][NP];
#pragma unroll
      for (int k = 0; k < N; ++k)
#pragma unroll
        for (int n = 0; n < NP; ++n) sb[k][n] = Ts->sub[k][n];
      const double b00 = Ts->b0[0];
      fill_st([&](int k, int n) -> double {
        if (k == N) return n == 0 ? b00 : 0.0;
        return sb[k < N ? k : k - N - 1][n];
      });
      // x-sweeps: y-interval means at the x-points, vy[G][iy]; Q3 in two
      // batches of rows (register file)
      double vy[NG][NS];
      double dep = st[N][N];
      if constexpr (N == 3) {
        dep = weno_rows<N, 0, 4>(st, vy, g.eps, raw, dep);
        dep = weno_rows<N, 4, NS - 4>(st, vy, g.eps, raw, dep);
      } else {
        dep = weno_rows<N, 0, NS>(st, vy, g.eps, raw, dep);
      }
      // y-sweeps at every x-point: uy[H][G] = u(x_G, y_H)
      double uy[NG][NG];
      dep = weno_rows<N, 0, NG>(vy, uy, g.eps, raw, dep);
      // the tensor projection
      const tab_sptr Tp = tab_after<N>(dep);
      double wb[NP][NG];  // wg[G] psi_n(r_G)
#pragma unroll
      for (int n = 0; n < NP; ++n)
#pragma unroll
        for (int G = 0; G < NG; ++G) wb[n][G] = Tp->wg[G] * Tp->bg[n][G];
      double sp[NG][NP];  // sp[G][n] = sum_H wg[H] u(G,H) psi_n(y_H)
#pragma unroll
      for (int G = 0; G < NG; ++G)
#pragma unroll
        for (int n = 0; n < NP; ++n) {
          double acc = 0.0;
#pragma unroll
          for (int H = 0; H < NG; ++H) acc += Tp->wg[H] * uy[H][G] * Tp->bg[n][H];
          sp[G][n] = acc;
        }
#pragma unroll
      for (int q = 1; q < NM; ++q) {
        const int m = q % NP, n = q / NP;
        double acc = 0.0;
#pragma unroll
        for (int G = 0; G < NG; ++G) acc += wb[m][G] * sp[G][n];
        side[(long)(v * NM + q) * plane + cell] = acc;
      }
      return;
    } else {
#pragma unroll
      for (int cy = 0; cy < 3; ++cy)
#pragma unroll
        for (int cx = 0; cx < 3; ++cx) {
          CellIdx ci = map_cell<BND>(g, i + cx - 1, j + cy - 1);
          double md[NM];
#pragma unroll
          for (int q = 0; q < NM; ++q) md[q] = cell_mode<NP, NM, 2>(u, plane, g, ci, v, q);
          const int x0 = cx == 0 ? 0 : (cx == 1 ? N : N + 1), x1 = cx == 0 ? N : (cx == 1 ? N + 1 : NS);
          const int y0 = cy == 0 ? 0 : (cy == 1 ? N : N + 1), y1 = cy == 0 ? N : (cy == 1 ? N + 1 : NS);
#pragma unroll
          for (int ix = 0; ix < NS; ++ix) {
            if (ix < x0 || ix >= x1) continue;
            double tn[NP];
#pragma unroll
            for (int n = 0; n < NP; ++n) {
              double s = 0.0;
#pragma unroll
              for (int m = 0; m < NP; ++m) s += md[m + NP * n] * interval_mean<N>(T, ix, m);
              tn[n] = s;
            }
#pragma unroll
            for (int iy = 0; iy < NS; ++iy) {
              if (iy < y0 || iy >= y1) continue;
              double s = 0.0;
#pragma unroll
              for (int n = 0; n < NP; ++n) s += tn[n] * interval_mean<N>(T, iy, n);
              st[iy][ix] = s;
            }
          }
        }
    }
    // x-sweeps: y-interval means at the x-points
    double vy[NG][NS];
#pragma unroll
    for (int iy = 0; iy < NS; ++iy) {
      double r[NG];
      if (BND && g.wtx) weno_row<N>(g.wtx[i], st[iy], r, g.eps, raw);
      else weno_row<N>(T, st[iy], r, g.eps, raw);
#pragma unroll
      for (int G = 0; G < NG; ++G) vy[G][iy] = r[G];
    }
    // y-sweeps at every x-point, then the tensor projection
    double s[NG][NP];  // s[G][n] = sum_H wg[H] u(G,H) psi_n(y_H)
#pragma unroll
    for (int G = 0; G < NG; ++G) {
      double u[NG];
      if (BND && g.wty) weno_row<N>(g.wty[j], vy[G], u, g.eps, raw);  // this row's stencil
      else weno_row<N>(T, vy[G], u, g.eps, raw);
#pragma unroll
      for (int n = 0; n < NP; ++n) {
        double acc = 0.0;
#pragma unroll
        for (int H = 0; H < NG; ++H) acc += T.wg[H] * u[H] * T.bg[n][H];
        s[G][n] = acc;
      }
    }
#pragma unroll
    for (int q = 1; q < NM; ++q) {
      const int m = q % NP, n = q / NP;
      double acc = 0.0;
#pragma unroll
      for (int G = 0; G < NG; ++G) acc += T.wg[G] * T.bg[m][G] * s[G][n];
      side[(long)(v * NM + q) * plane + cell] = acc;
    }
  }
}

// Thread t takes variable t / count of list entry t % count: a wavefront works
// on one variable of consecutive entries (neighbouring cells).
template <int N, int EQ, int DIM, bool BND>
__global__ __launch_bounds__(kBlock) void k_csweno(LimitArgs a) {
  constexpr int NV = Phys<EQ, DIM>::NV;
  if (a.check_done && a.sc->done) return;
  const long count = *a.count;
  const long total = count * NV;
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x)
    csweno_cell<N, EQ, DIM, BND>(a.u, a.side, a.geo, a.list[t % count], (int)(t / count));
}

// ---------------------------------------------------------------------------
// CSWENO in local characteristic fields (Euler; the paper limits systems in
// characteristic fields, end of Sec. 3).  One thread per troubled cell.
// ---------------------------------------------------------------------------

// Eigenvectors of the Euler flux Jacobian in direction dir at the conserved
// state w: R's columns are the right eigenvectors (eigenvalues u_n - c, u_n,
// u_n + c, and u_n for the 2D shear wave), L = R^-1.
template <int DIM>
__device__ inline void char_eig(double gam, int dir, const double (&w)[DIM + 2], double (&L)[DIM + 2][DIM + 2],
                                double (&R)[DIM + 2][DIM + 2]) {
  const double rho = w[0];
  const double un = (DIM == 1 ? w[1] : w[1 + dir]) / rho;
  const double ut = DIM == 1 ? 0.0 : w[2 - dir] / rho;
  const double E = w[DIM + 1];
  const double q2 = un * un + ut * ut;
  const double p = (gam - 1.0) * (E - 0.5 * rho * q2);
  const double c = sqrt(gam * p / rho), H = (E + p) / rho;
  const double b1 = (gam - 1.0) / (c * c), b2 = 0.5 * b1 * q2;
  if constexpr (DIM == 1) {
    const double Rm[3][3] = {{1.0, 1.0, 1.0}, {un - c, un, un + c}, {H - un * c, 0.5 * q2, H + un * c}};
    const double Lm[3][3] = {{0.5 * (b2 + un / c), -0.5 * (b1 * un + 1.0 / c), 0.5 * b1},
                             {1.0 - b2, b1 * un, -b1},
                             {0.5 * (b2 - un / c), -0.5 * (b1 * un - 1.0 / c), 0.5 * b1}};
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        R[a][b] = Rm[a][b];
        L[a][b] = Lm[a][b];
      }
  } else {
    // (normal, tangential) momentum ordering, then permuted back to (x, y)
    const double Rm[4][4] = {{1.0, 1.0, 1.0, 0.0},
                             {un - c, un, un + c, 0.0},
                             {ut, ut, ut, 1.0},
                             {H - un * c, 0.5 * q2, H + un * c, ut}};
    const double Lm[4][4] = {{0.5 * (b2 + un / c), -0.5 * (b1 * un + 1.0 / c), -0.5 * b1 * ut, 0.5 * b1},
                             {1.0 - b2, b1 * un, b1 * ut, -b1},
                             {0.5 * (b2 - un / c), -0.5 * (b1 * un - 1.0 / c), -0.5 * b1 * ut, 0.5 * b1},
                             {-ut, 0.0, 1.0, 0.0}};
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int pa = a == 1 ? 1 + dir : (a == 2 ? 2 - dir : a);
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int pb = b == 1 ? 1 + dir : (b == 2 ? 2 - dir : b);
        R[pa][b] = Rm[a][b];
        L[a][pb] = Lm[a][b];
      }
    }
  }
}

// Modes of variable v of cell (i, j) with the boundary reflections applied.
template <int NP, int NM, int DIM>
__device__ inline void load_var(const double *__restrict__ u, long plane, const Geometry &g, const CellIdx &c, int v,
                                double (&md)[NM]) {
#pragma unroll
  for (int q = 0; q < NM; ++q) md[q] = cell_mode<NP, NM, DIM>(u, plane, g, c, v, q);
}

template <int N, int DIM, bool BND = true>
__device__ inline void csweno_char_cell(const double *__restrict__ u, double *__restrict__ side, const Geometry &g,
                                        long cell) {
  constexpr int NP = N + 1, NM = DIM == 1 ? NP : NP * NP, NV = DIM + 2;
  constexpr int NS = 2 * N + 1, NG = num_points<N>();
  const OrderTables &T = c_tab[N];
  const long plane = (long)g.nx * g.ny;
  const bool raw = g.negw_raw != 0;
  const int i = (int)(cell % g.nx), j = (int)(cell / g.nx);
  const double k0 = DIM == 1 ? T.b0[0] : T.b0[0] * T.b0[0];
  double w0[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) w0[v] = u[(long)(v * NM) * plane + cell] * k0;
  double L[NV][NV], R[NV][NV];
  if constexpr (DIM == 1) {
    double a[NV][NS];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const CellIdx ci = map_cell<BND>(g, i + c - 1, 0);
      const int k0c = c == 0 ? 0 : (c == 1 ? N : N + 1), k1c = c == 0 ? N : (c == 1 ? N + 1 : NS);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        double md[NM];
        load_var<NP, NM, 1>(u, plane, g, ci, v, md);
#pragma unroll
        for (int k = 0; k < NS; ++k) {
          if (k < k0c || k >= k1c) continue;
          double s = 0.0;
#pragma unroll
          for (int n = 0; n < NP; ++n) s += md[n] * interval_mean<N>(T, k, n);
          a[v][k] = s;
        }
      }
    }
    char_eig<1>(g.gamma, 0, w0, L, R);
    double cG[NV][NG];
#pragma unroll
    for (int f = 0; f < NV; ++f) {
      double ch[NS];
#pragma unroll
      for (int k = 0; k < NS; ++k) {
        double s = 0.0;
#pragma unroll
        for (int v = 0; v < NV; ++v) s += L[f][v] * a[v][k];
        ch[k] = s;
      }
      if (BND && g.wtx) weno_row<N>(g.wtx[i], ch, cG[f], g.eps, raw);  // this column's stencil
      else weno_row<N>(T, ch, cG[f], g.eps, raw);
    }
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int n = 1; n < NP; ++n) {
        double s = 0.0;
#pragma unroll
        for (int G = 0; G < NG; ++G) {
          double uG = 0.0;
#pragma unroll
          for (int f = 0; f < NV; ++f) uG += R[v][f] * cG[f][G];
          s += T.wg[G] * uG * T.bg[n][G];
        }
        side[(long)(v * NM + n) * plane + cell] = s;
      }
  } else {
    // x-sweeps on every y-interval, in x-characteristic fields
    double vy[NV][NS][NG];
    char_eig<2>(g.gamma, 0, w0, L, R);
#pragma unroll 1
    for (int iy = 0; iy < NS; ++iy) {
      const int cy = iy < N ? 0 : (iy == N ? 1 : 2);
      double a[NV][NS];
#pragma unroll
      for (int cx = 0; cx < 3; ++cx) {
        const CellIdx ci = map_cell<BND>(g, i + cx - 1, j + cy - 1);
        const int x0 = cx == 0 ? 0 : (cx == 1 ? N : N + 1), x1 = cx == 0 ? N : (cx == 1 ? N + 1 : NS);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          double md[NM];
          load_var<NP, NM, 2>(u, plane, g, ci, v, md);
#pragma unroll
          for (int ix = 0; ix < NS; ++ix) {
            if (ix < x0 || ix >= x1) continue;
            double s = 0.0;
#pragma unroll
            for (int n = 0; n < NP; ++n) {
              double t = 0.0;
#pragma unroll
              for (int m = 0; m < NP; ++m) t += md[m + NP * n] * interval_mean<N>(T, ix, m);
              s += t * interval_mean<N>(T, iy, n);
            }
            a[v][ix] = s;
          }
        }
      }
      double cG[NV][NG];
      if constexpr (!BND) {  // the fields' rows batched, coefficients by phase (weno_rows)
        double ch[NV][NS], cGt[NG][NV];
#pragma unroll
        for (int f = 0; f < NV; ++f)
#pragma unroll
          for (int ix = 0; ix < NS; ++ix) {
            double s = 0.0;
#pragma unroll
            for (int v = 0; v < NV; ++v) s += L[f][v] * a[v][ix];
            ch[f][ix] = s;
          }
        weno_rows<N, 0, NV>(ch, cGt, g.eps, raw, ch[0][N]);
#pragma unroll
        for (int f = 0; f < NV; ++f)
#pragma unroll
          for (int G = 0; G < NG; ++G) cG[f][G] = cGt[G][f];
      } else {
#pragma unroll
        for (int f = 0; f < NV; ++f) {
          double ch[NS];
#pragma unroll
          for (int ix = 0; ix < NS; ++ix) {
            double s = 0.0;
#pragma unroll
            for (int v = 0; v < NV; ++v) s += L[f][v] * a[v][ix];
            ch[ix] = s;
          }
          if (BND && g.wtx) weno_row<N>(g.wtx[i], ch, cG[f], g.eps, raw);
          else weno_row<N>(T, ch, cG[f], g.eps, raw);
        }
      }
#pragma unroll
      for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int G = 0; G < NG; ++G) {
          double s = 0.0;
#pragma unroll
          for (int f = 0; f < NV; ++f) s += R[v][f] * cG[f][G];
          vy[v][iy][G] = s;
        }
    }
    // y-sweeps at every x-point, in y-characteristic fields, and the projection
    char_eig<2>(g.gamma, 1, w0, L, R);
    double out[NV][NM];
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int q = 0; q < NM; ++q) out[v][q] = 0.0;
#pragma unroll
    for (int G = 0; G < NG; ++G) {
      double cH[NV][NG];
      if constexpr (!BND) {
        double ch[NV][NS], cHt[NG][NV];
#pragma unroll
        for (int f = 0; f < NV; ++f)
#pragma unroll
          for (int iy = 0; iy < NS; ++iy) {
            double s = 0.0;
#pragma unroll
            for (int v = 0; v < NV; ++v) s += L[f][v] * vy[v][iy][G];
            ch[f][iy] = s;
          }
        weno_rows<N, 0, NV>(ch, cHt, g.eps, raw, ch[0][N]);
#pragma unroll
        for (int f = 0; f < NV; ++f)
#pragma unroll
          for (int H = 0; H < NG; ++H) cH[f][H] = cHt[H][f];
      } else {
#pragma unroll
        for (int f = 0; f < NV; ++f) {
          double ch[NS];
#pragma unroll
          for (int iy = 0; iy < NS; ++iy) {
            double s = 0.0;
#pragma unroll
            for (int v = 0; v < NV; ++v) s += L[f][v] * vy[v][iy][G];
            ch[iy] = s;
          }
          if (BND && g.wty) weno_row<N>(g.wty[j], ch, cH[f], g.eps, raw);  // this row's stencil
          else weno_row<N>(T, ch, cH[f], g.eps, raw);
        }
      }
#pragma unroll
      for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int n = 0; n < NP; ++n) {
          double sn = 0.0;
#pragma unroll
          for (int H = 0; H < NG; ++H) {
            double uH = 0.0;
#pragma unroll
            for (int f = 0; f < NV; ++f) uH += R[v][f] * cH[f][H];
            sn += T.wg[H] * uH * T.bg[n][H];
          }
#pragma unroll
          for (int m = 0; m < NP; ++m) out[v][m + NP * n] += T.wg[G] * T.bg[m][G] * sn;
        }
    }
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int q = 1; q < NM; ++q) side[(long)(v * NM + q) * plane + cell] = out[v][q];
  }
}

template <int N, int DIM, bool BND>
__global__ __launch_bounds__(kBlock) void k_csweno_char(LimitArgs a) {
  if (a.check_done && a.sc->done) return;
  const long total = *a.count;
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x)
    csweno_char_cell<N, DIM, BND>(a.u, a.side, a.geo, a.list[t]);
}

// Consecutive threads take consecutive list entries of one (variable, mode)
// plane, so a wavefront's accesses fall on the few cache lines that
// neighbouring troubled cells share.
template <int NM, int NV>
__global__ __launch_bounds__(kBlock) void k_scatter(LimitArgs a, double *dst) {
  if (a.check_done && a.sc->done) return;
  const long plane = (long)a.geo.nx * a.geo.ny;
  const long count = *a.count;
  const long total = count * NV * (NM - 1);
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
    const long e = t % count, r = t / count;  // r = v (NM - 1) + q - 1
    const int q = 1 + (int)(r % (NM - 1)), v = (int)(r / (NM - 1));
    const long k = (long)(v * NM + q) * plane + a.list[e];
    dst[k] = a.side[k];
  }
}

#include "dg_mlp.hpp"
#include "dg_batch.hpp"

// ---------------------------------------------------------------------------
// L2 projection of point values (rows j0..j0+nrows-1).
// ---------------------------------------------------------------------------
template <int N, int DIM>
__global__ __launch_bounds__(kBlock) void k_project(const double *__restrict__ pv, double *__restrict__ u,
                                                    Geometry g, int nv, int j0, int nrows) {
  constexpr int NP = N + 1, NM = DIM == 1 ? NP : NP * NP;
  const OrderTables &T = c_tab[N];
  const long rowcells = (long)nrows * g.nx;
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= rowcells * nv) return;
  const int v = (int)(t / rowcells);
  const long c = t % rowcells;  // cell within the given rows
  const long plane = (long)g.nx * g.ny;
  const long cell = (long)j0 * g.nx + c;
  const int nq = T.npq, nqy = DIM == 1 ? 1 : T.npq;
  double acc[NM];
#pragma unroll
  for (int q = 0; q < NM; ++q) acc[q] = 0.0;
  for (int b = 0; b < nqy; ++b)
    for (int aq = 0; aq < nq; ++aq) {
      double val = pv[((long)(v * nqy + b) * nq + aq) * rowcells + c];
#pragma unroll
      for (int q = 0; q < NM; ++q) {
        const int m = q % NP, n = q / NP;
        double w = T.wpq[aq] * T.bpq[m][aq];
        if (DIM == 2) w *= T.wpq[b] * T.bpq[n][b];
        acc[q] += w * val;
      }
    }
#pragma unroll
  for (int q = 0; q < NM; ++q) u[(long)(v * NM + q) * plane + cell] = acc[q];
}

// ---------------------------------------------------------------------------
// Dispatch on (dim, equation, order).
// ---------------------------------------------------------------------------
inline hipStream_t S(const LaunchCtx &c) { return (hipStream_t)c.stream; }

int check_launch() {
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? DG_OK : DG_ERR_HIP;
}

template <typename F>
int dispatch(const LaunchCtx &c, F &&f) {
#define DG_CASE(D, E, NN)                                     \
  if (c.dim == D && c.eq == E && c.N == NN) {                 \
    f(std::integral_constant<int, D>{}, std::integral_constant<int, E>{}, std::integral_constant<int, NN>{}); \
    return check_launch();                                    \
  }
  DG_CASE(1, 0, 1) DG_CASE(1, 0, 2) DG_CASE(1, 0, 3)
  DG_CASE(1, 1, 1) DG_CASE(1, 1, 2) DG_CASE(1, 1, 3)
  DG_CASE(2, 0, 1) DG_CASE(2, 0, 2) DG_CASE(2, 0, 3)
  DG_CASE(2, 1, 1) DG_CASE(2, 1, 2) DG_CASE(2, 1, 3)
#undef DG_CASE
  return DG_ERR_UNSUPPORTED;
}

dim3 cell_grid(const LaunchCtx &c, dim3 &block) {
  if (c.dim == 1) {
    block = dim3(kBlock, 1, 1);
    return dim3((c.geo.nx + kBlock - 1) / kBlock, 1, 1);
  }
  block = dim3(64, kBlock / 64, 1);
  return dim3((c.geo.nx + 63) / 64, (c.geo.ny + block.y - 1) / block.y, 1);
}

// Rows per marching wavefront: enough waves to fill 256 CUs several times.
int march_rows(const LaunchCtx &c, int strip = kStrip) {
  if (c.rows > 0) return c.rows;
  const long strips = (c.geo.nx + strip - 1) / strip;
  int rows = 32;
  while (rows > 4 && strips * ((c.geo.ny + rows - 1) / rows) < 8192) rows /= 2;
  return rows;
}

template <int D, int E, int NN, int STAGE>
void stage_launch(const LaunchCtx &c, const StageArgs &a) {
  constexpr bool march = D == 2 && E == 0;
  if (D == 2 && E == 1 && c.use_march) {
    constexpr int strip = euler_strip(NN);
    const int rows = march_rows(c, strip);
    dim3 grid((c.geo.nx + strip - 1) / strip, (c.geo.ny + rows - 1) / rows, 1);
    const bool off32 = euler_off32_fits(NN, (long long)c.geo.nx * c.geo.ny);
    if (c.special_bc) {
      if (off32) hipLaunchKernelGGL((k_stage_2d_euler<NN, STAGE, true, true>), grid, dim3(64), 0, S(c), a, rows);
      else hipLaunchKernelGGL((k_stage_2d_euler<NN, STAGE, true, false>), grid, dim3(64), 0, S(c), a, rows);
    } else {
      if (off32) hipLaunchKernelGGL((k_stage_2d_euler<NN, STAGE, false, true>), grid, dim3(64), 0, S(c), a, rows);
      else hipLaunchKernelGGL((k_stage_2d_euler<NN, STAGE, false, false>), grid, dim3(64), 0, S(c), a, rows);
    }
    return;
  }
  if (D == 2 && march && c.use_march) {
    const int rows = march_rows(c);
    dim3 grid((c.geo.nx + kStrip - 1) / kStrip, (c.geo.ny + rows - 1) / rows, 1);
    hipLaunchKernelGGL((k_stage_2d_march<NN, E, STAGE>), grid, dim3(64), 0, S(c), a, rows);
    return;
  }
  dim3 block, grid = cell_grid(c, block);
  if (D == 1) hipLaunchKernelGGL((k_stage_1d<NN, E, STAGE>), grid, block, 0, S(c), a);
  else hipLaunchKernelGGL((k_stage_2d<NN, E, STAGE>), grid, block, 0, S(c), a);
}

}  // namespace

// Stage kernels of one order (the largest share of the build): order 1 in
// part 0, order 2 in part 4, order 3 in part 5.  stage 0 is the residual.
#if DG_PART == 0 || DG_PART == 4 || DG_PART == 5
#if DG_PART == 0
#define DG_STAGE_N 1
#elif DG_PART == 4
#define DG_STAGE_N 2
#else
#define DG_STAGE_N 3
#endif
int DG_CAT(launch_stage_order, DG_STAGE_N)(const LaunchCtx &c, int stage, const double *u, const double *un,
                                           double *out, bool want_speed) {
  constexpr int n = DG_STAGE_N;
  StageArgs a{u, un, out, c.sc, c.geo, want_speed ? 1 : 0};
  auto go = [&](auto D, auto E) {
    constexpr int d = decltype(D)::value, e = decltype(E)::value;
    if (stage == 0) stage_launch<d, e, n, 0>(c, a);
    else if (stage == 1) stage_launch<d, e, n, 1>(c, a);
    else if (stage == 2) stage_launch<d, e, n, 2>(c, a);
    else stage_launch<d, e, n, 3>(c, a);
  };
  using I0 = std::integral_constant<int, 0>;
  using I1 = std::integral_constant<int, 1>;
  using I2 = std::integral_constant<int, 2>;
  if (c.N != n || stage < 0 || stage > 3) return DG_ERR_INVALID_ARG;
  if (c.dim == 1 && c.eq == 0) go(I1{}, I0{});
  else if (c.dim == 1 && c.eq == 1) go(I1{}, I1{});
  else if (c.dim == 2 && c.eq == 0) go(I2{}, I0{});
  else if (c.dim == 2 && c.eq == 1) go(I2{}, I1{});
  else return DG_ERR_UNSUPPORTED;
  return check_launch();
}
#endif  // DG_PART == 0 || DG_PART == 4 || DG_PART == 5

#if DG_PART == 0
int launch_stage(const LaunchCtx &c, int stage, const double *u, const double *un, double *out, bool want_speed) {
  if (stage < 1 || stage > 3) return DG_ERR_INVALID_ARG;
  switch (c.N) {
    case 1: return launch_stage_order1(c, stage, u, un, out, want_speed);
    case 2: return launch_stage_order2(c, stage, u, un, out, want_speed);
    case 3: return launch_stage_order3(c, stage, u, un, out, want_speed);
    default: return DG_ERR_UNSUPPORTED;
  }
}

int launch_residual(const LaunchCtx &c, const double *u, double *out) {
  switch (c.N) {
    case 1: return launch_stage_order1(c, 0, u, nullptr, out, false);
    case 2: return launch_stage_order2(c, 0, u, nullptr, out, false);
    case 3: return launch_stage_order3(c, 0, u, nullptr, out, false);
    default: return DG_ERR_UNSUPPORTED;
  }
}

#endif  // DG_PART == 0

#if DG_PART == 1
// Allocation-free limiter call (dg_limit_noalloc): scratch in a file-scope
// device array instead of a caller workspace.  Layout: DevScalars at 0, the
// troubled list at kStaticListOffset, the side buffer after it.
namespace {
std::mutex g_scratch_mu;
void *g_scratch_ptr[64];

__global__ void k_scratch_init(DevScalars *sc, double tb) {
  if (threadIdx.x != 0) return;
  sc->count[3] = 0;
  sc->status = 0;
  sc->done = 0;
  sc->tb = tb;
}
}  // namespace

int static_scratch(int device, void **ptr) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (device < 0 || device >= 64 || !ptr) return DG_ERR_HIP;
  if (!g_scratch_ptr[device]) {
    void *q = nullptr;
    if (hipGetSymbolAddress(&q, HIP_SYMBOL(scratch)) != hipSuccess || !q) return DG_ERR_HIP;
    g_scratch_ptr[device] = q;
  }
  *ptr = g_scratch_ptr[device];
  return DG_OK;
}

int launch_scratch_init(const LaunchCtx &c, double tb) {
  hipLaunchKernelGGL(k_scratch_init, dim3(1), dim3(64), 0, S(c), c.sc, tb);
  return check_launch();
}

// The troubled list rebuilt in row order from the flags the learned pass has
// written: that pass appends its cells per wavefront in 14-cell pieces of its
// strip, so the 64 consecutive entries a reconstruction or scatter wavefront
// takes would span about five rows.  The same cells; counted once, by the
// learned pass.
__global__ __launch_bounds__(kBlock) void k_list_from_flags(LimitArgs a) {
  const Geometry &g = a.geo;
  if (a.check_done && a.sc->done) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  const long cell = (long)j * g.nx + i;
  const bool flag = i < g.nx && j < g.ny && a.flags[cell] != 0;
  append_troubled_block(a, flag, cell, false);
}

int launch_limit(const LaunchCtx &c, double *u, double *side, int count_slot, uint8_t *flags, double *margin,
                 const uint8_t *flags_override) {
  LimitArgs a;
  a.u = u;
  a.side = side;
  a.sc = c.sc;
  a.count = &c.sc->count[count_slot];
  a.list = c.list;
  a.flags = flags;
  a.margin = margin;
  a.ovr = flags_override;
  a.geo = c.geo;
  a.mode = c.indicator;
  a.check_done = count_slot < 3 ? 1 : 0;
  auto body = [&](auto D, auto E, auto NN, auto B) {
    constexpr int d = decltype(D)::value, e = decltype(E)::value, n = decltype(NN)::value;
    constexpr bool bnd = decltype(B)::value;
    constexpr int NM = d == 1 ? n + 1 : (n + 1) * (n + 1);
    constexpr int NV = Phys<e, d>::NV;
    dim3 block, grid = cell_grid(c, block);
    bool learned = false;
    if constexpr (d == 2 && e == DG_EQ_EULER && !bnd) {  // (the learned indicator takes no special sides)
      if (c.indicator == DG_IND_LEARNED && !flags_override) {
        LearnedArgs L{c.mlp_w, c.mlp_m, MlpLayout{5 * NM * NV, (5 * NM * NV + 15) / 16 * 16}, (float)c.band_lo,
                      (float)c.band_hi, c.mlp_prob};
        constexpr int waves = lm_waves(n);
        const int groups = ((c.geo.nx + kLmStrip - 1) / kLmStrip + waves - 1) / waves;
        // the pass writes its flags (the problem's flag buffer if the caller
        // passed none) and its own list on a counter of its own; the list the
        // limiter reads is then rebuilt from the flags in row order
        LimitArgs al = a;
        if (!al.flags) al.flags = c.flags;
        al.count = &c.sc->count_scratch;
        hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, S(c), c.sc, 2);
        hipLaunchKernelGGL((k_indicator_learned<n, e, false>), dim3(groups, (c.geo.ny + kLmRows - 1) / kLmRows),
                           dim3(64 * waves), 0, S(c), al, L, kLmRows);
        LimitArgs ar = a;
        ar.flags = al.flags;
        hipLaunchKernelGGL(k_list_from_flags, grid, block, 0, S(c), ar);
        learned = true;
      }
    }
    if (!learned) {
      if (c.indicator == DG_IND_KXRCF) hipLaunchKernelGGL((k_indicator<n, e, d, bnd, true>), grid, block, 0, S(c), a);
      else hipLaunchKernelGGL((k_indicator<n, e, d, bnd, false>), grid, block, 0, S(c), a);
    }
    if (c.limiter != DG_LIM_NONE) {
      bool chr = false;
      if constexpr (e == DG_EQ_EULER) {
        if (c.limiter == DG_LIM_CSWENO_CHAR) {
          hipLaunchKernelGGL((k_csweno_char<n, d, bnd>), dim3(c.grid_cap), dim3(kBlock), 0, S(c), a);
          chr = true;
        }
      }
      if (!chr) hipLaunchKernelGGL((k_csweno<n, e, d, bnd>), dim3(c.grid_cap), dim3(kBlock), 0, S(c), a);
      hipLaunchKernelGGL((k_scatter<NM, NV>), dim3(c.grid_cap), dim3(kBlock), 0, S(c), a, u);
    }
  };
  // walls, inflow and switching sides get their own instantiations, so that
  // problems with periodic and transmissive sides only carry none of that code
  return dispatch(c, [&](auto D, auto E, auto NN) {
    if (c.special_bc) body(D, E, NN, std::true_type{});
    else body(D, E, NN, std::false_type{});
  });
}

#endif  // DG_PART == 1

#if DG_PART == 0
int launch_speed(const LaunchCtx &c, const double *u) {
  hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, S(c), c.sc, 1);
  const long cells = (long)c.geo.nx * c.geo.ny;
  dim3 grid((unsigned)std::min<long>((cells + kBlock - 1) / kBlock, 2048));
  return dispatch(c, [&](auto D, auto E, auto NN) {
    hipLaunchKernelGGL((k_speed<decltype(NN)::value, decltype(E)::value, decltype(D)::value>), grid, dim3(kBlock),
                       0, S(c), u, c.sc, c.geo);
  });
}

int launch_positivity(const LaunchCtx &c, double *u, int check_done) {
  if (c.eq != 1) return DG_ERR_UNSUPPORTED;
  const long cells = (long)c.geo.nx * c.geo.ny;
  dim3 grid((unsigned)std::max<long>(1, std::min<long>((cells + kBlock - 1) / kBlock, 4096)));
  auto go = [&](auto NN, auto D) {
    hipLaunchKernelGGL((k_positivity<decltype(NN)::value, decltype(D)::value>), grid, dim3(kBlock), 0, S(c), u, c.sc,
                       c.geo, check_done);
  };
  using I1 = std::integral_constant<int, 1>;
  using I2 = std::integral_constant<int, 2>;
  using I3 = std::integral_constant<int, 3>;
  if (c.dim == 1) {
    if (c.N == 1) go(I1{}, I1{}); else if (c.N == 2) go(I2{}, I1{}); else go(I3{}, I1{});
  } else {
    if (c.N == 1) go(I1{}, I2{}); else if (c.N == 2) go(I2{}, I2{}); else go(I3{}, I2{});
  }
  return check_launch();
}

int launch_set_tb(const LaunchCtx &c, double frac, double value) {
  hipLaunchKernelGGL(k_set_tb, dim3(1), dim3(64), 0, S(c), c.sc, frac, value);
  return check_launch();
}

int launch_dt_finalize(const LaunchCtx &c) {
  const bool nu = c.geo.hxa != nullptr;  // speeds are already per width
  hipLaunchKernelGGL(k_dt_finalize, dim3(1), dim3(64), 0, S(c), c.sc, c.dim, c.cfl, nu ? 1.0 : c.geo.hx,
                     nu ? 1.0 : c.geo.hy);
  return check_launch();
}

int launch_reset_counts(const LaunchCtx &c) {
  hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, S(c), c.sc, 0);
  return check_launch();
}

int launch_project(const LaunchCtx &c, const double *pv, int j0, int nrows, double *u) {
  const long work = (long)nrows * c.geo.nx * c.nv;
  dim3 grid((unsigned)((work + kBlock - 1) / kBlock));
  return dispatch(c, [&](auto D, auto E, auto NN) {
    hipLaunchKernelGGL((k_project<decltype(NN)::value, decltype(D)::value>), grid, dim3(kBlock), 0, S(c), pv, u,
                       c.geo, c.nv, j0, nrows);
  });
}


#endif  // DG_PART == 0

#if DG_PART == 2
int launch_mlp_features(const LaunchCtx &c, const double *u, float *f32, uint16_t *bf, int KP) {
  const long cells = (long)c.geo.nx * c.geo.ny;
  dim3 grid((unsigned)((cells + kBlock - 1) / kBlock));
  if (c.dim != 2) return DG_ERR_UNSUPPORTED;
  return dispatch(c, [&](auto D, auto E, auto NN) {
    constexpr int e = decltype(E)::value, n = decltype(NN)::value;
    hipLaunchKernelGGL((k_mlp_features<n, Phys<e, 2>::NV>), grid, dim3(kBlock), 0, S(c), u, c.geo, f32, bf, KP);
  });
}

template <typename F>
int kp_dispatch(int KP, F &&f) {
  switch (KP) {
    case 32: f(std::integral_constant<int, 32>{}); break;
    case 48: f(std::integral_constant<int, 48>{}); break;
    case 80: f(std::integral_constant<int, 80>{}); break;
    case 192: f(std::integral_constant<int, 192>{}); break;
    case 320: f(std::integral_constant<int, 320>{}); break;
    default: return DG_ERR_UNSUPPORTED;
  }
  return check_launch();
}

int mlp_layout(int F, int *KP, long *nmaster, long *nbf16) {
  if (F < 1) return DG_ERR_INVALID_ARG;
  MlpLayout lay{F, (F + 15) / 16 * 16};
  if (KP) *KP = lay.KP;
  if (nmaster) *nmaster = lay.nmaster();
  if (nbf16) *nbf16 = lay.nbf16();
  return DG_OK;
}

int launch_mlp_forward(const uint16_t *x, int n, int F, const uint16_t *W, const float *M, float *p, void *stream) {
  MlpLayout lay{F, (F + 15) / 16 * 16};
  if (n <= 0) return DG_OK;
  return kp_dispatch(lay.KP, [&](auto K) {
    hipLaunchKernelGGL((k_mlp_forward<decltype(K)::value>), dim3((n + 15) / 16), dim3(64), 0, (hipStream_t)stream, x,
                       n, W, M, lay, p);
  });
}

int launch_mlp_gradient(const uint16_t *x, const float *y, const float *w, int n, int F, const uint16_t *W,
                        const float *M, float *G, uint16_t *dh1, float *loss, void *stream) {
  MlpLayout lay{F, (F + 15) / 16 * 16};
  if (n <= 0) return DG_OK;
  const int ntiles = (n + 15) / 16;
  const int blocks = ntiles < 4096 ? ntiles : 4096;
  int rc = kp_dispatch(lay.KP, [&](auto K) {
    hipLaunchKernelGGL((k_mlp_train_tiles<decltype(K)::value>), dim3(blocks), dim3(64), 0, (hipStream_t)stream, x, y,
                       w, n, W, M, lay, G, dh1, loss);
  });
  if (rc) return rc;
  const int chunk = 1024;
  dim3 grid((lay.KP + 63) / 64, (n + chunk - 1) / chunk);
  return kp_dispatch(lay.KP, [&](auto K) {
    hipLaunchKernelGGL((k_mlp_wgrad1<decltype(K)::value>), grid, dim3(64), 0, (hipStream_t)stream, x, dh1, n, lay, G,
                       chunk);
  });
}

int launch_mlp_adam(float *M, float *m1, float *m2, float *G, uint16_t *W, int F, float lr, int step, void *stream) {
  MlpLayout lay{F, (F + 15) / 16 * 16};
  const long n = lay.nmaster() + lay.npad();
  hipLaunchKernelGGL(k_mlp_adam, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, (hipStream_t)stream, M,
                     m1, m2, G, W, lay, lr, step);
  return check_launch();
}

#endif  // DG_PART == 2

#if DG_PART == 3
// ---------------------------------------------------------------------------
// Batched execution launchers.
// ---------------------------------------------------------------------------
namespace {

template <typename F>
int order_dispatch(int order, F &&f) {
  switch (order) {
    case 1: f(std::integral_constant<int, 1>{}); break;
    case 2: f(std::integral_constant<int, 2>{}); break;
    case 3: f(std::integral_constant<int, 3>{}); break;
    default: return DG_ERR_UNSUPPORTED;
  }
  return check_launch();
}

}  // namespace

int batch_launch_decide(const BatchCtx &b, int finalize) {
  hipLaunchKernelGGL(k_batch_decide, dim3(1), dim3(1024), 0, (hipStream_t)b.stream, b.inst, b.n, b.queue, b.active,
                     finalize);
  return check_launch();
}

int batch_launch_speed(const BatchCtx &b, int order) {
  return order_dispatch(order, [&](auto NN) {
    hipLaunchKernelGGL((k_batch_speed<decltype(NN)::value>), dim3(b.grid_cap), dim3(64), 0, (hipStream_t)b.stream,
                       b.inst, b.queue + order);
  });
}

int batch_launch_stage(const BatchCtx &b, int order, int stage, int grid) {
  if (stage < 0 || stage > 3 || grid < 1) return DG_ERR_INVALID_ARG;
  return order_dispatch(order, [&](auto NN) {
    constexpr int n = decltype(NN)::value;
    const hipStream_t st = (hipStream_t)b.stream;
    const BatchQueue *q = b.queue + order;
    if (stage == 0) hipLaunchKernelGGL((k_batch_stage<n, 0>), dim3(grid), dim3(64), 0, st, b.inst, q);
    else if (stage == 1) hipLaunchKernelGGL((k_batch_stage<n, 1>), dim3(grid), dim3(64), 0, st, b.inst, q);
    else if (stage == 2) hipLaunchKernelGGL((k_batch_stage<n, 2>), dim3(grid), dim3(64), 0, st, b.inst, q);
    else hipLaunchKernelGGL((k_batch_stage<n, 3>), dim3(grid), dim3(64), 0, st, b.inst, q);
  });
}

int batch_launch_limit(const BatchCtx &b, int order, int slot) {
  if (slot < 0 || slot > 2) return DG_ERR_INVALID_ARG;
  if (b.indicator == DG_IND_LEARNED && !b.learned[order].W) return DG_ERR_INVALID_ARG;
  return order_dispatch(order, [&](auto NN) {
    constexpr int n = decltype(NN)::value;
    const hipStream_t st = (hipStream_t)b.stream;
    BatchQueue *q = b.queue + order;
    long long *list = b.list[order];
    const BatchLearned L = b.learned[order];
    auto go = [&](auto SL) {
      constexpr int s = decltype(SL)::value;
      if (b.indicator == DG_IND_LEARNED)
        hipLaunchKernelGGL((k_batch_learned<n, s>), dim3(b.grid_cap / 2), dim3(64 * lm_waves(n)), 0, st, b.inst, q,
                           list, L);
      else if (b.indicator == DG_IND_ALL)
        hipLaunchKernelGGL((k_batch_indicator<n, s, DG_IND_ALL>), dim3(4 * b.grid_cap), dim3(64), 0, st, b.inst, q,
                           list);
      else if (b.indicator == DG_IND_KXRCF)
        hipLaunchKernelGGL((k_batch_indicator<n, s, DG_IND_KXRCF>), dim3(4 * b.grid_cap), dim3(64), 0, st, b.inst,
                           q, list);
      else
        hipLaunchKernelGGL((k_batch_indicator<n, s, DG_IND_TVB>), dim3(4 * b.grid_cap), dim3(64), 0, st, b.inst, q,
                           list);
      if (b.limiter != DG_LIM_NONE) {
        if (b.limiter == DG_LIM_CSWENO_CHAR)
          hipLaunchKernelGGL((k_batch_csweno_char<n, s>), dim3(b.grid_cap), dim3(kBlock), 0, st, b.inst, q, list);
        else
          hipLaunchKernelGGL((k_batch_csweno<n, s>), dim3(b.grid_cap), dim3(kBlock), 0, st, b.inst, q, list);
        hipLaunchKernelGGL((k_batch_scatter<n, s>), dim3(b.grid_cap), dim3(kBlock), 0, st, b.inst, q, list);
      }
      if (b.positivity)
        hipLaunchKernelGGL((k_batch_positivity<n, s>), dim3(4 * b.grid_cap), dim3(64), 0, st, b.inst, q);
    };
    if (slot == 0) go(std::integral_constant<int, 0>{});
    else if (slot == 1) go(std::integral_constant<int, 1>{});
    else go(std::integral_constant<int, 2>{});
  });
}

#endif  // DG_PART == 3

}  // namespace dg
