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

#include <cmath>
#include <type_traits>

#include "dg_internal.h"

namespace dg {

__constant__ OrderTables c_tab[kMaxN + 1];

int upload_tables(const OrderTables *tabs) {
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
    double rho = u[0], vx = u[1] / rho, vy = u[2] / rho;
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
    double rho = u[0], vx = u[1] / rho, vy = u[2] / rho;
    double p = (g - 1.0) * (u[3] - 0.5 * rho * (vx * vx + vy * vy));
    bad |= !(rho > 0.0 && p > 0.0);
    return fabs(DIR == 0 ? vx : vy) + sqrt(g * p / rho);
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
// Cell access with boundary conditions: periodic wrap, or an even reflection
// of the adjacent cell (odd modes in the normal direction change sign).
// ---------------------------------------------------------------------------
struct CellIdx {
  long idx;
  bool fx, fy;
};

__device__ inline CellIdx map_cell(const Geometry &g, int i, int j) {
  CellIdx c;
  c.fx = c.fy = false;
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

template <int NP, int NM, int NV, int DIM>
__device__ inline void load_cell(const double *__restrict__ u, long plane, const CellIdx &c, double C[NV][NM]) {
#pragma unroll
  for (int v = 0; v < NV; ++v)
#pragma unroll
    for (int q = 0; q < NM; ++q) {
      int m = q % NP, n = q / NP;
      double s = u[(long)(v * NM + q) * plane + c.idx];
      bool flip = (c.fx && (m & 1)) != (DIM == 2 && c.fy && (n & 1));
      C[v][q] = flip ? -s : s;
    }
}

// ---------------------------------------------------------------------------
// Residual + SSP-RK3 stage.  STAGE 0: out = L(u).  1: u + dt L.  2: 3/4 un +
// 1/4 (u + dt L).  3: 1/3 un + 2/3 (u + dt L).
// ---------------------------------------------------------------------------
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
    double C[NV][NP], Nb[NV][NP], L[NV][NP];
    load_cell<NP, NP, NV, 1>(a.u, plane, map_cell(g, i, 0), C);
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
        double fw = g.rhx * T.wq[q] * f[v];
#pragma unroll
        for (int n = 0; n < NP; ++n) L[v][n] += fw * T.dbq[n][q];
      }
    }
    // faces
    double a_[NV], b_[NV], F[NV];
    load_cell<NP, NP, NV, 1>(a.u, plane, map_cell(g, i + 1, 0), Nb);
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
      for (int n = 0; n < NP; ++n) L[v][n] -= g.rhx * F[v] * T.bp[n];
    load_cell<NP, NP, NV, 1>(a.u, plane, map_cell(g, i - 1, 0), Nb);
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
      for (int n = 0; n < NP; ++n) L[v][n] += g.rhx * F[v] * T.bm[n];

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
        else r = a.un[k] / 3.0 + 2.0 * (C[v][n] + dt * L[v][n]) / 3.0;
        a.out[k] = r;
        if (n == 0) mean[v] = r * T.b0[0];
      }
    if (STAGE == 3 && a.want_speed) spd = P::template speed<0>(mean, g.gamma, bad);
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
    load_cell<NP, NM, NV, 2>(a.u, plane, map_cell(g, i, j), C);
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
          Fx[v][qx] = w * g.rhx * f[v];
          Gy[v][qx] = w * g.rhy * gg[v];
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
      load_cell<NP, NM, NV, 2>(a.u, plane, map_cell(g, i + di, j + dj), Nb);
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
      const double sc = face < 2 ? g.rhx : g.rhy;
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
        else r = a.un[k] / 3.0 + 2.0 * (C[v][q] + dt * L[v][q]) / 3.0;
        a.out[k] = r;
        if (q == 0) mean[v] = r * (T.b0[0] * T.b0[0]);
      }
    if (STAGE == 3 && a.want_speed) {
      spx = P::template speed<0>(mean, g.gamma, bad);
      spy = P::template speed<1>(mean, g.gamma, bad);
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
// Spectral radius of cell means (first step of a dg_step call, dg_cfl_dt).
// ---------------------------------------------------------------------------
template <int N, int EQ, int DIM>
__global__ __launch_bounds__(kBlock) void k_speed(const double *__restrict__ u, DevScalars *sc, Geometry g) {
  constexpr int NP = N + 1, NM = DIM == 1 ? NP : NP * NP, NV = Phys<EQ, DIM>::NV;
  using P = Phys<EQ, DIM>;
  const OrderTables &T = c_tab[N];
  const long plane = (long)g.nx * g.ny;
  const long cell = (long)blockIdx.x * blockDim.x + threadIdx.x;
  double sx = 0.0, sy = 0.0;
  bool bad = false;
  if (cell < plane) {
    const double k0 = DIM == 1 ? T.b0[0] : T.b0[0] * T.b0[0];
    double m[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) m[v] = u[(long)(v * NM) * plane + cell] * k0;
    sx = P::template speed<0>(m, g.gamma, bad);
    if (DIM == 2) sy = P::template speed<1>(m, g.gamma, bad);
  }
  if (bad) atomicOr(&sc->status, 1);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    sx = fmax(sx, __shfl_xor(sx, o));
    sy = fmax(sy, __shfl_xor(sy, o));
  }
  if (__lane_id() == 0) {
    atomicMax(&sc->smax[0], (unsigned long long)__double_as_longlong(sx));
    if (DIM == 2) atomicMax(&sc->smax[1], (unsigned long long)__double_as_longlong(sy));
  }
}

// One thread: time step of the CFL rule (or the fixed one), clipped at
// t_end; marks the run done; clears the per-step accumulators.
__global__ void k_dt_finalize(DevScalars *sc, int dim, double cfl, double hx, double hy) {
  if (threadIdx.x != 0 || sc->done) return;
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
  sc->t = last ? sc->t_end : sc->t + dt;
  sc->steps += 1;
  sc->smax[0] = 0ull;
  sc->smax[1] = 0ull;
  sc->count[0] = sc->count[1] = sc->count[2] = 0;
}

__global__ void k_reset(DevScalars *sc, int what) {
  if (threadIdx.x != 0) return;
  if (what == 0) {  // standalone limiter count
    sc->count[3] = 0;
  } else {  // speed accumulators
    sc->smax[0] = 0ull;
    sc->smax[1] = 0ull;
  }
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

template <int N, int EQ, int DIM>
__global__ __launch_bounds__(kBlock) void k_indicator(LimitArgs a) {
  constexpr int NP = N + 1, NM = DIM == 1 ? NP : NP * NP, NV = Phys<EQ, DIM>::NV;
  const OrderTables &T = c_tab[N];
  const Geometry &g = a.geo;
  if (a.check_done && a.sc->done) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = DIM == 1 ? 0 : blockIdx.y * blockDim.y + threadIdx.y;
  const long plane = (long)g.nx * g.ny;
  const bool active = i < g.nx && j < g.ny;
  const long cell = (long)j * g.nx + i;
  bool flag = false;
  double mg = INFINITY;
  if (active) {
    if (a.ovr) {
      flag = a.ovr[cell] != 0;
    } else if (a.mode == DG_IND_ALL) {
      flag = true;
    } else {
      const double k0 = DIM == 1 ? T.b0[0] : T.b0[0] * T.b0[0];
      double C[NV][NM];
      load_cell<NP, NM, NV, DIM>(a.u, plane, map_cell(g, i, j), C);
#pragma unroll
      for (int dir = 0; dir < DIM; ++dir) {
        const double Mh2 = dir == 0 ? g.tvb_Mx : g.tvb_My;
        const CellIdx cp = map_cell(g, i + (dir == 0), j + (dir == 1));
        const CellIdx cm = map_cell(g, i - (dir == 0), j - (dir == 1));
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          double mean = C[v][0] * k0;
          double mp = a.u[(long)(v * NM) * plane + cp.idx] * k0;
          double mm = a.u[(long)(v * NM) * plane + cm.idx] * k0;
          double up = 0.0, um = 0.0;
#pragma unroll
          for (int q = 0; q < NM; ++q) {
            int m = q % NP, n = q / NP;
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
            up += C[v][q] * bu;
            um += C[v][q] * bd;
          }
          double dp = mp - mean, dm = mean - mm;
          flag |= tvb_test(up - mean, dp, dm, Mh2, mg);
          flag |= tvb_test(mean - um, dp, dm, Mh2, mg);
        }
      }
    }
    if (a.flags) a.flags[cell] = flag ? 1 : 0;
    if (a.margin) a.margin[cell] = mg;
  }
  unsigned long long ballot = __ballot(flag);
  if (ballot) {
    const int lane = __lane_id();
    const int leader = __ffsll((long long)ballot) - 1;
    int base = 0;
    if (lane == leader) {
      base = atomicAdd(a.count, __popcll(ballot));
      atomicAdd(&a.sc->troubled_total, (unsigned long long)__popcll(ballot));
    }
    base = __shfl(base, leader);
    if (flag) a.list[base + __popcll(ballot & ((1ull << lane) - 1ull))] = (int32_t)cell;
  }
}

// ---------------------------------------------------------------------------
// CSWENO (Section 3).  One thread per (troubled cell, variable).
// ---------------------------------------------------------------------------

// WENO values at the Step-1 points of one row of 2N+1 stencil means.  The
// row is taken relative to the troubled cell's mean a[N] (the smoothness
// indicators only see derivatives and the normalised weights sum to one), so
// the quadratic forms do not cancel O(1) means.
template <int N>
__device__ inline void weno_row(const OrderTables &T, const double *a_in, double *out, double eps, bool raw) {
  constexpr int NP = N + 1, NG = num_points<N>(), NS = 2 * N + 1;
  const double a0 = a_in[N];
  double a[NS];
#pragma unroll
  for (int k = 0; k < NS; ++k) a[k] = a_in[k] - a0;
  double d[NP];
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
    double e = eps + beta;
    d[i] = 1.0 / (e * e);
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
      out[G] = a0 + (T.sp[G] * (up / wp) - T.sm[G] * (um / wm));
    } else {
      double ws = 0.0, us = 0.0;
#pragma unroll
      for (int i = 0; i < NP; ++i) {
        double x = T.gam[G][i] * d[i];
        ws += x;
        us += x * p[i];
      }
      out[G] = a0 + us / ws;
    }
  }
}

// mean of psi_n over stencil interval k (0..2N) of the compact stencil
template <int N>
__device__ inline double interval_mean(const OrderTables &T, int k, int n) {
  if (k == N) return n == 0 ? T.b0[0] : 0.0;
  return T.sub[k < N ? k : k - N - 1][n];
}

template <int N, int EQ, int DIM>
__global__ __launch_bounds__(kBlock) void k_csweno(LimitArgs a) {
  constexpr int NP = N + 1, NM = DIM == 1 ? NP : NP * NP, NV = Phys<EQ, DIM>::NV;
  constexpr int NS = 2 * N + 1, NG = num_points<N>();
  const OrderTables &T = c_tab[N];
  const Geometry &g = a.geo;
  if (a.check_done && a.sc->done) return;
  const long plane = (long)g.nx * g.ny;
  const long total = (long)(*a.count) * NV;
  const bool raw = g.negw_raw != 0;
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
    const int v = (int)(t % NV);
    const long cell = a.list[t / NV];
    const int i = (int)(cell % g.nx), j = (int)(cell / g.nx);
    if (DIM == 1) {
      double st[NS];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        CellIdx ci = map_cell(g, i + c - 1, 0);
        double md[NP];
#pragma unroll
        for (int n = 0; n < NP; ++n) {
          double s = a.u[(long)(v * NM + n) * plane + ci.idx];
          md[n] = (ci.fx && (n & 1)) ? -s : s;
        }
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
      weno_row<N>(T, st, uG, g.eps, raw);
#pragma unroll
      for (int n = 1; n < NP; ++n) {
        double s = 0.0;
#pragma unroll
        for (int G = 0; G < NG; ++G) s += T.wg[G] * uG[G] * T.bg[n][G];
        a.side[(long)(v * NM + n) * plane + cell] = s;
      }
    } else {
      // (2N+1)^2 sub-rectangle means of the 3x3 block, [iy][ix]
      double st[NS][NS];
#pragma unroll
      for (int cy = 0; cy < 3; ++cy)
#pragma unroll
        for (int cx = 0; cx < 3; ++cx) {
          CellIdx ci = map_cell(g, i + cx - 1, j + cy - 1);
          double md[NM];
#pragma unroll
          for (int q = 0; q < NM; ++q) {
            int m = q % NP, n = q / NP;
            double s = a.u[(long)(v * NM + q) * plane + ci.idx];
            bool flip = (ci.fx && (m & 1)) != (ci.fy && (n & 1));
            md[q] = flip ? -s : s;
          }
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
      // x-sweeps: y-interval means at the x-points
      double vy[NG][NS];
#pragma unroll
      for (int iy = 0; iy < NS; ++iy) {
        double r[NG];
        weno_row<N>(T, st[iy], r, g.eps, raw);
#pragma unroll
        for (int G = 0; G < NG; ++G) vy[G][iy] = r[G];
      }
      // y-sweeps at every x-point, then the tensor projection
      double s[NG][NP];  // s[G][n] = sum_H wg[H] u(G,H) psi_n(y_H)
#pragma unroll
      for (int G = 0; G < NG; ++G) {
        double u[NG];
        weno_row<N>(T, vy[G], u, g.eps, raw);
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
        a.side[(long)(v * NM + q) * plane + cell] = acc;
      }
    }
  }
}

template <int NM, int NV>
__global__ __launch_bounds__(kBlock) void k_scatter(LimitArgs a, double *dst) {
  if (a.check_done && a.sc->done) return;
  const long plane = (long)a.geo.nx * a.geo.ny;
  const long total = (long)(*a.count) * NV * (NM - 1);
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
    const int q = 1 + (int)(t % (NM - 1));
    const int v = (int)((t / (NM - 1)) % NV);
    const long cell = a.list[t / ((NM - 1) * NV)];
    const long k = (long)(v * NM + q) * plane + cell;
    dst[k] = a.side[k];
  }
}

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

template <int D, int E, int NN, int STAGE>
void stage_launch(const LaunchCtx &c, const StageArgs &a) {
  dim3 block, grid = cell_grid(c, block);
  if (D == 1) hipLaunchKernelGGL((k_stage_1d<NN, E, STAGE>), grid, block, 0, S(c), a);
  else hipLaunchKernelGGL((k_stage_2d<NN, E, STAGE>), grid, block, 0, S(c), a);
}

}  // namespace

int launch_residual(const LaunchCtx &c, const double *u, double *out) {
  StageArgs a{u, nullptr, out, c.sc, c.geo, 0};
  return dispatch(c, [&](auto D, auto E, auto NN) {
    stage_launch<decltype(D)::value, decltype(E)::value, decltype(NN)::value, 0>(c, a);
  });
}

int launch_stage(const LaunchCtx &c, int stage, const double *u, const double *un, double *out, bool want_speed) {
  StageArgs a{u, un, out, c.sc, c.geo, want_speed ? 1 : 0};
  return dispatch(c, [&](auto D, auto E, auto NN) {
    constexpr int d = decltype(D)::value, e = decltype(E)::value, n = decltype(NN)::value;
    if (stage == 1) stage_launch<d, e, n, 1>(c, a);
    else if (stage == 2) stage_launch<d, e, n, 2>(c, a);
    else stage_launch<d, e, n, 3>(c, a);
  });
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
  return dispatch(c, [&](auto D, auto E, auto NN) {
    constexpr int d = decltype(D)::value, e = decltype(E)::value, n = decltype(NN)::value;
    constexpr int NM = d == 1 ? n + 1 : (n + 1) * (n + 1);
    constexpr int NV = Phys<e, d>::NV;
    dim3 block, grid = cell_grid(c, block);
    hipLaunchKernelGGL((k_indicator<n, e, d>), grid, block, 0, S(c), a);
    if (c.limiter == DG_LIM_CSWENO) {
      hipLaunchKernelGGL((k_csweno<n, e, d>), dim3(c.grid_cap), dim3(kBlock), 0, S(c), a);
      hipLaunchKernelGGL((k_scatter<NM, NV>), dim3(c.grid_cap), dim3(kBlock), 0, S(c), a, u);
    }
  });
}

int launch_speed(const LaunchCtx &c, const double *u) {
  hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, S(c), c.sc, 1);
  const long cells = (long)c.geo.nx * c.geo.ny;
  dim3 grid((unsigned)((cells + kBlock - 1) / kBlock));
  return dispatch(c, [&](auto D, auto E, auto NN) {
    hipLaunchKernelGGL((k_speed<decltype(NN)::value, decltype(E)::value, decltype(D)::value>), grid, dim3(kBlock),
                       0, S(c), u, c.sc, c.geo);
  });
}

int launch_dt_finalize(const LaunchCtx &c) {
  hipLaunchKernelGGL(k_dt_finalize, dim3(1), dim3(64), 0, S(c), c.sc, c.dim, c.cfl, c.geo.hx, c.geo.hy);
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

}  // namespace dg
