/*
 * dg_oracle.c -- plain FP64 CPU reference of the RKDG step with the compact
 * subcell WENO (CSWENO) limiter of Kochi & Ramakrishna, "A compact subcell
 * WENO limiting strategy using immediate neighbors for Runge-Kutta
 * Discontinuous Galerkin Methods" (arXiv 1904.11147).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle the HIP path is checked
 * against.  Only the tests, the smoke check and the benchmark's CPU-baseline
 * leg may load it; the product library never does.  It shares no source,
 * header, table or generator with the HIP path: every coefficient it uses is
 * derived here, at run time, from the definitions in the paper.
 *
 * Style: straightforward loops, no blocking or fusion, double precision,
 * built without fast-math and without FMA contraction.  Where the paper is
 * silent or garbled the reading taken is stated at the point of use.
 *
 * Layout of a state: U[v][q][j][i] (i fastest), q = m + (N+1)*n where m is
 * the x-degree and n the y-degree of the tensor Legendre mode (1D: q = m).
 *
 * Parity pins: quadrature, P2 tables, P1 tables, residual, TVB and limiter
 * invariants are pinned by tests/test_oracle_*.py; the reflective wall,
 * inflow and switching boundary sides by mirror images, periodic images and
 * stage-time checks (test_oracle_boundary.py); the positivity scaling by
 * bisection on its defining property (test_oracle_positivity.py); the
 * non-uniform mesh tables, residual, limiter and design order
 * (test_oracle_nonuniform.py).  The P3 treatment of the
 * negative linear weights is "parity unpinned" (the paper does not say what
 * it does with them; see orc_weno_point).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAXN 3
#define ORC_MAXP 4  /* N+1 */
#define ORC_MAXS 7  /* 2N+1 stencil cells */
#define ORC_MAXG 4  /* reconstruction points */
#define ORC_MAXV 4  /* variables */
#define ORC_MAXM 16 /* modes per cell */
#define ORC_MAXPQ 10 /* projection nodes per direction: 2 panels x (N+2) */

enum { ORC_BURGERS = 0, ORC_EULER = 1 };
enum { ORC_BC_PERIODIC = 0, ORC_BC_TRANSMISSIVE = 1, ORC_BC_REFLECTIVE = 2, ORC_BC_INFLOW = 3 };
enum { ORC_LIM_NONE = 0, ORC_LIM_CSWENO = 1, ORC_LIM_CSWENO_CHAR = 2 };
enum { ORC_IND_TVB = 0, ORC_IND_ALL = 1, ORC_IND_KXRCF = 3 };
enum { ORC_NEGW_SPLIT = 0, ORC_NEGW_RAW = 1 };
enum { ORC_OK = 0, ORC_ERR_ARG = -1, ORC_ERR_NONPHYSICAL = -5, ORC_ERR_TABLE = -6 };

typedef struct {
  int32_t dim, equation, order, nx, ny;
  int32_t bc[4]; /* W, E, S, N */
  int32_t limiter, indicator, negw_mode;
  double gamma, x0, x1, y0, y1, tvb_M, weno_eps, cfl;
  /* Positivity-preserving scaling of Zhang & Shu (the component the paper
   * adds for the double Mach reflection, Example 11), after the limiter. */
  int32_t positivity;
  /* South/north sides may switch kind along x: kind bc[s] where the ghost
   * cell's centre x < a + b t, kind bc_beyond[s] from there on (-1: no
   * switch; west/east sides never switch). */
  int32_t bc_beyond[4];
  int32_t pad_;
  double bc_switch[4][2];   /* [side] {a, b} */
  double bc_state[4][2][4]; /* conserved ghost state of an inflow part [side][before, beyond][var] */
  double time;              /* time of the boundary data (orc_step: the step's start time) */
  /* Non-uniform tensor-product meshes: node coordinates x_0 < ... < x_nx
   * (and y_0 < ... < y_ny in 2D), or NULL for the uniform mesh on [x0,x1]. */
  const double *xn, *yn;
} orc_config;

/* ------------------------------------------------------------------------ */
/* Section 2: orthonormal Legendre basis on the reference cell r in [-1,1]. */
/* ------------------------------------------------------------------------ */

static double leg(int n, double r) {
  /* Bonnet recurrence (k+1) P_{k+1} = (2k+1) r P_k - k P_{k-1}. */
  if (n == 0) return 1.0;
  double p0 = 1.0, p1 = r;
  for (int k = 1; k < n; ++k) {
    double p2 = ((2.0 * k + 1.0) * r * p1 - k * p0) / (k + 1.0);
    p0 = p1;
    p1 = p2;
  }
  return p1;
}

static double dleg(int n, double r) {
  /* P_n' = sum over k = n-1, n-3, ... >= 0 of (2k+1) P_k. */
  double s = 0.0;
  for (int k = n - 1; k >= 0; k -= 2) s += (2.0 * k + 1.0) * leg(k, r);
  return s;
}

static double psi(int n, double r) { return sqrt((2.0 * n + 1.0) / 2.0) * leg(n, r); }
static double dpsi(int n, double r) { return sqrt((2.0 * n + 1.0) / 2.0) * dleg(n, r); }

/* n-point Gauss-Legendre rule on [-1,1], ascending nodes, by Newton on P_n. */
static void gauss_rule(int n, double *x, double *w) {
  for (int i = 0; i < n; ++i) {
    double r = -cos(M_PI * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double d = leg(n, r) / dleg(n, r);
      r -= d;
      if (fabs(d) < 1e-17) break;
    }
    double dp = dleg(n, r);
    x[i] = r;
    w[i] = 2.0 / ((1.0 - r * r) * dp * dp);
  }
}

/* n-point Gauss-Lobatto rule: end points and the roots of P_{n-1}'. */
static void gauss_lobatto_rule(int n, double *x, double *w) {
  x[0] = -1.0;
  x[n - 1] = 1.0;
  for (int i = 1; i < n - 1; ++i) {
    double r = -cos(M_PI * i / (n - 1.0));
    for (int it = 0; it < 100; ++it) {
      /* Legendre ODE: (1-r^2) P'' = 2 r P' - k(k+1) P with k = n-1. */
      int k = n - 1;
      double f = dleg(k, r);
      double fp = (2.0 * r * dleg(k, r) - k * (k + 1.0) * leg(k, r)) / (1.0 - r * r);
      double d = f / fp;
      r -= d;
      if (fabs(d) < 1e-17) break;
    }
    x[i] = r;
  }
  for (int i = 0; i < n; ++i) {
    double p = leg(n - 1, x[i]);
    w[i] = 2.0 / (n * (n - 1.0) * p * p);
  }
}

/* ------------------------------------------------------------------------ */
/* Small dense linear algebra (Gaussian elimination with partial pivoting). */
/* ------------------------------------------------------------------------ */

static int solve_dense(int n, double *A, double *b) { /* A row-major n x n, b overwritten */
  for (int c = 0; c < n; ++c) {
    int p = c;
    for (int r = c + 1; r < n; ++r)
      if (fabs(A[r * n + c]) > fabs(A[p * n + c])) p = r;
    if (A[p * n + c] == 0.0) return -1;
    if (p != c) {
      for (int k = 0; k < n; ++k) {
        double t = A[c * n + k];
        A[c * n + k] = A[p * n + k];
        A[p * n + k] = t;
      }
      double t = b[c];
      b[c] = b[p];
      b[p] = t;
    }
    for (int r = c + 1; r < n; ++r) {
      double f = A[r * n + c] / A[c * n + c];
      for (int k = c; k < n; ++k) A[r * n + k] -= f * A[c * n + k];
      b[r] -= f * b[c];
    }
  }
  for (int r = n - 1; r >= 0; --r) {
    double s = b[r];
    for (int k = r + 1; k < n; ++k) s -= A[r * n + k] * b[k];
    b[r] = s / A[r * n + r];
  }
  return 0;
}

static int solve_dense_ld(int n, long double *A, long double *b) { /* as solve_dense, in long double */
  for (int c = 0; c < n; ++c) {
    int p = c;
    for (int r = c + 1; r < n; ++r)
      if (fabsl(A[r * n + c]) > fabsl(A[p * n + c])) p = r;
    if (A[p * n + c] == 0.0L) return -1;
    if (p != c) {
      for (int k = 0; k < n; ++k) {
        long double t = A[c * n + k];
        A[c * n + k] = A[p * n + k];
        A[p * n + k] = t;
      }
      long double t = b[c];
      b[c] = b[p];
      b[p] = t;
    }
    for (int r = c + 1; r < n; ++r) {
      long double f = A[r * n + c] / A[c * n + c];
      for (int k = c; k < n; ++k) A[r * n + k] -= f * A[c * n + k];
      b[r] -= f * b[c];
    }
  }
  for (int r = n - 1; r >= 0; --r) {
    long double s = b[r];
    for (int k = r + 1; k < n; ++k) s -= A[r * n + k] * b[k];
    b[r] = s / A[r * n + r];
  }
  return 0;
}

static long double mono_mean_ld(int d, long double a, long double b) {
  return (powl(b, d + 1) - powl(a, d + 1)) / ((d + 1.0L) * (b - a));
}

/* Mean of xi^d over [a,b]. */
static double mono_mean(int d, double a, double b) {
  return (pow(b, d + 1) - pow(a, d + 1)) / ((d + 1.0) * (b - a));
}

/* Integral of xi^d over the troubled cell [-1/2, 1/2]. */
static double mono_int_centre(int d) { return (pow(0.5, d + 1) - pow(-0.5, d + 1)) / (d + 1.0); }

/* ------------------------------------------------------------------------ */
/* Section 3: CSWENO tables, derived in the order of steps 1-3.              */
/* ------------------------------------------------------------------------ */

typedef struct {
  int N, np;
  double rq[ORC_MAXP], wq[ORC_MAXP]; /* (N+1)-point Gauss: volume and edge rule */
  int ng;
  double rg[ORC_MAXG], wg[ORC_MAXG]; /* reconstruction rule (step 1) */
  double cl[ORC_MAXS], cr[ORC_MAXS]; /* stencil cells in xi = (x - x_j)/h_j */
  double Ainv[ORC_MAXP][ORC_MAXP][ORC_MAXP]; /* [i][d][k]: coefficient d of p_i from average k of S_i */
  double gam[ORC_MAXG][ORC_MAXP];            /* linear weights (step 3) */
  double gam_resid;                          /* max residual of the linear-weight system */
  int split[ORC_MAXG];                       /* point has a negative linear weight */
  double sub[ORC_MAXP][ORC_MAXP];            /* [k][n]: mean of psi_n over subcell k of [-1,1] */
  int npq;
  double rpq[ORC_MAXPQ], wpq[ORC_MAXPQ]; /* projection rule for initial data */
  /* basis values at the points the method evaluates: [n][point] */
  double bq[ORC_MAXP][ORC_MAXP], dbq[ORC_MAXP][ORC_MAXP]; /* psi_n, psi_n' at rq */
  double bm[ORC_MAXP], bp[ORC_MAXP], b0[ORC_MAXP];        /* psi_n(-1), psi_n(+1), psi_n(0) */
  double bg[ORC_MAXP][ORC_MAXG];                          /* psi_n at rg */
  double bpq[ORC_MAXP][ORC_MAXPQ];                        /* psi_n at rpq */
} orc_tables;

static orc_tables g_tab[ORC_MAXN + 1];
static int g_tab_ready[ORC_MAXN + 1];

/* Tables of order N for a troubled cell whose left and right neighbours are
 * rl and rr times as wide as itself (1, 1 on a uniform mesh). */
static int build_tables_into(orc_tables *T, int N, double rl, double rr) {
  memset(T, 0, sizeof(*T));
  T->N = N;
  T->np = N + 1;
  gauss_rule(N + 1, T->rq, T->wq);

  /* Step 1: a rule exact to the order the reconstruction needs.  P1: 2-point
   * Gauss; P2: 4-point Gauss-Lobatto; P3: 4-point Gauss. */
  if (N == 1) {
    T->ng = 2;
    gauss_rule(2, T->rg, T->wg);
  } else if (N == 2) {
    T->ng = 4;
    gauss_lobatto_rule(4, T->rg, T->wg);
  } else {
    T->ng = 4;
    gauss_rule(4, T->rg, T->wg);
  }

  /* Compact stencil: each immediate neighbour is cut into N equal subcells;
   * the troubled cell stays whole (for N = 1 the neighbours stay whole too).
   * Cells are numbered left to right. */
  int ns = 2 * N + 1;
  for (int k = 0; k < N; ++k) {
    T->cl[k] = (-0.5 - rl) + k * rl / N;
    T->cr[k] = (-0.5 - rl) + (k + 1) * rl / N;
    T->cl[N + 1 + k] = 0.5 + k * rr / N;
    T->cr[N + 1 + k] = 0.5 + (k + 1) * rr / N;
  }
  T->cl[N] = -0.5;
  T->cr[N] = 0.5;

  /* Step 2: p_i of degree N whose means on the N+1 cells of S_i = cells
   * i..i+N equal the data, and Q of degree 2N on all 2N+1 cells.  The small
   * systems are solved in long double (the moment matrices of the 7-cell P3
   * stencil lose about three digits), the results rounded once. */
  long double Ainv[ORC_MAXP][ORC_MAXP][ORC_MAXP];
  for (int i = 0; i <= N; ++i) {
    for (int k = 0; k <= N; ++k) {
      long double A[ORC_MAXP * ORC_MAXP], e[ORC_MAXP];
      for (int r = 0; r <= N; ++r)
        for (int d = 0; d <= N; ++d) A[r * (N + 1) + d] = mono_mean_ld(d, T->cl[i + r], T->cr[i + r]);
      for (int r = 0; r <= N; ++r) e[r] = (r == k) ? 1.0L : 0.0L;
      if (solve_dense_ld(N + 1, A, e)) return ORC_ERR_TABLE;
      for (int d = 0; d <= N; ++d) {
        Ainv[i][d][k] = e[d];
        T->Ainv[i][d][k] = (double)e[d];
      }
    }
  }
  long double AQinv[ORC_MAXS][ORC_MAXS];
  for (int k = 0; k < ns; ++k) {
    long double A[ORC_MAXS * ORC_MAXS], e[ORC_MAXS];
    for (int r = 0; r < ns; ++r)
      for (int d = 0; d < ns; ++d) A[r * ns + d] = mono_mean_ld(d, T->cl[r], T->cr[r]);
    for (int r = 0; r < ns; ++r) e[r] = (r == k) ? 1.0L : 0.0L;
    if (solve_dense_ld(ns, A, e)) return ORC_ERR_TABLE;
    for (int d = 0; d < ns; ++d) AQinv[d][k] = e[d];
  }

  /* Step 3: linear weights with Q(x_G) = sum_i gamma_i p_i(x_G) for every
   * data vector, i.e. 2N+1 equations in N+1 unknowns, solved in the least
   * squares sense (normal equations, long double); the residual is recorded
   * and must vanish. */
  T->gam_resid = 0.0;
  for (int G = 0; G < T->ng; ++G) {
    long double xi = 0.5L * T->rg[G];
    long double M[ORC_MAXS][ORC_MAXP], rhs[ORC_MAXS];
    for (int k = 0; k < ns; ++k) {
      long double q = 0.0L;
      for (int d = 0; d < ns; ++d) q += AQinv[d][k] * powl(xi, d);
      rhs[k] = q;
      for (int i = 0; i <= N; ++i) {
        long double t = 0.0L;
        if (k >= i && k <= i + N)
          for (int d = 0; d <= N; ++d) t += Ainv[i][d][k - i] * powl(xi, d);
        M[k][i] = t;
      }
    }
    long double NtN[ORC_MAXP * ORC_MAXP], Ntb[ORC_MAXP];
    for (int a = 0; a <= N; ++a) {
      Ntb[a] = 0.0L;
      for (int k = 0; k < ns; ++k) Ntb[a] += M[k][a] * rhs[k];
      for (int b = 0; b <= N; ++b) {
        long double s2 = 0.0L;
        for (int k = 0; k < ns; ++k) s2 += M[k][a] * M[k][b];
        NtN[a * (N + 1) + b] = s2;
      }
    }
    if (solve_dense_ld(N + 1, NtN, Ntb)) return ORC_ERR_TABLE;
    int neg = 0;
    for (int i = 0; i <= N; ++i) {
      T->gam[G][i] = (double)Ntb[i];
      if (Ntb[i] < 0.0L) neg = 1;
    }
    T->split[G] = neg;
    for (int k = 0; k < ns; ++k) {
      long double s2 = -rhs[k];
      for (int i = 0; i <= N; ++i) s2 += M[k][i] * Ntb[i];
      if (fabsl(s2) > T->gam_resid) T->gam_resid = (double)fabsl(s2);
    }
  }
  if (T->gam_resid > 1e-10) return ORC_ERR_TABLE;

  /* Means of psi_n over the N equal subcells of [-1,1] (N+1-point Gauss on
   * each subcell integrates psi_n exactly). */
  for (int k = 0; k < N; ++k) {
    double a = -1.0 + 2.0 * k / N, b = -1.0 + 2.0 * (k + 1) / N;
    for (int n = 0; n <= N; ++n) {
      double s = 0.0;
      for (int q = 0; q <= N; ++q) {
        double r = 0.5 * (a + b) + 0.5 * (b - a) * T->rq[q];
        s += 0.5 * T->wq[q] * psi(n, r);
      }
      T->sub[k][n] = s; /* (1/(b-a)) * (b-a)/2 * sum w psi */
    }
  }

  /* Projection of initial data: two panels [-1,0] and [0,1], each with an
   * (N+2)-point Gauss rule (exact to degree 2N+3 per panel), so a jump at a
   * cell face or a cell centre is integrated piecewise. */
  double px[ORC_MAXPQ], pw[ORC_MAXPQ];
  int m = N + 2;
  gauss_rule(m, px, pw);
  T->npq = 2 * m;
  for (int k = 0; k < m; ++k) {
    T->rpq[k] = -0.5 + 0.5 * px[k];
    T->wpq[k] = 0.5 * pw[k];
    T->rpq[m + k] = 0.5 + 0.5 * px[k];
    T->wpq[m + k] = 0.5 * pw[k];
  }
  for (int n = 0; n <= N; ++n) {
    for (int q = 0; q <= N; ++q) {
      T->bq[n][q] = psi(n, T->rq[q]);
      T->dbq[n][q] = dpsi(n, T->rq[q]);
    }
    T->bm[n] = psi(n, -1.0);
    T->bp[n] = psi(n, 1.0);
    T->b0[n] = psi(n, 0.0);
    for (int G = 0; G < T->ng; ++G) T->bg[n][G] = psi(n, T->rg[G]);
    for (int a = 0; a < T->npq; ++a) T->bpq[n][a] = psi(n, T->rpq[a]);
  }
  return ORC_OK;
}

static int build_tables(int N) {
  int rc = build_tables_into(&g_tab[N], N, 1.0, 1.0);
  if (rc == ORC_OK) g_tab_ready[N] = 1;
  return rc;
}

static const orc_tables *tables(int N) {
  if (N < 1 || N > ORC_MAXN) return NULL;
  if (!g_tab_ready[N] && build_tables(N) != ORC_OK) return NULL;
  return &g_tab[N];
}

/* ------------------------------------------------------------------------ */
/* Steps 2, 4, 5: one WENO reconstruction at point G from the 2N+1 stencil   */
/* means a[] (left to right).                                               */
/* ------------------------------------------------------------------------ */

static void small_poly(const orc_tables *T, int i, const double *a, double *c) {
  for (int d = 0; d <= T->N; ++d) {
    double s = 0.0;
    for (int k = 0; k <= T->N; ++k) s += T->Ainv[i][d][k] * a[i + k];
    c[d] = s;
  }
}

/* beta_i = sum_{l=1..N} int_{I_j} dx^{2l-1} (d^l p_i / dx^l)^2 dx, which in
 * the unit variable xi is sum_l int_{-1/2}^{1/2} (p_i^{(l)}(xi))^2 dxi. */
static double smoothness(int N, const double *c) {
  double beta = 0.0;
  for (int l = 1; l <= N; ++l) {
    double e[ORC_MAXP];
    int ne = N + 1 - l;
    for (int d = 0; d < ne; ++d) {
      double f = 1.0;
      for (int t = 0; t < l; ++t) f *= (double)(d + l - t);
      e[d] = c[d + l] * f;
    }
    for (int d1 = 0; d1 < ne; ++d1)
      for (int d2 = 0; d2 < ne; ++d2) beta += e[d1] * e[d2] * mono_int_centre(d1 + d2);
  }
  return beta;
}

static double orc_weno_point(const orc_tables *T, int G, const double *a_in, double eps, int negw_mode) {
  int N = T->N;
  double xi = 0.5 * T->rg[G];
  double p[ORC_MAXP], beta[ORC_MAXP];
  /* The reconstruction is taken on the means relative to the troubled cell's
   * mean a0: the derivatives in beta do not see the shift, and since the
   * normalised weights sum to one, u_G = a0 + (reconstruction of a - a0).
   * This is the same definition, without the cancellation of O(1) means in
   * the smoothness quadratic forms. */
  const double a0 = a_in[N];
  double a[ORC_MAXS];
  for (int k = 0; k < 2 * N + 1; ++k) a[k] = a_in[k] - a0;
  for (int i = 0; i <= N; ++i) {
    double c[ORC_MAXP];
    small_poly(T, i, a, c);
    double v = 0.0;
    for (int d = 0; d <= N; ++d) v += c[d] * pow(xi, d);
    p[i] = v;
    beta[i] = smoothness(N, c);
  }
  if (!T->split[G] || negw_mode == ORC_NEGW_RAW) {
    /* Step 5 with the nonlinear weights normalised to sum to one:
     * wbar_i = gamma_i / (eps + beta_i)^2. */
    double wsum = 0.0, usum = 0.0;
    for (int i = 0; i <= N; ++i) {
      double wb = T->gam[G][i] / ((eps + beta[i]) * (eps + beta[i]));
      wsum += wb;
      usum += wb * p[i];
    }
    return a0 + usum / wsum;
  }
  /* A point with a negative linear weight (P3 only): the paper is silent.
   * Reading taken: split the linear weights into a positive and a negative
   * group with theta = 3 (Shi, Hu and Shu, J. Comput. Phys. 175 (2002)),
   * form nonlinear weights within each group and combine
   * u = sigma+ u+ - sigma- u-.  Parity unpinned against the paper. */
  const double theta = 3.0;
  double gp[ORC_MAXP], gm[ORC_MAXP], sp = 0.0, sm = 0.0;
  for (int i = 0; i <= N; ++i) {
    double g = T->gam[G][i];
    gp[i] = 0.5 * (g + theta * fabs(g));
    gm[i] = gp[i] - g;
    sp += gp[i];
    sm += gm[i];
  }
  double wps = 0.0, ups = 0.0, wms = 0.0, ums = 0.0;
  for (int i = 0; i <= N; ++i) {
    double den = (eps + beta[i]) * (eps + beta[i]);
    double wp = (gp[i] / sp) / den, wm = (gm[i] / sm) / den;
    wps += wp;
    ups += wp * p[i];
    wms += wm;
    ums += wm * p[i];
  }
  return a0 + (sp * (ups / wps) - sm * (ums / wms));
}

/* ------------------------------------------------------------------------ */
/* Problem helpers                                                          */
/* ------------------------------------------------------------------------ */

typedef struct {
  const orc_config *c;
  const orc_tables *T;
  int N, np, nm, nv, nx, ny;
  double hx, hy;
  double kx_scale; /* KXRCF: 1 / h^((N+1)/2), h the radius of the cell's circumscribed circle */
  double time;     /* time of the boundary data */
  const orc_tables *tx, *ty; /* non-uniform meshes: tables per column and per row (limiter only) */
} orc_ctx;

static int make_ctx(const orc_config *c, orc_ctx *x) {
  if (!c || c->dim < 1 || c->dim > 2 || c->order < 1 || c->order > ORC_MAXN || c->nx < 1 || c->ny < 1)
    return ORC_ERR_ARG;
  if (c->dim == 1 && c->ny != 1) return ORC_ERR_ARG;
  if (c->equation != ORC_BURGERS && c->equation != ORC_EULER) return ORC_ERR_ARG;
  for (int s = 0; s < 4; ++s) {
    int k = c->bc[s], kb = c->bc_beyond[s];
    if (k < ORC_BC_PERIODIC || k > ORC_BC_INFLOW) return ORC_ERR_ARG;
    if (kb < -1 || kb > ORC_BC_INFLOW || kb == ORC_BC_PERIODIC) return ORC_ERR_ARG;
    if (kb >= 0 && (s < 2 || c->dim == 1 || k == ORC_BC_PERIODIC)) return ORC_ERR_ARG;
    if ((k == ORC_BC_REFLECTIVE || kb == ORC_BC_REFLECTIVE) && c->equation != ORC_EULER) return ORC_ERR_ARG;
  }
  if (c->positivity && c->equation != ORC_EULER) return ORC_ERR_ARG;
  if (c->xn || c->yn) { /* tensor-product meshes: nodes increasing, no moving switches */
    if (!c->xn || (c->dim == 2) != (c->yn != NULL)) return ORC_ERR_ARG;
    for (int i = 0; i < c->nx; ++i)
      if (!(c->xn[i + 1] > c->xn[i])) return ORC_ERR_ARG;
    if (c->dim == 2)
      for (int j = 0; j < c->ny; ++j)
        if (!(c->yn[j + 1] > c->yn[j])) return ORC_ERR_ARG;
    if (c->bc_beyond[2] >= 0 || c->bc_beyond[3] >= 0) return ORC_ERR_ARG;
  }
  x->tx = x->ty = NULL;
  x->c = c;
  x->time = c->time;
  x->T = tables(c->order);
  if (!x->T) return ORC_ERR_TABLE;
  x->N = c->order;
  x->np = c->order + 1;
  x->nm = c->dim == 1 ? x->np : x->np * x->np;
  x->nv = c->equation == ORC_BURGERS ? 1 : c->dim + 2;
  x->nx = c->nx;
  x->ny = c->ny;
  x->hx = (c->x1 - c->x0) / c->nx;
  x->hy = c->dim == 2 ? (c->y1 - c->y0) / c->ny : 1.0;
  {
    double rad = c->dim == 1 ? 0.5 * x->hx : 0.5 * sqrt(x->hx * x->hx + x->hy * x->hy);
    x->kx_scale = 1.0 / pow(rad, 0.5 * (c->order + 1));
  }
  return ORC_OK;
}

/* Width of column i (i in [-1, nx]: a ghost column has the width of the cell
 * it images, the periodic one or the mirrored adjacent one) and of row j. */
static double cell_hx(const orc_ctx *x, int i) {
  if (!x->c->xn) return x->hx;
  if (i < 0) i = x->c->bc[0] == ORC_BC_PERIODIC ? i + x->nx : -1 - i;
  else if (i >= x->nx) i = x->c->bc[1] == ORC_BC_PERIODIC ? i - x->nx : 2 * x->nx - 1 - i;
  return x->c->xn[i + 1] - x->c->xn[i];
}

static double cell_hy(const orc_ctx *x, int j) {
  if (!x->c->yn) return x->hy;
  if (j < 0) j = x->c->bc[2] == ORC_BC_PERIODIC ? j + x->ny : -1 - j;
  else if (j >= x->ny) j = x->c->bc[3] == ORC_BC_PERIODIC ? j - x->ny : 2 * x->ny - 1 - j;
  return x->c->yn[j + 1] - x->c->yn[j];
}

/* KXRCF scale 1 / h^((N+1)/2) of cell (i, j), h its circumscribed radius. */
static double cell_kx_scale(const orc_ctx *x, int i, int j) {
  if (!x->c->xn) return x->kx_scale;
  double hx = cell_hx(x, i), hy = cell_hy(x, j);
  double rad = x->c->dim == 1 ? 0.5 * hx : 0.5 * sqrt(hx * hx + hy * hy);
  return 1.0 / pow(rad, 0.5 * (x->c->order + 1));
}

static size_t at(const orc_ctx *x, int v, int q, int j, int i) {
  return (((size_t)v * x->nm + q) * x->ny + j) * x->nx + i;
}

/* Kind of boundary side s (0 W, 1 E, 2 S, 3 N) for a ghost cell whose
 * centre has tangential coordinate xt, at the context's time; *state gets
 * the inflow state of that part of the side. */
static int side_kind(const orc_ctx *x, int s, double xt, const double **state) {
  const orc_config *c = x->c;
  int beyond = c->bc_beyond[s] >= 0 && !(xt < c->bc_switch[s][0] + c->bc_switch[s][1] * x->time);
  *state = c->bc_state[s][beyond];
  return beyond ? c->bc_beyond[s] : c->bc[s];
}

/* Modes of cell (i,j), i in [-1,nx], j in [-1,ny], with the boundary
 * conditions.  Beyond a side the ghost cell is: the periodic image; the
 * even reflection of the adjacent interior cell (transmissive: odd modes in
 * the normal direction change sign); that reflection with the normal
 * momentum negated as well (reflective wall); or the constant inflow state
 * (all higher modes zero).  The x side is resolved first: a corner ghost
 * beyond an inflow west/east side is that inflow state; otherwise the
 * south/north rule applies to the column the x side mapped to. */
static void fetch_cell(const orc_ctx *x, const double *U, int i, int j, double out[ORC_MAXV][ORC_MAXM]) {
  int fx = 0, fy = 0, negx = 0, negy = 0;
  const double *inflow = NULL, *st;
  if (i < 0 || i >= x->nx) {
    int s = i < 0 ? 0 : 1;
    int k = side_kind(x, s, 0.0, &st);
    if (k == ORC_BC_PERIODIC) {
      i += s ? -x->nx : x->nx;
    } else {
      i = s ? x->nx - 1 : 0;
      fx = 1;
      negx = k == ORC_BC_REFLECTIVE;
      if (k == ORC_BC_INFLOW) inflow = st;
    }
  }
  if (!inflow && x->c->dim == 2 && (j < 0 || j >= x->ny)) {
    int s = j < 0 ? 2 : 3;
    int k = side_kind(x, s, x->c->x0 + (i + 0.5) * x->hx, &st);
    if (k == ORC_BC_PERIODIC) {
      j += s == 3 ? -x->ny : x->ny;
    } else {
      j = s == 3 ? x->ny - 1 : 0;
      fy = 1;
      negy = k == ORC_BC_REFLECTIVE;
      if (k == ORC_BC_INFLOW) inflow = st;
    }
  }
  if (inflow) {
    double k0 = x->c->dim == 1 ? x->T->b0[0] : x->T->b0[0] * x->T->b0[0];
    for (int v = 0; v < x->nv; ++v)
      for (int q = 0; q < x->nm; ++q) out[v][q] = q == 0 ? inflow[v] / k0 : 0.0;
    return;
  }
  for (int v = 0; v < x->nv; ++v)
    for (int q = 0; q < x->nm; ++q) {
      int m = q % x->np, n = q / x->np;
      double s = U[at(x, v, q, j, i)];
      if (fx && (m & 1)) s = -s;
      if (fy && (n & 1)) s = -s;
      if ((negx && v == 1) || (negy && v == 2)) s = -s;
      out[v][q] = s;
    }
}

/* Value of the cell polynomial at (r,s), given the basis values br[m] =
 * psi_m(r) and bs[n] = psi_n(s) (1D: bs ignored). */
static void point_value(const orc_ctx *x, double C[ORC_MAXV][ORC_MAXM], const double *br, const double *bs,
                        double *u) {
  for (int v = 0; v < x->nv; ++v) {
    double acc = 0.0;
    for (int q = 0; q < x->nm; ++q) {
      int m = q % x->np, n = q / x->np;
      double b = br[m];
      if (x->c->dim == 2) b *= bs[n];
      acc += C[v][q] * b;
    }
    u[v] = acc;
  }
}

static double cell_mean_factor(const orc_ctx *x) {
  /* mean over the cell of the lowest mode's basis function */
  return x->c->dim == 1 ? x->T->b0[0] : x->T->b0[0] * x->T->b0[0];
}

/* Physical flux in direction dir (0: x, 1: y) and its spectral radius. */
static int phys_flux(const orc_ctx *x, int dir, const double *u, double *f) {
  if (x->c->equation == ORC_BURGERS) {
    f[0] = 0.5 * u[0] * u[0];
    return 0;
  }
  double g = x->c->gamma;
  if (x->c->dim == 1) {
    double rho = u[0], vx = u[1] / rho;
    double p = (g - 1.0) * (u[2] - 0.5 * rho * vx * vx);
    f[0] = u[1];
    f[1] = u[1] * vx + p;
    f[2] = (u[2] + p) * vx;
    return !(rho > 0.0 && p > 0.0);
  }
  double rho = u[0], vx = u[1] / rho, vy = u[2] / rho;
  double p = (g - 1.0) * (u[3] - 0.5 * rho * (vx * vx + vy * vy));
  double vn = dir == 0 ? vx : vy;
  f[0] = dir == 0 ? u[1] : u[2];
  f[1] = u[1] * vn + (dir == 0 ? p : 0.0);
  f[2] = u[2] * vn + (dir == 1 ? p : 0.0);
  f[3] = (u[3] + p) * vn;
  return !(rho > 0.0 && p > 0.0);
}

static double spectral_radius(const orc_ctx *x, int dir, const double *u, int *bad) {
  if (x->c->equation == ORC_BURGERS) return fabs(u[0]);
  double g = x->c->gamma, rho = u[0];
  if (x->c->dim == 1) {
    double vx = u[1] / rho, p = (g - 1.0) * (u[2] - 0.5 * rho * vx * vx);
    if (!(rho > 0.0 && p > 0.0)) *bad = 1;
    return fabs(vx) + sqrt(g * p / rho);
  }
  double vx = u[1] / rho, vy = u[2] / rho;
  double p = (g - 1.0) * (u[3] - 0.5 * rho * (vx * vx + vy * vy));
  if (!(rho > 0.0 && p > 0.0)) *bad = 1;
  return fabs(dir == 0 ? vx : vy) + sqrt(g * p / rho);
}

/* Local Lax-Friedrichs flux between the left/lower state a and right/upper b,
 * with the dissipation coefficient taken pointwise from the two states. */
static void llf(const orc_ctx *x, int dir, const double *a, const double *b, double *F, int *bad) {
  double fa[ORC_MAXV], fb[ORC_MAXV];
  if (phys_flux(x, dir, a, fa)) *bad = 1;
  if (phys_flux(x, dir, b, fb)) *bad = 1;
  double al = fmax(spectral_radius(x, dir, a, bad), spectral_radius(x, dir, b, bad));
  for (int v = 0; v < x->nv; ++v) F[v] = 0.5 * (fa[v] + fb[v]) - 0.5 * al * (b[v] - a[v]);
}

/* ------------------------------------------------------------------------ */
/* Section 2, weak form: dU/dt = L(U) per cell in the orthonormal modal      */
/* basis (M = (h/2) I in each direction, so M^{-1} is the factor 2/h).       */
/* ------------------------------------------------------------------------ */

static int residual_cell(const orc_ctx *x, const double *U, int i, int j, double L[ORC_MAXV][ORC_MAXM]) {
  const orc_tables *T = x->T;
  int np = x->np, nv = x->nv, bad = 0;
  double C[ORC_MAXV][ORC_MAXM], Nb[ORC_MAXV][ORC_MAXM];
  double a[ORC_MAXV], b[ORC_MAXV], F[ORC_MAXV], f[ORC_MAXV], g[ORC_MAXV];
  double br[ORC_MAXP], bs[ORC_MAXP], dbr[ORC_MAXP], dbs[ORC_MAXP];
  fetch_cell(x, U, i, j, C);
  for (int v = 0; v < nv; ++v)
    for (int q = 0; q < x->nm; ++q) L[v][q] = 0.0;

  if (x->c->dim == 1) {
    double sx = 2.0 / cell_hx(x, i);
    for (int q = 0; q < np; ++q) { /* volume term: sum_q w_q f(u_q) psi_n'(r_q) */
      for (int n = 0; n < np; ++n) br[n] = T->bq[n][q];
      point_value(x, C, br, NULL, a);
      if (phys_flux(x, 0, a, f)) bad = 1;
      for (int v = 0; v < nv; ++v)
        for (int n = 0; n < np; ++n) L[v][n] += sx * T->wq[q] * f[v] * T->dbq[n][q];
    }
    /* right face x_{i+1/2} */
    fetch_cell(x, U, i + 1, j, Nb);
    point_value(x, C, T->bp, NULL, a);
    point_value(x, Nb, T->bm, NULL, b);
    llf(x, 0, a, b, F, &bad);
    for (int v = 0; v < nv; ++v)
      for (int n = 0; n < np; ++n) L[v][n] -= sx * F[v] * T->bp[n];
    /* left face x_{i-1/2} */
    fetch_cell(x, U, i - 1, j, Nb);
    point_value(x, Nb, T->bp, NULL, a);
    point_value(x, C, T->bm, NULL, b);
    llf(x, 0, a, b, F, &bad);
    for (int v = 0; v < nv; ++v)
      for (int n = 0; n < np; ++n) L[v][n] += sx * F[v] * T->bm[n];
    return bad;
  }

  double sx = 2.0 / cell_hx(x, i), sy = 2.0 / cell_hy(x, j);
  for (int qx = 0; qx < np; ++qx)
    for (int qy = 0; qy < np; ++qy) {
      double w = T->wq[qx] * T->wq[qy];
      for (int n = 0; n < np; ++n) {
        br[n] = T->bq[n][qx];
        dbr[n] = T->dbq[n][qx];
        bs[n] = T->bq[n][qy];
        dbs[n] = T->dbq[n][qy];
      }
      point_value(x, C, br, bs, a);
      if (phys_flux(x, 0, a, f)) bad = 1;
      if (phys_flux(x, 1, a, g)) bad = 1;
      for (int v = 0; v < nv; ++v)
        for (int q = 0; q < x->nm; ++q) {
          int m = q % np, n = q / np;
          L[v][q] += w * (sx * f[v] * dbr[m] * bs[n] + sy * g[v] * br[m] * dbs[n]);
        }
    }
  double Ce[ORC_MAXV][ORC_MAXM], Cw[ORC_MAXV][ORC_MAXM], Cn[ORC_MAXV][ORC_MAXM], Cs[ORC_MAXV][ORC_MAXM];
  fetch_cell(x, U, i + 1, j, Ce);
  fetch_cell(x, U, i - 1, j, Cw);
  fetch_cell(x, U, i, j + 1, Cn);
  fetch_cell(x, U, i, j - 1, Cs);
  for (int e = 0; e < np; ++e) {
    double w = T->wq[e], bt[ORC_MAXP];
    for (int n = 0; n < np; ++n) bt[n] = T->bq[n][e]; /* basis at the edge point */
    /* east face */
    point_value(x, C, T->bp, bt, a);
    point_value(x, Ce, T->bm, bt, b);
    llf(x, 0, a, b, F, &bad);
    for (int v = 0; v < nv; ++v)
      for (int q = 0; q < x->nm; ++q) L[v][q] -= sx * w * F[v] * T->bp[q % np] * bt[q / np];
    /* west face */
    point_value(x, Cw, T->bp, bt, a);
    point_value(x, C, T->bm, bt, b);
    llf(x, 0, a, b, F, &bad);
    for (int v = 0; v < nv; ++v)
      for (int q = 0; q < x->nm; ++q) L[v][q] += sx * w * F[v] * T->bm[q % np] * bt[q / np];
    /* north face */
    point_value(x, C, bt, T->bp, a);
    point_value(x, Cn, bt, T->bm, b);
    llf(x, 1, a, b, F, &bad);
    for (int v = 0; v < nv; ++v)
      for (int q = 0; q < x->nm; ++q) L[v][q] -= sy * w * F[v] * bt[q % np] * T->bp[q / np];
    /* south face */
    point_value(x, Cs, bt, T->bp, a);
    point_value(x, C, bt, T->bm, b);
    llf(x, 1, a, b, F, &bad);
    for (int v = 0; v < nv; ++v)
      for (int q = 0; q < x->nm; ++q) L[v][q] += sy * w * F[v] * bt[q % np] * T->bm[q / np];
  }
  return bad;
}

int orc_residual(const orc_config *c, const double *U, double *Lout) {
  orc_ctx x;
  int rc = make_ctx(c, &x);
  if (rc) return rc;
  int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
  for (int j = 0; j < x.ny; ++j)
    for (int i = 0; i < x.nx; ++i) {
      double L[ORC_MAXV][ORC_MAXM];
      bad |= residual_cell(&x, U, i, j, L);
      for (int v = 0; v < x.nv; ++v)
        for (int q = 0; q < x.nm; ++q) Lout[at(&x, v, q, j, i)] = L[v][q];
    }
  return bad ? ORC_ERR_NONPHYSICAL : ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Troubled-cell indicator: TVB-modified minmod (Cockburn and Shu).          */
/* ------------------------------------------------------------------------ */

static double minmod3(double a, double b, double c) {
  if (a > 0.0 && b > 0.0 && c > 0.0) return fmin(a, fmin(b, c));
  if (a < 0.0 && b < 0.0 && c < 0.0) return fmax(a, fmax(b, c));
  return 0.0;
}

/* One test: flagged when the modified minmod does not return a unchanged.
 * The margin is a lower bound on how far a, dp or dm must move to change
 * the outcome. */
static int tvb_test(double a, double dp, double dm, double Mh2, double *margin) {
  double aa = fabs(a);
  if (aa <= Mh2) {
    *margin = Mh2 - aa;
    return 0;
  }
  double m = fmin(aa - Mh2, fmin(fabs(aa - fabs(dp)), fabs(aa - fabs(dm))));
  *margin = m;
  return minmod3(a, dp, dm) != a;
}

static int indicator_cell(const orc_ctx *x, const double *U, int i, int j, double *margin) {
  double C[ORC_MAXV][ORC_MAXM], Nb[ORC_MAXV][ORC_MAXM], up[ORC_MAXV], um[ORC_MAXV];
  double mean[ORC_MAXV], mp[ORC_MAXV], mm[ORC_MAXV];
  double k0 = cell_mean_factor(x);
  int flag = 0;
  double mg = INFINITY, t;
  fetch_cell(x, U, i, j, C);
  for (int v = 0; v < x->nv; ++v) mean[v] = C[v][0] * k0;
  int ndir = x->c->dim;
  for (int dir = 0; dir < ndir; ++dir) {
    double h = dir == 0 ? cell_hx(x, i) : cell_hy(x, j), Mh2 = x->c->tvb_M * h * h;
    /* traces at the face midpoints of this direction */
    if (dir == 0) {
      point_value(x, C, x->T->bp, x->T->b0, up);
      point_value(x, C, x->T->bm, x->T->b0, um);
      fetch_cell(x, U, i + 1, j, Nb);
      for (int v = 0; v < x->nv; ++v) mp[v] = Nb[v][0] * k0;
      fetch_cell(x, U, i - 1, j, Nb);
      for (int v = 0; v < x->nv; ++v) mm[v] = Nb[v][0] * k0;
    } else {
      point_value(x, C, x->T->b0, x->T->bp, up);
      point_value(x, C, x->T->b0, x->T->bm, um);
      fetch_cell(x, U, i, j + 1, Nb);
      for (int v = 0; v < x->nv; ++v) mp[v] = Nb[v][0] * k0;
      fetch_cell(x, U, i, j - 1, Nb);
      for (int v = 0; v < x->nv; ++v) mm[v] = Nb[v][0] * k0;
    }
    for (int v = 0; v < x->nv; ++v) {
      double dp = mp[v] - mean[v], dm = mean[v] - mm[v];
      flag |= tvb_test(up[v] - mean[v], dp, dm, Mh2, &t);
      mg = fmin(mg, t);
      flag |= tvb_test(mean[v] - um[v], dp, dm, Mh2, &t);
      mg = fmin(mg, t);
    }
  }
  *margin = mg;
  return flag;
}

/* ------------------------------------------------------------------------ */
/* Troubled-cell indicator of Krivodonova, Xin, Remacle, Chevaugeon and      */
/* Flaherty (the paper's own, Sec. 3 step 1, by citation): per indicator     */
/* variable, the integral over the cell's inflow boundary of the jump        */
/* between the cell's trace and the neighbour's, divided by h^((N+1)/2), the */
/* inflow boundary's measure and the maximum of |u| over the cell's          */
/* quadrature points; troubled when it exceeds 1.  Inflow faces are those    */
/* where the cell-average characteristic velocity points into the cell      */
/* (Burgers: the mean itself; Euler: mean momentum / mean density); the      */
/* variables are u (Burgers) or density and total energy (Euler).  The       */
/* margin is min(|I - 1|, |v_x|, |v_y|).                                      */
/* ------------------------------------------------------------------------ */
static int kxrcf_cell(const orc_ctx *x, const double *U, int i, int j, double *margin) {
  const orc_tables *T = x->T;
  const int dim = x->c->dim, np = x->np;
  double C[ORC_MAXV][ORC_MAXM], Nb[ORC_MAXV][ORC_MAXM];
  fetch_cell(x, U, i, j, C);
  double k0 = cell_mean_factor(x);
  double vel[2] = {0.0, 0.0};
  if (x->c->equation == ORC_BURGERS) {
    vel[0] = vel[1] = C[0][0] * k0;
  } else {
    double rho = C[0][0] * k0;
    vel[0] = C[1][0] * k0 / rho;
    if (dim == 2) vel[1] = C[2][0] * k0 / rho;
  }
  int vars[2], nvar;
  if (x->c->equation == ORC_BURGERS) {
    vars[0] = 0;
    nvar = 1;
  } else {
    vars[0] = 0;
    vars[1] = dim + 1;
    nvar = 2;
  }
  double mg = fabs(vel[0]);
  if (dim == 2) mg = fmin(mg, fabs(vel[1]));
  int flag = 0;
  for (int k = 0; k < nvar; ++k) {
    const int v = vars[k];
    double J = 0.0, len = 0.0;
    for (int dir = 0; dir < dim; ++dir) {
      if (vel[dir] == 0.0) continue;
      const int minus = vel[dir] > 0.0; /* inflow through the west / south face */
      const int di = dir == 0 ? (minus ? -1 : 1) : 0, dj = dir == 1 ? (minus ? -1 : 1) : 0;
      fetch_cell(x, U, i + di, j + dj, Nb);
      const double *own = minus ? T->bm : T->bp, *nbr = minus ? T->bp : T->bm;
      if (dim == 1) {
        double a[ORC_MAXV], b[ORC_MAXV];
        point_value(x, C, own, NULL, a);
        point_value(x, Nb, nbr, NULL, b);
        J += a[v] - b[v];
        len += 1.0;
      } else {
        const double flen = dir == 0 ? cell_hy(x, j) : cell_hx(x, i);
        double integral = 0.0;
        for (int e = 0; e < np; ++e) {
          double bs[ORC_MAXP], a[ORC_MAXV], b[ORC_MAXV];
          for (int n = 0; n < np; ++n) bs[n] = T->bq[n][e];
          if (dir == 0) {
            point_value(x, C, own, bs, a);
            point_value(x, Nb, nbr, bs, b);
          } else {
            point_value(x, C, bs, own, a);
            point_value(x, Nb, bs, nbr, b);
          }
          integral += T->wq[e] * (a[v] - b[v]);
        }
        J += 0.5 * flen * integral;
        len += flen;
      }
    }
    /* maximum of |u| over the volume quadrature points */
    double norm = 0.0;
    for (int qy = 0; qy < (dim == 2 ? np : 1); ++qy)
      for (int qx = 0; qx < np; ++qx) {
        double bx[ORC_MAXP], by[ORC_MAXP], a[ORC_MAXV];
        for (int n = 0; n < np; ++n) {
          bx[n] = T->bq[n][qx];
          by[n] = T->bq[n][qy];
        }
        point_value(x, C, bx, by, a);
        norm = fmax(norm, fabs(a[v]));
      }
    const double I = (len > 0.0 && norm > 0.0) ? fabs(J) * cell_kx_scale(x, i, j) / (len * norm) : 0.0;
    flag |= I > 1.0;
    mg = fmin(mg, fabs(I - 1.0));
  }
  *margin = mg;
  return flag;
}

static int any_indicator(const orc_ctx *x, const double *U, int i, int j, double *margin) {
  if (x->c->indicator == ORC_IND_KXRCF) return kxrcf_cell(x, U, i, j, margin);
  return indicator_cell(x, U, i, j, margin);
}

int orc_indicator(const orc_config *c, const double *U, uint8_t *flags, double *margin) {
  orc_ctx x;
  int rc = make_ctx(c, &x);
  if (rc) return rc;
#pragma omp parallel for schedule(static)
  for (int j = 0; j < x.ny; ++j)
    for (int i = 0; i < x.nx; ++i) {
      double m;
      int f = any_indicator(&x, U, i, j, &m);
      size_t k = (size_t)j * x.nx + i;
      if (flags) flags[k] = (uint8_t)f;
      if (margin) margin[k] = m;
    }
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Section 3: CSWENO limiting of one troubled cell (all variables).         */
/* ------------------------------------------------------------------------ */

/* Mean of psi_n over stencil interval k of the compact stencil, measured in
 * the reference coordinate of the cell that interval belongs to. */
static double interval_mean(const orc_tables *T, int k, int n) {
  int N = T->N;
  if (k == N) return n == 0 ? T->b0[0] : 0.0; /* whole troubled cell */
  int sub = k < N ? k : k - N - 1;
  return T->sub[sub][n];
}

/* Eigenvectors of the Euler flux Jacobian in direction dir (0: x, 1: y) at
 * the conserved state w (1D: 3 components, 2D: 4): R holds the right
 * eigenvectors as columns (eigenvalues u_n - c, u_n, u_n + c and, in 2D,
 * u_n for the shear wave), L = R^-1 (rows: left eigenvectors). */
static void char_eig(int dim, double gamma, int dir, const double *w, double L[ORC_MAXV][ORC_MAXV],
                     double R[ORC_MAXV][ORC_MAXV]) {
  const double rho = w[0];
  double un, ut = 0.0, E;
  if (dim == 1) {
    un = w[1] / rho;
    E = w[2];
  } else {
    un = w[1 + dir] / rho;
    ut = w[2 - dir] / rho;
    E = w[3];
  }
  const double q2 = un * un + ut * ut;
  const double p = (gamma - 1.0) * (E - 0.5 * rho * q2);
  const double c = sqrt(gamma * p / rho), H = (E + p) / rho;
  const double b1 = (gamma - 1.0) / (c * c), b2 = 0.5 * b1 * q2;
  if (dim == 1) {
    const double Rm[3][3] = {{1.0, 1.0, 1.0}, {un - c, un, un + c}, {H - un * c, 0.5 * q2, H + un * c}};
    const double Lm[3][3] = {{0.5 * (b2 + un / c), -0.5 * (b1 * un + 1.0 / c), 0.5 * b1},
                             {1.0 - b2, b1 * un, -b1},
                             {0.5 * (b2 - un / c), -0.5 * (b1 * un - 1.0 / c), 0.5 * b1}};
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        R[a][b] = Rm[a][b];
        L[a][b] = Lm[a][b];
      }
    return;
  }
  /* in the (normal, tangential) ordering of the momentum components */
  const double Rm[4][4] = {{1.0, 1.0, 1.0, 0.0},
                           {un - c, un, un + c, 0.0},
                           {ut, ut, ut, 1.0},
                           {H - un * c, 0.5 * q2, H + un * c, ut}};
  const double Lm[4][4] = {{0.5 * (b2 + un / c), -0.5 * (b1 * un + 1.0 / c), -0.5 * b1 * ut, 0.5 * b1},
                           {1.0 - b2, b1 * un, b1 * ut, -b1},
                           {0.5 * (b2 - un / c), -0.5 * (b1 * un - 1.0 / c), -0.5 * b1 * ut, 0.5 * b1},
                           {-ut, 0.0, 1.0, 0.0}};
  /* back to (rho, rho u, rho v, E): the momentum rows of R and columns of L */
  const int perm[4] = {0, dir == 0 ? 1 : 2, dir == 0 ? 2 : 1, 3};
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) {
      R[perm[a]][b] = Rm[a][b];
      L[a][perm[b]] = Lm[a][b];
    }
}

int orc_char_eig(const orc_config *c, const double *w, int dir, double *L, double *R) {
  if (!c || c->equation != ORC_EULER || dir < 0 || dir >= c->dim) return ORC_ERR_ARG;
  double Lm[ORC_MAXV][ORC_MAXV], Rm[ORC_MAXV][ORC_MAXV];
  char_eig(c->dim, c->gamma, dir, w, Lm, Rm);
  const int nv = c->dim + 2;
  for (int a = 0; a < nv; ++a)
    for (int b = 0; b < nv; ++b) {
      L[a * nv + b] = Lm[a][b];
      R[a * nv + b] = Rm[a][b];
    }
  return ORC_OK;
}

/* Characteristic-field CSWENO (Euler; the paper limits systems in local
 * characteristic fields, end of Sec. 3): each sweep maps its stencil means to
 * characteristic fields with L of that sweep's direction, evaluated at the
 * troubled cell's mean state, reconstructs every field with the same WENO
 * and maps the point values back with R. */
/* Tables of the x-sweeps of column i and of the y-sweeps of row j. */
static const orc_tables *col_tables(const orc_ctx *x, int i) { return x->tx ? &x->tx[i] : x->T; }
static const orc_tables *row_tables(const orc_ctx *x, int j) { return x->ty ? &x->ty[j] : x->T; }

static void limit_cell_char(const orc_ctx *x, const double *Uin, int i, int j, double *Uout) {
  const orc_tables *T = col_tables(x, i), *Ty = row_tables(x, j);
  const int N = x->N, np = x->np, ns = 2 * N + 1, ng = T->ng, nv = x->nv;
  const double eps = x->c->weno_eps, k0 = cell_mean_factor(x);
  const int negw = x->c->negw_mode;
  double w0[ORC_MAXV];
  if (x->c->dim == 1) {
    double Cm[ORC_MAXV][ORC_MAXM], C0[ORC_MAXV][ORC_MAXM], Cp[ORC_MAXV][ORC_MAXM];
    fetch_cell(x, Uin, i - 1, j, Cm);
    fetch_cell(x, Uin, i, j, C0);
    fetch_cell(x, Uin, i + 1, j, Cp);
    for (int v = 0; v < nv; ++v) w0[v] = C0[v][0] * k0;
    double L[ORC_MAXV][ORC_MAXV], R[ORC_MAXV][ORC_MAXV];
    char_eig(1, x->c->gamma, 0, w0, L, R);
    double a[ORC_MAXV][ORC_MAXS], ch[ORC_MAXV][ORC_MAXS], cG[ORC_MAXV][ORC_MAXG];
    for (int v = 0; v < nv; ++v)
      for (int k = 0; k < ns; ++k) {
        double (*src)[ORC_MAXM] = k < N ? Cm : (k == N ? C0 : Cp);
        double s = 0.0;
        for (int n = 0; n < np; ++n) s += src[v][n] * interval_mean(T, k, n);
        a[v][k] = s;
      }
    for (int f = 0; f < nv; ++f)
      for (int k = 0; k < ns; ++k) {
        double s = 0.0;
        for (int v = 0; v < nv; ++v) s += L[f][v] * a[v][k];
        ch[f][k] = s;
      }
    for (int f = 0; f < nv; ++f)
      for (int G = 0; G < ng; ++G) cG[f][G] = orc_weno_point(T, G, ch[f], eps, negw);
    for (int v = 0; v < nv; ++v)
      for (int n = 1; n < np; ++n) {
        double s = 0.0;
        for (int G = 0; G < ng; ++G) {
          double uG = 0.0;
          for (int f = 0; f < nv; ++f) uG += R[v][f] * cG[f][G];
          s += T->wg[G] * uG * T->bg[n][G];
        }
        Uout[at(x, v, n, j, i)] = s;
      }
    return;
  }
  double B[3][3][ORC_MAXV][ORC_MAXM];
  for (int dy = -1; dy <= 1; ++dy)
    for (int dx = -1; dx <= 1; ++dx) fetch_cell(x, Uin, i + dx, j + dy, B[dy + 1][dx + 1]);
  for (int v = 0; v < nv; ++v) w0[v] = B[1][1][v][0] * k0;
  double Lx[ORC_MAXV][ORC_MAXV], Rx[ORC_MAXV][ORC_MAXV], Ly[ORC_MAXV][ORC_MAXV], Ry[ORC_MAXV][ORC_MAXV];
  char_eig(2, x->c->gamma, 0, w0, Lx, Rx);
  char_eig(2, x->c->gamma, 1, w0, Ly, Ry);
  double a[ORC_MAXV][ORC_MAXS][ORC_MAXS]; /* [v][iy][ix] */
  for (int v = 0; v < nv; ++v)
    for (int iy = 0; iy < ns; ++iy)
      for (int ix = 0; ix < ns; ++ix) {
        int cx = ix < N ? 0 : (ix == N ? 1 : 2), cy = iy < N ? 0 : (iy == N ? 1 : 2);
        double s = 0.0;
        for (int q = 0; q < x->nm; ++q) {
          int m = q % np, n = q / np;
          s += B[cy][cx][v][q] * interval_mean(T, ix, m) * interval_mean(T, iy, n);
        }
        a[v][iy][ix] = s;
      }
  /* x-sweeps in x-characteristic fields */
  double vy[ORC_MAXV][ORC_MAXS][ORC_MAXG];
  for (int iy = 0; iy < ns; ++iy) {
    double ch[ORC_MAXV][ORC_MAXS], cG[ORC_MAXV][ORC_MAXG];
    for (int f = 0; f < nv; ++f)
      for (int ix = 0; ix < ns; ++ix) {
        double s = 0.0;
        for (int v = 0; v < nv; ++v) s += Lx[f][v] * a[v][iy][ix];
        ch[f][ix] = s;
      }
    for (int f = 0; f < nv; ++f)
      for (int G = 0; G < ng; ++G) cG[f][G] = orc_weno_point(T, G, ch[f], eps, negw);
    for (int v = 0; v < nv; ++v)
      for (int G = 0; G < ng; ++G) {
        double s = 0.0;
        for (int f = 0; f < nv; ++f) s += Rx[v][f] * cG[f][G];
        vy[v][iy][G] = s;
      }
  }
  /* y-sweeps in y-characteristic fields */
  double u[ORC_MAXV][ORC_MAXG][ORC_MAXG]; /* [v][G][H] */
  for (int G = 0; G < ng; ++G) {
    double ch[ORC_MAXV][ORC_MAXS], cH[ORC_MAXV][ORC_MAXG];
    for (int f = 0; f < nv; ++f)
      for (int iy = 0; iy < ns; ++iy) {
        double s = 0.0;
        for (int v = 0; v < nv; ++v) s += Ly[f][v] * vy[v][iy][G];
        ch[f][iy] = s;
      }
    for (int f = 0; f < nv; ++f)
      for (int H = 0; H < ng; ++H) cH[f][H] = orc_weno_point(Ty, H, ch[f], eps, negw);
    for (int v = 0; v < nv; ++v)
      for (int H = 0; H < ng; ++H) {
        double s = 0.0;
        for (int f = 0; f < nv; ++f) s += Ry[v][f] * cH[f][H];
        u[v][G][H] = s;
      }
  }
  for (int v = 0; v < nv; ++v)
    for (int q = 1; q < x->nm; ++q) {
      int m = q % np, n = q / np;
      double s = 0.0;
      for (int G = 0; G < ng; ++G)
        for (int H = 0; H < ng; ++H) s += T->wg[G] * T->wg[H] * u[v][G][H] * T->bg[m][G] * T->bg[n][H];
      Uout[at(x, v, q, j, i)] = s;
    }
}

static void limit_cell(const orc_ctx *x, const double *Uin, int i, int j, double *Uout) {
  if (x->c->limiter == ORC_LIM_CSWENO_CHAR && x->c->equation == ORC_EULER) {
    limit_cell_char(x, Uin, i, j, Uout);
    return;
  }
  const orc_tables *T = col_tables(x, i), *Ty = row_tables(x, j);
  int N = x->N, np = x->np, ns = 2 * N + 1, ng = T->ng;
  double eps = x->c->weno_eps;
  int negw = x->c->negw_mode;
  if (x->c->dim == 1) {
    double Cm[ORC_MAXV][ORC_MAXM], C0[ORC_MAXV][ORC_MAXM], Cp[ORC_MAXV][ORC_MAXM];
    fetch_cell(x, Uin, i - 1, j, Cm);
    fetch_cell(x, Uin, i, j, C0);
    fetch_cell(x, Uin, i + 1, j, Cp);
    for (int v = 0; v < x->nv; ++v) {
      double a[ORC_MAXS], uG[ORC_MAXG];
      for (int k = 0; k < ns; ++k) {
        double (*src)[ORC_MAXM] = k < N ? Cm : (k == N ? C0 : Cp);
        double s = 0.0;
        for (int n = 0; n < np; ++n) s += src[v][n] * interval_mean(T, k, n);
        a[k] = s;
      }
      for (int G = 0; G < ng; ++G) uG[G] = orc_weno_point(T, G, a, eps, negw);
      /* Step 6: the mean is kept, the other moments are re-projected. */
      for (int n = 1; n < np; ++n) {
        double s = 0.0;
        for (int G = 0; G < ng; ++G) s += T->wg[G] * uG[G] * T->bg[n][G];
        Uout[at(x, v, n, j, i)] = s;
      }
    }
    return;
  }
  /* 2D, dimension by dimension: the 3x3 block gives (2N+1)^2 sub-rectangle
   * means; x-sweeps on every y-interval reconstruct y-interval means at the
   * x-points, then y-sweeps at every x-point give the tensor point values. */
  double B[3][3][ORC_MAXV][ORC_MAXM];
  for (int dy = -1; dy <= 1; ++dy)
    for (int dx = -1; dx <= 1; ++dx) fetch_cell(x, Uin, i + dx, j + dy, B[dy + 1][dx + 1]);
  for (int v = 0; v < x->nv; ++v) {
    double a[ORC_MAXS][ORC_MAXS]; /* [iy][ix] */
    for (int iy = 0; iy < ns; ++iy)
      for (int ix = 0; ix < ns; ++ix) {
        int cx = ix < N ? 0 : (ix == N ? 1 : 2), cy = iy < N ? 0 : (iy == N ? 1 : 2);
        double s = 0.0;
        for (int q = 0; q < x->nm; ++q) {
          int m = q % np, n = q / np;
          s += B[cy][cx][v][q] * interval_mean(T, ix, m) * interval_mean(T, iy, n);
        }
        a[iy][ix] = s;
      }
    double vy[ORC_MAXS][ORC_MAXG]; /* y-interval means at the x-points */
    for (int iy = 0; iy < ns; ++iy)
      for (int G = 0; G < ng; ++G) vy[iy][G] = orc_weno_point(T, G, a[iy], eps, negw);
    double u[ORC_MAXG][ORC_MAXG]; /* [G: x-point][H: y-point] */
    for (int G = 0; G < ng; ++G) {
      double col[ORC_MAXS];
      for (int iy = 0; iy < ns; ++iy) col[iy] = vy[iy][G];
      for (int H = 0; H < ng; ++H) u[G][H] = orc_weno_point(Ty, H, col, eps, negw);
    }
    for (int q = 1; q < x->nm; ++q) {
      int m = q % np, n = q / np;
      double s = 0.0;
      for (int G = 0; G < ng; ++G)
        for (int H = 0; H < ng; ++H) s += T->wg[G] * T->wg[H] * u[G][H] * T->bg[m][G] * T->bg[n][H];
      Uout[at(x, v, q, j, i)] = s;
    }
  }
}

static int positivity_state(const orc_ctx *x, double *U, double *theta);

/* Indicator + CSWENO with Jacobi semantics: every decision and every
 * reconstruction reads the state as it was before this call. */
static int limit_state(const orc_ctx *x0, double *U, double *work, uint8_t *flags_out, double *margin_out,
                       const uint8_t *flags_in) {
  orc_ctx xl = *x0, *x = &xl;
  orc_tables *tx = NULL, *ty = NULL;
  if (x->c->xn && x->c->limiter != ORC_LIM_NONE) {
    /* non-uniform mesh: the tables of every column and row, from the widths
     * of the cell and of its two neighbours (Steps 2-3 on that stencil) */
    tx = (orc_tables *)malloc(sizeof(orc_tables) * x->nx);
    ty = x->c->dim == 2 ? (orc_tables *)malloc(sizeof(orc_tables) * x->ny) : NULL;
    int bad = !tx || (x->c->dim == 2 && !ty);
    for (int i = 0; !bad && i < x->nx; ++i) {
      double h = cell_hx(x, i);
      bad = build_tables_into(&tx[i], x->N, cell_hx(x, i - 1) / h, cell_hx(x, i + 1) / h) != ORC_OK;
    }
    for (int j = 0; !bad && x->c->dim == 2 && j < x->ny; ++j) {
      double h = cell_hy(x, j);
      bad = build_tables_into(&ty[j], x->N, cell_hy(x, j - 1) / h, cell_hy(x, j + 1) / h) != ORC_OK;
    }
    if (bad) {
      free(tx);
      free(ty);
      return ORC_ERR_TABLE;
    }
    xl.tx = tx;
    xl.ty = ty;
  }
  size_t n = (size_t)x->nv * x->nm * x->ny * x->nx;
  memcpy(work, U, n * sizeof(double));
#pragma omp parallel for schedule(dynamic, 4)
  for (int j = 0; j < x->ny; ++j)
    for (int i = 0; i < x->nx; ++i) {
      size_t k = (size_t)j * x->nx + i;
      double m = INFINITY;
      int f;
      if (flags_in) f = flags_in[k] != 0;
      else if (x->c->indicator == ORC_IND_ALL) f = 1;
      else f = any_indicator(x, work, i, j, &m);
      if (flags_out) flags_out[k] = (uint8_t)f;
      if (margin_out) margin_out[k] = m;
      if (f && x->c->limiter != ORC_LIM_NONE) limit_cell(x, work, i, j, U);
    }
  free(tx);
  free(ty);
  return ORC_OK;
}

int orc_limit(const orc_config *c, double *U, uint8_t *flags_out, double *margin_out, const uint8_t *flags_in) {
  orc_ctx x;
  int rc = make_ctx(c, &x);
  if (rc) return rc;
  size_t n = (size_t)x.nv * x.nm * x.ny * x.nx;
  double *work = (double *)malloc(n * sizeof(double));
  if (!work) return ORC_ERR_ARG;
  rc = limit_state(&x, U, work, flags_out, margin_out, flags_in);
  free(work);
  if (!rc && c->positivity) rc = positivity_state(&x, U, NULL);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Positivity-preserving scaling of Zhang & Shu for rectangular meshes, the  */
/* component the paper adds to the limiter for Example 11.                   */
/* ------------------------------------------------------------------------ */

/* Points where density and pressure are kept at or above eps: the tensor
 * products of the face rule G ((N+1)-point Gauss) with the L-point
 * Gauss-Lobatto rule S (smallest L with 2L-3 >= N) in both orders, as Zhang
 * and Shu require, and also the volume points G x G, so that every point
 * where the scheme evaluates a flux is admissible.  1D: S and G. */
static int pos_points(const orc_ctx *x, double *r, double *s) {
  int N = x->N, L = N == 1 ? 2 : 3, n = 0;
  double g[ORC_MAXP], gw[ORC_MAXP], l[3], lw[3];
  gauss_rule(N + 1, g, gw);
  gauss_lobatto_rule(L, l, lw);
  if (x->c->dim == 1) {
    for (int a = 0; a < L; ++a) { r[n] = l[a]; s[n++] = 0.0; }
    for (int a = 0; a <= N; ++a) { r[n] = g[a]; s[n++] = 0.0; }
    return n;
  }
  for (int a = 0; a <= N; ++a)
    for (int b = 0; b < L; ++b) { r[n] = g[a]; s[n++] = l[b]; }
  for (int a = 0; a < L; ++a)
    for (int b = 0; b <= N; ++b) { r[n] = l[a]; s[n++] = g[b]; }
  for (int a = 0; a <= N; ++a)
    for (int b = 0; b <= N; ++b) { r[n] = g[a]; s[n++] = g[b]; }
  return n;
}

static double pressure(const orc_ctx *x, const double *w) {
  double ke = 0.0;
  for (int d = 1; d <= x->c->dim; ++d) ke += w[d] * w[d];
  return (x->c->gamma - 1.0) * (w[x->nv - 1] - 0.5 * ke / w[0]);
}

/* The t in [0,1] where the pressure along wb + t (wq - wb) falls to eps,
 * for p(wb) >= eps > p(wq) and positive density on the segment.  Multiplied
 * by the density, p = eps is a quadratic A t^2 + B t + C = 0 with C >= 0 and
 * A + B + C < 0; pressure is concave along the segment, so the crossing is
 * unique and is the root where the quadratic decreases,
 * (-B - sqrt(D)) / (2A) = 2C / (sqrt(D) - B) with D = B^2 - 4AC, taken in
 * the form without cancellation: the second for B <= 0, the first for B > 0
 * (where A < 0). */
static double pos_root(const orc_ctx *x, const double *wb, const double *wq, double eps) {
  int e = x->nv - 1;
  double ee = eps / (x->c->gamma - 1.0);
  double dr = wq[0] - wb[0], dE = wq[e] - wb[e], mm = 0.0, md = 0.0, dd = 0.0;
  for (int d = 1; d <= x->c->dim; ++d) {
    double dm = wq[d] - wb[d];
    mm += wb[d] * wb[d];
    md += wb[d] * dm;
    dd += dm * dm;
  }
  double A = dE * dr - 0.5 * dd;
  double B = wb[e] * dr + wb[0] * dE - md - ee * dr;
  double C = wb[e] * wb[0] - 0.5 * mm - ee * wb[0];
  if (!(C > 0.0)) return 0.0;
  double D = B * B - 4.0 * A * C;
  if (D < 0.0) D = 0.0;
  double t = B <= 0.0 ? 2.0 * C / (sqrt(D) - B) : (-B - sqrt(D)) / (2.0 * A);
  return t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
}

/* Floor of density and pressure.  Zhang and Shu use 1e-13; in double
 * precision the pressure of a scaled point value carries an absolute
 * rounding error near 1e-16 times the energy, which exceeds 1e-13 once the
 * energy is in the hundreds (about 560 behind the Mach 10 shock), and a
 * point left at -1e-14 breaks the sound speed.  1e-10 keeps a margin of
 * three orders over that error. */
#define ORC_POS_EPS 1e-10

/* One cell: density scaled towards its mean by theta1 so that it is >= eps
 * at every point, then the whole state by theta2 so that the pressure is >=
 * eps at every point; eps = min(ORC_POS_EPS, mean density, mean pressure).
 * The cell mean never changes.  Returns 1 if the mean itself is not admissible
 * (the cell is then left as it is). */
typedef struct {
  int n;
  double br[64][ORC_MAXP], bs[64][ORC_MAXP]; /* psi_m(r_k), psi_n(s_k) */
} pos_table;

static void pos_make_table(const orc_ctx *x, pos_table *P) {
  double r[64], sv[64];
  P->n = pos_points(x, r, sv);
  for (int k = 0; k < P->n; ++k)
    for (int n = 0; n <= x->N; ++n) {
      P->br[k][n] = psi(n, r[k]);
      P->bs[k][n] = psi(n, sv[k]);
    }
}

static int positivity_cell(const orc_ctx *x, const pos_table *P, double *U, int i, int j, double *th) {
  double C[ORC_MAXV][ORC_MAXM], wb[ORC_MAXV];
  double k0 = cell_mean_factor(x);
  for (int v = 0; v < x->nv; ++v) {
    for (int q = 0; q < x->nm; ++q) C[v][q] = U[at(x, v, q, j, i)];
    wb[v] = C[v][0] * k0;
  }
  th[0] = th[1] = 1.0;
  double pb = pressure(x, wb);
  if (!(wb[0] > 0.0 && pb > 0.0)) return 1;
  double eps = fmin(ORC_POS_EPS, fmin(wb[0], pb));
  double rmin = INFINITY;
  for (int k = 0; k < P->n; ++k) {
    double w[ORC_MAXV];
    point_value(x, C, P->br[k], P->bs[k], w);
    rmin = fmin(rmin, w[0]);
  }
  if (rmin < eps) {
    th[0] = (wb[0] - eps) / (wb[0] - rmin);
    for (int q = 1; q < x->nm; ++q) C[0][q] *= th[0];
  }
  for (int k = 0; k < P->n; ++k) {
    double w[ORC_MAXV];
    point_value(x, C, P->br[k], P->bs[k], w);
    if (pressure(x, w) < eps) th[1] = fmin(th[1], pos_root(x, wb, w, eps));
  }
  if (th[1] < 1.0)
    for (int v = 0; v < x->nv; ++v)
      for (int q = 1; q < x->nm; ++q) C[v][q] *= th[1];
  if (th[0] < 1.0 || th[1] < 1.0)
    for (int v = 0; v < x->nv; ++v)
      for (int q = 1; q < x->nm; ++q) U[at(x, v, q, j, i)] = C[v][q];
  return 0;
}

/* Every cell; theta (optional): [2][ny][nx] = theta1, theta2. */
static int positivity_state(const orc_ctx *x, double *U, double *theta) {
  int bad = 0;
  pos_table P;
  pos_make_table(x, &P);
#pragma omp parallel for schedule(static) reduction(| : bad)
  for (int j = 0; j < x->ny; ++j)
    for (int i = 0; i < x->nx; ++i) {
      double th[2];
      bad |= positivity_cell(x, &P, U, i, j, th);
      if (theta) {
        size_t k = (size_t)j * x->nx + i;
        theta[k] = th[0];
        theta[(size_t)x->nx * x->ny + k] = th[1];
      }
    }
  return bad ? ORC_ERR_NONPHYSICAL : ORC_OK;
}

int orc_positivity(const orc_config *c, double *U, double *theta) {
  orc_ctx x;
  int rc = make_ctx(c, &x);
  if (rc) return rc;
  if (c->equation != ORC_EULER) return ORC_ERR_ARG;
  return positivity_state(&x, U, theta);
}

/* Ghost cell (i, j) outside the mesh (or an interior cell) as the boundary
 * conditions give it at the configuration's time: out [nv][nm]. */
int orc_ghost(const orc_config *c, const double *U, int32_t i, int32_t j, double *out) {
  orc_ctx x;
  int rc = make_ctx(c, &x);
  if (rc) return rc;
  if (i < -1 || i > x.nx || j < (c->dim == 2 ? -1 : 0) || j > (c->dim == 2 ? x.ny : 0)) return ORC_ERR_ARG;
  double C[ORC_MAXV][ORC_MAXM];
  fetch_cell(&x, U, i, j, C);
  for (int v = 0; v < x.nv; ++v)
    for (int q = 0; q < x.nm; ++q) out[v * x.nm + q] = C[v][q];
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Time step: CFL rule on cell means (the paper states none).                */
/* ------------------------------------------------------------------------ */

int orc_max_speed(const orc_config *c, const double *U, double *sx, double *sy) {
  orc_ctx x;
  int rc = make_ctx(c, &x);
  if (rc) return rc;
  double k0 = cell_mean_factor(&x), mx = 0.0, my = 0.0;
  int bad = 0;
  for (int j = 0; j < x.ny; ++j)
    for (int i = 0; i < x.nx; ++i) {
      double u[ORC_MAXV];
      for (int v = 0; v < x.nv; ++v) u[v] = U[at(&x, v, 0, j, i)] * k0;
      mx = fmax(mx, spectral_radius(&x, 0, u, &bad));
      if (c->dim == 2) my = fmax(my, spectral_radius(&x, 1, u, &bad));
    }
  *sx = mx;
  *sy = my;
  return bad ? ORC_ERR_NONPHYSICAL : ORC_OK;
}

int orc_cfl_dt(const orc_config *c, const double *U, double *dt) {
  if (c->xn) { /* non-uniform: the largest spectral radius over width per direction */
    orc_ctx x;
    int rc = make_ctx(c, &x);
    if (rc) return rc;
    double k0 = cell_mean_factor(&x), mx = 0.0, my = 0.0;
    int bad = 0;
    for (int j = 0; j < x.ny; ++j)
      for (int i = 0; i < x.nx; ++i) {
        double u[ORC_MAXV];
        for (int v = 0; v < x.nv; ++v) u[v] = U[at(&x, v, 0, j, i)] * k0;
        mx = fmax(mx, spectral_radius(&x, 0, u, &bad) / cell_hx(&x, i));
        if (c->dim == 2) my = fmax(my, spectral_radius(&x, 1, u, &bad) / cell_hy(&x, j));
      }
    if (bad) return ORC_ERR_NONPHYSICAL;
    double den = mx + my;
    *dt = den > 0.0 ? c->cfl / den : INFINITY;
    return ORC_OK;
  }
  double sx, sy;
  int rc = orc_max_speed(c, U, &sx, &sy);
  if (rc) return rc;
  double hx = (c->x1 - c->x0) / c->nx;
  if (c->dim == 1) {
    *dt = sx > 0.0 ? c->cfl * hx / sx : INFINITY;
  } else {
    double hy = (c->y1 - c->y0) / c->ny;
    double den = sx / hx + sy / hy;
    *dt = den > 0.0 ? c->cfl / den : INFINITY;
  }
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Third-order TVD (SSP) Runge-Kutta with the limiter after every stage.     */
/* ------------------------------------------------------------------------ */

/* Boundary data are taken at the time each stage's input approximates:
 * t^n for the first residual, t^n + dt for the limiter after the first stage
 * and the second residual, t^n + dt/2 for the limiter after the second stage
 * and the third residual, t^n + dt after the last stage (c->time = t^n). */
int orc_step(const orc_config *c, double *U, double dt) {
  orc_ctx x;
  int rc = make_ctx(c, &x);
  if (rc) return rc;
  size_t n = (size_t)x.nv * x.nm * x.ny * x.nx;
  double *U1 = (double *)malloc(n * sizeof(double)), *U2 = (double *)malloc(n * sizeof(double));
  double *L = (double *)malloc(n * sizeof(double)), *W = (double *)malloc(n * sizeof(double));
  if (!U1 || !U2 || !L || !W) {
    free(U1); free(U2); free(L); free(W);
    return ORC_ERR_ARG;
  }
  int bad = 0;
  int lim = c->limiter != ORC_LIM_NONE;
  double tn = c->time;
  orc_config cs = *c;
  orc_ctx xs = x;
  xs.c = &cs;
  /* stage 1: u1 = u + dt L(u) */
  cs.time = tn;
  if (orc_residual(&cs, U, L)) bad = 1;
  for (size_t k = 0; k < n; ++k) U1[k] = U[k] + dt * L[k];
  cs.time = xs.time = tn + dt;
  if (lim) limit_state(&xs, U1, W, NULL, NULL, NULL);
  if (c->positivity && positivity_state(&xs, U1, NULL)) bad = 1;
  /* stage 2: u2 = 3/4 u + 1/4 (u1 + dt L(u1)) */
  if (orc_residual(&cs, U1, L)) bad = 1;
  for (size_t k = 0; k < n; ++k) U2[k] = 0.75 * U[k] + 0.25 * (U1[k] + dt * L[k]);
  cs.time = xs.time = tn + 0.5 * dt;
  if (lim) limit_state(&xs, U2, W, NULL, NULL, NULL);
  if (c->positivity && positivity_state(&xs, U2, NULL)) bad = 1;
  /* stage 3: u = 1/3 u + 2/3 (u2 + dt L(u2)) */
  if (orc_residual(&cs, U2, L)) bad = 1;
  for (size_t k = 0; k < n; ++k) U[k] = U[k] / 3.0 + 2.0 * (U2[k] + dt * L[k]) / 3.0;
  cs.time = xs.time = tn + dt;
  if (lim) limit_state(&xs, U, W, NULL, NULL, NULL);
  if (c->positivity && positivity_state(&xs, U, NULL)) bad = 1;
  free(U1); free(U2); free(L); free(W);
  return bad ? ORC_ERR_NONPHYSICAL : ORC_OK;
}

/* Advance to t_end (or max_steps).  dt_fixed > 0 uses that step, otherwise
 * the CFL rule; the last step is clipped so that t lands on t_end. */
int orc_run(const orc_config *c, double *U, double *t, double t_end, double dt_fixed, int32_t max_steps,
            int32_t *steps, double *dt_log, int32_t dt_log_len) {
  int s = 0, rc = ORC_OK;
  while (*t < t_end && s < max_steps) {
    double dt = dt_fixed;
    if (!(dt_fixed > 0.0)) {
      rc = orc_cfl_dt(c, U, &dt);
      if (rc) break;
    }
    int last = 0;
    if (*t + dt >= t_end) {
      dt = t_end - *t;
      last = 1;
    }
    orc_config cs = *c;
    cs.time = *t;
    rc = orc_step(&cs, U, dt);
    if (dt_log && s < dt_log_len) dt_log[s] = dt;
    ++s;
    *t = last ? t_end : *t + dt;
    if (rc) break;
  }
  *steps = s;
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Initial data: L2 projection of point values onto the modal basis.        */
/* pv layout: [v][qy][qx][j][i] at the nodes returned by orc_proj_nodes.     */
/* ------------------------------------------------------------------------ */

int orc_proj_nodes(int order, double *r, double *w, int32_t *nq) {
  const orc_tables *T = tables(order);
  if (!T) return ORC_ERR_ARG;
  *nq = T->npq;
  for (int k = 0; k < T->npq; ++k) {
    if (r) r[k] = T->rpq[k];
    if (w) w[k] = T->wpq[k];
  }
  return ORC_OK;
}

int orc_project(const orc_config *c, const double *pv, double *U) {
  orc_ctx x;
  int rc = make_ctx(c, &x);
  if (rc) return rc;
  const orc_tables *T = x.T;
  int nq = T->npq, nqy = c->dim == 2 ? nq : 1, np = x.np;
  size_t plane = (size_t)x.nx * x.ny;
#pragma omp parallel for schedule(static)
  for (int j = 0; j < x.ny; ++j)
    for (int i = 0; i < x.nx; ++i)
      for (int v = 0; v < x.nv; ++v)
        for (int q = 0; q < x.nm; ++q) {
          int m = q % np, n = q / np;
          double s = 0.0;
          for (int b = 0; b < nqy; ++b)
            for (int a = 0; a < nq; ++a) {
              double val = pv[(((size_t)v * nqy + b) * nq + a) * plane + (size_t)j * x.nx + i];
              double wgt = T->wpq[a] * T->bpq[m][a];
              if (c->dim == 2) wgt *= T->wpq[b] * T->bpq[n][b];
              s += wgt * val;
            }
          U[at(&x, v, q, j, i)] = s;
        }
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Introspection for the pin tests.                                         */
/* ------------------------------------------------------------------------ */

/* Reconstruction rule, linear weights, the rows T_i[k] giving p_i(x_G) from
 * the stencil means, and the smoothness quadratic forms B_i (beta_i = a^T B_i a
 * over the cells of S_i), evaluated through the oracle's own routines. */
static int weno_tables_of(const orc_tables *T, int order, int32_t *ng, double *rg, double *wg, double *gam,
                          double *rows, double *bmat, int32_t *split, double *gam_resid) {
  if (!T) return ORC_ERR_ARG;
  int N = order, ns = 2 * N + 1;
  *ng = T->ng;
  *gam_resid = T->gam_resid;
  for (int G = 0; G < T->ng; ++G) {
    rg[G] = T->rg[G];
    wg[G] = T->wg[G];
    split[G] = T->split[G];
    for (int i = 0; i <= N; ++i) {
      gam[G * (N + 1) + i] = T->gam[G][i];
      for (int k = 0; k < ns; ++k) {
        double a[ORC_MAXS] = {0}, c[ORC_MAXP];
        a[k] = 1.0;
        double v = 0.0;
        if (k >= i && k <= i + N) {
          small_poly(T, i, a, c);
          for (int d = 0; d <= N; ++d) v += c[d] * pow(0.5 * T->rg[G], d);
        }
        rows[(G * (N + 1) + i) * ns + k] = v;
      }
    }
  }
  /* polarisation of the quadratic form: B[k][l] = (b(e_k+e_l) - b(e_k) - b(e_l))/2 */
  for (int i = 0; i <= N; ++i)
    for (int k = 0; k <= N; ++k)
      for (int l = 0; l <= N; ++l) {
        double a[ORC_MAXS] = {0}, c[ORC_MAXP];
        a[i + k] += 1.0;
        a[i + l] += 1.0;
        small_poly(T, i, a, c);
        double bkl = smoothness(N, c);
        double bk, bl;
        memset(a, 0, sizeof(a));
        a[i + k] = 1.0;
        small_poly(T, i, a, c);
        bk = smoothness(N, c);
        memset(a, 0, sizeof(a));
        a[i + l] = 1.0;
        small_poly(T, i, a, c);
        bl = smoothness(N, c);
        double v = (k == l) ? bk : 0.5 * (bkl - bk - bl);
        bmat[(i * (N + 1) + k) * (N + 1) + l] = v;
      }
  return ORC_OK;
}

int orc_weno_tables(int order, int32_t *ng, double *rg, double *wg, double *gam, double *rows, double *bmat,
                    int32_t *split, double *gam_resid) {
  return weno_tables_of(tables(order), order, ng, rg, wg, gam, rows, bmat, split, gam_resid);
}

/* The same for a troubled cell whose neighbours are rl and rr times as wide
 * (non-uniform meshes); the stencil cells in units of the cell's width are
 * returned in cl, cr (2N+1 each). */
int orc_weno_tables_nu(int order, double rl, double rr, int32_t *ng, double *rg, double *wg, double *gam,
                       double *rows, double *bmat, int32_t *split, double *gam_resid, double *cl, double *cr) {
  if (order < 1 || order > ORC_MAXN || !(rl > 0.0) || !(rr > 0.0)) return ORC_ERR_ARG;
  orc_tables *T = (orc_tables *)malloc(sizeof(orc_tables));
  if (!T) return ORC_ERR_ARG;
  int rc = build_tables_into(T, order, rl, rr);
  if (!rc) rc = weno_tables_of(T, order, ng, rg, wg, gam, rows, bmat, split, gam_resid);
  if (!rc)
    for (int k = 0; k < 2 * order + 1; ++k) {
      cl[k] = T->cl[k];
      cr[k] = T->cr[k];
    }
  free(T);
  return rc;
}

/* One WENO reconstruction through the oracle's own routine (pin tests). */
int orc_weno_eval(int order, int G, const double *a, double eps, int negw_mode, double *out) {
  const orc_tables *T = tables(order);
  if (!T || G < 0 || G >= T->ng) return ORC_ERR_ARG;
  *out = orc_weno_point(T, G, a, eps, negw_mode);
  return ORC_OK;
}

int orc_subcell_means(int order, double *sub) {
  const orc_tables *T = tables(order);
  if (!T) return ORC_ERR_ARG;
  for (int k = 0; k < order; ++k)
    for (int n = 0; n <= order; ++n) sub[k * (order + 1) + n] = T->sub[k][n];
  return ORC_OK;
}

int orc_quadrature(int kind, int n, double *x, double *w) {
  if (n < 2 || n > 12) return ORC_ERR_ARG;
  if (kind == 0) gauss_rule(n, x, w);
  else gauss_lobatto_rule(n, x, w);
  return ORC_OK;
}

int orc_basis(int n, double r, double *val, double *der) {
  *val = psi(n, r);
  *der = dpsi(n, r);
  return ORC_OK;
}

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
