// Host-side derivation of the coefficient tables the kernels use, in long
// double, rounded once to double.
//
// Kochi & Ramakrishna (arXiv 1904.11147), Section 3:
//  * Step 1 fixes the reconstruction points: 2-point Gauss for P1, 4-point
//    Gauss-Lobatto for P2, 4-point Gauss for P3 (closed forms below);
//  * Step 2 defines p_i on the small stencils S_i and Q on the big stencil
//    T of the compact subcell stencil (neighbours cut into N equal parts).
//    Here p_i is obtained as the derivative of the Lagrange interpolant of
//    the primitive function through the cell edges of S_i;
//  * Step 3 defines the linear weights by Q(x_G) = sum_i gamma_i p_i(x_G),
//    solved here by forward substitution on the leftmost N+1 stencil cells
//    and verified on all 2N+1;
//  * Step 4 defines the smoothness indicators, stored as quadratic forms;
//  * Step 6 projects point values with the reconstruction rule's weights.
// Section 2 fixes the orthonormal Legendre basis psi_n = sqrt((2n+1)/2) P_n.
#include <cmath>
#include <cstring>

#include "dg_internal.h"

namespace dg {
namespace {

using ld = long double;

ld legendre(int n, ld r) {
  switch (n) {
    case 0: return 1.0L;
    case 1: return r;
    case 2: return 0.5L * (3.0L * r * r - 1.0L);
    case 3: return 0.5L * (5.0L * r * r * r - 3.0L * r);
    case 4: return 0.125L * (35.0L * r * r * r * r - 30.0L * r * r + 3.0L);
    default: {
      ld p0 = 1.0L, p1 = r;
      for (int k = 1; k < n; ++k) {
        ld p2 = ((2 * k + 1) * r * p1 - k * p0) / (k + 1);
        p0 = p1;
        p1 = p2;
      }
      return p1;
    }
  }
}

ld legendre_d(int n, ld r) {
  switch (n) {
    case 0: return 0.0L;
    case 1: return 1.0L;
    case 2: return 3.0L * r;
    case 3: return 0.5L * (15.0L * r * r - 3.0L);
    default: return n * (r * legendre(n, r) - legendre(n - 1, r)) / (r * r - 1.0L);
  }
}

ld norm(int n) { return std::sqrt((2.0L * n + 1.0L) / 2.0L); }

// antiderivative of P_n vanishing at r = -1
ld legendre_int(int n, ld r) {
  if (n == 0) return r + 1.0L;
  return (legendre(n + 1, r) - legendre(n - 1, r)) / (2.0L * n + 1.0L);
}

// n-point Gauss-Legendre on [-1,1] by Newton's method, ascending.
void gauss(int n, ld *x, ld *w) {
  for (int i = 0; i < n; ++i) {
    ld r = std::cos(3.14159265358979323846264338327950288L * (n - i - 0.25L) / (n + 0.5L));
    for (int it = 0; it < 200; ++it) {
      ld p = legendre(n, r);
      ld dp = n * (r * p - legendre(n - 1, r)) / (r * r - 1.0L);
      ld d = p / dp;
      r -= d;
      if (std::fabs(d) < 1e-21L) break;
    }
    ld dp = n * (r * legendre(n, r) - legendre(n - 1, r)) / (r * r - 1.0L);
    x[i] = r;
    w[i] = 2.0L / ((1.0L - r * r) * dp * dp);
  }
}

// Step 1 rules in closed form.
void recon_rule(int N, int *ng, ld *x, ld *w) {
  if (N == 1) {
    *ng = 2;
    x[0] = -1.0L / std::sqrt(3.0L);
    x[1] = -x[0];
    w[0] = w[1] = 1.0L;
  } else if (N == 2) {
    *ng = 4;
    x[0] = -1.0L;
    x[1] = -1.0L / std::sqrt(5.0L);
    x[2] = -x[1];
    x[3] = 1.0L;
    w[0] = w[3] = 1.0L / 6.0L;
    w[1] = w[2] = 5.0L / 6.0L;
  } else {
    *ng = 4;
    ld s = std::sqrt(30.0L);
    ld outer = std::sqrt(525.0L + 70.0L * s) / 35.0L, inner = std::sqrt(525.0L - 70.0L * s) / 35.0L;
    x[0] = -outer;
    x[1] = -inner;
    x[2] = inner;
    x[3] = outer;
    w[0] = w[3] = (18.0L - s) / 36.0L;
    w[1] = w[2] = (18.0L + s) / 36.0L;
  }
}

// Derivative at x of the Lagrange basis polynomial l of the nodes e[0..n-1].
ld lagrange_d(const ld *e, int n, int l, ld x) {
  ld s = 0.0L;
  for (int m = 0; m < n; ++m) {
    if (m == l) continue;
    ld t = 1.0L / (e[l] - e[m]);
    for (int k = 0; k < n; ++k)
      if (k != l && k != m) t *= (x - e[k]) / (e[l] - e[k]);
    s += t;
  }
  return s;
}

// Monomial coefficients (degree < n) of the Lagrange basis polynomial l.
void lagrange_coeffs(const ld *e, int n, int l, ld *c) {
  ld poly[16] = {1.0L};
  int deg = 0;
  ld den = 1.0L;
  for (int k = 0; k < n; ++k) {
    if (k == l) continue;
    for (int d = deg + 1; d >= 1; --d) poly[d] = poly[d - 1] - e[k] * poly[d];
    poly[0] = -e[k] * poly[0];
    ++deg;
    den *= e[l] - e[k];
  }
  for (int d = 0; d < n; ++d) c[d] = poly[d] / den;
}

// Reconstruction of the value at x from the means on cells c0..c0+nc-1 of the
// stencil with edges e[] and widths wdt[]: weights on each mean.
void stencil_row(const ld *edges, const ld *wdt, int c0, int nc, ld x, ld *row) {
  ld e[16];
  for (int l = 0; l <= nc; ++l) e[l] = edges[c0 + l];
  for (int c = 0; c < nc; ++c) {
    // a unit mean in cell c lifts the primitive by wdt at every edge right of it
    ld s = 0.0L;
    for (int l = c + 1; l <= nc; ++l) s += lagrange_d(e, nc + 1, l, x);
    row[c] = wdt[c0 + c] * s;
  }
}

// Monomial coefficients of p for a unit mean in cell c of stencil c0..c0+nc-1.
void stencil_poly(const ld *edges, const ld *wdt, int c0, int nc, int c, ld *coef /* nc */) {
  ld e[16], lc[16];
  for (int l = 0; l <= nc; ++l) e[l] = edges[c0 + l];
  ld P[16] = {0};
  for (int l = c + 1; l <= nc; ++l) {
    lagrange_coeffs(e, nc + 1, l, lc);
    for (int d = 0; d <= nc; ++d) P[d] += wdt[c0 + c] * lc[d];
  }
  for (int d = 0; d < nc; ++d) coef[d] = (d + 1) * P[d + 1];  // derivative of the primitive
}

ld int_centre(int d) {  // integral of xi^d over [-1/2, 1/2]
  if (d & 1) return 0.0L;
  return 2.0L * std::pow(0.5L, d + 1) / (d + 1);
}

}  // namespace

int build_weno_coef(int N, double rl_in, double rr_in, WenoCoef *o) {
  if (N < 1 || N > kMaxN || !(rl_in > 0.0) || !(rr_in > 0.0)) return DG_ERR_UNSUPPORTED;
  std::memset(o, 0, sizeof(*o));
  const int NP = N + 1, NS = 2 * N + 1;
  const ld rl = rl_in, rr = rr_in;
  int ng;
  ld rg[4], wg[4];
  recon_rule(N, &ng, rg, wg);

  // Step 2: the compact stencil in units of the troubled cell's width,
  // centred on it: N subcells of each neighbour around the whole cell (the
  // neighbours rl and rr times as wide as the cell).
  ld edges[16], wdt[16];
  for (int k = 0; k <= N; ++k) {
    edges[k] = (-0.5L - rl) + k * rl / N;
    edges[N + 1 + k] = 0.5L + k * rr / N;
  }
  for (int c = 0; c < NS; ++c) wdt[c] = edges[c + 1] - edges[c];

  ld Tl[4][4][4];
  for (int G = 0; G < ng; ++G) {
    ld xg = 0.5L * rg[G];
    for (int i = 0; i < NP; ++i) {
      ld row[8];
      stencil_row(edges, wdt, i, NP, xg, row);
      for (int k = 0; k < NP; ++k) {
        Tl[G][i][k] = row[k];
        o->T[G][i][k] = (double)row[k];
      }
    }
    ld qrow[8];
    stencil_row(edges, wdt, 0, NS, xg, qrow);
    // Step 3: triangular structure on the leftmost cells.
    ld gam[4];
    for (int k = 0; k < NP; ++k) {
      ld s = qrow[k];
      for (int i = 0; i < k; ++i) s -= gam[i] * Tl[G][i][k - i];
      gam[k] = s / Tl[G][k][0];
    }
    ld resid = 0.0L;
    for (int k = 0; k < NS; ++k) {
      ld s = -qrow[k];
      for (int i = 0; i < NP; ++i)
        if (k - i >= 0 && k - i < NP) s += gam[i] * Tl[G][i][k - i];
      resid = std::fmax(resid, std::fabs(s));
    }
    if (resid > 1e-14L) return DG_ERR_UNSUPPORTED;
    bool neg = false;
    for (int i = 0; i < NP; ++i) {
      o->gam[G][i] = (double)gam[i];
      if (gam[i] < 0.0L) neg = true;
    }
    o->split[G] = neg ? 1 : 0;
    // positive/negative groups (theta = 3) for points with a negative weight
    const ld theta = 3.0L;
    ld gp[4], gm[4], sp = 0.0L, sm = 0.0L;
    for (int i = 0; i < NP; ++i) {
      gp[i] = 0.5L * (gam[i] + theta * std::fabs(gam[i]));
      gm[i] = gp[i] - gam[i];
      sp += gp[i];
      sm += gm[i];
    }
    o->sp[G] = (double)sp;
    o->sm[G] = (double)sm;
    for (int i = 0; i < NP; ++i) {
      o->gpn[G][i] = (double)(gp[i] / sp);
      o->gmn[G][i] = (double)(gm[i] / sm);
    }
  }

  // Step 4: beta_i = sum_{l=1..N} int_{-1/2}^{1/2} (p_i^(l))^2 as a quadratic form.
  for (int i = 0; i < NP; ++i) {
    ld coef[4][8];
    for (int k = 0; k < NP; ++k) stencil_poly(edges, wdt, i, NP, k, coef[k]);
    for (int k = 0; k < NP; ++k)
      for (int l2 = 0; l2 < NP; ++l2) {
        ld s = 0.0L;
        for (int l = 1; l <= N; ++l)
          for (int d1 = l; d1 < NP; ++d1)
            for (int d2 = l; d2 < NP; ++d2) {
              ld f1 = 1.0L, f2 = 1.0L;
              for (int t = 0; t < l; ++t) {
                f1 *= (ld)(d1 - t);
                f2 *= (ld)(d2 - t);
              }
              s += coef[k][d1] * f1 * coef[l2][d2] * f2 * int_centre(d1 - l + d2 - l);
            }
        o->B[i][k][l2] = (double)s;
      }
  }

  return DG_OK;
}

int build_order_tables(int N, OrderTables *o) {
  if (N < 1 || N > kMaxN) return DG_ERR_UNSUPPORTED;
  std::memset(o, 0, sizeof(*o));
  const int NP = N + 1, NS = 2 * N + 1;
  o->N = N;

  // Section 2: volume/edge rule and basis values.
  ld rq[8], wq[8];
  gauss(NP, rq, wq);
  for (int q = 0; q < NP; ++q) o->wq[q] = (double)wq[q];
  for (int n = 0; n < NP; ++n) {
    for (int q = 0; q < NP; ++q) {
      o->bq[n][q] = (double)(norm(n) * legendre(n, rq[q]));
      o->dbq[n][q] = (double)(norm(n) * legendre_d(n, rq[q]));
    }
    o->bm[n] = (double)(norm(n) * legendre(n, -1.0L));
    o->bp[n] = (double)(norm(n) * legendre(n, 1.0L));
    o->b0[n] = (double)(norm(n) * legendre(n, 0.0L));
  }

  // Step 1.
  int ng;
  ld rg[4], wg[4];
  recon_rule(N, &ng, rg, wg);
  o->ng = ng;
  for (int G = 0; G < ng; ++G) {
    o->wg[G] = (double)wg[G];
    for (int n = 0; n < NP; ++n) o->bg[n][G] = (double)(norm(n) * legendre(n, rg[G]));
  }

  WenoCoef w;
  int rc = build_weno_coef(N, 1.0, 1.0, &w);
  if (rc) return rc;
  std::memcpy(o->T, w.T, sizeof(w.T));
  std::memcpy(o->gam, w.gam, sizeof(w.gam));
  std::memcpy(o->split, w.split, sizeof(w.split));
  std::memcpy(o->gpn, w.gpn, sizeof(w.gpn));
  std::memcpy(o->gmn, w.gmn, sizeof(w.gmn));
  std::memcpy(o->sp, w.sp, sizeof(w.sp));
  std::memcpy(o->sm, w.sm, sizeof(w.sm));
  std::memcpy(o->B, w.B, sizeof(w.B));

  // Means of psi_n over the N equal subcells of [-1,1].
  for (int k = 0; k < N; ++k) {
    ld a = -1.0L + 2.0L * k / N, b = -1.0L + 2.0L * (k + 1) / N;
    for (int n = 0; n < NP; ++n)
      o->sub[k][n] = (double)(norm(n) * (legendre_int(n, b) - legendre_int(n, a)) / (b - a));
  }

  // Projection rule: two panels, (N+2)-point Gauss on each.
  ld px[8], pw[8];
  int m = N + 2;
  gauss(m, px, pw);
  o->npq = 2 * m;
  for (int k = 0; k < m; ++k) {
    ld r0 = -0.5L + 0.5L * px[k], r1 = 0.5L + 0.5L * px[k];
    o->rpq[k] = (double)r0;
    o->rpq[m + k] = (double)r1;
    o->wpq[k] = o->wpq[m + k] = (double)(0.5L * pw[k]);
    for (int n = 0; n < NP; ++n) {
      o->bpq[n][k] = (double)(norm(n) * legendre(n, r0));
      o->bpq[n][m + k] = (double)(norm(n) * legendre(n, r1));
    }
  }
  return DG_OK;
}

}  // namespace dg
