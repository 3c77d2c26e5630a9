"""Pins of the oracle's derived tables against what the paper prints and what
the mathematics fixes (CPU only).

* quadrature nodes: Section 3, Step 1 prints them;
* P2 reconstruction rows, linear weights and smoothness indicators: Section 3,
  Steps 3-4 print them (golden fixture, with the misprints it lists fixed);
* P1: the textbook two-cell linear reconstruction (the paper says P1 is the
  standard WENO3 of Qiu and Shu);
* P3: the paper prints nothing; pinned by an independent exact derivation
  (sympy, primitive-function interpolation) and by polynomial reproduction.
"""
import json
import os

import numpy as np
import pytest
import sympy as sp

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "p2_weno_tables.json")


def _ev(expr):
    return float(sp.sympify(expr))


def test_quadrature_nodes_match_paper(oracle):
    g = json.load(open(GOLDEN))["quadrature_nodes"]
    for N, key in ((1, "P1"), (2, "P2"), (3, "P3")):
        t = oracle.weno_tables(N)
        want = np.array([_ev(e) for e in g[key]])
        np.testing.assert_allclose(t["rg"], want, rtol=0, atol=2e-16)
        assert abs(t["wg"].sum() - 2.0) < 1e-15


def test_gauss_rules_match_library(oracle):
    for n in range(2, 9):
        x, w = oracle.quadrature(0, n)
        xr, wr = np.polynomial.legendre.leggauss(n)
        np.testing.assert_allclose(x, xr, atol=1e-15)
        np.testing.assert_allclose(w, wr, atol=1e-15)
    x, w = oracle.quadrature(1, 4)
    np.testing.assert_allclose(x, [-1, -1 / np.sqrt(5), 1 / np.sqrt(5), 1], atol=1e-16)
    np.testing.assert_allclose(w, [1 / 6, 5 / 6, 5 / 6, 1 / 6], atol=1e-16)


def test_basis_is_orthonormal_legendre(oracle):
    xr, wr = np.polynomial.legendre.leggauss(10)
    for n in range(4):
        c = np.zeros(n + 1)
        c[n] = 1.0
        ref = np.sqrt((2 * n + 1) / 2) * np.polynomial.legendre.legval(xr, c)
        dref = np.sqrt((2 * n + 1) / 2) * np.polynomial.legendre.legval(xr, np.polynomial.legendre.legder(c))
        got = np.array([oracle.basis(n, r) for r in xr])
        np.testing.assert_allclose(got[:, 0], ref, atol=1e-14)
        np.testing.assert_allclose(got[:, 1], dref, atol=1e-13)
        for m in range(4):
            vm = np.array([oracle.basis(m, r)[0] for r in xr])
            assert abs((wr * got[:, 0] * vm).sum() - (n == m)) < 1e-14


def test_p2_tables_match_paper(oracle):
    g = json.load(open(GOLDEN))
    t = oracle.weno_tables(2)
    for G, pt in enumerate(g["points"]):
        assert abs(t["rg"][G] - _ev(pt["r"])) < 1e-15
        T = np.array([[_ev(e) for e in row] for row in pt["T"]])
        # rows p0, p1, p2 against the oracle's own reconstruction rows
        np.testing.assert_allclose(t["rows"][G], T[:3], atol=1e-14)
        gam = np.array([_ev(e) for e in pt["gamma"]])
        np.testing.assert_allclose(t["gamma"][G], gam, atol=1e-14)
        # the Q row must equal sum_i gamma_i p_i (the defining identity of Step 3)
        np.testing.assert_allclose(gam @ T[:3], T[3], atol=1e-14)


def test_p2_smoothness_indicators_match_paper(oracle):
    g = json.load(open(GOLDEN))["beta"]
    t = oracle.weno_tables(2)
    rng = np.random.default_rng(0)
    for _ in range(20):
        a = rng.normal(size=5)
        for i in range(3):
            spec = g[f"beta{i}"]
            want = 0.0
            for term, coef in spec["terms"].items():
                u, v = term.split("*")
                want += coef * a[int(u[1])] * a[int(v[1])]
            want /= spec["den"]
            B = t["beta"][i]
            got = a[i:i + 3] @ B @ a[i:i + 3]
            assert abs(got - want) < 1e-12 * max(1.0, abs(want))


def test_p1_is_textbook_weno3(oracle):
    t = oracle.weno_tables(1)
    s = np.sqrt(3) / 6
    np.testing.assert_allclose(t["rows"][0], [[s, 1 - s, 0], [0, 1 + s, -s]], atol=1e-15)
    np.testing.assert_allclose(t["rows"][1], [[-s, 1 + s, 0], [0, 1 - s, s]], atol=1e-15)
    np.testing.assert_allclose(t["gamma"], 0.5, atol=1e-15)
    a = np.array([0.3, -1.2, 2.0])
    for i in range(2):
        B = t["beta"][i]
        assert abs(a[i:i + 2] @ B @ a[i:i + 2] - (a[i + 1] - a[i]) ** 2) < 1e-14


def _exact_tables(N):
    """Independent exact derivation: p_i is the derivative of the Lagrange
    interpolant of the primitive function through the cell edges of S_i."""
    x = sp.Symbol("x")
    edges = [sp.Rational(-3, 2) + sp.Rational(k, N) for k in range(N + 1)]
    edges += [sp.Rational(1, 2) + sp.Rational(k, N) for k in range(N + 1)]
    widths = [edges[k + 1] - edges[k] for k in range(2 * N + 1)]
    if N == 1:
        pts = [-1 / sp.sqrt(3), 1 / sp.sqrt(3)]
    elif N == 2:
        pts = [-1, -1 / sp.sqrt(5), 1 / sp.sqrt(5), 1]
    else:
        pts = [-sp.sqrt(525 + 70 * sp.sqrt(30)) / 35, -sp.sqrt(525 - 70 * sp.sqrt(30)) / 35,
               sp.sqrt(525 - 70 * sp.sqrt(30)) / 35, sp.sqrt(525 + 70 * sp.sqrt(30)) / 35]

    def rows_for(cells):
        e = [edges[c] for c in cells] + [edges[cells[-1] + 1]]
        polys = []
        for k in cells:  # unit mean in cell k: primitive jumps by width_k at its right edge
            vals = [sum(widths[c] for c in cells if c == k and edges[c + 1] <= ee) for ee in e]
            P = sp.interpolate(list(zip(e, vals)), x)
            polys.append(sp.diff(P, x))
        return polys

    small = [rows_for(list(range(i, i + N + 1))) for i in range(N + 1)]
    big = rows_for(list(range(2 * N + 1)))
    out = []
    for r in pts:
        xi = sp.nsimplify(r) / 2
        R = [[sp.nsimplify(sp.expand(p.subs(x, xi))) for p in polys] for polys in small]
        Q = [sp.expand(p.subs(x, xi)) for p in big]
        out.append((R, Q))
    return out


@pytest.mark.parametrize("N", [1, 2, 3])
def test_tables_match_exact_derivation(oracle, N):
    t = oracle.weno_tables(N)
    ex = _exact_tables(N)
    for G, (R, Q) in enumerate(ex):
        for i in range(N + 1):
            want = np.zeros(2 * N + 1)
            want[i:i + N + 1] = [float(sp.N(v, 30)) for v in R[i]]
            np.testing.assert_allclose(t["rows"][G, i], want, atol=1e-12)
        # linear weights: the oracle's gamma reproduce Q exactly
        Qn = np.array([float(sp.N(v, 30)) for v in Q])
        np.testing.assert_allclose(t["gamma"][G] @ t["rows"][G], Qn, atol=1e-12)


def test_p3_inner_points_have_negative_weights(oracle):
    t = oracle.weno_tables(3)
    assert list(t["split"]) == [0, 1, 1, 0]
    assert t["gamma"][1].min() < -0.69 and t["gamma"][2].min() < -0.69
    np.testing.assert_allclose(t["gamma"].sum(axis=1), 1.0, atol=1e-13)


@pytest.mark.parametrize("N", [1, 2, 3])
def test_reconstruction_reproduces_polynomials(oracle, N):
    """Means of a polynomial of degree <= N are reconstructed exactly by every
    p_i, so the WENO value equals it for any weights (split form included)."""
    t = oracle.weno_tables(N)
    edges = np.concatenate([-1.5 + np.arange(N + 1) / N, 0.5 + np.arange(N + 1) / N])
    rng = np.random.default_rng(N)
    for _ in range(5):
        c = rng.normal(size=N + 1)
        P = np.polynomial.Polynomial(c)
        I = P.integ()
        a = np.array([(I(edges[k + 1]) - I(edges[k])) / (edges[k + 1] - edges[k]) for k in range(2 * N + 1)])
        for G in range(len(t["rg"])):
            want = P(0.5 * t["rg"][G])
            for mode in (0, 1):
                got = oracle.weno_eval(N, G, a, 1e-6, mode)
                assert abs(got - want) < 1e-11 * max(1.0, np.abs(a).max())


def test_subcell_means_closed_form(oracle):
    for N in (1, 2, 3):
        s = oracle.subcell_means(N)
        for k in range(N):
            a, b = -1 + 2 * k / N, -1 + 2 * (k + 1) / N
            for n in range(N + 1):
                c = np.zeros(n + 1)
                c[n] = 1.0
                I = np.polynomial.legendre.legint(c)
                want = np.sqrt((2 * n + 1) / 2) * (np.polynomial.legendre.legval(b, I)
                                                  - np.polynomial.legendre.legval(a, I)) / (b - a)
                assert abs(s[k, n] - want) < 1e-15
