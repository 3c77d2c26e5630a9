"""Pins of the oracle on non-uniform tensor-product meshes (the paper's
accuracy tests move every node of the uniform mesh by up to 10%).

* The stencil tables of a cell whose neighbours are rl, rr times as wide:
  every p_i reproduces polynomials of degree <= N from their exact stencil
  means, the linear weights make sum gamma_i p_i reproduce degree <= 2N (the
  big-stencil polynomial Q), beta of a linear profile is its exact integral;
  with rl = rr = 1 they are the uniform tables.
* The limiter reproduces polynomial data on a perturbed mesh (1D, 2D).
* The residual of a globally linear Burgers state equals the projection of
  -f(u)_x (-f_x - g_y in 2D) on the perturbed cells (widths enter through
  the 2/h factor of every cell).
* Free stream, conservation (sum of width times mean), the CFL rule, and
  the design order of the paper's Tables 1 and 3 on a 10%-perturbed mesh.
"""
import numpy as np
import pytest

from paper_1904_11147_amd import workloads as W
from tests import exact
from tests.dgutil import oracle_initial_state, oracle_problem, orders, psi_table


def _mono_mean(d, a, b):
    return (b ** (d + 1) - a ** (d + 1)) / ((d + 1) * (b - a))


@pytest.mark.parametrize("order", [1, 2, 3])
def test_stencil_tables_on_uneven_neighbours(oracle, order):
    rng = np.random.default_rng(order)
    N = order
    uni = oracle.weno_tables(N)
    same = oracle.weno_tables(N, 1.0, 1.0)
    np.testing.assert_array_equal(same["rows"], uni["rows"])
    np.testing.assert_array_equal(same["gamma"], uni["gamma"])
    for _ in range(6):
        rl, rr = rng.uniform(0.8, 1.25, 2)
        t = oracle.weno_tables(N, rl, rr)
        cells = t["cells"]
        np.testing.assert_allclose(cells[0], [-0.5 - rl, -0.5 - rl + rl / N], rtol=1e-15)
        np.testing.assert_allclose(cells[-1], [0.5 + rr - rr / N, 0.5 + rr], rtol=1e-15)
        xg = 0.5 * t["rg"]
        for d in range(2 * N + 1):
            means = np.array([_mono_mean(d, a, b) for a, b in cells])
            q = np.einsum("Gi,Gik,k->G", t["gamma"], t["rows"], means)  # sum_i gamma_i p_i(x_G)
            np.testing.assert_allclose(q, xg ** d, atol=1e-12)
            if d <= N:
                np.testing.assert_allclose(t["rows"] @ means, np.broadcast_to(xg[:, None] ** d, (len(xg), N + 1)),
                                           atol=1e-12)
        # beta of the linear profile x: p_i = x for every i, integral of 1 over the cell
        means = np.array([_mono_mean(1, a, b) for a, b in cells])
        for i in range(N + 1):
            a = means[i:i + N + 1]
            np.testing.assert_allclose(a @ t["beta"][i] @ a, 1.0, rtol=1e-11)
        assert t["gamma_residual"] < 1e-12


def _poly_state(prob, coef_x, coef_y=None, nv=1):
    """Projection of the polynomial sum_d coef_x[d] x^d (+ sum coef_y[d] y^d)."""
    X, Y = prob.node_coords()
    r, _ = prob.proj_nodes()
    px = np.polynomial.polynomial.polyval
    if prob.dim == 1:
        pv = np.stack([px(X, coef_x) * (1 + 0.1 * v) for v in range(nv)])[:, :, None, :]
    else:
        XX = np.broadcast_to(X[None, :, None, :], (len(r), len(r), prob.ny, prob.nx))
        YY = np.broadcast_to(Y[:, None, :, None], (len(r), len(r), prob.ny, prob.nx))
        pv = np.stack([(px(XX, coef_x) + px(YY, coef_y)) * (1 + 0.1 * v) for v in range(nv)])
    return prob.project(np.ascontiguousarray(pv))


@pytest.mark.parametrize("order", [1, 2, 3])
def test_limiter_reproduces_polynomials_on_perturbed_mesh(oracle, order):
    n = 12
    xn = W.perturbed_nodes(n, 0.0, 1.0, seed=10 + order)
    p = oracle.Problem(dim=1, equation=0, order=order, nx=n, bc=(1, 1, 0, 0), xn=xn)
    c = np.random.default_rng(order).normal(size=order + 1)
    U = _poly_state(p, c)
    out, f, _ = p.limit(U, flags=np.ones((1, n), dtype=np.uint8))
    inner = slice(1, n - 1)  # the mirrored ghosts are not the polynomial
    np.testing.assert_allclose(out[..., inner], U[..., inner], atol=1e-11)
    # 2D tensor mesh, polynomial in x plus polynomial in y
    yn = W.perturbed_nodes(10, 0.0, 1.0, seed=20 + order)
    p2 = oracle.Problem(dim=2, equation=0, order=order, nx=n, ny=10, bc=(1, 1, 1, 1), xn=xn, yn=yn)
    cy = np.random.default_rng(order + 5).normal(size=order + 1)
    U2 = _poly_state(p2, c, cy)
    out2, _, _ = p2.limit(U2, flags=np.ones((10, n), dtype=np.uint8))
    np.testing.assert_allclose(out2[..., 1:-1, 1:-1], U2[..., 1:-1, 1:-1], atol=1e-11)
    assert np.abs(U2[:, 1:]).max() > 0.01  # not a trivial state


@pytest.mark.parametrize("dim", [1, 2])
def test_residual_of_linear_burgers_state_on_perturbed_mesh(oracle, dim):
    """u = a + b x (+ c y) is continuous, so the LLF flux is the exact flux and
    the residual is the projection of -u (b + c), exactly (degree 1)."""
    n, order = 10, 2
    a, b, c = 0.3, 0.7, -0.4
    kw = dict(xn=W.perturbed_nodes(n, 0.0, 1.0, seed=3))
    if dim == 2:
        kw["yn"] = W.perturbed_nodes(n, 0.0, 1.0, seed=4)
    p = oracle.Problem(dim=dim, equation=0, order=order, nx=n, ny=n if dim == 2 else 1, bc=(0, 0, 0, 0), **kw)
    if dim == 1:
        U = _poly_state(p, [a, b])
        want = _poly_state(p, [-a * b, -b * b])
    else:
        U = _poly_state(p, [a, b], [0.0, c])
        s = b + c
        want = _poly_state(p, [-a * s, -b * s], [0.0, -c * s])
    L = p.residual(U)
    # periodic wrap breaks continuity at the domain boundary: interior cells only
    sl = (Ellipsis, slice(1, n - 1)) if dim == 1 else (Ellipsis, slice(1, n - 1), slice(1, n - 1))
    np.testing.assert_allclose(L[sl], want[sl], atol=1e-12)


def test_free_stream_and_cfl_on_perturbed_mesh(oracle):
    n = 9
    xn, yn = W.perturbed_nodes(n, 0.0, 1.0, seed=5), W.perturbed_nodes(n, 0.0, 2.0, seed=6)
    p = oracle.Problem(dim=2, equation=1, order=2, nx=n, ny=n, y1=2.0, bc=(1, 1, 1, 1), xn=xn, yn=yn, cfl=0.2)
    U = p.zeros()
    for v, c in enumerate(W.euler2d_conserved(1.2, 0.5, -0.3, 0.9)):
        U[v, 0] = 2.0 * float(c)
    assert np.abs(p.residual(U)).max() < 1e-12
    cs = np.sqrt(1.4 * 0.9 / 1.2)
    want = 0.2 / ((0.5 + cs) / np.diff(xn).min() + (0.3 + cs) / np.diff(yn).min())
    np.testing.assert_allclose(p.cfl_dt(U), want, rtol=1e-14)


def test_conservation_on_perturbed_mesh(oracle):
    wl = W.burgers1d(nx=40, order=2, t_end=0.6).nonuniform(seed=7)
    prob, U0 = oracle_initial_state(oracle, wl, limit=True)
    h = np.diff(wl.mesh["xn"])
    U, t, steps, _ = prob.run(U0, 0.0, wl.t_end)
    assert steps > 20
    mass = lambda V: float((h * V[0, 0, 0] / np.sqrt(2.0)).sum())  # noqa: E731
    assert abs(mass(U) - mass(U0)) < 1e-13


def _l1_1d(U, order, xn, f):
    r, w = np.polynomial.legendre.leggauss(order + 4)
    h = np.diff(xn)
    X = xn[None, :-1] + 0.5 * (1 + r[:, None]) * h[None, :]
    vals = np.einsum("nx,nq->qx", U[0, :, 0, :], psi_table(order, r))
    return float((w[:, None] * np.abs(vals - f(X)) * 0.5 * h[None, :]).sum() / (xn[-1] - xn[0]))


@pytest.mark.parametrize("order,min_order", [(1, 1.8), (2, 2.6), (3, 3.4)])
def test_burgers1d_design_order_on_perturbed_mesh(oracle, order, min_order):
    """The paper's Table 1 setting (Example 1, limiter on) on meshes with 10%
    node perturbation: order about N + 1 before the shock."""
    t_end = 0.5 / np.pi
    u0 = lambda x: 0.5 + np.sin(np.pi * x)  # noqa: E731
    du0 = lambda x: np.pi * np.cos(np.pi * x)  # noqa: E731
    errs = []
    for K in (20, 40, 80):
        wl = W.burgers1d(nx=K, order=order, t_end=t_end, cfl=0.1).nonuniform(seed=100 + K)
        prob, U = oracle_initial_state(oracle, wl, limit=True)
        U, t, _, _ = prob.run(U, 0.0, t_end)
        errs.append(_l1_1d(U, order, wl.mesh["xn"], lambda X: exact.burgers_characteristic(u0, du0, X, t_end)))
    o = orders(errs)
    assert o[-1] > min_order, (errs, o)


def test_density_wave_design_order_on_perturbed_mesh(oracle):
    """The paper's Table 3 setting (2D Euler density wave, Q2) on 10%-perturbed
    meshes, a short time: L1 error of the density falls at about order 3."""
    errs = []
    for K in (8, 16, 32):
        wl = W.density_wave(n=K, order=2, t_end=0.1).nonuniform(seed=200 + K)
        prob, U = oracle_initial_state(oracle, wl, limit=True)
        U, t, _, _ = prob.run(U, 0.0, wl.t_end)
        r, w = np.polynomial.legendre.leggauss(5)
        xn, yn = wl.mesh["xn"], wl.mesh["yn"]
        hx, hy = np.diff(xn), np.diff(yn)
        X = xn[None, :-1] + 0.5 * (1 + r[:, None]) * hx[None, :]
        Y = yn[None, :-1] + 0.5 * (1 + r[:, None]) * hy[None, :]
        P = psi_table(2, r)
        rho = np.einsum("nmji,mq,np->pqji", U[0].reshape(3, 3, K, K), P, P)
        ex = W.density_wave_exact(X[None, :, None, :], Y[:, None, :, None], t)
        W2 = (w[:, None] * w[None, :])[:, :, None, None] * (0.25 * hy[None, None, :, None] * hx[None, None, None, :])
        errs.append(float((W2 * np.abs(rho - ex)).sum() / ((xn[-1] - xn[0]) * (yn[-1] - yn[0]))))
    o = orders(errs)
    assert o[-1] > 2.6, (errs, o)
