"""Pins of the oracle's characteristic-field CSWENO (Euler systems limited in
local characteristic fields, end of Sec. 3): the eigenvectors against the flux
Jacobian (complex-step derivative of the Euler flux written out here), the
limiter's exactness on polynomials with every cell limited, cell means kept
bit for bit, and the Sod tube with P3, which componentwise limiting cannot run
(it loses positivity) while the characteristic limiter reaches t = 0.2 close
to the exact Riemann solution."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1904_11147_amd import workloads as W
from tests import exact
from tests.dgutil import eval_1d, oracle_initial_state, oracle_problem

G = 1.4


def _flux(w, dim, d):
    if dim == 1:
        rho, m, E = w
        u = m / rho
        p = (G - 1) * (E - 0.5 * rho * u * u)
        return np.array([m, m * u + p, (E + p) * u])
    rho, mx, my, E = w
    u, v = mx / rho, my / rho
    p = (G - 1) * (E - 0.5 * rho * (u * u + v * v))
    un = u if d == 0 else v
    return np.array([rho * un, mx * un + (p if d == 0 else 0), my * un + (p if d == 1 else 0), (E + p) * un])


def _jacobian(w, dim, d):
    n = len(w)
    A = np.zeros((n, n))
    h = 1e-30
    for k in range(n):
        z = np.array(w, dtype=complex)
        z[k] += 1j * h
        A[:, k] = _flux(z, dim, d).imag / h
    return A


@pytest.mark.parametrize("dim,d", [(1, 0), (2, 0), (2, 1)])
def test_eigenvectors_of_the_flux_jacobian(dim, d):
    rng = np.random.default_rng(5 + dim + d)
    p = O.Problem(dim=dim, equation=1, order=2, nx=4, ny=4 if dim == 2 else 1)
    for _ in range(5):
        rho, pr = 0.2 + rng.random(), 0.1 + rng.random()
        vel = rng.normal(size=dim)
        w = [rho, *(rho * vel), pr / (G - 1) + 0.5 * rho * (vel @ vel)]
        L, R = p.char_eig(w, d)
        A = _jacobian(w, dim, d)
        c = np.sqrt(G * pr / rho)
        un = vel[d]
        lam = [un - c, un, un + c] + ([un] if dim == 2 else [])
        assert np.allclose(A @ R, R @ np.diag(lam), rtol=0, atol=1e-11 * max(1, np.abs(A).max()))
        assert np.allclose(L @ R, np.eye(dim + 2), atol=1e-12)
        assert np.linalg.matrix_rank(R) == dim + 2


def _poly_state(op, order, dim):
    """A positive Euler state whose every component is a polynomial of degree
    <= order in each direction, projected exactly."""
    r, _ = op.proj_nodes()
    r = np.asarray(r)
    X = op.x0 + (np.arange(op.nx)[None, :] + 0.5 * (1 + r[:, None])) * op.hx
    if dim == 1:
        P = lambda a: a[0] + a[1] * X + a[2] * X ** min(order, 2) * (order >= 2)
        comps = [P((2.0, 0.3, 0.2)), P((0.4, -0.2, 0.1)), P((5.0, 0.5, -0.3))]
        return op.project(np.ascontiguousarray(np.stack(comps)[:, :, None, :]))
    hy = (op.y1 - op.y0) / op.ny
    Y = op.y0 + (np.arange(op.ny)[None, :] + 0.5 * (1 + r[:, None])) * hy
    XX, YY = np.broadcast_arrays(X[None, :, None, :], Y[:, None, :, None])
    P = lambda a: a[0] + a[1] * XX + a[2] * YY + a[3] * XX * YY
    comps = [P((2.0, 0.3, 0.2, 0.1)), P((0.4, -0.2, 0.1, 0.05)), P((-0.3, 0.1, 0.2, -0.1)), P((5.0, 0.5, -0.3, 0.2))]
    return op.project(np.ascontiguousarray(np.stack(comps)))


@pytest.mark.parametrize("dim", [1, 2])
@pytest.mark.parametrize("order", [1, 2, 3])
def test_polynomials_pass_unchanged_and_means_are_kept(dim, order):
    n = 12
    op = O.Problem(dim=dim, equation=1, order=order, nx=n, ny=n if dim == 2 else 1, x0=0.0, x1=1.0, y0=0.0,
                   y1=1.0, bc=(1, 1, 1, 1), limiter=O.LIM_CSWENO_CHAR)
    U = _poly_state(op, order, dim)
    flags = np.ones((op.ny, op.nx), dtype=np.uint8)
    V, _, _ = op.limit(U, flags=flags)
    inner = (slice(None), slice(None), slice(1, -1) if dim == 2 else slice(None), slice(1, -1))
    assert np.abs(V[inner] - U[inner]).max() <= 1e-11 * np.abs(U).max()
    assert (V[:, 0] == U[:, 0]).all()
    # rough data: the limiter does change it, the means still bit for bit
    rng = np.random.default_rng(order)
    Ur = U.copy()
    Ur[:, 1:] += 0.05 * rng.normal(size=Ur[:, 1:].shape)
    Vr, _, _ = op.limit(Ur, flags=flags)
    assert (Vr[:, 0] == Ur[:, 0]).all() and np.abs(Vr - Ur).max() > 1e-6


def test_sod_p3_runs_only_with_characteristic_limiting(oracle):
    wl = W.sod(nx=200, order=3)
    comp = oracle_problem(oracle, wl)
    comp, U = oracle_initial_state(oracle, wl, comp, limit=True)
    with pytest.raises(O.OracleError):
        comp.run(U, 0.0, wl.t_end)
    char = oracle_problem(oracle, wl, limiter=O.LIM_CSWENO_CHAR)
    char, U = oracle_initial_state(oracle, wl, char, limit=True)
    V, t, steps, _ = char.run(U, 0.0, wl.t_end)
    assert t == wl.t_end and np.isfinite(V).all()
    r, w = np.polynomial.legendre.leggauss(6)
    h = char.hx
    X = wl.x0 + (np.arange(wl.nx)[None, :] + 0.5 * (1 + r[:, None])) * h
    rho_ex, _, _ = exact.riemann_sample(wl.extra["left"], wl.extra["right"], (X - wl.extra["x_jump"]) / wl.t_end)
    err = float((w[:, None] * np.abs(eval_1d(V, 3, r)[0] - rho_ex)).sum() * 0.5 * h)
    assert err < 6e-3, err
