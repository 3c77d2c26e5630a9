"""Pins of the oracle's KXRCF troubled-cell indicator (the paper's own, by
citation) against closed forms.

For piecewise-constant data the indicator of the cell behind a jump is
|jump| * h^-((N+1)/2) * (inflow face length / inflow boundary length) /
max |u|, with h the radius of the cell's circumscribed circle (dx/2 in 1D,
sqrt(dx^2 + dy^2)/2 in 2D).  The oracle returns min(|I - 1|, |v_x|, |v_y|)
as the margin, which exposes I exactly where it is the smallest term."""
import numpy as np
import pytest

from oracle import oracle as O

SQ2 = np.sqrt(2.0)


def _burgers1d(order, nx, dx, bc=(1, 1, 0, 0)):
    return O.Problem(dim=1, equation=0, order=order, nx=nx, ny=1, x0=0.0, x1=nx * dx, bc=bc,
                     indicator_mode=O.IND_KXRCF)


def _const_1d(vals, order):
    U = np.zeros((1, order + 1, 1, len(vals)))
    U[0, 0, 0, :] = np.asarray(vals) * SQ2  # mean = mode 0 / sqrt(2)
    return U


@pytest.mark.parametrize("order", [1, 2, 3])
@pytest.mark.parametrize("delta", [0.004, 0.03, 0.045, 0.08])
def test_step_positive_velocity_closed_form(order, delta):
    dx, nx, k = 0.1, 12, 6
    p = _burgers1d(order, nx, dx)
    U = _const_1d([1.0 + delta] * k + [1.0] * (nx - k), order)
    flags, margin = p.indicator(U)
    I = delta * (dx / 2) ** (-(order + 1) / 2) / 1.0
    assert flags[0, k] == (I > 1.0)
    assert abs(margin[0, k] - min(abs(I - 1.0), 1.0)) <= 1e-12
    others = [i for i in range(nx) if i != k]
    assert not flags[0, others].any()


@pytest.mark.parametrize("order", [1, 2])
def test_step_negative_velocity_takes_the_other_face(order):
    dx, nx, k, delta = 0.1, 12, 6, 0.06
    p = _burgers1d(order, nx, dx)
    U = _const_1d([-(1.0 + delta)] * k + [-1.0] * (nx - k), order)
    flags, margin = p.indicator(U)
    # inflow through the east face: the cell left of the jump sees it
    I = delta * (dx / 2) ** (-(order + 1) / 2) / (1.0 + delta)
    assert flags[0, k - 1] == (I > 1.0) and not flags[0, k]
    assert abs(margin[0, k - 1] - min(abs(I - 1.0), 1.0 + delta)) <= 1e-12


def test_sloped_cell_trace_and_quadrature_norm():
    """Cell k linear (mean 1, slope s), the rest constant 1 + delta: the
    jump is taken between traces and the norm is the maximum over the
    2-point Gauss points of the P1 cell."""
    dx, nx, k, delta, s = 0.1, 10, 5, 0.02, 0.3
    p = _burgers1d(1, nx, dx)
    U = _const_1d([1.0 + delta] * nx, 1)
    U[0, 0, 0, k] = 1.0 * SQ2
    # u = mean + slope * (x - x_k) = mean + s * (dx/2) r ; psi_1 = sqrt(3/2) r
    U[0, 1, 0, k] = s * dx / 2 / np.sqrt(1.5)
    flags, margin = p.indicator(U)
    trace_w = 1.0 - s * dx / 2
    jump = trace_w - (1.0 + delta)
    norm = 1.0 + s * dx / 2 / np.sqrt(3.0)
    I = abs(jump) * (dx / 2) ** -1.0 / norm
    assert abs(margin[0, k] - min(abs(I - 1.0), 1.0)) <= 1e-12
    assert flags[0, k] == (I > 1.0)


def test_continuous_polynomial_data_is_never_troubled():
    for order in (1, 2, 3):
        nx, dx = 16, 0.05
        p = _burgers1d(order, nx, dx)
        wl_vals = lambda X: (0.7 + 0.4 * X + (0.2 * X * X if order >= 2 else 0.0),)
        r, _ = p.proj_nodes()
        X = (np.arange(nx)[None, :] + 0.5 * (1 + np.asarray(r)[:, None])) * dx
        pv = np.stack([np.asarray(v, dtype=float) for v in wl_vals(X)])[:, :, None, :]
        U = p.project(np.ascontiguousarray(pv))
        flags, margin = p.indicator(U)
        assert not flags.any()


@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("delta", [0.1, 0.2])
def test_euler2d_density_jump_radius_and_face_integral(order, delta):
    """rho = 1 + delta left of x = 0.5, 1 right; u = 1, v = 0.5, p = 1;
    dx = 0.1, dy = 0.2.  The first cell right of the jump has inflow west and
    south faces, the jump only on the west face."""
    g, nx, ny, dx, dy = 1.4, 10, 6, 0.1, 0.2
    p = O.Problem(dim=2, equation=1, order=order, nx=nx, ny=ny, x0=0.0, x1=nx * dx, y0=0.0, y1=ny * dy,
                  bc=(1, 1, 1, 1), indicator_mode=O.IND_KXRCF)
    nm = (order + 1) ** 2
    U = np.zeros((4, nm, ny, nx))
    rho = np.where(np.arange(nx) < 5, 1.0 + delta, 1.0)[None, :].repeat(ny, 0)
    u, v, pr = 1.0, 0.5, 1.0
    E = pr / (g - 1) + 0.5 * rho * (u * u + v * v)
    for var, val in enumerate((rho, rho * u, rho * v, E)):
        U[var, 0] = val * 2.0  # mean = mode 0 / 2
    flags, margin = p.indicator(U)
    h = 0.5 * np.hypot(dx, dy)
    kx = h ** (-(order + 1) / 2)
    I_rho = delta * dy * kx / (dx + dy)
    E_r = pr / (g - 1) + 0.5 * (u * u + v * v)
    I_E = 0.5 * (u * u + v * v) * delta * dy * kx / ((dx + dy) * E_r)
    want = min(abs(I_rho - 1.0), abs(I_E - 1.0), 1.0, 0.5)
    assert np.all(flags[:, 5] == (I_rho > 1.0 or I_E > 1.0))
    assert np.allclose(margin[:, 5], want, rtol=0, atol=1e-12)
    assert not flags[:, [0, 1, 2, 3, 4, 6, 7, 8, 9]].any()


def test_invariant_under_scaling_and_mirroring():
    rng = np.random.default_rng(3)
    # 1D Euler, positive states with random modes
    nx, order = 40, 2
    p = O.Problem(dim=1, equation=1, order=order, nx=nx, ny=1, x0=0.0, x1=1.0, bc=(1, 1, 0, 0),
                  indicator_mode=O.IND_KXRCF)
    U = np.zeros((3, order + 1, 1, nx))
    rho = 1.0 + 0.5 * rng.random(nx)
    mom = rng.normal(size=nx) * 0.5
    U[0, 0, 0] = rho * SQ2
    U[1, 0, 0] = mom * SQ2
    U[2, 0, 0] = (2.5 + mom ** 2 / rho) * SQ2
    U[:, 1:] = rng.normal(size=U[:, 1:].shape) * 0.05
    f0, m0 = p.indicator(U)
    f1, _ = p.indicator(3.7 * U)
    assert (f0 == f1).all() and f0.any() and not f0.all()
    # mirror x -> -x: reverse cells, flip odd modes and the momentum
    V = U[:, :, :, ::-1].copy()
    V[:, 1::2] *= -1
    V[1] *= -1
    f2, m2 = p.indicator(np.ascontiguousarray(V))
    assert (f2[:, ::-1] == f0).all()
    assert np.allclose(m2[:, ::-1], m0, rtol=1e-12, atol=1e-13)
