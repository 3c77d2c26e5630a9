"""Whole-method pins of the oracle on the CPU: design order on smooth
solutions against exact solutions (the paper's Tables 1-3 report order
about N+1 with the limiter on), conservation, and the exact Riemann solution
for the Sod and Lax shock tubes (Examples 7 and 8)."""
import numpy as np
import pytest

from paper_1904_11147_amd import workloads as W
from tests import exact
from tests.dgutil import (cell_means, l1_linf_1d, l1_linf_2d, oracle_initial_state, oracle_problem, orders,
                          eval_1d)


def _burgers_exact(t):
    u0 = lambda x: 0.5 + np.sin(np.pi * x)
    du0 = lambda x: np.pi * np.cos(np.pi * x)
    return lambda X: exact.burgers_characteristic(u0, du0, X, t)


@pytest.mark.parametrize("order,min_order", [(1, 1.8), (2, 2.6), (3, 3.5)])
def test_burgers1d_design_order_with_limiter(oracle, order, min_order):
    """The 1D Burgers problem on [0,2] is the paper's Example 1 under x' = pi x;
    its t = 0.5 becomes t = 0.5/pi (before the shock at t = 1/pi)."""
    t_end = 0.5 / np.pi
    errs = []
    for K in (20, 40, 80):
        wl = W.burgers1d(nx=K, order=order, t_end=t_end, cfl=0.1)
        prob, U = oracle_initial_state(oracle, wl, limit=True)
        U, t, steps, _ = prob.run(U, 0.0, t_end)
        assert t == t_end
        errs.append(l1_linf_1d(U, order, wl.x0, wl.x1, _burgers_exact(t_end))[0])
    o = orders(errs)
    assert o[-1] > min_order, (errs, o)


def test_burgers2d_design_order_with_limiter(oracle):
    """2D Burgers u0 = 0.5 + sin(pi (x+y)/2) on [0,4]^2: exact solution is the
    1D characteristic solution in s = x + y (Example 2 under a rescaling)."""
    t_end = 0.25 / np.pi
    u0 = lambda s: 0.5 + np.sin(np.pi * s / 2)
    du0 = lambda s: np.pi / 2 * np.cos(np.pi * s / 2)
    ex = lambda X, Y: exact.burgers_characteristic(u0, du0, X + Y, 2 * t_end)
    errs = []
    for K in (8, 16, 32):
        wl = W.burgers2d(n=K, order=2, t_end=t_end)
        prob, U = oracle_initial_state(oracle, wl, limit=True)
        U, t, steps, _ = prob.run(U, 0.0, t_end)
        errs.append(l1_linf_2d(U, 2, 0, 4, 0, 4, ex)[0])
    o = orders(errs)
    assert o[-1] > 2.5, (errs, o)


def test_density_wave_design_order(oracle):
    """Example 3 (2D Euler density wave), run to t = 0.5 to keep the CPU
    cost small; the exact density is 1 + 0.2 sin(x + y - t)."""
    t_end = 0.5
    errs = []
    for K in (6, 12, 24):
        wl = W.density_wave(n=K, order=2, t_end=t_end)
        prob, U = oracle_initial_state(oracle, wl, limit=True)
        U, t, steps, _ = prob.run(U, 0.0, t_end)
        errs.append(l1_linf_2d(U, 2, wl.x0, wl.x1, wl.y0, wl.y1,
                               lambda X, Y: W.density_wave_exact(X, Y, t_end))[0])
    o = orders(errs)
    assert o[-1] > 2.5, (errs, o)


def test_conservation_through_shock(oracle):
    """Periodic Burgers past shock formation: sum h * mean is conserved."""
    wl = W.burgers1d(nx=64, order=2, t_end=0.5)
    prob, U = oracle_initial_state(oracle, wl, limit=True)
    m0 = cell_means(U, 1).sum() * prob.hx
    U, t, steps, _ = prob.run(U, 0.0, wl.t_end)
    m1 = cell_means(U, 1).sum() * prob.hx
    assert abs(m1 - m0) < 1e-13 * steps * max(1.0, abs(m0))
    f, _ = prob.indicator(U)
    assert f.sum() >= 1  # the shock is flagged


@pytest.mark.parametrize("case", ["sod", "lax"])
@pytest.mark.parametrize("order", [1, 2])
def test_shock_tube_against_exact_riemann(oracle, case, order):
    errs = []
    for K in (100, 200):
        wl = (W.sod if case == "sod" else W.lax)(nx=K, order=order, cfl=0.1)
        prob, U = oracle_initial_state(oracle, wl, limit=True)
        U, t, steps, _ = prob.run(U, 0.0, wl.t_end)
        L, R = wl.extra["left"], wl.extra["right"]
        r, w = np.polynomial.legendre.leggauss(order + 3)
        h = prob.hx
        X = wl.x0 + (np.arange(K)[None, :] + 0.5 * (1 + r[:, None])) * h
        rho_ex, _, _ = exact.riemann_sample(L, R, (X - wl.extra["x_jump"]) / wl.t_end)
        rho = eval_1d(U, order, r)[0]
        errs.append(float((w[:, None] * np.abs(rho - rho_ex)).sum() * 0.5 * h))
        assert np.isfinite(U).all()
    assert errs[1] < errs[0]
    assert errs[1] < (6e-3 if case == "sod" else 1.5e-2), errs


def test_cfl_dt_rule(oracle):
    wl = W.burgers1d(nx=50, order=2)
    prob, U = oracle_initial_state(oracle, wl)
    sx, _ = prob.max_speed(U)
    means = cell_means(U, 1)[0, 0]
    assert abs(sx - np.abs(means).max()) < 1e-15 * sx
    assert abs(prob.cfl_dt(U) - 0.1 * prob.hx / sx) < 1e-18
