"""The 2D Euler Q2 scheme keeps a 1e-14 perturbation of its state at rounding
level, while Q3 with the positive/negative split of the negative linear
weights amplifies it by orders of magnitude within a few tens of steps (CPU,
oracle only).  This is why final-time GPU/oracle comparisons of Q3 Euler runs
are limited to their first steps."""
import numpy as np

from paper_1904_11147_amd import workloads as W
from tests.dgutil import oracle_initial_state, oracle_problem


def _growth(oracle, order, steps, n=16):
    wl = W.riemann2d(n=n, order=order, seed=3, t_end=1.0, cfl=0.05)
    op = oracle_problem(oracle, wl)
    op, U = oracle_initial_state(oracle, wl, op, limit=True)
    V = U * (1.0 + 1e-14 * np.random.default_rng(0).normal(size=U.shape))
    for _ in range(steps):
        dt = op.cfl_dt(U)
        U = op.step(U, dt)
        V = op.step(V, dt)
    return np.abs(U - V).max()


def test_q2_is_insensitive_q3_amplifies(oracle):
    assert _growth(oracle, 2, 30) < 1e-11
    assert _growth(oracle, 3, 30) > 1e-9
