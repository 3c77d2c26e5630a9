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


def test_kxrcf_on_a_flow_from_rest_is_sensitive_tvb_is_not(oracle):
    """Sod's problem starts at rest.  KXRCF takes its inflow faces from the
    sign of the mean velocity, which next to the waves is rounding-sized for
    some cells, so a 1e-15 perturbation of the initial state changes flags
    and the solution at t = 0.1 by ~1e-5; under TVB the same perturbation
    stays at ~1e-14.  Final-time GPU/oracle comparisons with KXRCF therefore
    use flows without resting regions."""
    wl = W.sod(nx=100, order=2).with_(t_end=0.1)
    out = {}
    for mode in (0, 3):
        op = oracle_problem(oracle, wl, indicator_mode=mode)
        op, U0 = oracle_initial_state(oracle, wl, op, limit=True)
        A = op.run(U0, 0.0, wl.t_end)[0]
        U1 = U0 * (1.0 + 1e-15 * np.random.default_rng(1).standard_normal(U0.shape))
        B = op.run(U1, 0.0, wl.t_end)[0]
        out[mode] = np.abs(A - B)[:, 0].mean()
    assert out[0] < 1e-12 and out[3] > 1e-8, out


def test_double_mach_q3_amplifies_q2_does_not(oracle):
    """The double Mach reflection (Mach 10, positivity scaling on): a 1e-15
    relative perturbation of the initial state stays near 1e-13 in L1 after
    20 Q2 steps, while Q3 reaches ~1e-9 after 20 steps (and ~5e-2 after 49 on
    this mesh), so Q3 final-time GPU/oracle comparisons of this problem stop
    after 5 steps."""
    from paper_1904_11147_amd import workloads as W
    from tests.dgutil import oracle_initial_state, oracle_problem
    from tests.test_gpu_runs import _l1_diff
    out = {}
    for order in (2, 3):
        wl = W.double_mach(48, order=order)
        op = oracle_problem(oracle, wl)
        op, U0 = oracle_initial_state(oracle, wl, op, limit=True)
        ref, _, s1, _ = op.run(U0, 0.0, 1.0, max_steps=20)
        U1 = U0 * (1 + 1e-15 * np.random.default_rng(1).standard_normal(U0.shape))
        got, _, s2, _ = op.run(U1, 0.0, 1.0, max_steps=20)
        assert s1 == s2 == 20
        out[order] = _l1_diff(got, ref, 2, order).max()
    assert out[2] < 1e-11 and out[3] > 1e-10, out
