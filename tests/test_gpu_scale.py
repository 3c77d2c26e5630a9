"""Parity at the workloads' scale beyond one step from the initial data:

* 2D Burgers Q2 at 256^2 to t = 0.5 (the 1024^2 workload's problem on a
  mesh the oracle finishes in seconds): final-time L1 difference <= 1e-10;
* the 2D Euler four-state Riemann problem of the benchmark (seed 12345) on a
  128^2 mesh: L1 difference <= 1e-10 at t = 0.06 and, at t = 0.25 (1765
  steps, about half of the cell-stages troubled), within 10x the oracle's
  own sensitivity to a 1e-15 perturbation of the initial state, against the
  oracle's solutions that tests/golden/make_riemann2d_128_final.py stored
  (about 37 minutes of oracle time per run on 8 host threads);
* the smallest and the largest instance of each order of the 256-instance
  batch, advanced together by dg_batch_step for three CFL steps, against
  three oracle steps each (1e-12 relative);
* the 2048^2 Q2 Euler mesh from a state with many troubled cells (a
  127 x 127 patchwork of random constant states: a jump every 16.1 cells,
  inside cells):
  three steps of dg_step with a fixed time step (the oracle's CFL step of
  the initial state), in the benchmark's launch configuration, checked on
  sampled windows recomputed by the oracle with an 18-cell halo (three steps
  of six cells each).

Every initial state is the oracle's own projection and limiting."""
import numpy as np
import pytest
import torch

from tests.gpu_common import assert_close
from tests.dgutil import oracle_initial_state, oracle_problem

pytestmark = pytest.mark.gpu


def test_burgers2d_256_q2_to_t05(oracle):
    from tests.test_gpu_runs import _run_both
    from paper_1904_11147_amd import workloads as W
    _run_both(oracle, W.burgers2d(n=256, order=2, t_end=0.5))


def test_riemann2d_128_q2_to_t025(oracle):
    """C4's problem at 128^2: to t = 0.06 (402 steps) the GPU must agree
    with the oracle within 1e-10 in L1; from there to t = 0.25 (1363 more
    steps, about half of the cell-stages troubled) the problem itself
    amplifies rounding-level differences: the oracle's own run from an
    initial state perturbed by 1e-15 (relative) ends 6e-7..4e-6 away in L1.
    There the GPU must stay within 10 times that self-sensitivity."""
    import os
    from paper_1904_11147_amd import dg
    from paper_1904_11147_amd import workloads as W
    from tests.test_gpu_runs import L1_TOL, _l1_diff
    g = np.load(os.path.join(os.path.dirname(__file__), "golden", "riemann2d_128_q2_final.npz"), allow_pickle=False)
    wl = W.riemann2d(n=int(g["n"]), order=int(g["order"]), seed=int(g["seed"]), t_end=float(g["t"]))
    op = oracle_problem(oracle, wl)
    _, U0 = oracle_initial_state(oracle, wl, prob=op, limit=True)
    gp = dg.problem_from_workload(wl)
    Ud = torch.from_numpy(U0).cuda()
    t, n = gp.step(Ud, 0.0, float(g["t_mid"]))
    assert t == float(g["t_mid"]) and n == int(g["steps_mid"]), (t, n)
    l1 = _l1_diff(Ud.cpu().numpy(), g["state_mid"], 2, wl.order)
    print(wl.name, f"t = {t}: {n} steps, L1 diff per var", l1, "oracle self-sensitivity", g["self_l1_mid"])
    assert (l1 <= L1_TOL).all(), l1
    t, n = gp.step(Ud, t, wl.t_end)
    gp.close()
    assert t == wl.t_end and n == int(g["steps_rest"]), (t, n)
    l1 = _l1_diff(Ud.cpu().numpy(), g["state"], 2, wl.order)
    print(wl.name, f"t = {t}: {n} more steps, L1 diff per var", l1, "oracle self-sensitivity", g["self_l1_end"])
    assert (l1 <= 10.0 * g["self_l1_end"]).all(), (l1, g["self_l1_end"])


def test_batch_extremes_three_steps(oracle):
    """Smallest and largest n of each order in the 256-instance batch."""
    from paper_1904_11147_amd import dg
    from paper_1904_11147_amd import workloads as W
    allw = W.riemann2d_batch()
    pick = []
    for order in (1, 2, 3):
        same = sorted((w for w in allw if w.order == order), key=lambda w: (w.nx, w.seed))
        pick += [same[0], same[-1]]
    b = dg.batch_from_workloads(pick, limit=False)
    ops, U0 = [], []
    for i, wl in enumerate(pick):
        op, U = oracle_initial_state(oracle, wl, limit=True)
        b.view(i).copy_(torch.from_numpy(U))
        ops.append(op)
        U0.append(U)
    t, steps, status, _ = b.step(0.0, [wl.t_end for wl in pick], max_steps=3)
    assert (steps == 3).all() and (status == 0).all(), (steps, status)
    for i, wl in enumerate(pick):
        op, U = ops[i], U0[i]
        tt = 0.0
        for _ in range(3):
            dt = op.cfl_dt(U)
            U = op.step(U, dt)
            tt += dt
        assert abs(t[i] - tt) <= 1e-13 * tt, (i, t[i], tt)
        e = assert_close(b.view(i).cpu().numpy(), U, what=f"{wl.name} ({wl.nx}^2) after 3 batched steps")
        print(wl.name, wl.nx, "order", wl.order, "rel diff", e)


HALO3 = 18  # three steps, six cells each


def _band_projection(O, wl, band=128):
    from tests.test_gpu_fullsize import _oracle_initial_state
    return _oracle_initial_state(O, wl, band)


def test_patchwork_2048_q2_three_steps(oracle):
    from paper_1904_11147_amd import dg
    from paper_1904_11147_amd import workloads as W
    wl = W.patchwork2d(n=2048, order=2, seed=4242, blocks=127)
    full = oracle_problem(oracle, wl)
    U0 = _band_projection(oracle, wl)
    flags, _ = full.indicator(U0)
    frac = float(flags.mean())
    print("troubled fraction of the initial state", frac)
    assert frac >= 0.10
    dt = full.cfl_dt(U0)
    p = dg.problem_from_workload(wl)
    u = torch.from_numpy(U0).cuda()
    p.autotune(u)
    p.profile_read(reset=True)
    t, n = p.step(u, 0.0, wl.t_end, dt=dt, max_steps=3)
    assert n == 3
    got = u.cpu().numpy()
    p.close()
    rng = np.random.default_rng(11)
    w = 24
    wins = [(0, 0), (2048 - w, 2048 - w), (1000, 0), (0, 1337), (2048 - w, 77)]
    wins += [tuple(int(v) for v in rng.integers(0, 2048 - w, size=2)) for _ in range(4)]
    hx = hy = 1.0 / 2048
    for ja, ia in wins:
        ilo, ihi = max(ia - HALO3, 0), min(ia + w + HALO3, 2048)
        jlo, jhi = max(ja - HALO3, 0), min(ja + w + HALO3, 2048)
        op = oracle.Problem(dim=2, equation=1, order=2, nx=ihi - ilo, ny=jhi - jlo, x0=ilo * hx, x1=ihi * hx,
                            y0=jlo * hy, y1=jhi * hy, bc=(1, 1, 1, 1), gamma=wl.gamma, cfl=wl.cfl)
        U = np.ascontiguousarray(U0[..., jlo:jhi, ilo:ihi])
        for _ in range(3):
            U = op.step(U, dt)
        oi, oj = ia - ilo, ja - jlo
        assert_close(got[..., ja:ja + w, ia:ia + w], U[..., oj:oj + w, oi:oi + w],
                     what=f"{wl.name} window ({ja},{ia}) after 3 steps")
