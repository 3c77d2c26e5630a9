"""GPU parity of the HIP path (through the C-ABI) against the FP64 CPU oracle,
element by element on the same seeded inputs, at sizes spanning several
64 x 4 tiles with ragged tails.  Tolerances: see tests/gpu_common.py."""
import numpy as np
import pytest
import torch

from tests.gpu_common import assert_close, configs, flags_agree, make_pair, rough_state, worst

pytestmark = pytest.mark.gpu

CASES = [  # (dim, eq, order, nx, ny, bc)
    (1, 0, 1, 301, 1, (0, 0, 0, 0)),
    (1, 0, 2, 517, 1, (0, 0, 0, 0)),
    (1, 0, 3, 300, 1, (1, 1, 1, 1)),
    (1, 1, 1, 257, 1, (1, 1, 1, 1)),
    (1, 1, 2, 333, 1, (1, 1, 1, 1)),
    (1, 1, 3, 260, 1, (0, 0, 0, 0)),
    (2, 0, 1, 150, 9, (0, 0, 0, 0)),
    (2, 0, 2, 131, 11, (1, 1, 0, 0)),
    (2, 0, 3, 70, 7, (0, 0, 1, 1)),
    (2, 1, 1, 130, 10, (1, 1, 1, 1)),
    (2, 1, 2, 150, 9, (1, 1, 1, 1)),
    (2, 1, 2, 67, 21, (0, 0, 0, 0)),
    (2, 1, 3, 66, 6, (1, 1, 0, 0)),
]
IDS = [f"d{c[0]}e{c[1]}n{c[2]}_{c[3]}x{c[4]}_bc{''.join(map(str, c[5]))}" for c in CASES]


@pytest.fixture(scope="module")
def libs(oracle):
    from paper_1904_11147_amd import dg
    dg.lib()
    return oracle, dg


def _pair(libs, case, **kw):
    O, D = libs
    dim, eq, order, nx, ny, bc = case
    cfg = configs(dim, eq, order, nx, ny, bc, **kw)
    return make_pair(O, D, cfg)


def _dev(U):
    return torch.from_numpy(np.ascontiguousarray(U)).cuda()


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_residual(libs, case):
    op, gp = _pair(libs, case)
    U = rough_state(libs[0], op, seed=11)
    ref = op.residual(U)
    got = gp.residual(_dev(U)).cpu().numpy()
    print(case, "residual rel err", assert_close(got, ref, what="residual"))


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_indicator_and_limiter(libs, case):
    op, gp = _pair(libs, case)
    U = rough_state(libs[0], op, seed=21)
    ref, rflags, rmargin = op.limit(U)
    assert rflags.sum() > 0
    # the indicator alone
    Ud = _dev(U)
    flags, margin, n = gp.limit(Ud)
    flags = flags.cpu().numpy()
    diff, ok = flags_agree(flags, rflags, rmargin)
    assert ok, f"flag mismatches away from the threshold: {diff[:10]}"
    assert n == int(flags.sum())
    m = margin.cpu().numpy()
    finite = np.isfinite(rmargin)
    assert np.allclose(m[finite], rmargin[finite], rtol=1e-9, atol=1e-12)
    # the limiter with the oracle's flags injected
    Ud = _dev(U)
    gp.limit(Ud, flags_override=torch.from_numpy(rflags))
    got = Ud.cpu().numpy()
    print(case, "limiter rel err", assert_close(got, ref, what="limiter"), "troubled", int(rflags.sum()))
    assert (got[:, 0] == U[:, 0]).all()  # means kept bit for bit


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_all_cells_limited(libs, case):
    op, gp = _pair(libs, case, indicator=1)
    U = rough_state(libs[0], op, seed=31)
    ref, _, _ = op.limit(U)
    Ud = _dev(U)
    flags, _, n = gp.limit(Ud)
    assert n == case[3] * case[4]
    print(case, "all-limited rel err", assert_close(Ud.cpu().numpy(), ref, what="all-limited"))


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_one_step(libs, case):
    op, gp = _pair(libs, case, cfl=0.05)
    U = rough_state(libs[0], op, seed=41, amplitude=0.2, extra_noise=0.01)
    dt = op.cfl_dt(U)
    assert abs(gp.cfl_dt(_dev(U)) - dt) <= 1e-14 * dt
    ref = op.step(U, dt)
    Ud = _dev(U)
    t, steps = gp.step(Ud, 0.0, 10.0, dt=dt, max_steps=1)
    assert steps == 1 and abs(t - dt) < 1e-18
    got = Ud.cpu().numpy()
    print(case, "step worst", worst(got, ref))
    print(case, "step rel err", assert_close(got, ref, what="step"))


@pytest.mark.parametrize("lim", ["none", "all"])
@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_one_step_fixed_limiting(libs, case, lim):
    """One step with the limiter off, or with every cell limited (no indicator
    decisions), separating rounding of the operator from flag decisions."""
    kw = dict(limiter=0) if lim == "none" else dict(indicator=1)
    op, gp = _pair(libs, case, cfl=0.05, **kw)
    U = rough_state(libs[0], op, seed=41, amplitude=0.2, extra_noise=0.01)
    dt = op.cfl_dt(U)
    ref = op.step(U, dt)
    Ud = _dev(U)
    gp.step(Ud, 0.0, 10.0, dt=dt, max_steps=1)
    got = Ud.cpu().numpy()
    print(case, lim, "step worst", worst(got, ref))
    print(case, lim, "step rel err", assert_close(got, ref, what=f"step limiter={lim}"))


@pytest.mark.parametrize("case", [c for c in CASES if c[2] == 2], ids=[i for c, i in zip(CASES, IDS) if c[2] == 2])
def test_projection(libs, case):
    from paper_1904_11147_amd import workloads as W
    from paper_1904_11147_amd import dg
    op, gp = _pair(libs, case)
    ic = W.random_state_1d(op.nx, op.order, op.equation, 5) if op.dim == 1 else W.random_state_2d(op.equation, 5)
    wl = W.Workload("p", op.dim, op.equation, op.order, op.nx, op.ny, op.x0, op.x1, op.y0, op.y1, op.bc, 0.1, 1.0, ic)
    r_o, _ = op.proj_nodes()
    r_g, w_g = gp.proj_nodes()
    np.testing.assert_allclose(r_g, r_o, atol=1e-15)
    ref = op.project(wl.point_values(r_o))
    got = dg.initial_state(gp, wl, limit=False, rows_per_chunk=4).cpu().numpy()
    assert_close(got, ref, what="projection")
