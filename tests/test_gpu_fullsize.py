"""Parity at the full workload sizes, in the launch configuration of the
benchmark (dg_step replaying its captured step after dg_autotune):

* 2D Euler four-state Riemann problem, 2048^2 cells, Q2 (seed 12345);
* 1D Euler shock/entropy-wave interaction, 4000 cells, P3;
* 2D Burgers, 1024^2 cells, Q2, periodic.

The initial state is the oracle's (projection in bands of rows, then one
limiter pass over the whole mesh); the GPU takes one SSP-RK3 step (CFL time
step) of the whole mesh from it; sampled windows are then recomputed by the
oracle from the same initial data and the oracle's CFL time step (which the
GPU's must equal bit for bit).  One step with limiting after each stage reads at most six
cells in each direction (per stage: one for the residual, one for the
limiter), so each window carries a six-cell halo (the true boundary condition
where it meets the domain boundary, wrapped data on periodic domains) and
only its interior is compared, at 1e-12 relative (the parity bar)."""
import numpy as np
import pytest
import torch

from tests.gpu_common import assert_close

pytestmark = pytest.mark.gpu

HALO = 6


def _oracle_initial_state(O, wl, band=128):
    """Projection of the initial data by the oracle, band by band of rows
    (each band a problem of its own: the projection is cell by cell), then
    the limiter once on the whole mesh."""
    from tests.dgutil import oracle_problem
    full = oracle_problem(O, wl)
    if wl.dim == 1:
        return full.limit(full.project(wl.point_values(full.proj_nodes()[0])))[0]
    U = full.zeros()
    hy = (wl.y1 - wl.y0) / wl.ny
    for j0 in range(0, wl.ny, band):
        nr = min(band, wl.ny - j0)
        sub = oracle_problem(O, wl, ny=nr, y0=wl.y0 + j0 * hy, y1=wl.y0 + (j0 + nr) * hy)
        U[..., j0:j0 + nr, :] = sub.project(wl.point_values(sub.proj_nodes()[0], j0, nr))
    return full.limit(U)[0]


def _gpu_one_step(wl, O):
    """One GPU step (CFL rule) from the oracle's initial state; returns that
    state (host), the GPU's result and the oracle's time step."""
    from paper_1904_11147_amd import dg
    from tests.dgutil import oracle_problem
    U0 = _oracle_initial_state(O, wl)
    dt = oracle_problem(O, wl).cfl_dt(U0)
    assert dt < wl.t_end
    p = dg.problem_from_workload(wl)
    u0 = torch.from_numpy(U0).cuda()
    p.autotune(u0)
    t, n = p.step(u0, 0.0, wl.t_end, max_steps=1)
    assert n == 1 and t == dt, (t, dt)  # the device's CFL rule gives the oracle's step exactly
    p.close()
    return torch.from_numpy(U0), u0, dt


def _window_1d(O, wl, u0, u1, dt, a, b):
    """Cells [a, b) of the 1D mesh."""
    nx = wl.nx
    lo, hi = max(a - HALO, 0), min(b + HALO, nx)
    h = (wl.x1 - wl.x0) / nx
    bc = (1, 1, 0, 0)  # transmissive sides: exact at a true boundary, contaminated halo elsewhere
    op = O.Problem(dim=1, equation=wl.equation, order=wl.order, nx=hi - lo, ny=1, x0=wl.x0 + lo * h,
                   x1=wl.x0 + hi * h, bc=bc, gamma=wl.gamma, cfl=wl.cfl)
    U = np.ascontiguousarray(u0[..., lo:hi].cpu().numpy())
    ref = op.step(U, dt)
    i0, i1 = a - lo, b - lo
    assert_close(u1[..., a:b].cpu().numpy(), ref[..., i0:i1], what=f"{wl.name} cells [{a},{b})")


def _window_2d(O, wl, u0, u1, dt, ja, ia, w):
    """Cells [ja, ja+w) x [ia, ia+w); periodic domains take wrapped halos."""
    ny, nx = wl.ny, wl.nx
    hx, hy = (wl.x1 - wl.x0) / nx, (wl.y1 - wl.y0) / ny
    periodic = wl.bc[0] == 0
    if periodic:
        ix = np.arange(ia - HALO, ia + w + HALO) % nx
        jy = np.arange(ja - HALO, ja + w + HALO) % ny
        U = u0.cpu().numpy()[..., jy[:, None], ix[None, :]]
        bc = (1, 1, 1, 1)
        x0, y0 = wl.x0 + (ia - HALO) * hx, wl.y0 + (ja - HALO) * hy
        nxw = nyw = w + 2 * HALO
        oi, oj = HALO, HALO
    else:
        ilo, ihi = max(ia - HALO, 0), min(ia + w + HALO, nx)
        jlo, jhi = max(ja - HALO, 0), min(ja + w + HALO, ny)
        U = u0[..., jlo:jhi, ilo:ihi].cpu().numpy()
        bc = (1, 1, 1, 1)
        x0, y0 = wl.x0 + ilo * hx, wl.y0 + jlo * hy
        nxw, nyw = ihi - ilo, jhi - jlo
        oi, oj = ia - ilo, ja - jlo
    op = O.Problem(dim=2, equation=wl.equation, order=wl.order, nx=nxw, ny=nyw, x0=x0, x1=x0 + nxw * hx, y0=y0,
                   y1=y0 + nyw * hy, bc=bc, gamma=wl.gamma, cfl=wl.cfl)
    ref = op.step(np.ascontiguousarray(U), dt)
    got = u1[..., ja:ja + w, ia:ia + w].cpu().numpy()
    assert_close(got, ref[..., oj:oj + w, oi:oi + w], what=f"{wl.name} window ({ja},{ia}) size {w}")


def test_riemann2d_2048_q2_full_size(oracle):
    from paper_1904_11147_amd import workloads as W
    wl = W.riemann2d(n=2048, order=2, seed=12345)
    u0, u1, dt = _gpu_one_step(wl, oracle)
    rng = np.random.default_rng(7)
    wins = [(1024 - 12, 1024 - 12), (0, 0), (2048 - 24, 2048 - 24), (0, 1500), (1017, 0)]
    wins += [tuple(int(v) for v in rng.integers(0, 2048 - 24, size=2)) for _ in range(3)]
    for ja, ia in wins:
        _window_2d(oracle, wl, u0, u1, dt, ja, ia, 24)


def test_shu_osher_k4000_p3_full_size(oracle):
    from paper_1904_11147_amd import workloads as W
    wl = W.shu_osher()
    u0, u1, dt = _gpu_one_step(wl, oracle)
    for a in (0, 90, 100, 1700, 3960):  # the shock sits near cell 100 (x = -4)
        _window_1d(oracle, wl, u0, u1, dt, a, a + 40)


def test_burgers2d_1024_q2_full_size(oracle):
    from paper_1904_11147_amd import workloads as W
    wl = W.burgers2d()
    u0, u1, dt = _gpu_one_step(wl, oracle)
    for ja, ia in ((0, 0), (1024 - 20, 1024 - 20), (500, 3), (7, 800), (333, 666)):
        _window_2d(oracle, wl, u0, u1, dt, ja, ia, 20)


def _window_dmr(O, wl, u0, u1, dt, ja, ia, w):
    """Window of the double Mach reflection: sides on the domain boundary keep
    their true kinds (inflow, wall, moving switch), inner sides are
    transmissive (contaminated halo)."""
    ny, nx = wl.ny, wl.nx
    hx, hy = (wl.x1 - wl.x0) / nx, (wl.y1 - wl.y0) / ny
    ilo, ihi = max(ia - HALO, 0), min(ia + w + HALO, nx)
    jlo, jhi = max(ja - HALO, 0), min(ja + w + HALO, ny)
    cfg = wl.config()
    at_edge = (ilo == 0, ihi == nx, jlo == 0, jhi == ny)
    bc = [wl.bc[k] if at_edge[k] else 1 for k in range(4)]
    beyond = [cfg["bc_beyond"][k] if at_edge[k] else -1 for k in range(4)]
    cfg.update(nx=ihi - ilo, ny=jhi - jlo, x0=wl.x0 + ilo * hx, x1=wl.x0 + ihi * hx, y0=wl.y0 + jlo * hy,
               y1=wl.y0 + jhi * hy, bc=tuple(bc), bc_beyond=tuple(beyond))
    op = O.Problem(**cfg)
    U = np.ascontiguousarray(u0[..., jlo:jhi, ilo:ihi].cpu().numpy())
    ref = op.step(U, dt)
    oi, oj = ia - ilo, ja - jlo
    got = u1[..., ja:ja + w, ia:ia + w].cpu().numpy()
    assert_close(got, ref[..., oj:oj + w, oi:oi + w], what=f"{wl.name} window ({ja},{ia}) size {w}")


def test_double_mach_1920x480_q2_full_size(oracle):
    """The paper's finest double Mach mesh, one step from t = 0: windows on
    the inflow west side, on both sides of the wall's start at x = 1/6, where
    the shock meets the north side, and inside."""
    from paper_1904_11147_amd import workloads as W
    wl = W.double_mach(1920, order=2)
    u0, u1, dt = _gpu_one_step(wl, oracle)
    w = 24
    foot = int(round(W.DMR_X0 * 480))  # the south side switches at column 80
    top = int((W.DMR_X0 + 1.0 / np.sqrt(3.0)) * 480)  # the shock meets y = 1 near column 357
    wins = [(0, 0), (0, foot - 12), (0, foot + 30), (480 - w, top - 12), (480 - w, 1920 - w), (200, 1000),
            (100, 300), (480 - w, 0)]
    for ja, ia in wins:
        _window_dmr(oracle, wl, u0, u1, dt, ja, ia, w)


def _window_sides(O, cfg, u0, u1, dt, ja, ia, w):
    """Window of a non-periodic mesh: sides on the domain boundary keep their
    true kinds, inner sides are transmissive (contaminated halo)."""
    nx, ny = cfg["nx"], cfg["ny"]
    hx, hy = (cfg["x1"] - cfg["x0"]) / nx, (cfg["y1"] - cfg["y0"]) / ny
    ilo, ihi = max(ia - HALO, 0), min(ia + w + HALO, nx)
    jlo, jhi = max(ja - HALO, 0), min(ja + w + HALO, ny)
    at_edge = (ilo == 0, ihi == nx, jlo == 0, jhi == ny)
    bc = tuple(cfg["bc"][k] if at_edge[k] else 1 for k in range(4))
    c = dict(cfg, nx=ihi - ilo, ny=jhi - jlo, x0=cfg["x0"] + ilo * hx, x1=cfg["x0"] + ihi * hx,
             y0=cfg["y0"] + jlo * hy, y1=cfg["y0"] + jhi * hy, bc=bc)
    op = O.Problem(**c)
    ref = op.step(np.ascontiguousarray(u0[..., jlo:jhi, ilo:ihi].cpu().numpy()), dt)
    oi, oj = ia - ilo, ja - jlo
    got = u1[..., ja:ja + w, ia:ia + w].cpu().numpy()
    assert_close(got, ref[..., oj:oj + w, oi:oi + w], what=f"window ({ja},{ia}) size {w}, sides {cfg['bc']}")


@pytest.mark.parametrize("bc", [(0, 0, 0, 0), (2, 1, 2, 1)], ids=["periodic", "walls"])
def test_large_mesh_64bit_offsets(oracle, bc):
    """2D Euler Q1 on 5840 x 5800 cells (4.3 GB of state): beyond
    32 (N+1)^2 cells = 2^32 bytes, so the stage kernel runs its form with
    64-bit addresses (with reflective west and south sides: its boundary-aware
    form).  A smooth seeded state built here from closed forms, one SSP-RK3
    step with a fixed dt and the limiter, windows against the oracle
    (corners, interior)."""
    from types import SimpleNamespace
    from paper_1904_11147_amd import dg
    from paper_1904_11147_amd import workloads as W
    nx, ny, order = 5840, 5800, 1
    assert 32 * (order + 1) ** 2 * nx * ny > 2 ** 32
    xc = (np.arange(nx) + 0.5) / nx
    yc = (np.arange(ny) + 0.5) / ny
    fx, gy = np.sin(2 * np.pi * xc)[None, :], np.cos(2 * np.pi * yc)[:, None]
    rho = 1.0 + 0.2 * fx * gy
    cons = W.euler2d_conserved(rho, 0.3, -0.2, 1.0 + 0.1 * fx * gy)
    U = np.empty((4, 4, ny, nx))
    for v in range(4):
        c = np.broadcast_to(cons[v], (ny, nx))
        U[v, 0] = 2.0 * c  # the mean is mode (0,0) / 2
        U[v, 1] = 0.01 * c * np.cos(2 * np.pi * xc)[None, :]  # psi_1(x) psi_0(y)
        U[v, 2] = 0.01 * c * np.sin(2 * np.pi * yc)[:, None]  # psi_0(x) psi_1(y)
        U[v, 3] = 0.002 * c * fx * gy
        del c
    h = 1.0 / nx
    dt = 0.02 * h
    cfg = dict(dim=2, equation=dg.EULER, order=order, nx=nx, ny=ny, x0=0.0, x1=1.0, y0=0.0, y1=1.0, bc=bc,
               gamma=1.4, cfl=0.1)
    p = dg.Problem(**cfg, limiter=dg.LIM_CSWENO, indicator=dg.IND_TVB)
    u1 = torch.from_numpy(U).cuda()
    t, n = p.step(u1, 0.0, 1.0, dt=dt, max_steps=1)
    assert n == 1 and t == dt
    p.close()
    u0 = torch.from_numpy(U)
    wins = ((0, 0), (ny - 16, nx - 16), (2900, 2920), (17, 5000), (4321, 1234), (0, 3000), (3000, 0))
    for ja, ia in wins:
        if bc[0] == 0:
            wl = SimpleNamespace(name="euler2d q1 5840x5800", bc=bc, equation=dg.EULER, order=order, gamma=1.4,
                                 cfl=0.1, **{k: cfg[k] for k in ("nx", "ny", "x0", "x1", "y0", "y1")})
            _window_2d(oracle, wl, u0, u1, dt, ja, ia, 16)
        else:
            _window_sides(oracle, cfg, u0, u1, dt, ja, ia, 16)
