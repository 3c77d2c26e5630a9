"""Seeded synthetic workloads: problem setups and initial data.

This module only describes problems -- domains, boundary conditions, orders,
initial conditions as point functions, seeded random quadrant states and
batch compositions.  It holds none of the method's arithmetic (no basis, no
quadrature, no flux, no limiter) and is the only code shared by the HIP path
and the CPU oracle: both evaluate its initial conditions at their own
projection nodes.

Workloads (names are what the problem is, with its sizes):

* ``burgers1d_k200_p2``   -- u_t + (u^2/2)_x = 0 on [0,2], periodic,
  u0 = 0.5 + sin(pi x), 200 cells, P2, CFL 0.1, t = 0.5 (after the shock
  forms at t = 1/pi).  The paper's Examples 1 and 5 on [0, 2 pi] under
  x' = pi x.
* ``shu_osher_k4000_p3``  -- 1D Euler shock/entropy-wave interaction on
  [-5,5], (rho,u,p) = (3.857143, 2.629369, 10.33333) for x < -4 and
  (1 + 0.2 sin 5x, 0, 1) elsewhere, 4000 cells, P3, CFL 0.05, t = 1.8,
  transmissive.  The paper's Example 9 in its standard scaling.
* ``burgers2d_1024_q2``   -- 2D Burgers on [0,4]^2, periodic,
  u0 = 0.5 + sin(pi (x+y)/2), 1024^2 cells, Q2, t = 0.5.
* ``riemann2d_2048_q2``   -- 2D Euler four-state Riemann problem on [0,1]^2,
  quadrant states drawn from a seed (rho in [0.1,1.5], u,v in [-1,1],
  p in [0.03,1.5]) around (0.5,0.5), 2048^2 cells, Q2, transmissive,
  t = 0.25.
* ``riemann2d_batch256``  -- 256 such problems, side n uniform in
  [64,512], order uniform in {1,2,3}.
* ``patchwork2d_2048_q2`` -- 2D Euler on [0,1]^2 from a 127 x 127 patchwork of
  random constant states in the same ranges (a jump every 16.1 cells, inside
  cells): a state with many troubled cells from the start, for limiter-heavy
  parity and timing.
* ``double_mach_960x240_q2`` -- the paper's Example 11: 2D Euler on
  [0,4]x[0,1], a Mach 10 shock through (1/6, 0) at 60 degrees to the x-axis
  moving right into (rho,u,v,p) = (1.4,0,0,1); behind it (8, 8.25 cos 30deg,
  -8.25 sin 30deg, 116.5).  Inflow of the post-shock state on the west side
  and on the south side for x < 1/6, a reflective wall on the rest of the
  south side, transmissive east side, and on the north side the exact
  motion of the shock (post-shock state for x < 1/6 + (1 + 20 t)/sqrt(3),
  pre-shock beyond); positivity-preserving scaling on; t = 0.2; 960x240 and
  1920x480 cells, Q2 and Q3.
* ``sod``, ``lax``, ``density_wave``, ``isentropic_vortex`` -- the paper's
  Examples 7, 8, 3 and 4, used by the tests.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import Callable, Optional

import numpy as np

BURGERS, EULER = 0, 1
PERIODIC, TRANSMISSIVE, REFLECTIVE, INFLOW = 0, 1, 2, 3
GAMMA = 1.4

# quadrant order used when drawing four-state Riemann data
QUADRANTS = ("NE", "NW", "SW", "SE")


@dataclass
class Workload:
    name: str
    dim: int
    equation: int
    order: int
    nx: int
    ny: int
    x0: float
    x1: float
    y0: float
    y1: float
    bc: tuple
    cfl: float
    t_end: float
    ic: Callable  # ic(X, Y) -> tuple of conserved-variable arrays
    gamma: float = GAMMA
    seed: Optional[int] = None
    extra: dict = field(default_factory=dict)
    # boundary switches, inflow states and positivity scaling, as keyword
    # arguments of a problem (bc_beyond, bc_switch, bc_state, positivity)
    bc_extra: dict = field(default_factory=dict)
    # non-uniform tensor-product mesh: {"xn": nodes (nx+1), "yn": nodes (ny+1)}
    mesh: dict = field(default_factory=dict)

    @property
    def nv(self):
        return 1 if self.equation == BURGERS else self.dim + 2

    @property
    def nm(self):
        return (self.order + 1) ** self.dim

    @property
    def cells(self):
        return self.nx * self.ny

    @property
    def dofs(self):
        return self.cells * self.nm * self.nv

    def with_(self, **kw):
        return replace(self, **kw)

    def config(self, **over):
        """Keyword dictionary shared by the oracle and the binding."""
        d = dict(dim=self.dim, equation=self.equation, order=self.order, nx=self.nx, ny=self.ny,
                 x0=self.x0, x1=self.x1, y0=self.y0, y1=self.y1, bc=tuple(self.bc), gamma=self.gamma,
                 cfl=self.cfl)
        d.update(self.bc_extra)
        d.update(self.mesh)
        d.update(over)
        return d

    def nonuniform(self, seed, frac=0.1):
        """The same problem on a mesh whose interior nodes are moved by up to
        frac of the uniform width, uniformly at random (the paper's accuracy
        tests use 10%); the end nodes stay on the domain boundary."""
        mesh = {"xn": perturbed_nodes(self.nx, self.x0, self.x1, seed, frac)}
        if self.dim == 2:
            mesh["yn"] = perturbed_nodes(self.ny, self.y0, self.y1, seed + 1, frac)
        return replace(self, name=f"{self.name}_nu{seed}", mesh=mesh)

    def _nodes(self, r, axis, j0=0, nrows=None):
        """Physical coordinates [q, cell] of the reference nodes r in every
        column (axis 0) or in rows j0.. (axis 1)."""
        key, lo, hi, n = ("xn", self.x0, self.x1, self.nx) if axis == 0 else ("yn", self.y0, self.y1, self.ny)
        idx = np.arange(n) if axis == 0 else np.arange(j0, j0 + nrows)
        if key in self.mesh:
            nodes = np.asarray(self.mesh[key], dtype=np.float64)
            left, width = nodes[idx], nodes[idx + 1] - nodes[idx]
            return left[None, :] + 0.5 * (1.0 + r[:, None]) * width[None, :]
        h = (hi - lo) / n
        return lo + (idx[None, :] + 0.5 * (1.0 + r[:, None])) * h

    def point_values(self, r_nodes, j0=0, nrows=None):
        """Initial data at the projection nodes r_nodes (reference coordinate in
        [-1,1]) of every cell of rows j0..j0+nrows-1.

        Returns an array [nv][nq_y][nq_x][nrows][nx] (1D: [nv][nq][1][nx])."""
        r = np.asarray(r_nodes, dtype=np.float64)
        X = self._nodes(r, 0)  # [q, i]
        if self.dim == 1:
            vals = self.ic(X, None)
            return np.ascontiguousarray(np.stack([np.asarray(v, dtype=np.float64) for v in vals])[:, :, None, :])
        if nrows is None:
            nrows = self.ny - j0
        Y = self._nodes(r, 1, j0, nrows)  # [q, j]
        XX = X[None, :, None, :]  # [qy, qx, j, i]
        YY = Y[:, None, :, None]
        XX, YY = np.broadcast_arrays(XX, YY)
        vals = self.ic(XX, YY)
        return np.ascontiguousarray(np.stack([np.asarray(v, dtype=np.float64) for v in vals]))


    def point_values_device(self, r_nodes, j0, nrows, device):
        """As point_values, built on a torch device, for four-state Riemann
        data (whose quadrant test separates into an x and a y part); None for
        other workloads.  Each node's conserved values are the same numbers
        point_values gives."""
        if "states" not in self.extra or self.dim != 2 or self.mesh:
            return None
        import torch
        st = self.extra["states"]
        xc, yc = self.extra.get("center", (0.5, 0.5))
        r = np.asarray(r_nodes, dtype=np.float64)
        hx = (self.x1 - self.x0) / self.nx
        hy = (self.y1 - self.y0) / self.ny
        X = self.x0 + (np.arange(self.nx)[None, :] + 0.5 * (1.0 + r[:, None])) * hx  # [qx, i]
        Y = self.y0 + (np.arange(j0, j0 + nrows)[None, :] + 0.5 * (1.0 + r[:, None])) * hy  # [qy, j]
        east = torch.from_numpy(X >= xc).to(device)[None, None, :, None, :]
        north = torch.from_numpy(Y >= yc).to(device)[None, :, None, :, None]
        cons = {q: torch.tensor([float(c) for c in euler2d_conserved(*st[q], gamma=self.gamma)],
                                dtype=torch.float64, device=device)[:, None, None, None, None]
                for q in QUADRANTS}
        return torch.where(north, torch.where(east, cons["NE"], cons["NW"]),
                           torch.where(east, cons["SE"], cons["SW"])).contiguous()


def perturbed_nodes(n, x0, x1, seed, frac=0.1):
    """Nodes of [x0, x1] in n cells, the n-1 interior ones moved by a uniform
    random fraction in [-frac, frac] of the uniform width (seeded)."""
    h = (x1 - x0) / n
    nodes = x0 + h * np.arange(n + 1, dtype=np.float64)
    nodes[1:-1] += frac * h * np.random.default_rng(seed).uniform(-1.0, 1.0, n - 1)
    nodes[0], nodes[-1] = x0, x1
    return nodes


# ---------------------------------------------------------------------------
# conserved variables from primitive ones (input preparation only)
# ---------------------------------------------------------------------------

def euler1d_conserved(rho, u, p, gamma=GAMMA):
    rho = np.asarray(rho, dtype=np.float64)
    u = np.broadcast_to(np.asarray(u, dtype=np.float64), rho.shape)
    p = np.broadcast_to(np.asarray(p, dtype=np.float64), rho.shape)
    return rho, rho * u, p / (gamma - 1.0) + 0.5 * rho * u * u


def euler2d_conserved(rho, u, v, p, gamma=GAMMA):
    rho = np.asarray(rho, dtype=np.float64)
    u = np.broadcast_to(np.asarray(u, dtype=np.float64), rho.shape)
    v = np.broadcast_to(np.asarray(v, dtype=np.float64), rho.shape)
    p = np.broadcast_to(np.asarray(p, dtype=np.float64), rho.shape)
    return rho, rho * u, rho * v, p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)


# ---------------------------------------------------------------------------
# 1D
# ---------------------------------------------------------------------------

def burgers1d(nx=200, order=2, t_end=0.5, cfl=0.1, x0=0.0, x1=2.0, omega=np.pi, shift=0.5):
    def ic(X, Y):
        return (shift + np.sin(omega * X),)
    return Workload(f"burgers1d_k{nx}_p{order}", 1, BURGERS, order, nx, 1, x0, x1, 0.0, 1.0,
                    (PERIODIC,) * 4, cfl, t_end, ic)


def shu_osher(nx=4000, order=3, t_end=1.8, cfl=0.05):
    def ic(X, Y):
        left = X < -4.0
        rho = np.where(left, 3.857143, 1.0 + 0.2 * np.sin(5.0 * X))
        u = np.where(left, 2.629369, 0.0)
        p = np.where(left, 10.33333, 1.0)
        return euler1d_conserved(rho, u, p)
    return Workload(f"shu_osher_k{nx}_p{order}", 1, EULER, order, nx, 1, -5.0, 5.0, 0.0, 1.0,
                    (TRANSMISSIVE,) * 4, cfl, t_end, ic)


def riemann1d(name, left, right, x_jump=0.5, nx=200, order=2, t_end=0.2, cfl=0.1, x0=0.0, x1=1.0):
    """Shock tube with primitive states left=(rho,u,p), right=(rho,u,p)."""
    def ic(X, Y):
        m = X < x_jump
        rho = np.where(m, left[0], right[0])
        u = np.where(m, left[1], right[1])
        p = np.where(m, left[2], right[2])
        return euler1d_conserved(rho, u, p)
    return Workload(f"{name}_k{nx}_p{order}", 1, EULER, order, nx, 1, x0, x1, 0.0, 1.0,
                    (TRANSMISSIVE,) * 4, cfl, t_end, ic, extra=dict(left=left, right=right, x_jump=x_jump))


def sod(nx=200, order=2, t_end=0.2, cfl=0.1):
    return riemann1d("sod", (1.0, 0.0, 1.0), (0.125, 0.0, 0.1), nx=nx, order=order, t_end=t_end, cfl=cfl)


def lax(nx=200, order=2, t_end=0.1, cfl=0.1):
    return riemann1d("lax", (0.445, 0.698, 3.528), (0.5, 0.0, 0.571), nx=nx, order=order, t_end=t_end, cfl=cfl)


def random_state_1d(nx, order, equation, seed, amplitude=0.3):
    """A seeded rough 1D profile (sum of a smooth wave, jumps and noise) used
    for limiter and residual parity cases.  Returns an ic callable."""
    rng = np.random.default_rng(seed)
    jumps = np.sort(rng.uniform(0.1, 0.9, size=3))
    levels = rng.uniform(-1.0, 1.0, size=4)
    k = rng.integers(1, 4)

    def ic(X, Y):
        s = np.searchsorted(jumps, X % 1.0)
        base = levels[s] + amplitude * np.sin(2 * np.pi * k * X)
        if equation == BURGERS:
            return (base,)
        rho = 1.0 + 0.4 * np.tanh(base)
        u = 0.5 * base
        p = 1.0 + 0.3 * np.cos(base)
        return euler1d_conserved(rho, u, p)
    return ic


# ---------------------------------------------------------------------------
# 2D
# ---------------------------------------------------------------------------

def burgers2d(n=1024, order=2, t_end=0.5, cfl=0.1, L=4.0, omega=np.pi / 2.0, shift=0.5):
    def ic(X, Y):
        return (shift + np.sin(omega * (X + Y)),)
    return Workload(f"burgers2d_{n}_q{order}", 2, BURGERS, order, n, n, 0.0, L, 0.0, L,
                    (PERIODIC,) * 4, cfl, t_end, ic)


def quadrant_states(seed):
    """Four primitive states (rho, u, v, p), in the order NE, NW, SW, SE, drawn
    with numpy's PCG64 generator from the given seed."""
    rng = np.random.default_rng(seed)
    out = {}
    for q in QUADRANTS:
        rho = rng.uniform(0.1, 1.5)
        u = rng.uniform(-1.0, 1.0)
        v = rng.uniform(-1.0, 1.0)
        p = rng.uniform(0.03, 1.5)
        out[q] = (rho, u, v, p)
    return out


def riemann2d(n=2048, order=2, seed=12345, t_end=0.25, cfl=None, xc=0.5, yc=0.5):
    if cfl is None:
        cfl = 0.05 if order == 3 else 0.1
    st = quadrant_states(seed)

    def ic(X, Y):
        east = X >= xc
        north = Y >= yc
        prim = []
        for k in range(4):
            ne, nw, sw, se = st["NE"][k], st["NW"][k], st["SW"][k], st["SE"][k]
            prim.append(np.where(north, np.where(east, ne, nw), np.where(east, se, sw)))
        return euler2d_conserved(*prim)
    return Workload(f"riemann2d_{n}_q{order}_s{seed}", 2, EULER, order, n, n, 0.0, 1.0, 0.0, 1.0,
                    (TRANSMISSIVE,) * 4, cfl, t_end, ic, seed=seed, extra=dict(states=st, center=(xc, yc)))


def patchwork2d(n=2048, order=2, seed=4242, blocks=127, t_end=0.25, cfl=None):
    """2D Euler on [0,1]^2, transmissive: a blocks x blocks patchwork of
    constant primitive states, each drawn (numpy PCG64, row by row) from the
    ranges of the four-state Riemann problem.  Jumps every n/blocks cells in
    both directions (inside cells unless blocks divides n) give a state with
    many troubled cells from the start, as a Riemann run has after its waves
    have spread."""
    if cfl is None:
        cfl = 0.05 if order == 3 else 0.1
    rng = np.random.default_rng(seed)
    prim = np.stack([rng.uniform(0.1, 1.5, size=(blocks, blocks)), rng.uniform(-1.0, 1.0, size=(blocks, blocks)),
                     rng.uniform(-1.0, 1.0, size=(blocks, blocks)), rng.uniform(0.03, 1.5, size=(blocks, blocks))])

    def ic(X, Y):
        bi = np.clip(np.floor(X * blocks).astype(np.int64), 0, blocks - 1)
        bj = np.clip(np.floor(Y * blocks).astype(np.int64), 0, blocks - 1)
        return euler2d_conserved(*[prim[k][bj, bi] for k in range(4)])
    return Workload(f"patchwork2d_{n}_q{order}_b{blocks}_s{seed}", 2, EULER, order, n, n, 0.0, 1.0, 0.0, 1.0,
                    (TRANSMISSIVE,) * 4, cfl, t_end, ic, seed=seed)


def riemann2d_batch(count=256, first_seed=10000, nmin=64, nmax=512, t_end=0.25):
    """Mixed batch of four-state Riemann problems: side n uniform integer in
    [nmin, nmax], order uniform in {1,2,3}, each from its own seed."""
    out = []
    for s in range(first_seed, first_seed + count):
        rng = np.random.default_rng(s + 7919 * 10**6)
        n = int(rng.integers(nmin, nmax + 1))
        order = int(rng.integers(1, 4))
        out.append(riemann2d(n=n, order=order, seed=s, t_end=t_end))
    return out


def density_wave(n=16, order=2, t_end=2 * np.pi, cfl=None, L=2 * np.pi):
    """Example 3: rho = 1 + 0.2 sin(x+y), u = 0.7, v = 0.3, p = 1, periodic."""
    if cfl is None:
        cfl = 0.05 if order == 3 else 0.1

    def ic(X, Y):
        return euler2d_conserved(1.0 + 0.2 * np.sin(X + Y), 0.7, 0.3, 1.0)
    return Workload(f"density_wave_{n}_q{order}", 2, EULER, order, n, n, 0.0, L, 0.0, L,
                    (PERIODIC,) * 4, cfl, t_end, ic)


def density_wave_exact(X, Y, t):
    return 1.0 + 0.2 * np.sin(X + Y - t)


def isentropic_vortex(n=16, order=2, t_end=2.0, cfl=None, x0=0.0, x1=10.0, y0=-5.0, y1=5.0,
                      xc=5.0, yc=0.0, beta=5.0):
    """Example 4 (domain [0,10] x [-5,5] assumed; the paper does not state it)."""
    if cfl is None:
        cfl = 0.05 if order == 3 else 0.1
    g = GAMMA

    def ic(X, Y):
        r2 = (X - xc) ** 2 + (Y - yc) ** 2
        e = np.exp(1.0 - r2)
        rho = (1.0 - (g - 1.0) / (16.0 * g * np.pi ** 2) * beta ** 2 * e ** 2) ** (1.0 / (g - 1.0))
        u = 1.0 - beta * e * (Y - yc) / (2 * np.pi)
        v = beta * e * (X - xc) / (2 * np.pi)
        return euler2d_conserved(rho, u, v, rho ** g)
    return Workload(f"isentropic_vortex_{n}_q{order}", 2, EULER, order, n, n, x0, x1, y0, y1,
                    (PERIODIC,) * 4, cfl, t_end, ic)


def random_state_2d(equation, seed, amplitude=0.3):
    """A seeded rough 2D field with curved jumps, used for parity cases."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.3, 0.7, size=2)
    rad = rng.uniform(0.15, 0.3)
    lev = rng.uniform(-1.0, 1.0, size=3)
    k = rng.uniform(1.0, 3.0, size=2)

    def ic(X, Y):
        d = np.sqrt((X - c[0]) ** 2 + (Y - c[1]) ** 2)
        base = np.where(d < rad, lev[0], np.where(X + 0.3 * Y < 0.6, lev[1], lev[2]))
        base = base + amplitude * np.sin(2 * np.pi * (k[0] * X + k[1] * Y))
        if equation == BURGERS:
            return (base,)
        rho = 1.0 + 0.4 * np.tanh(base)
        u = 0.5 * base
        v = -0.3 * base
        p = 1.0 + 0.3 * np.cos(base)
        return euler2d_conserved(rho, u, v, p)
    return ic


def by_name(name):
    table = {
        "burgers1d_k200_p2": lambda: burgers1d(),
        "shu_osher_k4000_p3": lambda: shu_osher(),
        "burgers2d_1024_q2": lambda: burgers2d(),
        "riemann2d_2048_q2": lambda: riemann2d(),
        "double_mach_960x240_q2": lambda: double_mach(960),
        "double_mach_1920x480_q2": lambda: double_mach(1920),
    }
    return table[name]()


# ---------------------------------------------------------------------------
# double Mach reflection (the paper's Example 11)
# ---------------------------------------------------------------------------

DMR_PRE = (1.4, 0.0, 0.0, 1.0)
DMR_POST = (8.0, 8.25 * np.cos(np.pi / 6.0), -8.25 * np.sin(np.pi / 6.0), 116.5)
DMR_X0 = 1.0 / 6.0
DMR_SHOCK_SPEED = 10.0


def double_mach(nx=960, ny=None, order=2, t_end=0.2, cfl=None):
    ny = ny or nx // 4
    cfl = cfl if cfl is not None else (0.05 if order == 3 else 0.1)
    s3 = np.sqrt(3.0)

    def ic(X, Y):
        behind = X < DMR_X0 + Y / s3
        prim = [np.where(behind, a, b) for a, b in zip(DMR_POST, DMR_PRE)]
        return euler2d_conserved(*prim)

    post = [float(c) for c in euler2d_conserved(*DMR_POST)]
    pre = [float(c) for c in euler2d_conserved(*DMR_PRE)]
    state = np.zeros((4, 2, 4))
    state[0, 0] = post  # west: inflow
    state[2, 0] = post  # south, x < 1/6: inflow
    state[3, 0] = post  # north, behind the shock
    state[3, 1] = pre   # north, ahead of it
    # the shock meets y = 1 at 1/6 + (1 + 20 t)/sqrt(3): normal speed 10 over sin 60deg
    extra = dict(bc_beyond=(-1, -1, REFLECTIVE, INFLOW),
                 bc_switch=((0.0, 0.0), (0.0, 0.0), (DMR_X0, 0.0),
                            (DMR_X0 + 1.0 / s3, DMR_SHOCK_SPEED / np.sin(np.pi / 3.0))),
                 bc_state=state, positivity=1)
    return Workload(f"double_mach_{nx}x{ny}_q{order}", 2, EULER, order, nx, ny, 0.0, 4.0, 0.0, 1.0,
                    (INFLOW, TRANSMISSIVE, INFLOW, INFLOW), cfl, t_end, ic, bc_extra=extra)
