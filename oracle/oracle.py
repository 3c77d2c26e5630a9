"""ctypes wrapper of the FP64 CPU oracle (``oracle/dg_oracle.c``).

Test infrastructure only: the tests, the smoke check and the benchmark's
CPU-baseline leg use it to check and to time the HIP path.  It imports
nothing from the product package and the product package never imports it.

The oracle follows Kochi & Ramakrishna (arXiv 1904.11147): Section 2 (modal
orthonormal-Legendre weak form, eq. weakFormScheme, with a Lax-Friedrichs
flux), Section 3 steps 1-6 (compact subcell WENO limiting) and the third-order
TVD Runge-Kutta scheme that closes Section 3.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dg_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

BURGERS, EULER = 0, 1
PERIODIC, TRANSMISSIVE, REFLECTIVE, INFLOW = 0, 1, 2, 3
LIM_NONE, LIM_CSWENO, LIM_CSWENO_CHAR = 0, 1, 2
IND_TVB, IND_ALL, IND_KXRCF = 0, 1, 3
NEGW_SPLIT, NEGW_RAW = 0, 1
ERR_NONPHYSICAL = -5


class OrcConfig(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32),
        ("equation", ctypes.c_int32),
        ("order", ctypes.c_int32),
        ("nx", ctypes.c_int32),
        ("ny", ctypes.c_int32),
        ("bc", ctypes.c_int32 * 4),
        ("limiter", ctypes.c_int32),
        ("indicator", ctypes.c_int32),
        ("negw_mode", ctypes.c_int32),
        ("gamma", ctypes.c_double),
        ("x0", ctypes.c_double),
        ("x1", ctypes.c_double),
        ("y0", ctypes.c_double),
        ("y1", ctypes.c_double),
        ("tvb_M", ctypes.c_double),
        ("weno_eps", ctypes.c_double),
        ("cfl", ctypes.c_double),
        ("positivity", ctypes.c_int32),
        ("bc_beyond", ctypes.c_int32 * 4),
        ("pad_", ctypes.c_int32),
        ("bc_switch", (ctypes.c_double * 2) * 4),
        ("bc_state", ((ctypes.c_double * 4) * 2) * 4),
        ("time", ctypes.c_double),
        ("xn", ctypes.POINTER(ctypes.c_double)),
        ("yn", ctypes.POINTER(ctypes.c_double)),
    ]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-fno-fast-math", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        P = ctypes.POINTER
        d, i32, u8 = ctypes.c_double, ctypes.c_int32, ctypes.c_uint8
        cfgp = P(OrcConfig)
        sig = {
            "orc_residual": [cfgp, P(d), P(d)],
            "orc_indicator": [cfgp, P(d), P(u8), P(d)],
            "orc_limit": [cfgp, P(d), P(u8), P(d), P(u8)],
            "orc_max_speed": [cfgp, P(d), P(d), P(d)],
            "orc_cfl_dt": [cfgp, P(d), P(d)],
            "orc_step": [cfgp, P(d), d],
            "orc_run": [cfgp, P(d), P(d), d, d, i32, P(i32), P(d), i32],
            "orc_proj_nodes": [ctypes.c_int, P(d), P(d), P(i32)],
            "orc_project": [cfgp, P(d), P(d)],
            "orc_weno_tables": [ctypes.c_int, P(i32), P(d), P(d), P(d), P(d), P(d), P(i32), P(d)],
            "orc_weno_eval": [ctypes.c_int, ctypes.c_int, P(d), d, ctypes.c_int, P(d)],
            "orc_weno_tables_nu": [ctypes.c_int, d, d, P(i32), P(d), P(d), P(d), P(d), P(d), P(i32), P(d), P(d),
                                   P(d)],
            "orc_subcell_means": [ctypes.c_int, P(d)],
            "orc_quadrature": [ctypes.c_int, ctypes.c_int, P(d), P(d)],
            "orc_basis": [ctypes.c_int, d, P(d), P(d)],
            "orc_num_threads": [],
            "orc_char_eig": [cfgp, P(d), ctypes.c_int, P(d), P(d)],
            "orc_positivity": [cfgp, P(d), P(d)],
            "orc_ghost": [cfgp, P(d), i32, i32, P(d)],
        }
        for name, args in sig.items():
            fn = getattr(_lib, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _u8p(a):
    if a is None:
        return None
    assert a.dtype == np.uint8 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"oracle {what} failed with code {code}")
        self.code = code


@dataclass
class Problem:
    """A discretised conservation law on a uniform Cartesian mesh."""

    dim: int = 1
    equation: int = BURGERS
    order: int = 2
    nx: int = 16
    ny: int = 1
    x0: float = 0.0
    x1: float = 1.0
    y0: float = 0.0
    y1: float = 1.0
    bc: tuple = (PERIODIC, PERIODIC, PERIODIC, PERIODIC)
    gamma: float = 1.4
    limiter: int = LIM_CSWENO
    indicator_mode: int = IND_TVB
    negw_mode: int = NEGW_SPLIT
    tvb_M: float = 1.0
    weno_eps: float = 1e-6
    cfl: float = 0.1
    positivity: int = 0
    # south/north sides may switch kind along x at a + b t: bc_beyond[s] = kind
    # beyond the switch (-1: none), bc_switch[s] = (a, b)
    bc_beyond: tuple = (-1, -1, -1, -1)
    bc_switch: tuple = ((0.0, 0.0),) * 4
    # conserved inflow ghost states [side][before, beyond][var]
    bc_state: object = None
    time: float = 0.0
    # non-uniform tensor-product mesh: node coordinates (nx+1, ny+1), or None
    xn: object = None
    yn: object = None
    _c: OrcConfig = field(default=None, repr=False)

    def __post_init__(self):
        if self.dim == 1:
            self.ny = 1
        c = OrcConfig()
        c.dim, c.equation, c.order, c.nx, c.ny = self.dim, self.equation, self.order, self.nx, self.ny
        for k in range(4):
            c.bc[k] = self.bc[k]
        c.limiter, c.indicator, c.negw_mode = self.limiter, self.indicator_mode, self.negw_mode
        c.gamma, c.x0, c.x1, c.y0, c.y1 = self.gamma, self.x0, self.x1, self.y0, self.y1
        c.tvb_M, c.weno_eps, c.cfl = self.tvb_M, self.weno_eps, self.cfl
        c.positivity = int(self.positivity)
        st = np.zeros((4, 2, 4)) if self.bc_state is None else np.asarray(self.bc_state, dtype=np.float64)
        for k in range(4):
            c.bc_beyond[k] = int(self.bc_beyond[k])
            for a in range(2):
                c.bc_switch[k][a] = float(self.bc_switch[k][a])
                for v in range(4):
                    c.bc_state[k][a][v] = float(st[k, a, v])
        c.time = float(self.time)
        self._nodes = []
        for name, n in (("xn", self.nx), ("yn", self.ny)):
            arr = getattr(self, name)
            if arr is None:
                continue
            arr = np.ascontiguousarray(arr, dtype=np.float64)
            assert arr.shape == (n + 1,), (name, arr.shape)
            self._nodes.append(arr)  # keeps the memory alive with the config
            setattr(c, name, _dp(arr))
        self._c = c

    def at_time(self, t):
        """The same problem with boundary data taken at time t."""
        import dataclasses
        return dataclasses.replace(self, time=float(t), _c=None)

    # -- shapes ---------------------------------------------------------
    @property
    def nv(self):
        return 1 if self.equation == BURGERS else self.dim + 2

    @property
    def nm(self):
        return (self.order + 1) ** self.dim

    @property
    def shape(self):
        return (self.nv, self.nm, self.ny, self.nx)

    @property
    def hx(self):
        return (self.x1 - self.x0) / self.nx

    @property
    def hy(self):
        return (self.y1 - self.y0) / self.ny if self.dim == 2 else 1.0

    def zeros(self):
        return np.zeros(self.shape, dtype=np.float64)

    # -- calls ----------------------------------------------------------
    def _chk(self, rc, what, allow_nonphysical=False):
        if rc != 0 and not (allow_nonphysical and rc == ERR_NONPHYSICAL):
            raise OracleError(rc, what)
        return rc

    def residual(self, U):
        U = np.ascontiguousarray(U, dtype=np.float64)
        L = np.empty_like(U)
        self._chk(lib().orc_residual(ctypes.byref(self._c), _dp(U), _dp(L)), "residual")
        return L

    def char_eig(self, w, direction=0):
        """(L, R): left/right eigenvectors of the Euler flux Jacobian in the given
        direction at the conserved state w."""
        nv = self.dim + 2
        w = np.ascontiguousarray(w, dtype=np.float64)
        L = np.zeros((nv, nv))
        R = np.zeros((nv, nv))
        self._chk(lib().orc_char_eig(ctypes.byref(self._c), _dp(w), int(direction), _dp(L), _dp(R)), "char_eig")
        return L, R

    def positivity_scale(self, U):
        """Positivity-preserving scaling of every cell.  Returns (state, theta)
        with theta[0] / theta[1] the density / pressure factors per cell."""
        out = np.array(U, dtype=np.float64, copy=True, order="C")
        th = np.empty((2, self.ny, self.nx), dtype=np.float64)
        self._chk(lib().orc_positivity(ctypes.byref(self._c), _dp(out), _dp(th)), "positivity")
        return out, th

    def ghost(self, U, i, j=0):
        """Modes [nv][nm] of cell (i, j), i in [-1, nx], j in [-1, ny], as the
        boundary conditions give it at the problem's time."""
        U = np.ascontiguousarray(U, dtype=np.float64)
        out = np.zeros((self.nv, self.nm))
        self._chk(lib().orc_ghost(ctypes.byref(self._c), _dp(U), int(i), int(j), _dp(out)), "ghost")
        return out

    def indicator(self, U):
        U = np.ascontiguousarray(U, dtype=np.float64)
        f = np.empty((self.ny, self.nx), dtype=np.uint8)
        m = np.empty((self.ny, self.nx), dtype=np.float64)
        self._chk(lib().orc_indicator(ctypes.byref(self._c), _dp(U), _u8p(f), _dp(m)), "indicator")
        return f, m

    def limit(self, U, flags=None):
        """Indicator + CSWENO once (Jacobi).  Returns (limited, flags, margins)."""
        out = np.array(U, dtype=np.float64, copy=True, order="C")
        f = np.empty((self.ny, self.nx), dtype=np.uint8)
        m = np.empty((self.ny, self.nx), dtype=np.float64)
        fin = None if flags is None else np.ascontiguousarray(flags, dtype=np.uint8)
        self._chk(lib().orc_limit(ctypes.byref(self._c), _dp(out), _u8p(f), _dp(m), _u8p(fin)), "limit")
        return out, f, m

    def max_speed(self, U):
        U = np.ascontiguousarray(U, dtype=np.float64)
        sx, sy = ctypes.c_double(), ctypes.c_double()
        self._chk(lib().orc_max_speed(ctypes.byref(self._c), _dp(U), ctypes.byref(sx), ctypes.byref(sy)),
                  "max_speed")
        return sx.value, sy.value

    def cfl_dt(self, U):
        U = np.ascontiguousarray(U, dtype=np.float64)
        dt = ctypes.c_double()
        self._chk(lib().orc_cfl_dt(ctypes.byref(self._c), _dp(U), ctypes.byref(dt)), "cfl_dt")
        return dt.value

    def step(self, U, dt):
        out = np.array(U, dtype=np.float64, copy=True, order="C")
        self._chk(lib().orc_step(ctypes.byref(self._c), _dp(out), float(dt)), "step")
        return out

    def run(self, U, t, t_end, dt=0.0, max_steps=10**9, log_dt=0):
        """Advance to t_end; returns (state, t, steps, dt_log)."""
        out = np.array(U, dtype=np.float64, copy=True, order="C")
        tt = ctypes.c_double(t)
        steps = ctypes.c_int32()
        log = np.zeros(max(log_dt, 1), dtype=np.float64)
        rc = lib().orc_run(ctypes.byref(self._c), _dp(out), ctypes.byref(tt), float(t_end), float(dt),
                           int(min(max_steps, 2**31 - 1)), ctypes.byref(steps), _dp(log), int(log_dt))
        self._chk(rc, "run")
        return out, tt.value, steps.value, log[: min(steps.value, log_dt)]

    # -- initial data -----------------------------------------------------
    def proj_nodes(self):
        r = np.zeros(16)
        w = np.zeros(16)
        nq = ctypes.c_int32()
        self._chk(lib().orc_proj_nodes(self.order, _dp(r), _dp(w), ctypes.byref(nq)), "proj_nodes")
        return r[: nq.value].copy(), w[: nq.value].copy()

    def node_coords(self):
        """Physical coordinates of the projection nodes: (X[qx, i], Y[qy, j])."""
        r, _ = self.proj_nodes()
        if self.xn is not None:
            xn = np.asarray(self.xn)
            X = xn[None, :-1] + 0.5 * (1.0 + r[:, None]) * np.diff(xn)[None, :]
        else:
            i = np.arange(self.nx)
            X = self.x0 + (i[None, :] + 0.5 * (1.0 + r[:, None])) * self.hx
        if self.dim == 1:
            return X, None
        if self.yn is not None:
            yn = np.asarray(self.yn)
            Y = yn[None, :-1] + 0.5 * (1.0 + r[:, None]) * np.diff(yn)[None, :]
        else:
            j = np.arange(self.ny)
            Y = self.y0 + (j[None, :] + 0.5 * (1.0 + r[:, None])) * self.hy
        return X, Y

    def project(self, pv):
        """pv: [nv][qy][qx][ny][nx] (1D: [nv][qx][1][nx]) point values at node_coords()."""
        pv = np.ascontiguousarray(pv, dtype=np.float64)
        U = self.zeros()
        self._chk(lib().orc_project(ctypes.byref(self._c), _dp(pv), _dp(U)), "project")
        return U


# -- table introspection (pin tests) -----------------------------------------

def weno_tables(order, rl=None, rr=None):
    """Linear weights, rows p_i(x_G) over the stencil means and the beta
    quadratic forms; with rl, rr the stencil of a cell whose left / right
    neighbours are rl / rr times as wide (non-uniform meshes), which also
    returns the stencil cells (in units of the cell's width)."""
    N = order
    ns = 2 * N + 1
    ng = ctypes.c_int32()
    rg, wg = np.zeros(4), np.zeros(4)
    gam = np.zeros(4 * (N + 1))
    rows = np.zeros(4 * (N + 1) * ns)
    bmat = np.zeros((N + 1) ** 3)
    split = np.zeros(4, dtype=np.int32)
    resid = ctypes.c_double()
    cl, cr = np.zeros(7), np.zeros(7)
    if rl is None:
        rc = lib().orc_weno_tables(order, ctypes.byref(ng), _dp(rg), _dp(wg), _dp(gam), _dp(rows), _dp(bmat),
                                   split.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), ctypes.byref(resid))
    else:
        rc = lib().orc_weno_tables_nu(order, float(rl), float(rr), ctypes.byref(ng), _dp(rg), _dp(wg), _dp(gam),
                                      _dp(rows), _dp(bmat), split.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                      ctypes.byref(resid), _dp(cl), _dp(cr))
    if rc:
        raise OracleError(rc, "weno_tables")
    G = ng.value
    return dict(
        cells=np.stack([cl[:ns], cr[:ns]], axis=1).copy(),
        rg=rg[:G].copy(), wg=wg[:G].copy(),
        gamma=gam[: G * (N + 1)].reshape(G, N + 1).copy(),
        rows=rows[: G * (N + 1) * ns].reshape(G, N + 1, ns).copy(),
        beta=bmat.reshape(N + 1, N + 1, N + 1).copy(),
        split=split[:G].copy(), gamma_residual=resid.value,
    )


def weno_eval(order, G, a, eps=1e-6, negw_mode=NEGW_SPLIT):
    a = np.ascontiguousarray(a, dtype=np.float64)
    out = ctypes.c_double()
    rc = lib().orc_weno_eval(order, G, _dp(a), eps, negw_mode, ctypes.byref(out))
    if rc:
        raise OracleError(rc, "weno_eval")
    return out.value


def subcell_means(order):
    s = np.zeros(order * (order + 1))
    rc = lib().orc_subcell_means(order, _dp(s))
    if rc:
        raise OracleError(rc, "subcell_means")
    return s.reshape(order, order + 1)


def quadrature(kind, n):
    x, w = np.zeros(n), np.zeros(n)
    rc = lib().orc_quadrature(kind, n, _dp(x), _dp(w))
    if rc:
        raise OracleError(rc, "quadrature")
    return x, w


def basis(n, r):
    v, d = ctypes.c_double(), ctypes.c_double()
    lib().orc_basis(n, float(r), ctypes.byref(v), ctypes.byref(d))
    return v.value, d.value


def num_threads():
    return lib().orc_num_threads()
