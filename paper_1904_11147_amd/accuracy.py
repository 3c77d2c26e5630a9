"""Accuracy studies in the style of the paper's Tables 1-4, run through the
library on the GPU: L1 and L-infinity errors and orders on meshes whose
nodes are moved by up to 10% (seeded), without the limiter and with CSWENO
under the TVB (M = 1) and the KXRCF indicator (the paper's).

    python -m paper_1904_11147_amd.accuracy [--out results/accuracy_nonuniform.json] [--quick]

* Table 1: 1D Burgers, u0 = 0.5 + sin x on [0, 2 pi], periodic, t = 0.5,
  P1-P3, K = 20 ... 320.
* Table 2: 2D Burgers, u0 = 0.5 + sin(x + y) on [0, 2 pi]^2, periodic,
  t = 0.25, Q1-Q3, K x K = 10^2 ... 80^2.
* Table 3: 2D Euler, rho = 1 + 0.2 sin(x + y), (u, v, p) = (0.7, 0.3, 1) on
  [0, 2 pi]^2, periodic, t = 2 pi, density errors.
* Table 4: 2D Euler isentropic vortex (strength 5, free stream (1, 0)) on
  [0, 10] x [-5, 5], periodic, t = 2, density errors, K = 20 ... 160.

Exact solutions: Burgers by Newton's method on the characteristic equation
u = u0(x - u t) (2D: in s = x + y with speed 2u), the Euler cases by
translation.  Time steps: the CFL rule (0.1; P3 0.05) for P1 and P2; for
P3 a fixed step, the smaller of that rule's initial step and 0.05 h^(4/3),
so that the third-order Runge-Kutta error stays below the spatial one.
Errors are (1/|D|) sum over cells of the integral of |u_h - u| and the
largest |u_h - u| over (N+4)-point Gauss nodes.
"""
import argparse
import json
import os
import time

import numpy as np
import torch

from . import dg
from . import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))


def _psi(order, r):
    out = np.empty((order + 1, len(r)))
    for n in range(order + 1):
        c = np.zeros(n + 1)
        c[n] = 1.0
        out[n] = np.sqrt((2 * n + 1) / 2.0) * np.polynomial.legendre.legval(r, c)
    return out


def _burgers_exact(u0, du0, s, t, speed=1.0):
    """u(s, t) of u_t + speed * u u_s = 0 with u(s, 0) = u0(s): Newton on
    xi + speed * u0(xi) t - s = 0, started from s."""
    xi = np.array(s, dtype=np.float64)
    for _ in range(100):
        f = xi + speed * u0(xi) * t - s
        d = f / (1.0 + speed * du0(xi) * t)
        xi -= d
        if np.abs(d).max() < 1e-15:
            break
    return u0(xi)


def _errors(U, wl, exact, var=0):
    nq = wl.order + 4
    r, w = np.polynomial.legendre.leggauss(nq)
    P = _psi(wl.order, r)
    xn = wl.mesh["xn"]
    hx = np.diff(xn)
    X = xn[None, :-1] + 0.5 * (1 + r[:, None]) * hx[None, :]  # [q, i]
    if wl.dim == 1:
        vals = np.einsum("nx,nq->qx", U[var, :, 0, :], P)
        e = np.abs(vals - exact(X))
        l1 = float((w[:, None] * e * 0.5 * hx[None, :]).sum() / (wl.x1 - wl.x0))
        return l1, float(e.max())
    yn = wl.mesh["yn"]
    hy = np.diff(yn)
    Y = yn[None, :-1] + 0.5 * (1 + r[:, None]) * hy[None, :]  # [p, j]
    NP = wl.order + 1
    vals = np.einsum("nmji,mq,np->pqji", U[var].reshape(NP, NP, wl.ny, wl.nx), P, P)
    e = np.abs(vals - exact(X[None, :, None, :], Y[:, None, :, None]))
    Wt = (w[:, None] * w[None, :])[:, :, None, None] * (0.25 * hy[None, None, :, None] * hx[None, None, None, :])
    return float((Wt * e).sum() / ((wl.x1 - wl.x0) * (wl.y1 - wl.y0))), float(e.max())


VARIANTS = (  # (name, limiter, indicator)
    ("no limiter", dg.LIM_NONE, dg.IND_TVB),
    ("CSWENO, TVB M=1", dg.LIM_CSWENO, dg.IND_TVB),
    ("CSWENO, KXRCF", dg.LIM_CSWENO, dg.IND_KXRCF),
)


def _run(wl, limiter, indicator, device):
    prob = dg.problem_from_workload(wl, device=device, limiter=limiter, indicator=indicator)
    state = dg.initial_state(prob, wl, limit=limiter != dg.LIM_NONE)
    h = np.diff(wl.mesh["xn"]).min()
    dt = 0.0
    if wl.order == 3:  # fixed step ~ h^(4/3): the RK3 error below the fourth-order spatial one
        dt = min(prob.cfl_dt(state), 0.05 * h ** (4.0 / 3.0))
    t, n = prob.step(state, 0.0, wl.t_end, dt=dt)
    U = state.cpu().numpy()
    prob.close()
    return U, t, n


def _table(name, make, exact, sizes, orders, device, var=0):
    rows = []
    for order in orders:
        for vname, lim, ind in VARIANTS:
            prev = None
            for K in sizes:
                wl = make(K, order).nonuniform(seed=1000 + K)
                a = time.perf_counter()
                try:
                    U, t, n = _run(wl, lim, ind, device)
                except dg.DGError as e:  # an under-resolved coarse mesh
                    rows.append({"table": name, "order": order, "variant": vname, "K": K, "status": str(e)})
                    print(f"{name} P{order} K={K}: {e}", flush=True)
                    prev = None
                    continue
                l1, li = _errors(U, wl, exact(t), var)
                row = {"table": name, "order": order, "variant": vname, "K": K, "steps": n, "t": t,
                       "l1": l1, "linf": li, "seconds": time.perf_counter() - a}
                if prev:
                    row["order_l1"] = float(np.log2(prev["l1"] / l1))
                    row["order_linf"] = float(np.log2(prev["linf"] / li))
                rows.append(row)
                prev = row
                print(f"{name} P{order} {vname} K={K}: L1 {l1:.3e} "
                      f"{row.get('order_l1', float('nan')):.2f}  Linf {li:.3e} {row.get('order_linf', float('nan')):.2f}",
                      flush=True)
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(HERE, "results", "accuracy_nonuniform.json"))
    ap.add_argument("--quick", action="store_true", help="three mesh sizes per table")
    ap.add_argument("--device", default="cuda:0")
    a = ap.parse_args()
    two_pi = 2.0 * np.pi
    u0 = lambda x: 0.5 + np.sin(x)  # noqa: E731
    du0 = lambda x: np.cos(x)  # noqa: E731
    s1 = (20, 40, 80) if a.quick else (20, 40, 80, 160, 320)
    s2 = (10, 20, 40) if a.quick else (10, 20, 40, 80)
    rows = []
    rows += _table("1: 1D Burgers", lambda K, o: W.burgers1d(nx=K, order=o, t_end=0.5, x0=0.0, x1=two_pi, omega=1.0),
                   lambda t: (lambda X: _burgers_exact(u0, du0, X, t)), s1, (1, 2, 3), a.device)
    rows += _table("2: 2D Burgers", lambda K, o: W.burgers2d(n=K, order=o, t_end=0.25, L=two_pi, omega=1.0),
                   lambda t: (lambda X, Y: _burgers_exact(u0, du0, X + Y, t, speed=2.0)), s2, (1, 2, 3), a.device)
    rows += _table("3: 2D Euler density wave", lambda K, o: W.density_wave(n=K, order=o),
                   lambda t: (lambda X, Y: W.density_wave_exact(X, Y, t)), s2, (1, 2, 3), a.device)

    def vortex_exact(t):
        wl = W.isentropic_vortex(n=4, order=1)

        def f(X, Y):
            Xs = wl.x0 + np.mod(X - t - wl.x0, wl.x1 - wl.x0)  # free stream (1, 0), periodic
            return wl.ic(Xs, Y)[0]
        return f
    rows += _table("4: 2D Euler isentropic vortex", lambda K, o: W.isentropic_vortex(n=K, order=o), vortex_exact,
                   tuple(2 * k for k in s2), (1, 2, 3), a.device)
    os.makedirs(os.path.dirname(a.out), exist_ok=True)
    meta = {"mesh": "tensor-product, interior nodes moved by up to 10% of the uniform width (seed 1000 + K)",
            "device": torch.cuda.get_device_name(0) if torch.cuda.is_available() else None}
    json.dump({"meta": meta, "rows": rows}, open(a.out, "w"), indent=1)
    print("wrote", a.out)


if __name__ == "__main__":
    main()
