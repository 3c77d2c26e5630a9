"""Test-side helpers: evaluate modal states with numpy's Legendre routines,
error norms, and oracle set-up from a workload (CPU only)."""
import numpy as np


def psi_table(order, r):
    """psi_n(r) = sqrt((2n+1)/2) P_n(r), rows n, columns r (numpy Legendre)."""
    r = np.asarray(r, dtype=np.float64)
    out = np.empty((order + 1, r.size))
    for n in range(order + 1):
        c = np.zeros(n + 1)
        c[n] = 1.0
        out[n] = np.sqrt((2 * n + 1) / 2.0) * np.polynomial.legendre.legval(r, c)
    return out


def eval_1d(U, order, r):
    """U [nv, N+1, 1, nx] -> values [nv, len(r), nx]."""
    P = psi_table(order, r)
    return np.einsum("vnx,nq->vqx", U[:, :, 0, :], P)


def eval_2d(U, order, r):
    """U [nv, (N+1)^2, ny, nx] -> values [nv, qy, qx, ny, nx] on the tensor nodes r x r."""
    P = psi_table(order, r)
    np_ = order + 1
    nv, nm, ny, nx = U.shape
    U5 = U.reshape(nv, np_, np_, ny, nx)  # [v, n(y), m(x), j, i]
    return np.einsum("vnmji,mq,np->vpqji", U5, P, P)


def cell_means(U, dim):
    return U[:, 0] / (np.sqrt(2.0) if dim == 1 else 2.0)


def l1_linf_1d(U, order, x0, x1, exact, nq=None):
    """(1/|D|) sum_cells int |u_h - u| and the max over the quadrature points."""
    nq = nq or order + 4
    r, w = np.polynomial.legendre.leggauss(nq)
    nx = U.shape[-1]
    h = (x1 - x0) / nx
    X = x0 + (np.arange(nx)[None, :] + 0.5 * (1 + r[:, None])) * h
    e = np.abs(eval_1d(U, order, r)[0] - exact(X))
    return float((w[:, None] * e).sum() * 0.5 * h / (x1 - x0)), float(e.max())


def l1_linf_2d(U, order, x0, x1, y0, y1, exact, var=0, nq=None):
    nq = nq or order + 3
    r, w = np.polynomial.legendre.leggauss(nq)
    ny, nx = U.shape[-2:]
    hx, hy = (x1 - x0) / nx, (y1 - y0) / ny
    X = x0 + (np.arange(nx)[None, :] + 0.5 * (1 + r[:, None])) * hx  # [q, i]
    Y = y0 + (np.arange(ny)[None, :] + 0.5 * (1 + r[:, None])) * hy  # [p, j]
    vals = eval_2d(U[var:var + 1], order, r)[0]  # [p, q, j, i]
    XX = X[None, :, None, :]
    YY = Y[:, None, :, None]
    e = np.abs(vals - exact(XX, YY))
    W = w[:, None, None, None] * w[None, :, None, None]
    return float((W * e).sum() * 0.25 * hx * hy / ((x1 - x0) * (y1 - y0))), float(e.max())


def oracle_problem(O, wl, **over):
    kw = dict(dim=wl.dim, equation=wl.equation, order=wl.order, nx=wl.nx, ny=wl.ny, x0=wl.x0, x1=wl.x1,
              y0=wl.y0, y1=wl.y1, bc=tuple(wl.bc), gamma=wl.gamma, cfl=wl.cfl)
    kw.update(wl.bc_extra)
    kw.update(wl.mesh)
    kw.update(over)
    return O.Problem(**kw)


def oracle_initial_state(O, wl, prob=None, limit=False):
    prob = prob or oracle_problem(O, wl)
    r, _ = prob.proj_nodes()
    pv = wl.point_values(r)
    U = prob.project(pv)
    if limit:
        U = prob.limit(U)[0]
    return prob, U


def orders(errors):
    e = np.asarray(errors)
    return np.log2(e[:-1] / e[1:])
