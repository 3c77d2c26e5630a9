"""Exact solutions the paper compares against (test helpers, CPU only).

* Burgers before shock formation: the characteristic solution
  u = u0(x - u t), solved pointwise by Newton's method (the paper cites
  Harten, Engquist, Osher and Chakravarthy for it).
* Shock tubes (Sod, Lax): the textbook exact Riemann solver for the ideal
  gas Euler equations (pressure-star Newton iteration, Toro, ch. 4).
"""
import numpy as np


def burgers_characteristic(u0, du0, x, t, iters=60):
    """Solve u = u0(x - u t) pointwise (valid before the shock forms)."""
    u = u0(x)
    for _ in range(iters):
        xi = x - u * t
        F = u - u0(xi)
        dF = 1.0 + t * du0(xi)
        u = u - F / dF
    return u


def _f_k(p, rho, pk, ck, g):
    if p > pk:  # shock
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pk
        q = np.sqrt(A / (p + B))
        return (p - pk) * q, q * (1.0 - 0.5 * (p - pk) / (p + B))
    # rarefaction
    pr = p / pk
    f = 2.0 * ck / (g - 1.0) * (pr ** ((g - 1.0) / (2.0 * g)) - 1.0)
    df = 1.0 / (rho * ck) * pr ** (-(g + 1.0) / (2.0 * g))
    return f, df


def riemann_star(L, R, g=1.4):
    rl, ul, pl = L
    rr, ur, pr = R
    cl, cr = np.sqrt(g * pl / rl), np.sqrt(g * pr / rr)
    p = max(1e-8, 0.5 * (pl + pr) - 0.125 * (ur - ul) * (rl + rr) * (cl + cr))
    for _ in range(100):
        fl, dfl = _f_k(p, rl, pl, cl, g)
        fr, dfr = _f_k(p, rr, pr, cr, g)
        dp = (fl + fr + ur - ul) / (dfl + dfr)
        pn = max(1e-10, p - dp)
        if abs(pn - p) < 1e-14 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _f_k(p, rl, pl, cl, g)
    fr, _ = _f_k(p, rr, pr, cr, g)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p, u


def riemann_sample(L, R, s, g=1.4):
    """Primitive (rho, u, p) of the exact solution at similarity s = x/t."""
    rl, ul, pl = L
    rr, ur, pr = R
    cl, cr = np.sqrt(g * pl / rl), np.sqrt(g * pr / rr)
    ps, us = riemann_star(L, R, g)
    s = np.asarray(s, dtype=np.float64)
    rho = np.empty_like(s)
    u = np.empty_like(s)
    p = np.empty_like(s)
    gm = (g - 1.0) / (g + 1.0)
    for k, sk in np.ndenumerate(s):
        if sk <= us:  # left of contact
            if ps > pl:  # left shock
                rls = rl * (ps / pl + gm) / (gm * ps / pl + 1.0)
                sl = ul - cl * np.sqrt((g + 1.0) / (2 * g) * ps / pl + (g - 1.0) / (2 * g))
                val = (rl, ul, pl) if sk <= sl else (rls, us, ps)
            else:  # left rarefaction
                cls = cl * (ps / pl) ** ((g - 1.0) / (2 * g))
                shl, stl = ul - cl, us - cls
                if sk <= shl:
                    val = (rl, ul, pl)
                elif sk >= stl:
                    val = (rl * (ps / pl) ** (1.0 / g), us, ps)
                else:
                    uu = 2.0 / (g + 1.0) * (cl + (g - 1.0) / 2.0 * ul + sk)
                    cc = 2.0 / (g + 1.0) * (cl + (g - 1.0) / 2.0 * (ul - sk))
                    rr_ = rl * (cc / cl) ** (2.0 / (g - 1.0))
                    val = (rr_, uu, pl * (cc / cl) ** (2.0 * g / (g - 1.0)))
        else:  # right of contact
            if ps > pr:  # right shock
                rrs = rr * (ps / pr + gm) / (gm * ps / pr + 1.0)
                sr = ur + cr * np.sqrt((g + 1.0) / (2 * g) * ps / pr + (g - 1.0) / (2 * g))
                val = (rr, ur, pr) if sk >= sr else (rrs, us, ps)
            else:
                crs = cr * (ps / pr) ** ((g - 1.0) / (2 * g))
                shr, stt = ur + cr, us + crs
                if sk >= shr:
                    val = (rr, ur, pr)
                elif sk <= stt:
                    val = (rr * (ps / pr) ** (1.0 / g), us, ps)
                else:
                    uu = 2.0 / (g + 1.0) * (-cr + (g - 1.0) / 2.0 * ur + sk)
                    cc = 2.0 / (g + 1.0) * (cr - (g - 1.0) / 2.0 * (ur - sk))
                    rr_ = rr * (cc / cr) ** (2.0 / (g - 1.0))
                    val = (rr_, uu, pr * (cc / cr) ** (2.0 * g / (g - 1.0)))
        rho[k], u[k], p[k] = val
    return rho, u, p
