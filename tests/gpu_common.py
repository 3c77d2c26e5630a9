"""Helpers of the GPU parity tests: matching oracle/GPU problems, seeded
inputs shared by both sides, and the comparison rules.

Tolerance (written in every test through ``assert_close``): the GPU result
must agree with the FP64 oracle to 1e-12 relative per call, measured as
max |gpu - oracle| / max(1, max |oracle|) per variable.  Troubled-cell flags
must be identical except in cells whose oracle margin is below 1e-10."""
import numpy as np

REL_TOL = 1e-12
MARGIN_TOL = 1e-10


def configs(dim, eq, order, nx, ny=1, bc=None, **kw):
    if bc is None:
        bc = (0, 0, 0, 0)
    d = dict(dim=dim, equation=eq, order=order, nx=nx, ny=ny if dim == 2 else 1, bc=tuple(bc),
             x0=kw.pop("x0", 0.0), x1=kw.pop("x1", 1.0), y0=kw.pop("y0", 0.0), y1=kw.pop("y1", 1.0))
    d.update(kw)
    return d


def make_pair(O, D, cfg, device="cuda"):
    oc = dict(cfg)
    if "indicator" in oc:
        oc["indicator_mode"] = oc.pop("indicator")
    return O.Problem(**oc), D.Problem(device=device, **cfg)


def rough_state(O, prob, seed, amplitude=0.3, extra_noise=0.05):
    """Projection of a seeded rough field plus seeded noise on the high modes."""
    from paper_1904_11147_amd import workloads as W
    if prob.dim == 1:
        ic = W.random_state_1d(prob.nx, prob.order, prob.equation, seed, amplitude)
    else:
        ic = W.random_state_2d(prob.equation, seed, amplitude)
    wl = W.Workload("rough", prob.dim, prob.equation, prob.order, prob.nx, prob.ny, prob.x0, prob.x1, prob.y0,
                    prob.y1, prob.bc, 0.1, 1.0, ic)
    r, _ = prob.proj_nodes()
    U0 = prob.project(wl.point_values(r))
    noise = np.random.default_rng(seed + 1000).normal(size=U0[:, 1:].shape)
    scale = np.abs(U0[:, :1]).mean(axis=(1, 2, 3), keepdims=True)
    for _ in range(30):  # Euler inputs must stay physical at every quadrature point
        U = U0.copy()
        U[:, 1:] += extra_noise * noise * scale
        try:
            prob.residual(U)
            return U
        except O.OracleError:
            extra_noise *= 0.5
    raise RuntimeError("could not build a physical rough state")


def worst(got, ref):
    """(var, mode, j, i) of the largest difference, for diagnostics."""
    d = np.abs(np.asarray(got) - np.asarray(ref))
    return np.unravel_index(np.argmax(d), d.shape), float(d.max())


def rel_err(got, ref):
    got = np.asarray(got)
    ref = np.asarray(ref)
    out = 0.0
    for v in range(ref.shape[0]):
        d = np.abs(got[v] - ref[v]).max()
        out = max(out, d / max(1.0, np.abs(ref[v]).max()))
    return out


def assert_close(got, ref, tol=REL_TOL, what=""):
    e = rel_err(got, ref)
    assert e <= tol, f"{what}: relative difference {e:.3e} > {tol:.1e}"
    return e


def flags_agree(gpu_flags, ref_flags, ref_margin, tol=MARGIN_TOL, what=""):
    """Cells whose flags differ, and whether every one of them is near the
    threshold by the oracle's margin.  Differing cells are listed (printed
    with their margins), as the parity bar asks."""
    diff = np.argwhere(np.asarray(gpu_flags) != np.asarray(ref_flags))
    near = [tuple(c) for c in diff if ref_margin[tuple(c)] < tol]
    if len(diff):
        cells = [(tuple(int(x) for x in c), float(ref_margin[tuple(c)])) for c in diff]
        print(f"flags differ {what}: {len(diff)} cell(s) (index, oracle margin): {cells}")
    return diff, len(near) == len(diff)
