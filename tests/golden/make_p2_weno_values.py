"""Writes p2_weno_values.json: P2 WENO point values computed from what the
paper prints, in 50-digit arithmetic.

Inputs are only the printed P2 data of Sec. 3 (in p2_weno_tables.json, with
the misprint fixes listed there): the reconstruction rows p0, p1, p2 of
T^3-T^6 (Step 3), the linear weights gamma of each point (Step 3) and the
smoothness indicators beta_0..beta_2 as quadratic forms in the five stencil
means (Step 4).  Step 5 is applied as written apart from the Sigma in the
printed denominator (reading: the Jiang-Shu form that the paper's cited
WENO builds on), so

    wbar_i = gamma_i / (eps + beta_i)^2,   w_i = wbar_i / sum_k wbar_k,
    u_G    = sum_i w_i p_i(x_G),           eps = 1e-6.

Nothing here calls the oracle or the GPU library.  Each stencil is stored as
the doubles the tests pass in (so the 50-digit evaluation starts from the
same binary inputs).  Run:  python tests/golden/make_p2_weno_values.py
"""
import json
import os

import mpmath as mp
import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
mp.mp.dps = 50
EPS = mp.mpf("1e-6")


def _mp(expr):
    """A printed entry ('(235-33*sqrt(5))/950') as a 50-digit number."""
    return mp.mpf(eval(expr, {"__builtins__": {}}, {"sqrt": lambda v: mp.sqrt(mp.mpf(v))}))


def _stencils():
    """Named five-mean stencils (two half-cells of the left neighbour, the
    troubled cell, two half-cells of the right neighbour)."""
    rng = np.random.default_rng(20190425)
    out = {
        # a jump between the troubled cell and its right neighbour
        "step_right": [1.0, 1.0, 1.0, 0.2, 0.2],
        # a jump inside the left neighbour
        "step_left": [-0.5, 0.75, 0.75, 0.75, 0.75],
        # a kink at the troubled cell's right edge: flat, then slope 1
        "kink": [0.0, 0.0, 0.0, 0.25, 0.75],
        # smooth data whose smoothness indicators are of the size of eps
        "smooth_beta_near_eps": [0.5 + 1e-3 * v for v in (-0.8, -0.3, 0.1, 0.45, 1.1)],
        # smooth quadratic of unit size (all betas >> eps)
        "smooth_large": [2.0 - 0.3 * v + 0.8 * v * v for v in (-1.25, -0.75, 0.0, 0.75, 1.25)],
    }
    for k in range(3):
        out[f"random_{k}"] = list(rng.normal(size=5))
    return {k: [float(np.float64(v)) for v in vals] for k, vals in out.items()}


def main():
    g = json.load(open(os.path.join(HERE, "p2_weno_tables.json")))
    beta_forms = []
    for i in range(3):
        spec = g["beta"][f"beta{i}"]
        terms = []
        for term, coef in spec["terms"].items():
            u, v = term.split("*")
            terms.append((int(u[1]), int(v[1]), mp.mpf(coef)))
        beta_forms.append((terms, mp.mpf(spec["den"])))
    points = []
    for pt in g["points"]:
        rows = [[_mp(e) for e in row] for row in pt["T"][:3]]
        gam = [_mp(e) for e in pt["gamma"]]
        points.append((pt["r"], rows, gam))

    cases = []
    for name, a in _stencils().items():
        A = [mp.mpf(v) for v in a]  # exact: every double is a 50-digit number
        beta = []
        for terms, den in beta_forms:
            beta.append(sum(c * A[u] * A[v] for u, v, c in terms) / den)
        vals = []
        for r, rows, gam in points:
            p = [sum(rows[i][k] * A[k] for k in range(5)) for i in range(3)]
            wb = [gam[i] / (EPS + beta[i]) ** 2 for i in range(3)]
            s = sum(wb)
            vals.append(mp.nstr(sum(wb[i] / s * p[i] for i in range(3)), 30))
        cases.append({"name": name, "means": a, "values": vals,
                      "beta": [mp.nstr(b, 20) for b in beta]})
    doc = {
        "source": "Kochi & Ramakrishna, arXiv 1904.11147, Section 3, Steps 3-5: P2 WENO values at the four "
                  "Gauss-Lobatto points r = -1, -1/sqrt(5), 1/sqrt(5), 1 from the printed T^3-T^6 rows, "
                  "linear weights and smoothness indicators",
        "reading": "Step 5 nonlinear weights wbar_i = gamma_i / (eps + beta_i)^2 normalised to sum to one "
                   "(the printed Sigma in the denominator would make every weight linear); eps = 1e-6",
        "generator": "tests/golden/make_p2_weno_values.py (50-digit mpmath; no oracle, no GPU)",
        "eps": 1e-6,
        "cases": cases,
    }
    with open(os.path.join(HERE, "p2_weno_values.json"), "w") as f:
        json.dump(doc, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
