"""Pins of the oracle's nonlinear WENO weights (Sec. 3, Step 5), CPU only.

Polynomial reproduction (in test_oracle_tables) holds for any weights, so it
cannot see a wrong Step 5.  Two pins that can:

* golden P2 values: the WENO value at every Step-1 point for jumps, a kink,
  smooth data whose smoothness indicators are of the size of eps, and random
  stencils, computed in 50-digit arithmetic from the printed T^3-T^6 rows,
  linear weights and smoothness indicators with wbar = gamma/(eps+beta)^2
  (tests/golden/make_p2_weno_values.py; no oracle involved);
* the ENO property for P1, P2, P3 (split form included): when some candidate
  stencils see constant data and the others cross a jump of size J, the
  value equals the constant up to a multiple of (eps/beta)^2 J, the decay
  that the power 2 in Step 5 fixes (power 1 would leave eps/beta).
"""
import json
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "p2_weno_values.json")


def test_p2_weno_values_match_printed_tables(oracle):
    g = json.load(open(GOLDEN))
    assert g["eps"] == 1e-6
    worst = 0.0
    for case in g["cases"]:
        a = np.array(case["means"])
        scale = max(1.0, np.abs(a).max())
        for G, want in enumerate(case["values"]):
            got = oracle.weno_eval(2, G, a, g["eps"], oracle.NEGW_SPLIT)
            err = abs(got - float(want)) / scale
            worst = max(worst, err)
            assert err <= 2e-14, (case["name"], G, got, want)
    assert worst <= 2e-14


def _jump_stencils(N):
    """(means, smooth value) pairs: a unit or small jump between two
    subcells, placed so that at least one candidate stencil (N+1 consecutive
    means) sees only the constant on the troubled cell's side."""
    n = 2 * N + 1
    out = []
    for J in (1.0, -3.0, 0.05):
        for cut in range(1, n):
            # constant c left of the cut, c + J right of it; the troubled cell is index N
            c = 0.4
            a = np.where(np.arange(n) < cut, c, c + J)
            left_smooth = cut >= N + 1          # stencil 0 = means 0..N is constant
            right_smooth = n - cut >= N + 1     # stencil N = means N..2N is constant
            if left_smooth or right_smooth:
                out.append((a, a[N], J))
    return out


@pytest.mark.parametrize("N", [1, 2, 3])
def test_eno_property_at_jumps(oracle, N):
    """With the jump outside the troubled cell's smooth candidate stencils,
    u_G equals the troubled cell's constant up to C (eps/beta_cross)^2 J."""
    t = oracle.weno_tables(N)
    eps = 1e-6
    for a, c, J in _jump_stencils(N):
        # smallest smoothness indicator of a stencil that crosses the jump
        bmin = np.inf
        for i in range(N + 1):
            s = a[i:i + N + 1] - a[N]
            b = s @ t["beta"][i] @ s
            if b > 0:
                bmin = min(bmin, b)
        bound = 50.0 * (eps / bmin) ** 2 * abs(J) + 1e-15
        for G in range(len(t["rg"])):
            got = oracle.weno_eval(N, G, a, eps, oracle.NEGW_SPLIT)
            assert abs(got - c) <= bound, (N, G, list(a), got - c, bound)


@pytest.mark.parametrize("N", [1, 2, 3])
@pytest.mark.parametrize("mode", ["raw", "split"])
def test_weights_tend_to_linear_on_smooth_data(oracle, N, mode):
    """On smooth data with beta >> eps the nonlinear weights are within
    O(beta differences) of the linear ones; as eps grows (beta << eps) they
    become exactly linear, so the value is the Q value gamma . p.  With the
    positive/negative split of the P3 inner points the same limit holds: the
    two normalised groups recombine to the linear weights (gamma = sigma+
    gamma+ - sigma- gamma-), so a wrong group sign, normalisation or factor
    fails here."""
    t = oracle.weno_tables(N)
    flag = oracle.NEGW_RAW if mode == "raw" else oracle.NEGW_SPLIT
    rng = np.random.default_rng(7 + N)
    for _ in range(5):
        a = 1.0 + 1e-4 * rng.normal(size=2 * N + 1)
        for G in range(len(t["rg"])):
            lin = t["gamma"][G] @ (t["rows"][G] @ a)
            got = oracle.weno_eval(N, G, a, 1e10, flag)
            assert abs(got - lin) <= 1e-13, (N, G, mode, got - lin)
