"""Pins of the oracle's troubled-cell indicator and CSWENO limiter (Section 3)
on the CPU: hand-derived TVB decisions, and invariants the method fixes
(exactness on polynomials, kept cell means, mirror symmetry, reduction of
2D to 1D on y-invariant data)."""
import numpy as np
import pytest

S2 = np.sqrt(2.0)
S32 = np.sqrt(1.5)


def _p1_state(means, jumps_right, jumps_left=None):
    """1D P1 Burgers state with given means and face offsets u(+1)-mean.
    With P1, u(+1)-mean = mean-u(-1) = U1 psi_1(1)."""
    means = np.asarray(means, float)
    U = np.zeros((1, 2, 1, means.size))
    U[0, 0, 0] = means * S2
    U[0, 1, 0] = np.asarray(jumps_right, float) / S32
    return U


def test_tvb_hand_cases(oracle):
    # 5 periodic cells of width 0.2 -> M h^2 = 0.04
    prob = oracle.Problem(dim=1, equation=0, order=1, nx=5, x0=0.0, x1=1.0, bc=(0, 0, 0, 0), tvb_M=1.0)
    # piecewise constant: nothing to flag
    f, _ = prob.indicator(_p1_state([0, 0, 1, 1, 1], [0, 0, 0, 0, 0]))
    assert f.tolist() == [[0, 0, 0, 0, 0]]
    # cell 2: offset 0.3 while its right difference is 0 -> minmod gives 0 -> flagged
    f, _ = prob.indicator(_p1_state([0, 0, 1, 1, 1], [0, 0, 0.3, 0, 0]))
    assert f.tolist() == [[0, 0, 1, 0, 0]]
    # below the TVB bound M h^2 = 0.04 the offset is kept whatever its sign
    f, _ = prob.indicator(_p1_state([0, 0, 1, 1, 1], [0, 0, -0.039, 0, 0]))
    assert f.tolist() == [[0, 0, 0, 0, 0]]
    # ramp: means 0, .5, 1, 1.5, 2 (periodic wrap makes cells 0 and 4 see a jump of -2)
    means = [0, 0.5, 1.0, 1.5, 2.0]
    f, _ = prob.indicator(_p1_state(means, [0.2, 0.2, 0.2, 0.2, 0.2]))
    assert f.tolist() == [[1, 0, 0, 0, 1]]
    # offset larger than the neighbour differences -> flagged
    f, _ = prob.indicator(_p1_state(means, [0.2, 0.2, 0.6, 0.2, 0.2]))
    assert f.tolist() == [[1, 0, 1, 0, 1]]
    # asymmetric differences: left difference 0.5, right difference 0.25, offset 0.3 > 0.25
    f, m = prob.indicator(_p1_state([0, 0.5, 1.0, 1.25, 1.5], [0.0, 0.0, 0.3, 0.0, 0.0]))
    assert f[0, 2] == 1
    # and the margin of that test is |0.3 - 0.25|
    assert abs(m[0, 2] - 0.05) < 1e-12


def test_tvb_2d_direction_or(oracle):
    """A y-direction violation flags the cell even when x is clean."""
    prob = oracle.Problem(dim=2, equation=0, order=1, nx=3, ny=3, bc=(0, 0, 0, 0))
    U = prob.zeros()
    U[0, 0] = 2.0 * np.array([[0, 0, 0], [1, 1, 1], [1, 1, 1]], float)  # means vary in y only
    f, _ = prob.indicator(U)
    assert f.sum() == 0
    U[0, 2, 1, 1] = 0.5 / S32 * S2  # mode (0,1): u(0,+1) - mean = U01 psi_0 psi_1(1)
    f, _ = prob.indicator(U)
    assert f[1, 1] == 1 and f.sum() == 1


def _poly_modes_1d(order, nx, coeffs, x0=0.0, x1=1.0):
    r, w = np.polynomial.legendre.leggauss(order + 6)
    h = (x1 - x0) / nx
    X = x0 + (np.arange(nx)[None, :] + 0.5 * (1 + r[:, None])) * h
    vals = np.polynomial.polynomial.polyval(X, coeffs)
    from tests.dgutil import psi_table
    P = psi_table(order, r)
    return np.einsum("q,nq,qx->nx", w, P, vals)


@pytest.mark.parametrize("order", [1, 2, 3])
@pytest.mark.parametrize("negw", [0, 1])
def test_limiter_exact_on_polynomials_1d(oracle, order, negw):
    nx = 9
    rng = np.random.default_rng(order)
    c = rng.normal(size=order + 1) * [1, 3, 5, 7][: order + 1]
    U = _poly_modes_1d(order, nx, c)[None, :, None, :]
    prob = oracle.Problem(dim=1, equation=0, order=order, nx=nx, bc=(0, 0, 0, 0), negw_mode=negw)
    flags = np.zeros((1, nx), np.uint8)
    flags[0, 1:-1] = 1  # interior cells: their neighbours carry the same polynomial
    out, f, _ = prob.limit(U, flags)
    np.testing.assert_allclose(out[..., 1:-1], U[..., 1:-1], atol=1e-11 * np.abs(U).max())
    assert (out[:, 0] == U[:, 0]).all()


@pytest.mark.parametrize("order", [1, 2, 3])
def test_limiter_exact_on_tensor_polynomials_2d(oracle, order):
    n = 6
    rng = np.random.default_rng(10 + order)
    cx = rng.normal(size=order + 1)
    cy = rng.normal(size=order + 1)
    ux = _poly_modes_1d(order, n, cx)
    uy = _poly_modes_1d(order, n, cy)
    np_ = order + 1
    U = np.zeros((1, np_ * np_, n, n))
    for m in range(np_):
        for k in range(np_):
            U[0, m + np_ * k] = uy[k][:, None] * ux[m][None, :]
    prob = oracle.Problem(dim=2, equation=0, order=order, nx=n, ny=n, bc=(0, 0, 0, 0))
    flags = np.zeros((n, n), np.uint8)
    flags[1:-1, 1:-1] = 1
    out, _, _ = prob.limit(U, flags)
    np.testing.assert_allclose(out[..., 1:-1, 1:-1], U[..., 1:-1, 1:-1], atol=1e-11 * np.abs(U).max())


def _rough_1d(order, nx, nv, seed):
    rng = np.random.default_rng(seed)
    U = np.zeros((nv, order + 1, 1, nx))
    U[:, 0, 0] = (np.sign(np.sin(np.arange(nx) * 0.7 + seed)) + 2.0 + 0.1 * rng.normal(size=(nv, nx))) * S2
    U[:, 1:, 0] = 0.3 * rng.normal(size=(nv, order, nx))
    return U


@pytest.mark.parametrize("order", [1, 2, 3])
def test_limiter_keeps_means_and_mirrors(oracle, order):
    nx = 24
    U = _rough_1d(order, nx, 3, order)
    prob = oracle.Problem(dim=1, equation=1, order=order, nx=nx, bc=(1, 1, 1, 1))
    out, f, _ = prob.limit(U)
    assert f.sum() > 0
    assert (out[:, 0] == U[:, 0]).all()  # Step 6 keeps the mean bit for bit
    # mirror x -> -x: reverse the cells and flip odd modes; momentum changes sign too
    sign_m = np.array([(-1) ** m for m in range(order + 1)], float)[None, :, None, None]
    sign_v = np.array([1, -1, 1], float)[:, None, None, None]
    Um = (U * sign_m * sign_v)[..., ::-1].copy()
    outm, fm, _ = prob.limit(Um)
    assert (fm[:, ::-1] == f).all()
    np.testing.assert_allclose((outm * sign_m * sign_v)[..., ::-1], out, atol=1e-13)


@pytest.mark.parametrize("order", [1, 2, 3])
def test_2d_limiter_on_y_invariant_data_equals_1d(oracle, order):
    nx, ny = 16, 5
    U1 = _rough_1d(order, nx, 1, 40 + order)
    p1 = oracle.Problem(dim=1, equation=0, order=order, nx=nx, bc=(0, 0, 0, 0))
    out1, f1, _ = p1.limit(U1)
    p2 = oracle.Problem(dim=2, equation=0, order=order, nx=nx, ny=ny, bc=(0, 0, 0, 0))
    U2 = p2.zeros()
    for m in range(order + 1):
        U2[0, m] = S2 * U1[0, m, 0][None, :]
    out2, f2, _ = p2.limit(U2)
    assert (f2 == f1).all()
    for m in range(order + 1):
        np.testing.assert_allclose(out2[0, m], np.broadcast_to(S2 * out1[0, m, 0], out2[0, m].shape), atol=1e-12)
    assert np.abs(out2[0, order + 1:]).max() < 1e-12


def test_limiter_x_mirror_2d(oracle):
    order, n = 2, 10
    rng = np.random.default_rng(77)
    prob = oracle.Problem(dim=2, equation=0, order=order, nx=n, ny=n, bc=(1, 1, 0, 0))
    U = prob.zeros()
    U[0, 0] = 2.0 * (np.where(np.add.outer(np.arange(n), 2 * np.arange(n)) > 12, 1.0, -0.5)
                     + 0.05 * rng.normal(size=(n, n)))
    U[0, 1:] = 0.2 * rng.normal(size=(8, n, n))
    out, f, _ = prob.limit(U)
    np_ = order + 1
    sgn = np.array([(-1) ** (q % np_) for q in range(np_ * np_)], float)[None, :, None, None]
    outm, fm, _ = prob.limit((U * sgn)[..., ::-1].copy())
    assert (fm[:, ::-1] == f).all()
    np.testing.assert_allclose((outm * sgn)[..., ::-1], out, atol=1e-13)


def test_all_flagged_equals_override(oracle):
    order, nx = 2, 12
    U = _rough_1d(order, nx, 1, 3)
    a = oracle.Problem(dim=1, equation=0, order=order, nx=nx, indicator_mode=1)
    b = oracle.Problem(dim=1, equation=0, order=order, nx=nx)
    oa, fa, _ = a.limit(U)
    ob, fb, _ = b.limit(U, np.ones((1, nx), np.uint8))
    assert fa.all() and fb.all()
    assert (oa == ob).all()
