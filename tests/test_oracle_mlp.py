"""Pins of the FP64 reference of the learned indicator (CPU): finite-difference
gradient check, Adam against its closed form on a quadratic, and feature
invariances that the definition fixes."""
import numpy as np

from oracle import mlp_oracle as M


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    F, n = 23, 40
    P = M.init_params(F, seed=1)
    for k in ("b1", "b2"):
        P[k] = rng.normal(size=P[k].shape) * 0.1
    X = rng.normal(size=(n, F))
    y = (rng.random(n) > 0.5).astype(float)
    w = 1.0 + rng.random(n)
    L, G = M.grads(P, X, y, w, bf16=False)
    eps = 1e-6
    for key in ("W1", "b1", "W2", "b2", "w3", "b3"):
        flat = P[key].reshape(-1)
        for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + eps
            lp, _ = M.loss(P, X, y, w, bf16=False)
            flat[idx] = old - eps
            lm, _ = M.loss(P, X, y, w, bf16=False)
            flat[idx] = old
            fd = (lp - lm) / (2 * eps)
            g = G[key].reshape(-1)[idx]
            assert abs(fd - g) <= 1e-6 * max(1.0, abs(fd)), (key, idx, fd, g)


def test_adam_first_step_moves_by_lr():
    """The first bias-corrected Adam step moves every parameter by lr sign(g)."""
    P = {"a": np.array([1.0, -2.0, 3.0])}
    G = {"a": np.array([0.5, -4.0, 1e-3])}
    st = {}
    M.adam(P, G, st, lr=0.01, eps=0.0)
    np.testing.assert_allclose(P["a"], [0.99, -1.99, 2.99], atol=1e-12)


def test_bf16_rounding_is_nearest_even():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -2.5, 3.140625])
    r = M.bf16_round(vals)
    np.testing.assert_array_equal(r, [1.0, 1.0, 1.0 + 2 ** -7, -2.5, 3.140625])


def test_features_are_invariant_to_offset_and_scale():
    rng = np.random.default_rng(4)
    U = rng.normal(size=(4, 9, 5, 6))
    f0 = M.features(U, 0.01, 1.0, (1, 1, 1, 1))
    V = U.copy()
    V[:, 0] += 7.0  # the same constant on every cell mean of every variable
    np.testing.assert_allclose(M.features(V, 0.01, 1.0, (1, 1, 1, 1)), f0, atol=1e-12)
    np.testing.assert_allclose(M.features(3.0 * U, 0.01, 1.0, (1, 1, 1, 1)), f0, atol=1e-12)
    assert np.abs(f0).max() <= 1.0 + 1e-15
    # the centre's own mean is always zero
    assert np.abs(f0[:, 0]).max() == 0.0


def test_features_normalise_each_variable_on_its_own():
    """s_v is per variable: scaling or shifting the means of one variable
    leaves every feature unchanged, and scaling one variable below M h^2
    changes only that variable's features."""
    rng = np.random.default_rng(5)
    U = rng.normal(size=(4, 9, 5, 6))
    bc = (0, 1, 0, 1)
    f0 = M.features(U, 0.01, 1.0, bc).reshape(30, 4, 5, 9)
    for v in range(4):
        V = U.copy()
        V[v] *= 25.0
        np.testing.assert_allclose(M.features(V, 0.01, 1.0, bc).reshape(30, 4, 5, 9), f0, atol=1e-12)
        V = U.copy()
        V[v, 0] -= 3.0
        np.testing.assert_allclose(M.features(V, 0.01, 1.0, bc).reshape(30, 4, 5, 9), f0, atol=1e-12)
        # variable v shrunk far below M h^2 = 1e-4: its own features scale
        # with it (s_v = M h^2), the others' stay as they were
        V = U.copy()
        V[v] *= 1e-7
        f = M.features(V, 0.01, 1.0, bc).reshape(30, 4, 5, 9)
        others = [w for w in range(4) if w != v]
        np.testing.assert_allclose(f[:, others], f0[:, others], atol=1e-12)
        assert np.abs(f[:, v]).max() < 1e-2


def test_features_follow_the_neighbour_order_and_ghost_rules():
    """Layout [v][C, W, E, S, N][mode]; a transmissive side mirrors the
    boundary cell (odd modes in the normal direction change sign), a periodic
    side wraps.  Checked on a field whose cells are labelled by position."""
    nx, ny = 4, 3
    U = np.zeros((1, 4, ny, nx))  # Q1 scalar: modes q = m + 2 n
    for j in range(ny):
        for i in range(nx):
            U[0, :, j, i] = [0.0, 1 + i + 10 * j, 2 + i + 10 * j, 3 + i + 10 * j]
    hx = 1.0  # M h^2 = 1 dominates nothing; s = max |entry|
    f = M.features(U, hx, 1e-9, (0, 0, 1, 1)).reshape(ny * nx, 1, 5, 4)
    for j in range(ny):
        for i in range(nx):
            blk = f[j * nx + i, 0]
            w = U[0, :, j, (i - 1) % nx]
            e = U[0, :, j, (i + 1) % nx]
            sgn = np.array([1, 1, -1, -1])  # modes odd in y flip across a south/north side
            so = U[0, :, j - 1, i] if j > 0 else U[0, :, 0, i] * sgn
            no = U[0, :, j + 1, i] if j < ny - 1 else U[0, :, ny - 1, i] * sgn
            cells = np.stack((U[0, :, j, i], w, e, so, no))
            want = cells / np.abs(cells).max()  # mode-0 entries are all zero here
            np.testing.assert_allclose(blk, want, atol=1e-12)
