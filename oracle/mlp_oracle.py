"""FP64 reference of the learned troubled-cell indicator (test infrastructure
only: tests, smoke check and benchmark baseline).

Not in the paper (its indicator is KXRCF, Sec. 3); specified by the workload:
a small MLP over normalised modal coefficients of a cell and its immediate
neighbours, trained on flags and limited/unlimited error pairs of the plain
method, with the TVB indicator as fallback in an uncertain probability band.

Features of cell (i, j), per variable v (in the order C, W, E, S, N, each with
its (N+1)^2 modes): the five mode-0 entries are shifted by the centre cell's
mode 0, then all 5 (N+1)^2 entries are divided by
s_v = max(max |entry|, M h_x^2).  Cells outside the mesh follow the boundary
condition (periodic wrap or even reflection).  Layout: [v][cell][mode].

Network: h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), z = w3 . h2 + b3,
p = sigmoid(z); W1, W2, w3 and the inputs and hidden activations are rounded
to bfloat16 (round to nearest even), accumulation in the reference is FP64.
Loss: weighted binary cross-entropy, mean over the batch.
"""
import numpy as np

HIDDEN = 64


def bf16_round(a):
    """Round float values to bfloat16 (nearest even), returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _ghost(U, i, j, bc):
    """Modes of cell (i, j) (one layer outside allowed) under the boundary
    conditions: U [nv][(N+1)^2][ny][nx]."""
    nv, nm, ny, nx = U.shape
    np_ = int(round(np.sqrt(nm)))
    fx = fy = False
    if i < 0:
        i, fx = (i + nx, False) if bc[0] == 0 else (0, True)
    elif i >= nx:
        i, fx = (i - nx, False) if bc[1] == 0 else (nx - 1, True)
    if j < 0:
        j, fy = (j + ny, False) if bc[2] == 0 else (0, True)
    elif j >= ny:
        j, fy = (j - ny, False) if bc[3] == 0 else (ny - 1, True)
    c = U[:, :, j, i].copy()
    for q in range(nm):
        m, n = q % np_, q // np_
        s = (-1) ** ((m if fx else 0) + (n if fy else 0))
        c[:, q] *= s
    return c


def features(U, hx, tvb_M, bc):
    """All cells' features, float64 [ny*nx][nv*5*(N+1)^2]."""
    nv, nm, ny, nx = U.shape
    out = np.zeros((ny * nx, nv * 5 * nm))
    Mh2 = tvb_M * hx * hx
    for j in range(ny):
        for i in range(nx):
            cells = [_ghost(U, i + di, j + dj, bc) for di, dj in ((0, 0), (-1, 0), (1, 0), (0, -1), (0, 1))]
            blk = np.stack(cells, axis=1)  # [v][cell][mode]
            blk[:, :, 0] -= blk[:, 0:1, 0]
            s = np.maximum(np.abs(blk).max(axis=(1, 2)), Mh2)
            blk = blk / s[:, None, None]
            out[j * nx + i] = blk.reshape(-1)
    return out


def init_params(F, seed=0):
    rng = np.random.default_rng(seed)
    return dict(W1=rng.normal(size=(HIDDEN, F)) * np.sqrt(2.0 / F), b1=np.zeros(HIDDEN),
                W2=rng.normal(size=(HIDDEN, HIDDEN)) * np.sqrt(2.0 / HIDDEN), b2=np.zeros(HIDDEN),
                w3=rng.normal(size=HIDDEN) * np.sqrt(1.0 / HIDDEN), b3=np.zeros(1))


def forward(P, X, bf16=True):
    r = bf16_round if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    x = r(X)
    a1 = x @ r(P["W1"]).T + P["b1"]
    h1 = np.maximum(a1, 0.0)
    h1r = r(h1)
    a2 = h1r @ r(P["W2"]).T + P["b2"]
    h2 = np.maximum(a2, 0.0)
    h2r = r(h2)
    z = h2r @ r(P["w3"]) + P["b3"][0]
    p = 1.0 / (1.0 + np.exp(-z))
    return dict(x=x, a1=a1, h1=h1r, a2=a2, h2=h2r, z=z, p=p)


def loss(P, X, y, w, bf16=True):
    c = forward(P, X, bf16)
    z = c["z"]
    # softplus form: -y log p - (1-y) log(1-p) = log(1+e^z) - y z
    l = np.logaddexp(0.0, z) - y * z
    return float(np.mean(w * l)), c


def grads(P, X, y, w, bf16=True):
    """Gradients of the mean weighted BCE through the bf16-rounded forward
    (the rounding is treated as the identity in the backward pass)."""
    r = bf16_round if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    L, c = loss(P, X, y, w, bf16)
    n = X.shape[0]
    dz = w * (c["p"] - y) / n
    g = {}
    g["w3"] = c["h2"].T @ dz
    g["b3"] = np.array([dz.sum()])
    dh2 = np.outer(dz, r(P["w3"])) * (c["a2"] > 0)
    g["W2"] = dh2.T @ c["h1"]
    g["b2"] = dh2.sum(axis=0)
    dh1 = (dh2 @ r(P["W2"])) * (c["a1"] > 0)
    g["W1"] = dh1.T @ c["x"]
    g["b1"] = dh1.sum(axis=0)
    return L, g


def adam(P, G, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    t = state.get("t", 0) + 1
    state["t"] = t
    for k in P:
        m = state.setdefault("m_" + k, np.zeros_like(P[k]))
        v = state.setdefault("v_" + k, np.zeros_like(P[k]))
        m[...] = b1 * m + (1 - b1) * G[k]
        v[...] = b2 * v + (1 - b2) * G[k] ** 2
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        P[k] = P[k] - lr * mh / (np.sqrt(vh) + eps)
    return P


def pack(P):
    """Master-parameter order shared with the library: W1 | W2 | w3 | b1 | b2 | b3."""
    return np.concatenate([P["W1"].ravel(), P["W2"].ravel(), P["w3"], P["b1"], P["b2"], P["b3"]])


def unpack(v, F):
    H = HIDDEN
    o = 0
    P = {}
    for k, shp in (("W1", (H, F)), ("W2", (H, H)), ("w3", (H,)), ("b1", (H,)), ("b2", (H,)), ("b3", (1,))):
        n = int(np.prod(shp))
        P[k] = np.asarray(v[o:o + n], dtype=np.float64).reshape(shp)
        o += n
    return P
