"""GPU checks of the learned indicator through the C-ABI against the FP64
reference (oracle/mlp_oracle.py): features, BF16-MFMA forward and gradients
(on the same bf16-rounded inputs), Adam, a training run, and the indicator's
decision rule inside dg_limit."""
import numpy as np
import pytest
import torch

from oracle import mlp_oracle as M
from tests.gpu_common import configs, make_pair, rough_state

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods(oracle):
    from paper_1904_11147_amd import dg, learned
    dg.lib()
    return oracle, dg, learned


def _to_bf16_tensor(X):
    """float64 -> bf16 bit patterns (int16 tensor) after the oracle's rounding."""
    r = M.bf16_round(X).astype(np.float32)
    bits = (r.view(np.uint32) >> 16).astype(np.uint16)
    return torch.from_numpy(bits.view(np.int16).copy()).cuda()


@pytest.mark.parametrize("order", [1, 2, 3])
def test_features_match_reference(mods, order):
    O, D, Lm = mods
    cfg = configs(2, 1, order, 70, 9, (1, 1, 0, 0))
    op, gp = make_pair(O, D, cfg)
    U = rough_state(O, op, seed=3)
    ref = M.features(U, op.hx, 1.0, op.bc)
    got = Lm.features(gp, torch.from_numpy(U).cuda(), bf16=False).cpu().numpy()
    np.testing.assert_allclose(got, ref, rtol=0, atol=2e-7)
    gb = Lm.features(gp, torch.from_numpy(U).cuda(), bf16=True).cpu().numpy()
    KP = gb.shape[1]
    assert KP % 16 == 0 and (gb[:, ref.shape[1]:] == 0).all()
    f = (gb.astype(np.uint16).astype(np.uint32) << 16).view(np.float32)[:, : ref.shape[1]]
    np.testing.assert_array_equal(f, M.bf16_round(got).astype(np.float32))


@pytest.mark.parametrize("F", [80, 180, 320])
def test_forward_and_gradient_match_reference(mods, F):
    O, D, Lm = mods
    rng = np.random.default_rng(F)
    n = 1000  # several tiles and a ragged tail
    P = M.init_params(F, seed=2)
    for k in ("b1", "b2", "b3"):
        P[k] = rng.normal(size=P[k].shape) * 0.1
    net = Lm.MLP(F, params=M.pack(P))
    X = rng.normal(size=(n, F))
    KP = net.KP
    Xp = np.zeros((n, KP))
    Xp[:, :F] = X
    xb = _to_bf16_tensor(Xp)
    y = (rng.random(n) > 0.5).astype(np.float64)
    w = 1.0 + rng.random(n)
    Pb = M.unpack(M.pack(P).astype(np.float32), F)  # the fp32 master values the GPU holds
    ref = M.forward(Pb, X)
    p = net.forward(xb).cpu().numpy()
    np.testing.assert_allclose(p, ref["p"], rtol=1e-2, atol=1e-3)
    L, G = M.grads(Pb, X, y, w)
    loss = net.gradient(xb, torch.from_numpy(y.astype(np.float32)).cuda(), torch.from_numpy(w.astype(np.float32)).cuda())
    assert abs(loss - L) <= 1e-2 * abs(L)
    g = net.grad.cpu().numpy().astype(np.float64)
    gref = M.pack(G)
    cos = g @ gref / (np.linalg.norm(g) * np.linalg.norm(gref))
    assert cos >= 0.999, cos
    got = M.unpack(g, F)
    for k in G:
        scale = np.abs(G[k]).max()
        assert np.abs(got[k] - G[k]).max() <= 5e-2 * scale, k


def test_adam_matches_reference(mods):
    O, D, Lm = mods
    F = 180
    P = M.init_params(F, seed=5)
    net = Lm.MLP(F, params=M.pack(P))
    rng = np.random.default_rng(9)
    gvec = rng.normal(size=net.master.numel()).astype(np.float32)
    st = {}
    Pr = M.unpack(M.pack(P).astype(np.float32), F)
    for step in range(3):
        net.grad.copy_(torch.from_numpy(gvec))
        net.adam_step(1e-3)
        Pr = M.adam(Pr, M.unpack(gvec.astype(np.float64), F), st, lr=1e-3)
    np.testing.assert_allclose(net.params_numpy(), M.pack(Pr), rtol=0, atol=2e-6)
    assert net.grad.abs().max().item() == 0.0


def test_training_reduces_loss(mods):
    O, D, Lm = mods
    F = 80
    rng = np.random.default_rng(1)
    n = 8192
    X = rng.normal(size=(n, F))
    y = (X[:, 0] + 0.5 * X[:, 3] > 0).astype(np.float32)
    Xp = np.zeros((n, 80))
    Xp[:, :F] = X
    xb = _to_bf16_tensor(Xp)
    net = Lm.MLP(F, seed=0)
    yy = torch.from_numpy(y).cuda()
    ww = torch.ones(n, device="cuda")
    hist = Lm.train(net, xb, yy, ww, epochs=8, batch=1024, lr=3e-3)
    assert hist[-1] < 0.5 * hist[0], hist
    acc = ((net.forward(xb).cpu().numpy() > 0.5) == (y > 0.5)).mean()
    assert acc > 0.95, acc


def test_learned_indicator_decision_rule(mods):
    """p > band_hi flags every cell, p < band_lo none, p inside the band
    defers to TVB (a network with zero weights has p = sigmoid(b3))."""
    O, D, Lm = mods
    cfg = configs(2, 1, 2, 70, 9, (1, 1, 1, 1))
    op, _ = make_pair(O, D, cfg)
    U = rough_state(O, op, seed=21)
    _, rflags, _ = op.limit(U)
    F = 180
    for b3, want in ((8.0, "all"), (-8.0, "none"), (0.0, "tvb")):
        P = M.init_params(F)
        for k in P:
            P[k] = np.zeros_like(P[k])
        P["b3"][:] = b3
        net = Lm.MLP(F, params=M.pack(P))
        kw = dict(cfg)
        kw["indicator"] = D.IND_LEARNED
        gp = D.Problem(**kw)
        probs = torch.empty(70 * 9, device="cuda")
        Lm.attach(gp, net, (0.2, 0.8), probs)
        Ud = torch.from_numpy(U.copy()).cuda()
        flags, _, n = gp.limit(Ud)
        f = flags.cpu().numpy()
        assert np.allclose(probs.cpu().numpy(), 1 / (1 + np.exp(-b3)), atol=1e-6)
        if want == "all":
            assert f.all() and n == f.size
        elif want == "none":
            assert not f.any() and n == 0
        else:
            assert (f == rflags).all()
