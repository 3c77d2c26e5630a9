"""Learned troubled-cell indicator: parameter buffers, training-data generation
from plain runs, and the training loop.  Every arithmetic step runs in the
library's kernels (features, BF16-MFMA forward/backward, Adam); torch holds the
buffers and selects samples.

Recipe (the workload's; the paper's own indicator is KXRCF):
* data: plain FP64 runs (TVB M = 1 + CSWENO) of seeded 64 x 64 four-state
  Riemann problems (Q2 Euler) to t = 0.25; every `every`-th step, the state
  after one *unlimited* SSP-RK3 step from the current limited state is the
  sample state.  Its features, a label and the change the limiter makes to
  each cell, c = |limited - unlimited|_1 / |unlimited|_1 (sample weight
  1 + c), are recorded for equal numbers of random troubled and untroubled
  cells (at most `cap` of each per sampled state).  The label is the TVB
  flag, or, with min_change > 0, the TVB flag of cells with c > min_change
  (the Q2 network: 3e-4; flagged cells below it are drawn first as
  negatives), so that the network learns to leave out the flagged cells the
  limiter hardly changes;
* training: weighted binary cross-entropy, Adam (lr 1e-3), FP32 master
  weights with BF16 copies;
* inference: p > 0.8 troubled, p < 0.2 untroubled, TVB in between.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import dg
from . import workloads as W

HIDDEN = 64


def layout(features):
    kp = ctypes.c_int32()
    nm = ctypes.c_int64()
    nb = ctypes.c_int64()
    rc = dg.lib().dg_mlp_layout(int(features), ctypes.byref(kp), ctypes.byref(nm), ctypes.byref(nb))
    if rc:
        raise dg.DGError(rc, "dg_mlp_layout")
    return kp.value, nm.value, nb.value


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class MLP:
    """Device buffers of one network with F input features."""

    def __init__(self, features, device="cuda", seed=0, params=None):
        self.F = int(features)
        self.KP, nmaster, nbf16 = layout(self.F)
        self.device = torch.device(device)
        if params is None:
            rng = np.random.default_rng(seed)
            H = HIDDEN
            params = np.concatenate([
                rng.normal(size=H * self.F) * np.sqrt(2.0 / self.F),
                rng.normal(size=H * H) * np.sqrt(2.0 / H),
                rng.normal(size=H) * np.sqrt(1.0 / H),
                np.zeros(2 * H + 1)])
        params = np.asarray(params, dtype=np.float32)
        assert params.size == nmaster
        self.master = torch.from_numpy(params.copy()).to(self.device)
        self.m = torch.zeros_like(self.master)
        self.v = torch.zeros_like(self.master)
        self.grad = torch.zeros_like(self.master)
        self.w = torch.zeros(nbf16, dtype=torch.int16, device=self.device)
        self.loss = torch.zeros(1, dtype=torch.float32, device=self.device)
        self.step_no = 0
        self._dh1 = None
        self.stream = torch.cuda.current_stream(self.device)
        self._adam(0.0, 0)  # bf16 copies from the master weights

    def _adam(self, lr, step):
        rc = dg.lib().dg_mlp_adam(_p(self.master), _p(self.m), _p(self.v), _p(self.grad), _p(self.w), self.F,
                                  ctypes.c_float(lr), int(step), ctypes.c_void_p(self.stream.cuda_stream))
        if rc:
            raise dg.DGError(rc, "dg_mlp_adam")

    def forward(self, x_bf16):
        n = x_bf16.shape[0]
        p = torch.empty(n, dtype=torch.float32, device=self.device)
        rc = dg.lib().dg_mlp_forward(_p(x_bf16), int(n), self.F, _p(self.w), _p(self.master), _p(p),
                                     ctypes.c_void_p(self.stream.cuda_stream))
        if rc:
            raise dg.DGError(rc, "dg_mlp_forward")
        return p

    def gradient(self, x_bf16, y, wgt, accumulate=False):
        """Adds the batch gradient to self.grad; returns the batch loss."""
        n = x_bf16.shape[0]
        if self._dh1 is None or self._dh1.numel() < n * HIDDEN:
            self._dh1 = torch.empty(n * HIDDEN, dtype=torch.int16, device=self.device)
        if not accumulate:
            self.grad.zero_()
        self.loss.zero_()
        rc = dg.lib().dg_mlp_gradient(_p(x_bf16), _p(y), _p(wgt), int(n), self.F, _p(self.w), _p(self.master),
                                      _p(self.grad), _p(self._dh1), _p(self.loss),
                                      ctypes.c_void_p(self.stream.cuda_stream))
        if rc:
            raise dg.DGError(rc, "dg_mlp_gradient")
        return float(self.loss.item())

    def adam_step(self, lr=1e-3):
        self.step_no += 1
        self._adam(lr, self.step_no)

    def params_numpy(self):
        return self.master.detach().cpu().numpy().astype(np.float64)

    def save(self, path):
        np.savez(path, master=self.master.cpu().numpy(), F=self.F)

    @classmethod
    def load(cls, path, device="cuda"):
        z = np.load(path, allow_pickle=False)
        return cls(int(z["F"]), device=device, params=z["master"])


def features(prob, state, bf16=True):
    """Features of every cell of a 2D problem's state (kernel)."""
    F = 5 * prob.nm * prob.nv
    KP, _, _ = layout(F)
    cells = prob.nx * prob.ny
    if bf16:
        out = torch.empty((cells, KP), dtype=torch.int16, device=prob.device)
        rc = dg.lib().dg_mlp_features(prob._h, _p(state), None, _p(out))
    else:
        out = torch.empty((cells, F), dtype=torch.float32, device=prob.device)
        rc = dg.lib().dg_mlp_features(prob._h, _p(state), _p(out), None)
    if rc:
        raise dg.DGError(rc, "dg_mlp_features")
    return out


def attach(prob, net, band=(0.2, 0.8), prob_out=None):
    rc = dg.lib().dg_set_learned(prob._h, _p(net.w), _p(net.master), float(band[0]), float(band[1]),
                                 _p(prob_out))
    if rc:
        raise dg.DGError(rc, "dg_set_learned")


SKIPPED = []  # (seed, time) of runs that met a non-physical state


def generate_samples(seeds, n=64, order=2, t_end=0.25, every=10, device="cuda", max_steps=100000, gen_seed=0,
                     cap=256, min_change=0.0):
    """Training samples from plain runs (see the module docstring).  A run
    that meets a non-physical state (no positivity limiter is applied) stops
    there; its earlier samples are kept and the seed is recorded in SKIPPED.
    min_change > 0: a TVB-flagged cell is labelled troubled only where the
    limiter changes it by more than min_change (relative, the weight's ratio);
    the flagged cells below it are the first negatives drawn.
    Returns (x bf16 [S][KP], y float [S], w float [S])."""
    g = torch.Generator(device="cpu").manual_seed(gen_seed)
    xs, ys, ws = [], [], []
    for seed in seeds:
        wl = W.riemann2d(n=n, order=order, seed=seed, t_end=t_end)
        plain = dg.problem_from_workload(wl, device=device)
        free = dg.problem_from_workload(wl, device=device, limiter=dg.LIM_NONE)
        state = dg.initial_state(plain, wl, limit=True)
        u = torch.empty_like(state)  # fixed buffers: the captured step graphs stay valid
        lim = torch.empty_like(state)
        t, k = 0.0, 0
        while t < t_end and k < max_steps:
            u.copy_(state)
            dt = plain.cfl_dt(u)
            free.step(u, 0.0, 1.0, dt=dt, max_steps=1, allow_nonphysical=True)
            lim.copy_(u)
            flags, _, _ = plain.limit(lim, want_margin=False)
            x = features(plain, u, bf16=True)
            flagged = flags.reshape(-1) != 0
            num = (lim - u).abs().sum(dim=(0, 1)).reshape(-1)
            den = u.abs().sum(dim=(0, 1)).reshape(-1).clamp_min(1e-300)
            chg = num / den
            wgt = (1.0 + chg).to(torch.float32)
            pos = flagged & (chg > min_change) if min_change > 0 else flagged
            f = pos.to(torch.float32)
            # finite samples only (bf16 exponent all ones = inf/nan)
            ok = ((x & 0x7F80) != 0x7F80).all(dim=1) & torch.isfinite(wgt)
            tr = torch.nonzero(pos & ok).reshape(-1)
            hard = torch.nonzero(flagged & ~pos & ok).reshape(-1)  # flagged, small change
            easy = torch.nonzero(~flagged & ok).reshape(-1)
            m = min(tr.numel(), hard.numel() + easy.numel(), cap)
            if m > 0:
                pt = torch.randperm(tr.numel(), generator=g)[:m].to(tr.device)
                mh = min(hard.numel(), m)
                parts = [tr[pt]]
                if mh > 0:
                    parts.append(hard[torch.randperm(hard.numel(), generator=g)[:mh].to(tr.device)])
                parts.append(easy[torch.randperm(easy.numel(), generator=g)[:m - mh].to(tr.device)])
                idx = torch.cat(parts)
                xs.append(x[idx])
                ys.append(f[idx])
                ws.append(wgt[idx])
            try:
                t, steps = plain.step(state, t, t_end, max_steps=every)
            except dg.DGError as e:
                if e.code != dg.DG_ERR_NONPHYSICAL:
                    raise
                SKIPPED.append((seed, t))
                break
            k += steps
        plain.close()
        free.close()
    return torch.cat(xs), torch.cat(ys), torch.cat(ws)


def train(net, x, y, w, epochs=3, batch=4096, lr=1e-3, seed=0, log=None, lr_final=None):
    """Mini-batch Adam over shuffled samples; the learning rate goes
    geometrically from lr to lr_final (default: constant) over the epochs.
    Returns the per-epoch mean loss."""
    gen = torch.Generator(device="cpu").manual_seed(seed)
    n = x.shape[0]
    hist = []
    lr0 = lr
    for ep in range(epochs):
        if lr_final is not None and epochs > 1:
            lr = lr0 * (lr_final / lr0) ** (ep / (epochs - 1))
        perm = torch.randperm(n, generator=gen).to(x.device)
        tot, cnt = 0.0, 0
        for s in range(0, n, batch):
            idx = perm[s:s + batch]
            loss = net.gradient(x[idx].contiguous(), y[idx].contiguous(), w[idx].contiguous())
            net.adam_step(lr)
            tot += loss * idx.numel()
            cnt += idx.numel()
        hist.append(tot / max(1, cnt))
        if log:
            log(f"epoch {ep}: loss {hist[-1]:.5f}")
    return hist


def _density_means(state, dim=2):
    return (state[0, 0] / 2.0).double()


def _average_down(fine_means, factor):
    ny, nx = fine_means.shape
    return fine_means.reshape(ny // factor, factor, nx // factor, factor).mean(dim=(1, 3))


def evaluate(net, seeds, n=128, order=2, t_end=0.25, band=(0.2, 0.8), device="cuda", probe_every=50, log=None):
    """Plain (TVB) vs learned runs of held-out problems: steps, troubled
    fraction, flag disagreement with TVB on the plain trajectory, and the L1
    error of the density means against the plain solution on the 2x-refined
    mesh averaged down.  Returns a list of per-seed dicts; log(text), if
    given, receives a line per finished run."""
    out = []
    say = log if log is not None else (lambda text: None)
    for seed in seeds:
        wl = W.riemann2d(n=n, order=order, seed=seed, t_end=t_end)
        res = {"seed": seed, "n": n}
        finals = {}
        for kind in ("plain", "learned"):
            kw = {} if kind == "plain" else {"indicator": dg.IND_LEARNED}
            prob = dg.problem_from_workload(wl, device=device, **kw)
            if kind == "learned":
                attach(prob, net, band)
            state = dg.initial_state(prob, wl, limit=True)
            prob.profile_read(reset=True)
            torch.cuda.synchronize()
            t, steps = prob.step(state, 0.0, t_end, allow_nonphysical=True)
            res[kind + "_nonphysical"] = prob.status() != 0
            _, troubled = prob.profile_read(reset=True)
            res[kind + "_steps"] = steps
            res[kind + "_troubled_fraction"] = troubled / max(1, 3 * wl.cells * steps)
            finals[kind] = _density_means(state)
            prob.close()
            say(f"eval seed {seed}: {kind} run, {steps} steps")
        # disagreement of the two indicators along the plain trajectory
        plain = dg.problem_from_workload(wl, device=device)
        learn = dg.problem_from_workload(wl, device=device, indicator=dg.IND_LEARNED)
        attach(learn, net, band)
        state = dg.initial_state(plain, wl, limit=True)
        t, dis, tot = 0.0, 0, 0
        while t < t_end:
            a = state.clone()
            b = state.clone()
            fa, _, _ = plain.limit(a, want_margin=False)
            fb, _, _ = learn.limit(b, want_margin=False)
            dis += int((fa != fb).sum().item())
            tot += fa.numel()
            t, k = plain.step(state, t, t_end, max_steps=probe_every, allow_nonphysical=True)
            if k == 0 or plain.status() != 0:  # a non-physical state stops the run
                break
        res["flag_disagreement"] = dis / max(1, tot)
        plain.close()
        learn.close()
        say(f"eval seed {seed}: flag disagreement {res['flag_disagreement']:.3f}")
        # reference: plain on the 2x-refined mesh, averaged down
        wf = W.riemann2d(n=2 * n, order=order, seed=seed, t_end=t_end)
        ref = dg.problem_from_workload(wf, device=device)
        rs = dg.initial_state(ref, wf, limit=True)
        ref.step(rs, 0.0, t_end, allow_nonphysical=True)
        res["reference_nonphysical"] = ref.status() != 0
        rmean = _average_down(_density_means(rs), 2)
        ref.close()
        for kind in ("plain", "learned"):
            res[kind + "_L1"] = float((finals[kind] - rmean).abs().mean().item())
        res["L1_learned_vs_plain"] = float((finals["learned"] - finals["plain"]).abs().mean().item())
        out.append(res)
    return out
