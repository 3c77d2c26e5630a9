"""Train the learned troubled-cell indicator on plain runs and evaluate it.

    python -m paper_1904_11147_amd.train_indicator --seeds 0:200 --out weights.npz
    python -m paper_1904_11147_amd.train_indicator --order 2 --epochs 30 --lr 2e-3 --lr-final 1e-4 \
        --min-change 3e-4 --out indicator_q2.npz --eval-json eval_q2.json   # the committed Q2 network

Data: seeded 64 x 64 four-state Riemann problems (2D Euler, Q1..Q3), see
paper_1904_11147_amd.learned.  Progress is printed per seed block and per
epoch; the evaluation compares plain and learned runs on held-out seeds.
"""
import argparse
import json
import time

import torch

from . import learned


def _range(s):
    a, b = s.split(":")
    return range(int(a), int(b))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--seeds", default="0:200")
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--order", type=int, default=2)
    ap.add_argument("--every", type=int, default=10)
    ap.add_argument("--epochs", type=int, default=6)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--lr-final", type=float, default=None, help="geometric decay to this rate by the last epoch")
    ap.add_argument("--out", default=None, help="default: indicator_q<order>.npz")
    ap.add_argument("--eval-seeds", default="1000:1004")
    ap.add_argument("--eval-n", type=int, default=128)
    ap.add_argument("--eval-json", default=None)
    ap.add_argument("--min-change", type=float, default=0.0,
                    help="label a TVB-flagged cell troubled only above this relative limiter change")
    ap.add_argument("--eval-only", default=None, help="evaluate this saved network (no data, no training)")
    args = ap.parse_args()
    if args.out is None:
        args.out = f"indicator_q{args.order}.npz"
    log = lambda s: print(s, flush=True)
    if args.eval_only:
        net = learned.MLP.load(args.eval_only)
        ev = learned.evaluate(net, list(_range(args.eval_seeds)), n=args.eval_n, order=args.order, log=log)
        for r in ev:
            print(json.dumps(r), flush=True)
        if args.eval_json:
            json.dump({"eval": ev, "args": vars(args)}, open(args.eval_json, "w"), indent=1)
        return

    seeds = list(_range(args.seeds))
    t0 = time.time()
    xs, ys, ws = [], [], []
    block = 20
    for k in range(0, len(seeds), block):
        x, y, w = learned.generate_samples(seeds[k:k + block], n=args.n, order=args.order,
                                           every=args.every, min_change=args.min_change)
        xs.append(x)
        ys.append(y)
        ws.append(w)
        print(f"data: seeds {seeds[k]}..{seeds[min(k + block, len(seeds)) - 1]} -> {x.shape[0]} samples "
              f"({time.time() - t0:.1f} s)", flush=True)
    x, y, w = torch.cat(xs), torch.cat(ys), torch.cat(ws)
    print(f"data: {x.shape[0]} samples, troubled fraction {y.mean().item():.3f}, F={x.shape[1]}; "
          f"runs stopped at a non-physical state: {learned.SKIPPED}", flush=True)
    net = learned.MLP(5 * (args.order + 1) ** 2 * 4, seed=0)
    t1 = time.time()
    hist = learned.train(net, x, y, w, epochs=args.epochs, batch=args.batch, lr=args.lr, lr_final=args.lr_final,
                         log=lambda s: print(s, flush=True))
    train_s = time.time() - t1
    p = net.forward(x)
    acc = ((p > 0.5).float() == y).float().mean().item()
    band = ((p > 0.2) & (p < 0.8)).float().mean().item()
    print(f"train: {args.epochs} epochs in {train_s:.1f} s, accuracy {acc:.4f}, in-band fraction {band:.4f}",
          flush=True)
    net.save(args.out)
    print(f"saved {args.out}", flush=True)
    ev = learned.evaluate(net, list(_range(args.eval_seeds)), n=args.eval_n, order=args.order, log=log)
    for r in ev:
        print(json.dumps(r), flush=True)
    if args.eval_json:
        json.dump({"train_samples": int(x.shape[0]), "nonphysical_runs": learned.SKIPPED, "train_loss": hist, "train_accuracy": acc,
                   "train_in_band": band, "train_seconds": train_s, "eval": ev,
                   "args": vars(args)}, open(args.eval_json, "w"), indent=1)


if __name__ == "__main__":
    main()
