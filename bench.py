"""Benchmark of the RKDG + CSWENO step on one MI355X.

Workload: 2D Euler four-state Riemann problem on [0,1]^2, 2048 x 2048 cells,
Q2 (9 modes x 4 variables per cell, FP64), transmissive sides, TVB (M = 1) +
CSWENO limiting after every SSP-RK3 stage, CFL 0.1, quadrant states from
seed 12345.  A step is one full SSP-RK3 step with limiting; the metric counts
cell-DOF updates per second, DOF = cells * 9 * 4.

Prints one JSON line.  The timed region runs the library's dg_step with its
kernel profiling on (HIP events around every launch on the problem's stream),
so the dominant kernel's average duration comes from the same region.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell-DOF updates/s, 2D Euler P2 (plain vs learned+batched) at equal L1"
HBM_PEAK_GBS = 8000.0
COPY_BYTES = 1 << 30
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_stage23_riemann2d_2048_q2.json")


def traffic_for(bytes_alg):
    """HBM bytes per launch of the stage kernel from the committed rocprofv3
    counter summary, if it was taken on the current kernel source."""
    try:
        t = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    from paper_1904_11147_amd.profiling import kernel_source_hash
    if t.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return t.get("hbm_bytes_per_launch")


def cpu_baseline(n_window=1024, seed=12345, min_seconds=10.0, max_steps=20):
    """The CPU oracle, as it stands, timed on SSP-RK3 steps of a n_window^2
    sub-block of the same problem (cells [512,1536)^2 of the 2048^2 mesh,
    i.e. [0.25,0.75]^2, which holds the quadrant corner), with its own
    projection of the initial data; steps are taken until at least
    min_seconds have passed."""
    from oracle import oracle as O
    from paper_1904_11147_amd import workloads as W
    full = W.riemann2d(n=2048, order=2, seed=seed)
    h = 1.0 / 2048
    lo = 512 * h
    wl = full.with_(nx=n_window, ny=n_window, x0=lo, x1=lo + n_window * h, y0=lo, y1=lo + n_window * h)
    op = O.Problem(dim=2, equation=1, order=2, nx=wl.nx, ny=wl.ny, x0=wl.x0, x1=wl.x1, y0=wl.y0, y1=wl.y1,
                   bc=tuple(wl.bc), cfl=wl.cfl)
    r, _ = op.proj_nodes()
    U = op.limit(op.project(wl.point_values(r)))[0]
    steps = 0
    t0 = time.perf_counter()
    while steps < max_steps and (steps == 0 or time.perf_counter() - t0 < min_seconds):
        U = op.step(U, op.cfl_dt(U))
        steps += 1
    el = time.perf_counter() - t0
    dofs = n_window * n_window * 36
    return {"value": dofs * steps / el, "unit": "cell-DOF updates/s", "cores": O.num_threads(), "kind": "oracle",
            "sample": f"{steps} SSP-RK3 steps (each 3 residuals + 3 TVB/CSWENO passes, CFL dt) of the "
                      f"{n_window}x{n_window} sub-block [0.25,0.75]^2 of the 2048^2 Q2 Euler Riemann problem, "
                      f"seed {seed}; {el:.2f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--seed", type=int, default=12345)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the timed region, run a plain 1 GiB device copy kernel three times "
                         "(the known-size reference for rocprofv3 FETCH_SIZE/WRITE_SIZE)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported by this build "
              "(the multi-GPU design is described in DESIGN.md).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1904_11147_amd import dg, workloads as W

    wl = W.riemann2d(n=args.n, order=2, seed=args.seed)
    prob = dg.problem_from_workload(wl, device="cuda:0")
    state = dg.initial_state(prob, wl, limit=True)
    torch.cuda.synchronize()
    t = 0.0
    if args.warmup:
        t, _ = prob.step(state, t, wl.t_end, max_steps=args.warmup)
    # timed region: kernel events on, the wall clock around it
    prob.profile(True)
    prob.profile_read(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t, steps = prob.step(state, t, wl.t_end, max_steps=args.steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    prof, troubled = prob.profile_read(reset=True)
    prob.profile(False)
    # the same number of steps replayed from the captured graph, for reference
    torch.cuda.synchronize()
    g0 = time.perf_counter()
    t, steps_g = prob.step(state, t, wl.t_end, max_steps=args.steps)
    torch.cuda.synchronize()
    el_graph = time.perf_counter() - g0

    if args.copy_calibration:
        src = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst

    dofs = wl.dofs
    state_bytes = dofs * 8
    value = dofs * steps / el
    ms_stage, n_stage = prof["stage23"]
    avg_ms = ms_stage / max(1, n_stage)
    bytes_launch = 3 * state_bytes  # reads u^(s) and u^n, writes u^(s+1)
    achieved = bytes_launch / (avg_ms * 1e-3) / 1e9
    kinds = {k: {"ms_total": v[0], "launches": v[1], "ms_avg": v[0] / max(1, v[1])} for k, v in prof.items()}
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-DOF updates/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * el / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"riemann2d_{args.n}_q2: 2D Euler four-state Riemann, {args.n}x{args.n} cells, Q2 "
                        f"(36 DOF/cell), seed {args.seed}, transmissive, TVB M=1 + CSWENO, SSP-RK3, CFL 0.1",
            "path": "plain",
            "cells": wl.cells,
            "dofs": dofs,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "k_stage_2d_euler_pair<2, stage 2|3>",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic_for(bytes_launch),
            "algorithmic_bytes_per_launch": bytes_launch,
            "avg_launch_ms": avg_ms,
        },
        "step": {
            "algorithmic_bytes": 64 * dofs,
            "hbm_frac_of_step": 64 * dofs / (el / steps) / 1e9 / HBM_PEAK_GBS,
            "ms_per_step_graph_replay": 1e3 * el_graph / max(1, steps_g),
            "kernels": kinds,
            "troubled_fraction": troubled / max(1, 3 * wl.cells * steps),
            "t_after": t,
        },
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(seed=args.seed)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
