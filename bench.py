"""Benchmark of the RKDG + CSWENO step on one MI355X.

Workload: 2D Euler four-state Riemann problem on [0,1]^2, 2048 x 2048 cells,
Q2 (9 modes x 4 variables per cell, FP64), transmissive sides, TVB (M = 1) +
CSWENO limiting after every SSP-RK3 stage, CFL 0.1, quadrant states from
seed 12345.  A step is one full SSP-RK3 step with limiting; the metric counts
cell-DOF updates per second, DOF = cells * 9 * 4.

Prints one JSON line.  `value` and `ms_per_step` come from K steps of
dg_step replaying its captured step graph (the production mode); the same
number of steps is run once more with the library's kernel profiling on (HIP
events around every launch on the problem's stream), which gives the
per-kernel times and the dominant kernel's average duration for `roofline`.
Further legs: a late-time window of the same run (t = 0.05), the learned
indicator, KXRCF and characteristic limiting on the same state, 2D Burgers
Q2 at 1024^2, the 1D Euler shock/entropy-wave problem (P3, 4000 cells) to
t = 1.8, the double Mach reflection, the 256-instance batch (sequential vs
batched, plain vs learned, Q2-only and all-order counts), a measured copy
bandwidth next to the vendor peak, and the CPU oracle (all host threads and
one thread) with the host's CPU model.
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
FP64_PEAK_TFLOPS = 78.6
COPY_BYTES = 1 << 30
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_stage23_riemann2d_2048_q2.json")
FP64_FILE = os.path.join(ROOT, "profiles", "fp64_stage23_riemann2d_2048_q2.json")


def fp64_per_launch():
    """FP64 flops per launch of the stage kernel (stages 2/3) from the committed
    rocprofv3 FP64 instruction counters, if taken on the current kernel source."""
    try:
        t = json.load(open(FP64_FILE))
    except (OSError, ValueError):
        return None
    from paper_1904_11147_amd.profiling import kernel_source_hash
    if t.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return t.get("fp64_flops_per_launch")


def copy_peak_gbs(nbytes=COPY_BYTES, reps=5):
    """Measured device copy bandwidth: torch's copy of nbytes (read once,
    written once) on torch's current stream, timed with events on that
    stream; the best of reps."""
    import torch
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = None
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    del src, dst
    return 2.0 * nbytes / (best * 1e-3) / 1e9


def host_info():
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "host_cpus_usable": usable, "host_cpus_total": os.cpu_count()}


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


def cpu_single_thread(seed=12345, n_window=256, min_seconds=6.0):
    """The oracle on one host thread (a child process with OMP_NUM_THREADS=1)
    on the 256^2 sub-block around the quadrant corner of the same problem."""
    import subprocess
    code = ("import json,sys; sys.path.insert(0, %r); import bench; "
            "print(json.dumps(bench.cpu_baseline(n_window=%d, seed=%d, min_seconds=%g, max_steps=50)))"
            % (ROOT, n_window, seed, min_seconds))
    env = dict(os.environ, OMP_NUM_THREADS="1")
    try:
        out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=300)
        return json.loads(out.stdout.strip().splitlines()[-1])
    except Exception as e:  # reported, not fatal
        return {"error": str(e)}


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
    lo = (1024 - n_window // 2) * h
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
                      f"{n_window}x{n_window} sub-block around the quadrant corner ([{lo:.4f},{lo + n_window * h:.4f}]^2)"
                      f" of the 2048^2 Q2 Euler Riemann problem, seed {seed}; {el:.2f} s"}


def learned_nets(device):
    """The committed trained indicators, by order (missing files are skipped)."""
    from paper_1904_11147_amd import learned
    nets = {}
    for o in (1, 2, 3):
        path = os.path.join(ROOT, "paper_1904_11147_amd", "weights", f"indicator_q{o}.npz")
        if os.path.exists(path):
            nets[o] = learned.MLP.load(path, device=device)
    return nets


def indicator_leg(wl, state0, t0, steps, warmup, indicator=0, net=None, limiter=1):
    """The same problem and state with another troubled-cell indicator (the
    learned one with its network, or KXRCF) or limiter (characteristic)."""
    import torch
    from paper_1904_11147_amd import dg, learned
    prob = dg.problem_from_workload(wl, device="cuda:0", indicator=indicator, limiter=limiter)
    if net is not None:
        learned.attach(prob, net)
    state = state0.clone()
    t, _ = prob.step(state, t0, wl.t_end, max_steps=warmup)
    prob.profile_read(reset=True)
    torch.cuda.synchronize()
    a = time.perf_counter()
    t, n = prob.step(state, t, wl.t_end, max_steps=steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - a
    _, troubled = prob.profile_read(reset=True)
    # the next steps once more with kernel events, for the per-kind times
    prob.profile(True)
    t, n2 = prob.step(state, t, wl.t_end, max_steps=steps)
    prof, _ = prob.profile_read(reset=True)
    prob.profile(False)
    prob.close()
    return {"value": wl.dofs * n / el, "ms_per_step": 1e3 * el / n, "steps": n,
            "troubled_fraction": troubled / max(1, 3 * wl.cells * n),
            "kernels_ms_per_step": {k: v[0] / max(1, n2) for k, v in prof.items()}}


def full_run_leg(wl, indicator=0, net=None, chunk=2000):
    """The whole run of the 2D Euler problem: from the projected and limited
    initial state to t_end by dg_step (captured step graph), wall time over
    every step (tile height autotuned first, untimed); troubled fraction over
    all limiter passes; progress on stderr after every `chunk` steps."""
    import torch
    from paper_1904_11147_amd import dg, learned
    prob = dg.problem_from_workload(wl, device="cuda:0", indicator=indicator)
    if net is not None:
        learned.attach(prob, net)
    state = dg.initial_state(prob, wl, limit=True)
    prob.autotune(state)
    torch.cuda.synchronize()
    t, total, troubled, status = 0.0, 0, 0, "ok"
    prob.profile_read(reset=True)
    a = time.perf_counter()
    while t < wl.t_end:
        try:
            t, n = prob.step(state, t, wl.t_end, max_steps=chunk)
        except dg.DGError as e:
            status = str(e)
            break
        total += n
        troubled += prob.profile_read(reset=True)[1]
        print(f"full run ({'learned' if net is not None else 'plain'}): t = {t:.5f} after {total} steps, "
              f"{time.perf_counter() - a:.1f} s", file=sys.stderr, flush=True)
        if n == 0:
            break
    torch.cuda.synchronize()
    el = time.perf_counter() - a
    prob.close()
    return {"t_end": wl.t_end, "t_reached": t, "steps": total, "seconds": el, "status": status,
            "ms_per_step": 1e3 * el / max(1, total), "value": wl.dofs * total / el, "unit": "cell-DOF updates/s",
            "troubled_fraction": troubled / max(1, 3 * wl.cells * total)}


def timed_steps(prob, state, t, t_end, steps, profile):
    """steps of dg_step from t; with profile: kernel events on.  Returns
    (t, steps taken, seconds, per-kind kernel times, troubled cells)."""
    import torch
    if profile:
        prob.profile(True)
    prob.profile_read(reset=True)
    torch.cuda.synchronize()
    a = time.perf_counter()
    t, n = prob.step(state, t, t_end, max_steps=steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - a
    prof, troubled = prob.profile_read(reset=True)
    if profile:
        prob.profile(False)
    return t, n, el, prof, troubled


def late_window_leg(prob, wl, state, t, t_late, steps, net=None):
    """The same C4 run advanced (untimed) to t_late, then `steps` steps timed
    by graph replay and once more with kernel events: the late-time cost,
    when the waves have spread and more cells are troubled; and the same
    steps from the same late state with the learned indicator."""
    import torch
    from paper_1904_11147_amd import dg
    torch.cuda.synchronize()
    a = time.perf_counter()
    n_adv = 0
    while t < t_late:  # in chunks, with progress on stderr
        t, n = prob.step(state, t, t_late, max_steps=2000)
        n_adv += n
        print(f"late window: advanced to t = {t:.5f} ({n_adv} steps, {time.perf_counter() - a:.1f} s)",
              file=sys.stderr, flush=True)
        if n == 0:
            break
    torch.cuda.synchronize()
    adv_s = time.perf_counter() - a
    late = state.clone()
    t1, n, el, _, troubled = timed_steps(prob, state, t, wl.t_end, steps, profile=False)
    t2, n2, el2, prof, troubled2 = timed_steps(prob, state, t1, wl.t_end, steps, profile=True)
    out = {"t_start": t, "advance_steps": n_adv, "advance_seconds": adv_s, "steps": n,
           "value": wl.dofs * n / el, "ms_per_step": 1e3 * el / n,
           "troubled_fraction": troubled2 / max(1, 3 * wl.cells * n2),
           "kernels_ms_per_step": {k: v[0] / max(1, n2) for k, v in prof.items()}}
    if net is not None:
        out["learned"] = indicator_leg(wl, late, t, steps, 2, dg.IND_LEARNED, net=net)
    del late
    return out


def burgers2d_leg(steps, warmup, n=1024):
    """2D Burgers Q2 on [0,4]^2, 1024^2 cells, periodic (the scalar 2D
    workload): throughput and its HBM floor of 64 B per DOF per step."""
    import torch
    from paper_1904_11147_amd import dg, workloads as W
    wl = W.burgers2d(n=n, order=2)
    prob = dg.problem_from_workload(wl, device="cuda:0")
    state = dg.initial_state(prob, wl, limit=True)
    rows, _ = prob.autotune(state)
    t, _ = prob.step(state, 0.0, wl.t_end, max_steps=warmup)
    t, k, el, _, _ = timed_steps(prob, state, t, wl.t_end, steps, profile=False)
    t, k2, el2, prof, troubled = timed_steps(prob, state, t, wl.t_end, steps, profile=True)
    prob.close()
    floor = 64.0 * wl.dofs
    ms23 = prof["stage23"][0] / max(1, prof["stage23"][1])
    return {"workload": f"{wl.name}: 2D Burgers, u0 = 0.5 + sin(pi (x+y)/2) on [0,4]^2, {n}x{n} cells, Q2, periodic, "
                        "TVB M=1 + CSWENO, CFL 0.1",
            "value": wl.dofs * k / el, "unit": "cell-DOF updates/s", "ms_per_step": 1e3 * el / k, "steps": k,
            "step_algorithmic_bytes": floor, "hbm_frac_of_step": floor / (el / k) / 1e9 / HBM_PEAK_GBS,
            "stage23_ms": ms23, "stage23_frac": 3 * 8 * wl.dofs / (ms23 * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "troubled_fraction": troubled / max(1, 3 * wl.cells * k2), "autotuned_rows": rows,
            "kernels_ms_per_step": {kk: v[0] / max(1, k2) for kk, v in prof.items()}}


def shu_osher_leg():
    """1D Euler shock/entropy-wave interaction (Example 9 in its standard
    scaling), 4000 cells, P3, to t = 1.8.  With the workload's componentwise
    limiter at CFL 0.05 the P3 solution loses positivity in step 22
    (t = 6.0e-4; the oracle does the same, componentwise and characteristic
    alike).  With the positivity-preserving scaling it gets to t = 0.24
    (componentwise) and 0.26 (characteristic), where a cell mean itself turns
    non-physical (the scaling keeps means admissible only under a CFL bound on
    point speeds); at CFL 0.01 with the scaling the componentwise run reaches
    t = 1.8, which is the run whose throughput is reported."""
    import torch
    from paper_1904_11147_amd import dg, workloads as W
    wl = W.shu_osher()
    out = {"workload": f"{wl.name}: 1D Euler, {wl.nx} cells, P3, t = {wl.t_end}, transmissive, TVB M=1 + CSWENO"}
    for name, lim, pos, cfl in (("componentwise_cfl0.05", dg.LIM_CSWENO, 0, 0.05),
                                ("componentwise_positivity_cfl0.05", dg.LIM_CSWENO, 1, 0.05),
                                ("characteristic_positivity_cfl0.05", dg.LIM_CSWENO_CHAR, 1, 0.05),
                                ("componentwise_positivity_cfl0.01", dg.LIM_CSWENO, 1, 0.01)):
        wl = wl.with_(cfl=cfl)
        prob = dg.problem_from_workload(wl, device="cuda:0", limiter=lim, positivity=pos)
        state = dg.initial_state(prob, wl, limit=True)
        prob.status()
        torch.cuda.synchronize()
        a = time.perf_counter()
        t, k = prob.step(state, 0.0, wl.t_end, allow_nonphysical=True)
        torch.cuda.synchronize()
        el = time.perf_counter() - a
        ok = prob.status() == 0
        out[name] = {"t_reached": t, "steps": k, "seconds": el, "status": "ok" if ok else "non-physical",
                     "value": wl.dofs * k / el, "ms_per_step": 1e3 * el / max(1, k)}
        prob.close()
    return out


def double_mach_leg(steps, warmup, n=1920, order=2, to_end=False):
    """The paper's Example 11 on its finest mesh: double Mach reflection,
    n x n/4 cells, walls, inflow and the moving shock on the north side,
    positivity scaling after every limiter pass.  Optionally the whole run to
    t = 0.2 as well."""
    import torch
    from paper_1904_11147_amd import dg, workloads as W
    wl = W.double_mach(n, order=order)
    prob = dg.problem_from_workload(wl, device="cuda:0")
    state = dg.initial_state(prob, wl, limit=True)
    rows, _ = prob.autotune(state)
    t, _ = prob.step(state, 0.0, wl.t_end, max_steps=warmup)
    prob.profile(True)
    prob.profile_read(reset=True)
    torch.cuda.synchronize()
    a = time.perf_counter()
    t, k = prob.step(state, t, wl.t_end, max_steps=steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - a
    prof, troubled = prob.profile_read(reset=True)
    prob.profile(False)
    res = {"workload": f"{wl.name}: 2D Euler, Mach 10 shock at 60 degrees on [0,4]x[0,1], {wl.nx}x{wl.ny} cells, "
                       f"Q{order}, TVB M=1 + CSWENO + positivity scaling, CFL {wl.cfl}",
           "value": wl.dofs * k / el, "unit": "cell-DOF updates/s", "ms_per_step": 1e3 * el / k, "steps": k,
           "troubled_fraction": troubled / max(1, 3 * wl.cells * k), "autotuned_rows": rows,
           "kernels_ms_per_step": {kk: v[0] / k for kk, v in prof.items()}}
    if to_end:
        torch.cuda.synchronize()
        a = time.perf_counter()
        try:
            t, k2 = prob.step(state, t, wl.t_end)
            status = "ok"
        except dg.DGError as e:
            k2, status = 0, str(e)
        torch.cuda.synchronize()
        res["to_t_end"] = {"t": t, "steps_total": warmup + k + k2, "seconds_rest": time.perf_counter() - a,
                           "status": status}
    prob.close()
    return res


def batched_leg(steps, warmup, count=256, nets=None, positivity=0):
    """256 mixed four-state Riemann problems (side uniform in [64,512], order
    uniform in {1,2,3}, one seed each): every instance advanced alone through
    dg_step, then all together through dg_batch_step (autotuned tiles), plain
    TVB and with the learned indicators.  Each instance takes the same number
    of steps in every variant; cell-DOF updates / wall time of the stepping.
    Instances that reach a non-physical state within those steps are listed
    and left out of all variants.  positivity=1: the same with the
    positivity-preserving scaling on in every run (no learned variant)."""
    import numpy as np
    import torch
    from paper_1904_11147_amd import dg, workloads as W
    wls_all = W.riemann2d_batch(count=count)
    # each instance alone
    el_seq, keep, excluded = 0.0, [], []
    for wl in wls_all:
        p = dg.problem_from_workload(wl, device="cuda:0", positivity=positivity)
        st = dg.initial_state(p, wl, limit=True)
        t, _ = p.step(st, 0.0, wl.t_end, max_steps=warmup, allow_nonphysical=True)
        bad = p.status() != 0
        if not bad:
            torch.cuda.synchronize()
            a = time.perf_counter()
            p.step(st, t, wl.t_end, max_steps=steps, allow_nonphysical=True)
            torch.cuda.synchronize()
            el = time.perf_counter() - a
            bad = p.status() != 0
        if bad:
            excluded.append({"seed": wl.seed, "n": wl.nx, "order": wl.order})
        else:
            el_seq += el
            keep.append(wl)
        p.close()
        del st
    wls = keep
    dofs = np.array([wl.dofs for wl in wls], dtype=np.float64)
    t_end = np.array([wl.t_end for wl in wls])
    q2 = np.array([wl.order == 2 for wl in wls])
    res = {"workload": f"riemann2d_batch{count}: {count} 2D Euler four-state Riemann problems, side uniform in "
                       "[64,512], order uniform in {1,2,3} (CFL 0.1, Q3 0.05), seeds 10000+, transmissive, "
                       "TVB M=1 + CSWENO" + (" + positivity scaling" if positivity else ""),
           "instances": len(wls), "excluded_nonphysical": excluded, "dofs": int(dofs.sum()),
           "orders": {o: int(sum(w.order == o for w in wls)) for o in (1, 2, 3)}, "steps_each": steps,
           "sequential": {"value": dofs.sum() * steps / el_seq, "value_q2_only": dofs[q2].sum() * steps / el_seq,
                          "ms_per_step": 1e3 * el_seq / steps}}
    b = dg.batch_from_workloads(wls, device="cuda:0", positivity=positivity)
    init = b.states.clone()

    def run(batch):
        t, _, _, _ = batch.step(0.0, t_end, max_steps=warmup)
        torch.cuda.synchronize()
        a = time.perf_counter()
        t, n, status, troubled = batch.step(t, t_end, max_steps=steps, allow_nonphysical=True)
        torch.cuda.synchronize()
        el = time.perf_counter() - a
        cells = float(sum(wl.cells * k for wl, k in zip(wls, n)))
        return {"value": float((dofs * n).sum() / el), "value_q2_only": float((dofs * n)[q2].sum() / el),
                "ms_per_step": 1e3 * el / steps,
                "troubled_fraction": troubled / max(1.0, 3.0 * cells), "nonphysical": int((status != 0).sum())}

    res["autotune"] = {str(o): {"rows": r, "tiles": n, "stage_ms": ms} for o, (r, n, ms) in b.autotune().items()}
    res["batched"] = run(b)
    b.close()
    del b
    if nets and not positivity and all(o in nets for o in (1, 2, 3)):
        cfgs = [dict(dim=2, equation=wl.equation, order=wl.order, nx=wl.nx, ny=wl.ny, x0=wl.x0, x1=wl.x1, y0=wl.y0,
                     y1=wl.y1, bc=tuple(wl.bc), gamma=wl.gamma, cfl=wl.cfl, indicator=dg.IND_LEARNED) for wl in wls]
        bl = dg.Batch(cfgs, device="cuda:0")
        bl.states.copy_(init)
        for o in (1, 2, 3):
            bl.set_learned(o, nets[o].w, nets[o].master)
        bl.autotune()
        res["batched_learned"] = run(bl)
        bl.close()
    res["speedup_batched_vs_sequential"] = res["batched"]["value"] / res["sequential"]["value"]
    if "batched_learned" in res:
        res["speedup_batched_learned_vs_sequential"] = res["batched_learned"]["value"] / res["sequential"]["value"]
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--seed", type=int, default=12345)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the 256-instance batched comparison")
    ap.add_argument("--batched-steps", type=int, default=10)
    ap.add_argument("--no-double-mach", action="store_true", help="skip the double Mach reflection leg")
    ap.add_argument("--double-mach-only", action="store_true",
                    help="run only the double Mach reflection leg and print its record (for profiling)")
    ap.add_argument("--double-mach-to-end", action="store_true",
                    help="also run the double Mach reflection to t = 0.2 (about a minute)")
    ap.add_argument("--full-run", action="store_true",
                    help="only run the 2D Euler problem to t_end, plain and with the learned indicator, and print "
                         "their records (a few minutes)")
    ap.add_argument("--no-late", action="store_true", help="skip the late-time window of the 2D Euler run")
    ap.add_argument("--late-t", type=float, default=0.05, help="time at which the late window starts")
    ap.add_argument("--no-burgers2d", action="store_true", help="skip the 2D Burgers 1024^2 leg")
    ap.add_argument("--no-shu-osher", action="store_true", help="skip the 1D Euler Shu-Osher leg to t = 1.8")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the timed region, run a plain 1 GiB device copy kernel three times "
                         "(the known-size reference for rocprofv3 FETCH_SIZE/WRITE_SIZE)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the library has no multi-GPU path).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1904_11147_amd import dg, workloads as W

    if args.double_mach_only:
        print(json.dumps({"double_mach": double_mach_leg(args.steps, args.warmup, to_end=args.double_mach_to_end)}),
              flush=True)
        return
    wl = W.riemann2d(n=args.n, order=2, seed=args.seed)
    if args.full_run:
        nets = learned_nets("cuda:0")
        res = {"workload": f"{wl.name}: 2D Euler four-state Riemann problem, {wl.nx}x{wl.ny} cells, Q2, "
                           f"TVB M=1 + CSWENO, CFL {wl.cfl}, to t = {wl.t_end}",
               "plain": full_run_leg(wl)}
        if 2 in nets:
            res["learned"] = full_run_leg(wl, dg.IND_LEARNED, nets[2])
        print(json.dumps({"full_run": res}), flush=True)
        return
    prob = dg.problem_from_workload(wl, device="cuda:0")
    state = dg.initial_state(prob, wl, limit=True)
    tuned_rows, tuned_ms = prob.autotune(state)
    torch.cuda.synchronize()
    t = 0.0
    if args.warmup:
        t, _ = prob.step(state, t, wl.t_end, max_steps=args.warmup)
    state_warm, t_warm = state.clone(), t
    # timed region: K steps replaying the captured step graph
    t, steps, el, _, troubled = timed_steps(prob, state, t, wl.t_end, args.steps, profile=False)
    # the same number of steps with kernel events on the problem's stream
    t, steps_p, el_p, prof, troubled_p = timed_steps(prob, state, t, wl.t_end, args.steps, profile=True)

    dofs = wl.dofs
    state_bytes = dofs * 8
    value = dofs * steps / el
    ms_stage, n_stage = prof["stage23"]
    avg_ms = ms_stage / max(1, n_stage)
    bytes_launch = 3 * state_bytes  # reads u^(s) and u^n, writes u^(s+1)
    achieved = bytes_launch / (avg_ms * 1e-3) / 1e9
    copy_gbs = copy_peak_gbs()
    if args.copy_calibration:  # the known-size copy for rocprofv3 FETCH_SIZE / WRITE_SIZE
        src = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst
    flops = fp64_per_launch()
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
            "kernel": "k_stage_2d_euler<2, stage 2|3>",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic_for(bytes_launch),
            "algorithmic_bytes_per_launch": bytes_launch,
            "avg_launch_ms": avg_ms,
            "autotuned_rows": tuned_rows,
            "peak_measured_copy": copy_gbs,
            "frac_of_measured_copy": achieved / copy_gbs,
            "fp64_flops_per_launch": flops,
            "fp64_tflops": (flops / (avg_ms * 1e-3) / 1e12) if flops else None,
            "fp64_frac": (flops / (avg_ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS) if flops else None,
            "fp64_peak_tflops": FP64_PEAK_TFLOPS,
        },
        "step": {
            "algorithmic_bytes": 64 * dofs,
            "hbm_frac_of_step": 64 * dofs / (el / steps) / 1e9 / HBM_PEAK_GBS,
            "hbm_frac_of_step_measured_copy": 64 * dofs / (el / steps) / 1e9 / copy_gbs,
            "ms_per_step_profiled": 1e3 * el_p / max(1, steps_p),
            "kernels": kinds,
            "troubled_fraction": troubled_p / max(1, 3 * wl.cells * steps_p),
            "t_after": t,
        },
    }
    nets = learned_nets("cuda:0")
    out["learned"] = (indicator_leg(wl, state_warm, t_warm, args.steps, 2, dg.IND_LEARNED, net=nets[2])
                      if 2 in nets else None)
    out["kxrcf"] = indicator_leg(wl, state_warm, t_warm, args.steps, 2, dg.IND_KXRCF)
    out["characteristic"] = indicator_leg(wl, state_warm, t_warm, args.steps, 2, limiter=dg.LIM_CSWENO_CHAR)
    del state_warm
    if not args.no_late:
        out["late_window"] = late_window_leg(prob, wl, state, t, args.late_t, args.steps, net=nets.get(2))
    prob.close()
    del state
    torch.cuda.empty_cache()
    if not args.no_burgers2d:
        out["burgers2d"] = burgers2d_leg(args.steps, args.warmup)
        torch.cuda.empty_cache()
    if not args.no_shu_osher:
        out["shu_osher"] = shu_osher_leg()
    if not args.no_double_mach:
        out["double_mach"] = double_mach_leg(args.steps, 2, to_end=args.double_mach_to_end)
        torch.cuda.empty_cache()
    if not args.no_batched:
        out["batched"] = batched_leg(args.batched_steps, 2, nets=nets)
        torch.cuda.empty_cache()
        out["batched_positivity"] = batched_leg(args.batched_steps, 2, positivity=1)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(seed=args.seed)
        out["cpu_baseline"].update(host_info())
        out["cpu_baseline"]["single_thread"] = cpu_single_thread(seed=args.seed)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
