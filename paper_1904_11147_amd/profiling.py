"""Summaries of rocprofv3 output for the committed profiles.

    python -m paper_1904_11147_amd.profiling stats  <kernel_stats.csv> --cmd "<command>" --out <summary.txt>
    python -m paper_1904_11147_amd.profiling traffic --fetch <csv> --write <csv> --kernel <regex>
            --copy-kernel <regex> --copy-bytes <B> --cmd "<command>" --out <traffic.json>
    python -m paper_1904_11147_amd.profiling counters <counter_collection.csv> --cmd "<command>" --out <summary.txt>
    python -m paper_1904_11147_amd.profiling fp64 <counter_collection.csv> --kernel <regex> --cmd "<command>"
            --out <fp64.json>

`stats` shortens the kernel names of a `--kernel-trace --stats` CSV and keeps
calls, total, average, min and max duration.  `traffic` turns two `--pmc`
runs (FETCH_SIZE, then WRITE_SIZE, both in KiB per dispatch) into HBM bytes
per launch of one kernel, each counter scaled by what it reads for a plain
copy kernel that moves a known number of bytes (read once, written once).
The result records the hash of the kernel source it was taken on, so that a
reader can tell when the kernel has changed since.  `fp64` turns a `--pmc`
run of SQ_INSTS_VALU_ADD_F64, _MUL_F64, _FMA_F64 and _TRANS_F64 (wavefront
instructions per dispatch) into FP64 flops per launch of one kernel: 64
lanes per instruction, two flops per FMA (inactive lanes count too, so this
is an upper bound on the useful flops).
"""
import argparse
import csv
import hashlib
import json
import os
import re
import statistics

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KERNEL_SOURCE = os.path.join(ROOT, "paper_1904_11147_amd", "csrc", "dg_kernels.hip")


def kernel_source_hash():
    return hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()[:16]


def short_name(k):
    k = k.replace("void ", "").replace("dg::(anonymous namespace)::", "").replace("(anonymous namespace)::", "")
    k = re.sub(r"\(.*$", "", k)
    return k[:110]


def stats(path, cmd, out):
    rows = list(csv.DictReader(open(path)))
    lines = [f"# rocprofv3 kernel statistics", f"# command: {cmd}", "#",
             f"{'kernel':<110} {'calls':>7} {'total_ms':>10} {'avg_us':>10} {'min_us':>10} {'max_us':>10} {'pct':>6}"]
    for r in rows:
        lines.append(f"{short_name(r['Name']):<110} {int(r['Calls']):>7} {float(r['TotalDurationNs']) / 1e6:>10.3f} "
                     f"{float(r['AverageNs']) / 1e3:>10.2f} {float(r['MinNs']) / 1e3:>10.2f} "
                     f"{float(r['MaxNs']) / 1e3:>10.2f} {float(r['Percentage']):>6.2f}")
    open(out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def _per_dispatch(path, counter):
    """{kernel name: [value per dispatch]} of one counter (KiB per dispatch)."""
    acc = {}
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        key = (r["Kernel_Name"], r["Dispatch_Id"])
        acc[key] = acc.get(key, 0.0) + float(r["Counter_Value"])
    res = {}
    for (k, _), v in acc.items():
        res.setdefault(k, []).append(v)
    return res


def _pick(d, pattern):
    hits = [k for k in d if re.search(pattern, k)]
    if not hits:
        raise SystemExit(f"no kernel matching {pattern!r} among {sorted(map(short_name, d))}")
    vals = [v for k in hits for v in d[k]]
    return hits, vals


def traffic(fetch, write, kernel, copy_kernel, copy_bytes, cmd, out):
    f = _per_dispatch(fetch, "FETCH_SIZE")
    w = _per_dispatch(write, "WRITE_SIZE")
    _, cf = _pick(f, copy_kernel)
    _, cw = _pick(w, copy_kernel)
    kf_names, kf = _pick(f, kernel)
    _, kw = _pick(w, kernel)
    fetch_scale = copy_bytes / (statistics.median(cf) * 1024)
    write_scale = copy_bytes / (statistics.median(cw) * 1024)
    fetch_b = statistics.mean(kf) * 1024 * fetch_scale
    write_b = statistics.mean(kw) * 1024 * write_scale
    res = {
        "kernel": short_name(kf_names[0]),
        "kernel_source_sha256_16": kernel_source_hash(),
        "dispatches": {"fetch": len(kf), "write": len(kw)},
        "fetch_kib_per_launch_raw": statistics.mean(kf),
        "write_kib_per_launch_raw": statistics.mean(kw),
        "copy_kernel": short_name(_pick(f, copy_kernel)[0][0]),
        "copy_bytes_each_way": copy_bytes,
        "copy_fetch_kib_raw": statistics.median(cf),
        "copy_write_kib_raw": statistics.median(cw),
        "fetch_scale": fetch_scale,
        "write_scale": write_scale,
        "fetch_bytes_per_launch": fetch_b,
        "write_bytes_per_launch": write_b,
        "hbm_bytes_per_launch": fetch_b + write_b,
        "command": cmd,
    }
    json.dump(res, open(out, "w"), indent=1)
    print(json.dumps(res, indent=1))


def counters(path, cmd, out):
    """Per-kernel averages per dispatch of SQ counters, and per-wavefront
    figures (cycles, VALU / LDS / vector-memory instructions, the fraction of
    a wavefront's cycles with a VALU instruction active or waiting)."""
    acc, disp = {}, {}
    for r in csv.DictReader(open(path)):
        k = short_name(r["Kernel_Name"])
        acc.setdefault(k, {}).setdefault(r["Counter_Name"], 0.0)
        acc[k][r["Counter_Name"]] += float(r["Counter_Value"])
        disp.setdefault(k, set()).add(r["Dispatch_Id"])
    lines = ["# rocprofv3 SQ counters, averages per dispatch", f"# command: {cmd}", "#",
             f"{'kernel':<40} {'disp':>5} {'waves':>8} {'cyc/wave':>9} {'valu/wave':>10} {'lds/wave':>9} "
             f"{'vmem/wave':>10} {'valu_act':>9} {'wait':>6}"]
    for k in sorted(acc):
        n = len(disp[k])
        d = {c: v / n for c, v in acc[k].items()}
        waves = max(d.get("SQ_WAVES", 0.0), 1.0)
        wc = max(d.get("SQ_WAVE_CYCLES", 0.0), 1.0)
        lines.append(f"{k[:40]:<40} {n:>5} {waves:>8.0f} {wc / waves:>9.0f} {d.get('SQ_INSTS_VALU', 0) / waves:>10.0f} "
                     f"{d.get('SQ_INSTS_LDS', 0) / waves:>9.0f} {d.get('SQ_INSTS_VMEM_RD', 0) / waves:>10.0f} "
                     f"{d.get('SQ_ACTIVE_INST_VALU', 0) / wc:>9.3f} {d.get('SQ_WAIT_INST_ANY', 0) / wc:>6.3f}")
    open(out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def fp64(path, kernel, cmd, out):
    names = ("SQ_INSTS_VALU_ADD_F64", "SQ_INSTS_VALU_MUL_F64", "SQ_INSTS_VALU_FMA_F64", "SQ_INSTS_VALU_TRANS_F64")
    per = {c: _pick(_per_dispatch(path, c), kernel) for c in names}
    hits = per[names[0]][0]
    mean = {c: statistics.mean(v[1]) for c, v in per.items()}
    flops = 64.0 * (mean[names[0]] + mean[names[1]] + mean[names[3]]) + 128.0 * mean[names[2]]
    res = {"kernel": short_name(hits[0]), "kernel_source_sha256_16": kernel_source_hash(),
           "dispatches": len(per[names[0]][1]), "wave_instructions_per_launch": mean,
           "fp64_flops_per_launch": flops, "command": cmd}
    json.dump(res, open(out, "w"), indent=1)
    print(json.dumps(res, indent=1))


def legs(path, before, window, cmd, out):
    """Per-kernel mean durations in the last two legs of one kernel trace
    (rocprofv3 kernel_trace.csv): the `window` dispatches that end two
    dispatches after the last one matching `before` (that leg's last limiter
    pass: indicator, reconstruction, scatter), and every dispatch after them
    (the next leg)."""
    rows = sorted(csv.DictReader(open(path)), key=lambda r: int(r["Start_Timestamp"]))
    last = max(i for i, r in enumerate(rows) if re.search(before, r["Kernel_Name"]))
    cut = min(len(rows), last + 3)
    lines = ["# rocprofv3 kernel trace, per-kernel mean durations of two legs", f"# command: {cmd}",
             f"# first leg: the {window} dispatches up to the last limiter pass after {before!r}; second leg: the rest", "#"]
    for label, part in (("first leg", rows[max(0, cut - window):cut]), ("second leg", rows[cut:])):
        acc = {}
        for r in part:
            acc.setdefault(short_name(r["Kernel_Name"]), []).append(
                (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
        lines.append(f"== {label}: {len(part)} dispatches")
        lines.append(f"{'kernel':<60} {'calls':>7} {'avg_us':>10} {'total_ms':>10}")
        for k, v in sorted(acc.items(), key=lambda kv: -sum(kv[1])):
            lines.append(f"{k[:60]:<60} {len(v):>7} {sum(v) / len(v):>10.1f} {sum(v) / 1e3:>10.2f}")
    open(out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--cmd", required=True)
    s.add_argument("--out", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--kernel", required=True, help="regular expression on the kernel name")
    t.add_argument("--copy-kernel", required=True, help="regular expression on the kernel name")
    t.add_argument("--copy-bytes", type=float, required=True)
    t.add_argument("--cmd", required=True)
    t.add_argument("--out", required=True)
    c = sub.add_parser("counters")
    c.add_argument("csv")
    c.add_argument("--cmd", required=True)
    c.add_argument("--out", required=True)
    g = sub.add_parser("legs")
    g.add_argument("csv")
    g.add_argument("--before", required=True, help="regular expression on the kernel name")
    g.add_argument("--window", type=int, required=True)
    g.add_argument("--cmd", required=True)
    g.add_argument("--out", required=True)
    f = sub.add_parser("fp64")
    f.add_argument("csv")
    f.add_argument("--kernel", required=True, help="regular expression on the kernel name")
    f.add_argument("--cmd", required=True)
    f.add_argument("--out", required=True)
    a = ap.parse_args()
    if a.what == "legs":
        legs(a.csv, a.before, a.window, a.cmd, a.out)
    elif a.what == "fp64":
        fp64(a.csv, a.kernel, a.cmd, a.out)
    elif a.what == "stats":
        stats(a.csv, a.cmd, a.out)
    elif a.what == "counters":
        counters(a.csv, a.cmd, a.out)
    else:
        traffic(a.fetch, a.write, a.kernel, a.copy_kernel, a.copy_bytes, a.cmd, a.out)


if __name__ == "__main__":
    main()
