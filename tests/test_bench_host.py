"""Host-side checks of bench.py (no GPU): more than one GPU is refused with
a message before any device work, and the HBM traffic figure is used only
when the committed counter summary was taken on the current kernel source."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_traffic_only_for_the_current_kernel_source(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    from paper_1904_11147_amd.profiling import kernel_source_hash
    f = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.traffic_for(1.0) is None  # no file
    f.write_text(json.dumps({"kernel_source_sha256_16": kernel_source_hash(), "hbm_bytes_per_launch": 123.0}))
    assert bench.traffic_for(1.0) == 123.0
    f.write_text(json.dumps({"kernel_source_sha256_16": "0" * 16, "hbm_bytes_per_launch": 123.0}))
    assert bench.traffic_for(1.0) is None  # stale: the kernels changed since


def test_fp64_figure_only_for_the_current_kernel_source(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    from paper_1904_11147_amd.profiling import kernel_source_hash
    f = tmp_path / "fp64.json"
    monkeypatch.setattr(bench, "FP64_FILE", str(f))
    assert bench.fp64_per_launch() is None
    f.write_text(json.dumps({"kernel_source_sha256_16": kernel_source_hash(), "fp64_flops_per_launch": 7.0}))
    assert bench.fp64_per_launch() == 7.0
    f.write_text(json.dumps({"kernel_source_sha256_16": "1" * 16, "fp64_flops_per_launch": 7.0}))
    assert bench.fp64_per_launch() is None


def test_host_info_names_the_cpu():
    sys.path.insert(0, ROOT)
    import bench
    h = bench.host_info()
    assert h["host_cpus_usable"] >= 1 and h["host_cpus_total"] >= h["host_cpus_usable"]
    assert h["cpu_model"]


def test_trace_legs_split(tmp_path):
    """profiling.legs: the first leg ends with the limiter pass (indicator,
    reconstruction, scatter) of the last dispatch matching `before`, and the
    second leg is every dispatch after it, whatever order the CSV lists them in."""
    import csv
    sys.path.insert(0, ROOT)
    from paper_1904_11147_amd import profiling
    rows, t = [], 0

    def add(name, us):
        nonlocal t
        rows.append({"Kernel_Name": f"void dg::(anonymous namespace)::{name}(int)", "Start_Timestamp": t,
                     "End_Timestamp": t + 1000 * us})
        t += 1000 * us + 7

    for _ in range(4):  # first leg: TVB passes
        for k, us in (("k_stage", 10), ("k_indicator<2, 1, 2, false, false>", 3), ("k_csweno", 5), ("k_scatter", 2)):
            add(k, us)
    for _ in range(3):  # second leg: learned passes
        for k, us in (("k_stage", 10), ("k_indicator_learned<2, 1, false>", 6), ("k_csweno", 8), ("k_scatter", 4)):
            add(k, us)
    path = tmp_path / "trace.csv"
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=list(rows[0]))
        w.writeheader()
        for r in reversed(rows):  # out of order on purpose
            w.writerow(r)
    out = tmp_path / "legs.txt"
    profiling.legs(str(path), r"k_indicator<2, 1, 2, false, false>", 8, "test", str(out))
    text = out.read_text()
    first, second = text.split("== second leg")
    assert "8 dispatches" in first and "k_indicator_learned" not in first
    assert "12 dispatches" in second and "k_indicator<2" not in second
    line = [l for l in second.splitlines() if l.startswith("k_csweno")][0].split()
    assert int(line[1]) == 3 and abs(float(line[2]) - 8.0) < 1e-9
