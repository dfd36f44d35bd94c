"""The benchmark line's contract, checked on the CPU.

* More than one GPU is refused with a message, before anything touches a GPU.
* The HBM traffic the line reports for the D = 100 evaluation kernel comes
  from a committed counter summary that was taken on the current kernel
  sources (the summary records a SHA-256 of them); a kernel edit without new
  counters fails here instead of silently dropping the figure.
* That summary's traffic follows from its own counter readings: the fetched
  and written KiB per dispatch, each scaled by what the same counter reads
  for a device copy of known size.
"""
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _summary(b):
    with open(b.HBM_PROFILE) as f:
        kv = dict(l.split(":", 1) for l in f if ":" in l and not l.startswith(" "))
    return {k.strip(): v.strip() for k, v in kv.items()}


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_summary_matches_the_kernel_sources():
    b = _bench()
    kv = _summary(b)
    assert kv["source_sha256"] == b.kernel_source_hash(), \
        "the D = 100 kernel sources changed since the HBM counters were taken: retake FETCH_SIZE and WRITE_SIZE"
    assert b.measured_traffic() is not None


def test_traffic_follows_from_the_counters_and_the_copy_calibration():
    kv = _summary(_bench())
    copy_bytes = float(kv["copy_bytes"].split()[0])
    fetch_scale = copy_bytes / (float(kv["copy_fetch_kib_per_dispatch"]) * 1024)
    write_scale = copy_bytes / (float(kv["copy_write_kib_per_dispatch"]) * 1024)
    assert abs(fetch_scale - float(kv["fetch_scale"])) < 1e-4
    assert abs(write_scale - float(kv["write_scale"])) < 1e-4
    traffic = (float(kv["fetch_kib_per_dispatch"]) * 1024 * float(kv["fetch_scale"])
               + float(kv["write_kib_per_dispatch"]) * 1024 * float(kv["write_scale"]))
    assert abs(traffic - float(kv["traffic_bytes_per_launch"])) <= 1.0
    ratio = float(kv["traffic_bytes_per_launch"]) / float(kv["algorithmic_bytes_per_launch"])
    assert abs(ratio - float(kv["traffic_over_algorithmic"])) < 1e-3
