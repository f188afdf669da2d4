"""Host tests of the benchmark's pieces that run without a GPU: the one-GPU
refusal and the CPU baseline (the oracle, timed on a bounded sample)."""
import importlib.util
import os
import subprocess
import sys

from paper_1707_05354_amd import workload as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BENCH = os.path.join(ROOT, "bench.py")


def _load_bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", BENCH)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, BENCH, "--gpus", "2"], capture_output=True, text=True,
                       timeout=300, cwd=ROOT)
    assert r.returncode == 2
    assert r.stdout.strip() == ""  # no JSON line: nothing was measured
    assert "one GPU" in r.stderr


def test_world_size_above_one_is_refused():
    env = dict(os.environ, WORLD_SIZE="2", RANK="0", LOCAL_RANK="0")
    r = subprocess.run([sys.executable, BENCH], capture_output=True, text=True, timeout=300,
                       cwd=ROOT, env=env)
    assert r.returncode == 2
    assert r.stdout.strip() == ""


def test_cpu_baseline_times_the_oracle_on_a_bounded_sample():
    bench = _load_bench()
    w = W.tiny()
    cb = bench.cpu_baseline(w, budget_s=0.2)
    assert cb["kind"] == "oracle" and cb["cores"] == 1
    assert cb["unit"] == "M updates/s" and cb["value"] > 0
    assert cb["sample"].startswith("first ") and ("of %d update batches" % w.R) in cb["sample"]
    n_done = int(cb["sample"].split()[1])
    assert 1 <= n_done <= w.R
    assert cb["seconds"] >= 0 and cb["host_cpus"] == os.cpu_count()
    assert isinstance(cb["cpu_model"], str) and cb["cpu_model"]
