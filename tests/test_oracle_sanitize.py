"""Run the CPU oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

``oracle/sanitize_check.cpp`` drives both oracles through every C entry point
on seeded random streams (insert, delete, mixed and coalesced batches, partial
batches, cleanups, rejected batch sizes) and checks that the dictionary the
cascade layout encodes equals the map oracle's after every step.  Built here
with g++ and the sanitizers set to abort on the first report, so an
out-of-bounds access, use after free, leak or undefined operation in the
oracle fails this test.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")


def _build_and_run(tmp_path, oracle_src):
    exe = str(tmp_path / "oracle_sanitize")
    build = subprocess.run(
        ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
         "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
         os.path.join(ORACLE, "sanitize_check.cpp"), oracle_src, "-o", exe],
        capture_output=True, text=True, timeout=300)
    if build.returncode != 0 and "sanitize" in build.stderr and "cannot find" in build.stderr:
        pytest.skip("sanitizer runtime not installed: " + build.stderr.strip()[:200])
    assert build.returncode == 0, build.stderr
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    return subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_oracle_is_clean_under_sanitizers(tmp_path):
    run = _build_and_run(tmp_path, os.path.join(ORACLE, "lsm_oracle.cpp"))
    assert run.returncode == 0, run.stdout + run.stderr
    assert "runtime error" not in run.stderr and "Sanitizer" not in run.stderr, run.stderr
    assert "oracle sanitize check: ok" in run.stdout


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_planted_overflow_is_reported(tmp_path):
    # A copy of the oracle whose level copy reads one element past the end:
    # the run must stop with an AddressSanitizer report, which shows that
    # the checks above are live.
    src = open(os.path.join(ORACLE, "lsm_oracle.cpp")).read()
    old = "for (size_t p = 0; p < L.size(); ++p) {"
    assert src.count(old) == 1
    bad = tmp_path / "lsm_oracle_overflow.cpp"
    bad.write_text(src.replace(old, "for (size_t p = 0; p <= L.size(); ++p) {"))
    run = _build_and_run(tmp_path, str(bad))
    assert run.returncode != 0
    assert "AddressSanitizer" in run.stderr, run.stderr[-2000:]
