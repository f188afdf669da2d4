"""Run the HIP library's host code under AddressSanitizer and
UndefinedBehaviorSanitizer, on the CPU.

``csrc/lsm_api.hip`` (everything of the library that runs on the host) is
compiled as C++ with g++ against ``tests/host_sanitize/``: a stand-in for the
HIP runtime calls it makes (device memory is host memory) and stand-in
kernel launchers that touch the first and last element of every range the
real kernel would read or write.  The scratch-layout functions the launchers
need (sort scratch carving, scan and cleanup tile counts) are copied out of
the kernel source at build time, so the touched ranges follow the library's
real layout.  ``driver.cpp`` then calls every C entry point on seeded random
operation streams with allocation and launch failures injected; a sanitizer
report or a failed status check fails the test.  A second case plants a
one-element-short scratch allocation in a copy of the host code and checks
that the run reports it.  A third case checks the sort-scratch carving
itself: regions inside the allocation, disjoint, per-slot ones 16-byte
aligned.  A fourth builds the same host code with ThreadSanitizer and drives
handles from four threads at once (calls on different handles are
independent).
"""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1707_05354_amd", "csrc")
HERE = os.path.join(ROOT, "tests", "host_sanitize")
KERNELS = os.path.join(CSRC, "lsm_kernels.hip")

# Host functions and constants of the kernel source the stand-ins use.
LAYOUT = [
    r"^constexpr int kCleanItems = .*;$",
    r"^constexpr uint32_t kCleanTile = .*;$",
    r"^inline unsigned grid_for\(.*\}$",
    r"^size_t sort_meta_words\(uint32_t b\) \{",
    r"^SortMeta sort_meta_carve\(uint32_t\* base, uint32_t b, int parity, int slot\) \{",
    r"^int sort_kernel_count\(const SortArgs& a\) \{",
    r"^size_t scan_status_words\(uint32_t nq\) \{.*\}$",
    r"^uint32_t clean_tiles\(uint32_t n\) \{.*\}$",
]


def extract_layout(src: str) -> str:
    lines = src.splitlines()
    out = []
    for pat in LAYOUT:
        hits = [i for i, l in enumerate(lines) if re.match(pat, l)]
        assert len(hits) == 1, "kernel source: %r matched %d lines" % (pat, len(hits))
        i = hits[0]
        if lines[i].rstrip().endswith(("}", ";")):
            out.append(lines[i])
            continue
        j = i
        while lines[j] != "}":
            j += 1
        out.extend(lines[i:j + 1])
    return "\n".join(out) + "\n"


def build_and_run(tmp_path, api_src, sanitize="address,undefined", args=()):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    gen = tmp_path / "gen"
    gen.mkdir()
    (gen / "layout_gen.inc").write_text(extract_layout(open(KERNELS).read()))
    exe = str(tmp_path / "host_sanitize")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-pthread",
           "-fsanitize=" + sanitize, "-fno-sanitize-recover=all",
           "-I", HERE, "-I", str(gen), "-I", CSRC, "-I", os.path.join(ROOT, "include"),
           "-x", "c++", api_src, "-x", "none",
           os.path.join(HERE, "stand_in.cpp"), os.path.join(HERE, "driver.cpp"), "-o", exe]
    build = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    if build.returncode != 0 and "sanitize" in build.stderr and "cannot find" in build.stderr:
        pytest.skip("sanitizer runtime not installed: " + build.stderr.strip()[:200])
    assert build.returncode == 0, build.stderr[-4000:]
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["TSAN_OPTIONS"] = "halt_on_error=1"
    return subprocess.run([exe] + list(args), capture_output=True, text=True, timeout=600,
                          env=env)


def test_host_code_is_clean_under_sanitizers(tmp_path):
    run = build_and_run(tmp_path, os.path.join(CSRC, "lsm_api.hip"))
    assert run.returncode == 0, (run.stdout + run.stderr)[-6000:]
    assert "runtime error" not in run.stderr and "Sanitizer" not in run.stderr, run.stderr[-4000:]
    assert "host sanitize check: ok" in run.stdout
    m = re.search(r"(\d+) calls failed with LSM_ENOMEM, (\d+) with LSM_EHIP", run.stdout)
    assert m and int(m.group(1)) > 20 and int(m.group(2)) > 20, run.stdout  # both paths ran


def test_planted_short_scratch_is_reported(tmp_path):
    # The copy allocates the per-slot scatter buffers one element short: the
    # stand-in scatter's last write then lands past the allocation.
    src = open(os.path.join(CSRC, "lsm_api.hip")).read()
    old = "(s = dev_alloc(h, &p, kSortSlots * bb)) == LSM_OK)\n    for (int i = 0; i < kSortSlots; ++i) h->scat_kv[i]"
    assert src.count(old) == 1
    bad = tmp_path / "lsm_api_short.hip"
    bad.write_text(src.replace(old, old.replace("kSortSlots * bb", "kSortSlots * bb - 4")))
    run = build_and_run(tmp_path, str(bad))
    assert run.returncode != 0
    assert "AddressSanitizer" in run.stderr, run.stderr[-3000:]


def test_sort_scratch_layout(tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    gen = tmp_path / "gen"
    gen.mkdir()
    (gen / "layout_gen.inc").write_text(extract_layout(open(KERNELS).read()))
    exe = str(tmp_path / "layout_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-I", HERE, "-I", str(gen), "-I", CSRC,
           os.path.join(HERE, "layout_check.cpp"), "-o", exe]
    build = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    if build.returncode != 0 and "sanitize" in build.stderr and "cannot find" in build.stderr:
        pytest.skip("sanitizer runtime not installed: " + build.stderr.strip()[:200])
    assert build.returncode == 0, build.stderr[-4000:]
    run = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert run.returncode == 0, (run.stdout + run.stderr)[-4000:]
    assert "sort scratch layout: ok" in run.stdout


def test_handles_on_threads_under_thread_sanitizer(tmp_path):
    run = build_and_run(tmp_path, os.path.join(CSRC, "lsm_api.hip"), sanitize="thread",
                        args=("1", "threads"))
    assert run.returncode == 0, (run.stdout + run.stderr)[-6000:]
    assert "ThreadSanitizer" not in run.stderr, run.stderr[-4000:]
    assert "host sanitize check, threads: ok" in run.stdout
