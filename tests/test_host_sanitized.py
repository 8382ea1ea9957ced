"""Host code of the library (the planner and the staged work-list builders,
plain C++ without HIP) built with g++ and the address and undefined-behaviour
sanitizers, and run over many plan sizes and random batches: every input
column is covered once, every launch reads only its own item list within its
size (including batches whose plans all take the windowed product), every
transform is listed once.  No GPU."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2004_11610_amd", "csrc")


@pytest.mark.slow
def test_planner_and_work_lists_under_sanitizers(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not found")
    exe = str(tmp_path / "worklist_check")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           os.path.join(CSRC, "planner.cpp"), os.path.join(CSRC, "worklist.cpp"),
           os.path.join(ROOT, "tests", "host", "worklist_check.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    print(r.stdout[-2000:])
    assert r.returncode == 0, (r.stdout[-4000:], r.stderr[-4000:])
    assert "failures 0" in r.stdout
