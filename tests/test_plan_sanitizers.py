"""The host planner (plan.cpp, plain C++) under AddressSanitizer and UBSan,
driven over seeded random matrices and options by tests/native/plan_fuzz.cpp
(CPU only; nothing here touches a GPU)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_planner_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "plan_fuzz")
    src = [os.path.join(ROOT, "tests", "native", "plan_fuzz.cpp"),
           os.path.join(ROOT, "paper_2606_22482_amd", "csrc", "plan.cpp")]
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-pthread",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_2606_22482_amd", "csrc")] + src + ["-o", exe]
    subprocess.check_call(cmd)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1", SPMM_PLAN_THREADS="3")
    r = subprocess.run([exe, "300"], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "ok 300 cases" in r.stdout


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_planner_threads_under_tsan(tmp_path):
    """The planner's threaded column stage and row ranges (3 threads forced)
    under ThreadSanitizer: no data race on fuzzed inputs."""
    exe = str(tmp_path / "plan_fuzz_tsan")
    src = [os.path.join(ROOT, "tests", "native", "plan_fuzz.cpp"),
           os.path.join(ROOT, "paper_2606_22482_amd", "csrc", "plan.cpp")]
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-pthread", "-fsanitize=thread",
           "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_2606_22482_amd", "csrc")] + src + ["-o", exe]
    subprocess.check_call(cmd)
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1", SPMM_PLAN_THREADS="3")
    r = subprocess.run([exe, "100"], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "ok 100 cases" in r.stdout
