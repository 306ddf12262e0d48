"""The library's host code under sanitizers, on the CPU: the planner and
pattern validation built with AddressSanitizer and UndefinedBehaviorSanitizer
over random patterns and motif sets (every pattern edge covered exactly once,
columns a permutation), and the batch planning pool and the plan cache that
server workers share built with ThreadSanitizer under concurrent use.  The
checks are tests/sanitize/host_checks.cpp, compiled here with g++ (host
code only; nothing here touches a GPU)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = [os.path.join(ROOT, "tests", "sanitize", "host_checks.cpp"),
       os.path.join(ROOT, "paper_2508_21287_amd", "csrc", "planner.cpp")]


def build(tmp_path, name, flags):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not found")
    out = str(tmp_path / name)
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-I" + os.path.join(ROOT, "include"),
           "-I/opt/rocm/include"] + flags + SRC + ["-o", out, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    return out


def run(exe, mode, env_extra):
    env = dict(os.environ)
    env.update(env_extra)
    r = subprocess.run([exe, mode], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    return r.stdout


def test_planner_under_asan_ubsan(tmp_path):
    exe = build(tmp_path, "host_checks_asan", ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"])
    out = run(exe, "plan", {"ASAN_OPTIONS": "detect_leaks=1:abort_on_error=0",
                            "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"})
    assert "0 failures" in out, out


def test_pool_and_plan_cache_under_tsan(tmp_path):
    exe = build(tmp_path, "host_checks_tsan", ["-fsanitize=thread"])
    out = run(exe, "threads", {"TSAN_OPTIONS": "halt_on_error=1:second_deadlock_stack=1"})
    assert "0 failures" in out, out
