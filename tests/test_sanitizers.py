"""Address and undefined-behaviour sanitizer runs of the host-side code (CPU).

Four programs are built with -fsanitize=address,undefined (any finding
aborts the run) and run on seeded random inputs:
  - tests/native/oracle_check.c drives every entry point of the C oracle
    and checks its results against the invariants they must satisfy and
    against each other (summarize, its direction/label extension, the
    fixed-count iteration and the strided step);
  - tests/native/resolve_check.cpp drives the host-side resolution of
    update batches (csrc/bsim_resolve.h, the same header the library
    compiles) against a plain sequential model of the operations, valid
    and invalid batches alike (also built with the thread sanitizer, for
    the passes that split a large batch over host threads);
  - tests/native/pool_check.cpp drives the host thread pool of those
    passes: every share once, concurrent callers, exceptions (built with
    each sanitizer);
  - tests/native/sched_check.cpp drives the serving loop's scheduler
    (csrc/bsim_sched.h) from submitter, worker and poller threads with a
    fake executor, built once with the thread sanitizer and once with the
    address and undefined-behaviour sanitizers.
No GPU is involved."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def _build(compiler, std, sources, exe_name, san=None):
    if shutil.which(compiler) is None:
        pytest.skip(compiler + " not found")
    out_dir = os.path.join(ROOT, "_build")
    os.makedirs(out_dir, exist_ok=True)
    exe = os.path.join(out_dir, "%s_%d" % (exe_name, os.getpid()))  # one per test process
    cmd = [compiler, std, "-Wall", "-Wextra"] + (san or SAN) + [
        "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2111_12493_amd", "csrc")] + [
        os.path.join(ROOT, s) for s in sources] + ["-o", exe, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


def _run(exe, seed):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
               TSAN_OPTIONS="halt_on_error=1:second_deadlock_stack=1")
    r = subprocess.run([exe, str(seed)], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert r.stdout.strip().startswith("ok "), r.stdout
    assert "runtime error" not in r.stderr, r.stderr[-4000:]
    assert "WARNING: ThreadSanitizer" not in r.stderr, r.stderr[-4000:]
    return int(r.stdout.split()[1])


@pytest.fixture(scope="module")
def oracle_exe():
    return _build("gcc", "-std=c99", ["oracle/bsim_oracle.c", "tests/native/oracle_check.c"], "oracle_check")


@pytest.fixture(scope="module")
def resolve_exe():
    return _build("g++", "-std=c++17", ["tests/native/resolve_check.cpp"], "resolve_check")


@pytest.mark.parametrize("seed", [1, 2])
def test_oracle_under_sanitizers(oracle_exe, seed):
    assert _run(oracle_exe, seed) > 300


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_update_resolution_under_sanitizers(resolve_exe, seed):
    assert _run(resolve_exe, seed) > 400


@pytest.mark.parametrize("san", ["asan", "tsan"])
def test_resolution_thread_pool_under_sanitizers(san):
    flags = ["-O1", "-g", "-fsanitize=thread"] if san == "tsan" else None
    exe = _build("g++", "-std=c++17", ["tests/native/pool_check.cpp"], "pool_check_" + san, flags)
    assert _run(exe, 1) > 400


def test_update_resolution_under_the_thread_sanitizer():
    # the large batches split their checks, sorts and emit passes over
    # several host threads
    exe = _build("g++", "-std=c++17", ["tests/native/resolve_check.cpp"], "resolve_check_tsan",
                 ["-O1", "-g", "-fsanitize=thread"])
    assert _run(exe, 1) > 400


@pytest.fixture(scope="module")
def sched_exes():
    src = ["tests/native/sched_check.cpp"]
    return [_build("g++", "-std=c++17", src, "sched_check_tsan", ["-O1", "-g", "-fsanitize=thread"]),
            _build("g++", "-std=c++17", src, "sched_check_asan")]


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_scheduler_under_sanitizers(sched_exes, seed):
    for exe in sched_exes:
        assert _run(exe, seed) > 1000
