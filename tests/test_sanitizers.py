"""Host code under sanitizers (no GPU): the multi-core lockless CPU table
under ThreadSanitizer, a CPU-thread model of the GPU kernels' protocols under
ThreadSanitizer (with planted ordering mistakes it must catch) and, for the
exploration without level barriers, also built without a sanitizer and run
many times, and the tuning-file reader under AddressSanitizer and
UndefinedBehaviorSanitizer with mutated inputs."""
import os
import shutil
import subprocess

import pytest

from conftest import ROOT

HERE = os.path.join(ROOT, "tests", "sanitize")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_cpu_table_under_thread_sanitizer(tmp_path):
    exe = str(tmp_path / "cpu_table_threads")
    subprocess.check_call(["g++", "-O1", "-g", "-std=c++17", "-fsanitize=thread", "-pthread",
                           os.path.join(HERE, "cpu_table_threads.cpp"),
                           os.path.join(ROOT, "cpu_table", "cpu_table.cpp"), "-o", exe])
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600,
                       env=dict(os.environ, TSAN_OPTIONS="halt_on_error=1 exitcode=66"))
    assert "ThreadSanitizer" not in r.stderr, r.stderr[-4000:]
    assert r.returncode == 0, r.stdout + r.stderr[-2000:]


def _protocol_model(tmp_path, plant):
    exe = str(tmp_path / f"gpu_protocol_model_{plant}")
    subprocess.check_call(["g++", "-O1", "-g", "-std=c++17", "-fsanitize=thread", "-pthread", f"-DPLANT={plant}",
                           os.path.join(HERE, "gpu_protocol_model.cpp"), "-o", exe])
    return subprocess.run([exe], capture_output=True, text=True, timeout=600,
                          env=dict(os.environ, TSAN_OPTIONS="halt_on_error=1 exitcode=66"))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_gpu_protocol_model_under_thread_sanitizer(tmp_path):
    """Find-or-put's claim / row write / publish / bounded wait, the batch
    ring with last-tile level finalisation, the ring alone, and the
    persistent server (admission into running workers, completion records,
    draining and relaunch, slot reuse), the merge of a pass's equal
    successors, and segmented appends to the next frontier with the cap's
    abort, modelled with threads and the kernels' orderings: no race, every
    result equals a sequential BFS, no merged pass loses a state, and every
    appended state is listed once (gpu_protocol_model.cpp)."""
    r = _protocol_model(tmp_path, 0)
    assert "ThreadSanitizer" not in r.stderr, r.stderr[-4000:]
    assert r.returncode == 0 and "errors 0" in r.stdout, r.stdout + r.stderr[-2000:]
    assert "WRONG" not in r.stdout


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
@pytest.mark.parametrize("plant,what", [
    (1, "DONE published before the row is written"),
    (2, "DONE published without release"),
    (3, "matching row compared without waiting for DONE"),
    (4, "ring cell freed before its item is read"),
    (5, "finished tile counted without ordering"),
    (6, "admission tail raised without release"),
    (7, "completion record published without release"),
    (8, "completion record filled after it is published"),
    (9, "successors merged on a tag match without comparing the vectors"),
    (10, "another lane's successor read without the pass barrier"),
    (11, "a flush placed past the end of its segment"),
    (12, "abort raised on the workgroup's own estimate, without the cursors"),
    (13, "a queue entry written without release"),
    (14, "held-back states counted as open only once appended"),
])
def test_gpu_protocol_model_catches_planted_mistakes(tmp_path, plant, what):
    r = _protocol_model(tmp_path, plant)
    assert "ThreadSanitizer: data race" in r.stderr or r.returncode != 0, f"not caught: {what}"


def _stress(tmp_path, plant, part, reps):
    exe = str(tmp_path / f"gpu_protocol_model_o2_{plant}")
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-pthread", f"-DPLANT={plant}",
                           os.path.join(HERE, "gpu_protocol_model.cpp"), "-o", exe])
    return subprocess.run([exe, part, str(reps)], capture_output=True, text=True, timeout=600)


def _exploration_stress(tmp_path, plant):
    return _stress(tmp_path, plant, "part7", 20)


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_persistent_server_stress(tmp_path):
    """The persistent server, 200 runs of 160 queries without a sanitizer:
    every query's result equals a sequential BFS and no producer waits for
    a cell that is never freed.  (Keeping an admitted query's first tile
    while holding a ring position, an earlier rule, stops here in about one
    run of 20 to 500.)"""
    r = _stress(tmp_path, 0, "part4", 200)
    assert r.returncode == 0 and r.stdout.strip().endswith("errors 0"), r.stdout[-3000:]


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_exploration_without_levels_stress(tmp_path):
    """The exploration without level barriers, 20 x 128 runs without a
    sanitizer (threads interleave finely): every run lists the reachable set
    once, expands every entry once and ends with no open state, and no
    worker leaves while states are still to be found."""
    r = _exploration_stress(tmp_path, 0)
    assert r.returncode == 0 and r.stdout.strip().endswith("errors 0"), r.stdout[-3000:]


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_exploration_stress_catches_late_count(tmp_path):
    """Planted: states appended in the middle of a tile enter the work count
    only when the tile ends.  A workgroup that expands them first can take
    the count to zero while the tile is open; idle workgroups then leave with
    chunks that later states land in, and those states are never expanded."""
    r = _exploration_stress(tmp_path, 15)
    assert r.returncode != 0 and "WRONG" in r.stdout


HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="needs hipcc")
def test_tune_reader_under_address_sanitizer(tmp_path):
    exe = str(tmp_path / "tune_reader_fuzz")
    csrc = os.path.join(ROOT, "paper_1004_2772_amd", "csrc")
    # host code only: every sanitizer flag is scoped to the host pass
    subprocess.check_call([HIPCC, "-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer",
                           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                           "-I" + os.path.join(ROOT, "include"), "-I" + csrc,
                           os.path.join(HERE, "tune_reader_fuzz.cpp"), os.path.join(csrc, "tune.cpp"), "-o", exe],
                          stderr=subprocess.DEVNULL)
    r = subprocess.run([exe, os.path.join(ROOT, "paper_1004_2772_amd", "tune.json"), "4000",
                        str(tmp_path / "mutated.json")],
                       capture_output=True, text=True, timeout=600,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1",
                                UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1"))
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
    assert r.returncode == 0 and "iterations 4000" in r.stdout, r.stdout + r.stderr[-2000:]
