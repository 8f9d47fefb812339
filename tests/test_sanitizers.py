"""Host code under sanitizers (no GPU): the multi-core lockless CPU table
under ThreadSanitizer, and the tuning-file reader under AddressSanitizer and
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
