"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

Two drivers are built with gcc/g++ and the sanitizers, and run:
* tests/sanitize/oracle_synth_check.c runs every entry point of the C
  oracle and of the seeded generators, edge cases included, with output
  buffers of exactly the size each call needs;
* tests/sanitize/hostbook_check.cpp runs the serving arena's allocator and
  the stream's window cutter (the library's host-side bookkeeping, which
  needs no GPU) under random operation sequences against brute-force models.
Any out-of-bounds access, leak or undefined operation fails the run.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def _build_and_run(tmp_path, compiler, std, sources, extra=()):
    if shutil.which(compiler) is None:
        pytest.skip("%s not available" % compiler)
    exe = str(tmp_path / "check")
    cmd = [compiler, std] + SAN + list(extra) + ["-o", exe] + [os.path.join(ROOT, s) for s in sources] + ["-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr


def test_oracle_and_generators_under_sanitizers(tmp_path):
    _build_and_run(tmp_path, "gcc", "-std=c11", ["tests/sanitize/oracle_synth_check.c", "oracle/oracle.c",
                                                  "oracle/bpe_train.c", "synth/synth.c"])


def test_host_bookkeeping_under_sanitizers(tmp_path):
    _build_and_run(tmp_path, "g++", "-std=c++17", ["tests/sanitize/hostbook_check.cpp"],
                   extra=["-I", os.path.join(ROOT, "paper_2601_05531_amd", "csrc")])
