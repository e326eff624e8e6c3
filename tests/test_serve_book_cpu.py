"""CPU concurrency check of the serving loop's bookkeeping (serve_book.h: tickets, the
bounded admission queue, chunked delivery): tests/serve_book_check.cpp runs many
submitting, waiting and racing threads against a scheduler and four delivery threads,
with and without a failure part-way, built once under ThreadSanitizer and once under
AddressSanitizer + UndefinedBehaviorSanitizer; any report fails the test."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("san", ["thread", "address,undefined"])
def test_serve_book_under_sanitizer(tmp_path, san):
    exe = str(tmp_path / "serve_book_check")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-g", "-Wall", f"-fsanitize={san}",
                           "-fno-sanitize-recover=all",
                           "-I", os.path.join(ROOT, "include"),
                           "-I", os.path.join(ROOT, "paper_2410_14117_amd", "csrc"),
                           os.path.join(ROOT, "tests", "serve_book_check.cpp"), "-o", exe,
                           "-lpthread"])
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 exitcode=66",
               ASAN_OPTIONS="halt_on_error=1", UBSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=240, env=env)
    print(r.stdout, r.stderr[-4000:])
    assert r.returncode == 0, r.stderr[-4000:]
    assert "0 failures" in r.stdout and "WARNING" not in r.stderr
