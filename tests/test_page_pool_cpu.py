"""CPU unit check of the serving loop's page pool / admission logic (page_pool.h)."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_page_pool(tmp_path):
    exe = str(tmp_path / "page_pool_check")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-Wall", "-fsanitize=address,undefined",
                           "-I", os.path.join(ROOT, "paper_2410_14117_amd", "csrc"),
                           os.path.join(ROOT, "tests", "page_pool_check.cpp"), "-o", exe])
    r = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    print(r.stdout, r.stderr)
    assert r.returncode == 0 and "0 failures" in r.stdout
