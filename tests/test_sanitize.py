"""The input generators and every oracle routine under AddressSanitizer and
UndefinedBehaviorSanitizer (host code only): ``sanitize_driver.c`` runs
them over generated, degenerate and invalid inputs; the sanitizers abort on
any out-of-bounds access, use after free, leak, overflow or other undefined
behaviour, and the driver exits non-zero on an unexpected result."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SOURCES = [os.path.join(ROOT, "tests", "sanitize_driver.c"),
           os.path.join(ROOT, "oracle", "oracle.c"),
           os.path.join(ROOT, "paper_1508_03619_amd", "inputs", "gen.c")]


def test_oracle_and_generators_under_asan_ubsan(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no gcc")
    exe = str(tmp_path / "sanitize_driver")
    cmd = [gcc, "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-fopenmp",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-Wall", "-Wextra",
           "-Werror", *SOURCES, "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "asan" in r.stderr.lower() and "cannot find" in r.stderr.lower():
        pytest.skip("the sanitizer runtime is not installed")
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="4")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert "all checks passed" in r.stdout
