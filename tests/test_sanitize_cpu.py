"""The seeded generators and the CPU oracle under AddressSanitizer and
UndefinedBehaviorSanitizer (host code only, gcc): tests/sanitize_driver.c
calls every exported C function on small and degenerate inputs; any
out-of-bounds access, leak or undefined behaviour fails the run."""
import os
import shutil
import subprocess

import pytest

from conftest import ROOT


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_generators_and_oracle_under_asan_ubsan(tmp_path):
    exe = tmp_path / "sanitize_driver"
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-o", str(exe),
           os.path.join(ROOT, "tests", "sanitize_driver.c"),
           os.path.join(ROOT, "graphgen", "graphgen.c"),
           os.path.join(ROOT, "oracle", "oracle.c"), "-lm"]
    build = subprocess.run(cmd, capture_output=True, text=True)
    if build.returncode != 0 and "cannot find" in build.stderr and "asan" in build.stderr:
        pytest.skip("the sanitizer runtime libraries are not installed")
    assert build.returncode == 0, build.stderr
    # (verify_asan_link_order=0: the environment may preload other libraries)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert run.returncode == 0, run.stdout + run.stderr
    assert "sanitized driver ok" in run.stdout
