"""The FP64 oracle under AddressSanitizer and UndefinedBehaviorSanitizer:
tests/sanitize/oracle_driver.c calls every oracle entry point (every system
on each lattice of its dimension, odd grid sizes, shifted and unshifted
storage, BGK / TRT / regularized collisions, source and coefficient fields,
the adjoint), built with the oracle's own source as one translation unit.
Any out-of-bounds access, leak or undefined operation aborts the run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_is_clean_under_address_and_undefined_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    build = subprocess.run(
        ["gcc", "-std=gnu11", "-O1", "-g", "-fopenmp", "-ffp-contract=off", "-fno-omit-frame-pointer",
         "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-Wall", "-Wno-unknown-pragmas",
         "-I" + os.path.join(ROOT, "oracle"), os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"),
         "-o", exe, "-lm"], capture_output=True, text=True, timeout=300)
    assert build.returncode == 0, build.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1",
               OMP_NUM_THREADS="2")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stderr[-4000:]
    assert r.stdout.startswith("ok 144 cases"), r.stdout
