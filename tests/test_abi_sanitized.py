"""The C ABI's host logic under AddressSanitizer and UndefinedBehaviorSanitizer:
lbm_api.cpp rebuilt with host-side instrumentation (device code as usual),
linked with the library's other objects into tests/sanitize/api_driver.cpp,
which creates a handle for every system and lattice and walks the
parameter, storage, reference, sizing and error paths that need no device.
Any out-of-bounds access, leak or undefined operation fails the run."""
import glob
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIBDIR = os.path.join(ROOT, "paper_2607_05668_amd", "_lib")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang++"


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="ROCm compilers not available")
def test_abi_host_code_is_clean_under_address_and_undefined_sanitizers(tmp_path):
    objs = [p for p in glob.glob(os.path.join(LIBDIR, "*.o")) if not p.endswith("lbm_api.o")]
    if not any(p.endswith("kernels.o") for p in objs):
        pytest.skip("library objects not built (run __graft_entry__.build())")
    api = str(tmp_path / "api_san.o")
    cc = subprocess.run(
        [HIPCC, "-O1", "-g", "-std=c++17", "-fPIC", "-I" + os.path.join(ROOT, "paper_2607_05668_amd", "csrc"),
         "-I" + os.path.join(ROOT, "include"), "-x", "hip", "--offload-arch=gfx950",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
         "-Xarch_host", "-fno-omit-frame-pointer",
         "-c", os.path.join(ROOT, "paper_2607_05668_amd", "csrc", "lbm_api.cpp"), "-o", api],
        capture_output=True, text=True, timeout=600)
    assert cc.returncode == 0, cc.stderr[-4000:]
    exe = str(tmp_path / "api_driver")
    ld = subprocess.run(
        [CLANG, "-std=c++17", "-g", "-O1", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
         "-I" + os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "sanitize", "api_driver.cpp"), api]
        + sorted(objs) + ["-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", exe],
        capture_output=True, text=True, timeout=600)
    assert ld.returncode == 0, ld.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stderr[-4000:]
    assert r.stdout.startswith("ok 20 handles"), r.stdout
