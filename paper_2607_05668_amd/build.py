"""Build the HIP library ``_lib/liblbm.so`` for gfx950 with hipcc.

Every HIP source is compiled with packed-FP32 instructions disabled
(``-Xclang -target-feature -Xclang -packed-fp32-ops``).  The library is
built in-tree so that it travels with the source tree.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_lib")
LIB = os.path.join(OUT_DIR, "liblbm.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
          "-I" + SRC, "-I" + os.path.join(ROOT, "include")]
DEVICE = ["-x", "hip", "--offload-arch=" + ARCH,
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose: bool = False, jobs: int = 0, out_dir: str = OUT_DIR, defines=()) -> str:
    """Compile the library into out_dir, at most `jobs` translation units at
    a time (0: up to 8, bounded by the CPU count); defines: extra -D tuning
    macros."""
    os.makedirs(out_dir, exist_ok=True)
    lib = os.path.join(out_dir, "liblbm.so")
    jobs = jobs or max(1, min(8, os.cpu_count() or 1))
    units = [(name, True) for name in sorted(os.listdir(SRC)) if name.endswith(".hip")] + [("lbm_api.cpp", True)]
    cmds, objs = [], []
    for name, dev in units:
        obj = os.path.join(out_dir, os.path.splitext(name)[0] + ".o")
        cmds.append([HIPCC] + COMMON + ["-D" + d for d in defines] + (DEVICE if dev else []) +
                    ["-c", os.path.join(SRC, name), "-o", obj])
        objs.append(obj)
    running, failed = [], False
    for cmd in cmds:
        if verbose:
            print(" ".join(cmd), flush=True)
        running.append(subprocess.Popen(cmd))
        while len(running) >= jobs:
            failed |= running.pop(0).wait() != 0
    for p in running:
        failed |= p.wait() != 0
    if failed:
        raise RuntimeError("hipcc failed")
    tmp = lib + ".tmp"
    _run([HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs, verbose)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
