"""Build the HIP library (liboss.so) for gfx950 in-tree.

    python -m paper_1707_05647_amd.build

compiles every ``csrc/*.hip`` file with hipcc (one object per file, in
parallel) and links them into ``liboss.so`` next to this file.  The build
always recompiles.
"""
from __future__ import annotations

import glob
import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "liboss.so")
ARCH = os.environ.get("OSS_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # no packed fp32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
]


def sources():
    return sorted(glob.glob(os.path.join(PKG, "csrc", "*.hip")))


def _jobs() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    inc = ["-I", os.path.join(ROOT, "include")]
    work = tempfile.mkdtemp(prefix="oss_build_", dir=PKG)
    try:
        def compile_one(src):
            obj = os.path.join(work, os.path.basename(src) + ".o")
            cmd = [hipcc, *HIPCC_FLAGS, *inc, "-c", "-o", obj, src]
            res = subprocess.run(cmd, capture_output=True, text=True)
            if res.returncode != 0:
                raise RuntimeError(f"hipcc failed on {src}:\n" + res.stderr[-8000:])
            if verbose:
                print(" ".join(cmd))
            return obj

        with ThreadPoolExecutor(_jobs()) as ex:
            objs = list(ex.map(compile_one, sources()))
        fd, tmp = tempfile.mkstemp(suffix=".so", dir=PKG)
        os.close(fd)
        try:
            cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
            res = subprocess.run(cmd, capture_output=True, text=True)
            if res.returncode != 0:
                raise RuntimeError("link failed:\n" + res.stderr[-8000:])
            if verbose:
                print(" ".join(cmd))
            os.chmod(tmp, 0o755)
            os.replace(tmp, LIB)
        finally:
            if os.path.exists(tmp):
                os.unlink(tmp)
    finally:
        shutil.rmtree(work, ignore_errors=True)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
