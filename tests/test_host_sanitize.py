"""The library's host code and the C oracle under AddressSanitizer and
UndefinedBehaviorSanitizer, on the CPU: every source of the library with the
sanitizers on its host side (the device code is built but never runs), the
oracle's C source, and a driver
(`host_sanitize/driver.cpp`) that calls the host-side entry points and checks
their results against the oracle.  A sanitizer report or a wrong result
fails the test."""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# sanitizers on the host side only
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host",
       "-fno-omit-frame-pointer"]


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(" ".join(cmd) + "\n" + res.stderr[-6000:])


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
def test_host_code_under_asan_and_ubsan(tmp_path):
    import glob
    srcs = sorted(glob.glob(os.path.join(ROOT, "paper_1707_05647_amd", "csrc", "*.hip")))
    inc = ["-I", os.path.join(ROOT, "include")]
    # device code is compiled (the objects need their fat binaries to link)
    # but never runs here, so unoptimised; the sanitizers are host-only
    common = ["--offload-arch=gfx950", "-O1", "-Xarch_device", "-O0", "-g", "-std=c++17", "-fPIC",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *SAN, *inc]

    def compile_one(src):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        _run([HIPCC, *common, "-c", "-o", obj, src])
        return obj

    jobs = max(1, min(8, len(os.sched_getaffinity(0))))
    with ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(compile_one, srcs))
    oracle_obj = str(tmp_path / "oracle.o")
    _run([HIPCC, "-x", "c", "--offload-host-only", "-O1", "-g", "-fPIC", *SAN, "-c", "-o",
          oracle_obj, os.path.join(ROOT, "oracle", "oss_oracle.c")])
    driver_obj = str(tmp_path / "driver.o")
    _run([HIPCC, *common, "-c", "-o", driver_obj,
          os.path.join(ROOT, "tests", "host_sanitize", "driver.cpp")])
    exe = str(tmp_path / "driver")
    _run([HIPCC, "--offload-arch=gfx950", *SAN, "-o", exe, driver_obj, *objs, oracle_obj])
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "halt_on_error=1:abort_on_error=0:detect_leaks=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env.pop("LD_PRELOAD", None)
    res = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    out = res.stdout + res.stderr
    assert res.returncode == 0, out[-6000:]
    assert "all checks passed" in res.stdout
    assert "runtime error" not in out and "AddressSanitizer" not in out
    shutil.rmtree(tmp_path, ignore_errors=True)
