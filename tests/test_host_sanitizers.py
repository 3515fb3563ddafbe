"""The C ABI's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(host code only; device code is built as usual).  The sanitizer build of the
four library sources takes a few minutes, so the test runs only when
SHG_HOST_SANITIZERS=1:

    SHG_HOST_SANITIZERS=1 python -m pytest tests/test_host_sanitizers.py -v
"""
import concurrent.futures as cf
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2410_04994_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined"]

pytestmark = pytest.mark.skipif(os.environ.get("SHG_HOST_SANITIZERS") != "1",
                                reason="set SHG_HOST_SANITIZERS=1 (builds the library with sanitizers)")


def test_abi_host_code_under_sanitizers(tmp_path):
    common = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-I" + os.path.join(ROOT, "include"),
              "-I" + CSRC, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              "-Wno-unused-command-line-argument", *SAN]

    def compile_one(name):
        obj = str(tmp_path / (name[:-4] + ".o"))
        subprocess.run([HIPCC, *common, "-c", os.path.join(CSRC, name), "-o", obj], check=True,
                       capture_output=True)
        return obj

    srcs = sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))
    with cf.ThreadPoolExecutor(4) as ex:
        objs = list(ex.map(compile_one, srcs))
    exe = str(tmp_path / "abi_harness")
    harness = os.path.join(ROOT, "tests", "sanitize", "abi_harness.c")
    rocm_lib = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "lib")
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-g", *SAN, "-I" + os.path.join(ROOT, "include"),
                    "-x", "c", harness, "-x", "none", *objs, "-o", exe, "-L" + rocm_lib,
                    "-Wl,-rpath," + rocm_lib, "-lrocsolver", "-lrocblas"], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    print(r.stdout, r.stderr[-4000:])
    assert r.returncode == 0, r.stderr[-4000:]
    assert "0 failure(s)" in r.stdout
