"""The host code of the HIP library built with AddressSanitizer (host side
only; device code is compiled as usual) and driven by tests/host_checks.c
through the C ABI: option validation, workspace queries, argument errors,
status strings, and a clean failure of cl_create where no device can be
used.  No GPU is needed; any heap error or leak fails the run."""
import concurrent.futures as cf
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2209_08189_amd", "csrc")
OUT = os.path.join(ROOT, "_build", "asan")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang"

# host-side sanitizer flags only (each -fsanitize= behind -Xarch_host)
HOST_ASAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer"]


def _compile(src):
    obj = os.path.join(OUT, os.path.basename(src)[:-4] + ".o")
    cmd = [HIPCC, "--offload-arch=gfx950", "-O1", "-fPIC", "-std=c++17",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           *HOST_ASAN, "-I", os.path.join(ROOT, "include"), "-c", src, "-o", obj]
    subprocess.run(cmd, check=True, capture_output=True)
    return obj


@pytest.mark.slow
def test_host_code_under_asan():
    if not (os.path.exists(HIPCC) and os.path.exists(CLANG)) or shutil.which("gcc") is None:
        pytest.skip("ROCm toolchain not found")
    os.makedirs(OUT, exist_ok=True)
    srcs = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    lib = os.path.join(OUT, "libclairehip_asan.so")
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", lib, *objs], check=True,
                   capture_output=True)
    exe = os.path.join(OUT, "host_checks")
    subprocess.run([CLANG, "-fsanitize=address", "-g", "-I", os.path.join(ROOT, "include"),
                    os.path.join(HERE, "host_checks.c"), "-L", OUT, "-lclairehip_asan",
                    "-Wl,-rpath," + OUT, "-o", exe], check=True, capture_output=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=23", HIP_VISIBLE_DEVICES="")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    print(r.stdout, r.stderr[-4000:])
    assert r.returncode == 0, r.stderr[-4000:]
    assert "0 failure(s)" in r.stdout
