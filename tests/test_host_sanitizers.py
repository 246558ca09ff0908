"""The library's host code (argument validation, size queries, Table 2
coefficients, the workspace carving) built with AddressSanitizer and
UndefinedBehaviorSanitizer on the host side only, driven by
tests/sanitize/host_checks.c.  No GPU: every call is refused on the host or
answers a size query.  The device code is built as usual; the sanitizers
never apply to it."""
import glob
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2207_14589_amd", "csrc")
INCLUDE = os.path.join(ROOT, "include")
DRIVER = os.path.join(ROOT, "tests", "sanitize", "host_checks.c")
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang"
CLANGXX = "/opt/rocm/llvm/bin/clang++"

# each sanitizer flag applies to the host compilation only
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="ROCm toolchain not installed")
def test_host_code_under_asan_and_ubsan(tmp_path):
    objs = []

    def compile_one(src):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        cmd = [HIPCC, "-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-Xclang", "-target-feature",
               "-Xclang", "-packed-fp32-ops", "-Wno-unused-command-line-argument", f"-I{INCLUDE}", *HOST_SAN,
               "-c", src, "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-2000:]
        return obj

    with ThreadPoolExecutor(8) as ex:
        objs = list(ex.map(compile_one, sorted(glob.glob(os.path.join(CSRC, "*.hip")))))
    rt = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
    assert rt, "sanitizer runtime not found"
    rtdir = os.path.dirname(rt[0])
    lib = str(tmp_path / "libsped_san.so")
    san = ["-fsanitize=address,undefined", "-shared-libsan"]
    r = subprocess.run([CLANGXX, "-shared", *san, "-o", lib, *objs, "-L/opt/rocm/lib", "-lamdhip64",
                        "-Wl,-rpath,/opt/rocm/lib"], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    exe = str(tmp_path / "host_checks")
    r = subprocess.run([CLANG, "-g", *san, f"-I{INCLUDE}", DRIVER, "-o", exe, f"-L{tmp_path}", "-lsped_san",
                        f"-Wl,-rpath,{tmp_path}", "-Wl,-rpath,/opt/rocm/lib", f"-Wl,-rpath,{rtdir}"],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-4000:]
    assert out.startswith("ok:"), out[-2000:]
