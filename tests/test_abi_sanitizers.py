"""The host side of the C-ABI under the host sanitizers: a copy of the library whose host code
is built with AddressSanitizer and UndefinedBehaviorSanitizer (the device code as usual) is
driven by a sanitized C++ program through configuration validation, the host-only entry
points and the argument checks of the device entry points (tests/abi_sanitize_driver.cpp).
Any invalid access, leak of the library's own or undefined operation fails the test."""
import os
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

CLANG = "/opt/rocm/llvm/bin/clang++"
pytestmark = pytest.mark.skipif(not (os.path.exists(CLANG) and (shutil.which("hipcc") or os.path.exists("/opt/rocm/bin/hipcc"))),
                                reason="the ROCm toolchain is required")

# host code only: each sanitizer flag is scoped to the host compilation
HOST_SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                 "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def test_abi_host_code_under_sanitizers():
    from paper_2411_14413_amd import build as B
    with tempfile.TemporaryDirectory() as tmp:
        objs = []
        for src in B.SOURCES:
            obj = os.path.join(tmp, os.path.splitext(src)[0] + ".o")
            r = subprocess.run([B.hipcc()] + B.FLAGS + HOST_SANITIZE + ["-c", os.path.join(B.CSRC, src), "-o", obj],
                               capture_output=True, text=True)
            assert r.returncode == 0, r.stderr[-3000:]
            objs.append(obj)
        lib = os.path.join(tmp, "libspx.so")
        r = subprocess.run([B.hipcc(), f"--offload-arch={B.ARCH}", "-shared", "-fPIC", "-o", lib] + objs,
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        exe = os.path.join(tmp, "driver")
        r = subprocess.run([CLANG, "-std=c++17", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                            "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "include"),
                            os.path.join(HERE, "abi_sanitize_driver.cpp"), "-L", tmp, "-lspx", f"-Wl,-rpath,{tmp}",
                            "-o", exe], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        # leaks are reported only for the library's own allocations: the HIP runtime it loads
        # keeps process-lifetime state that the sanitizer cannot tell from a leak
        supp = os.path.join(tmp, "lsan.supp")
        open(supp, "w").write("leak:libamdhip64\nleak:libhsa-runtime64\nleak:libamd_comgr\nleak:librocprofiler\n")
        env = dict(os.environ, ASAN_OPTIONS="halt_on_error=1:detect_leaks=1",
                   LSAN_OPTIONS=f"suppressions={supp}:print_suppressions=0",
                   UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
        r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
        assert r.returncode == 0 and r.stdout.strip().endswith("ok"), (r.stdout[-3000:], r.stderr[-4000:])
