"""The oracle and the library's host code under AddressSanitizer and
UndefinedBehaviorSanitizer (CPU only).

The oracle is built with clang and the library with hipcc, whose host half is
instrumented (`-Xarch_host` before each sanitizer flag; the device code is
built as usual and never runs here).  The oracle pins and the C-ABI tests then
run in a child process with the sanitizer runtime preloaded and the two builds
named by APPD_ORACLE_LIB and APPD_LIB; any report stops the child with an
error.  The ABI tests reach the host argument checks, the workspace layout and
the batch plan construction (which ends at its first device copy when no GPU
is present)."""
import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
from paper_2407_07058_amd import _build  # noqa: E402

CLANG = "/opt/rocm/llvm/bin/clang"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SAN = ["-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all",
       "-shared-libsan", "-fno-omit-frame-pointer"]


def runtime():
    libs = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return libs[-1] if libs else None


def build_libraries(out):
    oracle = os.path.join(out, "liboracle_san.so")
    subprocess.run([CLANG, "-std=c11", "-O1", "-g", "-fPIC", "-shared", "-ffp-contract=off", *SAN,
                    "-o", oracle, os.path.join(ROOT, "oracle", "appd_oracle.c"), "-lm"], check=True)
    host_san = [f for flag in SAN for f in ("-Xarch_host", flag)]
    flags = [f for f in _build.HIPCC_FLAGS if f not in ("-shared", "-O3")]
    inc = ["-I", os.path.join(ROOT, "include"), "-I", _build.CSRC]

    def obj(src):
        o = os.path.join(out, src.replace(".hip", ".o"))
        r = subprocess.run([HIPCC, *flags, "-O1", "-g", *host_san, *inc, "-c", "-o", o,
                            os.path.join(_build.CSRC, src)], capture_output=True, text=True)
        if r.returncode:
            raise RuntimeError(r.stderr[-2000:])
        return o

    with ThreadPoolExecutor(min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(obj, _build.SOURCES))
    lib = os.path.join(out, "libappd_san.so")
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", *host_san, "-o", lib, *objs],
                   check=True, capture_output=True)
    return oracle, lib


@pytest.mark.timeout(900)
def test_pins_and_abi_under_asan_ubsan(tmp_path):
    rt = runtime()
    if rt is None or not os.path.exists(CLANG):
        pytest.skip("clang sanitizer runtime not installed")
    oracle, lib = build_libraries(str(tmp_path))
    env = dict(os.environ)
    env.update(LD_PRELOAD=rt, APPD_LIB=lib, APPD_ORACLE_LIB=oracle,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-s", "-m", "not gpu", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                        os.path.join(ROOT, "tests", "test_abi.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=800)
    tail = (r.stdout + r.stderr)[-4000:]
    assert r.returncode == 0, tail
    assert "ERROR: AddressSanitizer" not in tail and "runtime error" not in tail, tail
