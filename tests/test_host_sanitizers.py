"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

constants.cpp, general.cpp and rl0.cpp (the argument checks, the host constants: score
tables of the Gaussian and the general laws, thresholds, c rule, the batched planner's
checks, the bf16 packer, the host validator) are rebuilt with g++
-fsanitize=address,undefined and linked with the unchanged device objects of the normal
build into a second copy of librl0.so.  The host-only tests of tests/test_capi_host.py,
those of tests/test_capi_general.py that do not wait on the oracle (general-law tables,
given tables and their checks) and the checkpoint reader's checks of
tests/test_capi_checkpoint.py then run against that copy (the binding loads the
library named by RL0_LIBRARY) in a child process with the sanitizer runtime preloaded: any
heap or stack overflow, use after free, signed overflow, misaligned or out-of-bounds
access in those paths ends the child with an error.  No GPU is used."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1704_09012_amd", "csrc")
OUT_DIR = os.path.join(ROOT, "_build", "host_sanitize")
HOST_SOURCES = ("constants.cpp", "general.cpp", "rl0.cpp")
DEVICE_OBJECTS = ("kernels.hip", "batched.hip", "mlp.hip", "noalloc.hip")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer"]


def _runtime(name: str) -> str:
    p = subprocess.run(["g++", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else ""


def _build_sanitized() -> str:
    from paper_1704_09012_amd import build as B

    os.makedirs(OUT_DIR, exist_ok=True)
    dev_objs = []
    for src in DEVICE_OBJECTS:
        obj = os.path.join(B.BUILD_DIR, src + ".o")
        if not os.path.exists(obj):
            os.makedirs(B.BUILD_DIR, exist_ok=True)
            obj = B._compile(src)            # the normal hipcc build of that file
        dev_objs.append(obj)
    host_objs = []
    for src in HOST_SOURCES:
        obj = os.path.join(OUT_DIR, src + ".o")
        cmd = ["g++", "-std=c++17", "-O1", "-g", "-fPIC", *SAN, "-D__HIP_PLATFORM_AMD__",
               "-I/opt/rocm/include", "-I" + os.path.join(ROOT, "include"), "-c", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-4000:]
        host_objs.append(obj)
    lib = os.path.join(OUT_DIR, "librl0.so")
    cmd = ["g++", "-shared", *SAN, *host_objs, *dev_objs, "-L/opt/rocm/lib", "-lamdhip64",
           "-Wl,-rpath,/opt/rocm/lib", "-o", lib]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    return lib


@pytest.mark.timeout(900)
def test_host_paths_are_clean_under_asan_and_ubsan():
    if not shutil.which("g++") or not os.path.exists("/opt/rocm/lib/libamdhip64.so"):
        pytest.skip("g++ or the HIP runtime is not installed")
    asan = _runtime("libasan.so")
    if not asan or not _runtime("libubsan.so"):
        pytest.skip("the sanitizer runtimes are not installed")
    lib = _build_sanitized()
    env = dict(os.environ)
    env.update({
        "RL0_LIBRARY": lib,
        "LD_PRELOAD": asan,
        # the Python interpreter and the HIP runtime are not instrumented: their own
        # allocations are not leak-checked
        "ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1:abort_on_error=0",
        "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1",
    })
    probe = ("import os, paper_1704_09012_amd.rl0 as R; R.lib(); "
             "maps = open('/proc/self/maps').read(); "
             "assert R.LIB_PATH == os.environ['RL0_LIBRARY'] and R.LIB_PATH in maps and 'libasan' in maps; "
             "print('sanitized library loaded')")
    r = subprocess.run([sys.executable, "-c", probe], cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and "sanitized library loaded" in r.stdout, r.stdout[-2000:] + r.stderr[-4000:]
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
                        "-k", "not match_the_oracle", os.path.join(ROOT, "tests", "test_capi_host.py"),
                        os.path.join(ROOT, "tests", "test_capi_general.py"),
                        os.path.join(ROOT, "tests", "test_capi_checkpoint.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=800)
    tail = r.stdout[-3000:] + r.stderr[-6000:]
    assert r.returncode == 0, tail
    assert "passed" in r.stdout and "ERROR: AddressSanitizer" not in tail and "runtime error" not in tail, tail
