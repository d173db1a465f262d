"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The FP64 oracle (oracle/oracle.c) is built with gcc and driven over small and
edge-case shapes with exactly sized buffers (tests/sanitize/oracle_driver.c).
The library's host code (argument checks, plan shapes, bin frequencies, the
batch's job table, the fault-injection paths) is built from every csrc/*.hip
with the sanitizers on the host side only and driven without a GPU
(tests/sanitize/host_driver.cpp).  Objects are cached under
_build/sanitize/<hash of the sources>.
"""
import hashlib
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2108_03948_amd", "csrc")
SAN = os.path.join(ROOT, "tests", "sanitize")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang++"
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def _hash(paths):
    h = hashlib.sha256()
    for p in sorted(paths):
        h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def test_oracle_under_asan_ubsan(tmp_path):
    if not shutil.which("gcc"):
        pytest.skip("gcc missing")
    exe = str(tmp_path / "oracle_san")
    cmd = ["gcc", "-std=gnu11", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", os.path.join(ROOT, "oracle", "oracle.c"),
           os.path.join(SAN, "oracle_driver.c"), "-o", exe, "-lm"]
    subprocess.run(cmd, check=True, capture_output=True)
    r = subprocess.run([exe], env=dict(ENV, ASAN_OPTIONS="detect_leaks=1"), capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0 and "oracle driver: ok" in r.stdout, r.stdout + r.stderr


@pytest.mark.slow
def test_library_host_code_under_asan_ubsan(tmp_path):
    if not (os.path.exists(HIPCC) and os.path.exists(CLANG)):
        pytest.skip("ROCm toolchain missing")
    import torch
    if torch.cuda.is_available():
        pytest.skip("the driver passes stand-in device pointers: CPU only")
    srcs = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hip", ".h"))]
    hips = sorted(p for p in srcs if p.endswith(".hip"))
    drv = os.path.join(SAN, "host_driver.cpp")
    key = _hash(srcs + [drv, os.path.join(ROOT, "include", "thzspec.h")])
    obj_dir = os.path.join(ROOT, "_build", "sanitize", key)
    os.makedirs(obj_dir, exist_ok=True)
    flags = ["-O1", "-g", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-fno-omit-frame-pointer",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}"]

    def compile_one(src):
        obj = os.path.join(obj_dir, os.path.basename(src)[:-4] + ".o")
        if not os.path.exists(obj):
            subprocess.run([HIPCC, *flags, "-c", src, "-o", obj + ".tmp"], check=True, capture_output=True)
            os.replace(obj + ".tmp", obj)
        return obj

    with ThreadPoolExecutor(max_workers=8) as ex:
        objs = list(ex.map(compile_one, hips))
    dobj = str(tmp_path / "host_driver.o")
    subprocess.run([CLANG, "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                    f"-I{os.path.join(ROOT, 'include')}", "-c", drv, "-o", dobj], check=True, capture_output=True)
    exe = str(tmp_path / "host_san")
    subprocess.run([CLANG, "-fsanitize=address,undefined", dobj, *objs, "-L/opt/rocm/lib", "-lamdhip64",
                    "-Wl,-rpath,/opt/rocm/lib", "-o", exe], check=True, capture_output=True)
    r = subprocess.run([exe], env=ENV, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and "host driver: ok" in r.stdout, r.stdout + r.stderr[-4000:]
