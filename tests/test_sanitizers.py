"""CPU-only sanitizer runs (AddressSanitizer + UndefinedBehaviorSanitizer).

1. The FP64 oracle (oracle/gsn_oracle.c) built with gcc -fsanitize=address,
   undefined and driven through every entry point on small grids
   (tests/host_oracle_check.c), leak detection on.
2. The C ABI's host-side argument validation: the library sources compiled
   for the host only (no device code; an empty device image is embedded, so
   no kernel can run) with the sanitizers on host code, linked to a driver
   (tests/host_abi_check.cpp) that checks every rejection path returns the
   documented status before any HIP call.
Any invalid access, leak (oracle) or undefined behaviour aborts the program.
"""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1909_08354_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/lib/llvm/bin/clang++"
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, (" ".join(cmd), r.stdout[-3000:], r.stderr[-3000:])
    return r


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_address_and_ub_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_check")
    _run(["gcc", "-O1", "-g", "-std=gnu11", "-fopenmp"] + SAN +
         ["-o", exe, os.path.join(HERE, "host_oracle_check.c"), os.path.join(ROOT, "oracle", "gsn_oracle.c"),
          "-lm"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", OMP_NUM_THREADS="2")
    r = _run([exe], env=env, timeout=300)
    assert "fails 0" in r.stdout


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="ROCm compilers not available")
def test_abi_validation_under_address_and_ub_sanitizers(tmp_path):
    empty = tmp_path / "empty.hipfb"
    empty.write_bytes(b"")
    host_san = []
    for f in SAN:
        host_san += ["-Xarch_host", f]

    def compile_one(src):
        obj = str(tmp_path / (os.path.splitext(src)[0] + ".o"))
        _run([HIPCC, "--cuda-host-only", "-O1", "-g", "-std=c++17"] + host_san +
             ["-Xclang", "-fcuda-include-gpubinary", "-Xclang", str(empty),
              "-I" + os.path.join(ROOT, "include"), "-I" + CSRC, "-c", "-o", obj, os.path.join(CSRC, src)],
             timeout=600)
        return obj

    srcs = ["gsn_api.hip", "gsn_batch.hip", "gsn_corrector.hip", "gsn_local.hip", "gsn_c128.hip"]
    with ThreadPoolExecutor(len(srcs)) as ex:
        objs = list(ex.map(compile_one, srcs))
    drv = str(tmp_path / "drv.o")
    _run([CLANG, "-O1", "-g", "-std=c++17"] + SAN + ["-I" + os.path.join(ROOT, "include"), "-c", "-o", drv,
                                                      os.path.join(HERE, "host_abi_check.cpp")])
    exe = str(tmp_path / "abi_check")
    _run([CLANG] + SAN + ["-o", exe, drv] + objs + ["-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1")
    r = _run([exe], env=env, timeout=120)
    assert "fails 0" in r.stdout
