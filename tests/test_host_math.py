"""Host-side checks of device math helpers: the phase passes' FP64 sincos
routines (series after a pi/2 reduction, and the 256-entry table form) are
inline __host__ __device__ functions, compiled here for the CPU from the same
header and compared with libm over every quadrant and large arguments."""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_sincos_fp64_matches_libm(tmp_path):
    exe = tmp_path / "host_sincos"
    subprocess.run([HIPCC, "-O2", "-std=c++17", "--offload-arch=gfx950",
                    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                    "-I" + os.path.join(ROOT, "paper_1909_08354_amd", "csrc"),
                    "-o", str(exe), os.path.join(HERE, "host_sincos.hip")],
                   check=True, capture_output=True)
    rng = np.random.default_rng(3)
    th = np.concatenate([rng.uniform(-8, 8, 4000), rng.uniform(-1e5, 1e5, 2000),
                         [0.0, -0.0, 1e-300, math.pi / 4, -math.pi / 4, math.pi / 2, math.pi,
                          -3 * math.pi / 2, 2 * math.pi, 1.5e6]])
    out = subprocess.run([str(exe)], input="\n".join(repr(float(t)) for t in th),
                         capture_output=True, text=True, check=True).stdout.split("\n")
    sc = np.array([[float(v) for v in line.split()] for line in out if line.strip()])
    assert sc.shape == (th.size, 4)
    for s_col, c_col in ((0, 1), (2, 3)):   # sincos_fp64, then sincos_tab
        assert np.max(np.abs(sc[:, s_col] - np.sin(th))) < 4e-16 * np.maximum(1, np.abs(th) / 1e5).max()
        assert np.max(np.abs(sc[:, c_col] - np.cos(th))) < 4e-16 * np.maximum(1, np.abs(th) / 1e5).max()
        # the nonlinear step must be unitary to FP64 accuracy (no systematic norm drift)
        assert np.max(np.abs(sc[:, s_col] ** 2 + sc[:, c_col] ** 2 - 1)) < 5e-16


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_persistent_queue_decode_and_progress(tmp_path):
    """The batched persistent kernel's item decode equals the phase-by-phase
    definition, every dependency is numbered earlier (no deadlock with items
    handed out in order), and a random in-order scheduler always finishes."""
    exe = tmp_path / "host_queue"
    subprocess.run([HIPCC, "-O2", "-std=c++17", "--offload-arch=gfx950",
                    "-I" + os.path.join(ROOT, "paper_1909_08354_amd", "csrc"),
                    "-o", str(exe), os.path.join(HERE, "host_queue.hip")],
                   check=True, capture_output=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout[-2000:]
    assert "failures 0" in r.stdout


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_log_and_exp_fp64_match_libm(tmp_path):
    """The phase pass's own FP64 ln and exp (series after a 2^e / ln 2
    reduction) against libm, over the dynamic range the pressure term meets."""
    exe = tmp_path / "host_logexp"
    subprocess.run([HIPCC, "-O2", "-std=c++17", "--offload-arch=gfx950",
                    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                    "-I" + os.path.join(ROOT, "paper_1909_08354_amd", "csrc"),
                    "-o", str(exe), os.path.join(HERE, "host_logexp.hip")],
                   check=True, capture_output=True)
    rng = np.random.default_rng(4)
    xl = np.concatenate([10.0 ** rng.uniform(-300, 300, 3000), rng.uniform(0.5, 2.0, 3000),
                         [1.0, 2.0, 0.5, math.sqrt(0.5), math.sqrt(2.0), 1e-300, 5e-324, 1.7e308]])
    out = subprocess.run([str(exe)], input="\n".join(repr(float(t)) for t in xl),
                         capture_output=True, text=True, check=True).stdout.split("\n")
    le = np.array([[float(v) for v in line.split()] for line in out if line.strip()])
    ref = np.log(xl)
    assert np.max(np.abs(le[:, 0] - ref) / np.maximum(1.0, np.abs(ref))) < 4e-16
    assert le[list(xl).index(1.0), 0] == 0.0
    xe = np.concatenate([rng.uniform(-700, 700, 3000), rng.uniform(-1, 1, 3000), [0.0, 1.0, -1.0, 709.0, -745.0]])
    out = subprocess.run([str(exe)], input="\n".join(repr(float(t)) for t in xe),
                         capture_output=True, text=True, check=True).stdout.split("\n")
    ee = np.array([[float(v) for v in line.split()] for line in out if line.strip()])[:, 1]
    refe = np.exp(xe)
    ok = refe > 1e-300
    assert np.max(np.abs(ee[ok] - refe[ok]) / refe[ok]) < 6e-16
    assert ee[list(xe).index(0.0)] == 1.0
    assert np.all(ee[~ok] < 1e-300)
