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
