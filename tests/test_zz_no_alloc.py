"""gsn_create_static: a grid on the library's static per-device workspace
(no device allocation) gives the same results as gsn_create with a caller
workspace (GPU).  Two grids in a row, the second smaller, so the second runs
on an array that still holds the first one's contents."""
import sys

import numpy as np
import pytest

from paper_1909_08354_amd import gsn, inputs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def run(n, static, steps=25):
    L = tuple(float(v) for v in n)
    rng = np.random.default_rng(31 + len(n))
    cs, ws, vs = inputs.random_lumps(rng, n, L, 3, (min(n) / 8, min(n) / 5))
    psi0 = inputs.to_c64(inputs.lumps(n, L, cs, ws, vs))
    g = gsn.Grid(n, L, static_workspace=static)
    g.set_kernel(1.0, 0.3, 0.2, 0.0)
    g.set_coefficients(0.5, -0.5, 2e-3)
    g.set_psi(psi0)
    g.step(steps)
    out = g.get_psi(np.complex64)
    m = g.mass()
    e = g.energy()
    th = g.phase()
    g.close()
    return out, m, e, th


@pytest.mark.parametrize("n", [(64, 128, 32), (32, 64)])
def test_static_workspace_grid_matches_caller_workspace(n):
    """First a 3-D grid, then a smaller 2-D one on the same static array."""
    say("static-workspace grid", n)
    a = run(n, True)
    b = run(n, False)
    rel = np.linalg.norm(a[0] - b[0]) / np.linalg.norm(b[0])
    say(f"{n}: static vs caller workspace rel_l2 {rel:.3e}")
    assert rel < 1e-5
    assert np.array_equal(a[0], b[0])
    assert a[1] == b[1] and a[3] == b[3]
    assert a[2]["total"] == b[2]["total"]


def test_static_workspace_limits():
    g = gsn.Grid((32, 32), (32.0, 32.0), static_workspace=True)
    try:
        with pytest.raises(gsn.GsnError) as ei:
            gsn.Grid((16, 16), (16.0, 16.0), static_workspace=True)
        assert ei.value.status == gsn.GSN_ESTATE
    finally:
        g.close()
    with pytest.raises(gsn.GsnError) as ei:
        gsn.Grid((512, 512, 64), (512.0, 512.0, 64.0), static_workspace=True)
    assert ei.value.status == gsn.GSN_EWORKSPACE
    g = gsn.Grid((16, 16), (16.0, 16.0), static_workspace=True)   # free again
    g.close()
