"""GPU parity of the FP64-storage grids (gsn_create_ex with GSN_C128) against
the FP64 oracle: with psi, the half spectra and every LDS exchange in double
precision, a step rounds nothing below FP64, so the only differences are the
order of the FP64 operations (Stockham radix-16/8/4 against radix-2, table
products against direct cos/sin): ~1e-16 per operation, ~1e-15 per transform.
Bar: relative L2 <= 1e-12 after tens of steps (the complex64 grids' bar is
1e-5), and <= 1e-10 after the 1000 steps of the 256^3 workload."""
import json
import os
import sys

import numpy as np
import pytest

from oracle import oracle as orc
from paper_1909_08354_amd import gsn, inputs

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
import goldens  # noqa: E402

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
REL_L2 = 1e-12


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def lumps(n, seed):
    rng = np.random.default_rng(seed)
    L = tuple(float(v) for v in n)
    w = max(2.0, min(n) / 6.0)
    cs, ws, vs = inputs.random_lumps(rng, n, L, 2, (w, 1.5 * w))
    return inputs.phase_noise(inputs.lumps(n, L, cs, ws, vs), 1e-3, seed + 1), L


def run(n, L, psi0, kern, g, dz, steps, storage=np.complex128, schedule=None, mode=0, chunks=None):
    grid = gsn.Grid(n, L, storage=storage)
    grid.set_kernel(*kern)
    grid.set_coefficients(0.5, g, dz)
    if schedule is not None:
        grid.set_schedule(schedule)
    grid.set_nonlinear_mode(mode)
    grid.set_psi(np.ascontiguousarray(psi0, dtype=np.complex128))
    for c in chunks or [steps]:
        grid.step(c)
    return grid


@pytest.mark.parametrize("n", [(64, 128), (32, 32, 64), (16, 64)])
@pytest.mark.parametrize("schedule,mode", [(0, 0), (1, 1), (4, 0), (3, 1)])
def test_fp64_storage_matches_oracle(n, schedule, mode):
    psi0, L = lumps(n, 41)
    kern, g, dz, steps = (1.0, 0.3, 0.4, 0.05), -0.4, 2e-3, 24
    say("fp64", n, "schedule", schedule, "mode", mode)
    grid = run(n, L, psi0, kern, g, dz, steps, schedule=schedule, mode=mode, chunks=[7, 17])
    ref = orc.evolve(psi0, L, kern, 0.5, g, dz, steps)
    err = orc.rel_l2(grid.get_psi(), ref)
    # the same run on a complex64 grid, for scale
    err64 = orc.rel_l2(run(n, L, psi0, kern, g, dz, steps, storage=np.complex64, schedule=schedule,
                           mode=mode, chunks=[7, 17]).get_psi(), ref)
    say(f"  rel_l2 c128 {err:.3e}   c64 {err64:.3e}")
    assert err < REL_L2
    assert err64 > 1e3 * err
    m = grid.mass()
    ob = orc.observables(ref, L, kern, 0.5, g)
    assert abs(m / ob["mass"] - 1) < 1e-13
    e = grid.energy()
    scale = abs(ob["kinetic"]) + abs(ob["local"]) + abs(ob["nonlocal"])
    for k in ("total", "kinetic", "local", "nonlocal"):
        assert abs(e[k] - ob[k]) < 1e-11 * scale, k


def test_fp64_storage_helmholtz_equation_and_io_dtypes():
    import torch
    n, L = (64, 64), (64.0, 64.0)
    psi0, _ = lumps(n, 42)
    eq = (-0.5, -1.0, 2.5 * (2 * np.pi / 64) ** 2, 0.05)
    grid = gsn.Grid(n, L, storage=np.complex128)
    grid.set_coefficients(0.5, -0.3, 2e-3)
    grid.set_equation(*eq)
    grid.set_psi(torch.from_numpy(psi0).cuda())          # complex128 from the device
    grid.step(20)
    ref = orc.evolve_equation(psi0, L, eq, -0.3, 2e-3, 20)
    assert orc.rel_l2(grid.get_psi(), ref) < REL_L2
    assert orc.rel_l2(grid.get_psi(np.complex128, device=True).cpu().numpy(), ref) < REL_L2
    # complex64 in and out round at the boundary only
    p64 = inputs.to_c64(psi0)
    grid.set_psi(p64)
    assert np.array_equal(grid.get_psi(np.complex64), p64)
    grid.set_psi(torch.from_numpy(p64).cuda())
    assert np.array_equal(grid.get_psi(np.complex128), p64.astype(np.complex128))


def test_fp64_storage_unsupported_calls():
    grid = gsn.Grid((16, 16), (8.0, 8.0), storage=np.complex128)
    with pytest.raises(gsn.GsnError) as ei:
        grid.set_local_terms(-0.5, 1.0, 0.0, 1e-6)
    assert ei.value.status == gsn.GSN_EUNSUPPORTED
    grid.set_local_terms(0.0, 1.0, 0.0, 0.0)   # all zero: the model itself
    grid.set_psi(np.ones((16, 16), np.complex128))
    import torch
    with pytest.raises(gsn.GsnError) as ei:
        grid.potential(torch.empty((16, 16), dtype=torch.float32, device="cuda"))
    assert ei.value.status == gsn.GSN_EUNSUPPORTED


def test_fp64_storage_256_matches_oracle_after_1000_steps():
    """The 256^3 workload from the same complex128(complex64(psi0)) bits as the
    stored 1000-step oracle result, on an FP64-storage grid: the three whole
    central planes element by element, the central x line and the mass."""
    import torch
    rec, ref = goldens.load("gsn3d_256_newton_yukawa")
    w = inputs.WORKLOADS["gsn3d_256_newton_yukawa"]
    grid = gsn.Grid(w["n"], w["L"], storage=np.complex128)
    grid.set_kernel(*w["kern"])
    grid.set_coefficients(w["a"], w["g"], w["dz"])
    dev0 = torch.from_numpy(inputs.as_oracle_input(inputs.gaussian_3d_256())).cuda()
    grid.set_psi(dev0)
    say("fp64 256^3 autotune:", grid.autotune(3))
    grid.set_psi(dev0)
    grid.step(w["steps"])
    out = grid.get_psi(np.complex128, device=True)
    res = goldens.compare(goldens.device_planes(out, rec), ref)
    xl = rec["x_line"]
    ref_line = np.array(xl["re"]) + 1j * np.array(xl["im"])
    got_line = out[xl["z"], xl["y"], :].cpu().numpy()
    del out
    rel_l = np.linalg.norm(got_line - ref_line) / np.linalg.norm(ref_line)
    m = grid.mass()
    drift = abs(m / rec["observables_start"]["mass"] - 1)
    for k, (r, mx) in res.items():
        say(f"fp64 256^3 plane {k}: rel_l2 {r:.3e} max|diff|/max|psi| {mx:.3e}")
    say(f"fp64 256^3: rel_l2 line {rel_l:.3e} drift {drift:.3e}")
    for k, (r, mx) in res.items():
        assert r < 1e-10 and mx < 1e-10, (k, r, mx)
    assert rel_l < 1e-10
    assert drift < 1e-12
