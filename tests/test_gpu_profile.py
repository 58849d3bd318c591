"""Per-pass timing through the C ABI (gsn_profile_passes): it advances the state
bit for bit as gsn_step does, and the kernel durations it reports (a start and
a stop event bound to every dispatch) add up to the wall time of the same
steps, since one stream runs the passes one after another."""
import sys
import time

import numpy as np
import pytest

from paper_1909_08354_amd import gsn, inputs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def make(n, L, psi0, schedule=None):
    grid = gsn.Grid(n, L)
    grid.set_kernel(1.0, 0.3, 0.1, 0.0)
    grid.set_coefficients(0.5, -0.2, 1e-3)
    if schedule is not None:
        grid.set_schedule(schedule)
    grid.set_psi(inputs.to_c64(psi0))
    return grid


@pytest.mark.parametrize("schedule,steps", [(0, 6), (2, 6), (2, 70)])
def test_profile_passes_advances_like_step(schedule, steps):
    """70 steps: more launches than one batch of timing events (256), so the
    events are reused after a synchronisation."""
    n, L = (32, 64, 64), (32.0, 64.0, 64.0)
    rng = np.random.default_rng(3)
    cs, ws, vs = inputs.random_lumps(rng, n, L, 2, (5.0, 8.0))
    psi0 = inputs.lumps(n, L, cs, ws, vs)
    a, b = make(n, L, psi0, schedule), make(n, L, psi0, schedule)
    a.step(steps)
    prof = b.profile_passes(steps)
    say("profile", schedule, {k: round(v, 4) for k, v in prof.items() if v > 0})
    assert np.array_equal(a.get_psi(np.complex64), b.get_psi(np.complex64))
    assert a.mass() == b.mass()
    assert a.phase() == b.phase()
    for name in ("kinetic_y", "kinetic", "x_density", "y_fwd_rho", "kernel", "y_inv_phi",
                 "x_phase"):
        assert prof[name] > 0.0, name
    for name in ("y_fwd_sqrt", "laplacian", "x_source"):
        assert prof[name] == 0.0, name


def test_profile_pass_durations_add_up_to_the_step_time():
    import torch
    n, L = (256, 256, 256), (256.0,) * 3
    grid = gsn.Grid(n, L)
    grid.set_kernel(1.0, 0.3, 0.1, 0.0)
    grid.set_coefficients(0.5, 0.0, 5e-4)
    grid.set_psi(torch.from_numpy(inputs.to_c64(inputs.gaussian_3d_256())).cuda())
    grid.set_schedule(2)
    grid.step(10)
    grid.sync()
    steps = 100
    walls = []
    for _ in range(2):
        t0 = time.perf_counter()
        grid.step(steps)
        grid.sync()
        walls.append(1e3 * (time.perf_counter() - t0) / steps)
    prof = grid.profile_passes(20)
    wall = max(walls)
    steady = sum(v for k, v in prof.items() if k not in ("x_entry_fft", "x_exit_ifft"))
    say(f"256^3: wall {wall:.4f} ms/step, sum of pass kernels {steady:.4f} ms")
    # kernels of one stream do not overlap: their sum stays within the wall
    # time (timer noise aside), and back-to-back launches leave little idle
    assert steady < 1.05 * wall
    assert steady > 0.8 * wall


def test_profile_passes_advances_like_step_with_eq15_terms_and_fields():
    import torch
    n, L = (32, 32, 64), (32.0, 32.0, 64.0)
    psi0 = inputs.fluid_gaussian(n, L, 25.0, 4.0, noise=1e-3, seed=12)
    xs = np.meshgrid(*[inputs.axis_coords(N, Ld) for N, Ld in zip(n, L)], indexing="ij")
    V = torch.from_numpy((0.1 * np.cos(2 * np.pi * xs[2] / L[2])).astype(np.float32)).cuda()
    grids = []
    for _ in range(2):
        grid = gsn.Grid(n, L)
        grid.set_kernel(0.5, 0.0, 0.0, 0.0)
        grid.set_coefficients(0.5, 0.0, 1e-3)
        grid.set_local_terms(-1.02, 1.0, -1.0, 1e-10)
        grid.set_source_fields(None, None, V)
        grid.set_schedule(3)
        grid.set_psi(inputs.to_c64(psi0))
        grids.append(grid)
    grids[0].step(5)
    prof = grids[1].profile_passes(5)
    say("profile eq15", {k: round(v, 4) for k, v in prof.items() if v > 0})
    assert np.array_equal(grids[0].get_psi(np.complex64), grids[1].get_psi(np.complex64))
    for name in ("y_fwd_sqrt", "laplacian", "y_inv_lap", "x_phase", "x_density"):
        assert prof[name] > 0.0, name


def test_profile_passes_advances_like_step_on_fp64_storage():
    n, L = (16, 32, 64), (16.0, 32.0, 64.0)
    rng = np.random.default_rng(5)
    cs, ws, vs = inputs.random_lumps(rng, n, L, 2, (3.0, 5.0))
    psi0 = inputs.lumps(n, L, cs, ws, vs)
    grids = []
    for _ in range(2):
        grid = gsn.Grid(n, L, storage=np.complex128)
        grid.set_kernel(1.0, 0.3, 0.4, 0.0)
        grid.set_coefficients(0.5, -0.2, 1e-3)
        grid.set_psi(psi0)
        grids.append(grid)
    grids[0].step(4)
    prof = grids[1].profile_passes(4)
    assert np.array_equal(grids[0].get_psi(np.complex128), grids[1].get_psi(np.complex128))
    assert grids[0].mass() == grids[1].mass()
    assert prof["kernel"] > 0.0 and prof["x_phase"] > 0.0
