"""GPU parity of the position-dependent coupling (Eq. (9)-(12)): the source
s = gamma rho + beta lap(rho) that the kernel acts on, the static potential
V_ext, and the non-minimal-coupling fields, against the FP64 oracle through
the C ABI.  The oracle is given the same float32 field values the GPU reads.
Bar: relative L2 <= 1e-5."""
import sys

import numpy as np
import pytest

from oracle import oracle as orc
from paper_1909_08354_amd import gsn, inputs

pytestmark = pytest.mark.gpu

REL_L2 = 1e-5


def say(*a):
    print(*a, file=sys.stderr, flush=True)


SHAPES = {"2d": ((64, 128), (32.0, 64.0)), "3d": ((32, 32, 64), (32.0, 32.0, 64.0))}


def smooth_fields(n, L, seed):
    rng = np.random.default_rng(seed)
    xs = np.meshgrid(*[inputs.axis_coords(N, Ld) for N, Ld in zip(n, L)], indexing="ij")
    def wave(amp, base):
        m = [int(v) for v in rng.integers(1, 3, len(n))]
        ph = rng.uniform(0, 2 * np.pi)
        return (base + amp * np.cos(sum(2 * np.pi * mi * x / Ld for mi, x, Ld in zip(m, xs, L)) + ph)).astype(np.float32)
    return wave(0.3, 0.7), wave(0.4, 0.1), wave(0.5, 0.0)


def dev(a):
    import torch
    return None if a is None else torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def host64(a):
    return None if a is None else np.asarray(a.cpu().numpy() if hasattr(a, "cpu") else a, dtype=np.float64)


CASES = {
    "gamma": (True, False, False, None),
    "beta": (False, True, False, None),
    "gamma_beta": (True, True, False, None),
    "V": (False, False, True, None),
    "all_eq15": (True, True, True, (-0.5, 1.0, -1.0, 1e-10)),
}


@pytest.mark.parametrize("shape", ["2d", "3d"])
@pytest.mark.parametrize("case", list(CASES))
def test_source_fields_match_oracle(shape, case):
    use_g, use_b, use_v, local = CASES[case]
    n, L = SHAPES[shape]
    psi0 = inputs.fluid_gaussian(n, L, 25.0, 4.0, seed=12)
    gm, bt, V = smooth_fields(n, L, 3)
    gm, bt, V = (f if u else None for f, u in zip((gm, bt, V), (use_g, use_b, use_v)))
    kern, g, dz, steps = (0.8, 0.0, 0.0, 0.0), -0.2, 1e-3, 20
    say("fields", case, shape)
    grid = gsn.Grid(n, L)
    grid.set_kernel(*kern)
    grid.set_coefficients(0.5, g, dz)
    if local:
        grid.set_local_terms(*local)
    grid.set_source_fields(dev(gm), dev(bt), dev(V))
    grid.set_psi(inputs.to_c64(psi0))
    grid.step(8)
    grid.step(12)
    ref = orc.evolve_fields(inputs.as_oracle_input(psi0), L, kern, 0.5, g, dz, steps,
                            (host64(gm), host64(bt), host64(V)), local=local)
    err = orc.rel_l2(grid.get_psi(), ref)
    say(f"  rel_l2 {err:.3e}")
    assert err < REL_L2
    # the fields changed the evolution
    plain = orc.evolve(inputs.as_oracle_input(psi0), L, kern, 0.5, g, dz, steps, local=local)
    assert orc.rel_l2(ref, plain) > 1e-4


@pytest.mark.parametrize("schedule,mode", [(1, 0), (4, 1), (3, 1), (2, 0)])
def test_source_fields_all_schedules(schedule, mode):
    n, L = SHAPES["3d"]
    psi0 = inputs.fluid_gaussian(n, L, 25.0, 4.0, seed=13)
    gm, bt, V = smooth_fields(n, L, 4)
    kern, dz, steps = (0.8, 0.0, 0.0, 0.0), 1e-3, 12
    grid = gsn.Grid(n, L)
    grid.set_kernel(*kern)
    grid.set_coefficients(0.5, 0.0, dz)
    grid.set_source_fields(dev(gm), dev(bt), dev(V))
    grid.set_schedule(schedule)
    grid.set_nonlinear_mode(mode)
    grid.set_psi(inputs.to_c64(psi0))
    grid.step(steps)
    ref = orc.evolve_fields(inputs.as_oracle_input(psi0), L, kern, 0.5, 0.0, dz, steps,
                            (host64(gm), host64(bt), host64(V)))
    assert orc.rel_l2(grid.get_psi(), ref) < REL_L2


@pytest.mark.parametrize("shape", ["2d", "3d"])
def test_nmc_fields_match_oracle(shape):
    n, L = SHAPES[shape]
    grid = gsn.Grid(n, L)
    c = [1.5 * (i + 1) for i in range(len(n))]
    for lam in (1.0, 2.5):
        got = [host64(f) for f in grid.nmc_fields(lam, 1.9, 1.3, center=c)]
        ref = orc.nmc_fields(n, L, lam, 1.9, 1.3, center=c)
        for a, b in zip(got, ref):
            assert np.max(np.abs(a - b)) <= 2e-7 * np.max(np.abs(b)) + 1e-30


def test_clearing_fields_restores_the_model_and_unsupported_calls():
    n, L = SHAPES["2d"]
    psi0 = inputs.fluid_gaussian(n, L, 25.0, 4.0, seed=14)
    gm, bt, V = smooth_fields(n, L, 5)
    outs = []
    for with_fields in (False, True):
        grid = gsn.Grid(n, L)
        grid.set_kernel(0.8, 0.0, 0.0, 0.0)
        grid.set_coefficients(0.5, -0.2, 1e-3)
        if with_fields:
            keep = (dev(gm), dev(bt), dev(V))
            grid.set_source_fields(*keep)
            with pytest.raises(gsn.GsnError) as ei:
                grid.energy()
            assert ei.value.status == gsn.GSN_EUNSUPPORTED
            grid.set_kernel(0.8, 0.2, 0.5, 0.0)          # K(0) != 0 with a source field
            grid.set_psi(inputs.to_c64(psi0))
            with pytest.raises(gsn.GsnError) as ei:
                grid.step(1)
            assert ei.value.status == gsn.GSN_EUNSUPPORTED
            grid.set_kernel(0.8, 0.0, 0.0, 0.0)
            grid.set_source_fields(None, None, None)
        grid.set_psi(inputs.to_c64(psi0))
        grid.step(9)
        outs.append(grid.get_psi(np.complex64))
    assert np.array_equal(outs[0], outs[1])


def test_nmc_256_full_size_matches_oracle():
    """The 256^3 fluid under the non-minimal coupling with the Eq. (15) local
    terms (the paper's model), in the benchmark's configuration: 3 steps against
    the oracle on the whole grid, and mass conservation over 200 steps."""
    import torch
    w = inputs.WORKLOADS["gsn3d_256_nmc"]
    psi0 = inputs.fluid_gaussian(w["n"], w["L"], w["mass"], w["waist"], seed=w["seed"])
    dev0 = torch.from_numpy(inputs.to_c64(psi0)).cuda()
    grid = gsn.Grid(w["n"], w["L"])
    grid.set_kernel(*w["kern"])
    grid.set_coefficients(w["a"], w["g"], w["dz"])
    grid.set_local_terms(*w["local"])
    nm = w["nmc"]
    fields = grid.nmc_fields(nm["lam"], nm["r0"], nm["nu"])
    grid.set_source_fields(*fields)
    grid.set_psi(dev0)
    say("nmc 256^3 autotune:", grid.autotune(3))
    grid.set_psi(dev0)
    grid.step(3)
    out = grid.get_psi(np.complex128)
    say("nmc 256^3: oracle 3 steps")
    ref = orc.evolve_fields(inputs.as_oracle_input(psi0), w["L"], w["kern"], w["a"], w["g"], w["dz"], 3,
                            tuple(host64(f) for f in fields), local=w["local"])
    err = orc.rel_l2(out, ref)
    say(f"nmc 256^3: rel_l2 {err:.3e}")
    assert err < REL_L2
    m0 = grid.mass()
    grid.step(w["steps"] - 3)
    drift = abs(grid.mass() / m0 - 1)
    say(f"nmc 256^3: norm drift over {w['steps']} steps {drift:.3e}")
    assert drift < 1e-6


@pytest.mark.parametrize("shape", ["2d", "3d"])
def test_static_potential_energy_matches_oracle(shape):
    """With V_ext alone the energy stays the Hamiltonian: its local part holds
    -dV sum V rho (with the Eq. (15) terms on as well)."""
    n, L = SHAPES[shape]
    psi0 = inputs.fluid_gaussian(n, L, 25.0, 4.0, seed=15)
    _, _, V = smooth_fields(n, L, 6)
    kern, g, local = (0.8, 0.2, 0.4, 0.0), -0.2, (-0.5, 1.0, -1.0, 1e-10)
    grid = gsn.Grid(n, L)
    grid.set_kernel(*kern)
    grid.set_coefficients(0.5, g, 1e-3)
    grid.set_local_terms(*local)
    keep = dev(V)
    grid.set_source_fields(None, None, keep)
    grid.set_psi(inputs.to_c64(psi0))
    grid.step(6)
    psi = grid.get_psi()
    e = grid.energy()
    eo = orc.observables(psi, L, kern, 0.5, g, local=local, V=host64(V))
    scale = abs(eo["kinetic"]) + abs(eo["local"]) + abs(eo["nonlocal"])
    for k in ("total", "kinetic", "local", "nonlocal"):
        assert abs(e[k] - eo[k]) < 1e-6 * scale, k
    ref = orc.evolve_fields(inputs.as_oracle_input(psi0), L, kern, 0.5, g, 1e-3, 6, (None, None, host64(V)),
                            local=local)
    assert orc.rel_l2(psi, ref) < REL_L2


def test_field_counts_are_checked():
    import ctypes
    n, L = SHAPES["2d"]
    grid = gsn.Grid(n, L)
    f = dev(np.ones(n, np.float32))
    lib = gsn.load()
    P = int(np.prod(n))
    assert lib.gsn_set_source_fields(grid.h, ctypes.c_void_p(f.data_ptr()), None, None, P - 1) == gsn.GSN_EINVAL
    assert lib.gsn_set_source_fields(grid.h, None, None, None, 0) == gsn.GSN_OK
    assert lib.gsn_nmc_fields(grid.h, 1.0, 2.0, 1.0, None, 0.5, ctypes.c_void_p(f.data_ptr()), None, None,
                              P - 1) == gsn.GSN_EINVAL
