"""GPU tests of the batched solver (many 2-D instances in one graph).

The grouped launches run the very same tile code as a single grid, so every
instance must equal an independent gsn_grid run with the same schedule bit for
bit; a subset is also checked against the FP64 oracle at the solver's bar.
"""
import sys

import numpy as np
import pytest

from oracle import oracle as orc
from paper_1909_08354_amd import gsn, inputs

pytestmark = pytest.mark.gpu

# batch family order: kinetic, density, kernel, phase, x entry/exit
FAM_TO_PASS = {"kinetic": "kinetic", "x_density": "x_density", "kernel": "kernel",
               "x_phase": "x_phase", "x_fft": ("x_entry_fft", "x_exit_ifft")}


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def grid_schedule(grid, variants):
    names = grid.pass_names()
    v = [0] * len(names)
    for fam, var in zip(gsn.BATCH_FAMILIES, variants):
        targets = FAM_TO_PASS[fam]
        for t in (targets if isinstance(targets, tuple) else (targets,)):
            v[names.index(t)] = var
    return v


def make_instances(shapes, seed, dz=None):
    """dz=None: a different dz per instance (so members of one shape group
    have different kinetic tables); else that dz for all."""
    rng = np.random.default_rng(seed)
    out = []
    for n in shapes:
        L = (float(n[0]), float(n[1]))
        w = max(1.5, min(n) / 6)
        cs, ws, vs = inputs.random_lumps(rng, n, L, int(rng.integers(1, 4)), (w, 1.5 * w))
        kern = (1.0, float(rng.uniform(0, 1)), float(rng.uniform(0.05, 0.5)), 0.0)
        ddz = float(rng.uniform(1e-3, 3e-3))
        out.append(dict(n=n, L=L, kern=kern, a=0.5, g=-0.5, dz=ddz if dz is None else dz,
                        psi=inputs.lumps(n, L, cs, ws, vs)))
    return out


SHAPES = [(32, 32), (64, 32), (32, 32), (16, 64), (64, 32), (128, 128), (32, 32)]


@pytest.mark.parametrize("variants,nlmode,dz,grid_variants", [
    ((0, 0, 0, 1, 0), 0, None, None), ((1, 1, 1, 0, 1), 1, None, None),
    # persistent grouped passes (one table set per shape group)
    ((2, 2, 2, 3, 0), 1, 2e-3, None), ((3, 3, 3, 2, 1), 0, 1.5e-3, None),
    # persistent variants asked for, but the members' tables differ: the
    # group runs the one-tile-per-block passes of the same radix plan
    ((2, 3, 2, 3, 0), 1, None, (0, 1, 0, 1, 0))])
def test_batch_equals_independent_grids(variants, nlmode, dz, grid_variants):
    inst = make_instances(SHAPES, 5, dz)
    b = gsn.Batch([d["n"] for d in inst], [d["L"] for d in inst])
    b.set_schedule(list(variants), nlmode)
    for i, d in enumerate(inst):
        b.set(i, d["kern"], d["a"], d["g"], d["dz"], inputs.to_c64(d["psi"]))
    steps = 17
    b.step(steps)
    masses = b.masses()
    for i, d in enumerate(inst):
        say("instance", i, d["n"])
        g = gsn.Grid(d["n"], d["L"])
        g.set_kernel(*d["kern"])
        g.set_coefficients(d["a"], d["g"], d["dz"])
        g.set_schedule(grid_schedule(g, grid_variants or variants))
        g.set_nonlinear_mode(nlmode)
        g.set_psi(inputs.to_c64(d["psi"]))
        g.step(steps)
        assert np.array_equal(b.get(i, np.complex64), g.get_psi(np.complex64))
        assert b.phase(i) == g.phase()
        assert masses[i] == g.mass()
        if i < 3:
            ref = orc.evolve(inputs.as_oracle_input(d["psi"]), d["L"], d["kern"], d["a"], d["g"],
                             d["dz"], steps)
            assert orc.rel_l2(b.get(i), ref) < 1e-5


def test_batch_autotune_keeps_states_and_matches_independent_grids():
    """gsn_batch_autotune picks a schedule per shape group; the instances'
    states are unchanged by it, and afterwards every instance equals an
    independent gsn_grid run with its group's tuned schedule bit for bit,
    and a subset matches the FP64 oracle at the solver's bar."""
    inst = make_instances(SHAPES, 11, 2e-3)
    b = gsn.Batch([d["n"] for d in inst], [d["L"] for d in inst])
    for i, d in enumerate(inst):
        b.set(i, d["kern"], d["a"], d["g"], d["dz"], inputs.to_c64(d["psi"]))
    b.step(3)
    before = [b.get(i, np.complex64) for i in range(len(inst))]
    ph_before = [b.phase(i) for i in range(len(inst))]
    b.autotune(2)
    for i in range(len(inst)):
        assert np.array_equal(b.get(i, np.complex64), before[i])
        assert b.phase(i) == ph_before[i]
    scheds = {}
    for i, d in enumerate(inst):
        scheds.setdefault(d["n"], b.schedule(i))
        assert b.schedule(i) == scheds[d["n"]]
    say("tuned batch schedules:", scheds)
    for i, d in enumerate(inst):
        b.set(i, d["kern"], d["a"], d["g"], d["dz"], inputs.to_c64(d["psi"]))
    steps = 17
    b.step(steps)
    masses = b.masses()
    for i, d in enumerate(inst):
        variants, nlmode = b.schedule(i)
        g = gsn.Grid(d["n"], d["L"])
        g.set_kernel(*d["kern"])
        g.set_coefficients(d["a"], d["g"], d["dz"])
        g.set_schedule(grid_schedule(g, variants))
        g.set_nonlinear_mode(nlmode)
        g.set_psi(inputs.to_c64(d["psi"]))
        g.step(steps)
        assert np.array_equal(b.get(i, np.complex64), g.get_psi(np.complex64)), (i, d["n"], variants)
        assert b.phase(i) == g.phase()
        assert masses[i] == g.mass()
        g.close()
        if i < 3:
            ref = orc.evolve(inputs.as_oracle_input(d["psi"]), d["L"], d["kern"], d["a"], d["g"],
                             d["dz"], steps)
            assert orc.rel_l2(b.get(i), ref) < 1e-5


def test_batch_autotune_needs_every_state():
    inst = make_instances(SHAPES[:2], 3, 2e-3)
    b = gsn.Batch([d["n"] for d in inst], [d["L"] for d in inst])
    b.set(0, inst[0]["kern"], 0.5, -0.5, 2e-3, inputs.to_c64(inst[0]["psi"]))
    with pytest.raises(gsn.GsnError) as ei:
        b.autotune(1)
    assert ei.value.status == gsn.GSN_ESTATE


def test_graph_replays_and_direct_mode_agree():
    """Several replays of one captured graph, with eager work in between, equal
    the same steps issued as direct launches."""
    inst = make_instances(SHAPES[:4], 9)
    res = []
    for mode in (0, 2):
        b = gsn.Batch([d["n"] for d in inst], [d["L"] for d in inst])
        b.set_mode(mode)
        for i, d in enumerate(inst):
            b.set(i, d["kern"], d["a"], d["g"], d["dz"], inputs.to_c64(d["psi"]))
        snaps = []
        for _ in range(3):
            b.step(6)
            snaps.append([b.get(i, np.complex64) for i in range(len(inst))])
            b.masses()
        res.append(snaps)
    for r0, r1 in zip(*res):
        for a, c in zip(r0, r1):
            assert np.array_equal(a, c)
    assert not np.array_equal(res[0][0][0], res[0][1][0])


def test_batch_sweep_64_full_size():
    """The 64-instance sweep of 256^2/512^2/1024^2 grids, 500 steps: norm
    conservation for all, bitwise equality with single grids for one instance
    per size, and the first 20 steps of one instance per size vs the oracle."""
    w = inputs.WORKLOADS["gsn2d_batch64_sweep"]
    inst = inputs.batch_sweep(w["count"], w["seed"], w["sizes"])
    b = gsn.Batch([d["n"] for d in inst], [d["L"] for d in inst])
    sched = (2, 3, 2, 3, 0)   # the default: persistent passes, stored real-space psi
    b.set_schedule(list(sched), 1)
    for i, d in enumerate(inst):
        b.set(i, d["kern"], d["a"], d["g"], d["dz"], inputs.to_c64(d["psi"]))
    m0 = b.masses()
    b.step(w["steps"])
    m1 = b.masses()
    drift = np.max(np.abs(m1 / m0 - 1))
    say(f"batch 64 x 500 steps: worst norm drift {drift:.3e}")
    assert drift < 1e-6
    firsts = {}
    for i, d in enumerate(inst):
        firsts.setdefault(d["n"], i)
    for n, i in sorted(firsts.items()):
        d = inst[i]
        say("check instance", i, n)
        g = gsn.Grid(d["n"], d["L"])
        g.set_kernel(*d["kern"])
        g.set_coefficients(d["a"], d["g"], d["dz"])
        g.set_schedule(grid_schedule(g, sched))
        g.set_nonlinear_mode(1)
        g.set_psi(inputs.to_c64(d["psi"]))
        g.step(w["steps"])
        assert np.array_equal(b.get(i, np.complex64), g.get_psi(np.complex64))
        g.set_psi(inputs.to_c64(d["psi"]))
        g.step(20)
        ref = orc.evolve(inputs.as_oracle_input(d["psi"]), d["L"], d["kern"], d["a"], d["g"], d["dz"], 20)
        assert orc.rel_l2(g.get_psi(), ref) < 1e-5


PSHAPES = [(128, 128), (256, 128), (128, 256), (256, 256), (128, 128), (512, 256)]


@pytest.mark.parametrize("nlmode", [0, 1])
def test_persistent_mode_matches_graph_mode(nlmode):
    """The persistent work-queue kernel runs the same per-line arithmetic as the
    grouped launches with x passes at 8 and y passes at 16 points per thread."""
    inst = make_instances(PSHAPES, 21)
    outs = []
    for mode in (0, 1):
        b = gsn.Batch([d["n"] for d in inst], [d["L"] for d in inst])
        b.set_schedule([0, 1, 0, 1, 1], nlmode)
        for i, d in enumerate(inst):
            b.set(i, d["kern"], d["a"], d["g"], d["dz"], inputs.to_c64(d["psi"]))
        b.set_mode(mode)
        b.step(13)
        b.step(4)
        outs.append([b.get(i) for i in range(len(inst))])
    for i, (x, y) in enumerate(zip(*outs)):
        assert orc.rel_l2(y, x) < 1e-12, i
    d = inst[1]
    ref = orc.evolve(inputs.as_oracle_input(d["psi"]), d["L"], d["kern"], d["a"], d["g"], d["dz"], 17)
    assert orc.rel_l2(outs[1][1], ref) < 1e-5


def test_persistent_queue_error_is_reported():
    inst = make_instances(PSHAPES[:3], 22)
    b = gsn.Batch([d["n"] for d in inst], [d["L"] for d in inst])
    for i, d in enumerate(inst):
        b.set(i, d["kern"], d["a"], d["g"], d["dz"], inputs.to_c64(d["psi"]))
    b.set_mode(1)
    b.set_queue_limits(fail_item=40)
    b.step(3)
    with pytest.raises(gsn.GsnError) as ei:
        b.sync()
    assert ei.value.status == gsn.GSN_EHIP
    # the next run without the hook completes normally
    b.set_queue_limits(fail_item=-1)
    for i, d in enumerate(inst):
        b.set(i, d["kern"], d["a"], d["g"], d["dz"], inputs.to_c64(d["psi"]))
    b.step(3)
    b.sync()
