"""Full-size checks of the HIP solver in the benchmark's launch configuration.

256^3 (Newton + Yukawa, 1000 steps): the three whole planes through the grid
centre, element by element, and the central x line against the FP64 oracle's
stored result (tests/golden, written by make_gsn3d_256_golden.py from the
oracle alone), plus mass and energy.
512^3 (8 moving lumps): 20 steps against the stored oracle result
(make_gsn3d_512_golden.py): the three planes through the densest point
(256 x 256 windows), mass and energy, for the autotuned schedule and for each
persistent schedule on every pass; and, over the full 2000 steps, properties
that hold at any size -- norm conservation, time reversibility and bounded
energy drift.
"""
import os
import sys

import numpy as np
import pytest

from paper_1909_08354_amd import gsn, inputs

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
import goldens  # noqa: E402

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))

# the goal's bar for complex64 storage against the FP64 oracle
REL_L2 = 1e-5
# largest pointwise difference per plane, relative to the plane's largest
# |psi|: each pass rounds psi to complex64 (2^-24 relative), and the
# differences after n steps are a sum of about 8n such roundings
MAX_ABS = 2e-5


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def check_planes(tag, grid, rec, ref, rel=REL_L2, mx=MAX_ABS):
    out = grid.get_psi(np.complex64, device=True)
    res = goldens.compare(goldens.device_planes(out, rec), ref)
    del out
    for k, (r, m) in res.items():
        say(f"{tag} plane {k}: rel_l2 {r:.3e} max|diff|/max|psi| {m:.3e}")
    for k, (r, m) in res.items():
        assert r < rel and m < mx, (tag, k, r, m)


def test_gsn3d_256_matches_oracle_after_1000_steps():
    import torch
    rec, ref = goldens.load("gsn3d_256_newton_yukawa")
    w = inputs.WORKLOADS["gsn3d_256_newton_yukawa"]
    assert rec["steps"] == w["steps"] == 1000 and tuple(rec["n"]) == w["n"]
    grid = gsn.Grid(w["n"], w["L"])
    grid.set_kernel(*w["kern"])
    grid.set_coefficients(w["a"], w["g"], w["dz"])
    dev0 = torch.from_numpy(inputs.to_c64(inputs.gaussian_3d_256())).cuda()
    grid.set_psi(dev0)
    say("256^3 autotune:", grid.autotune(5))
    grid.set_psi(dev0)
    grid.step(w["steps"])
    check_planes("256^3", grid, rec, ref)
    out = grid.get_psi(np.complex128, device=True)
    xl = rec["x_line"]
    ref_line = np.array(xl["re"]) + 1j * np.array(xl["im"])
    got_line = out[xl["z"], xl["y"], :].cpu().numpy()
    del out
    rel_l = np.linalg.norm(got_line - ref_line) / np.linalg.norm(ref_line)
    m = grid.mass()
    m_ref0 = rec["observables_start"]["mass"]
    m_ref1 = rec["observables_end"]["mass"]
    e = grid.energy()
    eo = rec["observables_end"]
    scale = abs(eo["kinetic"]) + abs(eo["local"]) + abs(eo["nonlocal"])
    say(f"256^3: rel_l2 line {rel_l:.3e} drift {abs(m / m_ref0 - 1):.3e} "
        f"dE {abs(e['total'] - eo['total']) / scale:.3e}")
    assert rel_l < REL_L2
    assert abs(m / m_ref0 - 1) < 1e-6 and abs(m / m_ref1 - 1) < 1e-6
    assert abs(e["total"] - eo["total"]) < 1e-6 * scale
    assert abs(e["nonlocal"] - eo["nonlocal"]) < 1e-6 * scale
    assert abs(e["kinetic"] - eo["kinetic"]) < 1e-6 * scale


@pytest.mark.parametrize("schedule", ["autotuned", "p16", "p8"])
def test_gsn3d_512_matches_oracle_after_20_steps(schedule):
    """The 512^3 multi-body workload from the stored 20-step oracle result:
    the autotuned schedule (what the benchmark times) and each persistent
    schedule on every pass (several tiles per block on every strided pass)."""
    import torch
    rec, ref = goldens.load("gsn3d_512_lumps")
    w = inputs.WORKLOADS["gsn3d_512_lumps"]
    assert tuple(rec["n"]) == w["n"] and rec["dz"] == w["dz"]
    say(f"512^3 {schedule}: building the lumps")
    dev0 = torch.from_numpy(inputs.lumps_3d(w["n"], w["seed"], 8, dtype=np.complex64)).cuda()
    grid = gsn.Grid(w["n"], w["L"])
    grid.set_kernel(*w["kern"])
    grid.set_coefficients(w["a"], w["g"], w["dz"])
    grid.set_psi(dev0)
    if schedule == "autotuned":
        say("512^3 autotune:", grid.autotune(3))
    else:
        grid.set_schedule(gsn.variant_names().index(schedule))
        grid.set_nonlinear_mode(1)
    grid.set_psi(dev0)
    del dev0
    e0 = grid.energy()
    m0 = grid.mass()
    grid.step(rec["steps"])
    check_planes(f"512^3 {schedule}", grid, rec, ref)
    m = grid.mass()
    e = grid.energy()
    o0, o1 = rec["observables_start"], rec["observables_end"]
    scale = abs(o1["kinetic"]) + abs(o1["local"]) + abs(o1["nonlocal"])
    say(f"512^3 {schedule}: mass {m:.12e} vs {o1['mass']:.12e}, energy {e['total']:.9e} vs "
        f"{o1['total']:.9e}")
    assert abs(m0 / o0["mass"] - 1) < 1e-6 and abs(m / o1["mass"] - 1) < 1e-6
    assert abs(e0["total"] - o0["total"]) < 1e-6 * scale
    for k in ("kinetic", "nonlocal", "total"):
        assert abs(e[k] - o1[k]) < 1e-6 * scale, (k, e[k], o1[k])
    grid.close()


@pytest.mark.parametrize("plain,piped", [(0, 2), (1, 3)])
def test_gsn3d_256_pipelined_passes_match_plain(plain, piped):
    """The persistent prefetching LM passes (p16 / p8: several tiles per
    block at this size) against the one-tile-per-block passes of the same
    radix plan, 20 steps from the same state."""
    import torch
    w = inputs.WORKLOADS["gsn3d_256_newton_yukawa"]
    dev0 = torch.from_numpy(inputs.to_c64(inputs.gaussian_3d_256())).cuda()
    outs = []
    for v in (plain, piped):
        grid = gsn.Grid(w["n"], w["L"])
        grid.set_kernel(*w["kern"])
        grid.set_coefficients(w["a"], w["g"], w["dz"])
        grid.set_schedule(v)
        grid.set_nonlinear_mode(1)
        grid.set_psi(dev0)
        grid.step(20)
        outs.append(grid.get_psi(np.complex64, device=True))
        grid.close()
    diff = torch.max(torch.abs(outs[0] - outs[1])).item()
    top = torch.max(torch.abs(outs[0])).item()
    say(f"256^3 variant {plain} vs {piped}: max |diff| {diff:.3e} of max |psi| {top:.3e}")
    assert diff <= 1e-6 * top


def test_gsn3d_512_lumps_invariants():
    import torch
    w = inputs.WORKLOADS["gsn3d_512_lumps"]
    say("building 512^3 lumps")
    psi0 = inputs.lumps_3d(w["n"], w["seed"], 8, dtype=np.complex64)
    grid = gsn.Grid(w["n"], w["L"])
    grid.set_kernel(*w["kern"])
    grid.set_coefficients(w["a"], w["g"], w["dz"])
    dev0 = torch.from_numpy(psi0).cuda()
    grid.set_psi(dev0)
    say("512^3 autotune:", grid.autotune(3))
    m0 = grid.mass()
    e0 = grid.energy()
    scale = abs(e0["kinetic"]) + abs(e0["local"]) + abs(e0["nonlocal"])
    worst_e = 0.0
    for chunk in range(4):
        grid.step(w["steps"] // 4)
        e = grid.energy()
        worst_e = max(worst_e, abs(e["total"] - e0["total"]) / scale)
    m1 = grid.mass()
    say(f"512^3: drift {abs(m1 / m0 - 1):.3e} worst energy drift {worst_e:.3e}")
    assert abs(m1 / m0 - 1) < 1e-6
    assert worst_e < 1e-5
    # reversibility: 300 steps back with -dz from a state 300 steps in
    grid.set_psi(dev0)
    grid.step(300)
    grid.set_coefficients(w["a"], w["g"], -w["dz"])
    grid.step(300)
    back = grid.get_psi(np.complex64, device=True)
    rel = (torch.linalg.vector_norm((back - dev0).flatten()) / torch.linalg.vector_norm(dev0.flatten())).item()
    say(f"512^3 reversal rel_l2 {rel:.3e}")
    assert rel < 1e-5
