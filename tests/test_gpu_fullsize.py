"""Full-size checks of the HIP solver in the benchmark's launch configuration.

256^3 (Newton + Yukawa, 1000 steps): sampled points and the central x line
against the FP64 oracle's stored result (tests/golden, written by
make_gsn3d_256_golden.py from the oracle alone), plus mass and energy.
512^3 (8 moving lumps): properties that hold at any size -- norm
conservation, time reversibility and bounded energy drift -- since the oracle
cannot run 2000 steps of 512^3 in test time.
"""
import json
import os
import sys

import numpy as np
import pytest

from paper_1909_08354_amd import gsn, inputs

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def test_gsn3d_256_matches_oracle_after_1000_steps():
    import torch
    rec = json.load(open(os.path.join(HERE, "golden", "gsn3d_256_newton_yukawa.json")))
    w = inputs.WORKLOADS["gsn3d_256_newton_yukawa"]
    assert rec["steps"] == w["steps"] == 1000 and tuple(rec["n"]) == w["n"]
    grid = gsn.Grid(w["n"], w["L"])
    grid.set_kernel(*w["kern"])
    grid.set_coefficients(w["a"], w["g"], w["dz"])
    grid.set_psi(torch.from_numpy(inputs.to_c64(inputs.gaussian_3d_256())).cuda())
    say("256^3 autotune:", grid.autotune(5))
    grid.step(w["steps"])
    out = grid.get_psi(np.complex128, device=True)
    idx = [tuple(s[0]) for s in rec["samples"]]
    ref = np.array([s[1] + 1j * s[2] for s in rec["samples"]])
    zi, yi, xi = (torch.tensor([i[a] for i in idx], device="cuda") for a in range(3))
    got = out[zi, yi, xi].cpu().numpy()
    xl = rec["x_line"]
    ref_line = np.array(xl["re"]) + 1j * np.array(xl["im"])
    got_line = out[xl["z"], xl["y"], :].cpu().numpy()
    rel_s = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    rel_l = np.linalg.norm(got_line - ref_line) / np.linalg.norm(ref_line)
    m = grid.mass()
    m_ref0 = rec["observables_start"]["mass"]
    m_ref1 = rec["observables_end"]["mass"]
    e = grid.energy()
    eo = rec["observables_end"]
    scale = abs(eo["kinetic"]) + abs(eo["local"]) + abs(eo["nonlocal"])
    say(f"256^3: rel_l2 samples {rel_s:.3e} line {rel_l:.3e} drift {abs(m / m_ref0 - 1):.3e} "
        f"dE {abs(e['total'] - eo['total']) / scale:.3e}")
    assert rel_s < 1e-5 and rel_l < 1e-5
    assert abs(m / m_ref0 - 1) < 1e-6 and abs(m / m_ref1 - 1) < 1e-6
    assert abs(e["total"] - eo["total"]) < 1e-5 * scale
    assert abs(e["nonlocal"] - eo["nonlocal"]) < 1e-5 * scale


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
    assert worst_e < 1e-4
    # reversibility: 300 steps back with -dz from a state 300 steps in
    grid.set_psi(dev0)
    grid.step(300)
    grid.set_coefficients(w["a"], w["g"], -w["dz"])
    grid.step(300)
    back = grid.get_psi(np.complex64, device=True)
    rel = (torch.linalg.vector_norm((back - dev0).flatten()) / torch.linalg.vector_norm(dev0.flatten())).item()
    say(f"512^3 reversal rel_l2 {rel:.3e}")
    assert rel < 1e-5
