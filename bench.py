#!/usr/bin/env python3
"""Benchmark of the split-step Schroedinger-Newton hot path on one MI355X.

Headline workload: one 3-D instance on a 512^3 periodic grid (dx = 1),
complex64 storage with FP64 arithmetic, 8 Gaussian lumps (waist U[4,10],
seeded centres and phase-gradient velocities), Newtonian kernel plus a Yukawa
correction 0.3/(k^2 + 0.1^2), g = 0, dz = 2.5e-4.  A "step" is one symmetric
split step over the whole grid (8 HBM passes).  The timed region is one
gsn_step(K) call with psi already resident in HBM.

Prints ONE JSON line.  Besides throughput it reports the dominant pass's
roofline (algorithmic bytes / HIP-event duration on the solver's stream), the
step's HBM fraction on the method's pass model (104 B per point), the norm and
energy drift of the timed run, and secondary legs: the 256^3 single grid, the
FP64-storage grid, the Eq. (15) fluids, the batched sweep and the learned
corrector; last, the FP64 CPU oracle timed on a bounded sample on this host
(a baseline, not a target).
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
# the headline workload (the largest single-GPU configuration: 8 moving lumps
# on 512^3) and the secondary single-grid leg (a centred cloud on 256^3)
WORKLOAD = "gsn3d_512_lumps"
WORKLOAD_256 = "gsn3d_256_newton_yukawa"
# bytes per grid point of one 3-D step in the pass model of the method
# (8 HBM passes: reads 56 + writes 48)
MODEL_BPP = 104.0


# the sources of the single-grid passes (the batched and corrector files do
# not change them)
PASS_SOURCES = ("gsn_api.hip", "gsn_fft.hpp", "gsn_host.hpp", "gsn_kernels.hpp")


# the Eq. (15) and coupling-field legs also run the kernels of gsn_local.hip,
# the FP64-storage leg those of gsn_c128.hip
LEG_SOURCES = PASS_SOURCES + ("gsn_local.hip", "gsn_c128.hip")
FP64_LEG = "gsn3d_256_newton_yukawa:c128"


def csrc_hash(files=PASS_SOURCES):
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1909_08354_amd", "csrc")
    for f in files:
        with open(os.path.join(d, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel_pass, variant, workload, mode=None):
    """HBM bytes per launch of a pass in a schedule variant (and, for the
    density and phase passes, nonlinear mode) on a workload, from committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE runs (profiles/traffic.json), only when
    they were taken on the current kernel sources; else None."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    try:
        rec = json.load(open(p))
    except ValueError:
        return None
    if rec.get("csrc_hash") != csrc_hash():
        return None
    by_variant = rec.get("workloads", {}).get(workload, {}).get("passes", {}).get(kernel_pass, {})
    b = by_variant.get(f"{variant}:m{mode}", by_variant.get(variant))
    if b is None:
        return None
    return {"bytes": b, "source": "rocprofv3 FETCH_SIZE x %.3g + WRITE_SIZE x %.3g per launch, "
            "committed in profiles/traffic.json for these kernel sources (hash %s), not re-measured "
            "in this run" % (rec["calibration"]["fetch_factor"], rec["calibration"]["write_factor"],
                             rec["csrc_hash"])}


def measured_leg_traffic(workload, kernel_pass, variant):
    """The same for a pass of the Eq. (15) / coupling-field legs."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    try:
        rec = json.load(open(p))
    except ValueError:
        return None
    legs = rec.get("legs", {})
    if legs.get("legs_hash") != csrc_hash(LEG_SOURCES):
        return None
    return legs.get(workload, {}).get(kernel_pass, {}).get(variant)


def progress(msg):
    """One line on stderr as each leg ends (the JSON line stays alone on stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo) and logical CPU count."""
    name = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    name = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": name, "logical_cpus": os.cpu_count()}


def oracle_step_rate(w, psi0_c128, nthreads):
    """Oracle step rate with nthreads threads: evolve(1) and evolve(2) on the
    same input; the difference is one merged step without table setup."""
    from oracle import oracle as orc
    args = (w["L"], w["kern"], w["a"], w["g"], w["dz"])
    t0 = time.perf_counter()
    orc.evolve(psi0_c128, *args, 1, nthreads=nthreads)
    t1 = time.perf_counter()
    orc.evolve(psi0_c128, *args, 2, nthreads=nthreads)
    t2 = time.perf_counter()
    per_step = max((t2 - t1) - (t1 - t0), 1e-9)
    return int(np.prod(w["n"])) / per_step


def cpu_baseline(legs):
    """The FP64 oracle's step rate on this host (a baseline, not a target).
    legs: (name, workload dict, complex128 input, thread counts); the first
    leg at its first thread count is the headline figure.  The thread share
    is OMP_NUM_THREADS when set (the GPU host's share), else every logical CPU."""
    share = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1)
    out = dict(cpu_model())
    out["thread_share"] = share
    runs = []
    for name, w, psi, threads in legs:
        for nt in threads:
            nt = share if nt == 0 else nt
            t0 = time.perf_counter()
            rate = oracle_step_rate(w, psi, nt)
            runs.append({"workload": name, "threads": nt, "value": rate,
                         "unit": "grid-pt updates/s", "seconds": time.perf_counter() - t0})
            progress(f"oracle {name} with {nt} threads: {rate:.3e} grid-pt updates/s")
    head = runs[0]
    out.update({"value": head["value"], "unit": "grid-pt updates/s", "cores": head["threads"],
                "kind": "oracle",
                "sample": f"one merged step of {head['workload']} (evolve(2) - evolve(1)) "
                          f"with {head['threads']} threads; the other runs listed in 'runs'",
                "runs": runs})
    return out


def single_grid_leg(name, psi0, steps, warmup, autotune_iters, profile_steps, traffic=True):
    """One grid of a workload: autotune, warm up, time gsn_step(steps) with psi
    resident in HBM, then the per-pass kernel durations (HIP events bound to
    each dispatch on the solver's stream) for the dominant pass's roofline,
    and the norm and energy drift of the timed run."""
    import torch
    from paper_1909_08354_amd import gsn, inputs
    w = inputs.WORKLOADS[name]
    n, L = w["n"], w["L"]
    P = int(np.prod(n))
    grid = gsn.Grid(n, L)
    grid.set_kernel(*w["kern"])
    grid.set_coefficients(w["a"], w["g"], w["dz"])
    dev0 = torch.from_numpy(psi0).cuda()
    grid.set_psi(dev0)
    schedule = grid.autotune(autotune_iters) if autotune_iters > 0 else grid.schedule()
    grid.set_psi(dev0)
    del dev0
    m0 = grid.mass()
    e0 = grid.energy()
    if warmup:
        grid.step(warmup)
    grid.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    grid.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    grid.sync()
    elapsed = t1 - t0
    m1 = grid.mass()
    e1 = grid.energy()
    ms_per_step = 1e3 * elapsed / steps
    prof = grid.profile_passes(profile_steps)
    bpp = dict(zip(grid.pass_names(), grid.pass_bytes_per_point()))
    steady = {k: v for k, v in prof.items() if k not in ("x_entry_fft", "x_exit_ifft")}
    dom = max(steady, key=steady.get)
    achieved = bpp[dom] * P / (steady[dom] * 1e-3) / 1e9
    executed = sum(bpp[k] for k in steady)
    scale = abs(e0["kinetic"]) + abs(e0["local"]) + abs(e0["nonlocal"])
    mode = grid.nonlinear_mode()
    grid.close()
    tr = measured_traffic(dom, schedule.get(dom), name, mode) if traffic else None
    return {
        "workload": name, "grid": list(n), "steps": steps, "warmup": warmup,
        "value": P * steps / elapsed, "unit": "grid-pt updates/s", "ms_per_step": ms_per_step,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBPS,
                     "traffic": None if tr is None else tr["bytes"],
                     "traffic_source": None if tr is None else tr["source"],
                     "algorithmic_bytes_per_launch": bpp[dom] * P,
                     "avg_launch_ms": steady[dom]},
        # the pass model of the method: 104 B per point per 3-D step
        "model_bytes_per_point": MODEL_BPP,
        "model_step_gbps": MODEL_BPP * P / (ms_per_step * 1e-3) / 1e9,
        "model_step_hbm_frac": MODEL_BPP * P / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBPS,
        # what the chosen schedule moves (stored real-space psi: +8 B per point)
        "executed_bytes_per_point": executed,
        "executed_step_hbm_frac": executed * P / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBPS,
        "pass_ms": {k: round(v, 5) for k, v in prof.items()},
        "pass_sum_ms_per_step": sum(steady.values()),
        "schedule": schedule, "nonlinear_mode": mode,
        "kernel": {"c_newton": w["kern"][0], "c_yukawa": w["kern"][1], "m_yukawa": w["kern"][2]},
        "dz": w["dz"], "g": w["g"], "ic": w["ic"],
        "norm_drift": abs(m1 / m0 - 1),
        "energy_drift": abs(e1["total"] - e0["total"]) / scale,
    }


def batch_bench(steps, autotune_iters=0):
    """The 64-instance sweep (256^2/512^2/1024^2, per-instance Yukawa couplings):
    one gsn_batch_step graph launch, with the schedule gsn_batch_autotune picks
    per shape group, vs the same instances run one after another through
    gsn_step (a) with each group's batch schedule (bit-identical results,
    checked on one instance per shape) and (b) with each shape's own
    single-grid autotuned schedule."""
    import torch
    from paper_1909_08354_amd import gsn, inputs
    w = inputs.WORKLOADS["gsn2d_batch64_sweep"]
    inst = inputs.batch_sweep(w["count"], w["seed"], w["sizes"])
    total_pts = sum(int(np.prod(d["n"])) for d in inst)
    b = gsn.Batch([d["n"] for d in inst], [d["L"] for d in inst])

    def reset():
        for i, d in enumerate(inst):
            b.set(i, d["kern"], d["a"], d["g"], d["dz"], inputs.to_c64(d["psi"]))

    reset()
    m0 = b.masses()
    t_tune = 0.0
    if autotune_iters > 0:
        t0 = time.perf_counter()
        b.autotune(autotune_iters)
        t_tune = time.perf_counter() - t0
    names = gsn.variant_names()
    scheds = {}
    for i, d in enumerate(inst):
        if d["n"] not in scheds:
            v, m = b.schedule(i)
            scheds[d["n"]] = (v, m)
    b.step(steps)            # captures and instantiates the graph
    b.sync()
    reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(steps)
    b.sync()
    t_batch = time.perf_counter() - t0
    drift = float(np.max(np.abs(b.masses() / m0 - 1)))
    first = {}
    for i, d in enumerate(inst):
        first.setdefault(d["n"], i)
    batch_out = {n: b.get(i, np.complex64) for n, i in first.items()}
    t_pers = None
    if all(256 <= n[0] <= 1024 and 256 <= n[1] <= 1024 for n in (d["n"] for d in inst)):
        b.set_mode(1)
        reset()
        b.step(2)
        b.sync()
        reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.step(steps)
        b.sync()
        t_pers = time.perf_counter() - t0
        b.set_mode(0)
    # family order of the batch schedule: kinetic, density, kernel, phase, x entry/exit
    fam_pass = (("kinetic",), ("x_density",), ("kernel",), ("x_phase",), ("x_entry_fft", "x_exit_ifft"))

    def make_grids(tuned):
        out, sched = [], {}
        for d in inst:
            g = gsn.Grid(d["n"], d["L"])
            g.set_kernel(*d["kern"])
            g.set_coefficients(d["a"], d["g"], d["dz"])
            g.set_psi(inputs.to_c64(d["psi"]))
            pn = g.pass_names()
            if not tuned:
                v, m = scheds[d["n"]]
                sv = [0] * len(pn)
                for fv, passes in zip(v, fam_pass):
                    for nm in passes:
                        sv[pn.index(nm)] = fv
                g.set_schedule(sv)
                g.set_nonlinear_mode(m)
            elif d["n"] not in sched:
                g.autotune(5)
                sched[d["n"]] = (g.schedule(), g.nonlinear_mode())
            else:
                vn = {nm: v for v, nm in enumerate(names)}
                s0, m = sched[d["n"]]
                g.set_schedule([vn[s0[nm]] for nm in pn])
                g.set_nonlinear_mode(m)
            out.append(g)
        return out

    def time_seq(grids):
        grids[0].step(2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for g in grids:
            g.step(steps)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    grids = make_grids(False)
    t_seq = time_seq(grids)
    # the first instance of every shape again, from its initial state: equal
    # bits to the batch run
    same = True
    for n, i in first.items():
        d = inst[i]
        grids[i].set_psi(inputs.to_c64(d["psi"]))
        grids[i].step(steps)
        same = same and bool(np.array_equal(grids[i].get_psi(np.complex64), batch_out[n]))
    del grids
    grids = make_grids(True)
    t_tuned = time_seq(grids)
    del grids
    model_bytes = 56.0 * total_pts * steps
    return {"workload": "gsn2d_batch64_sweep", "instances": len(inst), "steps": steps,
            "grid_points": total_pts, "value": total_pts * steps / t_batch,
            "unit": "grid-pt updates/s", "ms_batch_graph": 1e3 * t_batch,
            "model_bytes_per_point": 56.0,
            "model_hbm_frac": model_bytes / t_batch / 1e9 / HBM_PEAK_GBPS,
            "autotune_iters": autotune_iters, "autotune_s": t_tune,
            "schedules": {"%dx%d" % n: {"families": dict(zip(("kinetic", "x_density", "kernel", "x_phase",
                                                                "x_fft"), [names[x] for x in v])),
                                          "nonlinear_mode": m} for n, (v, m) in scheds.items()},
            "ms_sequential_gsn_step": 1e3 * t_seq, "speedup": t_seq / t_batch,
            "ms_sequential_autotuned": 1e3 * t_tuned, "speedup_vs_autotuned": t_tuned / t_batch,
            "ms_batch_persistent": None if t_pers is None else 1e3 * t_pers,
            "speedup_persistent": None if t_pers is None else t_seq / t_pers,
            "max_norm_drift": drift,
            "bit_identical_to_sequential": same,
            "accuracy": "bit-identical to the sequential runs with the same schedule (checked on the "
                        "first instance of every shape)"}


def corrector_bench(ntrain, epochs, neval, ncoarse, tol):
    """Learned corrector on 512^2 lump states: train on solver-generated pairs
    (seeds 10000..), then on held-out seeds (20000..) compare, after ncoarse
    coarse steps (ratio 8), the plain coarse solver and the corrected one with
    the fine solver (the reference): relative L2 errors, share of seeds within tol,
    and device time of the fine and corrected runs."""
    from paper_1909_08354_amd import corrector_train as ct
    from paper_1909_08354_amd import gsn, inputs
    w = inputs.WORKLOADS["gsn2d_512_corrector"]
    t0 = time.perf_counter()
    data = ct.generate_pairs(list(range(w["train_seeds"][0], w["train_seeds"][0] + ntrain)))
    t_gen = time.perf_counter() - t0
    insc, outsc = ct.fit_scales(*data)
    corr = gsn.Corrector(*w["n"], max_batch=8)
    rng = np.random.default_rng(1)
    theta = []
    for ci, co in ((3, 32), (32, 32), (32, 32), (32, 2)):
        theta.append(rng.standard_normal(9 * co * ci) * 0.5 * np.sqrt(2.0 / (9 * ci)))
        theta.append(np.zeros(co))
    corr.set_weights(np.concatenate(theta).astype(np.float32))
    corr.set_scales(insc, outsc)
    tr = ct.train(corr, data, epochs=epochs, batch=8, lr=2e-3, lr_final=1e-4)
    del data
    ev = ct.evaluate(corr, list(range(w["heldout_seeds"][0], w["heldout_seeds"][0] + neval)), ncoarse=ncoarse)
    within_c = float(np.mean(np.array(ev["err_corrected"]) <= tol))
    within_k = float(np.mean(np.array(ev["err_coarse"]) <= tol))
    return {"workload": "gsn2d_512_corrector", "train_pairs": 2 * ntrain, "train_trajectories": ntrain,
            "epochs": epochs, "train_s": tr["seconds"], "gen_s": t_gen, "loss_first": tr["first_loss"],
            "loss_final": tr["final_loss"], "heldout_seeds": neval, "coarse_steps": ncoarse,
            "ratio": w["ratio"], "tol_rel_l2": tol,
            "err_coarse_mean": ev["err_coarse_mean"], "err_coarse_max": ev["err_coarse_max"],
            "err_corrected_mean": ev["err_corrected_mean"], "err_corrected_max": ev["err_corrected_max"],
            "share_within_tol_coarse": within_k, "share_within_tol_corrected": within_c,
            "ms_fine": 1e3 * ev["t_fine"] / neval, "ms_corrected": 1e3 * ev["t_corrected"] / neval,
            "ms_coarse": 1e3 * ev["t_coarse"] / neval, "speedup": ev["t_fine"] / ev["t_corrected"]}


def eq15_bench(steps, autotune_iters, profile_steps, workload="gsn3d_256_eq15"):
    """A 256^3 Eq. (15) fluid (pressure and Bohm terms on; with "nmc" in the
    workload also the position-dependent coupling of Eq. (9)-(12)): step rate,
    the per-pass times and the roofline of its dominant pass, and its
    invariants (no energy with source fields)."""
    import torch
    from paper_1909_08354_amd import gsn, inputs
    w = inputs.WORKLOADS[workload]
    n, L = w["n"], w["L"]
    P = int(np.prod(n))
    psi0 = inputs.fluid_gaussian(n, L, w["mass"], w["waist"], seed=w["seed"])
    grid = gsn.Grid(n, L)
    grid.set_kernel(*w["kern"])
    grid.set_coefficients(w["a"], w["g"], w["dz"])
    grid.set_local_terms(*w["local"])
    fields = None
    if "nmc" in w:
        fields = grid.nmc_fields(w["nmc"]["lam"], w["nmc"]["r0"], w["nmc"]["nu"])
        grid.set_source_fields(*fields)
    dev0 = torch.from_numpy(inputs.to_c64(psi0)).cuda()
    grid.set_psi(dev0)
    schedule = grid.autotune(autotune_iters) if autotune_iters > 0 else grid.schedule()
    grid.set_psi(dev0)
    m0 = grid.mass()
    e0 = grid.energy() if fields is None else None
    grid.step(10)
    grid.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    grid.step(steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    grid.sync()
    m1 = grid.mass()
    e1 = grid.energy() if fields is None else None
    prof = grid.profile_passes(profile_steps)
    bpp = dict(zip(grid.pass_names(), grid.pass_bytes_per_point()))
    steady = {k: v for k, v in prof.items() if k not in ("x_entry_fft", "x_exit_ifft") and bpp[k] > 0}
    dom = max(steady, key=steady.get)
    achieved = bpp[dom] * P / (steady[dom] * 1e-3) / 1e9
    step_bytes = sum(bpp[k] for k in steady) * P
    ms = 1e3 * elapsed / steps
    grid.close()
    edrift = None
    if e0 is not None:
        scale = abs(e0["kinetic"]) + abs(e0["local"]) + abs(e0["nonlocal"])
        edrift = abs(e1["total"] - e0["total"]) / scale
    return {"workload": workload, "grid": list(n), "local": list(w["local"]), "nmc": w.get("nmc"),
            "kernel": list(w["kern"]), "steps": steps, "value": P * steps / elapsed,
            "unit": "grid-pt updates/s", "ms_per_step": ms,
            "model_bytes_per_point": step_bytes / P,
            "model_step_hbm_frac": step_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS,
            "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBPS,
                         "unit": "GB/s", "frac": achieved / HBM_PEAK_GBPS,
                         "traffic": measured_leg_traffic(workload, dom, schedule.get(dom)),
                         "algorithmic_bytes_per_launch": bpp[dom] * P, "avg_launch_ms": steady[dom]},
            "pass_ms": {k: round(v, 5) for k, v in steady.items()}, "schedule": schedule,
            "norm_drift": abs(m1 / m0 - 1), "energy_drift": edrift}


def fp64_bench(steps, autotune_iters, profile_steps):
    """The 256^3 workload on an FP64-storage grid (complex128 in HBM and LDS):
    step rate, per-pass times, the roofline of its dominant pass, invariants."""
    import torch
    from paper_1909_08354_amd import gsn, inputs
    w = inputs.WORKLOADS[WORKLOAD_256]
    n, L = w["n"], w["L"]
    P = int(np.prod(n))
    grid = gsn.Grid(n, L, storage=np.complex128)
    grid.set_kernel(*w["kern"])
    grid.set_coefficients(w["a"], w["g"], w["dz"])
    dev0 = torch.from_numpy(inputs.as_oracle_input(inputs.gaussian_3d_256())).cuda()
    grid.set_psi(dev0)
    schedule = grid.autotune(autotune_iters) if autotune_iters > 0 else grid.schedule()
    grid.set_psi(dev0)
    m0 = grid.mass()
    e0 = grid.energy()
    grid.step(10)
    grid.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    grid.step(steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    grid.sync()
    m1 = grid.mass()
    e1 = grid.energy()
    prof = grid.profile_passes(profile_steps)
    bpp = dict(zip(grid.pass_names(), grid.pass_bytes_per_point()))
    steady = {k: v for k, v in prof.items() if k not in ("x_entry_fft", "x_exit_ifft") and bpp[k] > 0}
    dom = max(steady, key=steady.get)
    achieved = bpp[dom] * P / (steady[dom] * 1e-3) / 1e9
    step_bytes = sum(bpp[k] for k in steady) * P
    ms = 1e3 * elapsed / steps
    scale = abs(e0["kinetic"]) + abs(e0["local"]) + abs(e0["nonlocal"])
    grid.close()
    return {"workload": WORKLOAD_256, "storage": "c128", "grid": list(n), "steps": steps,
            "value": P * steps / elapsed, "unit": "grid-pt updates/s", "ms_per_step": ms,
            "model_bytes_per_point": step_bytes / P,
            "model_step_hbm_frac": step_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS,
            "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBPS,
                         "unit": "GB/s", "frac": achieved / HBM_PEAK_GBPS,
                         "traffic": measured_leg_traffic(FP64_LEG, dom, schedule.get(dom)),
                         "algorithmic_bytes_per_launch": bpp[dom] * P, "avg_launch_ms": steady[dom]},
            "pass_ms": {k: round(v, 5) for k, v in steady.items()}, "schedule": schedule,
            "norm_drift": abs(m1 / m0 - 1), "energy_drift": abs(e1["total"] - e0["total"]) / scale}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500,
                    help="timed steps of the 512^3 headline workload")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-steps", type=int, default=10)
    ap.add_argument("--autotune-iters", type=int, default=5)
    ap.add_argument("--steps-256", type=int, default=1000,
                    help="timed steps of the 256^3 single-grid leg (0 skips it)")
    ap.add_argument("--batch-steps", type=int, default=500,
                    help="steps of the 64-instance batched sweep (0 skips it)")
    ap.add_argument("--batch-autotune-iters", type=int, default=3,
                    help="iterations per variant of the batch autotuner (0: default schedule)")
    ap.add_argument("--corrector-train", type=int, default=2000,
                    help="training trajectories of the corrector leg (0 skips it)")
    ap.add_argument("--corrector-epochs", type=int, default=4)
    ap.add_argument("--fp64-steps", type=int, default=200,
                    help="steps of the 256^3 FP64-storage leg (0 skips it)")
    ap.add_argument("--eq15-steps", type=int, default=200,
                    help="steps of the 256^3 Eq. (15) fluid legs, without and with the "
                         "non-minimal coupling (0 skips them)")
    ap.add_argument("--corrector-eval", type=int, default=100)
    ap.add_argument("--copy-probe", action="store_true",
                    help="run one plain 1 GiB device copy first (calibrates HBM byte counters)")
    ap.add_argument("--only-256", action="store_true",
                    help="run the 256^3 leg in place of the 512^3 headline (profiling runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
              "(the solver is single-GPU; multi-GPU sharding is design-only).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1909_08354_amd import inputs

    if args.copy_probe:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    psi256 = inputs.to_c64(inputs.gaussian_3d_256())
    if args.only_256:
        head_name, head_psi, head_steps = WORKLOAD_256, psi256, args.steps
    else:
        w = inputs.WORKLOADS[WORKLOAD]
        head_name, head_steps = WORKLOAD, args.steps
        head_psi = inputs.lumps_3d(w["n"], w["seed"], 8, dtype=np.complex64)
    progress(f"{head_name}: state built")
    head = single_grid_leg(head_name, head_psi, head_steps, args.warmup, args.autotune_iters,
                           args.profile_steps)
    progress(f"{head_name}: {head['ms_per_step']:.4f} ms/step")
    w = inputs.WORKLOADS[head_name]
    line = {
        "metric": "split-step grid-pt updates/s + %HBM peak; batched/corrected speedup at fixed err",
        "value": head["value"],
        "unit": "grid-pt updates/s",
        "n_gpus": 1,
        "steps": head_steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "storage": "c64",
        "data": "synthetic",
        "config": {"workload": head_name, "grid": list(w["n"]), "dz": w["dz"],
                   "kernel": head["kernel"], "g": w["g"], "ic": w["ic"],
                   "passes_per_step": len([k for k, v in head["pass_ms"].items()
                                           if v > 0 and k not in ("x_entry_fft", "x_exit_ifft")])},
        "roofline": head["roofline"],
    }
    for k in ("model_bytes_per_point", "model_step_gbps", "model_step_hbm_frac",
              "executed_bytes_per_point", "executed_step_hbm_frac", "pass_ms",
              "pass_sum_ms_per_step", "schedule", "nonlinear_mode", "norm_drift", "energy_drift"):
        line[k] = head[k]
    line.update({"single_256": None, "batched_speedup": None, "batched": None,
                 "corrected_speedup": None, "corrected": None, "eq15": None, "nmc": None,
                 "fp64": None})
    del head_psi
    if args.steps_256 > 0 and not args.only_256:
        line["single_256"] = single_grid_leg(WORKLOAD_256, psi256, args.steps_256, args.warmup,
                                             args.autotune_iters, args.profile_steps)
        progress("256^3 leg done")
    if args.fp64_steps > 0:
        line["fp64"] = fp64_bench(args.fp64_steps, min(args.autotune_iters, 5), args.profile_steps)
        progress("FP64-storage leg done")
    if args.eq15_steps > 0:
        line["eq15"] = eq15_bench(args.eq15_steps, min(args.autotune_iters, 5), args.profile_steps)
        line["nmc"] = eq15_bench(args.eq15_steps, min(args.autotune_iters, 5), args.profile_steps,
                                 "gsn3d_256_nmc")
        progress("Eq. (15) legs done")
    if args.batch_steps > 0:
        line["batched"] = batch_bench(args.batch_steps, args.batch_autotune_iters)
        line["batched_speedup"] = line["batched"]["speedup"]
        progress("batched leg done")
    if args.corrector_train > 0:
        line["corrected"] = corrector_bench(args.corrector_train, args.corrector_epochs,
                                            args.corrector_eval, 10, 1e-4)
        line["corrected_speedup"] = line["corrected"]["speedup"]
        progress("corrector leg done")
    if not args.no_cpu_baseline:
        legs = []
        if not args.only_256:
            w4 = inputs.WORKLOADS[WORKLOAD]
            psi4 = inputs.lumps_3d(w4["n"], w4["seed"], 8, dtype=np.complex64).astype(np.complex128)
            legs.append((WORKLOAD, w4, psi4, (0,)))
        w2 = inputs.WORKLOADS[WORKLOAD_256]
        legs.append((WORKLOAD_256, w2, psi256.astype(np.complex128), (0, 1)))
        line["cpu_baseline"] = cpu_baseline(legs)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
