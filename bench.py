#!/usr/bin/env python3
"""Benchmark of the split-step Schroedinger-Newton hot path on one MI355X.

Workload: one 3-D instance, 256^3 periodic grid (dx = 1), complex64 storage
with FP64 arithmetic, centred Gaussian cloud of waist 6, Newtonian kernel plus
a Yukawa correction 0.3/(k^2 + 0.1^2), g = 0, dz = 5e-4.  A "step" is one
symmetric split step over the whole grid (8 HBM passes).  The timed region is
one gsn_step(K) call with psi already resident in HBM.

Prints ONE JSON line.  Besides throughput it reports the dominant pass's
roofline (algorithmic bytes / HIP-event duration on the solver's stream), the
norm and energy drift of the timed run, and the FP64 CPU oracle timed on a
bounded sample on this host (a baseline, not a target).
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
WORKLOAD = "gsn3d_256_newton_yukawa"


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


def measured_traffic(kernel_pass, variant):
    """HBM bytes per launch of a pass in a schedule variant, from committed
    rocprofv3 counter runs, only when they were taken on the current kernel
    sources."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    try:
        rec = json.load(open(p))
    except ValueError:
        return None
    if rec.get("csrc_hash") != csrc_hash():
        return None
    return rec.get("passes", {}).get(kernel_pass, {}).get(variant)


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


def cpu_baseline(w, psi0_c128, budget_s=30.0):
    """Oracle step rate on this host: time evolve(1) and evolve(3) on the same
    input; the difference is two merged steps without table setup."""
    from oracle import oracle as orc
    nthreads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or min(16, os.cpu_count() or 1)
    args = (w["L"], w["kern"], w["a"], w["g"], w["dz"])
    t0 = time.perf_counter()
    orc.evolve(psi0_c128, *args, 1, nthreads=nthreads)
    t1 = time.perf_counter()
    if (t1 - t0) * 3 > budget_s:
        per_step = t1 - t0
        sample = "1 merged step incl. table setup (budget)"
    else:
        orc.evolve(psi0_c128, *args, 3, nthreads=nthreads)
        t2 = time.perf_counter()
        per_step = max((t2 - t1) - (t1 - t0), 1e-9) / 2
        sample = "2 merged 256^3 steps (evolve(3) - evolve(1))"
    P = int(np.prod(w["n"]))
    return {"value": P / per_step, "unit": "grid-pt updates/s", "cores": nthreads,
            "kind": "oracle", "sample": sample}


def batch_bench(steps):
    """The 64-instance sweep (256^2/512^2/1024^2, per-instance Yukawa couplings):
    one gsn_batch_step graph launch vs the same instances run one after another
    through gsn_step, with the batch's schedule (bit-identical results) and with
    each shape's autotuned schedule."""
    import torch
    from paper_1909_08354_amd import gsn, inputs
    w = inputs.WORKLOADS["gsn2d_batch64_sweep"]
    inst = inputs.batch_sweep(w["count"], w["seed"], w["sizes"])
    total_pts = sum(int(np.prod(d["n"])) for d in inst)
    b = gsn.Batch([d["n"] for d in inst], [d["L"] for d in inst])
    for i, d in enumerate(inst):
        b.set(i, d["kern"], d["a"], d["g"], d["dz"], inputs.to_c64(d["psi"]))
    m0 = b.masses()
    b.step(steps)            # captures and instantiates the graph
    b.sync()
    for i, d in enumerate(inst):
        b.set(i, d["kern"], d["a"], d["g"], d["dz"], inputs.to_c64(d["psi"]))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(steps)
    b.sync()
    t_batch = time.perf_counter() - t0
    drift = float(np.max(np.abs(b.masses() / m0 - 1)))
    t_pers = None
    if all(256 <= n[0] <= 1024 and 256 <= n[1] <= 1024 for n in (d["n"] for d in inst)):
        b.set_mode(1)
        for i, d in enumerate(inst):
            b.set(i, d["kern"], d["a"], d["g"], d["dz"], inputs.to_c64(d["psi"]))
        b.step(2)
        b.sync()
        for i, d in enumerate(inst):
            b.set(i, d["kern"], d["a"], d["g"], d["dz"], inputs.to_c64(d["psi"]))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.step(steps)
        b.sync()
        t_pers = time.perf_counter() - t0
    # the plain form: every instance through gsn_step, (a) with the batch's own
    # schedule (the batch default: persistent kinetic/kernel p16, density/phase
    # p8, x entry/exit e16, stored real-space psi), bit-identical results;
    # (b) with each shape's own autotuned schedule
    fam = {"kinetic": 2, "x_density": 3, "kernel": 2, "x_phase": 3}

    def make_grids(tuned):
        out, sched = [], {}
        for d in inst:
            g = gsn.Grid(d["n"], d["L"])
            g.set_kernel(*d["kern"])
            g.set_coefficients(d["a"], d["g"], d["dz"])
            g.set_psi(inputs.to_c64(d["psi"]))
            if not tuned:
                g.set_schedule([fam.get(nm, 0) for nm in g.pass_names()])
                g.set_nonlinear_mode(1)
            elif d["n"] not in sched:
                g.autotune(5)
                sched[d["n"]] = (g.schedule(), g.nonlinear_mode())
            else:
                names = g.pass_names()
                vn = {nm: v for v, nm in enumerate(gsn.variant_names())}
                s0, m = sched[d["n"]]
                g.set_schedule([vn[s0[nm]] for nm in names])
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
    del grids
    grids = make_grids(True)
    t_tuned = time_seq(grids)
    del grids
    return {"workload": "gsn2d_batch64_sweep", "instances": len(inst), "steps": steps,
            "grid_points": total_pts, "value": total_pts * steps / t_batch,
            "unit": "grid-pt updates/s", "ms_batch_graph": 1e3 * t_batch,
            "ms_sequential_gsn_step": 1e3 * t_seq, "speedup": t_seq / t_batch,
            "ms_sequential_autotuned": 1e3 * t_tuned, "speedup_vs_autotuned": t_tuned / t_batch,
            "ms_batch_persistent": None if t_pers is None else 1e3 * t_pers,
            "speedup_persistent": None if t_pers is None else t_seq / t_pers,
            "max_norm_drift": drift,
            "accuracy": "bit-identical to the sequential runs (same kernels and schedule)"}


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
    w = inputs.WORKLOADS[WORKLOAD]
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
    return {"workload": WORKLOAD, "storage": "c128", "grid": list(n), "steps": steps,
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
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-steps", type=int, default=20)
    ap.add_argument("--autotune-iters", type=int, default=10)
    ap.add_argument("--batch-steps", type=int, default=500,
                    help="steps of the 64-instance batched sweep (0 skips it)")
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
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
              "(the solver is single-GPU; multi-GPU sharding is design-only).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1909_08354_amd import gsn, inputs

    if args.copy_probe:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    w = inputs.WORKLOADS[WORKLOAD]
    n, L = w["n"], w["L"]
    P = int(np.prod(n))
    psi0 = inputs.gaussian_3d_256()
    grid = gsn.Grid(n, L)
    grid.set_kernel(*w["kern"])
    grid.set_coefficients(w["a"], w["g"], w["dz"])
    grid.set_psi(torch.from_numpy(inputs.to_c64(psi0)).cuda())
    schedule = grid.autotune(args.autotune_iters) if args.autotune_iters > 0 else grid.schedule()
    m0 = grid.mass()
    e0 = grid.energy()

    if args.warmup:
        grid.step(args.warmup)
    grid.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    grid.step(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    grid.sync()
    elapsed = t1 - t0
    m1 = grid.mass()
    e1 = grid.energy()
    value = P * args.steps / elapsed
    ms_per_step = 1e3 * elapsed / args.steps

    # per-pass kernel durations: HIP events bound to each pass's dispatch on
    # the solver's stream, the launches back to back as in the timed steps
    prof = grid.profile_passes(args.profile_steps)
    bpp = dict(zip(grid.pass_names(), grid.pass_bytes_per_point()))
    steady = {k: v for k, v in prof.items() if k not in ("x_entry_fft", "x_exit_ifft")}
    dom = max(steady, key=steady.get)
    achieved = bpp[dom] * P / (steady[dom] * 1e-3) / 1e9
    traffic = measured_traffic(dom, schedule.get(dom))
    step_bytes = sum(bpp[k] for k in steady) * P
    scale = abs(e0["kinetic"]) + abs(e0["local"]) + abs(e0["nonlocal"])

    line = {
        "metric": "split-step grid-pt updates/s + %HBM peak; batched/corrected speedup at fixed err",
        "value": value,
        "unit": "grid-pt updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "storage": "c64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "grid": list(n), "dz": w["dz"],
                   "kernel": {"c_newton": w["kern"][0], "c_yukawa": w["kern"][1],
                              "m_yukawa": w["kern"][2]},
                   "g": w["g"], "ic": w["ic"], "passes_per_step": len(steady)},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBPS, "traffic": traffic,
                     "algorithmic_bytes_per_launch": bpp[dom] * P,
                     "avg_launch_ms": steady[dom]},
        "model_step_gbps": step_bytes / (ms_per_step * 1e-3) / 1e9,
        "model_step_hbm_frac": step_bytes / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBPS,
        "pass_ms": {k: round(v, 5) for k, v in prof.items()},
        "pass_sum_ms_per_step": sum(steady.values()),
        "schedule": schedule,
        "nonlinear_mode": grid.nonlinear_mode(),
        "norm_drift": abs(m1 / m0 - 1),
        "energy_drift": abs(e1["total"] - e0["total"]) / scale,
        "batched_speedup": None,
        "batched": None,
        "corrected_speedup": None,
        "corrected": None,
        "eq15": None,
        "nmc": None,
        "fp64": None,
    }
    if args.batch_steps > 0 or args.corrector_train > 0 or args.eq15_steps > 0 or args.fp64_steps > 0:
        grid.close()
        del grid
    if args.fp64_steps > 0:
        line["fp64"] = fp64_bench(args.fp64_steps, min(args.autotune_iters, 5), args.profile_steps)
    if args.eq15_steps > 0:
        line["eq15"] = eq15_bench(args.eq15_steps, min(args.autotune_iters, 5), args.profile_steps)
        line["nmc"] = eq15_bench(args.eq15_steps, min(args.autotune_iters, 5), args.profile_steps,
                                 "gsn3d_256_nmc")
    if args.batch_steps > 0:
        line["batched"] = batch_bench(args.batch_steps)
        line["batched_speedup"] = line["batched"]["speedup"]
    if args.corrector_train > 0:
        line["corrected"] = corrector_bench(args.corrector_train, args.corrector_epochs,
                                            args.corrector_eval, 10, 1e-4)
        line["corrected_speedup"] = line["corrected"]["speedup"]
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(w, inputs.as_oracle_input(psi0))
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
