"""Training and evaluation of the learned coarse-step corrector.

Orchestration only: the solver generates every training pair (a coarse step
of ratio * dz and the ratio fine steps from the same state), the library's
kernels pack features, run the network forward and backward and take Adam
steps.  Data stay on the GPU as torch tensors.

Workload (synthetic): 2-D 512^2 periodic grids (dx = 1) of 1-4 Gaussian lumps
(waist U[2,6], velocity U[-0.5,0.5]^2), Newtonian kernel, g = -0.5,
dz_fine = 5e-3, dz_coarse = 8 dz_fine; training seeds 10000-11999, held-out
seeds 20000-20099.
"""
import time

import numpy as np

from . import gsn, inputs


def _grid(w, ratio, psi=None, tune=5):
    """A solver grid of the workload; with an initial state, its FFT schedule
    is autotuned on it (the fine and coarse steps share the schedule)."""
    g = gsn.Grid(w["n"], w["L"])
    g.set_kernel(*w["kern"])
    g.set_coefficients(w["a"], w["g"], w["dz_fine"])
    g.set_coarse_ratio(ratio)
    if psi is not None:
        g.set_psi(psi)
        if tune:
            g.autotune(tune)
    return g


def generate_pairs(seeds, w=None, pre_steps=(0, 24), ratio=None):
    """For every seed and every pre-step count: the state after that many fine
    steps, one coarse step from it (psi_c, phi_c) and the ratio fine steps
    from it (psi_f).  Returns device tensors (psi_c, phi_c, psi_f)."""
    import torch
    w = w or inputs.WORKLOADS["gsn2d_512_corrector"]
    ratio = ratio or w["ratio"]
    g = _grid(w, ratio, inputs.corrector_state_device(seeds[0], w["n"]))
    npair = len(seeds) * len(pre_steps)
    H, W = w["n"]
    psi_c = torch.empty((npair, H, W), dtype=torch.complex64, device="cuda")
    psi_f = torch.empty_like(psi_c)
    phi_c = torch.empty((npair, H, W), dtype=torch.float32, device="cuda")
    k = 0
    for s in seeds:
        ic = inputs.corrector_state_device(s, w["n"])
        for pre in pre_steps:
            g.set_psi(ic)
            if pre:
                g.step(pre)
            start = g.get_psi(np.complex64, device=True)
            g.step_coarse(1)
            psi_c[k] = g.get_psi(np.complex64, device=True)
            g.potential(phi_c[k])
            g.set_psi(start)
            g.step(ratio)
            psi_f[k] = g.get_psi(np.complex64, device=True)
            k += 1
    torch.cuda.synchronize()
    return psi_c, phi_c, psi_f


def fit_scales(psi_c, phi_c, psi_f):
    """Input scales bring features to O(1); the residual scale makes the
    targets O(1/4) (4 x the RMS residual)."""
    import torch
    a = float(torch.max(torch.abs(psi_c)).item())
    p = float(torch.max(torch.abs(phi_c)).item())
    r = float(torch.sqrt(torch.mean(torch.abs(psi_f - psi_c) ** 2)).item())
    return (1.0 / a, 1.0 / a, 1.0 / max(p, 1e-30)), 4.0 * max(r, 1e-30)


def train(corr, data, epochs=4, batch=8, lr=2e-3, lr_final=2e-4, seed=0, log=None):
    """Adam over shuffled minibatches of the pairs; cosine-free linear decay."""
    import torch
    psi_c, phi_c, psi_f = data
    n = psi_c.shape[0]
    rng = np.random.default_rng(seed)
    steps = epochs * (n // batch)
    losses = []
    t0 = time.perf_counter()
    it = 0
    for ep in range(epochs):
        order = rng.permutation(n)
        for j in range(n // batch):
            idx = order[j * batch:(j + 1) * batch]
            for b, i in enumerate(idx):
                corr.pack(b, psi_c[i], phi_c[i])
                corr.pack_target(b, psi_f[i], psi_c[i])
            frac = it / max(1, steps - 1)
            cur = lr * (1 - frac) + lr_final * frac
            losses.append(corr.train_step(batch, cur))
            it += 1
        if log:
            log(f"epoch {ep}: mean loss {np.mean(losses[-(n // batch):]):.4e}")
    torch.cuda.synchronize()
    return {"steps": it, "final_loss": float(np.mean(losses[-max(1, n // batch):])),
            "first_loss": float(losses[0]), "seconds": time.perf_counter() - t0, "losses": losses}


def evaluate(corr, seeds, ncoarse=10, w=None, ratio=None, audit_every=0, tol=0.0):
    """Relative L2 error after ncoarse steps of the plain coarse solver and of
    the corrected one, both against ratio * ncoarse fine steps (the reference),
    with device timings of the fine and corrected runs."""
    import torch
    w = w or inputs.WORKLOADS["gsn2d_512_corrector"]
    ratio = ratio or w["ratio"]
    ic0 = inputs.corrector_state_device(seeds[0], w["n"])
    gf, gc, gk = (_grid(w, ratio, ic0) for _ in range(3))
    res = {"err_coarse": [], "err_corrected": [], "t_fine": 0.0, "t_corrected": 0.0, "t_coarse": 0.0,
           "fallbacks": 0}
    for s in seeds:
        ic = inputs.corrector_state_device(s, w["n"])
        for g in (gf, gc, gk):
            g.set_psi(ic)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        gf.step(ratio * ncoarse)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        nfb, _ = gc.step_corrected(corr, ncoarse, audit_every, tol)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        gk.step_coarse(ncoarse)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        fine = gf.get_psi(np.complex128, device=True)
        nrm = torch.linalg.vector_norm(fine).item()
        res["err_corrected"].append(torch.linalg.vector_norm(gc.get_psi(np.complex128, device=True) - fine).item() / nrm)
        res["err_coarse"].append(torch.linalg.vector_norm(gk.get_psi(np.complex128, device=True) - fine).item() / nrm)
        res["t_fine"] += t1 - t0
        res["t_corrected"] += t2 - t1
        res["t_coarse"] += t3 - t2
        res["fallbacks"] += nfb
    for k in ("err_coarse", "err_corrected"):
        res[k + "_mean"] = float(np.mean(res[k]))
        res[k + "_max"] = float(np.max(res[k]))
    return res
