"""Stored oracle results (tests/golden/) and their comparison with a HIP run.

The records are written by the scripts in tests/golden/, which call only the
FP64 oracle and the input module.  Planes are compared element by element on
the device copy of psi: relative L2 over each plane and the largest absolute
difference relative to the plane's largest |psi|.
"""
import json
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(name):
    """(record, planes) of a stored oracle result; planes maps xy / xz / yz to
    complex128 arrays."""
    rec = json.load(open(os.path.join(GOLDEN, name + ".json")))
    with np.load(os.path.join(GOLDEN, rec["planes"]["file"]), allow_pickle=False) as z:
        planes = {k: z[k] for k in ("xy", "xz", "yz")}
    return rec, planes


def plane_indices(rec):
    """Index arrays (iz, iy, ix) of the stored window on each axis and the
    fixed index of each plane: the whole central planes of the 256^3 record,
    the windows around the densest point of the 512^3 one."""
    n = rec["n"]
    if "origin" in rec["planes"]:
        win = rec["window"]
        idx = [(np.arange(win) + o) % N for o, N in zip(rec["planes"]["origin"], n)]
        fixed = rec["densest"]
    else:
        idx = [np.arange(N) for N in n]
        fixed = rec["planes"]["center"]
    return idx, fixed


def device_planes(psi_dev, rec):
    """The same planes cut from a device tensor psi (shape n, complex), as
    complex128 numpy arrays."""
    import torch
    (iz, iy, ix), (cz, cy, cx) = plane_indices(rec)
    dev = psi_dev.device
    tz, ty, tx = (torch.from_numpy(a).to(dev) for a in (iz, iy, ix))
    xy = psi_dev[cz].index_select(0, ty).index_select(1, tx)
    xz = psi_dev[:, cy, :].index_select(0, tz).index_select(1, tx)
    yz = psi_dev[:, :, cx].index_select(0, tz).index_select(1, ty)
    return {k: v.cpu().numpy().astype(np.complex128) for k, v in (("xy", xy), ("xz", xz), ("yz", yz))}


def compare(got, ref):
    """Per plane: (relative L2, max |diff| / max |ref|)."""
    out = {}
    for k in ref:
        d = got[k] - ref[k]
        out[k] = (float(np.linalg.norm(d) / np.linalg.norm(ref[k])),
                  float(np.max(np.abs(d)) / np.max(np.abs(ref[k]))))
    return out
