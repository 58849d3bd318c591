"""Write tests/golden/gsn3d_256_newton_yukawa.json from the FP64 oracle.

Workload: 256^3 periodic grid, dx = 1, centred Gaussian of waist 6 (real),
K = 1/k^2 (k = 0 dropped) + 0.3/(k^2 + 0.1^2), g = 0, a = 1/2, dz = 5e-4,
1000 merged symmetric split steps from complex128(complex64(psi0)).  Stored:
psi at 4096 seeded sample points and along the central x line, at the final
step, plus mass and energy at the start and the end.  Only oracle/ and the
input module are used.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as orc  # noqa: E402
from paper_1909_08354_amd import inputs  # noqa: E402

NAME = "gsn3d_256_newton_yukawa"
SAMPLE_SEED = 20260


def sample_indices(n, count=4096, seed=SAMPLE_SEED):
    rng = np.random.default_rng(seed)
    return [tuple(int(rng.integers(0, N)) for N in n) for _ in range(count)]


def main(nthreads=0, steps=None):
    w = inputs.WORKLOADS[NAME]
    steps = w["steps"] if steps is None else steps
    psi0 = inputs.as_oracle_input(inputs.gaussian_3d_256())
    args = (w["L"], w["kern"], w["a"], w["g"])
    ob0 = orc.observables(psi0, *args, nthreads=nthreads)
    t = time.time()
    psi = orc.evolve(psi0, *args, w["dz"], steps, nthreads=nthreads)
    el = time.time() - t
    ob1 = orc.observables(psi, *args, nthreads=nthreads)
    idx = sample_indices(w["n"])
    c = [N // 2 for N in w["n"]]
    rec = {
        "workload": NAME, "steps": steps, "dz": w["dz"], "kern": w["kern"], "a": w["a"],
        "g": w["g"], "n": w["n"], "L": w["L"], "sample_seed": SAMPLE_SEED,
        "oracle_seconds": el,
        "observables_start": ob0, "observables_end": ob1,
        "samples": [[list(i), psi[i].real, psi[i].imag] for i in idx],
        "x_line": {"z": c[0], "y": c[1],
                   "re": psi[c[0], c[1], :].real.tolist(), "im": psi[c[0], c[1], :].imag.tolist()},
    }
    out = os.path.join(HERE, NAME + ".json")
    with open(out + ".tmp", "w") as fh:
        json.dump(rec, fh)
    os.replace(out + ".tmp", out)
    print(out, el)


if __name__ == "__main__":
    main(nthreads=int(sys.argv[1]) if len(sys.argv) > 1 else 0)
