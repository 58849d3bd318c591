"""Seeded synthetic initial states and workload recipes.

This module holds only input generation: grid coordinates, Gaussian lumps with
phase-gradient velocities and seeded random draws.  It contains none of the
solver's arithmetic, so both the HIP path and the CPU oracle can be fed from it.

The paper starts its simulations from a Gaussian distribution of the number
density (Sec. IV) and reaches a fluid velocity through the Madelung form
psi = sqrt(rho) exp(i S / nu), v = grad S (Sec. II, before Eq. (15)); a lump
moving with velocity v is therefore exp(-|x - c|^2 / w^2) exp(i v.(x - c)) with
nu = 1.  The paper gives no grid, box or duration, so every workload here is
synthetic; the recipes are listed in WORKLOADS.

Conventions: C-order arrays, slowest axis first; x_j = -L/2 + j L/N on each
axis; ``waist`` w is the optics convention psi = A exp(-r^2 / w^2); lumps use
minimum-image displacements on the periodic box.
"""
import numpy as np


def axis_coords(N, L):
    """Cell coordinates x_j = -L/2 + j L/N, j = 0..N-1."""
    return -0.5 * L + np.arange(N, dtype=np.float64) * (L / N)


def _min_image(d, L):
    return (d + 0.5 * L) % L - 0.5 * L


def gaussian(n, L, waist, amplitude=1.0, center=None, velocity=None):
    """Separable Gaussian lump amplitude*exp(-|x-c|^2/w^2)*exp(i v.(x-c))."""
    nd = len(n)
    center = np.zeros(nd) if center is None else np.asarray(center, dtype=np.float64)
    velocity = np.zeros(nd) if velocity is None else np.asarray(velocity, dtype=np.float64)
    out = np.array(amplitude, dtype=np.complex128)
    for ax in range(nd):
        x = axis_coords(n[ax], L[ax])
        d = _min_image(x - center[ax], L[ax])
        f = np.exp(-(d * d) / (waist * waist)) * np.exp(1j * velocity[ax] * d)
        shape = [1] * nd
        shape[ax] = n[ax]
        out = out * f.reshape(shape)
    return np.ascontiguousarray(np.broadcast_to(out, tuple(n)), dtype=np.complex128)


def lumps(n, L, centers, waists, velocities, amplitude=1.0):
    """Sum of Gaussian lumps (complex128)."""
    psi = np.zeros(tuple(n), dtype=np.complex128)
    for c, w, v in zip(centers, waists, velocities):
        psi += gaussian(n, L, w, amplitude, c, v)
    return psi


def phase_noise(psi, size, seed):
    """psi * exp(i size xi), xi i.i.d. U[-1, 1] per grid point from default_rng(seed)."""
    rng = np.random.default_rng(seed)
    xi = rng.uniform(-1.0, 1.0, size=psi.shape)
    return psi * np.exp(1j * size * xi)


def random_lumps(rng, n, L, count, waist_range, vel_range=0.5):
    """Draw ``count`` lumps in the order: centre, waist, velocity (per lump)."""
    nd = len(n)
    cs, ws, vs = [], [], []
    for _ in range(count):
        cs.append(rng.uniform(0.0, 1.0, size=nd) * np.asarray(L, dtype=np.float64))
        ws.append(rng.uniform(*waist_range))
        vs.append(rng.uniform(-vel_range, vel_range, size=nd))
    return cs, ws, vs


def to_c64(psi):
    """The bits both sides start from: the HIP path gets complex64 ..."""
    return np.ascontiguousarray(psi, dtype=np.complex64)


def as_oracle_input(psi):
    """... and the oracle gets complex128(complex64(psi)), so IC rounding is shared."""
    return np.ascontiguousarray(to_c64(psi), dtype=np.complex128)


# --------------------------------------------------------------------------
# workload recipes (every one synthetic; see module docstring)
# kern = (c_N, c_Y, m_Y, c_0); a = 1/2 (Eq. (3) with k = k0 = 1)
# --------------------------------------------------------------------------
WORKLOADS = {
    "gsn2d_128_kerr_newton": dict(
        n=(128, 128), L=(40.0, 40.0), kern=(1.0, 0.0, 0.0, 0.0), a=0.5, g=-0.5,
        dz=1e-3, steps=200, seed=1909,
        ic="gaussian A=1 w=3 centred, phase noise 1e-3*U[-1,1]"),
    "gsn3d_256_newton_yukawa": dict(
        n=(256, 256, 256), L=(256.0, 256.0, 256.0), kern=(1.0, 0.3, 0.1, 0.0), a=0.5,
        g=0.0, dz=5e-4, steps=1000, seed=2, ic="gaussian A=1 w=6 centred, real"),
    "gsn2d_batch64_sweep": dict(
        count=64, sizes=(256, 512, 1024), a=0.5, g=-0.5, dz=1e-3, steps=500, seed=3,
        ic="1-4 lumps, centres U[0,L)^2, w U[2,6], v U[-0.5,0.5]^2; c_Y U[0,1], m_Y U[0.05,0.5]"),
    "gsn3d_512_lumps": dict(
        n=(512, 512, 512), L=(512.0, 512.0, 512.0), kern=(1.0, 0.3, 0.1, 0.0), a=0.5,
        g=0.0, dz=2.5e-4, steps=2000, seed=4,
        ic="8 lumps, centres U[0,512)^3, w U[4,10], v U[-0.5,0.5]^3"),
    # Eq. (15) fluid: a Gaussian number density of total mass M0 (Sec. IV:
    # M0 = 25, nu = 1, w = 1.02, n = 1), so a = nu/2, c_bohm = -nu,
    # c_pressure = -w/nu and c_newton = gamma/nu with gamma = 1/2 (GR)
    "gsn3d_256_eq15": dict(
        n=(256, 256, 256), L=(256.0, 256.0, 256.0), kern=(0.5, 0.0, 0.0, 0.0), a=0.5,
        g=0.0, local=(-1.02, 1.0, -1.0, 1e-10), dz=5e-4, steps=200, seed=5, mass=25.0,
        waist=6.0, ic="Gaussian number density, total mass 25, waist 6, phase noise 1e-3"),
    # the same fluid under the pure non-minimal coupling (Eq. (9)-(12), alpha = 0,
    # lambda = 1, r0 = M0 / (4 pi)), with c_newton = 1/nu acting on the source
    # gamma rho + beta lap(rho) and V = -phi_C / nu
    "gsn3d_256_nmc": dict(
        n=(256, 256, 256), L=(256.0, 256.0, 256.0), kern=(1.0, 0.0, 0.0, 0.0), a=0.5,
        g=0.0, local=(-1.02, 1.0, -1.0, 1e-10), dz=5e-4, steps=200, seed=5, mass=25.0,
        waist=6.0, nmc=dict(lam=1.0, r0=25.0 / (4 * np.pi), nu=1.0),
        ic="Gaussian number density, total mass 25, waist 6, phase noise 1e-3"),
    "gsn2d_512_corrector": dict(
        n=(512, 512), L=(512.0, 512.0), kern=(1.0, 0.0, 0.0, 0.0), a=0.5, g=-0.5,
        dz_fine=5e-3, ratio=8, train_seeds=(10000, 12000), heldout_seeds=(20000, 20100),
        ic="1-4 lumps, centres U[0,L)^2, w U[2,6], v U[-0.5,0.5]^2"),
}


def gaussian_2d_128(seed=None):
    """128^2 on [-20,20)^2: Gaussian A=1 w=3 with 1e-3 phase noise."""
    w = WORKLOADS["gsn2d_128_kerr_newton"]
    psi = gaussian(w["n"], w["L"], 3.0)
    return phase_noise(psi, 1e-3, w["seed"] if seed is None else seed)


def fluid_gaussian(n, L, mass, waist, noise=1e-3, seed=5):
    """psi = sqrt(rho) for a Gaussian number density rho = rho0 exp(-|x|^2/w^2)
    of total mass ``mass`` (rho0 = mass / (pi w^2)^(D/2)), times a phase noise
    of size ``noise``."""
    rho0 = mass / (np.pi * waist * waist) ** (len(n) / 2)
    psi = gaussian(n, L, np.sqrt(2.0) * waist, amplitude=np.sqrt(rho0))
    return phase_noise(psi, noise, seed) if noise else psi


def gaussian_3d_256(n=None):
    """Centred real Gaussian cloud, waist 6 grid units (dx = 1)."""
    w = WORKLOADS["gsn3d_256_newton_yukawa"]
    n = w["n"] if n is None else n
    return gaussian(n, tuple(float(v) for v in n), 6.0)


def lumps_3d(n=(512, 512, 512), seed=4, count=8, dtype=np.complex128):
    """``count`` lumps, waist U[4,10], velocities U[-0.5,0.5]^3 (dx = 1).
    Built slab by slab from the separable 1-D factors, so a 512^3 complex64
    state needs no full-size complex128 temporaries."""
    rng = np.random.default_rng(seed)
    L = tuple(float(v) for v in n)
    cs, ws, vs = random_lumps(rng, n, L, count, (4.0, 10.0))
    psi = np.zeros(tuple(n), dtype=dtype)
    for c, w, v in zip(cs, ws, vs):
        f = []
        for ax in range(3):
            d = _min_image(axis_coords(n[ax], L[ax]) - c[ax], L[ax])
            f.append(np.exp(-(d * d) / (w * w)) * np.exp(1j * v[ax] * d))
        yx = np.outer(f[1], f[2])
        for z in range(n[0]):
            psi[z] += (f[0][z] * yx).astype(dtype)
    return psi


def batch_sweep(count=64, seed=3, sizes=(256, 512, 1024)):
    """Instances of the batched sweep, in draw order size, c_Y, m_Y, lump count,
    then per lump centre, waist, velocity.  Returns a list of dicts."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        N = int(sizes[rng.integers(0, len(sizes))])
        cY = float(rng.uniform(0.0, 1.0))
        mY = float(rng.uniform(0.05, 0.5))
        nl = int(rng.integers(1, 5))
        n, L = (N, N), (float(N), float(N))
        cs, ws, vs = random_lumps(rng, n, L, nl, (2.0, 6.0))
        out.append(dict(n=n, L=L, kern=(1.0, cY, mY, 0.0), a=0.5, g=-0.5, dz=1e-3,
                        psi=lumps(n, L, cs, ws, vs)))
    return out


def corrector_lumps(seed, n=(512, 512)):
    """Lump parameters (centres, waists, velocities) of one seeded corrector
    state: 1-4 lumps, waist U[2,6], velocity U[-0.5,0.5]^2, dx = 1."""
    rng = np.random.default_rng(seed)
    L = tuple(float(v) for v in n)
    nl = int(rng.integers(1, 5))
    return random_lumps(rng, n, L, nl, (2.0, 6.0))


def corrector_state(seed, n=(512, 512)):
    """One seeded 2-D lump state for the learned-corrector workload."""
    L = tuple(float(v) for v in n)
    cs, ws, vs = corrector_lumps(seed, n)
    return lumps(n, L, cs, ws, vs)


def corrector_state_device(seed, n=(512, 512), device="cuda"):
    """The same state built on a torch device (complex64) from the separable
    1-D factors, for generating many training states quickly."""
    import torch
    L = tuple(float(v) for v in n)
    cs, ws, vs = corrector_lumps(seed, n)
    psi = torch.zeros(tuple(n), dtype=torch.complex128, device=device)
    for c, w, v in zip(cs, ws, vs):
        f = []
        for ax in range(2):
            d = _min_image(axis_coords(n[ax], L[ax]) - c[ax], L[ax])
            f.append(torch.from_numpy(np.exp(-(d * d) / (w * w)) * np.exp(1j * v[ax] * d)).to(device))
        psi += torch.outer(f[0], f[1])
    return psi.to(torch.complex64)
