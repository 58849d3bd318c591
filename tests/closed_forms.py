"""Closed forms for superpositions of plane waves on a periodic grid, for
checks at sizes no CPU transform reaches.

psi(x) = sum_j A_j exp(i k_j . x) with k_j = 2 pi m_j / L (integer m_j, taken
into the grid's range [-N/2, N/2) per axis) and x_d = idx_d L_d / N_d:

* under the kinetic term alone (i psi_z = -a lap psi) every mode keeps its
  amplitude and turns its phase by exp(-i a |k_j|^2 z);
* the density |psi|^2 holds exactly the modes k_i - k_j with coefficients
  A_i conj(A_j), so phi = IDFT[K DFT rho] is the sum of K(k_i - k_j) A_i
  conj(A_j) exp(i (k_i - k_j) . x), the terms i = j giving the uniform part
  K(0) sum_j |A_j|^2.

Grid indices enter as integers (m idx mod N), so the phases are exact up to
one FP64 rounding."""
import numpy as np


def alias(m, N):
    """Integer mode m as the grid's wavenumber index in [-N/2, N/2)."""
    return ((int(m) + N // 2) % N) - N // 2


def k2_of(m, n, L):
    return sum((2.0 * np.pi * alias(md, Nd) / Ld) ** 2 for md, Nd, Ld in zip(m, n, L))


def kernel_value(k2, kern):
    """K(k) = c_N / |k|^2 (k != 0) + c_Y / (|k|^2 + m_Y^2) + c_0."""
    cN, cY, mY, c0 = kern
    K = c0
    if cY != 0.0:
        K += cY / (k2 + mY * mY)
    if k2 > 0.0:
        K += cN / k2
    return K


def mode_phase(m, n, idx):
    """exp(i k . x) at the grid indices idx (npts x ndim integer array)."""
    turns = np.zeros(idx.shape[0], dtype=np.float64)
    for d, (md, Nd) in enumerate(zip(m, n)):
        turns += ((alias(md, Nd) * idx[:, d].astype(np.int64)) % Nd) / Nd
    return np.exp(2j * np.pi * turns)


def free_waves(modes, amps, n, L, idx, a=0.5, z=0.0):
    """psi at idx after propagating a distance z under -a lap alone."""
    out = np.zeros(idx.shape[0], dtype=np.complex128)
    for m, A in zip(modes, amps):
        out += A * np.exp(-1j * a * k2_of(m, n, L) * z) * mode_phase(m, n, idx)
    return out


def wave_potential(modes, amps, n, L, kern, idx, include_k0=True):
    """phi of the density of the superposition at idx."""
    out = np.zeros(idx.shape[0], dtype=np.complex128)
    for i, (mi, Ai) in enumerate(zip(modes, amps)):
        for j, (mj, Aj) in enumerate(zip(modes, amps)):
            if i == j and not include_k0:
                continue
            d = tuple(alias(p - q, Nd) for p, q, Nd in zip(mi, mj, n))
            out += kernel_value(k2_of(d, n, L), kern) * Ai * np.conj(Aj) * mode_phase(d, n, idx)
    return out.real


def axis_factors(m, n):
    """Per-axis factors exp(i 2 pi alias(m_d) idx_d / N_d), idx_d = 0..N_d-1:
    their outer product is the plane wave on the whole grid."""
    return [np.exp(2j * np.pi * ((alias(md, Nd) * np.arange(Nd, dtype=np.int64)) % Nd) / Nd)
            for md, Nd in zip(m, n)]


def all_indices(n):
    return np.indices(n).reshape(len(n), -1).T
