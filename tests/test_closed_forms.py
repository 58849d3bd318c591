"""The plane-wave closed forms used by the large-grid GPU checks, pinned to
the FP64 oracle on grids it transforms in milliseconds."""
import numpy as np
import pytest

from oracle import oracle as orc

import closed_forms as cf

MODES3 = [(3, -5, 7), (-2, 6, -13), (1, 7, 16), (-4, -8, 2)]   # 16 on an axis of 32: its Nyquist mode
AMPS = [0.6, 0.5 * np.exp(0.3j), 0.4 * np.exp(-1.1j), 0.25 * np.exp(2.0j)]


def grid_psi(modes, amps, n):
    psi = np.zeros(n, dtype=np.complex128)
    for m, A in zip(modes, amps):
        f = cf.axis_factors(m, n)
        psi += A * np.einsum("i,j,k->ijk", *f) if len(n) == 3 else A * np.outer(*f)
    return psi


@pytest.mark.parametrize("n,L", [((8, 16, 32), (5.0, 7.0, 11.0)), ((16, 32), (3.0, 9.0))])
def test_free_waves_match_the_oracle(n, L):
    modes = MODES3 if len(n) == 3 else [m[1:] for m in MODES3]
    psi0 = grid_psi(modes, AMPS, n)
    idx = cf.all_indices(n)
    assert np.allclose(psi0.reshape(-1), cf.free_waves(modes, AMPS, n, L, idx), rtol=0, atol=1e-13)
    dz, steps = 0.013, 7
    ref = orc.evolve(psi0, L, (0.0, 0.0, 0.0, 0.0), 0.5, 0.0, dz, steps)
    got = cf.free_waves(modes, AMPS, n, L, idx, a=0.5, z=dz * steps).reshape(n)
    assert orc.rel_l2(got, ref) < 1e-12
    # the modes really turned
    assert orc.rel_l2(ref, psi0) > 1e-2


@pytest.mark.parametrize("kern", [(1.0, 0.0, 0.0, 0.0), (0.7, 0.3, 0.5, 0.2), (0.0, 1.0, 0.25, 0.0)])
@pytest.mark.parametrize("n,L", [((8, 16, 32), (5.0, 7.0, 11.0)), ((16, 32), (3.0, 9.0))])
def test_wave_potential_matches_the_oracle(n, L, kern):
    modes = MODES3 if len(n) == 3 else [m[1:] for m in MODES3]
    psi0 = grid_psi(modes, AMPS, n)
    rho = np.abs(psi0) ** 2
    ref = orc.potential(rho, L, kern)
    idx = cf.all_indices(n)
    got = cf.wave_potential(modes, AMPS, n, L, kern, idx, include_k0=True).reshape(n)
    assert np.max(np.abs(got - ref)) < 1e-12 * np.max(np.abs(ref))
    # without the uniform part: the same up to the constant K(0) sum |A|^2
    got0 = cf.wave_potential(modes, AMPS, n, L, kern, idx, include_k0=False).reshape(n)
    k0 = cf.kernel_value(0.0, kern) * sum(abs(A) ** 2 for A in AMPS)
    assert np.max(np.abs(got0 + k0 - ref)) < 1e-12 * np.max(np.abs(ref))


def test_alias_takes_modes_into_the_grid_range():
    assert [cf.alias(m, 8) for m in (-5, -4, -1, 0, 3, 4, 12)] == [3, -4, -1, 0, 3, -4, -4]
