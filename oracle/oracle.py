"""ctypes wrapper around the FP64 CPU oracle (``liboracle.so``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py``.  The product path never imports
this module, and this module imports nothing from the product package.

Conventions (arXiv:1909.08354 Sec. II Eq. (1)-(3), Sec. III):
  * arrays are numpy complex128 in C order, shape ``n`` (slowest axis first);
  * ``kern`` = (c_N, c_Y, m_Y, c_0): K(k) = c_N/|k|^2 [k != 0]
    + c_Y/(|k|^2 + m_Y^2) + c_0;
  * ``a`` kinetic coefficient (1/2 for Eq. (3) with k = k0 = 1),
    ``g`` local (Kerr) coefficient, ``dz`` the step;
  * ``eq`` = (A, B, C, D): Eq. (1)-(2) with their own constants,
    i psi_t = A lap psi + B phi psi + G psi, lap phi + C phi = D rho, so that
    a = -A and K = B D / (|k|^2 - C) (C > 0: Helmholtz, resonances rejected);
  * ``fields`` = (gamma, beta, V) or None (each an array of the grid's shape or
    None): the kernel acts on s = gamma rho + beta lap(rho) and V joins the
    phase (position-dependent coupling of Eq. (9)-(12));
  * ``local`` = (c_p, n_p, c_B, rho_f) or None: the local terms of Eq. (15),
    U = g rho + c_p f_n(max(rho, rho_f)) + c_B lap(sqrt rho) / (2 max(sqrt rho,
    sqrt rho_f)) with f_1 = ln rho, f_n = n/(n-1) rho^(n-1) (Sec. II C).
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b  # type: ignore
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int)
    lib.orc_fft.argtypes = [dp, ctypes.c_int, ip, ctypes.c_int, ctypes.c_int]
    lib.orc_dft_brute.argtypes = [dp, dp, ctypes.c_int, ip, ctypes.c_int]
    lib.orc_potential.argtypes = [dp, dp, ctypes.c_int, ip, dp, dp, ctypes.c_int]
    lib.orc_evolve.argtypes = [dp, ctypes.c_int, ip, dp, dp, ctypes.c_double,
                               ctypes.c_double, ctypes.c_double, ctypes.c_longlong,
                               ctypes.c_int, ctypes.c_int]
    lib.orc_observables.argtypes = [dp, ctypes.c_int, ip, dp, dp, ctypes.c_double,
                                    ctypes.c_double, dp, ctypes.c_int]
    lib.orc_evolve_local.argtypes = [dp, ctypes.c_int, ip, dp, dp, ctypes.c_double,
                                     ctypes.c_double, dp, ctypes.c_double, ctypes.c_longlong,
                                     ctypes.c_int, ctypes.c_int]
    lib.orc_observables_local.argtypes = [dp, ctypes.c_int, ip, dp, dp, ctypes.c_double,
                                          ctypes.c_double, dp, dp, ctypes.c_int]
    lib.orc_local_potential.argtypes = [dp, ctypes.c_int, ip, dp, ctypes.c_double, dp, dp,
                                        ctypes.c_int]
    d = ctypes.c_double
    lib.orc_evolve_equation.argtypes = [dp, ctypes.c_int, ip, dp, d, d, d, d, d, dp, d,
                                        ctypes.c_longlong, ctypes.c_int, ctypes.c_int]
    lib.orc_potential_equation.argtypes = [dp, dp, ctypes.c_int, ip, dp, d, d, d, ctypes.c_int]
    lib.orc_observables_equation.argtypes = [dp, ctypes.c_int, ip, dp, d, d, d, d, d, dp, dp,
                                             ctypes.c_int]
    lib.orc_evolve_fields.argtypes = [dp, ctypes.c_int, ip, dp, dp, d, d, dp, dp, dp, dp, d,
                                      ctypes.c_longlong, ctypes.c_int, ctypes.c_int]
    lib.orc_potential_fields.argtypes = [dp, dp, ctypes.c_int, ip, dp, dp, dp, dp, ctypes.c_int]
    lib.orc_nmc_fields.argtypes = [ctypes.c_int, ip, dp, d, d, d, dp, d, dp, dp, dp]
    lib.orc_observables_vext.argtypes = [dp, ctypes.c_int, ip, dp, dp, d, d, dp, dp, dp, ctypes.c_int]
    lib.orc_max_threads.argtypes = []
    for f in ("orc_fft", "orc_dft_brute", "orc_potential", "orc_evolve",
              "orc_observables", "orc_evolve_local", "orc_observables_local",
              "orc_local_potential", "orc_evolve_equation", "orc_potential_equation",
              "orc_observables_equation", "orc_evolve_fields", "orc_potential_fields",
              "orc_nmc_fields", "orc_observables_vext", "orc_max_threads"):
        getattr(lib, f).restype = ctypes.c_int
    _lib = lib
    return lib


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _shape_args(shape, L=None):
    n = (ctypes.c_int * len(shape))(*[int(s) for s in shape])
    if L is None:
        return n, None
    Larr = np.ascontiguousarray(np.asarray(L, dtype=np.float64).reshape(len(shape)))
    return n, Larr


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what} failed with code {rc}")


def max_threads():
    return _load().orc_max_threads()


def fft(x, inverse=False, nthreads=0):
    """Unnormalised forward DFT (exp(-i k.x)); inverse carries 1/P."""
    a = np.array(x, dtype=np.complex128, order="C", copy=True)
    n, _ = _shape_args(a.shape)
    _check(_load().orc_fft(_dptr(a), a.ndim, n, 1 if inverse else -1, nthreads), "fft")
    return a


def dft_brute(x, inverse=False):
    """O(P^2) DFT with the same normalisation as :func:`fft` (pin only)."""
    a = np.ascontiguousarray(x, dtype=np.complex128)
    out = np.empty_like(a)
    n, _ = _shape_args(a.shape)
    _check(_load().orc_dft_brute(_dptr(a), _dptr(out), a.ndim, n, 1 if inverse else -1),
           "dft_brute")
    return out


def potential(rho, L, kern, nthreads=0):
    """phi = Re IDFT[K DFT rho] for a real density on a periodic box."""
    r = np.ascontiguousarray(rho, dtype=np.float64)
    phi = np.empty_like(r)
    n, Larr = _shape_args(r.shape, L)
    k = np.ascontiguousarray(kern, dtype=np.float64)
    _check(_load().orc_potential(_dptr(r), _dptr(phi), r.ndim, n, _dptr(Larr), _dptr(k),
                                 nthreads), "potential")
    return phi


def _local_arr(local):
    if local is None:
        return None
    arr = np.ascontiguousarray(local, dtype=np.float64).reshape(4)
    return arr


def evolve(psi, L, kern, a, g, dz, nsteps, merged=True, nthreads=0, local=None):
    """nsteps symmetric split steps of the equation; returns a new array."""
    p = np.array(psi, dtype=np.complex128, order="C", copy=True)
    n, Larr = _shape_args(p.shape, L)
    k = np.ascontiguousarray(kern, dtype=np.float64)
    lp = _local_arr(local)
    if lp is None:
        rc = _load().orc_evolve(_dptr(p), p.ndim, n, _dptr(Larr), _dptr(k), float(a), float(g),
                                float(dz), int(nsteps), 1 if merged else 0, nthreads)
    else:
        rc = _load().orc_evolve_local(_dptr(p), p.ndim, n, _dptr(Larr), _dptr(k), float(a),
                                      float(g), _dptr(lp), float(dz), int(nsteps),
                                      1 if merged else 0, nthreads)
    _check(rc, "evolve")
    return p


def observables(psi, L, kern, a, g, nthreads=0, local=None, V=None):
    """dict(mass, kinetic, local, nonlocal, total, pressure, bohm) of psi;
    ``local`` (the total local energy) includes the pressure and Bohm parts and,
    with a static potential V, -dV sum V rho."""
    p = np.ascontiguousarray(psi, dtype=np.complex128)
    n, Larr = _shape_args(p.shape, L)
    k = np.ascontiguousarray(kern, dtype=np.float64)
    out = np.zeros(7)
    lp = _local_arr(local)
    if V is not None:
        Va = np.ascontiguousarray(V, dtype=np.float64)
        if Va.shape != p.shape:
            raise ValueError("V shape differs from the grid")
        rc = _load().orc_observables_vext(_dptr(p), p.ndim, n, _dptr(Larr), _dptr(k), float(a), float(g),
                                          None if lp is None else _dptr(lp), _dptr(Va), _dptr(out), nthreads)
    elif lp is None:
        rc = _load().orc_observables(_dptr(p), p.ndim, n, _dptr(Larr), _dptr(k), float(a),
                                     float(g), _dptr(out), nthreads)
    else:
        rc = _load().orc_observables_local(_dptr(p), p.ndim, n, _dptr(Larr), _dptr(k), float(a),
                                           float(g), _dptr(lp), _dptr(out), nthreads)
    _check(rc, "observables")
    return {"mass": out[0], "kinetic": out[1], "local": out[2], "nonlocal": out[3],
            "total": out[4], "pressure": out[5], "bohm": out[6]}


def local_potential(psi, L, g, local, nthreads=0):
    """The local potential U(x) of psi (Kerr + pressure + Bohm), real array."""
    p = np.ascontiguousarray(psi, dtype=np.complex128)
    n, Larr = _shape_args(p.shape, L)
    U = np.empty(p.shape, dtype=np.float64)
    lp = _local_arr(local)
    _check(_load().orc_local_potential(_dptr(p), p.ndim, n, _dptr(Larr), float(g),
                                       None if lp is None else _dptr(lp), _dptr(U), nthreads),
           "local_potential")
    return U


def rel_l2(x, ref):
    """||x - ref||_2 / ||ref||_2 in FP64."""
    x = np.asarray(x, dtype=np.complex128)
    ref = np.asarray(ref, dtype=np.complex128)
    return float(np.linalg.norm((x - ref).ravel()) / np.linalg.norm(ref.ravel()))


def evolve_equation(psi, L, eq, g, dz, nsteps, merged=True, nthreads=0, local=None):
    """nsteps symmetric split steps of Eq. (1)-(2) with constants eq = (A, B, C, D)."""
    p = np.array(psi, dtype=np.complex128, order="C", copy=True)
    n, Larr = _shape_args(p.shape, L)
    lp = _local_arr(local)
    A, B, C, D = (float(v) for v in eq)
    _check(_load().orc_evolve_equation(_dptr(p), p.ndim, n, _dptr(Larr), A, B, C, D, float(g),
                                       None if lp is None else _dptr(lp), float(dz), int(nsteps),
                                       1 if merged else 0, nthreads), "evolve_equation")
    return p


def potential_equation(rho, L, eq, nthreads=0):
    """This file's phi (= -B phi of Eq. (2)) for a real density: Re IDFT[B D/(|k|^2 - C) DFT rho]."""
    r = np.ascontiguousarray(rho, dtype=np.float64)
    phi = np.empty_like(r)
    n, Larr = _shape_args(r.shape, L)
    _, B, C, D = (float(v) for v in eq)
    _check(_load().orc_potential_equation(_dptr(r), _dptr(phi), r.ndim, n, _dptr(Larr), B, C, D,
                                          nthreads), "potential_equation")
    return phi


def observables_equation(psi, L, eq, g, nthreads=0, local=None):
    """observables() for Eq. (1)-(2) with constants eq = (A, B, C, D)."""
    p = np.ascontiguousarray(psi, dtype=np.complex128)
    n, Larr = _shape_args(p.shape, L)
    out = np.zeros(7)
    lp = _local_arr(local)
    A, B, C, D = (float(v) for v in eq)
    _check(_load().orc_observables_equation(_dptr(p), p.ndim, n, _dptr(Larr), A, B, C, D, float(g),
                                            None if lp is None else _dptr(lp), _dptr(out), nthreads),
           "observables_equation")
    return {"mass": out[0], "kinetic": out[1], "local": out[2], "nonlocal": out[3],
            "total": out[4], "pressure": out[5], "bohm": out[6]}


def _field(f, shape):
    if f is None:
        return None
    a = np.ascontiguousarray(f, dtype=np.float64)
    if a.shape != tuple(shape):
        raise ValueError("field shape differs from the grid")
    return a


def evolve_fields(psi, L, kern, a, g, dz, nsteps, fields, merged=True, nthreads=0, local=None):
    """evolve() with position-dependent source fields and a static potential."""
    p = np.array(psi, dtype=np.complex128, order="C", copy=True)
    n, Larr = _shape_args(p.shape, L)
    k = np.ascontiguousarray(kern, dtype=np.float64)
    lp = _local_arr(local)
    gm, bt, V = (_field(f, p.shape) for f in fields)
    ptr = lambda x: None if x is None else _dptr(x)
    _check(_load().orc_evolve_fields(_dptr(p), p.ndim, n, _dptr(Larr), _dptr(k), float(a), float(g),
                                     ptr(lp), ptr(gm), ptr(bt), ptr(V), float(dz), int(nsteps),
                                     1 if merged else 0, nthreads), "evolve_fields")
    return p


def potential_fields(rho, L, kern, gamma=None, beta=None, nthreads=0):
    """phi = Re IDFT[K DFT s], s = gamma rho + beta lap(rho)."""
    r = np.ascontiguousarray(rho, dtype=np.float64)
    phi = np.empty_like(r)
    n, Larr = _shape_args(r.shape, L)
    k = np.ascontiguousarray(kern, dtype=np.float64)
    gm, bt = _field(gamma, r.shape), _field(beta, r.shape)
    ptr = lambda x: None if x is None else _dptr(x)
    _check(_load().orc_potential_fields(_dptr(r), _dptr(phi), r.ndim, n, _dptr(Larr), _dptr(k),
                                        ptr(gm), ptr(bt), nthreads), "potential_fields")
    return phi


def nmc_fields(n, L, lam, r0, nu, center=None, r_min=None):
    """(gamma, beta, V) of the pure non-minimal coupling, Eq. (9)-(11), with
    V = -phi_C / nu and phi_C cut at r_min (default half the smallest spacing)."""
    n = tuple(int(v) for v in n)
    na, Larr = _shape_args(n, L)
    c = np.zeros(len(n)) if center is None else np.ascontiguousarray(center, dtype=np.float64)
    rmin = 0.5 * min(Ld / N for N, Ld in zip(n, L)) if r_min is None else float(r_min)
    gm, bt, V = (np.empty(n) for _ in range(3))
    _check(_load().orc_nmc_fields(len(n), na, _dptr(Larr), float(lam), float(r0), float(nu), _dptr(c),
                                  rmin, _dptr(gm), _dptr(bt), _dptr(V)), "nmc_fields")
    return gm, bt, V
