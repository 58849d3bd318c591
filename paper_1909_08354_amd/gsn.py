"""Thin ctypes binding of the C ABI in include/gsn.h (libgsn.so).

Argument marshalling only: every step of the solver runs in the HIP kernels of
libgsn.so.  PyTorch provides device memory (the caller-owned workspace and
device-side psi buffers) and the stream.  If the library is missing, loading
fails loudly; there is no CPU fallback.
"""
import ctypes
import os
import re

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libgsn.so")
HEADER = os.path.join(os.path.dirname(PKG), "include", "gsn.h")

GSN_OK, GSN_EINVAL, GSN_EUNSUPPORTED, GSN_EWORKSPACE, GSN_EHIP, GSN_ENONFINITE, GSN_ESTATE = range(7)
GSN_C64, GSN_C128 = 0, 1
STATUS_NAMES = {0: "GSN_OK", 1: "GSN_EINVAL", 2: "GSN_EUNSUPPORTED", 3: "GSN_EWORKSPACE",
                4: "GSN_EHIP", 5: "GSN_ENONFINITE", 6: "GSN_ESTATE"}


class GsnError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class gsn_kernel(ctypes.Structure):
    _fields_ = [("c_newton", ctypes.c_double), ("c_yukawa", ctypes.c_double),
                ("m_yukawa", ctypes.c_double), ("c_contact", ctypes.c_double)]


_lib = None
vp = ctypes.c_void_p
i32p = ctypes.POINTER(ctypes.c_int32)
dp = ctypes.POINTER(ctypes.c_double)

_SIGNATURES = {
    "gsn_workspace_bytes": [ctypes.c_int, i32p, ctypes.POINTER(ctypes.c_size_t)],
    "gsn_create": [ctypes.POINTER(vp), ctypes.c_int, i32p, dp, vp, ctypes.c_size_t, vp],
    "gsn_create_static": [ctypes.POINTER(vp), ctypes.c_int, i32p, dp, vp],
    "gsn_workspace_bytes_ex": [ctypes.c_int, i32p, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)],
    "gsn_create_ex": [ctypes.POINTER(vp), ctypes.c_int, i32p, dp, ctypes.c_int, vp, ctypes.c_size_t, vp],
    "gsn_destroy": [vp],
    "gsn_set_kernel": [vp, ctypes.POINTER(gsn_kernel)],
    "gsn_set_coefficients": [vp, ctypes.c_double, ctypes.c_double, ctypes.c_double],
    "gsn_set_local_terms": [vp, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double],
    "gsn_set_equation": [vp, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double],
    "gsn_set_source_fields": [vp, vp, vp, vp, ctypes.c_size_t],
    "gsn_nmc_fields": [vp, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.POINTER(ctypes.c_double),
                       ctypes.c_double, vp, vp, vp, ctypes.c_size_t],
    "gsn_set_psi": [vp, vp, ctypes.c_int, ctypes.c_int],
    "gsn_step": [vp, ctypes.c_int64],
    "gsn_sync": [vp],
    "gsn_get_psi": [vp, vp, ctypes.c_int, ctypes.c_int],
    "gsn_mass": [vp, dp],
    "gsn_energy": [vp, dp],
    "gsn_phase": [vp, dp, ctypes.POINTER(ctypes.c_int64)],
    "gsn_profile_passes": [vp, ctypes.c_int64, dp, ctypes.c_int],
    "gsn_autotune": [vp, ctypes.c_int],
    "gsn_get_schedule": [vp, ctypes.POINTER(ctypes.c_int), ctypes.c_int],
    "gsn_set_schedule": [vp, ctypes.POINTER(ctypes.c_int), ctypes.c_int],
    "gsn_set_nonlinear_mode": [vp, ctypes.c_int],
    "gsn_set_coarse_ratio": [vp, ctypes.c_int],
    "gsn_step_coarse": [vp, ctypes.c_int64],
    "gsn_potential": [vp, vp],
    "gsn_step_corrected": [vp, vp, ctypes.c_int64, ctypes.c_int, ctypes.c_double,
                           ctypes.POINTER(ctypes.c_int64), dp],
    "gsn_corrector_workspace_bytes": [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)],
    "gsn_corrector_create": [ctypes.POINTER(vp), ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, ctypes.c_size_t, vp],
    "gsn_corrector_destroy": [vp],
    "gsn_corrector_set_weights": [vp, ctypes.POINTER(ctypes.c_float), ctypes.c_size_t],
    "gsn_corrector_get_weights": [vp, ctypes.POINTER(ctypes.c_float), ctypes.c_size_t],
    "gsn_corrector_set_scales": [vp, ctypes.POINTER(ctypes.c_float), ctypes.c_float],
    "gsn_corrector_pack": [vp, ctypes.c_int, vp, vp],
    "gsn_corrector_pack_target": [vp, ctypes.c_int, vp, vp],
    "gsn_corrector_forward": [vp, ctypes.c_int, vp],
    "gsn_corrector_gradients": [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float)],
    "gsn_corrector_train_step": [vp, ctypes.c_int, ctypes.c_float, ctypes.POINTER(ctypes.c_float)],
    "gsn_corrector_apply": [vp, ctypes.c_int, vp, vp],
    "gsn_batch_workspace_bytes": [ctypes.c_int, ctypes.c_int, i32p, ctypes.POINTER(ctypes.c_size_t)],
    "gsn_batch_create": [ctypes.POINTER(vp), ctypes.c_int, ctypes.c_int, i32p, dp, vp, ctypes.c_size_t, vp],
    "gsn_batch_destroy": [vp],
    "gsn_batch_set": [vp, ctypes.c_int, ctypes.POINTER(gsn_kernel), ctypes.c_double, ctypes.c_double,
                      ctypes.c_double, vp, ctypes.c_int, ctypes.c_int],
    "gsn_batch_step": [vp, ctypes.c_int64],
    "gsn_batch_sync": [vp],
    "gsn_batch_get": [vp, ctypes.c_int, vp, ctypes.c_int, ctypes.c_int],
    "gsn_batch_mass": [vp, dp],
    "gsn_batch_phase": [vp, ctypes.c_int, dp, ctypes.POINTER(ctypes.c_int64)],
    "gsn_batch_set_mode": [vp, ctypes.c_int],
    "gsn_batch_set_queue_limits": [vp, ctypes.c_uint, ctypes.c_longlong],
    "gsn_batch_set_schedule": [vp, ctypes.POINTER(ctypes.c_int), ctypes.c_int, ctypes.c_int],
    "gsn_batch_autotune": [vp, ctypes.c_int],
    "gsn_batch_get_schedule": [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.c_int,
                               ctypes.POINTER(ctypes.c_int)],
    "gsn_get_nonlinear_mode": [vp, ctypes.POINTER(ctypes.c_int)],
}


def header_functions(path=HEADER):
    """Names of every function declared in include/gsn.h."""
    txt = open(path).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(gsn_[a-z0-9_]+)\s*\(", txt)))


def load(path=LIB_PATH):
    """Load libgsn.so (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built: run `python -c 'import __graft_entry__ as g; g.build()'`")
    # torch ships its own HIP runtime; loading it first makes the library
    # resolve libamdhip64 to that same copy (two runtimes in one process do
    # not share the device: the second one's calls fail)
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    for name, args in _SIGNATURES.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.gsn_last_error.argtypes = []
    lib.gsn_last_error.restype = ctypes.c_char_p
    lib.gsn_pass_count.argtypes = [vp]
    lib.gsn_pass_count.restype = ctypes.c_int
    lib.gsn_pass_name.argtypes = [vp, ctypes.c_int]
    lib.gsn_pass_name.restype = ctypes.c_char_p
    lib.gsn_pass_bytes_per_point.argtypes = [vp, ctypes.c_int]
    lib.gsn_pass_bytes_per_point.restype = ctypes.c_double
    lib.gsn_variant_count.argtypes = []
    lib.gsn_variant_count.restype = ctypes.c_int
    lib.gsn_variant_name.argtypes = [ctypes.c_int]
    lib.gsn_variant_name.restype = ctypes.c_char_p
    _lib = lib
    return lib


def check(status):
    if status != GSN_OK:
        raise GsnError(status, load().gsn_last_error().decode())
    return status


def _i32(seq):
    return (ctypes.c_int32 * len(seq))(*[int(v) for v in seq])


def _f64(seq):
    return (ctypes.c_double * len(seq))(*[float(v) for v in seq])


def gsn_workspace_bytes(n, storage=None):
    out = ctypes.c_size_t(0)
    if storage is None:
        check(load().gsn_workspace_bytes(len(n), _i32(n), ctypes.byref(out)))
    else:
        check(load().gsn_workspace_bytes_ex(len(n), _i32(n), _storage_code(storage), ctypes.byref(out)))
    return out.value


def _storage_code(storage):
    if storage in (np.complex64, "c64"):
        return GSN_C64
    if storage in (np.complex128, "c128"):
        return GSN_C128
    raise ValueError("storage must be complex64 or complex128")


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no HIP device visible to torch")
    return torch


def _ptr_and_flag(x):
    """(pointer, on_device, dtype code, keepalive) for a numpy array or torch tensor."""
    if isinstance(x, np.ndarray):
        if x.dtype == np.complex64:
            code = GSN_C64
        elif x.dtype == np.complex128:
            code = GSN_C128
        else:
            raise TypeError("psi must be complex64 or complex128")
        x = np.ascontiguousarray(x)
        return x.ctypes.data, 0, code, x
    torch = _torch()
    if x.dtype == torch.complex64:
        code = GSN_C64
    elif x.dtype == torch.complex128:
        code = GSN_C128
    else:
        raise TypeError("psi must be complex64 or complex128")
    x = x.contiguous()
    return x.data_ptr(), 1 if x.is_cuda else 0, code, x


class Grid:
    """One periodic 2-D or 3-D grid on the current HIP device (gsn_create;
    storage=np.complex128: gsn_create_ex with FP64 storage)."""

    def __init__(self, n, L, stream=None, storage=np.complex64, static_workspace=False):
        torch = _torch()
        lib = load()
        self.n = tuple(int(v) for v in n)
        self.L = tuple(float(v) for v in L)
        self.P = int(np.prod(self.n))
        self.storage = _storage_code(storage)
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        if static_workspace:
            # gsn_create_static: the library's per-device static workspace,
            # no device allocation anywhere (complex64 storage only)
            if self.storage != GSN_C64:
                raise ValueError("the static workspace holds complex64 grids only")
            self._ws = None
            h = vp()
            check(lib.gsn_create_static(ctypes.byref(h), len(self.n), _i32(self.n), _f64(self.L),
                                        vp(stream.cuda_stream)))
            self.h = h
            return
        nbytes = gsn_workspace_bytes(self.n, storage)
        self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        base = self._ws.data_ptr()
        aligned = (base + 255) & ~255
        h = vp()
        check(lib.gsn_create_ex(ctypes.byref(h), len(self.n), _i32(self.n), _f64(self.L), self.storage,
                                vp(aligned), nbytes, vp(stream.cuda_stream)))
        self.h = h

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            check(load().gsn_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_kernel(self, c_newton=0.0, c_yukawa=0.0, m_yukawa=0.0, c_contact=0.0):
        k = gsn_kernel(c_newton, c_yukawa, m_yukawa, c_contact)
        check(load().gsn_set_kernel(self.h, ctypes.byref(k)))

    def set_coefficients(self, a, g, dz):
        check(load().gsn_set_coefficients(self.h, a, g, dz))

    def set_equation(self, A, B, C, D):
        """Eq. (1)-(2) constants: a = -A, K = B D / (|k|^2 - C)."""
        check(load().gsn_set_equation(self.h, A, B, C, D))

    def _field_ptr(self, f):
        if f is None:
            return None
        t = _torch()
        if not (isinstance(f, t.Tensor) and f.is_cuda and f.dtype == t.float32 and f.is_contiguous()
                and tuple(f.shape) == tuple(self.n)):
            raise ValueError("fields must be contiguous float32 device tensors of the grid's shape")
        return f.data_ptr()

    def set_source_fields(self, gamma=None, beta=None, V_ext=None):
        """Position-dependent coupling s = gamma rho + beta lap(rho) and a static
        potential V_ext (device float32 tensors; references are kept while set)."""
        ptrs = [self._field_ptr(f) for f in (gamma, beta, V_ext)]
        check(load().gsn_set_source_fields(self.h, *ptrs, self.P))
        self._fields = (gamma, beta, V_ext)

    def nmc_fields(self, lam, r0, nu, center=None, r_min=None):
        """(gamma, beta, V_ext) of the pure non-minimal coupling, Eq. (9)-(11),
        as device float32 tensors; r_min defaults to half the smallest spacing."""
        t = _torch()
        out = [t.empty(tuple(self.n), dtype=t.float32, device="cuda") for _ in range(3)]
        c = None if center is None else _f64(center)
        rmin = 0.5 * min(Ld / N for N, Ld in zip(self.n, self.L)) if r_min is None else r_min
        check(load().gsn_nmc_fields(self.h, lam, r0, nu, c, rmin, *[o.data_ptr() for o in out], self.P))
        return tuple(out)

    def set_local_terms(self, c_pressure=0.0, n_pressure=1.0, c_bohm=0.0, rho_floor=0.0):
        """Pressure and Bohm terms of Eq. (15) (all zero: the Kerr model)."""
        check(load().gsn_set_local_terms(self.h, c_pressure, n_pressure, c_bohm, rho_floor))

    def set_psi(self, psi):
        ptr, dev, code, keep = _ptr_and_flag(psi)
        if tuple(keep.shape) != self.n:
            raise ValueError(f"psi shape {tuple(keep.shape)} != grid {self.n}")
        check(load().gsn_set_psi(self.h, vp(ptr), dev, code))
        self._keep = keep

    def step(self, nsteps):
        check(load().gsn_step(self.h, int(nsteps)))

    def sync(self):
        check(load().gsn_sync(self.h))

    def get_psi(self, dtype=np.complex128, device=False):
        if device:
            torch = _torch()
            tdt = torch.complex128 if dtype == np.complex128 else torch.complex64
            out = torch.empty(self.n, dtype=tdt, device="cuda")
            check(load().gsn_get_psi(self.h, vp(out.data_ptr()), 1,
                                     GSN_C128 if dtype == np.complex128 else GSN_C64))
            return out
        out = np.empty(self.n, dtype=dtype)
        check(load().gsn_get_psi(self.h, vp(out.ctypes.data), 0,
                                 GSN_C128 if dtype == np.complex128 else GSN_C64))
        return out

    def mass(self):
        m = ctypes.c_double(0)
        check(load().gsn_mass(self.h, ctypes.byref(m)))
        return m.value

    def energy(self):
        e = (ctypes.c_double * 4)()
        check(load().gsn_energy(self.h, e))
        return {"total": e[0], "kinetic": e[1], "local": e[2], "nonlocal": e[3]}

    def phase(self):
        th = ctypes.c_double(0)
        st = ctypes.c_int64(0)
        check(load().gsn_phase(self.h, ctypes.byref(th), ctypes.byref(st)))
        return th.value, st.value

    def pass_names(self):
        lib = load()
        return [lib.gsn_pass_name(self.h, i).decode() for i in range(lib.gsn_pass_count(self.h))]

    def pass_bytes_per_point(self):
        lib = load()
        return [lib.gsn_pass_bytes_per_point(self.h, i) for i in range(lib.gsn_pass_count(self.h))]

    def autotune(self, iters=20):
        check(load().gsn_autotune(self.h, int(iters)))
        return self.schedule()

    def schedule(self):
        lib = load()
        npass = lib.gsn_pass_count(self.h)
        v = (ctypes.c_int * npass)()
        check(lib.gsn_get_schedule(self.h, v, npass))
        return dict(zip(self.pass_names(), [lib.gsn_variant_name(i).decode() for i in v]))

    def nonlinear_mode(self):
        m = ctypes.c_int(0)
        check(load().gsn_get_nonlinear_mode(self.h, ctypes.byref(m)))
        return m.value

    def set_nonlinear_mode(self, mode):
        check(load().gsn_set_nonlinear_mode(self.h, int(mode)))

    def set_schedule(self, variants):
        """variants: one variant index per pass, or a single index for all."""
        lib = load()
        npass = lib.gsn_pass_count(self.h)
        if isinstance(variants, int):
            variants = [variants] * npass
        v = (ctypes.c_int * npass)(*variants)
        check(lib.gsn_set_schedule(self.h, v, npass))

    def set_coarse_ratio(self, ratio):
        check(load().gsn_set_coarse_ratio(self.h, int(ratio)))

    def step_coarse(self, nsteps):
        check(load().gsn_step_coarse(self.h, int(nsteps)))

    def potential(self, out=None):
        """phi of the current psi (float32 device tensor, no uniform k=0 part)."""
        torch = _torch()
        if out is None:
            out = torch.empty(self.n, dtype=torch.float32, device="cuda")
        check(load().gsn_potential(self.h, vp(out.data_ptr())))
        return out

    def step_corrected(self, corrector, ncoarse, audit_every=0, tol=0.0):
        nfb = ctypes.c_int64(0)
        worst = ctypes.c_double(0)
        check(load().gsn_step_corrected(self.h, corrector.h, int(ncoarse), int(audit_every), float(tol),
                                        ctypes.byref(nfb), ctypes.byref(worst)))
        return nfb.value, worst.value

    def profile_passes(self, nsteps):
        lib = load()
        npass = lib.gsn_pass_count(self.h)
        ms = (ctypes.c_double * npass)()
        check(lib.gsn_profile_passes(self.h, int(nsteps), ms, npass))
        return dict(zip(self.pass_names(), list(ms)))


BATCH_FAMILIES = ("kinetic", "x_density", "kernel", "x_phase", "x_fft")


def equation_optics():
    """(A, B) of Eq. (3) with k = k0 = 1: i psi_z = -lap psi / 2 - Delta n psi."""
    return (-0.5, -1.0)


def equation_thermo_optic(sigma, zeta, mu, kappa):
    """(A, B, C, D) of a thermo-optical medium, Eq. (4):
    lap Delta n - Delta n / sigma^2 = -(zeta mu / kappa) |E|^2."""
    return equation_optics() + (-1.0 / sigma ** 2, -zeta * mu / kappa)


def equation_nematic(nu, q):
    """(A, B, C, D) of a nematic liquid crystal, Eq. (5) divided by nu:
    lap theta - (2 q / nu) theta = -(2 / nu) |E|^2, with Delta n = theta."""
    return equation_optics() + (-2.0 * q / nu, -2.0 / nu)


def variant_names():
    """Names of the FFT schedule variants by index (gsn_variant_name)."""
    lib = load()
    return [lib.gsn_variant_name(i).decode() for i in range(lib.gsn_variant_count())]


class Batch:
    """Many independent 2-D instances advanced together (gsn_batch_create)."""

    def __init__(self, shapes, boxes, stream=None):
        torch = _torch()
        lib = load()
        self.shapes = [tuple(int(v) for v in n) for n in shapes]
        self.boxes = [tuple(float(v) for v in L) for L in boxes]
        self.count = len(self.shapes)
        flat_n = [v for n in self.shapes for v in n]
        flat_L = [v for L in self.boxes for v in L]
        nb = ctypes.c_size_t(0)
        check(lib.gsn_batch_workspace_bytes(self.count, 2, _i32(flat_n), ctypes.byref(nb)))
        self._ws = torch.empty(nb.value + 256, dtype=torch.uint8, device="cuda")
        aligned = (self._ws.data_ptr() + 255) & ~255
        stream = torch.cuda.current_stream() if stream is None else stream
        self.stream = stream
        h = vp()
        check(lib.gsn_batch_create(ctypes.byref(h), self.count, 2, _i32(flat_n), _f64(flat_L),
                                   vp(aligned), nb.value, vp(stream.cuda_stream)))
        self.h = h
        self._keep = {}

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            check(load().gsn_batch_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set(self, i, kern, a, g, dz, psi):
        k = gsn_kernel(*kern)
        ptr, dev, code, keep = _ptr_and_flag(psi)
        if tuple(keep.shape) != self.shapes[i]:
            raise ValueError("psi shape does not match instance %d" % i)
        check(load().gsn_batch_set(self.h, int(i), ctypes.byref(k), a, g, dz, vp(ptr), dev, code))
        self._keep[i] = keep

    def step(self, nsteps):
        check(load().gsn_batch_step(self.h, int(nsteps)))

    def sync(self):
        check(load().gsn_batch_sync(self.h))

    def get(self, i, dtype=np.complex128):
        out = np.empty(self.shapes[i], dtype=dtype)
        check(load().gsn_batch_get(self.h, int(i), vp(out.ctypes.data), 0,
                                   GSN_C128 if dtype == np.complex128 else GSN_C64))
        return out

    def masses(self):
        m = (ctypes.c_double * self.count)()
        check(load().gsn_batch_mass(self.h, m))
        return np.array(list(m))

    def phase(self, i):
        th = ctypes.c_double(0)
        st = ctypes.c_int64(0)
        check(load().gsn_batch_phase(self.h, int(i), ctypes.byref(th), ctypes.byref(st)))
        return th.value, st.value

    def set_mode(self, mode):
        check(load().gsn_batch_set_mode(self.h, int(mode)))

    def set_queue_limits(self, spin_limit=1 << 22, fail_item=-1):
        check(load().gsn_batch_set_queue_limits(self.h, int(spin_limit), int(fail_item)))

    def set_schedule(self, variants, nonlinear_mode=0):
        v = (ctypes.c_int * len(variants))(*variants)
        check(load().gsn_batch_set_schedule(self.h, v, len(variants), int(nonlinear_mode)))

    def autotune(self, iters=3):
        check(load().gsn_batch_autotune(self.h, int(iters)))

    def schedule(self, i):
        """(variant index per family in BATCH_FAMILIES, nonlinear mode) of
        instance i's shape group."""
        v = (ctypes.c_int * len(BATCH_FAMILIES))()
        m = ctypes.c_int(0)
        check(load().gsn_batch_get_schedule(self.h, int(i), v, len(BATCH_FAMILIES), ctypes.byref(m)))
        return list(v), m.value


CORRECTOR_NPARAMS = 19970


class Corrector:
    """The learned coarse-step corrector (gsn_corrector_create)."""

    def __init__(self, H, W, max_batch=1, stream=None):
        torch = _torch()
        lib = load()
        self.H, self.W, self.max_batch = int(H), int(W), int(max_batch)
        nb = ctypes.c_size_t(0)
        check(lib.gsn_corrector_workspace_bytes(self.H, self.W, self.max_batch, ctypes.byref(nb)))
        self._ws = torch.empty(nb.value + 256, dtype=torch.uint8, device="cuda")
        aligned = (self._ws.data_ptr() + 255) & ~255
        stream = torch.cuda.current_stream() if stream is None else stream
        h = vp()
        check(lib.gsn_corrector_create(ctypes.byref(h), self.H, self.W, self.max_batch, vp(aligned),
                                       nb.value, vp(stream.cuda_stream)))
        self.h = h

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            check(load().gsn_corrector_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_weights(self, w):
        w = np.ascontiguousarray(w, dtype=np.float32)
        check(load().gsn_corrector_set_weights(self.h, w.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), w.size))

    def get_weights(self):
        w = np.empty(CORRECTOR_NPARAMS, dtype=np.float32)
        check(load().gsn_corrector_get_weights(self.h, w.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), w.size))
        return w

    def set_scales(self, in_scale, out_scale):
        a = (ctypes.c_float * 3)(*[float(v) for v in in_scale])
        check(load().gsn_corrector_set_scales(self.h, a, float(out_scale)))

    def pack(self, b, psi, phi):
        check(load().gsn_corrector_pack(self.h, int(b), vp(psi.data_ptr()), vp(phi.data_ptr())))

    def pack_target(self, b, psi_fine, psi_coarse):
        check(load().gsn_corrector_pack_target(self.h, int(b), vp(psi_fine.data_ptr()),
                                               vp(psi_coarse.data_ptr())))

    def forward(self, B):
        torch = _torch()
        out = torch.empty((B, self.H, self.W, 2), dtype=torch.float32, device="cuda")
        check(load().gsn_corrector_forward(self.h, int(B), vp(out.data_ptr())))
        return out

    def gradients(self, B):
        g = np.empty(CORRECTOR_NPARAMS, dtype=np.float32)
        loss = ctypes.c_float(0)
        check(load().gsn_corrector_gradients(self.h, int(B), g.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                             ctypes.byref(loss)))
        return loss.value, g

    def train_step(self, B, lr):
        loss = ctypes.c_float(0)
        check(load().gsn_corrector_train_step(self.h, int(B), float(lr), ctypes.byref(loss)))
        return loss.value

    def apply(self, b, psi_c, psi_out):
        check(load().gsn_corrector_apply(self.h, int(b), vp(psi_c.data_ptr()), vp(psi_out.data_ptr())))
