"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and validates arguments before any HIP call."""
import ctypes
import os

import pytest

from paper_1909_08354_amd import gsn

pytestmark = pytest.mark.skipif(not os.path.exists(gsn.LIB_PATH), reason="libgsn.so not built")


def test_every_header_symbol_is_exported():
    lib = gsn.load()
    names = gsn.header_functions()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def _create(ndim, n, L, ws, nbytes):
    lib = gsn.load()
    h = ctypes.c_void_p()
    st = lib.gsn_create(ctypes.byref(h), ndim, gsn._i32(n) if n is not None else None,
                        gsn._f64(L) if L is not None else None, ctypes.c_void_p(ws), nbytes, None)
    return st, h


@pytest.mark.parametrize("ndim,n,expect", [
    (1, (64,), gsn.GSN_EUNSUPPORTED), (4, (8, 8, 8, 8), gsn.GSN_EUNSUPPORTED),
    (2, (12, 16), gsn.GSN_EUNSUPPORTED), (2, (4, 16), gsn.GSN_EUNSUPPORTED),
    (3, (4096, 8, 8), gsn.GSN_EUNSUPPORTED), (2, (0, 8), gsn.GSN_EUNSUPPORTED)])
def test_workspace_bytes_rejects_bad_shapes(ndim, n, expect):
    lib = gsn.load()
    out = ctypes.c_size_t(0)
    assert lib.gsn_workspace_bytes(ndim, gsn._i32(n), ctypes.byref(out)) == expect
    assert lib.gsn_last_error()


def test_workspace_bytes_scales_with_grid():
    b2 = gsn.gsn_workspace_bytes((128, 128))
    b3 = gsn.gsn_workspace_bytes((256, 256, 256))
    P = 256 ** 3
    assert b2 >= 24 * 128 * 128
    # psi + scratch + two half spectra (rho and sqrt rho) (+ small tables)
    assert 24 * P <= b3 <= 25 * P


def test_create_validates_before_any_hip_call():
    lib = gsn.load()
    n, L = (64, 64), (10.0, 10.0)
    need = gsn.gsn_workspace_bytes(n)
    fake = 1 << 20   # an aligned address that is never dereferenced
    assert _create(2, n, L, None, need)[0] == gsn.GSN_EINVAL
    assert _create(2, n, None, fake, need)[0] == gsn.GSN_EINVAL
    assert _create(2, n, (10.0, -1.0), fake, need)[0] == gsn.GSN_EINVAL
    assert _create(2, n, (10.0, float("nan")), fake, need)[0] == gsn.GSN_EINVAL
    assert _create(2, n, L, fake + 8, need)[0] == gsn.GSN_EWORKSPACE
    assert _create(2, n, L, fake, need - 1)[0] == gsn.GSN_EWORKSPACE
    assert b"workspace" in lib.gsn_last_error()
    assert _create(3, (8, 8, 12), (1.0, 1.0, 1.0), fake, need)[0] == gsn.GSN_EUNSUPPORTED
    assert b"power of two" in lib.gsn_last_error()


def test_null_handles_are_rejected():
    lib = gsn.load()
    k = gsn.gsn_kernel(1.0, 0.0, 0.0, 0.0)
    assert lib.gsn_set_kernel(None, ctypes.byref(k)) == gsn.GSN_EINVAL
    assert lib.gsn_set_coefficients(None, 0.5, 0.0, 1e-3) == gsn.GSN_EINVAL
    assert lib.gsn_step(None, 1) == gsn.GSN_EINVAL
    assert lib.gsn_destroy(None) == gsn.GSN_EINVAL
    m = ctypes.c_double()
    assert lib.gsn_mass(None, ctypes.byref(m)) == gsn.GSN_EINVAL
    assert lib.gsn_get_psi(None, None, 0, 0) == gsn.GSN_EINVAL


def test_library_shares_torch_hip_runtime():
    """The binding loads libgsn after torch, whose wheel carries its own HIP
    runtime: the library then resolves libamdhip64 to that copy.  Loaded
    first, it mapped the system runtime and torch, imported afterwards, a
    second one, and the library's own HIP calls failed on the GPU.  Checked
    in a fresh process: one libamdhip64 and one libhsa-runtime64 mapped after
    load() and a later import of torch."""
    import subprocess
    import sys
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_1909_08354_amd import gsn\n"
            "gsn.load()\n"
            "import torch\n"
            "maps = open('/proc/self/maps').read().splitlines()\n"
            "libs = {l.split()[-1] for l in maps if 'libamdhip64' in l or 'libhsa-runtime64' in l}\n"
            "print(sorted(libs))\n"
            "assert len([p for p in libs if 'libamdhip64' in p]) == 1, libs\n"
            "assert len([p for p in libs if 'libhsa-runtime64' in p]) == 1, libs\n"
            % os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
