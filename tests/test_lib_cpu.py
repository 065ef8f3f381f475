"""CPU-side checks of the C ABI: the library loads, exports every function
that include/drot.h declares, and rejects invalid arguments before any GPU
work (these paths never touch a device)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    with open(os.path.join(ROOT, "include", "drot.h")) as fh:
        text = fh.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(drot_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2110_11738_amd import drot
    return drot.lib()


def test_header_declares_the_documented_entry_points():
    names = _declared()
    for must in ("drot_solve", "drot_bind", "drot_iterate", "drot_poll", "drot_finish",
                 "drot_solve_cost", "drot_bind_cost",
                 "drot_ctx_create", "drot_ctx_destroy", "drot_get_trace", "drot_last_error",
                 "drot_strerror", "drot_version"):
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def test_binding_covers_every_export():
    from paper_2110_11738_amd import drot
    assert set(_declared()) == set(drot.EXPORTED)


def test_struct_layouts_match_header(lib):
    from paper_2110_11738_amd import drot
    # drot_params: 2 doubles, 1 int64, 10 int32 -> 64 bytes;
    # drot_result: int64, 2 int32, 11 doubles, int64, double -> 120 bytes
    assert ctypes.sizeof(drot.Params) == 64
    assert ctypes.sizeof(drot.Result) == 120
    assert ctypes.sizeof(drot.Cost) == 48


def test_version_and_strerror(lib):
    from paper_2110_11738_amd import drot
    assert b"gfx950" in lib.drot_version()
    for code in (drot.OK, drot.MAXITER, drot.EINVAL, drot.EMASS, drot.ENONFINITE, drot.ENOMEM,
                 drot.EDEVICE, drot.EUNSUPPORTED, drot.ESTATE):
        assert lib.drot_strerror(code) != b"unknown status"


def _solve(lib, m=4, n=5, dtype=0, C=1, ldc=None, p=2, q=3, prm=None, X=4096, ldx=None,
           mu0=None, nu0=None, out=True):
    from paper_2110_11738_amd import drot
    prm = prm if prm is not None else drot.make_params(0.1, 1e-4, 100)
    res = drot.Result()
    return lib.drot_solve(None, m, n, dtype, C and C * 4096, n if ldc is None else ldc,
                          p and p * 4096 * 1000, q and q * 4096 * 2000, ctypes.byref(prm),
                          X and X * 100000, n if ldx is None else ldx, None, None, mu0, nu0,
                          ctypes.byref(res) if out else None, None)


def test_argument_validation_without_device(lib):
    from paper_2110_11738_amd import drot
    assert _solve(lib, out=False) == drot.EINVAL
    assert _solve(lib, m=0) == drot.EINVAL
    assert _solve(lib, n=-3) == drot.EINVAL
    assert _solve(lib, dtype=7) == drot.EINVAL
    assert _solve(lib, ldc=3) == drot.EINVAL
    assert _solve(lib, ldx=2) == drot.EINVAL
    assert _solve(lib, prm=drot.make_params(0.0)) == drot.EINVAL
    assert _solve(lib, prm=drot.make_params(float("nan"))) == drot.EINVAL
    assert _solve(lib, prm=drot.make_params(0.1, -1.0)) == drot.EINVAL
    assert _solve(lib, prm=drot.make_params(0.1, 1e-4, 0)) == drot.EINVAL
    assert _solve(lib, prm=drot.make_params(0.1, tol_mode=5)) == drot.EINVAL
    assert _solve(lib, prm=drot.make_params(0.1, x0_mode=3)) == drot.EINVAL
    assert _solve(lib, prm=drot.make_params(0.1, flags=0x80)) == drot.EINVAL
    assert _solve(lib, C=None) == drot.EINVAL
    assert _solve(lib, mu0=ctypes.c_void_p(8 * 77)) == drot.EINVAL  # nu0 missing
    assert "mu0 and nu0" in drot.last_error()
    # C and X overlapping
    assert _solve(lib, C=1, X=None) == drot.EINVAL
    # every argument valid: the NULL context is the first thing rejected
    assert _solve(lib) == drot.EINVAL
    assert "ctx" in drot.last_error()


def test_context_creation_reports_missing_device(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    from paper_2110_11738_amd import drot
    h = ctypes.c_void_p()
    assert lib.drot_ctx_create(ctypes.byref(h), 0) == drot.EDEVICE
    assert lib.drot_ctx_destroy(None) == drot.OK


def test_product_path_does_not_import_the_oracle():
    import subprocess
    import sys
    code = ("import sys; sys.path.insert(0, %r); import paper_2110_11738_amd, bench; "
            "from paper_2110_11738_amd import drot; drot.lib(); "
            "bad = [m for m in sys.modules if m == 'oracle' or m.startswith('oracle.')]; "
            "print(bad); assert not bad" % ROOT)
    subprocess.run([sys.executable, "-c", code], check=True, cwd=ROOT)


def test_cost_descriptor_validation_without_device(lib):
    from paper_2110_11738_amd import drot
    prm = drot.make_params(0.1, 1e-4, 100)
    res = drot.Result()

    def go(cost, dtype=0):
        return lib.drot_solve_cost(None, 4, 8, dtype, ctypes.byref(cost) if cost else None,
                                   4096 * 1000, 4096 * 2000, ctypes.byref(prm), 4096 * 5000, 8,
                                   None, None, None, None, ctypes.byref(res), None)
    assert go(None) == drot.EINVAL
    assert go(drot.Cost(7, 0, 4096, 8, None, None, 0.0)) == drot.EINVAL
    assert go(drot.Cost(drot.COST_COORDS, 5, None, 0, 4096, 8192, 0.0)) == drot.EINVAL
    assert go(drot.Cost(drot.COST_COORDS, 2, None, 0, None, 8192, 0.0)) == drot.EINVAL
    assert go(drot.Cost(drot.COST_COORDS, 2, None, 0, 4096, 8192, -1.0)) == drot.EINVAL
    assert go(drot.Cost(drot.COST_BF16, 0, 4096, 8, None, None, 0.0), dtype=1) == drot.EUNSUPPORTED
    assert go(drot.Cost(drot.COST_BF16, 0, 4096, 4, None, None, 0.0)) == drot.EINVAL  # ld < n
    # a valid descriptor reaches the context check
    assert go(drot.Cost(drot.COST_COORDS, 3, None, 0, 4096, 8192, 0.0)) == drot.EINVAL
    assert "ctx" in drot.last_error()


def test_noalloc_refuses_oversized_problem_before_device_work():
    """drot_solve_noalloc checks the workspace of the problem against its
    static scratch before any HIP call (here without a GPU): a 20000 x 20000
    problem is refused with DROT_EINVAL."""
    import ctypes
    from paper_2110_11738_amd import drot
    L = drot.lib()
    r = drot.Result()
    prm = drot.make_params(1e-5, 0.0, 10)
    vp = ctypes.c_void_p
    big = 20000
    rc = L.drot_solve_noalloc(big, big, drot.F32, vp(1 << 12), big, vp(1 << 44), vp(1 << 44),
                              ctypes.byref(prm), vp(1 << 40), big, None, None, None, None,
                              ctypes.byref(r), None)
    assert rc == drot.EINVAL
    assert "static scratch" in drot.last_error()
