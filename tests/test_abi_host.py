"""Host-side checks of the C ABI: the library loads, exports every declared symbol, and its
pure host logic (workspace sizing, defaults, argument validation that fails before any
device work) behaves as documented. No kernel is launched here."""
import ctypes
import os
import re

import pytest

from paper_1611_03220_amd import krr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "krr.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(krr_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    L = krr.lib()
    names = _declared()
    assert set(names) >= {"krr_features", "krr_precond_factor", "krr_kernel_matmat",
                          "krr_pcg_solve", "krr_grad", "krr_workspace_bytes", "krr_last_error"}
    for name in names:
        assert hasattr(L, name), name
    assert set(krr.EXPORTED) <= set(names)


def test_version_and_defaults():
    assert "gfx950" in krr.version()
    o = krr.PCGOpts()
    krr.lib().krr_pcg_defaults(ctypes.byref(o))
    assert (o.tol, o.max_iter, o.prec, o.use_precond, o.check_every, o.lambda_p,
            o.true_residual, o.refine, o.warm_start) == (1e-6, 1000, 1, 1, 1, 0.0, 1, 0, 0)


def test_workspace_sizes_scale_sensibly():
    ws = krr.workspace_bytes
    a = ws(krr.OP_KERNEL_MATMAT, 1000, 1000, 54, 0, 7, 1)
    b = ws(krr.OP_KERNEL_MATMAT, 4000, 4000, 54, 0, 7, 1)
    assert 0 < a < b
    # mixed points: 4 split arrays of rows_pad x 64 halves at least
    assert b >= 4 * 4032 * 64 * 2
    assert ws(krr.OP_PCG_SOLVE, 65536, 65536, 54, 2048, 7, 1) > 65536 * 7 * 8 * 6
    assert ws(krr.OP_PRECOND_FACTOR, 65536, 65536, 0, 2048, 0, 1) > 2 * 2048 * 65536 * 2
    assert ws(krr.OP_FEATURES, 100, 100, 8, 20, 0, 1) > 0
    assert ws(99, 10, 10, 1, 1, 1, 1) == 0


def test_argument_validation_before_device_work():
    L = krr.lib()
    null = None
    # null pointers
    st = L.krr_kernel_matmat(null, 10, 3, null, 10, 3, 3, 1.0, 0.0, null, 1, 1, null, 1, 0, 1,
                             null, 0, null)
    assert st == krr.E_ARG and "null" in krr.last_error()
    fake = ctypes.c_void_p(256)  # never dereferenced: validation fails first
    # sigma <= 0
    st = L.krr_kernel_matmat(fake, 10, 3, fake, 10, 3, 3, 0.0, 0.0, fake, 1, 1, fake, 1, 0, 1,
                             fake, 1 << 30, null)
    assert st == krr.E_ARG and "sigma" in krr.last_error()
    # shift with n1 != n2
    st = L.krr_kernel_matmat(fake, 10, 3, fake, 11, 3, 3, 1.0, 0.5, fake, 1, 1, fake, 1, 0, 1,
                             fake, 1 << 30, null)
    assert st == krr.E_ARG and "shift" in krr.last_error()
    # unknown precision
    st = L.krr_kernel_matmat(fake, 10, 3, fake, 10, 3, 3, 1.0, 0.0, fake, 1, 1, fake, 1, 0, 9,
                             fake, 1 << 30, null)
    assert st == krr.E_ARG
    # workspace too small / misaligned
    st = L.krr_kernel_matmat(fake, 10, 3, fake, 10, 3, 3, 1.0, 0.0, fake, 1, 1, fake, 1, 0, 1,
                             fake, 16, null)
    assert st == krr.E_WORKSPACE
    st = L.krr_kernel_matmat(fake, 10, 3, fake, 10, 3, 3, 1.0, 0.0, fake, 1, 1, fake, 1, 0, 1,
                             ctypes.c_void_p(257), 1 << 30, null)
    assert st == krr.E_WORKSPACE
    # pcg: lambda <= 0, tol <= 0, s >= n
    o = krr.PCGOpts()
    L.krr_pcg_defaults(ctypes.byref(o))
    st = L.krr_pcg_solve(fake, 10, 3, 3, 1.0, 0.0, fake, 4, 4, fake, 1, fake, 1, 1,
                         ctypes.byref(o), None, fake, 1 << 30, null)
    assert st == krr.E_ARG and "lambda" in krr.last_error()
    o.tol = 0.0
    st = L.krr_pcg_solve(fake, 10, 3, 3, 1.0, 1.0, fake, 4, 4, fake, 1, fake, 1, 1,
                         ctypes.byref(o), None, fake, 1 << 30, null)
    assert st == krr.E_ARG and "tol" in krr.last_error()
    o.tol = 1e-6
    st = L.krr_pcg_solve(fake, 10, 3, 3, 1.0, 1.0, fake, 10, 10, fake, 1, fake, 1, 1,
                         ctypes.byref(o), None, fake, 1 << 30, null)
    assert st == krr.E_ARG and "s < n" in krr.last_error()
    info = ctypes.c_int64(7)
    st = L.krr_precond_factor(fake, 10, 10, 10, 1.0, fake, fake, 10, fake, 1 << 30,
                              ctypes.byref(info), null)
    assert st == krr.E_ARG and info.value == 0
    st = L.krr_precond_factor(fake, 10, 4, 4, -1.0, fake, fake, 4, fake, 1 << 30,
                              ctypes.byref(info), null)
    assert st == krr.E_ARG and "lambda_p" in krr.last_error()
    # dimension limit of the BF16X3 (VALU-accumulate) product
    st = L.krr_kernel_matmat(fake, 10, 300, fake, 10, 300, 300, 1.0, 0.0, fake, 1, 1, fake, 1, 0,
                             2, fake, 1 << 40, null)
    assert st == krr.E_ARG and "254" in krr.last_error()


def test_python_binding_rejects_host_tensors():
    import torch
    with pytest.raises(TypeError):
        krr.kernel_matmat(torch.zeros(4, 2), torch.zeros(4, 2), 1.0, torch.zeros(4, 1, dtype=torch.float64))
