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


def test_dsigma_inner_validation_before_device_work():
    L = krr.lib()
    fake = ctypes.c_void_p(256)
    out = ctypes.c_double(7.0)
    st = L.krr_kernel_dsigma_inner(None, 10, 3, fake, 12, 3, 3, 1.0, fake, 2, 2, fake, 2,
                                   ctypes.byref(out), 0, fake, 1 << 30, None)
    assert st == krr.E_ARG and "null" in krr.last_error()
    st = L.krr_kernel_dsigma_inner(fake, 10, 3, fake, 12, 3, 3, -1.0, fake, 2, 2, fake, 2,
                                   ctypes.byref(out), 0, fake, 1 << 30, None)
    assert st == krr.E_ARG and "sigma" in krr.last_error()
    st = L.krr_kernel_dsigma_inner(fake, 10, 3, fake, 12, 3, 3, 1.0, fake, 2, 1, fake, 2,
                                   ctypes.byref(out), 0, fake, 1 << 30, None)
    assert st == krr.E_ARG
    st = L.krr_kernel_dsigma_inner(fake, 10, 3, fake, 12, 3, 3, 1.0, fake, 2, 2, fake, 2,
                                   ctypes.byref(out), 0, fake, 64, None)
    assert st == krr.E_WORKSPACE and out.value == 7.0
    a = krr.workspace_bytes(krr.OP_DSIGMA_INNER, 1000, 3000, 54, 0, 7, 0)
    b = krr.workspace_bytes(krr.OP_DSIGMA_INNER, 1000, 6000, 54, 0, 7, 0)
    assert 0 < a < b


def test_python_binding_rejects_host_tensors():
    import torch
    with pytest.raises(TypeError):
        krr.kernel_matmat(torch.zeros(4, 2), torch.zeros(4, 2), 1.0, torch.zeros(4, 1, dtype=torch.float64))


def _c_layout(struct, fields):
    """sizeof and offsetof of a header struct, compiled with gcc against include/krr.h."""
    import subprocess
    import tempfile
    body = "\n".join(f'  printf("%zu\\n", offsetof({struct}, {f}));' for f in fields)
    src = (f'#include <stddef.h>\n#include <stdio.h>\n#include "krr.h"\nint main(void) {{\n'
           f'  printf("%zu\\n", sizeof({struct}));\n{body}\n  return 0;\n}}\n')
    with tempfile.TemporaryDirectory() as d:
        c, exe = os.path.join(d, "l.c"), os.path.join(d, "l")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout.split()
    return [int(v) for v in out]


@pytest.mark.parametrize("struct,cls", [("krr_pcg_opts", krr.PCGOpts),
                                        ("krr_pcg_report", krr.PCGReport),
                                        ("krr_batch_problem", krr.BatchProblem),
                                        ("krr_batch_report", krr.BatchReport),
                                        ("krr_kernel", krr.Kernel),
                                        ("krr_precond_test_report", krr.PrecondTestReport)])
def test_binding_structs_match_header_layout(struct, cls):
    names = [f[0] for f in cls._fields_]
    cnames = ["lambda" if n == "lam" else n for n in names]
    got = _c_layout(struct, cnames)
    assert got[0] == ctypes.sizeof(cls)
    assert got[1:] == [getattr(cls, n).offset for n in names]


def test_precond_apply_validation_before_device_work():
    L = krr.lib()
    fake = ctypes.c_void_p(256)
    other = ctypes.c_void_p(512)
    st = L.krr_precond_apply(fake, 10, 10, 10, 1.0, other, 1, 1, fake, 1, fake, 1 << 30, None)
    assert st == krr.E_ARG and "s < n" in krr.last_error()
    st = L.krr_precond_apply(fake, 10, 4, 4, 0.0, other, 1, 1, fake, 1, fake, 1 << 30, None)
    assert st == krr.E_ARG and "lambda_p" in krr.last_error()
    st = L.krr_precond_apply(fake, 10, 4, 4, 1.0, other, 2, 1, fake, 2, fake, 1 << 30, None)
    assert st == krr.E_ARG
    st = L.krr_precond_apply(fake, 10, 4, 4, 1.0, other, 1, 1, other, 1, fake, 1 << 30, None)
    assert st == krr.E_ARG and "alias" in krr.last_error()
    st = L.krr_precond_apply(fake, 10, 4, 4, 1.0, other, 1, 1, fake, 1, fake, 8, None)
    assert st == krr.E_WORKSPACE
    assert krr.workspace_bytes(krr.OP_PRECOND_APPLY, 65536, 65536, 0, 2048, 7, 0) > 2048 * 7 * 8


def test_batch_plan_validation_before_device_work():
    L = krr.lib()
    fake = ctypes.c_void_p(256)
    probs = (krr.BatchProblem * 2)()
    for p in probs:
        p.X, p.n, p.d, p.ldx, p.sigma, p.lam = fake, 100, 3, 3, 1.0, 1.0
        p.Y, p.ldy, p.alpha, p.lda, p.m = fake, 2, fake, 2, 2
    o = krr.PCGOpts()
    L.krr_pcg_defaults(ctypes.byref(o))
    h = ctypes.c_void_p(None)
    probs[1].m, probs[1].ldy, probs[1].lda = 17, 17, 17
    st = L.krr_batch_plan_create(probs, 2, ctypes.byref(o), ctypes.byref(h), None)
    assert st == krr.E_ARG and "problem 1" in krr.last_error() and not h
    probs[1].m, probs[1].ldy, probs[1].lda = 2, 2, 2
    probs[0].sigma = -1.0
    st = L.krr_batch_plan_create(probs, 2, ctypes.byref(o), ctypes.byref(h), None)
    assert st == krr.E_ARG and "sigma" in krr.last_error()
    probs[0].sigma = 1.0
    probs[0].Ut, probs[0].s, probs[0].ldu = fake, 100, 100
    st = L.krr_batch_plan_create(probs, 2, ctypes.byref(o), ctypes.byref(h), None)
    assert st == krr.E_ARG and "s < n" in krr.last_error()
    probs[0].Ut = None
    o.prec = 0
    st = L.krr_batch_plan_create(probs, 2, ctypes.byref(o), ctypes.byref(h), None)
    assert st == krr.E_ARG and "F16X3" in krr.last_error()
    o.prec = 1
    st = L.krr_batch_plan_create(probs, 0, ctypes.byref(o), ctypes.byref(h), None)
    assert st == krr.E_ARG
    st = L.krr_batch_solve(None, None, None)
    assert st == krr.E_ARG
    L.krr_batch_plan_destroy(None)


def test_kernel_descriptor_validation_before_device_work():
    L = krr.lib()
    fake = ctypes.c_void_p(256)
    null = None

    def mm(k, prec=1, deriv=0):
        return L.krr_kernel_matmat_k(ctypes.byref(k) if k is not None else None, fake, 10, 3, fake,
                                     10, 3, 3, 0.0, fake, 1, 1, fake, 1, deriv, prec, fake, 1 << 30,
                                     null)
    assert mm(None) == krr.E_ARG and "descriptor" in krr.last_error()
    assert mm(krr.Kernel.gaussian(-1.0)) == krr.E_ARG and "sigma" in krr.last_error()
    assert mm(krr.Kernel.polynomial(1.0, 1.0, 0)) == krr.E_ARG and "degree" in krr.last_error()
    assert mm(krr.Kernel.polynomial(1.0, 1.0, 17)) == krr.E_ARG
    assert mm(krr.Kernel.polynomial(-0.5, 1.0, 2)) == krr.E_ARG and "gamma" in krr.last_error()
    assert mm(krr.Kernel.polynomial(1.0, float("nan"), 2)) == krr.E_ARG
    assert mm(krr.Kernel.polynomial(1.0, 1.0, 2), prec=2) == krr.E_ARG and "F16X3" in krr.last_error()
    assert mm(krr.Kernel.polynomial(1.0, 1.0, 2), deriv=1) == krr.E_ARG and "deriv" in krr.last_error()
    k = krr.Kernel(7, 1, 1.0, 0.0, 0.0)
    assert mm(k) == krr.E_ARG and "kind" in krr.last_error()
    o = krr.PCGOpts()
    L.krr_pcg_defaults(ctypes.byref(o))
    st = L.krr_pcg_solve_k(None, fake, 10, 3, 3, 1.0, fake, 4, 4, fake, 1, fake, 1, 1,
                           ctypes.byref(o), None, fake, 1 << 30, null)
    assert st == krr.E_ARG and "descriptor" in krr.last_error()
    o.prec = 2
    st = L.krr_pcg_solve_k(ctypes.byref(krr.Kernel.polynomial(1.0, 1.0, 3)), fake, 10, 3, 3, 1.0,
                           fake, 4, 4, fake, 1, fake, 1, 1, ctypes.byref(o), None, fake, 1 << 30, null)
    assert st == krr.E_ARG and "F16X3" in krr.last_error()


def test_tensorsketch_validation_before_device_work():
    L = krr.lib()
    fake = ctypes.c_void_p(256)
    ts = L.krr_tensorsketch
    assert ts(None, 10, 3, 3, 1.0, 1.0, 2, fake, fake, 64, fake, 64, None) == krr.E_ARG
    assert ts(fake, 10, 3, 3, 1.0, 1.0, 2, fake, fake, 48, fake, 64, None) == krr.E_ARG
    assert "power of two" in krr.last_error()
    assert ts(fake, 10, 3, 3, 1.0, 1.0, 2, fake, fake, 16384, fake, 16384, None) == krr.E_ARG
    assert ts(fake, 10, 3, 3, 1.0, 1.0, 0, fake, fake, 64, fake, 64, None) == krr.E_ARG
    assert ts(fake, 10, 3, 3, -1.0, 1.0, 2, fake, fake, 64, fake, 64, None) == krr.E_ARG
    assert ts(fake, 10, 3, 3, 1.0, 1.0, 2, fake, fake, 64, fake, 32, None) == krr.E_ARG


def test_tune_cache_round_trip(tmp_path):
    """The tuning table's file: entries written for this build's digest read back; a file of
    another build (digest) or architecture is ignored."""
    dg = krr.tune_digest()
    assert dg and dg != "unversioned"
    src = tmp_path / "tune.json"
    src.write_text('{"arch": "gfx950", "digest": "%s", "entries": [\n'
                   '  [1, 0, 64, 3, 16, 4, 0, 1.500000, 1.400000],\n'
                   '  [0, 0, 800, 4, 18, 8, 32, 420.0, 400.0]\n]}\n' % dg)
    krr.tune_cache_clear()
    assert krr.tune_cache_size() == 0
    assert krr.tune_cache_load(str(src))
    assert krr.tune_cache_size() == 2
    out = tmp_path / "out.json"
    assert krr.tune_cache_save(str(out))
    krr.tune_cache_clear()
    assert krr.tune_cache_load(str(out)) and krr.tune_cache_size() == 2
    txt = out.read_text()
    assert "[1, 0, 64, 3, 16, 4, 0, 1.500000, 1.400000]" in txt and dg in txt
    krr.tune_cache_clear()
    other = tmp_path / "other.json"
    other.write_text(txt.replace(dg, "0000000000000000"))
    assert not krr.tune_cache_load(str(other)) and krr.tune_cache_size() == 0
    assert not krr.tune_cache_load(str(tmp_path / "missing.json"))
    krr.tune_cache_clear()
