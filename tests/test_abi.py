"""C-ABI contract tests that run without a GPU.

The library must load, export every function include/firal.h declares, and
reject bad arguments with FIRAL_EINVAL before any device work; without a
device, a well-formed firal_create must fail with FIRAL_EHIP (not crash).
"""
import ctypes
import os
import re

import pytest

from paper_2409_07392_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "firal.h")


def header_functions():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|double|const char\*)\s+(firal_\w+)\s*\(", txt, re.M)))


def test_header_declares_the_binding_exports():
    assert header_functions() == sorted(_lib.EXPORTS)


def test_library_loads_and_exports_every_declared_symbol():
    lib = _lib.load()
    for name in header_functions():
        assert hasattr(lib, name), name
    # the ELF dynamic symbol table has them as global functions
    out = os.popen(f"nm -D --defined-only {_lib.LIB_PATH}").read()
    for name in header_functions():
        assert re.search(rf"\bT {name}\b", out), name


def test_strerror_covers_codes():
    lib = _lib.load()
    for code in (0, 1, -1, -2, -3, -4, -5, -6):
        assert lib.firal_strerror(code).decode() != "unknown return code"
    assert lib.firal_strerror(-99).decode() == "unknown return code"


def _create(lib, **kw):
    args = dict(n_pool=10, n_lab=2, d=4, c=3, s_max=2, prec=1, X=1, H=1)
    args.update(kw)
    ctx = ctypes.c_void_p()
    rc = lib.firal_create(ctypes.byref(ctx), args["n_pool"], args["n_lab"], args["d"], args["c"],
                          args["s_max"], args["prec"], args["X"], args["H"], None)
    return rc, ctx


@pytest.mark.parametrize("bad", [dict(n_pool=0), dict(n_lab=-1), dict(d=0), dict(c=1),
                                 dict(s_max=0), dict(prec=7), dict(X=None), dict(H=None)])
def test_create_rejects_bad_arguments(bad):
    lib = _lib.load()
    rc, ctx = _create(lib, **bad)
    assert rc == _lib.EINVAL
    assert ctx.value is None
    assert lib.firal_last_error().decode() != ""


def test_create_null_output_pointer():
    lib = _lib.load()
    assert lib.firal_create(None, 10, 0, 4, 3, 2, 1, 1, 1, None) == _lib.EINVAL


def test_calls_reject_null_context():
    lib = _lib.load()
    info = _lib.Info()
    assert lib.firal_hvp(None, None, 1, 0.0, 1, 2, 1, None) == _lib.EINVAL
    assert lib.firal_build_precond(None, None, 0.0, None, None, ctypes.byref(info), None) == _lib.EINVAL
    assert lib.firal_pcg_solve(None, None, 0.0, 1, 1, 2, 1, 1e-6, 10, 0, ctypes.byref(info),
                               None) == _lib.EINVAL
    assert lib.firal_grad_z(None, 1, 2, 1, 3, None) == _lib.EINVAL
    assert lib.firal_probes(None, 1, 1, 1, 1, None) == _lib.EINVAL
    assert lib.firal_relax_step(None, 1, 1.0, 1e-3, 0.1, 1, 1, 1, 1e-6, 10, 0, None,
                                ctypes.byref(info), None) == _lib.EINVAL
    it = ctypes.c_int32()
    assert lib.firal_relax_solve(None, 1.0, 1e-3, -1.0, 1, 5, 1, 1e-6, 10, 0, 0.0, 1, None,
                                 None, ctypes.byref(it), ctypes.byref(info), None) == _lib.EINVAL
    best = ctypes.c_int32()
    etas = (ctypes.c_double * 2)(1.0, 2.0)
    assert lib.firal_round_eta_sweep(None, 1, 1e-3, etas, 2, 3, 0, 1, None, ctypes.byref(best),
                                     None) == _lib.EINVAL
    assert lib.firal_destroy(None) == _lib.OK


def test_noalloc_product_refuses_before_any_device_call():
    # argument errors and partial sums beyond the fixed device array are found on the host
    lib = _lib.load()
    assert lib.firal_hvp_noalloc(None, 1, 10, 8, 3, None, 0.0, 1, 2, 1, None) == _lib.EINVAL
    assert lib.firal_hvp_noalloc(1, 1, 10, 8, 3, None, 0.0, 1, 1, 1, None) == _lib.EINVAL
    assert lib.firal_hvp_noalloc(1, 1, 10, 200, 3, None, 0.0, 1, 2, 1, None) == _lib.ENOTSUP
    # d = 128, c = 128: one probe per tile, so s = 4096 probes need 4096 x 128 x 128 floats
    rc = lib.firal_hvp_noalloc(1, 1, 100000, 128, 128, None, 0.0, 1, 2, 4096, None)
    assert rc == _lib.EINVAL
    assert "fixed device array" in lib.firal_last_error().decode()


def test_default_beta0_is_the_entropic_mirror_descent_step():
    # sqrt(2 ln n / T) (host arithmetic only; no device needed)
    import math
    lib = _lib.load()
    for n, T in [(2000, 50), (50000, 100), (1, 1), (1280000, 20)]:
        assert lib.firal_default_beta0(n, T) == pytest.approx(math.sqrt(2 * math.log(n) / T),
                                                              rel=1e-15, abs=0)
    assert lib.firal_default_beta0(0, 5) == 0.0


def test_create_without_device_reports_hip_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    lib = _lib.load()
    rc, ctx = _create(lib)
    assert rc == _lib.EHIP
    assert ctx.value is None


def test_binding_refuses_cpu_tensors():
    import torch
    from paper_2409_07392_amd import RelaxContext
    X = torch.zeros(5, 3, dtype=torch.float32)
    H = torch.full((5, 2), 0.5, dtype=torch.float32)
    with pytest.raises(ValueError):
        RelaxContext(X, H, n_pool=4, s_max=2, prec="f32")
