"""The allocation-free Hessian product (firal_hvp_noalloc) against firal_hvp.

firal_hvp_noalloc runs the same fused FP32 kernels as a context's firal_hvp, with the partial
sums in the library's fixed device array instead of the context's workspace, so its output
must equal firal_hvp's bit for bit (and so meet the FP32 bar against the oracle, which
firal_hvp's own tests check).  Two calls in a row on one device, the second with a smaller
input, show that the array's contents left by a call do not leak into the next.
"""
import ctypes

import numpy as np
import pytest
import torch

from oracle import relax as orc
from paper_2409_07392_amd import RelaxContext, _lib
from synthdata import make_small

pytestmark = pytest.mark.gpu


def _noalloc(lib, X, H, omega, shift, B, out):
    N, d = X.shape
    c = H.shape[1]
    s = B.shape[1]
    rc = lib.firal_hvp_noalloc(X.data_ptr(), H.data_ptr(), N, d, c,
                               None if omega is None else omega.data_ptr(), float(shift),
                               B.data_ptr(), out.data_ptr(), s,
                               torch.cuda.current_stream().cuda_stream)
    return rc


def test_noalloc_product_equals_the_context_product_twice():
    lib = _lib.load()
    # the second call is smaller in every dimension (rows, d, c, s)
    for n, nl, d, c, s, seed in [(3001, 7, 100, 10, 20, 31), (517, 3, 37, 13, 3, 32)]:
        p = make_small(n=n, n_lab=nl, d=d, c=c, s=s, seed=seed)
        Xh = np.asarray(p.X, np.float32)
        Hh = np.asarray(p.H, np.float32)
        X = torch.as_tensor(Xh, device="cuda").contiguous()
        H = torch.as_tensor(Hh, device="cuda").contiguous()
        rng = np.random.default_rng(seed)
        Bh = rng.standard_normal((d, s, c)).astype(np.float32)
        B = torch.as_tensor(Bh, device="cuda").contiguous()
        om = torch.as_tensor(rng.uniform(0.0, 2.0, p.N), device="cuda")
        ctx = RelaxContext(X, H, p.n_pool, s, "f32")
        ref = ctx.hvp(B, omega=om, shift=0.25)
        out = torch.full_like(B, float("nan"))
        assert _noalloc(lib, X, H, om, 0.25, B, out) == 0, lib.firal_last_error().decode()
        torch.cuda.synchronize()
        assert torch.equal(out, ref), (n, d, c, s)
        # and the FP32 bar against the oracle
        want = orc.hvp(Xh.astype(np.float64), Hh.astype(np.float64), om.cpu().numpy(), 0.25,
                       Bh.astype(np.float64))
        got = out.cpu().numpy().astype(np.float64)
        assert np.linalg.norm(got - want) <= 1e-5 * np.linalg.norm(want)
        ctx.close()


def test_noalloc_no_rows_and_refusals():
    lib = _lib.load()
    d, s, c = 8, 2, 3
    X = torch.zeros(4, d, device="cuda")
    H = torch.full((4, c), 1.0 / c, device="cuda")
    B = torch.randn(d, s, c, device="cuda")
    out = torch.empty_like(B)
    rc = lib.firal_hvp_noalloc(X.data_ptr(), H.data_ptr(), 0, d, c, None, 1.5, B.data_ptr(),
                               out.data_ptr(), s, torch.cuda.current_stream().cuda_stream)
    assert rc == 0
    torch.cuda.synchronize()
    assert torch.equal(out, (1.5 * B.double()).float())
    # d above the fused kernel's range
    assert lib.firal_hvp_noalloc(1, 1, 10, 200, 3, None, 0.0, 1, 2, 1, None) == _lib.ENOTSUP
