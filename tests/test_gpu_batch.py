"""Extension (2): the kernel-variant tuner and graph-captured batches of Relax problems.

A batch replays one captured Relax iteration of every problem; each problem's weights after
every replay must equal those of the same number of ordinary firal_relax_step calls on a
second context with the same tuned variants (same kernels, same order: equal up to the last
bit, checked at 1e-12), and a small FP64 batch must follow the oracle's trajectory.
"""
import numpy as np
import pytest
import torch

from oracle import relax as orc
from paper_2409_07392_amd import FiralError, RelaxBatch, RelaxContext, default_beta0
from synthdata import make_small

pytestmark = pytest.mark.gpu

SHAPES = [  # n_pool, n_lab, d, c, s: uneven problems
    (1500, 5, 24, 10, 8),
    (700, 3, 70, 33, 4),
    (3000, 9, 40, 5, 16),
    (900, 2, 130, 130, 2),
    (2200, 4, 16, 64, 6),
]


def dev(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def problem(i, shape, prec):
    n, nl, d, c, s = shape
    p = make_small(n=n, n_lab=nl, d=d, c=c, s=s, seed=40 + i, whiten_x=True, probs="maxprob")
    dt = torch.float64 if prec == "f64" else torch.float32
    X = np.asarray(p.X, dtype=np.float32).astype(np.float64)
    H = np.asarray(p.H, dtype=np.float32).astype(np.float64)
    return p, X, H, dt


def test_autotune_choice_is_cached_and_keeps_parity():
    p, X, H, dt = problem(0, (3001, 7, 100, 10, 20), "f32")
    ctx = RelaxContext(dev(X, dt), dev(H, dt), p.n_pool, p.s, "f32")
    ch = ctx.autotune()
    # a fused tiling (column blocks per wave, workgroup target 256 << k, k <= 2) or row-tiled
    assert 0 <= ch < 32 and (ch >> 3) <= 2 and not (ch & 1 and ch & (4 | 24))
    assert ctx.autotune() == ch
    rng = np.random.default_rng(2)
    B = rng.standard_normal((p.d, p.s, p.c)).astype(np.float32).astype(np.float64)
    got = ctx.hvp(dev(B, dt), shift=1e-3).cpu().numpy().astype(np.float64)
    ref = orc.hvp(X, H, None, 1e-3, B)
    assert np.linalg.norm(got - ref) <= 1e-5 * np.linalg.norm(ref)


def test_autotune_on_a_wide_shape_keeps_parity():
    # d > 128 and c > 128: no fused tiling fits; the tuner times the context's default (wide)
    # path against the row-tiled kernels and the product keeps the FP32 bar either way
    p, X, H, dt = problem(3, (1500, 10, 136, 257, 2), "f32")
    ctx = RelaxContext(dev(X, dt), dev(H, dt), p.n_pool, p.s, "f32")
    ch = ctx.autotune()
    assert ch & ~3 == 0   # no fused bits: the default path (0) or the row-tiled one (1)
    rng = np.random.default_rng(4)
    B = rng.standard_normal((p.d, p.s, p.c)).astype(np.float32).astype(np.float64)
    got = ctx.hvp(dev(B, dt), shift=1e-3).cpu().numpy().astype(np.float64)
    ref = orc.hvp(X, H, None, 1e-3, B)
    assert np.linalg.norm(got - ref) <= 1e-5 * np.linalg.norm(ref)


@pytest.mark.parametrize("prec", ["f32", "bf16x3"])
def test_batch_replays_equal_sequential_steps(prec):
    T = 3
    probs, refs = [], []
    for i, shape in enumerate(SHAPES):
        p, X, H, dt = problem(i, shape, prec)
        a = RelaxContext(dev(X, dt), dev(H, dt), p.n_pool, p.s, prec)
        b = RelaxContext(dev(X, dt), dev(H, dt), p.n_pool, p.s, prec)
        wa = torch.full((p.n_pool,), 1.0 / p.n_pool, dtype=torch.float64, device="cuda")
        wb = wa.clone()
        beta0 = default_beta0(p.n_pool, 30)
        probs.append(dict(ctx=a, w=wa, b=p.b, lam=1e-3, beta0=beta0, seed=p.probe_seed, t0=1,
                          s=p.s, tol=1e-6, max_iter=60, project=True))
        refs.append((b, wb, p, beta0))
    batch = RelaxBatch(probs)
    for _, (b, wb, p, _) in zip(probs, refs):
        b.autotune(p.s)   # same bucket: the batch context's tuned variants
    for k in range(T):
        batch.run(1)
        torch.cuda.synchronize()
        for i, (q, (b, wb, p, beta0)) in enumerate(zip(probs, refs)):
            info = b.relax_step(wb, p.b, 1e-3, beta0, p.probe_seed, k + 1, p.s, 1e-6, 60,
                                project=True)
            bi = batch.info(i)
            assert bi["cg_iters"] == info["cg_iters"], (i, k)
            diff = (q["w"] - wb).abs().max().item()
            assert diff <= 1e-12 * wb.abs().max().item(), (i, k, diff)
            assert abs(q["w"].sum().item() - 1.0) < 1e-12
    for i in range(len(probs)):
        assert batch.next_t(i) == T + 1
    batch.close()


def test_batch_f64_follows_the_oracle():
    shapes = [(600, 3, 12, 4, 5), (900, 5, 20, 6, 3)]
    probs, data = [], []
    for i, shape in enumerate(shapes):
        p, X, H, dt = problem(10 + i, shape, "f64")
        ctx = RelaxContext(dev(X, dt), dev(H, dt), p.n_pool, p.s, "f64")
        w = torch.full((p.n_pool,), 1.0 / p.n_pool, dtype=torch.float64, device="cuda")
        beta0 = default_beta0(p.n_pool, 10)
        probs.append(dict(ctx=ctx, w=w, b=p.b, lam=1e-3, beta0=beta0, seed=p.probe_seed, t0=1,
                          s=p.s, tol=0.0, max_iter=30, project=True))
        data.append((p, X, H, beta0))
    batch = RelaxBatch(probs)
    batch.run(2)
    torch.cuda.synchronize()
    for q, (p, X, H, beta0) in zip(probs, data):
        w = np.full(p.n_pool, 1.0 / p.n_pool)
        for t in (1, 2):
            w, _ = orc.relax_iteration(X, H, p.n_pool, w, p.b, 1e-3, beta0, p.probe_seed, t, p.s,
                                       0.0, 30, project=True)
        got = q["w"].cpu().numpy()
        assert np.abs(got - w).max() <= 1e-9 * np.abs(w).max()
    batch.close()


def test_batch_rejects_a_shared_context():
    p, X, H, dt = problem(20, (300, 2, 8, 3, 2), "f32")
    ctx = RelaxContext(dev(X, dt), dev(H, dt), p.n_pool, p.s, "f32")
    w1 = torch.full((p.n_pool,), 1.0 / p.n_pool, dtype=torch.float64, device="cuda")
    w2 = w1.clone()
    q = dict(ctx=ctx, b=p.b, lam=1e-3, beta0=0.1, seed=1)
    with pytest.raises(FiralError):
        RelaxBatch([dict(q, w=w1), dict(q, w=w2)])
