"""GPU parity: every C-ABI entry point against the FP64 oracle on the same inputs.

Tolerances (normwise relative error ||gpu - oracle|| / ||oracle||, plus an
elementwise bound scaled by the largest oracle entry):
* FP64 mode: 1e-10.  Both sides compute in FP64; they differ only in the
  order of the sums (tiles, split-K partials), so the error is a small
  multiple of eps * sqrt(terms) ~ 1e-13.
* FP32 mode: 1e-5.  The oracle runs on the FP32-rounded inputs, so the gap is
  FP32 arithmetic alone: products accumulated over d or n terms in FP32.
Iterative results (PCG, Relax) are compared with the same probes and either
the same stopping rule (iteration counts must match) or a fixed number of
iterations on both sides.
"""
import os

import numpy as np
import pytest
import torch

from oracle import dense
from oracle import relax as orc
from paper_2409_07392_amd import FiralError, RelaxContext, _lib
from synthdata import make_problem, make_small

pytestmark = pytest.mark.gpu

DT = {"f64": torch.float64, "f32": torch.float32}
NPDT = {"f64": np.float64, "f32": np.float32}
TOL = {"f64": 1e-10, "f32": 1e-5}


def dev(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def rounded(a, prec):
    return np.asarray(a, dtype=NPDT[prec]).astype(np.float64)


def relerr(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def assert_close(got, ref, tol, what=""):
    e = relerr(got, ref)
    assert e <= tol, f"{what}: normwise relative error {e:.3e} > {tol:.1e}"
    scale = np.abs(ref).max() if ref.size else 1.0
    worst = np.abs(got - ref).max() if ref.size else 0.0
    assert worst <= 10 * tol * max(scale, 1e-300), f"{what}: max abs error {worst:.3e}"


def context(p, prec, s_max):
    X = rounded(p.X, prec)
    H = rounded(p.H, prec)
    ctx = RelaxContext(dev(X, DT[prec]), dev(H, DT[prec]), p.n_pool, s_max, prec)
    return ctx, X, H


SHAPES = [  # n_pool, n_lab, d, c, s
    (2000, 50, 20, 5, 10),     # configuration 1 shape
    (3001, 7, 100, 10, 20),    # configuration 2 shape, ragged n
    (517, 3, 37, 13, 3),       # nothing a multiple of a tile
    (300, 0, 1, 2, 1),         # degenerate d = 1, c = 2, s = 1, no labeled rows
    (1000, 10, 130, 33, 2),    # d over two 64-tiles
]


# --------------------------------------------------------------------- probes

@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_probes_bit_exact(prec):
    p = make_small(n=50, n_lab=1, d=13, c=7, s=5)
    ctx, _, _ = context(p, prec, 9)
    for seed, t, s in [(0, 1, 5), (2002, 3, 9), (2**64 - 5, 7, 1), (123456789, 100, 4)]:
        V = host(ctx.probes(seed, t, s))
        assert np.array_equal(V, orc.probes(seed, t, 13, s, 7)), (seed, t, s)


# ------------------------------------------------------------------------ hvp

@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("shape", SHAPES)
def test_hvp_matches_oracle(prec, shape):
    n, nl, d, c, s = shape
    p = make_small(n=n, n_lab=nl, d=d, c=c, s=s, seed=5)
    ctx, X, H = context(p, prec, s)
    rng = np.random.default_rng(1)
    B = rounded(rng.standard_normal((d, s, c)), prec)
    om = rng.uniform(0.0, 2.0, p.N)
    got = host(ctx.hvp(dev(B, DT[prec]), omega=dev(om, torch.float64), shift=0.25))
    assert_close(got, orc.hvp(X, H, om, 0.25, B), TOL[prec], f"hvp {prec} {shape}")
    # H_p: pool rows only, unit weights, no shift
    got = host(ctx.hvp(dev(B, DT[prec]), n_rows=n))
    assert_close(got, orc.hvp(X[:n], H[:n], None, 0.0, B), TOL[prec], f"H_p {prec} {shape}")


@pytest.mark.parametrize("unfused", ["0", "1", "ncb1"])
@pytest.mark.parametrize("shape", [(3001, 7, 100, 10, 20), (1200, 9, 256, 100, 5),
                                   (900, 3, 130, 33, 11), (650, 2, 20, 5, 10)])
def test_hvp_f32_fused_and_general_paths(shape, unfused, monkeypatch):
    # FIRAL_UNFUSED=1 forces the row-tiled product, ncb1 the fused kernel's one-block tiles
    # (next chunk fetched ahead); all must meet the FP32 bar
    monkeypatch.setenv("FIRAL_UNFUSED", "1" if unfused == "1" else "0")
    monkeypatch.setenv("FIRAL_FUSED_MAX_NCB", "1" if unfused == "ncb1" else "2")
    n, nl, d, c, s = shape
    p = make_small(n=n, n_lab=nl, d=d, c=c, s=s, seed=15)
    ctx, X, H = context(p, "f32", s)
    rng = np.random.default_rng(11)
    B = rounded(rng.choice([-1.0, 1.0], size=(d, s, c)), "f32")
    om = rng.uniform(0.0, 1.0, p.N)
    got = host(ctx.hvp(dev(B, torch.float32), omega=dev(om, torch.float64), shift=1e-3))
    assert_close(got, orc.hvp(X, H, om, 1e-3, B), TOL["f32"], f"hvp {shape} unfused={unfused}")
    got = host(ctx.hvp(dev(B[:, :1].copy(), torch.float32), n_rows=n))   # s = 1 < s_max
    assert_close(got, orc.hvp(X[:n], H[:n], None, 0.0, B[:, :1]), TOL["f32"], "s=1")


# Column modes of the row-tiled kernels (any d, c): whole probes per tile with short (c <= 32)
# or long segments, probes cut into column windows (c above the tile width), one-column last
# windows, d over many pipeline stages, and configuration 4's d and c.
TILED_SHAPES = [  # n_pool, n_lab, d, c, s
    (700, 5, 40, 300, 2),       # c > 128: three product windows, five gradient windows
    (400, 3, 70, 129, 3),       # a one-column last product window
    (350, 1, 24, 64, 3),        # two probes per product tile, one per gradient tile
    (520, 4, 33, 65, 2),        # a one-column last gradient window
    (300, 2, 300, 7, 17),       # 16 short probes per tile plus a ragged tile; 19 k-stages
    (1500, 10, 384, 1000, 2),   # configuration 4's d and c
]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("shape", TILED_SHAPES)
def test_tiled_hvp_and_grad(prec, shape, monkeypatch):
    monkeypatch.setenv("FIRAL_UNFUSED", "1")
    n, nl, d, c, s = shape
    p = make_small(n=n, n_lab=nl, d=d, c=c, s=s, seed=25)
    ctx, X, H = context(p, prec, s)
    rng = np.random.default_rng(21)
    B = rounded(rng.standard_normal((d, s, c)), prec)
    om = rng.uniform(0.0, 2.0, p.N)
    got = host(ctx.hvp(dev(B, DT[prec]), omega=dev(om, torch.float64), shift=0.5))
    assert_close(got, orc.hvp(X, H, om, 0.5, B), TOL[prec], f"hvp {prec} {shape}")
    got = host(ctx.hvp(dev(B, DT[prec]), n_rows=n))
    assert_close(got, orc.hvp(X[:n], H[:n], None, 0.0, B), TOL[prec], f"H_p {prec} {shape}")
    U = rounded(rng.choice([-1.0, 1.0], size=(d, s, c)), prec)
    g = host(ctx.grad_z(dev(U, DT[prec]), dev(B, DT[prec])))
    assert_close(g, orc.grad_contract(X[:n], H[:n], U, B), 10 * TOL[prec], f"grad {shape}")


def test_hvp_f32_full_configuration_2():
    # the bench workload at full size, in the launch configuration the bench times
    p = make_problem(2)
    ctx, X, H = context(p, "f32", p.s)
    V = ctx.probes(p.probe_seed, 1, p.s)
    om = np.concatenate([np.full(p.n_pool, p.b / p.n_pool), np.ones(p.n_lab)])
    got = host(ctx.hvp(V, omega=dev(om, torch.float64), shift=p.lam))
    ref = orc.hvp(X, H, om, p.lam, host(V))
    assert_close(got, ref, TOL["f32"], "hvp cfg2 full size")


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_hvp_row_chunks(prec, monkeypatch):
    monkeypatch.setenv("FIRAL_CHUNK_ROWS", "333")
    p = make_small(n=2100, n_lab=17, d=29, c=6, s=4, seed=9)
    ctx, X, H = context(p, prec, 4)
    B = rounded(np.random.default_rng(2).standard_normal((29, 4, 6)), prec)
    got = host(ctx.hvp(dev(B, DT[prec]), shift=0.5))
    assert_close(got, orc.hvp(X, H, None, 0.5, B), TOL[prec], "chunked hvp")


def test_hvp_no_rows_is_the_shift():
    p = make_small(n=20, n_lab=2, d=5, c=3, s=2)
    ctx, _, _ = context(p, "f64", 2)
    B = np.random.default_rng(3).standard_normal((5, 2, 3))
    got = host(ctx.hvp(dev(B, torch.float64), n_rows=0, shift=1.5))
    assert np.array_equal(got, 1.5 * B)


def test_hvp_is_deterministic():
    p = make_small(n=3001, n_lab=7, d=100, c=10, s=20, seed=4)
    ctx, _, _ = context(p, "f32", 20)
    B = dev(np.random.default_rng(4).standard_normal((100, 20, 10)), torch.float32)
    a = ctx.hvp(B, shift=0.1)
    b = ctx.hvp(B, shift=0.1)
    assert torch.equal(a, b)


# ------------------------------------------------------------- preconditioner

@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("shape", [(2000, 50, 20, 5), (3001, 7, 100, 10), (517, 3, 37, 13),
                                   (700, 4, 130, 3), (900, 2, 200, 2), (800, 1, 300, 2),
                                   (700, 2, 257, 2), (1000, 2, 384, 2), (1300, 3, 601, 2),
                                   (5000, 2, 1100, 2, 1.0), (6000, 2, 1201, 2, 1.0),
                                   (600, 3, 45, 40), (500, 5, 24, 70), (400, 2, 27, 130)])
def test_precond_matches_oracle(prec, shape):
    # class tiles of 32, 64 and 128 (the last ones partial), pair tiles cut by d; the factor
    # by the sweeps in registers (d <= 256), the global-memory sweep with 16-pivot panels
    # (d = 257: one pivot in its last panel; 300, 384) and 8-pivot panels (d = 601, 1100), and
    # the column-at-a-time factor (d = 1201).  Shift 1e-3 unless given: at d > 1000 it leaves
    # kappa(P_k) near 5e7, past FP32 (kappa u > 1: the FP32 Gram block is not SPD), so those
    # shapes take shift 1
    n, nl, d, c, *rest = shape
    shift = rest[0] if rest else 1e-3
    p = make_small(n=n, n_lab=nl, d=d, c=c, s=1, seed=6)
    ctx, X, H = context(p, prec, 1)
    om = np.random.default_rng(5).uniform(0.0, 1.0, p.N)
    L, Pinv, info = ctx.build_precond(dev(om, torch.float64), shift=shift)
    assert info["bad_block"] == -1
    P = orc.precond_blocks(X, H, om, shift)
    Lr, bad = orc.precond_factor(P)
    assert bad == -1
    L = host(L)
    assert np.all(np.triu(L, 1) == 0.0)
    # the block arithmetic (FP32 or FP64 SYRK) meets the precision's bar on P = L L^T; the
    # factor and the inverse move by up to kappa(P_k) times that (perturbation bounds)
    assert_close(L @ np.transpose(L, (0, 2, 1)), P, TOL[prec], "blocks L L^T")
    kappa = max(np.linalg.cond(Pk) for Pk in P)
    assert_close(L, Lr, TOL[prec] * max(1.0, kappa), "Cholesky factor")
    assert_close(host(Pinv), np.linalg.inv(P), TOL[prec] * max(10.0, 10 * kappa), "block inverse")


@pytest.mark.parametrize("wide", ["0", "1"])
@pytest.mark.parametrize("shape", [(2000, 50, 20, 70), (3001, 7, 100, 130), (1500, 3, 132, 300),
                                   (700, 2, 384, 65), (1500, 3, 384, 200)])
def test_precond_f32_gram_forms(shape, wide, monkeypatch):
    # c > 64, d a multiple of 4: the Gram kernel with its waves along the pairs (default) and the
    # classic tiling (FIRAL_GRAM_WIDE=0), one class tile with 64 row splits of 33 rows, two and
    # three class tiles with the last partial, a-blocks cut by d; d = 384, c = 200: 600
    # workgroups of the wide form, more than the 512 slots of a 256-CU device, so its row splits
    # are chosen by rounds (5 there); both at the FP32 bar
    monkeypatch.setenv("FIRAL_GRAM_WIDE", wide)
    n, nl, d, c = shape
    p = make_small(n=n, n_lab=nl, d=d, c=c, s=1, seed=33)
    ctx, X, H = context(p, "f32", 1)
    om = np.random.default_rng(34).uniform(0.0, 1.0, p.N)
    L, Pinv, info = ctx.build_precond(dev(om, torch.float64), shift=1e-3)
    assert info["bad_block"] == -1
    P = orc.precond_blocks(X, H, om, 1e-3)
    L = host(L)
    assert_close(L @ np.transpose(L, (0, 2, 1)), P, TOL["f32"], "blocks L L^T")
    _, Pinv1, info = ctx.build_precond(None, shift=1e-3, want_L=False)
    assert info["bad_block"] == -1
    P1 = orc.precond_blocks(X, H, np.ones(p.N), 1e-3)
    kappa1 = max(np.linalg.cond(Pk) for Pk in P1)
    assert_close(host(Pinv1), np.linalg.inv(P1), TOL["f32"] * max(10.0, 10 * kappa1),
                 "block inverse, unit weights")


@pytest.mark.parametrize("d", [6, 300])
@pytest.mark.parametrize("want_L", [True, False])
def test_precond_reports_non_spd_block(want_L, d):
    # want_L=False: the inverse alone (the blocked sweep for d <= 128); d = 300: the
    # global-memory sweep
    p = make_small(n=200 if d < 100 else 700, n_lab=3, d=d, c=4, s=1, seed=7)
    H = p.H.copy()
    H[:, 2] = 0.0
    ctx = RelaxContext(dev(p.X, torch.float64), dev(H, torch.float64), p.n_pool, 1, "f64")
    with pytest.raises(FiralError) as ei:
        ctx.build_precond(shift=0.0, want_L=want_L)
    assert ei.value.code == _lib.ENOTSPD


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("shape", [(2000, 50, 20, 5), (3001, 7, 100, 10), (517, 3, 37, 13),
                                   (777, 5, 128, 3), (600, 3, 45, 40), (300, 2, 1, 3),
                                   (800, 1, 300, 2), (1300, 3, 520, 2), (5000, 2, 1100, 2, 1.0)])
def test_precond_inverse_alone_matches_oracle(prec, shape):
    # without the factor, d <= 128 takes the blocked sweep in registers (16-pivot blocks;
    # d = 1, 37, 45: partial blocks padded with the identity, d = 128: eight full blocks), and
    # d = 300, 520 the global-memory sweep (16-pivot panels, the last one partial), d = 1100
    # its 8-pivot panels (the last one partial; shift 1, as in the test above)
    n, nl, d, c, *rest = shape
    shift = rest[0] if rest else 1e-3
    p = make_small(n=n, n_lab=nl, d=d, c=c, s=1, seed=8)
    ctx, X, H = context(p, prec, 1)
    om = np.random.default_rng(9).uniform(0.0, 1.0, p.N)
    L, Pinv, info = ctx.build_precond(dev(om, torch.float64), shift=shift, want_L=False)
    assert L is None and info["bad_block"] == -1
    P = orc.precond_blocks(X, H, om, shift)
    kappa = max(np.linalg.cond(Pk) for Pk in P)
    assert_close(host(Pinv), np.linalg.inv(P), TOL[prec] * max(10.0, 10 * kappa), "block inverse")


# ------------------------------------------------------------------------ pcg

@pytest.mark.parametrize("unfused", ["0", "1"])
@pytest.mark.parametrize("project", [True, False])
def test_pcg_f64_matches_oracle(project, unfused, monkeypatch):
    monkeypatch.setenv("FIRAL_UNFUSED", unfused)   # column-local CG step / separate kernels
    p = make_small(n=1500, n_lab=20, d=12, c=5, s=6, seed=8)
    ctx, X, H = context(p, "f64", 6)
    rng = np.random.default_rng(6)
    om = np.concatenate([rng.uniform(0, 0.02, p.n_pool), np.ones(p.n_lab)])
    B = rng.standard_normal((12, 6, 5))
    _, Pinv, _ = ctx.build_precond(dev(om, torch.float64), shift=1e-3)
    L, _ = orc.precond_factor(orc.precond_blocks(X, H, om, 1e-3))
    # same number of iterations on both sides: the same arithmetic sequence
    Xs, info = ctx.pcg_solve(dev(B, torch.float64), Pinv, omega=dev(om, torch.float64),
                             shift=1e-3, tol=0.0, max_iter=40, project=project)
    xr, it, _ = orc.pcg(X, H, om, 1e-3, L, B, 0.0, 40, project)
    assert info["cg_iters"][0] == it == 40
    # the two sides round in different orders; each CG iteration can move the iterate by
    # about kappa(A) u relative, so after k iterations the bar is max(1e-10, kappa u k): the
    # FP64 bar itself with the projection (kappa ~ 10 on the complement), 8e-10 without it
    # (kappa = 1.8e5: the lambda eigenspace)
    A = dense.sum_fisher(X, H, om) + 1e-3 * np.eye(12 * 5)
    ev = np.linalg.eigvalsh(A)
    kappa = ev[-1] / ev[0] if not project else 1.0
    bar = max(TOL["f64"], kappa * np.finfo(np.float64).eps / 2 * 40)
    e = relerr(host(Xs), xr)
    print(f"FP64 PCG iterate after 40 iterations (project={project}): rel err {e:.2e}, "
          f"bar {bar:.2e}")
    assert_close(host(Xs), xr, bar, "pcg iterate after 40 iterations")
    # stopping rule: with the projection (kappa ~ 10) the counts agree exactly; without it
    # (kappa ~ 1e4, the lambda eigenspace) finite-precision CG loses orthogonality and the
    # summation order moves the crossing of tol by a few percent of the count (113 against
    # 117 has been seen), and the two solutions agree to about kappa * tol.
    Xs, info = ctx.pcg_solve(dev(B, torch.float64), Pinv, omega=dev(om, torch.float64),
                             shift=1e-3, tol=1e-9, max_iter=2000, project=project)
    xr, it, rr = orc.pcg(X, H, om, 1e-3, L, B, 1e-9, 2000, project)
    assert info["rc"] == 0 and info["converged"]
    assert info["relres_max"] <= 1e-9
    if project:
        assert info["cg_iters"][0] == it
        assert_close(host(Xs), xr, TOL["f64"], "pcg solution")
    else:
        # both sides stop with ||r|| <= tol ||b||, so their solutions differ by at most
        # 2 kappa(A) tol relative to the solution (A = sum omega_i H_i + shift I, 2-norm)
        assert abs(info["cg_iters"][0] - it) <= max(3, 0.05 * it)
        A = dense.sum_fisher(X, H, om) + 1e-3 * np.eye(12 * 5)
        ev = np.linalg.eigvalsh(A)
        bar = 2.0 * (ev[-1] / ev[0]) * 1e-9
        e = relerr(host(Xs), xr)
        print(f"literal PCG at tol 1e-9: rel diff {e:.2e}, kappa-derived bar {bar:.2e}")
        assert e <= bar, (e, bar)


@pytest.mark.parametrize("unfused", ["0", "1"])
def test_pcg_f32_fixed_iterations(unfused, monkeypatch):
    monkeypatch.setenv("FIRAL_UNFUSED", unfused)
    p = make_small(n=3001, n_lab=7, d=100, c=10, s=20, seed=10, whiten_x=True, probs="maxprob")
    ctx, X, H = context(p, "f32", 20)
    rng = np.random.default_rng(7)
    om = np.concatenate([np.full(p.n_pool, 100.0 / p.n_pool), np.ones(p.n_lab)])
    B = rounded(rng.choice([-1.0, 1.0], size=(100, 20, 10)), "f32")
    _, Pinv, _ = ctx.build_precond(dev(om, torch.float64), shift=1e-3)
    Xs, info = ctx.pcg_solve(dev(B, torch.float32), Pinv, omega=dev(om, torch.float64),
                             shift=1e-3, tol=0.0, max_iter=12, project=True)
    assert info["cg_iters"][0] == 12
    L, _ = orc.precond_factor(orc.precond_blocks(X, H, om, 1e-3))
    xr, _, _ = orc.pcg(X, H, om, 1e-3, L, B, 0.0, 12, True)
    e = relerr(host(Xs), xr)
    print(f"FP32 PCG iterate after 12 iterations: rel err {e:.2e}")
    assert e <= TOL["f32"], e


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("shape", [(1500, 10, 600, 5, 6), (2600, 4, 2100, 2, 3)])
def test_pcg_apply_groups_large_d(prec, shape):
    # d c > 2340: the separate-kernel CG step, with the preconditioner applied in groups of 4
    # probes (512 < d <= 2048; s = 6: a full and a partial group) and of 2 (d > 2048; s = 3).
    # Shift 1 and small pool weights keep the spectrum of A in [1, ~c x 260] (the blocks' kappa is
    # at most ~260), so the rounding drift after 8 iterations, about kappa u k < 1e-12, stays
    # under the FP64 bar
    n, nl, d, c, s = shape
    p = make_small(n=n, n_lab=nl, d=d, c=c, s=s, seed=40)
    ctx, X, H = context(p, prec, s)
    rng = np.random.default_rng(41)
    om = np.concatenate([rng.uniform(0, 0.02, p.n_pool), np.ones(p.n_lab)])
    B = rounded(rng.standard_normal((d, s, c)), prec)
    _, Pinv, _ = ctx.build_precond(dev(om, torch.float64), shift=1.0)
    Xs, info = ctx.pcg_solve(dev(B, DT[prec]), Pinv, omega=dev(om, torch.float64), shift=1.0,
                             tol=0.0, max_iter=8, project=True)
    assert info["cg_iters"][0] == 8
    L, _ = orc.precond_factor(orc.precond_blocks(X, H, om, 1.0))
    xr, it, _ = orc.pcg(X, H, om, 1.0, L, B, 0.0, 8, True)
    assert it == 8
    assert_close(host(Xs), xr, TOL[prec], f"pcg iterate after 8 iterations {prec} {shape}")


@pytest.mark.parametrize("unfused", ["0", "1"])
def test_pcg_breakdown_and_not_converged(unfused, monkeypatch):
    monkeypatch.setenv("FIRAL_UNFUSED", unfused)
    p = make_small(n=300, n_lab=3, d=4, c=3, s=2, seed=11)
    ctx, _, _ = context(p, "f64", 2)
    _, Pinv, _ = ctx.build_precond(shift=1.0)
    B = dev(np.random.default_rng(8).standard_normal((4, 2, 3)), torch.float64)
    with pytest.raises(FiralError) as ei:
        ctx.pcg_solve(B, Pinv, shift=-1e4, tol=1e-8, max_iter=50)
    assert ei.value.code == _lib.EBREAKDOWN
    _, info = ctx.pcg_solve(B, Pinv, shift=1e-3, tol=1e-14, max_iter=1)
    assert info["rc"] == _lib.WARN_NOT_CONVERGED and not info["converged"]
    assert info["cg_iters"][0] == 1


# ----------------------------------------------------------------------- grad

@pytest.mark.parametrize("unfused", ["0", "1"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("shape", SHAPES)
def test_grad_matches_oracle(prec, shape, unfused, monkeypatch):
    # FP32 with d <= 128: the fused one-pass gradient, or (FIRAL_UNFUSED=1) the row-tiled passes
    monkeypatch.setenv("FIRAL_UNFUSED", unfused)
    n, nl, d, c, s = shape
    p = make_small(n=n, n_lab=nl, d=d, c=c, s=s, seed=12)
    ctx, X, H = context(p, prec, s)
    rng = np.random.default_rng(9)
    U = rounded(rng.choice([-1.0, 1.0], size=(d, s, c)), prec)
    W = rounded(rng.standard_normal((d, s, c)), prec)
    g = host(ctx.grad_z(dev(U, DT[prec]), dev(W, DT[prec])))
    assert_close(g, orc.grad_contract(X[:n], H[:n], U, W), 10 * TOL[prec], f"grad {shape}")


# ---------------------------------------------------------------------- relax

@pytest.mark.parametrize("unfused", ["0", "1"])
def test_relax_f64_trajectory_matches_oracle(unfused, monkeypatch):
    monkeypatch.setenv("FIRAL_UNFUSED", unfused)
    p = make_problem(1)
    ctx, X, H = context(p, "f64", p.s)
    beta0 = orc.default_beta0(p.n_pool, p.T)
    w = torch.full((p.n_pool,), 1.0 / p.n_pool, dtype=torch.float64, device="cuda")
    g = torch.empty_like(w)
    wr = np.full(p.n_pool, 1.0 / p.n_pool)
    for t in range(1, 4):
        info = ctx.relax_step(w, p.b, p.lam, beta0, p.probe_seed, t, p.s, p.tol, 1000,
                              project=True, g_out=g)
        wr, ir = orc.relax_iteration(X, H, p.n_pool, wr, p.b, p.lam, beta0, p.probe_seed, t, p.s,
                                     p.tol, 1000, project=True)
        assert info["cg_iters"] == ir["cg_iters"], t
        assert abs(info["f_hat"] - ir["f_hat"]) <= TOL["f64"] * abs(ir["f_hat"])
        assert abs(info["g_absmax"] - ir["g_absmax"]) <= TOL["f64"] * ir["g_absmax"]
        assert_close(host(g), ir["g"], TOL["f64"], f"gradient t={t}")
        assert_close(host(w), wr, TOL["f64"], f"weights t={t}")
    wh = host(w)
    assert abs(wh.sum() - 1.0) < 1e-12 and np.all(wh > 0)


def test_relax_literal_mode_f64():
    p = make_small(n=400, n_lab=5, d=6, c=4, s=4, seed=13)
    ctx, X, H = context(p, "f64", 4)
    w0 = np.full(p.n_pool, 1.0 / p.n_pool)
    # fixed CG count: identical sequence of operations on both sides
    w = torch.full((p.n_pool,), 1.0 / p.n_pool, dtype=torch.float64, device="cuda")
    info = ctx.relax_step(w, 5.0, 1e-3, 0.3, 77, 1, 4, 0.0, 60, project=False)
    wr, ir = orc.relax_iteration(X, H, p.n_pool, w0, 5.0, 1e-3, 0.3, 77, 1, 4, 0.0, 60,
                                 project=False)
    assert info["cg_iters"] == ir["cg_iters"] == (60, 60)
    e = relerr(host(w), wr)
    print(f"literal Relax step at 60 fixed CG iterations: weights rel err {e:.2e}")
    assert_close(host(w), wr, TOL["f64"], "weights (literal, 60 CG iterations)")
    # tolerance-based stop (kappa ~ 1e4 here): counts within 3, weights close
    w = torch.full((p.n_pool,), 1.0 / p.n_pool, dtype=torch.float64, device="cuda")
    info = ctx.relax_step(w, 5.0, 1e-3, 0.3, 77, 1, 4, 1e-8, 3000, project=False)
    wr, ir = orc.relax_iteration(X, H, p.n_pool, w0, 5.0, 1e-3, 0.3, 77, 1, 4, 1e-8, 3000,
                                 project=False)
    assert all(abs(a - b) <= 3 for a, b in zip(info["cg_iters"], ir["cg_iters"]))
    assert relerr(host(w), wr) <= 1e-6


def test_relax_not_spd_leaves_weights():
    p = make_small(n=200, n_lab=0, d=5, c=3, s=2, seed=14)
    H = p.H.copy()
    H[:, 1] = 0.0
    ctx = RelaxContext(dev(p.X, torch.float64), dev(H, torch.float64), p.n_pool, 2, "f64")
    w0 = torch.full((p.n_pool,), 1.0 / p.n_pool, dtype=torch.float64, device="cuda")
    w = w0.clone()
    with pytest.raises(FiralError) as ei:
        ctx.relax_step(w, 5.0, 0.0, 0.3, 1, 1, 2, 1e-8, 100)
    assert ei.value.code == _lib.ENOTSPD
    assert torch.equal(w, w0)


def test_relax_f32_gradient_error_fixed_iterations():
    # FP32 against the FP64 oracle with the same probes and the same fixed CG count
    p = make_problem(2, n=5000)
    ctx, X, H = context(p, "f32", p.s)
    beta0 = orc.default_beta0(p.n_pool, p.T)
    w = torch.full((p.n_pool,), 1.0 / p.n_pool, dtype=torch.float64, device="cuda")
    g = torch.empty_like(w)
    info = ctx.relax_step(w, p.b, p.lam, beta0, p.probe_seed, 1, p.s, 0.0, 15, project=True,
                          g_out=g)
    wr, ir = orc.relax_iteration(X, H, p.n_pool, np.full(p.n_pool, 1.0 / p.n_pool), p.b, p.lam,
                                 beta0, p.probe_seed, 1, p.s, 0.0, 15, project=True)
    assert info["cg_iters"] == (15, 15)
    e = relerr(host(g), ir["g"])
    print(f"FP32 Relax gradient at 15 CG iterations: rel err {e:.2e}")
    assert e <= TOL["f32"], e
    assert abs(info["f_hat"] - ir["f_hat"]) <= TOL["f32"] * abs(ir["f_hat"])
    assert relerr(host(w), wr) <= TOL["f32"]


# -------------------------------------------------------------------- bf16x3
# Each FP32 product is taken as hi*hi + hi*lo + lo*hi of bf16 halves (FP32 sums): the
# dropped lo*lo term and the rounding of lo leave ~2^-16 relative error per product, so
# the bar for these results is 1e-4 normwise (the gradient gate of the metric).

BF3_TOL = 1e-4


@pytest.mark.parametrize("ncb", ["1", "2"])
@pytest.mark.parametrize("shape", [(3001, 7, 100, 10, 20), (650, 2, 20, 5, 10), (900, 3, 37, 13, 3),
                                   (300, 0, 1, 2, 1)])
def test_hvp_bf16x3(shape, ncb, monkeypatch):
    monkeypatch.setenv("FIRAL_FUSED_MAX_NCB", ncb)
    n, nl, d, c, s = shape
    p = make_small(n=n, n_lab=nl, d=d, c=c, s=s, seed=17, whiten_x=True, probs="maxprob")
    X = rounded(p.X, "f32")
    H = rounded(p.H, "f32")
    ctx = RelaxContext(dev(X, torch.float32), dev(H, torch.float32), p.n_pool, s, "bf16x3")
    rng = np.random.default_rng(19)
    for B in (rng.choice([-1.0, 1.0], size=(d, s, c)), rounded(rng.standard_normal((d, s, c)), "f32")):
        om = rng.uniform(0.0, 1.0, p.N)
        got = host(ctx.hvp(dev(B, torch.float32), omega=dev(om, torch.float64), shift=1e-3))
        ref = orc.hvp(X, H, om, 1e-3, B)
        assert relerr(got, ref) <= BF3_TOL, relerr(got, ref)


@pytest.mark.parametrize("gram3", ["0", "1"])
@pytest.mark.parametrize("shape", [(2000, 50, 20, 70), (3001, 7, 100, 130), (1500, 3, 132, 300),
                                   (700, 2, 384, 65), (1500, 3, 384, 200), (517, 3, 37, 70),
                                   (600, 3, 44, 40)])
def test_precond_bf16x3_matches_oracle(shape, gram3, monkeypatch):
    # FIRAL_BF3_GRAM=1 with c > 64 and d a multiple of 4: the Gram blocks as bf16x3 products (one
    # class tile with 64 row splits of 33 rows; two and three class tiles, the last partial;
    # a-blocks cut by d); d = 37, c = 40 and the default keep the FP32 Gram in the bf16x3
    # context.  Blocks at the bf16x3 bar, factor and inverse within kappa(P_k) times it
    monkeypatch.setenv("FIRAL_BF3_GRAM", gram3)
    n, nl, d, c = shape
    p = make_small(n=n, n_lab=nl, d=d, c=c, s=1, seed=31)
    X = rounded(p.X, "f32")
    H = rounded(p.H, "f32")
    ctx = RelaxContext(dev(X, torch.float32), dev(H, torch.float32), p.n_pool, 1, "bf16x3")
    om = np.random.default_rng(32).uniform(0.0, 1.0, p.N)
    L, Pinv, info = ctx.build_precond(dev(om, torch.float64), shift=1e-3)
    assert info["bad_block"] == -1
    P = orc.precond_blocks(X, H, om, 1e-3)
    Lr, bad = orc.precond_factor(P)
    assert bad == -1
    L = host(L)
    assert np.all(np.triu(L, 1) == 0.0)
    assert_close(L @ np.transpose(L, (0, 2, 1)), P, BF3_TOL, "blocks L L^T")
    kappa = max(np.linalg.cond(Pk) for Pk in P)
    assert_close(L, Lr, BF3_TOL * max(1.0, kappa), "Cholesky factor")
    assert_close(host(Pinv), np.linalg.inv(P), BF3_TOL * max(10.0, 10 * kappa), "block inverse")
    # without row weights (omega = 1): the kernel's unit-weight path
    _, Pinv1, info = ctx.build_precond(None, shift=1e-3, want_L=False)
    assert info["bad_block"] == -1
    P1 = orc.precond_blocks(X, H, np.ones(p.N), 1e-3)
    kappa1 = max(np.linalg.cond(Pk) for Pk in P1)
    assert_close(host(Pinv1), np.linalg.inv(P1), BF3_TOL * max(10.0, 10 * kappa1),
                 "block inverse, unit weights")


@pytest.mark.parametrize("chunk", [None, "333"])
@pytest.mark.parametrize("shape", TILED_SHAPES)
def test_tiled_bf16x3_hvp_and_grad(shape, chunk, monkeypatch):
    # the row-tiled kernels with split products (FIRAL_UNFUSED=1 keeps small shapes off the
    # fused kernel): every column mode, one chunk or chunks of 320 rows, against the FP64
    # oracle at the bf16x3 bar
    monkeypatch.setenv("FIRAL_UNFUSED", "1")
    if chunk:
        monkeypatch.setenv("FIRAL_CHUNK_ROWS", chunk)
    n, nl, d, c, s = shape
    p = make_small(n=n, n_lab=nl, d=d, c=c, s=s, seed=27, whiten_x=True, probs="maxprob")
    X = rounded(p.X, "f32")
    H = rounded(p.H, "f32")
    ctx = RelaxContext(dev(X, torch.float32), dev(H, torch.float32), p.n_pool, s, "bf16x3")
    rng = np.random.default_rng(23)
    B = rounded(rng.standard_normal((d, s, c)), "f32")
    om = rng.uniform(0.0, 1.0, p.N)
    got = host(ctx.hvp(dev(B, torch.float32), omega=dev(om, torch.float64), shift=1e-3))
    e = relerr(got, orc.hvp(X, H, om, 1e-3, B))
    assert e <= BF3_TOL, ("hvp", e)
    U = rng.choice([-1.0, 1.0], size=(d, s, c))
    g = host(ctx.grad_z(dev(U, torch.float32), dev(B, torch.float32)))
    e = relerr(g, orc.grad_contract(X[:n], H[:n], U, B))
    assert e <= BF3_TOL, ("grad", e)


def test_relax_bf16x3_gradient_error_fixed_iterations():
    p = make_problem(2, n=5000)
    X = rounded(p.X, "f32")
    H = rounded(p.H, "f32")
    ctx = RelaxContext(dev(X, torch.float32), dev(H, torch.float32), p.n_pool, p.s, "bf16x3")
    beta0 = orc.default_beta0(p.n_pool, p.T)
    w = torch.full((p.n_pool,), 1.0 / p.n_pool, dtype=torch.float64, device="cuda")
    g = torch.empty_like(w)
    info = ctx.relax_step(w, p.b, p.lam, beta0, p.probe_seed, 1, p.s, 0.0, 15, project=True,
                          g_out=g)
    _, ir = orc.relax_iteration(X, H, p.n_pool, np.full(p.n_pool, 1.0 / p.n_pool), p.b, p.lam,
                                beta0, p.probe_seed, 1, p.s, 0.0, 15, project=True)
    assert info["cg_iters"] == (15, 15)
    e = relerr(host(g), ir["g"])
    assert e <= BF3_TOL, e


# ------------------------------------------------------------- wide FP32 path
# d > 128 (a multiple of 4) and c > 128 in an FP32 context: the transposed-operand GEMMs with the
# row step split between the first kernel's epilogue (alpha per column window) and the second
# kernel's staging.  Shapes: configuration 4's d and c; d with a 4-deep last stage (132); a
# one-column last window (c = 129); ragged rows and several chunks (FIRAL_CHUNK_ROWS, rounded
# down to 32 rows); H_p over the pool rows only (the labeled rows follow in the same chunk).
NT_SHAPES = [  # n_pool, n_lab, d, c, s, chunk rows
    (1500, 10, 384, 1000, 2, None),
    (900, 7, 132, 129, 3, None),
    (777, 3, 260, 300, 5, "320"),
    (2050, 14, 136, 257, 1, "100"),
    (1100, 6, 520, 140, 2, "400"),    # five 128-row output tiles
]


@pytest.mark.parametrize("shape", NT_SHAPES)
def test_wide_fp32_product_matches_oracle(shape, monkeypatch):
    n, nl, d, c, s, chunk = shape
    if chunk:
        monkeypatch.setenv("FIRAL_CHUNK_ROWS", chunk)
    p = make_small(n=n, n_lab=nl, d=d, c=c, s=s, seed=33, whiten_x=True, probs="maxprob")
    ctx, X, H = context(p, "f32", s)
    rng = np.random.default_rng(34)
    B = rounded(rng.standard_normal((d, s, c)), "f32")
    om = rng.uniform(0.0, 2.0, p.N)
    got = host(ctx.hvp(dev(B, torch.float32), omega=dev(om, torch.float64), shift=0.5))
    assert_close(got, orc.hvp(X, H, om, 0.5, B), TOL["f32"], f"wide hvp {shape}")
    got = host(ctx.hvp(dev(B, torch.float32), n_rows=n))
    assert_close(got, orc.hvp(X[:n], H[:n], None, 0.0, B), TOL["f32"], f"wide H_p {shape}")
    # the same call twice: bitwise identical (fixed-order sums)
    a = ctx.hvp(dev(B, torch.float32), shift=0.5)
    b = ctx.hvp(dev(B, torch.float32), shift=0.5)
    assert torch.equal(a, b)


def test_wide_fp32_relax_step_matches_oracle():
    p = make_small(n=2000, n_lab=9, d=132, c=130, s=3, seed=35, whiten_x=True, probs="maxprob")
    ctx, X, H = context(p, "f32", p.s)
    w = torch.full((p.n_pool,), 1.0 / p.n_pool, dtype=torch.float64, device="cuda")
    g = torch.empty_like(w)
    info = ctx.relax_step(w, 20.0, 1e-3, 0.4, 7, 1, p.s, 0.0, 12, project=True, g_out=g)
    assert info["cg_iters"] == (12, 12)
    wr, ir = orc.relax_iteration(X, H, p.n_pool, np.full(p.n_pool, 1.0 / p.n_pool), 20.0, 1e-3,
                                 0.4, 7, 1, p.s, 0.0, 12, project=True)
    e = relerr(host(g), ir["g"])
    print(f"wide FP32 Relax step at 12 CG iterations: gradient rel err {e:.2e}")
    assert e <= TOL["f32"], e
    assert relerr(host(w), wr) <= TOL["f32"]


NT3_SHAPES = [  # n_pool, n_lab, d, c, s, chunk rows: d a multiple of 8 for the bf16x3 form
    (1500, 10, 384, 1000, 2, None),   # second contraction over all output rows (d <= 384)
    (900, 7, 136, 129, 3, None),
    (777, 3, 264, 300, 5, "320"),
    (2050, 14, 136, 257, 1, "100"),
    (1100, 6, 520, 140, 2, "400"),    # d > 384: one workgroup per 128-row output tile
]


@pytest.mark.parametrize("shape", NT3_SHAPES)
def test_wide_bf16x3_product_matches_oracle(shape, monkeypatch):
    # the bf16x3 form of the wide path (X from the context's hi/lo planes in both layouts, V^T
    # split once per call, G' split while staged) at the bf16x3 bar
    n, nl, d, c, s, chunk = shape
    if chunk:
        monkeypatch.setenv("FIRAL_CHUNK_ROWS", chunk)
    p = make_small(n=n, n_lab=nl, d=d, c=c, s=s, seed=36, whiten_x=True, probs="maxprob")
    X = rounded(p.X, "f32")
    H = rounded(p.H, "f32")
    ctx = RelaxContext(dev(X, torch.float32), dev(H, torch.float32), p.n_pool, s, "bf16x3")
    rng = np.random.default_rng(37)
    B = rounded(rng.standard_normal((d, s, c)), "f32")
    om = rng.uniform(0.0, 2.0, p.N)
    got = host(ctx.hvp(dev(B, torch.float32), omega=dev(om, torch.float64), shift=0.5))
    e = relerr(got, orc.hvp(X, H, om, 0.5, B))
    assert e <= BF3_TOL, ("hvp", shape, e)
    got = host(ctx.hvp(dev(B, torch.float32), n_rows=n))
    e = relerr(got, orc.hvp(X[:n], H[:n], None, 0.0, B))
    print(f"wide bf16x3 {shape}: H_p rel err {e:.2e}")
    assert e <= BF3_TOL, ("H_p", shape, e)


def test_wide_bf16x3_relax_step_matches_oracle():
    p = make_small(n=2000, n_lab=9, d=136, c=130, s=3, seed=38, whiten_x=True, probs="maxprob")
    X = rounded(p.X, "f32")
    H = rounded(p.H, "f32")
    ctx = RelaxContext(dev(X, torch.float32), dev(H, torch.float32), p.n_pool, p.s, "bf16x3")
    w = torch.full((p.n_pool,), 1.0 / p.n_pool, dtype=torch.float64, device="cuda")
    g = torch.empty_like(w)
    info = ctx.relax_step(w, 20.0, 1e-3, 0.4, 7, 1, p.s, 0.0, 12, project=True, g_out=g)
    assert info["cg_iters"] == (12, 12)
    wr, ir = orc.relax_iteration(X, H, p.n_pool, np.full(p.n_pool, 1.0 / p.n_pool), 20.0, 1e-3,
                                 0.4, 7, 1, p.s, 0.0, 12, project=True)
    e = relerr(host(g), ir["g"])
    print(f"wide bf16x3 Relax step at 12 CG iterations: gradient rel err {e:.2e}")
    assert e <= BF3_TOL, e


def test_wide_bf16x3_gram_relax_step_to_tolerance(monkeypatch):
    # the bf16x3 Gram blocks (FIRAL_BF3_GRAM=1) change the preconditioner by ~1e-5 relative: PCG
    # run to a tolerance on both sides reaches the same gradient at the bf16x3 bar
    monkeypatch.setenv("FIRAL_BF3_GRAM", "1")
    p = make_small(n=2000, n_lab=9, d=136, c=130, s=3, seed=38, whiten_x=True, probs="maxprob")
    X = rounded(p.X, "f32")
    H = rounded(p.H, "f32")
    ctx = RelaxContext(dev(X, torch.float32), dev(H, torch.float32), p.n_pool, p.s, "bf16x3")
    w = torch.full((p.n_pool,), 1.0 / p.n_pool, dtype=torch.float64, device="cuda")
    g = torch.empty_like(w)
    info = ctx.relax_step(w, 20.0, 1e-3, 0.4, 7, 1, p.s, 1e-6, 400, project=True, g_out=g)
    wr, ir = orc.relax_iteration(X, H, p.n_pool, np.full(p.n_pool, 1.0 / p.n_pool), 20.0, 1e-3,
                                 0.4, 7, 1, p.s, 1e-6, 400, project=True)
    e = relerr(host(g), ir["g"])
    print(f"wide bf16x3 Relax step, bf16x3 Gram, PCG to 1e-6: CG {info['cg_iters']} "
          f"(oracle {ir.get('cg_iters')}), gradient rel err {e:.2e}")
    assert e <= BF3_TOL, e
