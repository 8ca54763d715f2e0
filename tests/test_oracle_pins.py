"""Pins of the FP64 oracle against things other than itself.

Each test checks one oracle function against a brute force that forms the
Fisher matrices with np.kron (eq. 2), a closed form, a published value, an
exact special case (a complete Hadamard probe set), finite differences, or an
invariant.  All CPU; tiny shapes.
"""
import math
import os

import numpy as np
import pytest

from oracle import dense
from oracle import relax as orc
from synthdata import make_small

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def tiny(n=9, n_lab=3, d=3, c=4, s=3, seed=3):
    return make_small(n=n, n_lab=n_lab, d=d, c=c, s=s, seed=seed)


def dense_apply(S, B):
    d, s, c = B.shape
    return orc.vecs_to_block(S @ orc.block_to_vecs(B), d, c)


# --------------------------------------------------------------------- probes

def test_splitmix64_published_outputs():
    vals = [int(l, 16) for l in open(os.path.join(GOLDEN, "splitmix64_seed0.txt"))
            if l.strip() and not l.startswith("#")]
    got = [int(v) for v in orc.splitmix64_stream(0, 3)]
    assert got == vals


def test_probes_are_signs_balanced_and_continue_across_iterations():
    d, s, c = 7, 5, 3
    V = orc.probes(123, 1, d, s, c)
    assert set(np.unique(V)) <= {-1.0, 1.0}
    big = orc.probes(99, 1, 16, 64, 16)
    assert abs(big.mean()) < 0.02
    # iteration t draws the counters right after iteration t-1's: the probes of
    # t = 1..3 with s probes equal those of t = 1 with 3s probes.
    cat = np.concatenate([orc.probes(5, t, d, s, c) for t in (1, 2, 3)], axis=1)
    assert np.array_equal(cat, orc.probes(5, 1, d, 3 * s, c))
    assert not np.array_equal(orc.probes(5, 1, d, s, c), orc.probes(5, 2, d, s, c))


# ------------------------------------------------------------------------ hvp

@pytest.mark.parametrize("shape", [(9, 3, 3, 4, 3), (12, 0, 5, 2, 2), (6, 2, 1, 3, 4)])
def test_hvp_equals_dense_kronecker(shape):
    n, nl, d, c, s = shape
    p = make_small(n=n, n_lab=nl, d=d, c=c, s=s, seed=11)
    rng = np.random.default_rng(0)
    omega = rng.uniform(0.1, 2.0, p.N)
    B = rng.standard_normal((d, s, c))
    S = dense.sum_fisher(p.X, p.H, omega) + 0.37 * np.eye(d * c)
    np.testing.assert_allclose(orc.hvp(p.X, p.H, omega, 0.37, B), dense_apply(S, B),
                               rtol=1e-12, atol=1e-12)


def test_hvp_row_chunks_do_not_change_the_sum():
    p = tiny(n=40, n_lab=5)
    B = np.random.default_rng(1).standard_normal((p.d, p.s, p.c))
    a = orc.hvp(p.X, p.H, None, 0.0, B)
    b = orc.hvp(p.X, p.H, None, 0.0, B, row_chunk=7)
    np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-12)


def test_hvp_annihilates_class_constant_vectors_and_is_symmetric():
    p = tiny()
    rng = np.random.default_rng(2)
    u = rng.standard_normal((p.d, p.s, 1)) * np.ones((1, 1, p.c))   # 1_c (x) u
    assert np.abs(orc.hvp(p.X, p.H, None, 0.0, u)).max() < 1e-12
    A = rng.standard_normal((p.d, p.s, p.c))
    B = rng.standard_normal((p.d, p.s, p.c))
    om = rng.uniform(0, 1, p.N)
    np.testing.assert_allclose(orc.col_dot(A, orc.hvp(p.X, p.H, om, 0.1, B)),
                               orc.col_dot(B, orc.hvp(p.X, p.H, om, 0.1, A)), rtol=1e-11)


# -------------------------------------------------------------- preconditioner

def test_precond_blocks_are_the_dense_block_diagonal():
    p = tiny(n=11, d=4, c=3)
    z = np.random.default_rng(3).uniform(0, 1, p.n_pool)
    S = dense.sigma(p.X, p.H, p.n_pool, z, 0.2)
    om = np.concatenate([z, np.ones(p.n_lab)])
    np.testing.assert_allclose(orc.precond_blocks(p.X, p.H, om, 0.2),
                               dense.block_diagonal(S, p.d, p.c), rtol=1e-12, atol=1e-12)


def test_precond_factor_reconstructs_and_reports_bad_block():
    p = tiny(n=30, d=4, c=3)
    P = orc.precond_blocks(p.X, p.H, None, 1e-3)
    L, bad = orc.precond_factor(P)
    assert bad == -1
    np.testing.assert_allclose(L @ np.transpose(L, (0, 2, 1)), P, rtol=1e-12, atol=1e-12)
    assert np.all(np.triu(L, 1) == 0.0)
    H = p.H.copy()
    H[:, 1] = 0.0                       # class 1 never predicted: its block is the zero matrix
    _, bad = orc.precond_factor(orc.precond_blocks(p.X, H, None, 0.0))
    assert bad == 1
    R = np.random.default_rng(4).standard_normal((p.d, 2, p.c))
    Z = orc.precond_apply(L, R)
    for k in range(p.c):
        np.testing.assert_allclose(P[k] @ Z[:, :, k], R[:, :, k], rtol=1e-10, atol=1e-12)


# ------------------------------------------------------------------------ pcg

@pytest.mark.parametrize("project", [False, True])
def test_pcg_matches_dense_solve(project):
    p = tiny(n=25, n_lab=4, d=3, c=4, s=3)
    rng = np.random.default_rng(5)
    z = rng.uniform(0.1, 1, p.n_pool)
    om = np.concatenate([z, np.ones(p.n_lab)])
    S = dense.sigma(p.X, p.H, p.n_pool, z, 1e-2)
    L, _ = orc.precond_factor(orc.precond_blocks(p.X, p.H, om, 1e-2))
    B = rng.standard_normal((p.d, p.s, p.c))
    x, it, rr = orc.pcg(p.X, p.H, om, 1e-2, L, B, 1e-13, 500, project)
    rhs = orc.project_perp(B) if project else B
    ref = orc.vecs_to_block(np.linalg.solve(S, orc.block_to_vecs(rhs)), p.d, p.c)
    np.testing.assert_allclose(x, ref, rtol=1e-9, atol=1e-9 * np.abs(ref).max())
    assert rr.max() <= 1e-13
    assert it <= 4 * p.d * p.c
    # tol = 0 runs exactly max_iter iterations
    _, it0, _ = orc.pcg(p.X, p.H, om, 1e-2, L, B, 0.0, 3, project)
    assert it0 == 3


def test_pcg_reports_breakdown_on_indefinite_operator():
    p = tiny()
    L, _ = orc.precond_factor(orc.precond_blocks(p.X, p.H, None, 1.0))
    B = np.random.default_rng(6).standard_normal((p.d, p.s, p.c))
    with pytest.raises(orc.PCGBreakdown):
        orc.pcg(p.X, p.H, None, -50.0, L, B, 1e-10, 50)


# -------------------------------------------------------- exact dense gradient

def test_dense_gradient_matches_finite_differences():
    p = tiny(n=8, n_lab=3, d=3, c=3)
    z = np.random.default_rng(7).uniform(0.2, 1.0, p.n_pool)
    g = dense.exact_gradient(p.X, p.H, p.n_pool, z, 1e-2)
    h = 1e-5
    for i in range(p.n_pool):
        e = np.zeros(p.n_pool)
        e[i] = h
        fd = (dense.objective(p.X, p.H, p.n_pool, z + e, 1e-2)
              - dense.objective(p.X, p.H, p.n_pool, z - e, 1e-2)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i]))
    assert np.all(g <= 0)


def test_two_class_reduces_to_binary_design_formula():
    p = make_small(n=10, n_lab=3, d=3, c=2, s=2, seed=21)
    z = np.random.default_rng(8).uniform(0.1, 1, p.n_pool)
    lam = 1e-2
    # h = (p, 1-p): Gamma = 2p(1-p) e e^T with e = (1,-1)/sqrt(2), so Sigma and H_p act as
    # S + lam and S_p on the e-direction (weights 2p(1-p)) and as lam on the other one.
    wgt = 2 * p.H[:, 0] * (1 - p.H[:, 0])
    S = sum(wgt[i] * np.outer(p.X[i], p.X[i]) * (z[i] if i < p.n_pool else 1.0)
            for i in range(p.N)) + lam * np.eye(p.d)
    Sp = sum(wgt[i] * np.outer(p.X[i], p.X[i]) for i in range(p.n_pool))
    Si = np.linalg.inv(S)
    f_ref = np.trace(Si @ Sp)
    g_ref = np.array([-wgt[i] * p.X[i] @ Si @ Sp @ Si @ p.X[i] for i in range(p.n_pool)])
    assert abs(dense.objective(p.X, p.H, p.n_pool, z, lam) - f_ref) < 1e-10 * abs(f_ref)
    np.testing.assert_allclose(dense.exact_gradient(p.X, p.H, p.n_pool, z, lam), g_ref,
                               rtol=1e-9, atol=1e-12 * np.abs(g_ref).max())


def test_constant_probabilities_closed_form():
    rng = np.random.default_rng(9)
    n, nl, d, c, lam = 7, 2, 3, 4, 0.05
    X = rng.standard_normal((n + nl, d))
    h = rng.dirichlet(np.ones(c))
    H = np.tile(h, (n + nl, 1))
    z = rng.uniform(0.1, 1, n)
    # Gamma = Q diag(mu) Q^T: Sigma splits into c blocks mu_k S_z + lam, H_p into mu_k S_p.
    mu, _ = np.linalg.eigh(np.diag(h) - np.outer(h, h))
    Sz = sum(np.outer(X[i], X[i]) * (z[i] if i < n else 1.0) for i in range(n + nl))
    Sp = sum(np.outer(X[i], X[i]) for i in range(n))
    f_ref, g_ref = 0.0, np.zeros(n)
    for m in mu:
        A = np.linalg.inv(m * Sz + lam * np.eye(d))
        f_ref += m * np.trace(A @ Sp)
        g_ref -= m * m * np.einsum("ia,ab,ib->i", X[:n], A @ Sp @ A, X[:n])
    assert abs(dense.objective(X, H, n, z, lam) - f_ref) < 1e-10 * abs(f_ref)
    np.testing.assert_allclose(dense.exact_gradient(X, H, n, z, lam), g_ref, rtol=1e-9)


# ---------------------------------------------------------- Hutchinson gradient

def hadamard_block(d, c):
    m = int(round(math.log2(d * c)))
    assert 2 ** m == d * c
    return orc.vecs_to_block(dense.hadamard(m), d, c)      # s = dc probes


@pytest.mark.parametrize("project", [False, True])
def test_complete_hadamard_probes_give_the_exact_gradient(project):
    p = make_small(n=14, n_lab=4, d=4, c=4, s=16, seed=31)
    z = np.random.default_rng(10).uniform(0.2, 1.0, p.n_pool)
    w = z / z.sum()
    b = z.sum()
    V = hadamard_block(p.d, p.c)
    _, info = orc.relax_iteration(p.X, p.H, p.n_pool, w, b, 1e-2, 0.1, 0, 1, p.s,
                                  1e-14, 1000, project=project, V=V)
    g_ref = dense.exact_gradient(p.X, p.H, p.n_pool, z, 1e-2)
    np.testing.assert_allclose(info["g"], g_ref, rtol=1e-8, atol=1e-9 * np.abs(g_ref).max())
    f_ref = dense.objective(p.X, p.H, p.n_pool, z, 1e-2)
    assert abs(info["f_hat"] - f_ref) < 1e-9 * f_ref


def test_configuration_1_gradient_with_the_complete_probe_set():
    # Configuration 1's shape (n = 2000 + 50, d = 20, c = 5: dc = 100) and its data.  With the
    # complete set of scaled unit probes sqrt(dc) e_k (s = dc), (1/s) sum_j v_j^T A v_j = Tr(A)
    # for every A, so the Hutchinson gradient of Algorithm 2 (eq. 11) is the exact gradient of
    # eq. 6, formed here from the dense dc x dc matrices H_i = Gamma_i (x) x_i x_i^T.
    from synthdata import make_problem
    p = make_problem(1)
    dc = p.d * p.c
    w = np.full(p.n_pool, 1.0 / p.n_pool)
    z = p.b * w
    V = orc.vecs_to_block(math.sqrt(dc) * np.eye(dc), p.d, p.c)
    _, info = orc.relax_iteration(p.X, p.H, p.n_pool, w, p.b, p.lam, 0.1, 0, 1, dc, 1e-13,
                                  2000, project=True, V=V)
    g_ref = dense.exact_gradient(p.X, p.H, p.n_pool, z, p.lam)
    np.testing.assert_allclose(info["g"], g_ref, rtol=1e-7, atol=1e-9 * np.abs(g_ref).max())
    f_ref = dense.objective(p.X, p.H, p.n_pool, z, p.lam)
    assert abs(info["f_hat"] - f_ref) < 1e-9 * f_ref


def test_grad_contract_equals_dense_quadratic_forms():
    p = tiny(n=6, n_lab=0, d=3, c=3, s=2)
    rng = np.random.default_rng(12)
    U = rng.standard_normal((p.d, p.s, p.c))
    W = rng.standard_normal((p.d, p.s, p.c))
    g = orc.grad_contract(p.X, p.H, U, W)
    Uv, Wv = orc.block_to_vecs(U), orc.block_to_vecs(W)
    ref = [-np.mean([Uv[:, j] @ dense.fisher(p.X[i], p.H[i]) @ Wv[:, j] for j in range(p.s)])
           for i in range(p.n_pool)]
    np.testing.assert_allclose(g, ref, rtol=1e-12, atol=1e-12)


def test_gradient_and_hvp_are_consistent():
    # sum_i z_i g_i = -(1/s) sum_j <V_j, H_z W_j> by linearity in the row weights.
    p = tiny(n=30, n_lab=4, d=4, c=3, s=5)
    rng = np.random.default_rng(13)
    V = rng.standard_normal((p.d, p.s, p.c))
    W = rng.standard_normal((p.d, p.s, p.c))
    z = rng.uniform(0, 1, p.n_pool)
    g = orc.grad_contract(p.X[:p.n_pool], p.H[:p.n_pool], V, W)
    rhs = -orc.col_dot(V, orc.hvp(p.X[:p.n_pool], p.H[:p.n_pool], z, 0.0, W)).sum() / p.s
    assert abs(z @ g - rhs) < 1e-11 * abs(rhs)


def test_hutchinson_mean_over_seeds_tends_to_exact():
    p = make_small(n=12, n_lab=3, d=3, c=3, s=8, seed=41)
    z = np.full(p.n_pool, 0.5)
    g_ref = dense.exact_gradient(p.X, p.H, p.n_pool, z, 1e-2)
    acc = np.zeros(p.n_pool)
    T = 60
    for t in range(1, T + 1):
        _, info = orc.relax_iteration(p.X, p.H, p.n_pool, z / z.sum(), z.sum(), 1e-2, 0.1,
                                      77, t, p.s, 1e-12, 500)
        acc += info["g"]
    err = np.linalg.norm(acc / T - g_ref) / np.linalg.norm(g_ref)
    assert err < 0.15


# ------------------------------------------------------------ adjoint gradient

def test_adjoint_gradient_matches_finite_differences_of_sampled_objective():
    p = make_small(n=10, n_lab=3, d=3, c=3, s=4, seed=51)
    rng = np.random.default_rng(14)
    z = rng.uniform(0.2, 1.0, p.n_pool)
    V = orc.probes(9, 1, p.d, p.s, p.c)
    f, g = orc.sampled_objective_grad(p.X, p.H, p.n_pool, z, 1e-2, V, 1e-14, 1000)
    h = 1e-5
    for i in range(0, p.n_pool, 3):
        e = np.zeros(p.n_pool)
        e[i] = h
        fp, *_ = orc.sampled_objective(p.X, p.H, p.n_pool, z + e, 1e-2, V, 1e-14, 1000)
        fm, *_ = orc.sampled_objective(p.X, p.H, p.n_pool, z - e, 1e-2, V, 1e-14, 1000)
        assert abs((fp - fm) / (2 * h) - g[i]) <= 1e-6 * max(1.0, abs(g[i]))


def test_adjoint_with_hadamard_probes_is_exact():
    p = make_small(n=9, n_lab=2, d=2, c=4, s=8, seed=61)
    z = np.random.default_rng(15).uniform(0.2, 1.0, p.n_pool)
    V = hadamard_block(p.d, p.c)
    f, g = orc.sampled_objective_grad(p.X, p.H, p.n_pool, z, 1e-2, V, 1e-14, 1000)
    np.testing.assert_allclose(g, dense.exact_gradient(p.X, p.H, p.n_pool, z, 1e-2),
                               rtol=1e-8)
    assert abs(f - dense.objective(p.X, p.H, p.n_pool, z, 1e-2)) < 1e-9 * f


# ------------------------------------------------------------ mirror descent

def test_mirror_step_invariants():
    rng = np.random.default_rng(16)
    w = rng.dirichlet(np.ones(50))
    g = -rng.uniform(0, 3, 50)
    wn, beta, gmax = orc.mirror_step(w, g, 0.3)
    assert abs(wn.sum() - 1) < 1e-14 and np.all(wn > 0)
    assert abs(beta - 0.3 / gmax) < 1e-15
    ratio = wn / w                      # w_i exp(-beta g_i) / Z: ratio ordered like -g
    assert np.all(np.diff(ratio[np.argsort(g)]) <= 1e-15)
    wc, _, _ = orc.mirror_step(w, np.full(50, -2.5), 0.7)
    np.testing.assert_allclose(wc, w, rtol=1e-13)


def test_relax_keeps_simplex_and_decreases_exact_objective():
    p = make_small(n=16, n_lab=4, d=2, c=4, s=8, seed=71)
    V = hadamard_block(p.d, p.c)
    w = np.full(p.n_pool, 1.0 / p.n_pool)
    b, lam = 4.0, 1e-2
    fs = [dense.objective(p.X, p.H, p.n_pool, b * w, lam)]
    for t in range(1, 6):
        w, info = orc.relax_iteration(p.X, p.H, p.n_pool, w, b, lam, 0.05, 0, t, p.s, 1e-13,
                                      500, V=V)
        assert abs(w.sum() - 1) < 1e-13 and np.all(w > 0)
        fs.append(dense.objective(p.X, p.H, p.n_pool, b * w, lam))
    assert all(f1 < f0 for f0, f1 in zip(fs, fs[1:]))


def test_projected_and_literal_modes_agree():
    p = make_small(n=40, n_lab=5, d=3, c=4, s=4, seed=81)
    w = np.full(p.n_pool, 1.0 / p.n_pool)
    out = {}
    for proj in (False, True):
        out[proj] = orc.relax_iteration(p.X, p.H, p.n_pool, w, 5.0, 1e-3, 0.2, 17, 1, p.s,
                                        1e-13, 2000, project=proj)
    (w0, i0), (w1, i1) = out[False], out[True]
    assert abs(i0["f_hat"] - i1["f_hat"]) < 1e-9 * abs(i0["f_hat"])
    np.testing.assert_allclose(i0["g"], i1["g"], rtol=1e-7, atol=1e-9 * np.abs(i0["g"]).max())
    np.testing.assert_allclose(w0, w1, rtol=1e-9)


# ------------------------------------------------------------ stop rule

def test_relative_change_stop_rule_hand_values():
    # |f_t - f_{t-1}| <= tol |f_{t-1}| (experiments section: relative change below 1e-4)
    assert orc.relative_change_small(100.0, 100.005, 1e-4)
    assert orc.relative_change_small(1024.0, 1023.0, 2.0 ** -10)  # exactly on the bound
    assert not orc.relative_change_small(1024.0, 1022.0, 2.0 ** -10)
    assert not orc.relative_change_small(100.0, 100.02, 1e-4)
    assert orc.relative_change_small(-50.0, -50.004, 1e-4)
    assert not orc.relative_change_small(-50.0, -49.99, 1e-4)


def test_relax_stop_rule_ends_at_the_first_small_change():
    p = make_small(n=60, n_lab=4, d=3, c=4, s=4, seed=91)
    full_w = []
    _, full = orc.relax(p.X, p.H, p.n_pool, 4.0, 1e-3, 0.3, 5, 25, p.s, 1e-10, 500,
                        project=True, callback=lambda t, w, info: full_w.append(w.copy()))
    f = [h["f_hat"] for h in full]
    rel = [abs(f[t] - f[t - 1]) / abs(f[t - 1]) for t in range(1, len(f))]
    stop_rel = float(np.median(rel))      # some change along the run passes, earlier ones do not
    want = 1 + next(t for t in range(1, len(f)) if rel[t - 1] <= stop_rel)
    z, hist = orc.relax(p.X, p.H, p.n_pool, 4.0, 1e-3, 0.3, 5, 25, p.s, 1e-10, 500,
                        project=True, stop_rel=stop_rel)
    assert len(hist) == want
    assert [h["f_hat"] for h in hist] == f[:want]
    np.testing.assert_allclose(z, 4.0 * full_w[want - 1], rtol=0, atol=0)
