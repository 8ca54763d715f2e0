"""Pins of the diagonal Round oracle (Algorithm 3) against things other than itself.

* Algorithm 1's Round step on dense dc x dc matrices with block-diagonal Fisher
  matrices (``dense.round_exact_blockdiag``: explicit Sigma^-1/2 transform,
  dense trace of the inverse, FTRL action from a dense eigendecomposition, nu
  by Brent's method) selects the same rows with the same nu.
* The diagonal objective and the dense one differ by the row-independent
  Tr[B_t^-1 Sigma] and the factor -eta, at every round (the proposition of
  Section 3.2); the printed variant with Sigma^-1 in the numerator does not.
* The block Sherman-Morrison formula (Lemma 2) against a direct inverse.
* nu solves Tr(A^-2) = 1 with the eigenvalues of the generalized problem
  (H)_k v = lambda Sigma_k v (scipy's generalized eigensolver, a different
  route to the spectrum of Sigma^-1/2 H Sigma^-1/2).
* Invariants: distinct selections, (H)_k = H_o + sum of the selected rows'
  blocks after b rounds, nu_1 = sqrt(dc).
All CPU; tiny shapes.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import dense
from oracle import round as orr
from synthdata import dirichlet_weights, make_small


def problem(n=30, n_lab=4, d=3, c=3, seed=5, b=6.0):
    p = make_small(n=n, n_lab=n_lab, d=d, c=c, s=2, seed=seed)
    z = dirichlet_weights(np.random.default_rng(seed + 1), n, b)
    return p, z


@pytest.mark.parametrize("shape", [(30, 4, 3, 3, 5), (24, 0, 2, 4, 8), (20, 3, 4, 2, 9),
                                   (16, 2, 1, 3, 12)])
@pytest.mark.parametrize("eta", [0.5, 3.0, 20.0])
def test_diagonal_round_matches_dense_algorithm_1(shape, eta):
    n, nl, d, c, seed = shape
    p, z = problem(n, nl, d, c, seed)
    b = 6
    sel, nus, _ = dense.round_exact_blockdiag(p.X, p.H, p.n_pool, z, 1e-3, eta, b)
    res = orr.round_diag(p.X, p.H, p.n_pool, z, 1e-3, eta, b)
    assert np.array_equal(sel, res["selected"])
    np.testing.assert_allclose(res["nu"], nus, rtol=1e-11)


def test_diagonal_objective_is_the_dense_trace_up_to_a_row_constant():
    p, z = problem()
    eta, b = 3.0, 6
    sel, _, objs = dense.round_exact_blockdiag(p.X, p.H, p.n_pool, z, 1e-3, eta, b)
    st = orr.DiagonalRound(p.X, p.H, p.n_pool, z, 1e-3, eta, b)
    for t in range(b):
        tr = sum(np.trace(st.Binv[k] @ st.Sig[k]) for k in range(st.c))
        lhs = objs[t]
        m = np.isfinite(lhs)
        rhs = tr - eta * st.scores()
        np.testing.assert_allclose(rhs[m], lhs[m], rtol=1e-12)
        st.step(int(sel[t]))


def test_printed_inverse_in_the_numerator_breaks_the_identity():
    # the stated objective prints (Sigma_o)_k^-1 between the two B^-1; with it the
    # difference to the dense trace is no longer constant over rows
    p, z = problem()
    eta = 3.0
    _, _, objs = dense.round_exact_blockdiag(p.X, p.H, p.n_pool, z, 1e-3, eta, 6)
    st = orr.DiagonalRound(p.X, p.H, p.n_pool, z, 1e-3, eta, 6)
    Xp, Gp = st.X[:st.n_pool], st.G[:st.n_pool]
    alt = np.zeros(st.n_pool)
    for k in range(st.c):
        Y = Xp @ st.Binv[k]
        q1 = np.sum(Y * Xp, axis=1)
        q2 = np.sum((Y @ np.linalg.inv(st.Sig[k])) * Y, axis=1)
        alt += Gp[:, k] * q2 / (1 + eta * Gp[:, k] * q1)
    diff = objs[0] + eta * alt
    assert np.ptp(diff) > 1e-3 * np.abs(diff).max()
    diff_ok = objs[0] + eta * st.scores()
    assert np.ptp(diff_ok) <= 1e-12 * np.abs(diff_ok).max()


def test_block_sherman_morrison():
    rng = np.random.default_rng(3)
    d, c = 4, 3
    blocks = []
    for _ in range(c):
        M = rng.standard_normal((d, d))
        blocks.append(M @ M.T + d * np.eye(d))
    A = sla.block_diag(*blocks)
    x = rng.standard_normal(d)
    gam = rng.uniform(0.1, 2.0, c)
    direct = np.linalg.inv(A + np.kron(np.diag(gam), np.outer(x, x)))
    for k in range(c):
        Ai = np.linalg.inv(blocks[k])
        f = Ai - gam[k] * np.outer(Ai @ x, Ai @ x) / (1 + gam[k] * x @ Ai @ x)
        np.testing.assert_allclose(direct[k * d:(k + 1) * d, k * d:(k + 1) * d], f, rtol=1e-12,
                                   atol=1e-14)


def test_nu_solves_the_trace_condition_with_generalized_eigenvalues():
    p, z = problem(n=40, n_lab=5, d=4, c=3, seed=21)
    eta, b = 5.0, 5
    st = orr.DiagonalRound(p.X, p.H, p.n_pool, z, 1e-3, eta, b)
    assert st.nu == math.sqrt(p.d * p.c)
    for _ in range(b):
        st.step()
        lam = np.concatenate([sla.eigh(st.Hk[k], st.Sig[k], eigvals_only=True)
                              for k in range(st.c)])
        np.testing.assert_allclose(np.sort(lam), np.sort(st.lams.ravel()), rtol=1e-9,
                                   atol=1e-12)
        assert abs(np.sum((st.nu + eta * lam) ** -2.0) - 1.0) < 1e-12


def test_round_invariants_and_eta_sweep():
    p, z = problem(n=25, n_lab=3, d=3, c=4, seed=2)
    b = 7
    res = orr.round_diag(p.X, p.H, p.n_pool, z, 1e-3, 2.0, b)
    sel = res["selected"]
    assert len(set(sel.tolist())) == b and sel.min() >= 0 and sel.max() < p.n_pool
    st = res["state"]
    G = orr.class_weights(p.H)
    want = st.Ho + sum(G[i][:, None, None] * np.outer(p.X[i], p.X[i])[None] for i in sel)
    np.testing.assert_allclose(st.Hk, want, rtol=1e-12, atol=1e-13)
    assert res["criterion"] == pytest.approx(min(np.linalg.eigvalsh(want[k])[0]
                                                 for k in range(p.c)), rel=1e-10)
    sw = orr.eta_sweep(p.X, p.H, p.n_pool, z, 1e-3, [0.5, 2.0, 8.0], b)
    assert sw["best"] == sw["etas"][int(np.argmax(sw["criterion"]))]
    # the whole pool, one round each: every row is taken exactly once
    full = orr.round_diag(p.X, p.H, p.n_pool, z, 1e-3, 2.0, p.n_pool)
    assert sorted(full["selected"].tolist()) == list(range(p.n_pool))


def test_float32_decision_follows_the_float64_one_up_to_rounding():
    # the float32 objective differs from the float64 one by float32 rounding only, and the
    # float32 argmax of a well-separated round is the float64 one
    p, z = problem(n=60, n_lab=4, d=5, c=3, seed=31)
    st64 = orr.DiagonalRound(p.X, p.H, p.n_pool, z, 1e-3, 4.0, 6)
    st32 = orr.DiagonalRound(p.X, p.H, p.n_pool, z, 1e-3, 4.0, 6, fp32=True)
    for _ in range(6):
        r64, r32 = st64.scores(), st32.scores()
        assert np.linalg.norm(r32 - r64) <= 1e-5 * np.linalg.norm(r64)
        top = np.sort(r64[st64.available])[::-1]
        if top[0] - top[1] > 1e-4 * top[0]:
            assert st32.argmax(r32) == st64.argmax(r64)
        i = st64.argmax(r64)
        st64.step(i)
        st32.step(i)
