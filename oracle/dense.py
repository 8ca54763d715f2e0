"""Dense brute force for tiny Relax problems (test infrastructure only).

Every Fisher matrix is formed explicitly, H_i = [diag(h_i) - h_i h_i^T] (x)
x_i x_i^T (eq. 2), with ``np.kron`` acting on column-stacked vectors (the
paper's vec), so none of Lemma 1's algebra is reused here.  Sums follow eq. 3,
Sigma_z follows eq. 7 plus the regulariser lam*I, the objective is eq. 4-5's
Tr(Sigma_z^-1 H_p) and the exact gradient is eq. 6,
g_i = -<H_i, Sigma_z^-1 H_p Sigma_z^-1>_F.  Only for dc up to a few hundred.
"""
from __future__ import annotations

import numpy as np


def gamma(h: np.ndarray) -> np.ndarray:
    """Gamma_i = diag(h_i) - h_i h_i^T."""
    return np.diag(h) - np.outer(h, h)


def fisher(x: np.ndarray, h: np.ndarray) -> np.ndarray:
    """H_i = Gamma_i (x) x_i x_i^T, a dc x dc matrix (eq. 2)."""
    return np.kron(gamma(h), np.outer(x, x))


def sum_fisher(X: np.ndarray, H: np.ndarray, weights: np.ndarray) -> np.ndarray:
    """sum_i weights_i H_i over the rows of X (eq. 3)."""
    d, c = X.shape[1], H.shape[1]
    S = np.zeros((d * c, d * c))
    for x, h, w in zip(X, H, weights):
        if w != 0.0:
            S += w * fisher(x, h)
    return S


def sigma(X, H, n_pool, z, lam):
    """Sigma_z = H_o + H_z + lam*I (eq. 7 with the regulariser)."""
    N = X.shape[0]
    wts = np.concatenate([z, np.ones(N - n_pool)])
    S = sum_fisher(X, H, wts)
    return S + lam * np.eye(S.shape[0])


def hp(X, H, n_pool):
    """H_p = sum of the pool rows' Fisher matrices (eq. 3)."""
    return sum_fisher(X[:n_pool], H[:n_pool], np.ones(n_pool))


def objective(X, H, n_pool, z, lam) -> float:
    """f(z) = Tr(Sigma_z^-1 H_p) (eq. 4-5)."""
    return float(np.trace(np.linalg.solve(sigma(X, H, n_pool, z, lam), hp(X, H, n_pool))))


def exact_gradient(X, H, n_pool, z, lam) -> np.ndarray:
    """g_i = -<H_i, Sigma_z^-1 H_p Sigma_z^-1>_F for every pool row (eq. 6)."""
    S = sigma(X, H, n_pool, z, lam)
    Si = np.linalg.inv(S)
    M = Si @ hp(X, H, n_pool) @ Si
    return np.array([-np.sum(fisher(X[i], H[i]) * M) for i in range(n_pool)])


def block_diagonal(S: np.ndarray, d: int, c: int) -> np.ndarray:
    """B(S): the c diagonal d x d blocks of a dc x dc matrix (Definition 1)."""
    return np.stack([S[k * d:(k + 1) * d, k * d:(k + 1) * d] for k in range(c)])


def hadamard(m: int) -> np.ndarray:
    """Sylvester-Hadamard matrix of order 2^m (entries +-1, H H^T = 2^m I)."""
    Hm = np.ones((1, 1))
    for _ in range(m):
        Hm = np.block([[Hm, Hm], [Hm, -Hm]])
    return Hm


# ---------------------------------------------------------------- Round step

def block_diag_part(S: np.ndarray, d: int, c: int) -> np.ndarray:
    """S with every off-diagonal d x d block set to zero (the block-diagonal
    assumption of the new Round step, Section 3.2)."""
    M = np.zeros_like(S)
    for k in range(c):
        sl = slice(k * d, (k + 1) * d)
        M[sl, sl] = S[sl, sl]
    return M


def round_exact_blockdiag(X, H, n_pool, z, lam, eta, b):
    """Algorithm 1's Round step on dense dc x dc matrices, every Fisher matrix
    reduced to its block diagonal: the transform H~ = Sigma^-1/2 H Sigma^-1/2
    (Section 2.3) formed explicitly, the per-point objective
    Tr[(A_t + (eta/b) H~_o + eta H~_i)^-1] by a dense inverse, the FTRL action
    A_1 = sqrt(dc) I and A_{t+1} = V (nu I + Lambda) V^T from the
    eigendecomposition of eta H~ (nu from Tr(A^-2) = 1, found by Brent's method).
    A point is selected at most once; ties go to the lowest index.

    Returns (selected rows, [nu_1 .. nu_{b+1}], per-round objective arrays).
    """
    from scipy.optimize import brentq

    N, d = X.shape
    c = H.shape[1]
    dc = d * c
    bd = lambda S: block_diag_part(S, d, c)
    Hi = [bd(fisher(X[i], H[i])) for i in range(N)]
    Sig = bd(sigma(X, H, n_pool, z, lam))
    Ho = sum(Hi[n_pool:], np.zeros((dc, dc)))
    ev, U = np.linalg.eigh(Sig)
    Smh = (U / np.sqrt(ev)) @ U.T
    tl = lambda M: Smh @ M @ Smh
    Ho_t = tl(Ho)
    Hi_t = [tl(Hi[i]) for i in range(n_pool)]
    A = np.sqrt(dc) * np.eye(dc)
    Ht = np.zeros((dc, dc))
    sel, nus, objs = [], [float(np.sqrt(dc))], []
    for _ in range(b):
        r = np.full(n_pool, np.inf)
        for i in range(n_pool):
            if i not in sel:
                r[i] = np.trace(np.linalg.inv(A + (eta / b) * Ho_t + eta * Hi_t[i]))
        objs.append(r)
        it = int(np.argmin(r))
        Ht = Ht + Ho_t / b + Hi_t[it]
        lam_, V = np.linalg.eigh(eta * Ht)
        f = lambda nu: float(np.sum((nu + lam_) ** -2.0)) - 1.0
        lo = 1.0 - lam_.min()
        hi = np.sqrt(dc) - lam_.min()
        nu = lo if f(lo) == 0.0 else (hi if f(hi) == 0.0 else
                                      brentq(f, lo, hi, xtol=1e-15, rtol=4 * np.finfo(float).eps,
                                             maxiter=500))
        A = (V * (nu + lam_)) @ V.T
        sel.append(it)
        nus.append(float(nu))
    return np.array(sel, dtype=np.int64), np.array(nus), objs
