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
