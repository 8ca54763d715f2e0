"""Seeded synthetic inputs for the Approx-FIRAL Relax step.

This module only *draws inputs*: Gaussian-mixture feature rows, an optional
whitening of them, and class-probability rows h_i = softmax(tau * W^T x_i)
from a random linear model (the multinomial logistic model of eq. 1, here with
all c classes).  It holds none of the Relax arithmetic (no Hessian products,
no preconditioner, no solver, no gradient), so the CPU oracle and the GPU
path can both take their inputs from it without sharing any method code.

The shapes follow the paper's workloads (Table 4 for the accuracy datasets,
Section 4.2 for the ImageNet-1k single-GPU runs); the datasets themselves are
replaced by mixtures with the same n, d, c.  Every array is a deterministic
function of the integer seed it is given.

Row layout everywhere: X is (n_pool + n_lab) x d with the pool rows first,
H is (n_pool + n_lab) x c with the same row order.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Problem", "gaussian_mixture", "whiten", "softmax_rows", "tune_tau_maxprob",
    "entropy_spread_probs", "make_problem", "dirichlet_weights", "labeled_mixture", "CONFIGS",
]


@dataclasses.dataclass
class Problem:
    """One Relax problem instance plus the hyper-parameters it is run with."""
    name: str
    X: np.ndarray          # (n_pool + n_lab, d) float64, pool rows first
    H: np.ndarray          # (n_pool + n_lab, c) float64, rows sum to 1
    n_pool: int
    n_lab: int
    d: int
    c: int
    s: int                 # number of Rademacher probes
    b: float               # budget: sum of the relaxed weights z
    lam: float             # regulariser added to Sigma_z (lam * I)
    tol: float             # PCG relative-residual tolerance
    T: int                 # mirror-descent iterations
    probe_seed: int

    @property
    def N(self) -> int:
        return self.n_pool + self.n_lab

    def astype(self, dtype) -> "Problem":
        return dataclasses.replace(self, X=np.ascontiguousarray(self.X, dtype=dtype),
                                   H=np.ascontiguousarray(self.H, dtype=dtype))


def gaussian_mixture(rng: np.random.Generator, n: int, d: int, k: int,
                     mean_std: float = 2.0) -> np.ndarray:
    """n rows from k equally weighted unit-variance clusters with means ~ N(0, mean_std^2 I)."""
    means = rng.standard_normal((k, d)) * mean_std
    lab = rng.integers(0, k, size=n)
    out = rng.standard_normal((n, d))
    out += means[lab]
    return out


def labeled_mixture(rng: np.random.Generator, n: int, d: int, c: int,
                    mean_std: float = 0.5) -> tuple:
    """n rows from c equally weighted unit-variance clusters with means ~ N(0, mean_std^2 I),
    and each row's cluster as its class label (for active-learning loops with known labels)."""
    means = rng.standard_normal((c, d)) * mean_std
    y = rng.integers(0, c, size=n)
    X = rng.standard_normal((n, d)) + means[y]
    return X, y


def whiten(X: np.ndarray) -> np.ndarray:
    """Centre, rotate to the sample-covariance eigenbasis, scale each component to unit variance."""
    mu = X.mean(axis=0)
    Xc = X - mu
    cov = (Xc.T @ Xc) / max(X.shape[0] - 1, 1)
    evals, evecs = np.linalg.eigh(cov)
    evals = np.maximum(evals, 1e-12)
    return (Xc @ evecs) / np.sqrt(evals)


def softmax_rows(L: np.ndarray) -> np.ndarray:
    """Row-wise softmax of a score matrix (max-subtracted)."""
    m = L.max(axis=1, keepdims=True)
    E = np.exp(L - m)
    E /= E.sum(axis=1, keepdims=True)
    return E


def tune_tau_maxprob(L: np.ndarray, target: float = 0.70, iters: int = 60) -> float:
    """Bisect a scalar temperature tau so that mean_i max_k softmax(tau*L)_ik == target."""
    lo, hi = 0.0, 1.0
    while softmax_rows(hi * L).max(axis=1).mean() < target:
        hi *= 2.0
        if hi > 1e6:
            break
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        if softmax_rows(mid * L).max(axis=1).mean() < target:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def entropy_spread_probs(L: np.ndarray, rng: np.random.Generator, lo: float = 0.2,
                         hi: float = 0.9, iters: int = 40, chunk: int = 65536) -> np.ndarray:
    """Per-row temperatures so that entropy(h_i) = U[lo, hi] * log c for each row.

    The entropy of softmax(tau * l) falls monotonically in tau > 0, so each row's
    tau_i is found by bisection (vectorised over a chunk of rows).
    """
    n, c = L.shape
    target = rng.uniform(lo, hi, size=n) * math.log(c)
    out = np.empty_like(L)
    for r0 in range(0, n, chunk):
        Lc = L[r0:r0 + chunk]
        tc = target[r0:r0 + chunk]
        t_lo = np.zeros(Lc.shape[0])
        t_hi = np.full(Lc.shape[0], 1.0)
        for _ in range(60):   # grow the bracket until entropy(t_hi) <= target
            P = softmax_rows(t_hi[:, None] * Lc)
            ent = -(P * np.log(np.maximum(P, 1e-300))).sum(axis=1)
            grow = ent > tc
            if not grow.any():
                break
            t_hi[grow] *= 2.0
        for _ in range(iters):
            mid = 0.5 * (t_lo + t_hi)
            P = softmax_rows(mid[:, None] * Lc)
            ent = -(P * np.log(np.maximum(P, 1e-300))).sum(axis=1)
            above = ent > tc
            t_lo = np.where(above, mid, t_lo)
            t_hi = np.where(above, t_hi, mid)
        out[r0:r0 + chunk] = softmax_rows((0.5 * (t_lo + t_hi))[:, None] * Lc)
    return out


def dirichlet_weights(rng: np.random.Generator, n: int, b: float) -> np.ndarray:
    """z ~ b * Dirichlet(1_n): positive weights summing to b."""
    g = rng.standard_exponential(n)
    return b * g / g.sum()


# Configuration table: the five workloads of the build (pool n, labeled n_o, d, c,
# probes s, budget b, regulariser, PCG tolerance, mirror-descent iterations).
CONFIGS = {
    1: dict(n=2000, n_lab=50, d=20, c=5, s=10, b=10.0, lam=1e-3, tol=1e-8, T=50,
            K=5, whiten=False, probs="tau1"),
    2: dict(n=50000, n_lab=10, d=100, c=10, s=20, b=100.0, lam=1e-3, tol=1e-6, T=100,
            K=10, whiten=True, probs="maxprob"),
    3: dict(n=200000, n_lab=100, d=256, c=100, s=32, b=1000.0, lam=1e-3, tol=1e-6, T=1,
            K=100, whiten=True, probs="maxprob"),
    4: dict(n=1280000, n_lab=2000, d=384, c=1000, s=16, b=1000.0, lam=1e-3, tol=1e-5, T=20,
            K=1000, whiten=False, probs="entropy"),
}


def make_problem(cfg: int, n: int | None = None, n_lab: int | None = None,
                 d: int | None = None, c: int | None = None, s: int | None = None,
                 seed: int | None = None, **over) -> Problem:
    """Build configuration `cfg` (1-4), optionally with some sizes overridden.

    Data seed 1000+cfg and probe seed 2000+cfg unless `seed` is given (then the
    probe seed is seed+1000).  Overrides keep the recipe (mixture, whitening,
    probability model) and change only the sizes, so reduced problems have the
    same value distributions as the full ones.
    """
    p = dict(CONFIGS[cfg])
    p.update({k: v for k, v in dict(n=n, n_lab=n_lab, d=d, c=c, s=s).items() if v is not None})
    p.update(over)
    dseed = 1000 + cfg if seed is None else seed
    rng = np.random.default_rng(dseed)
    nt = p["n"] + p["n_lab"]
    K = min(p["K"], p["c"]) if "K" not in over else p["K"]
    X = gaussian_mixture(rng, nt, p["d"], K)
    if p["whiten"]:
        X = whiten(X)
    W = rng.standard_normal((p["d"], p["c"]))
    L = X @ W
    if p["probs"] == "tau1":
        H = softmax_rows(L)
    elif p["probs"] == "maxprob":
        H = softmax_rows(tune_tau_maxprob(L, 0.70) * L)
    elif p["probs"] == "entropy":
        H = entropy_spread_probs(L, rng)
    else:
        raise ValueError(p["probs"])
    return Problem(name=f"cfg{cfg}", X=np.ascontiguousarray(X), H=np.ascontiguousarray(H),
                   n_pool=p["n"], n_lab=p["n_lab"], d=p["d"], c=p["c"], s=p["s"],
                   b=float(p["b"]), lam=float(p["lam"]), tol=float(p["tol"]), T=int(p["T"]),
                   probe_seed=(2000 + cfg) if seed is None else seed + 1000)


def make_small(n: int, n_lab: int, d: int, c: int, s: int, seed: int = 7, b: float = 5.0,
               lam: float = 1e-3, tol: float = 1e-10, T: int = 5, whiten_x: bool = False,
               probs: str = "tau1") -> Problem:
    """A tiny problem with the config-1 recipe (mixture with c clusters, tau = 1 softmax)."""
    rng = np.random.default_rng(seed)
    X = gaussian_mixture(rng, n + n_lab, d, max(c, 2))
    if whiten_x:
        X = whiten(X)
    W = rng.standard_normal((d, c))
    L = X @ W
    H = softmax_rows(L) if probs == "tau1" else softmax_rows(tune_tau_maxprob(L) * L)
    return Problem(name=f"small{n}x{d}x{c}", X=X, H=H, n_pool=n, n_lab=n_lab, d=d, c=c, s=s,
                   b=b, lam=lam, tol=tol, T=T, probe_seed=seed + 1000)
