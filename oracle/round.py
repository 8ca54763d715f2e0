"""FP64 oracle of the diagonal Round step of Approx-FIRAL (Algorithm 3).

Test infrastructure only (see the package docstring).  Plain NumPy in float64;
matmul, ``eigh``/``eigvalsh`` and ``inv`` serve as single steps, everything
else follows Algorithm 3 in the paper's order and notation.

Every d x d quantity is block diagonal with c blocks of d x d (Section 3.2:
each H_i keeps only its diagonal blocks, g_ik x_i x_i^T with
g_ik = h_ik (1 - h_ik)); a block-diagonal matrix is held as a (c, d, d) array.

Round t (1-based) selects

    i_t = argmax over the unselected pool rows of
          sum_k g_ik * x_i^T (B_t)_k^-1 (Sigma_o)_k (B_t)_k^-1 x_i
                     / (1 + eta g_ik x_i^T (B_t)_k^-1 x_i)

with B_1 = sqrt(dc) Sigma_o + (eta/b) H_o and, after the update of (H)_k,
the eigenvalues lambda_kj of (H~)_k = (Sigma_o)_k^-1/2 (H)_k (Sigma_o)_k^-1/2,
nu_{t+1} with sum_kj (nu + eta lambda_kj)^-2 = 1 (bisection), and
B_{t+1} = nu_{t+1} Sigma_o + eta H + (eta/b) H_o.

Readings of the paper taken here (each is listed with its reason in the
design notes):
* Sigma_o (the paper's Sigma at z_o) keeps the Relax step's regulariser:
  its blocks are lam*I + (H_o)_k + (H_{z_o})_k, i.e. the blocks of Sigma_z
  at z = z_o.
* The numerator of the per-point objective holds (Sigma_o)_k itself: the
  proof of the diagonal objective reaches Tr[(B_t + eta H_i)^-1 Sigma_o],
  and the block Sherman-Morrison formula then gives x^T B^-1 Sigma_o B^-1 x;
  the inverse printed in the stated objective contradicts that derivation.
  ``tests/test_oracle_round.py`` pins this against the dense trace of the
  exact Round objective.
* A point is selected at most once (the selected set grows by one point per
  round); ties go to the lowest index.
* nu is found by bisection on [1 - eta*lambda_min, sqrt(dc) - eta*lambda_min],
  where sum_kj (nu + eta lambda_kj)^-2 - 1 changes sign, until the bracket
  stops shrinking in float64.
* The eta criterion of the experiments section is min_k lambda_min((H)_k)
  of Algorithm 3's (H)_k after the b rounds (which include H_o).
* Decision precision: the paper's implementation computes in single
  precision (Section 3.3).  With fp32=True the per-point objective (the two
  quadratic forms, the class terms and their sum) is evaluated in float32
  and the argmax taken on those float32 values, as the GPU's FP32 mode does;
  the block state (Sigma_o, B^-1, eigenvalues, nu) stays float64 either way.
"""
from __future__ import annotations

import math

import numpy as np


def class_weights(H: np.ndarray) -> np.ndarray:
    """g_ik = h_ik (1 - h_ik): the diagonal of Gamma_i, which scales block k of H_i."""
    return H * (1.0 - H)


def gram_blocks(X: np.ndarray, G: np.ndarray, w: np.ndarray) -> np.ndarray:
    """(c, d, d) blocks sum_r w_r G_rk x_r x_r^T (the block diagonal of sum_r w_r H_r)."""
    c = G.shape[1]
    return np.stack([(X * (w * G[:, k])[:, None]).T @ X for k in range(c)])


def inv_sqrt_spd(S: np.ndarray) -> np.ndarray:
    """S^-1/2 of a symmetric positive definite matrix through its eigendecomposition."""
    ev, U = np.linalg.eigh(S)
    return (U / np.sqrt(ev)) @ U.T


def nu_bisection(lam: np.ndarray, eta: float) -> float:
    """The unique nu > -eta*min(lam) with sum_j (nu + eta lam_j)^-2 = 1 (bisection)."""
    lam = np.asarray(lam, dtype=np.float64).ravel()
    m = eta * lam.min()
    lo, hi = 1.0 - m, math.sqrt(lam.size) - m

    def phi(nu):
        return float(np.sum((nu + eta * lam) ** -2.0))

    for _ in range(2000):
        mid = 0.5 * (lo + hi)
        if mid <= lo or mid >= hi:
            break
        if phi(mid) > 1.0:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


class DiagonalRound:
    """State of Algorithm 3 on a problem (X, H) with relaxed weights z (pool rows).

    X: (n_pool + n_lab, d), pool rows first; H: same rows x c probabilities;
    z: (n_pool,) relaxed weights z_o; lam: regulariser of Sigma_o; eta > 0;
    b: number of rounds.
    """

    def __init__(self, X, H, n_pool, z, lam, eta, b, fp32: bool = False):
        self.X = np.asarray(X, dtype=np.float64)
        self.H = np.asarray(H, dtype=np.float64)
        self.n_pool = int(n_pool)
        self.N, self.d = self.X.shape
        self.c = self.H.shape[1]
        self.eta = float(eta)
        self.b = int(b)
        self.fp32 = bool(fp32)
        self.G = class_weights(self.H)
        d, c = self.d, self.c
        w_lab = np.concatenate([np.zeros(self.n_pool), np.ones(self.N - self.n_pool)])
        w_all = np.concatenate([np.asarray(z, dtype=np.float64), np.ones(self.N - self.n_pool)])
        # the blocks of Sigma_o = H_o + H_{z_o} (+ lam I)
        self.Ho = gram_blocks(self.X, self.G, w_lab)
        self.Sig = gram_blocks(self.X, self.G, w_all) + lam * np.eye(d)[None]
        self.Sig_mh = np.stack([inv_sqrt_spd(self.Sig[k]) for k in range(c)])
        # first round: B_1 = sqrt(dc) Sigma_o + (eta/b) H_o (A_1 = sqrt(dc) I)
        self.nu = math.sqrt(d * c)
        self.Binv = np.linalg.inv(self.nu * self.Sig + (self.eta / self.b) * self.Ho)
        # the accumulated (H)_k start at zero
        self.Hk = np.zeros((c, d, d))
        self.t = 1
        self.selected: list[int] = []
        self.available = np.ones(self.n_pool, dtype=bool)
        self.nus = [self.nu]
        self.lams = None

    def scores(self) -> np.ndarray:
        """The diagonal Round objective of every pool row at the current B_t
        (selected rows included; the caller masks them)."""
        ft = np.float32 if self.fp32 else np.float64
        Xp = self.X[:self.n_pool].astype(ft)
        Gp = self.G[:self.n_pool].astype(ft)
        eta = ft(self.eta)
        r = np.zeros(self.n_pool, dtype=ft)
        for k in range(self.c):
            Bk = self.Binv[k].astype(ft)
            Y = Xp @ Bk                                               # rows (B_k^-1 x_i)^T
            q1 = np.sum(Y * Xp, axis=1, dtype=ft)                     # x^T B_k^-1 x
            q2 = np.sum((Y @ self.Sig[k].astype(ft)) * Y, axis=1, dtype=ft)
            g = Gp[:, k]                                              # x^T B^-1 Sigma B^-1 x above
            r += g * q2 / (ft(1.0) + eta * g * q1)
        return r.astype(np.float64)

    def argmax(self, r: np.ndarray) -> int:
        """Largest score among the unselected rows, lowest index on ties."""
        masked = np.where(self.available, r, -np.inf)
        return int(np.argmax(masked))

    def step(self, i: int | None = None) -> int:
        """One round: the selection (or the given index), the update of (H)_k, the
        eigenvalues, nu and the next B^-1."""
        if i is None:
            i = self.argmax(self.scores())
        if not self.available[i]:
            raise ValueError(f"row {i} was already selected")
        x = self.X[i]
        # (H)_k += H_o,k / b + g_ik x x^T
        self.Hk += self.Ho / self.b + self.G[i][:, None, None] * np.outer(x, x)[None]
        # eigenvalues of (H~)_k = Sigma_k^-1/2 (H)_k Sigma_k^-1/2
        self.lams = np.stack([np.linalg.eigvalsh(self.Sig_mh[k] @ self.Hk[k] @ self.Sig_mh[k])
                              for k in range(self.c)])
        # nu_{t+1} from Tr(A_{t+1}^-2) = 1
        self.nu = nu_bisection(self.lams, self.eta)
        # B_{t+1}^-1
        self.Binv = np.linalg.inv(self.nu * self.Sig + self.eta * self.Hk
                                  + (self.eta / self.b) * self.Ho)
        # the selected set grows by the row
        self.selected.append(i)
        self.available[i] = False
        self.nus.append(self.nu)
        self.t += 1
        return i

    def criterion(self) -> float:
        """min over k of lambda_min((H)_k), the quantity the eta sweep maximises."""
        return float(min(np.linalg.eigvalsh(self.Hk[k])[0] for k in range(self.c)))


def round_diag(X, H, n_pool, z, lam, eta, b, rounds: int | None = None,
               fp32: bool = False) -> dict:
    """Run `rounds` (default b) rounds of Algorithm 3; returns the selected rows,
    nu_1..nu_{rounds+1}, the winning score of each round and the criterion."""
    st = DiagonalRound(X, H, n_pool, z, lam, eta, b, fp32=fp32)
    smax = []
    for _ in range(b if rounds is None else rounds):
        r = st.scores()
        i = st.argmax(r)
        smax.append(float(r[i]))
        st.step(i)
    return dict(selected=np.array(st.selected, dtype=np.int64), nu=np.array(st.nus),
                score_max=np.array(smax), criterion=st.criterion(), state=st)


def eta_sweep(X, H, n_pool, z, lam, etas, b, fp32: bool = False) -> dict:
    """The eta choice of the experiments section: run the Round step for each eta
    and keep the one whose selection maximises min_k lambda_min((H)_k) (the first
    such eta in the list on ties)."""
    runs = [round_diag(X, H, n_pool, z, lam, e, b, fp32=fp32) for e in etas]
    crit = [r["criterion"] for r in runs]
    best = int(np.argmax(crit))
    return dict(etas=list(etas), criterion=crit, best=etas[best], best_index=best,
                selected=runs[best]["selected"])
