"""Matrix-free FP64 oracle of the Approx-FIRAL Relax step (Algorithm 2).

Test infrastructure only (see the package docstring).  Plain NumPy/SciPy in
float64; library primitives (matmul, Cholesky, triangular solves) serve as
single steps, everything else is written out in the order of the paper.

Block layout
------------
A "block" holds s vectors of length dc as a (d, s, c) array B: element
(a, j, k) is entry k*d + a of the paper's j-th vector, i.e. v_j = vec(V_j)
with V_j = B[:, j, :] the d x c matrix whose columns are stacked (notation
table, Lemma 1).  The row-major order (a, j, k) is also the device layout.

Readings of the paper taken here (each is listed with its reason in the
design notes):
* h has c columns (a full softmax); the ABI takes whatever columns it is given.
* Sigma_z = H_o + H_z + lam*I; H_p has no regulariser.
* The iterate is w on the simplex and z = b*w (Algorithm 2 normalises z to
  sum 1 inside the loop and scales by b at the end; eq. 5 has sum z = b).
* beta_t = beta0 / max_i |g_i|, the update done in the log domain.
* Probes are SplitMix64 signs keyed by a counter (the paper leaves the
  generator open), fresh for every iteration t.
* PCG starts from x0 = 0, freezes each column once its recurrence residual
  satisfies ||r_j|| <= tol*||b_j||, and stops when all columns are frozen or
  after max_iter iterations; tol = 0 runs exactly max_iter iterations.
* Optional projected mode: the right-hand sides and the preconditioner are
  projected onto the complement of the near-null space {1_c (x) u}, which
  every H_i annihilates; this leaves H_p*Sigma^-1*V, f_hat and g unchanged
  per sample (see ``project_perp``).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla

GOLDEN_GAMMA = 0x9E3779B97F4A7C15
_MASK64 = (1 << 64) - 1

# ----------------------------------------------------------------------------
# Rademacher probes (Algorithm 2, probe matrix V in R^{dc x s}; eq. 11)
# ----------------------------------------------------------------------------


def splitmix64(state: np.ndarray) -> np.ndarray:
    """SplitMix64 output function (Steele, Lea & Flood, OOPSLA 2014) on uint64 words."""
    z = np.asarray(state, dtype=np.uint64).copy()
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def splitmix64_stream(seed: int, count: int, start: int = 0) -> np.ndarray:
    """Outputs start..start+count-1 of the SplitMix64 sequence whose state starts at `seed`.

    Output number m (0-based) is the mix of seed + (m+1)*golden_gamma (mod 2^64).
    """
    m = np.arange(start, start + count, dtype=np.uint64)
    with np.errstate(over="ignore"):
        st = np.uint64(seed & _MASK64) + (m + np.uint64(1)) * np.uint64(GOLDEN_GAMMA)
    return splitmix64(st)


def probes(seed: int, t: int, d: int, s: int, c: int) -> np.ndarray:
    """Block of s Rademacher vectors for mirror-descent iteration t (1-based).

    Entry (a, j, k) is -1 if the top bit of SplitMix64 output number
    ctr = ((t-1)*s + j)*(d*c) + (k*d + a) is set, else +1; k*d + a is the
    entry's index in the paper's vec ordering.
    """
    a = np.arange(d, dtype=np.int64)[:, None, None]
    j = np.arange(s, dtype=np.int64)[None, :, None]
    k = np.arange(c, dtype=np.int64)[None, None, :]
    ctr = (((t - 1) * s + j) * (d * c) + (k * d + a)).astype(np.uint64)
    with np.errstate(over="ignore"):
        st = np.uint64(seed & _MASK64) + (ctr + np.uint64(1)) * np.uint64(GOLDEN_GAMMA)
    top = splitmix64(st) >> np.uint64(63)
    return np.where(top == 1, -1.0, 1.0)


# ----------------------------------------------------------------------------
# Vectorisation helpers (notation table: vec stacks columns)
# ----------------------------------------------------------------------------


def block_to_vecs(B: np.ndarray) -> np.ndarray:
    """(d, s, c) block -> (dc, s) matrix whose column j is vec(B[:, j, :])."""
    d, s, c = B.shape
    return np.transpose(B, (2, 0, 1)).reshape(c * d, s)


def vecs_to_block(V: np.ndarray, d: int, c: int) -> np.ndarray:
    """(dc, s) matrix of vec-ordered columns -> (d, s, c) block."""
    s = V.shape[1]
    return np.ascontiguousarray(np.transpose(V.reshape(c, d, s), (1, 2, 0)))


def project_perp(B: np.ndarray) -> np.ndarray:
    """Project each vector onto the complement of {1_c (x) u : u in R^d}.

    With a full softmax, Gamma_i 1_c = 0, so every H_i = Gamma_i (x) x_i x_i^T
    annihilates 1_c (x) u; removing that component means subtracting, for each
    feature a and probe j, the mean over the c classes.
    """
    return B - B.mean(axis=2, keepdims=True)


def col_dot(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Per-probe inner products <A_j, B_j> of two blocks."""
    return np.einsum("ajk,ajk->j", A, B)


# ----------------------------------------------------------------------------
# Matrix-free Hessian product (Lemma 1 and the aggregated sum that follows it)
# ----------------------------------------------------------------------------


def hvp(X: np.ndarray, H: np.ndarray, omega: np.ndarray | None, shift: float,
        B: np.ndarray, row_chunk: int = 32768) -> np.ndarray:
    """Out = sum_i omega_i H_i v_j + shift*v_j for every probe j, without forming H_i.

    Lemma 1 gives H_i v in four steps: (1) gamma = V^T x_i, (2) alpha =
    gamma . h_i, (3) gamma <- (gamma - alpha) * h_i, (4) H_i v = vec(x_i
    gamma^T).  Summed over rows, step 4 becomes X^T [gamma_1; ...; gamma_N]
    (the H_p v formula after Lemma 1).  omega=None means weight 1 on every
    row of X.  Rows are taken in slices only to bound memory.
    """
    N, d = X.shape
    c = H.shape[1]
    s = B.shape[1]
    Bm = B.reshape(d, s * c)
    out = np.zeros((d, s * c))
    for r0 in range(0, N, row_chunk):
        Xr = X[r0:r0 + row_chunk]
        Hr = H[r0:r0 + row_chunk]
        n = Xr.shape[0]
        gamma = (Xr @ Bm).reshape(n, s, c)                       # step 1
        alpha = np.einsum("isk,ik->is", gamma, Hr)               # step 2
        gamma = (gamma - alpha[:, :, None]) * Hr[:, None, :]     # step 3
        if omega is not None:
            gamma *= omega[r0:r0 + row_chunk, None, None]
        out += Xr.T @ gamma.reshape(n, s * c)                    # step 4, summed
    return out.reshape(d, s, c) + shift * B


# ----------------------------------------------------------------------------
# Block-diagonal preconditioner (Definition 1, eq. 12)
# ----------------------------------------------------------------------------


def precond_blocks(X: np.ndarray, H: np.ndarray, omega: np.ndarray | None,
                   shift: float) -> np.ndarray:
    """The c diagonal d x d blocks of sum_i omega_i H_i + shift*I.

    By eq. 12 the k-th diagonal block of H_i is h_ik (1 - h_ik) x_i x_i^T.
    """
    N, d = X.shape
    c = H.shape[1]
    om = np.ones(N) if omega is None else omega
    P = np.empty((c, d, d))
    for k in range(c):
        u = om * H[:, k] * (1.0 - H[:, k])
        P[k] = (X * u[:, None]).T @ X + shift * np.eye(d)
    return P


def precond_factor(P: np.ndarray) -> tuple[np.ndarray, int]:
    """Lower Cholesky factor of every block; returns (L, bad) with bad = -1 or the first failing k."""
    c, d, _ = P.shape
    L = np.zeros_like(P)
    for k in range(c):
        try:
            L[k] = np.linalg.cholesky(P[k])
        except np.linalg.LinAlgError:
            return L, k
    return L, -1


def precond_apply(L: np.ndarray, R: np.ndarray) -> np.ndarray:
    """Z = B(Sigma)^-1 R: for each class k, solve P_k Z[:, :, k] = R[:, :, k] with the factor."""
    Z = np.empty_like(R)
    for k in range(L.shape[0]):
        Z[:, :, k] = sla.cho_solve((L[k], True), R[:, :, k])
    return Z


# ----------------------------------------------------------------------------
# Block-Jacobi preconditioned CG over s right-hand sides (Algorithm 2, solves)
# ----------------------------------------------------------------------------


class PCGBreakdown(RuntimeError):
    """p_j^T q_j <= 0 for an active column: the operator is not SPD on that column."""


def pcg(X, H, omega, shift, L, Bb, tol, max_iter, project=False):
    """Solve (sum_i omega_i H_i + shift I) X_j = B_j for all probes j at once.

    Standard preconditioned CG run on every column in lock-step, x0 = 0.
    Returns (x, iters, relres) where relres[j] = ||r_j|| / ||b_j|| of the
    recurrence residual at exit.
    """
    b = project_perp(Bb) if project else Bb.copy()

    def M(r):
        if project:
            return project_perp(precond_apply(L, project_perp(r)))
        return precond_apply(L, r)

    s = b.shape[1]
    bnorm = np.sqrt(col_dot(b, b))
    x = np.zeros_like(b)
    r = b.copy()
    z = M(r)
    p = z.copy()
    rho = col_dot(r, z)
    done = bnorm == 0.0
    it = 0
    while not done.all() and it < max_iter:
        q = hvp(X, H, omega, shift, p)
        pq = col_dot(p, q)
        act = ~done
        if np.any(pq[act] <= 0.0):
            raise PCGBreakdown(f"p^T q <= 0 at iteration {it + 1}")
        alpha = np.where(act, rho / np.where(act, pq, 1.0), 0.0)
        x += alpha[None, :, None] * p
        r -= alpha[None, :, None] * q
        it += 1
        rnorm = np.sqrt(col_dot(r, r))
        done = done | (rnorm <= tol * bnorm)
        z = M(r)
        rho_new = col_dot(r, z)
        act = ~done
        beta = np.where(act, rho_new / np.where(rho != 0.0, rho, 1.0), 0.0)
        p = np.where(act[None, :, None], z + beta[None, :, None] * p, p)
        rho = np.where(act, rho_new, rho)
    rnorm = np.sqrt(col_dot(r, r))
    relres = np.where(bnorm > 0, rnorm / np.where(bnorm > 0, bnorm, 1.0), 0.0)
    return x, it, relres


# ----------------------------------------------------------------------------
# Hutchinson gradient (eq. 11; Algorithm 2 gradient line)
# ----------------------------------------------------------------------------


def grad_contract(Xp: np.ndarray, Hp: np.ndarray, U: np.ndarray, W: np.ndarray,
                  row_chunk: int = 32768) -> np.ndarray:
    """g_i = -(1/s) sum_j u_j^T H_i w_j for every row of Xp.

    With a = U_j^T x_i and b = W_j^T x_i (c-vectors), Lemma 1 gives
    u_j^T H_i w_j = a^T Gamma_i b = sum_k a_k h_ik b_k - (a . h_i)(b . h_i).
    """
    n, d = Xp.shape
    s, c = U.shape[1], U.shape[2]
    g = np.empty(n)
    Um = U.reshape(d, s * c)
    Wm = W.reshape(d, s * c)
    for r0 in range(0, n, row_chunk):
        Xr = Xp[r0:r0 + row_chunk]
        Hr = Hp[r0:r0 + row_chunk]
        m = Xr.shape[0]
        A = (Xr @ Um).reshape(m, s, c)
        Bq = (Xr @ Wm).reshape(m, s, c)
        q = (np.einsum("isk,ik,isk->is", A, Hr, Bq)
             - np.einsum("isk,ik->is", A, Hr) * np.einsum("isk,ik->is", Bq, Hr))
        g[r0:r0 + row_chunk] = -q.sum(axis=1) / s
    return g


# ----------------------------------------------------------------------------
# One Relax iteration (Algorithm 2) and the loop
# ----------------------------------------------------------------------------


def default_beta0(n: int, T: int) -> float:
    """sqrt(2 ln n / T): the textbook entropic mirror-descent step for T iterations."""
    return math.sqrt(2.0 * math.log(n) / max(T, 1))


def mirror_step(w: np.ndarray, g: np.ndarray, beta0: float) -> tuple[np.ndarray, float, float]:
    """w_i <- w_i exp(-beta g_i) / sum_l w_l exp(-beta g_l) with beta = beta0 / max|g|.

    Evaluated as exp(log w_i - beta g_i - m) with m the maximum exponent, which
    the normalisation makes exact in real arithmetic.
    """
    gmax = float(np.abs(g).max()) if g.size else 0.0
    beta = beta0 / gmax if gmax > 0.0 else 0.0
    e = np.log(w) - beta * g
    e -= e.max()
    wn = np.exp(e)
    return wn / wn.sum(), beta, gmax


def relax_iteration(X, H, n_pool, w, b, lam, beta0, seed, t, s, tol, max_iter,
                    project=False, V=None):
    """One pass of Algorithm 2's loop body at iteration t (1-based).

    z = b*w; omega = [z; 1] over pool then labeled rows; V = probes(seed, t)
    unless given; preconditioner blocks of Sigma_z and their factors; W1 =
    Sigma^-1 V; Y = H_p W1; W2 = Sigma^-1 Y; g = Hutchinson gradient; w <-
    mirror step.  Returns (w_new, info).
    """
    N, d = X.shape
    c = H.shape[1]
    z = b * w
    omega = np.concatenate([z, np.ones(N - n_pool)])
    if V is None:
        V = probes(seed, t, d, s, c)
    P = precond_blocks(X, H, omega, lam)
    L, bad = precond_factor(P)
    if bad >= 0:
        raise np.linalg.LinAlgError(f"preconditioner block {bad} is not SPD")
    W1, it1, rr1 = pcg(X, H, omega, lam, L, V, tol, max_iter, project)
    Y = hvp(X[:n_pool], H[:n_pool], None, 0.0, W1)
    f_hat = float(col_dot(V, Y).sum() / s)
    W2, it2, rr2 = pcg(X, H, omega, lam, L, Y, tol, max_iter, project)
    g = grad_contract(X[:n_pool], H[:n_pool], V, W2)
    w_new, beta, gmax = mirror_step(w, g, beta0)
    info = dict(cg_iters=(it1, it2), relres=max(rr1.max(), rr2.max()), f_hat=f_hat,
                g=g, g_absmax=gmax, beta=beta, W1=W1, Y=Y, W2=W2, V=V)
    return w_new, info


def relative_change_small(f_prev: float, f_cur: float, stop_rel: float) -> bool:
    """The stop test of the experiments section: the objective moved by at most stop_rel
    relative to its previous value, |f_cur - f_prev| <= stop_rel * |f_prev|."""
    return abs(f_cur - f_prev) <= stop_rel * abs(f_prev)


def relax(X, H, n_pool, b, lam, beta0, seed, T, s, tol, max_iter, project=False,
          w0=None, callback=None, stop_rel=0.0):
    """Algorithm 2 from w = 1/n for at most T iterations; returns (z = b*w, history).

    stop_rel > 0 adds the termination of the experiments section: after iteration t >= 2
    the loop ends when the objective estimate f_hat of iteration t differs from that of
    iteration t-1 by at most stop_rel times the latter (the weights of iteration t are kept).
    len(history) is the number of iterations run.
    """
    w = np.full(n_pool, 1.0 / n_pool) if w0 is None else w0.copy()
    hist = []
    for t in range(1, T + 1):
        w, info = relax_iteration(X, H, n_pool, w, b, lam, beta0, seed, t, s, tol,
                                  max_iter, project)
        hist.append({k: v for k, v in info.items() if k in ("cg_iters", "relres", "f_hat",
                                                               "g_absmax", "beta")})
        if callback is not None:
            callback(t, w, info)
        if stop_rel > 0.0 and t >= 2 and relative_change_small(hist[-2]["f_hat"],
                                                                hist[-1]["f_hat"], stop_rel):
            break
    return b * w, hist


# ----------------------------------------------------------------------------
# Adjoint gradient of the sampled objective (autograd backward)
# ----------------------------------------------------------------------------


def sampled_objective(X, H, n_pool, z, lam, V, tol, max_iter, project=False):
    """f_V(z) = (1/s) sum_j v_j^T Sigma_z^-1 H_p v_j with Sigma_z = H_o + H_z + lam I.

    Returns (f, U, Yp, L): U = Sigma^-1 V, Yp = H_p V and the preconditioner factor
    (reused by the adjoint).
    """
    N, d = X.shape
    s = V.shape[1]
    omega = np.concatenate([z, np.ones(N - n_pool)])
    L, bad = precond_factor(precond_blocks(X, H, omega, lam))
    if bad >= 0:
        raise np.linalg.LinAlgError(f"preconditioner block {bad} is not SPD")
    U, _, _ = pcg(X, H, omega, lam, L, V, tol, max_iter, project)
    Yp = hvp(X[:n_pool], H[:n_pool], None, 0.0, V)
    f = float(col_dot(U, Yp).sum() / s)
    return f, U, Yp, L


def sampled_objective_grad(X, H, n_pool, z, lam, V, tol, max_iter, project=False):
    """Gradient of f_V w.r.t. z: d f_V / d z_i = -(1/s) sum_j (Sigma^-1 v_j)^T H_i (Sigma^-1 H_p v_j).

    Differentiating Sigma_z^-1 gives -Sigma^-1 (dSigma/dz_i) Sigma^-1 with
    dSigma/dz_i = H_i, so two solves (U = Sigma^-1 V, Y' = Sigma^-1 H_p V)
    and the per-row contraction of eq. 11's form give the exact derivative of
    the sampled objective.
    """
    N = X.shape[0]
    f, U, Yp, L = sampled_objective(X, H, n_pool, z, lam, V, tol, max_iter, project)
    omega = np.concatenate([z, np.ones(N - n_pool)])
    Y2, _, _ = pcg(X, H, omega, lam, L, Yp, tol, max_iter, project)
    g = grad_contract(X[:n_pool], H[:n_pool], U, Y2)
    return f, g
