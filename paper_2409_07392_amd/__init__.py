"""MI355X (gfx950) Relax and Round steps of Approx-FIRAL (Chen, Wen & Biros, SC24).

Every step of the path runs in the hand-written HIP kernels of libfiral.so
(see include/firal.h); this module only marshals arguments: torch tensors
supply device memory and the current stream.  There is no CPU fallback:
constructing a context without the built library or without a GPU raises.
"""
from __future__ import annotations

import torch

from . import _lib
from ._lib import (BF16X3, F32, F64, PCG_PROJECT, ROUND_FP32, FiralError, Info,
                   WARN_NOT_CONVERGED, check, load)

__all__ = ["RelaxContext", "RelaxBatch", "RelaxObjective", "RoundSolver", "round_eta_sweep",
           "FiralError", "default_beta0", "F64", "F32", "BF16X3", "load"]

_DTYPE = {F64: torch.float64, F32: torch.float32, BF16X3: torch.float32}


def default_beta0(n: int, T: int) -> float:
    """The library's default mirror-descent step scale for T iterations over n weights
    (firal_default_beta0)."""
    return float(load().firal_default_beta0(int(n), int(T)))


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _ptr(t):
    return None if t is None else t.data_ptr()


class RelaxContext:
    """One Relax problem on the current GPU.

    X: (n_pool + n_lab, d) and H: (n_pool + n_lab, c) CUDA tensors, pool rows
    first, float64 for prec 'f64' and float32 otherwise.  The context borrows
    them (keeps references) and owns all workspace for up to s_max probes.
    """

    def __init__(self, X: torch.Tensor, H: torch.Tensor, n_pool: int, s_max: int,
                 prec: str = "f32"):
        self.lib = load()
        self.prec = _lib.PREC[prec]
        self.dtype = _DTYPE[self.prec]
        if not (X.is_cuda and H.is_cuda):
            raise ValueError("X and H must be CUDA tensors")
        if X.dtype != self.dtype or H.dtype != self.dtype:
            raise ValueError(f"X and H must be {self.dtype} for prec={prec}")
        if X.dim() != 2 or H.dim() != 2 or X.shape[0] != H.shape[0]:
            raise ValueError("X must be (N, d) and H (N, c) with the same N")
        self.X = X.contiguous()
        self.H = H.contiguous()
        self.N, self.d = self.X.shape
        self.c = self.H.shape[1]
        self.n_pool = int(n_pool)
        self.n_lab = self.N - self.n_pool
        self.s_max = int(s_max)
        self._ctx = _lib.ctypes.c_void_p()
        check(self.lib.firal_create(_lib.ctypes.byref(self._ctx), self.n_pool, self.n_lab,
                                    self.d, self.c, self.s_max, self.prec, _ptr(self.X),
                                    _ptr(self.H), _stream()))

    # ------------------------------------------------------------ helpers
    def block(self, s: int) -> torch.Tensor:
        return torch.empty((self.d, s, self.c), dtype=self.dtype, device=self.X.device)

    def _blk(self, B: torch.Tensor) -> torch.Tensor:
        if B.dtype != self.dtype or not B.is_cuda or B.dim() != 3 or \
                B.shape[0] != self.d or B.shape[2] != self.c:
            raise ValueError(f"block must be a CUDA {self.dtype} tensor of shape (d, s, c)")
        return B.contiguous()

    @staticmethod
    def _f64(t, n):
        if t is None:
            return None
        if t.dtype != torch.float64 or not t.is_cuda or t.numel() != n:
            raise ValueError(f"expected a CUDA float64 tensor with {n} elements")
        return t.contiguous()

    # -------------------------------------------------------------- calls
    def hvp(self, B, omega=None, shift=0.0, n_rows=None, out=None):
        B = self._blk(B)
        n_rows = self.N if n_rows is None else int(n_rows)
        omega = self._f64(omega, n_rows)
        out = torch.empty_like(B) if out is None else out
        check(self.lib.firal_hvp(self._ctx, _ptr(omega), n_rows, float(shift), _ptr(B),
                                 _ptr(out), B.shape[1], _stream()))
        return out

    def build_precond(self, omega=None, shift=0.0, want_L=True):
        omega = self._f64(omega, self.N)
        shape = (self.c, self.d, self.d)
        L = torch.empty(shape, dtype=torch.float64, device=self.X.device) if want_L else None
        Pinv = torch.empty(shape, dtype=torch.float64, device=self.X.device)
        info = Info()
        rc = self.lib.firal_build_precond(self._ctx, _ptr(omega), float(shift), _ptr(L),
                                          _ptr(Pinv), _lib.ctypes.byref(info), _stream())
        check(rc)
        return L, Pinv, info.as_dict()

    def pcg_solve(self, B, Pinv, omega=None, shift=0.0, tol=1e-6, max_iter=1000, project=False):
        B = self._blk(B)
        omega = self._f64(omega, self.N)
        Xsol = torch.empty_like(B)
        info = Info()
        rc = self.lib.firal_pcg_solve(self._ctx, _ptr(omega), float(shift), _ptr(Pinv), _ptr(B),
                                      _ptr(Xsol), B.shape[1], float(tol), int(max_iter),
                                      PCG_PROJECT if project else 0, _lib.ctypes.byref(info),
                                      _stream())
        check(rc)
        d = info.as_dict()
        d["rc"] = rc
        return Xsol, d

    def grad_z(self, U, W, g=None):
        U = self._blk(U)
        W = self._blk(W)
        g = torch.empty(self.n_pool, dtype=torch.float64, device=self.X.device) if g is None else g
        check(self.lib.firal_grad_z(self._ctx, _ptr(U), _ptr(W), U.shape[1], _ptr(g), _stream()))
        return g

    def probes(self, seed: int, t: int, s: int):
        V = self.block(s)
        check(self.lib.firal_probes(self._ctx, int(seed) & (2**64 - 1), int(t), int(s), _ptr(V),
                                    _stream()))
        return V

    def relax_step(self, w, b, lam, beta0, seed, t, s=None, tol=1e-6, max_iter=1000,
                   project=False, g_out=None):
        """One Algorithm 2 iteration on w (in place).  Returns the info dict (with 'rc')."""
        s = self.s_max if s is None else int(s)
        w = self._f64(w, self.n_pool)
        g_out = self._f64(g_out, self.n_pool)
        info = Info()
        rc = self.lib.firal_relax_step(self._ctx, _ptr(w), float(b), float(lam), float(beta0),
                                       int(seed) & (2**64 - 1), int(t), s, float(tol),
                                       int(max_iter), PCG_PROJECT if project else 0, _ptr(g_out),
                                       _lib.ctypes.byref(info), _stream())
        check(rc)
        d = info.as_dict()
        d["rc"] = rc
        return d

    def relax(self, b, lam, seed, T, s=None, tol=1e-6, max_iter=1000, project=False,
              beta0=None, stop_rel=0.0):
        """The Relax solve (firal_relax_solve): up to T iterations from the uniform weights, with
        the relative-change stop when stop_rel > 0.  beta0=None takes the library's default.
        Returns (z = b w as a CUDA float64 tensor, dict with f_hat and cg_iters per iteration,
        iters, rc and the last iteration's info)."""
        import numpy as np
        s = self.s_max if s is None else int(s)
        z = torch.empty(self.n_pool, dtype=torch.float64, device=self.X.device)
        f_hist = np.zeros(int(T), dtype=np.float64)
        cg_hist = np.zeros(2 * int(T), dtype=np.int32)
        iters = _lib.ctypes.c_int32()
        info = Info()
        rc = self.lib.firal_relax_solve(
            self._ctx, float(b), float(lam), -1.0 if beta0 is None else float(beta0),
            int(seed) & (2**64 - 1), int(T), s, float(tol), int(max_iter),
            PCG_PROJECT if project else 0, float(stop_rel), _ptr(z),
            f_hist.ctypes.data_as(_lib.ctypes.c_void_p),
            cg_hist.ctypes.data_as(_lib.ctypes.c_void_p), _lib.ctypes.byref(iters),
            _lib.ctypes.byref(info), _stream())
        check(rc)
        n = iters.value
        out = info.as_dict()
        out.update(rc=rc, iters=n, f_hat_hist=f_hist[:n].tolist(),
                   cg_hist=[(int(cg_hist[2 * i]), int(cg_hist[2 * i + 1])) for i in range(n)])
        return z, out

    def sampled_objective(self, z, lam, V, tol=1e-10, max_iter=1000, project=True, grad=True):
        """f_V(z) = (1/s) sum_j v_j^T Sigma_z^-1 H_p v_j and, if grad, df_V/dz (FP64 CUDA)."""
        z = self._f64(z, self.n_pool)
        V = self._blk(V)
        g = torch.empty(self.n_pool, dtype=torch.float64, device=self.X.device) if grad else None
        f = _lib.ctypes.c_double()
        info = Info()
        rc = self.lib.firal_sampled_objective(self._ctx, _ptr(z), float(lam), _ptr(V), V.shape[1],
                                              float(tol), int(max_iter),
                                              PCG_PROJECT if project else 0,
                                              _lib.ctypes.byref(f), _ptr(g),
                                              _lib.ctypes.byref(info), _stream())
        check(rc)
        d = info.as_dict()
        d["rc"] = rc
        return f.value, g, d

    def autotune(self, s=None):
        """Time the kernel variants on this problem and keep the faster ones (firal_autotune).

        Returns the choice bits: 1 = row-tiled product, 2 = separate-kernel PCG, 4 = fused
        product with two column blocks per wave, bits 3-4 = code k of the fused product's
        workgroup target 256 << k.  The work blocks and preconditioner of the
        context are overwritten."""
        s = self.s_max if s is None else int(s)
        ch = _lib.ctypes.c_int32()
        check(self.lib.firal_autotune(self._ctx, s, _lib.ctypes.byref(ch), _stream()))
        return ch.value

    def profile_begin(self, kernel: str = "product"):
        """Start timing every launch of one kernel with event pairs attached to its launches:
        'product' (the product's main kernel: the fused kernel, or the row-tiled first
        contraction X V with the row step), 'product_t' (the row-tiled X^T G' contraction) or
        'round_score' (the Round step's scoring kernel)."""
        k = {"product": _lib.PROF_PRODUCT, "product_t": _lib.PROF_PRODUCT_T,
             "round_score": _lib.PROF_ROUND_SCORE}[kernel]
        check(self.lib.firal_profile_begin(self._ctx, k))

    def profile_end(self):
        """Stop timing; returns (total kernel milliseconds, number of launches)."""
        ms = _lib.ctypes.c_double()
        n = _lib.ctypes.c_int64()
        check(self.lib.firal_profile_end(self._ctx, _lib.ctypes.byref(ms), _lib.ctypes.byref(n)))
        return ms.value, n.value

    def close(self):
        if getattr(self, "_ctx", None) is not None and self._ctx.value:
            self.lib.firal_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class RelaxBatch:
    """Independent Relax problems advanced together by one captured HIP graph (extension 2).

    problems: list of dicts with keys ctx (a RelaxContext, one per problem), w (CUDA float64
    simplex weights, advanced in place), b, lam, beta0, seed, and optionally t0 (1), s
    (ctx.s_max), tol (1e-6), max_iter (100), project (True).  Every replay runs one Relax
    iteration of every problem; each PCG solve enqueues exactly max_iter iterations whose
    kernels return once all columns have converged.
    """

    def __init__(self, problems):
        self.lib = load()
        self.problems = list(problems)
        arr = (_lib.BatchProblem * len(self.problems))()
        for i, q in enumerate(self.problems):
            ctx = q["ctx"]
            w = RelaxContext._f64(q["w"], ctx.n_pool)
            if w.data_ptr() != q["w"].data_ptr():
                raise ValueError("w must be a contiguous CUDA float64 tensor (updated in place)")
            arr[i] = _lib.BatchProblem(ctx._ctx.value, w.data_ptr(), float(q["b"]), float(q["lam"]),
                                       float(q["beta0"]), int(q["seed"]) & (2**64 - 1),
                                       int(q.get("t0", 1)), int(q.get("s", ctx.s_max)),
                                       float(q.get("tol", 1e-6)), int(q.get("max_iter", 100)),
                                       PCG_PROJECT if q.get("project", True) else 0)
        self._b = _lib.ctypes.c_void_p()
        check(self.lib.firal_batch_create(_lib.ctypes.byref(self._b), len(self.problems), arr,
                                          _stream()))

    def run(self, iters=1):
        check(self.lib.firal_batch_run(self._b, int(iters), _stream()))

    def info(self, i):
        info = Info()
        rc = self.lib.firal_batch_info(self._b, int(i), _lib.ctypes.byref(info), _stream())
        check(rc)
        d = info.as_dict()
        d["rc"] = rc
        return d

    def next_t(self, i):
        t = _lib.ctypes.c_int32()
        check(self.lib.firal_batch_next_t(self._b, int(i), _lib.ctypes.byref(t)))
        return t.value

    def close(self):
        if getattr(self, "_b", None) is not None and self._b.value:
            self.lib.firal_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class RoundSolver:
    """Diagonal Round step (Algorithm 3) on a RelaxContext's rows.

    z: CUDA float64 relaxed weights of the pool rows (read at construction); lam: regulariser of
    Sigma_o's blocks; eta: learning rate; b: rounds (points to select); fp32: evaluate the
    per-point objective and its argmax in FP32 (the paper's precision) instead of FP64.  The
    block state is FP64; step() only enqueues.  Keep the context alive while the solver lives.
    """

    def __init__(self, ctx: RelaxContext, z: torch.Tensor, lam: float, eta: float, b: int,
                 fp32: bool = False):
        self.lib = load()
        self.ctx = ctx
        self.b = int(b)
        self.fp32 = bool(fp32)
        z = RelaxContext._f64(z, ctx.n_pool)
        self._r = _lib.ctypes.c_void_p()
        check(self.lib.firal_round_create(_lib.ctypes.byref(self._r), ctx._ctx, _ptr(z),
                                          float(lam), float(eta), self.b,
                                          ROUND_FP32 if self.fp32 else 0, _stream()))

    def step(self, rounds: int = 1):
        check(self.lib.firal_round_step(self._r, int(rounds), _stream()))

    def run(self):
        """All remaining rounds; returns the selected pool rows (int64 numpy array)."""
        t = self.result()["t"]
        self.step(self.b - t)
        return self.result()["selected"]

    def scores(self, out=None):
        """The per-point objective of every pool row at the current round (-inf if selected)."""
        if out is None:
            out = torch.empty(self.ctx.n_pool, dtype=torch.float64, device=self.ctx.X.device)
        out = RelaxContext._f64(out, self.ctx.n_pool)
        check(self.lib.firal_round_scores(self._r, _ptr(out), _stream()))
        return out

    def result(self):
        import numpy as np
        sel = np.zeros(self.b, dtype=np.int64)
        nu = np.zeros(self.b + 1, dtype=np.float64)
        smax = np.zeros(self.b, dtype=np.float64)
        t = _lib.ctypes.c_int32()
        check(self.lib.firal_round_result(
            self._r, sel.ctypes.data_as(_lib.ctypes.c_void_p),
            nu.ctypes.data_as(_lib.ctypes.c_void_p), smax.ctypes.data_as(_lib.ctypes.c_void_p),
            _lib.ctypes.byref(t), _stream()))
        n = t.value
        return dict(t=n, selected=sel[:n], nu=nu[:n + 1], score_max=smax[:n])

    def criterion(self) -> float:
        """min_k lambda_min((H)_k) after the rounds done so far."""
        out = _lib.ctypes.c_double()
        check(self.lib.firal_round_criterion(self._r, _lib.ctypes.byref(out), _stream()))
        return out.value

    def close(self):
        if getattr(self, "_r", None) is not None and self._r.value:
            self.lib.firal_round_destroy(self._r)
            self._r = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def round_eta_sweep(ctx: RelaxContext, z: torch.Tensor, lam: float, etas, b: int,
                    fp32: bool = False) -> dict:
    """The eta choice of the experiments section (firal_round_eta_sweep): the Round step for
    every eta, keeping the selection that maximises min_k lambda_min((H)_k)."""
    import numpy as np
    lib = load()
    etas = [float(e) for e in etas]
    z = RelaxContext._f64(z, ctx.n_pool)
    e_arr = np.asarray(etas, dtype=np.float64)
    sel = np.zeros(int(b), dtype=np.int64)
    crit = np.zeros(len(etas), dtype=np.float64)
    best = _lib.ctypes.c_int32()
    check(lib.firal_round_eta_sweep(ctx._ctx, _ptr(z), float(lam),
                                    e_arr.ctypes.data_as(_lib.ctypes.c_void_p), len(etas),
                                    int(b), ROUND_FP32 if fp32 else 0,
                                    sel.ctypes.data_as(_lib.ctypes.c_void_p),
                                    crit.ctypes.data_as(_lib.ctypes.c_void_p),
                                    _lib.ctypes.byref(best), _stream()))
    return dict(etas=etas, criterion=crit.tolist(), best=etas[best.value],
                best_index=best.value, selected=sel)


class RelaxObjective(torch.autograd.Function):
    """f_V(z) = (1/s) sum_j v_j^T Sigma_z^-1 H_p v_j as a differentiable function of z.

    The backward pass is the adjoint of the sampled objective,
    df_V/dz_i = -(1/s) sum_j (Sigma^-1 v_j)^T H_i (Sigma^-1 H_p v_j): two PCG solves and the
    per-point contraction, all in the library (firal_sampled_objective).  The forward computes
    the gradient along with f when z requires it (the solves it needs are shared).

        f = RelaxObjective.apply(z, relax_ctx, V, lam, tol, max_iter, project)
    """

    @staticmethod
    def forward(ctx, z, relax_ctx, V, lam, tol=1e-10, max_iter=1000, project=True):
        need = ctx.needs_input_grad[0]
        f, g, _ = relax_ctx.sampled_objective(z.detach(), lam, V, tol, max_iter, project,
                                              grad=need)
        if need:
            ctx.save_for_backward(g)
        return torch.tensor(f, dtype=torch.float64, device=z.device)

    @staticmethod
    def backward(ctx, grad_f):
        (g,) = ctx.saved_tensors
        return grad_f * g, None, None, None, None, None, None
