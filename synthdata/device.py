"""The same input recipes as `synthdata.make_problem`, drawn on a torch device.

Configurations 3 and 4 (200k x 256 with 100 classes, 1.28M x 384 with 1000
classes and per-row entropy-tuned probabilities) take minutes and tens of GB
in NumPy; here the mixture, the optional whitening and the probability model
are drawn with a seeded torch.Generator on the device.  The values are a
deterministic function of the seed and device type, but not the same numbers
as the NumPy generator (different random streams): results on these inputs
are compared with the GPU's own FP64 mode or with properties, never with
stored values.  Like the rest of this package it holds none of the Relax
arithmetic.
"""
from __future__ import annotations

import dataclasses
import math

import torch

from . import CONFIGS


@dataclasses.dataclass
class DeviceProblem:
    name: str
    X: torch.Tensor        # (n_pool + n_lab, d), pool rows first
    H: torch.Tensor        # (n_pool + n_lab, c), rows sum to 1
    n_pool: int
    n_lab: int
    d: int
    c: int
    s: int
    b: float
    lam: float
    tol: float
    T: int
    probe_seed: int

    @property
    def N(self) -> int:
        return self.n_pool + self.n_lab

    def astype(self, dtype) -> "DeviceProblem":
        return dataclasses.replace(self, X=self.X.to(dtype), H=self.H.to(dtype))


def _softmax_rows(L: torch.Tensor, tau) -> torch.Tensor:
    return torch.softmax(L * tau, dim=1)


def _entropy(P: torch.Tensor) -> torch.Tensor:
    return -(P * torch.log(P.clamp_min(1e-30))).sum(dim=1)


def make_problem_device(cfg: int, device="cuda", dtype=torch.float32, n: int | None = None,
                        n_lab: int | None = None, chunk: int = 131072) -> DeviceProblem:
    """Configuration `cfg` drawn on `device` (data seed 1000+cfg, probe seed 2000+cfg)."""
    p = dict(CONFIGS[cfg])
    if n is not None:
        p["n"] = n
    if n_lab is not None:
        p["n_lab"] = n_lab
    return draw_device(f"cfg{cfg}", p, 1000 + cfg, 2000 + cfg, device, dtype, chunk)


def batch_problems_device(count: int = 64, device="cuda", dtype=torch.float32, seed0: int = 5000,
                          n_range=(5000, 100000), chunk: int = 131072) -> list:
    """The batch workload: problem p (seed seed0 + p) has n ~ U{n_range}, d ~ U{64, 128, 256},
    c ~ U{10, 50, 100}, n_lab = c labeled rows, s = 16, b = c, a mixture of c clusters,
    whitened, with mean max-probability 0.7; tol 1e-6, 30 iterations."""
    out = []
    for q in range(count):
        g = torch.Generator(device="cpu")
        g.manual_seed(seed0 + q)
        n = int(torch.randint(n_range[0], n_range[1] + 1, (1,), generator=g))
        d = (64, 128, 256)[int(torch.randint(0, 3, (1,), generator=g))]
        c = (10, 50, 100)[int(torch.randint(0, 3, (1,), generator=g))]
        p = dict(n=n, n_lab=c, d=d, c=c, s=16, b=float(c), lam=1e-3, tol=1e-6, T=30, K=c,
                 whiten=True, probs="maxprob")
        out.append(draw_device(f"batch{q}", p, seed0 + q, seed0 + 1000 + q, device, dtype, chunk))
    return out


def draw_device(name: str, p: dict, seed: int, probe_seed: int, device, dtype,
                chunk: int = 131072) -> DeviceProblem:
    """One problem of recipe p (keys n, n_lab, d, c, s, b, lam, tol, T, K, whiten, probs)."""
    d, c = p["d"], p["c"]
    N = p["n"] + p["n_lab"]
    K = min(p["K"], c)
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    f32 = dict(device=device, dtype=torch.float32)
    means = torch.randn(K, d, generator=gen, **f32) * 2.0
    lab = torch.randint(0, K, (N,), generator=gen, device=device)
    X = torch.randn(N, d, generator=gen, **f32)
    X += means[lab]
    del lab
    if p["whiten"]:
        mu = X.double().mean(dim=0)
        Xc = X - mu.float()
        cov = torch.zeros(d, d, device=device, dtype=torch.float64)
        for r0 in range(0, N, chunk):
            xc = Xc[r0:r0 + chunk].double()
            cov += xc.T @ xc
        cov /= max(N - 1, 1)
        evals, evecs = torch.linalg.eigh(cov)
        proj = (evecs / torch.sqrt(evals.clamp_min(1e-12))).float()
        X = Xc @ proj
        del Xc
    W = torch.randn(d, c, generator=gen, **f32)
    H = torch.empty(N, c, **f32)
    if p["probs"] == "maxprob":
        # one temperature for all rows: mean max-probability 0.70 (bisection)
        def mean_max(tau):
            acc = 0.0
            for r0 in range(0, N, chunk):
                acc += _softmax_rows(X[r0:r0 + chunk] @ W, tau).max(dim=1).values.double().sum().item()
            return acc / N
        lo, hi = 0.0, 1.0
        while mean_max(hi) < 0.70 and hi < 1e6:
            hi *= 2.0
        for _ in range(40):
            mid = 0.5 * (lo + hi)
            if mean_max(mid) < 0.70:
                lo = mid
            else:
                hi = mid
        tau = 0.5 * (lo + hi)
        for r0 in range(0, N, chunk):
            H[r0:r0 + chunk] = _softmax_rows(X[r0:r0 + chunk] @ W, tau)
    elif p["probs"] == "entropy":
        # per-row temperatures: entropy(h_i) = U[0.2, 0.9] log c (bisection per row)
        target = (0.2 + 0.7 * torch.rand(N, generator=gen, **f32)) * math.log(c)
        for r0 in range(0, N, chunk):
            L = X[r0:r0 + chunk] @ W
            tc = target[r0:r0 + chunk]
            t_lo = torch.zeros(L.shape[0], **f32)
            t_hi = torch.ones(L.shape[0], **f32)
            for _ in range(60):
                grow = _entropy(_softmax_rows(L, t_hi[:, None])) > tc
                if not bool(grow.any()):
                    break
                t_hi = torch.where(grow, 2.0 * t_hi, t_hi)
            for _ in range(40):
                mid = 0.5 * (t_lo + t_hi)
                above = _entropy(_softmax_rows(L, mid[:, None])) > tc
                t_lo = torch.where(above, mid, t_lo)
                t_hi = torch.where(above, t_hi, mid)
            H[r0:r0 + chunk] = _softmax_rows(L, (0.5 * (t_lo + t_hi))[:, None])
    elif p["probs"] == "tau1":
        for r0 in range(0, N, chunk):
            H[r0:r0 + chunk] = _softmax_rows(X[r0:r0 + chunk] @ W, 1.0)
    else:
        raise ValueError(p["probs"])
    return DeviceProblem(name=name, X=X.to(dtype).contiguous(), H=H.to(dtype).contiguous(),
                         n_pool=p["n"], n_lab=p["n_lab"], d=d, c=c, s=p["s"], b=float(p["b"]),
                         lam=float(p["lam"]), tol=float(p["tol"]), T=int(p["T"]),
                         probe_seed=probe_seed)
