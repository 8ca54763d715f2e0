"""Benchmark of the Relax step (Algorithm 2) on one MI355X.

Default (the headline): configuration 4, n = 1,280,000 pool points + 2000 labeled, d = 384,
c = 1000, s = 16 probes, b = 1000, PCG tol 1e-5; Gaussian-mixture features (1000 clusters)
and softmax probabilities whose entropies are spread uniformly over [0.2, 0.9] log c, drawn on
the GPU.  A "step" is one full Hessian product of Lemma 1 over all 1,282,000 rows with all 16
probes (4 N c d s = 3.15e13 flop), the operation every PCG iteration of Algorithm 2 spends its
time in; `value` is its rate in TFLOP/s for the FP32 leg.  Measured beside it, for FP32 and for
bf16x3 (products as three bf16 MFMA passes), and reported in `precision_legs`:
  * the product's rate and the time of its kernels (event pairs attached to their launches);
  * one full Relax iteration (Algorithm 2 from w = 1/n: probes, preconditioner with FP64
    factors, two PCG solves to the relative residual 1e-5, the H_p product, the gradient, the
    mirror step), its wall time and CG counts;
  * the relative error of the eq. 11 gradient against the GPU's FP64 mode with the same
    probes and the same fixed CG count (the FP64 mode is itself held to the oracle at 1e-10 on
    a 1% row sample of this workload by the test suite).

    python bench.py [--steps K] [--warmup W] [--relax-iters R] [--no-cpu-baseline]

Prints one JSON line.  --gpus N > 1 is refused: the library runs on one GPU.

Other workloads (not the bench line): --workload 2 (configuration 2: n = 50,000, d = 100,
c = 10, s = 20; whole Relax iterations per step, plus the Round step), 3 (configuration 3:
the sampled objective and its adjoint gradient), 5 (64 uneven problems as a batch), studies
(convergence and scaling studies), al (a synthetic active-learning loop).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Relax iter time + HVP TFLOP/s, FP32 vs bf16x3 at ≤1e-4 rel grad error"
# TFLOP/s, MI355X dense MFMA; bf16x3 counts the FP32-equivalent products of three bf16 passes
PEAK = {"f32": 157.3, "f64": 78.6, "bf16x3": 2500.0 / 3}
HBM_PEAK = 8.0e12   # bytes/s, MI355X HBM3E


def hbm_frac(traffic, launch_us):
    """Measured HBM bytes per launch over the launch time, as a fraction of the HBM peak."""
    if traffic is None or not launch_us:
        return None
    return traffic / (launch_us * 1e-6) / HBM_PEAK


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="4", choices=["2", "3", "4", "5", "studies", "al"])
    ap.add_argument("--prec", default="f32", choices=["f32", "f64", "bf16x3"],
                    help="workloads 2 and 5: the precision of the main leg")
    ap.add_argument("--no-bf16x3", action="store_true", help="skip the bf16x3 leg")
    ap.add_argument("--only-bf16x3", action="store_true",
                    help="configuration 4: the bf16x3 leg alone (the line then reports it)")
    ap.add_argument("--literal", action="store_true", help="PCG without the null-space projection")
    ap.add_argument("--hvp-reps", type=int, default=50)
    ap.add_argument("--prof-reps", type=int, default=3,
                    help="configuration 4: product calls timed kernel by kernel")
    ap.add_argument("--relax-iters", type=int, default=1,
                    help="configuration 4: Relax iterations timed per precision (tol 1e-5)")
    ap.add_argument("--relax-max-cg", type=int, default=200,
                    help="configuration 4: cap on the CG iterations of each solve")
    ap.add_argument("--grad-cg", type=int, default=10,
                    help="configuration 4: fixed CG iterations of the gradient-error runs")
    ap.add_argument("--no-grad-error", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (counter calibration)")
    ap.add_argument("--study", default="fig1,fig4,fig5",
                    help="--workload studies: comma-separated subset of fig1, fig4, fig5")
    ap.add_argument("--no-round", action="store_true", help="skip the Round-step leg")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="configuration 3: the product legs only (no objective, adjoint or "
                         "gradient-error runs)")
    ap.add_argument("--round-rounds", type=int, default=0,
                    help="configurations 3/4: Round-step rounds timed per decision precision")
    ap.add_argument("--round-only", action="store_true",
                    help="configurations 3/4: only the Round-step leg")
    ap.add_argument("--eta", type=float, default=None,
                    help="Round-step learning rate (default 8 sqrt(dc), the theorem's value at "
                         "epsilon = 1)")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {time.strftime('%H:%M:%S')} {msg}", file=sys.stderr, flush=True)


def read_traffic(summary: str):
    """HBM bytes per launch from a committed counter summary under profiles/ (FETCH_SIZE and
    WRITE_SIZE, each scaled by the copy-kernel calibration): the summary's
    `traffic_bytes_per_launch:` line, or None when the summary is missing or the kernel's source
    file (`source:` and `source_sha256:` lines) has changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", summary)
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = re.search(r"^traffic_bytes_per_launch:\s*([0-9.eE+]+)", txt, re.M)
    src = re.search(r"^source:\s*(\S+)", txt, re.M)
    sha = re.search(r"^source_sha256:\s*([0-9a-f]+)", txt, re.M)
    if not (m and src and sha):
        return None
    fpath = os.path.join(ROOT, src.group(1))
    if not os.path.exists(fpath):
        return None
    if hashlib.sha256(open(fpath, "rb").read()).hexdigest() != sha.group(1):
        return None
    return float(m.group(1))


def host_threads():
    from threadpoolctl import threadpool_info
    return max([i.get("num_threads", 1) for i in threadpool_info()] or [1])


# --------------------------------------------------------------- configuration 4

def product_leg(ctx, p, prec, steps, warmup, prof_reps):
    """Time `steps` full products after `warmup`, then each row-tiled kernel on its own."""
    import torch
    flops = 4.0 * p.N * p.c * p.d * p.s
    B = ctx.probes(p.probe_seed, 1, p.s)
    out = torch.empty_like(B)
    om = torch.full((p.N,), 1.0, dtype=torch.float64, device="cuda:0")
    om[:p.n_pool] = p.b / p.n_pool
    for _ in range(warmup):
        ctx.hvp(B, omega=om, shift=p.lam, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.hvp(B, omega=om, shift=p.lam, out=out)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    leg = {"hvp_ms": 1e3 * el / steps, "hvp_tflops": flops * steps / el / 1e12}
    # the kernels of the product, each with event pairs attached to its launches; each of the
    # two contractions does half of the product's algorithmic flops (2 N c d s)
    kern = {}
    for name in ("product", "product_t"):
        ctx.profile_begin(name)
        for _ in range(prof_reps):
            ctx.hvp(B, omega=om, shift=p.lam, out=out)
        ms, n = ctx.profile_end()
        if n == 0:
            continue
        half = 2.0 * p.N * p.c * p.d * p.s * prof_reps
        kern[name] = {"launches_per_product": n // prof_reps, "ms_per_product": ms / prof_reps,
                      "avg_launch_us": 1e3 * ms / n, "tflops": half / (ms / 1e3) / 1e12}
    leg["kernels"] = kern
    return leg, el


def relax_leg(ctx, p, iters, max_cg):
    """Whole Relax iterations t = 1..iters from w = 1/n at the workload's PCG tolerance."""
    import torch

    from paper_2409_07392_amd import default_beta0
    w = torch.full((p.n_pool,), 1.0 / p.n_pool, dtype=torch.float64, device="cuda:0")
    beta0 = default_beta0(p.n_pool, p.T)
    out = []
    for t in range(1, iters + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = ctx.relax_step(w, p.b, p.lam, beta0, p.probe_seed, t, p.s, p.tol, max_cg, True)
        torch.cuda.synchronize()
        out.append({"t": t, "s": time.perf_counter() - t0, "cg_iters": list(info["cg_iters"]),
                    "converged": info["converged"], "relres_max": info["relres_max"],
                    "f_hat": info["f_hat"]})
        log(f"  Relax iteration {t}: {out[-1]['s']:.2f} s, CG {info['cg_iters']}")
    return out


def fixed_cg_gradient(ctx, p, n_cg):
    """The eq. 11 gradient of iteration 1 with exactly n_cg CG iterations per solve."""
    import torch

    from paper_2409_07392_amd import default_beta0
    w = torch.full((p.n_pool,), 1.0 / p.n_pool, dtype=torch.float64, device="cuda:0")
    g = torch.empty_like(w)
    ctx.relax_step(w, p.b, p.lam, default_beta0(p.n_pool, p.T), p.probe_seed, 1, p.s, 0.0, n_cg,
                   True, g_out=g)
    return g.cpu().numpy()


def cpu_baseline_products(p, rows=12820, budget_s=15.0):
    """The FP64 oracle's product (Lemma 1, NumPy) on the first `rows` rows (1%) of the same
    workload, timed on the host: TFLOP/s over whole calls, repeated for about budget_s seconds."""
    import numpy as np

    from oracle import relax as orc
    X = p.X[:rows].double().cpu().numpy()
    H = p.H[:rows].double().cpu().numpy()
    from oracle.relax import probes
    B = probes(p.probe_seed, 1, p.d, p.s, p.c)
    om = np.full(rows, p.b / p.n_pool)
    flops = 4.0 * rows * p.c * p.d * p.s
    t0 = time.perf_counter()
    calls = 0
    while calls < 1 or (time.perf_counter() - t0 < budget_s and calls < 64):
        orc.hvp(X, H, om, p.lam, B)
        calls += 1
    dt = time.perf_counter() - t0
    return {"value": flops * calls / dt / 1e12, "unit": "TFLOP/s", "cores": int(host_threads()),
            "kind": "oracle",
            "sample": f"{calls} calls of the FP64 NumPy product over the first {rows} rows (1%) "
                      f"of the same workload ({p.d} x {p.s} x {p.c} blocks), {dt:.1f} s; the "
                      "rate is per Hessian-product flop, as `value`"}


def dirichlet_weights_device(p, seed):
    """z = b x Dirichlet(1) over the pool, drawn on the GPU (the weights of the Round legs)."""
    import torch
    g = torch.Generator(device="cuda:0")
    g.manual_seed(seed)
    e = -torch.log(torch.rand(p.n_pool, generator=g, device="cuda:0", dtype=torch.float64))
    return p.b * e / e.sum()


def round_legs(p, args, seed):
    """The Round step from Dirichlet weights, FP32 and FP64 decisions (`--round-rounds`)."""
    import torch
    z = dirichlet_weights_device(p, seed)
    eta = 8.0 * (p.d * p.c) ** 0.5 if args.eta is None else args.eta
    rounds = {}
    for fp32 in (True, False):
        log(f"Round step, {'FP32' if fp32 else 'FP64'} decision")
        rounds["fp32_decision" if fp32 else "fp64_decision"] = round_large(
            p, z, eta, args.round_rounds, fp32)
        torch.cuda.empty_cache()
    return rounds


def headline(args):
    import numpy as np
    import torch

    from paper_2409_07392_amd import RelaxContext
    from synthdata.device import make_problem_device
    log("drawing configuration 4 on the GPU")
    p = make_problem_device(4, device="cuda:0")
    flops = 4.0 * p.N * p.c * p.d * p.s
    rounds = round_legs(p, args, 4004) if args.round_rounds > 0 else {}
    if args.round_only:
        print(json.dumps({"workload": "configuration 4", "round_step": rounds}), flush=True)
        return
    legs, grads, main = {}, {}, None
    precs = ["bf16x3"] if args.only_bf16x3 else ["f32"] + ([] if args.no_bf16x3 else ["bf16x3"])
    for prec in precs:
        log(f"{prec}: context")
        ctx = RelaxContext(p.X, p.H, p.n_pool, p.s, prec)
        log(f"{prec}: {args.steps} timed products")
        leg, el = product_leg(ctx, p, prec, args.steps, args.warmup, args.prof_reps)
        if main is None:
            main = (leg, el, prec)
        log(f"{prec}: {leg['hvp_ms']:.1f} ms per product; Relax iterations at tol {p.tol}")
        leg["relax_iterations"] = relax_leg(ctx, p, args.relax_iters, args.relax_max_cg)
        leg["relax_iter_s"] = (float(np.median([r["s"] for r in leg["relax_iterations"]]))
                               if leg["relax_iterations"] else None)
        if not args.no_grad_error:
            log(f"{prec}: gradient at {args.grad_cg} fixed CG iterations")
            grads[prec] = fixed_cg_gradient(ctx, p, args.grad_cg)
        legs[prec] = leg
        ctx.close()
        del ctx
        torch.cuda.empty_cache()
    if not args.no_grad_error:
        log("f64: reference gradient")
        ctx = RelaxContext(p.X.double(), p.H.double(), p.n_pool, p.s, "f64")
        ref = fixed_cg_gradient(ctx, p, args.grad_cg)
        ctx.close()
        del ctx
        torch.cuda.empty_cache()
        nrm = np.linalg.norm(ref)
        for k in grads:
            legs[k]["rel_grad_err_vs_f64"] = float(np.linalg.norm(grads[k] - ref) / nrm)
            legs[k]["grad_error_cg_iters"] = args.grad_cg
    leg, el, mprec = main
    kern = leg["kernels"]
    dom = max(kern, key=lambda k: kern[k]["ms_per_product"])
    pre = "k_nt" if mprec == "f32" else "k_nt3"
    kname = {"product": f"{pre}_xv (first contraction X V^T with the row sums of Lemma 1, "
                        f"{mprec})",
             "product_t": f"{pre}_xtg{'_m<3>' if p.d <= 384 else ''} (second contraction "
                          f"X^T G'^T with the row step, {mprec})"}[dom]
    traffic_file = {"product": f"{pre}_xv_cfg4_traffic.md",
                    "product_t": f"{pre}_xtg_cfg4_traffic.md"}[dom]
    res = {
        "metric": METRIC,
        "value": flops * args.steps / el / 1e12,
        "unit": "TFLOP/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * el / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": mprec,
        "data": "synthetic",
        "config": {"workload": "cfg4: full Hessian product (Lemma 1) per step, n=1280000+2000 "
                               "labeled, d=384, c=1000, s=16, b=1000, PCG tol 1e-5",
                   "step_flop": flops, "pcg": "projected",
                   "relax_iter_s_f32": legs.get("f32", {}).get("relax_iter_s"),
                   "relax_iter_s_bf16x3": legs.get("bf16x3", {}).get("relax_iter_s")},
        "precision_legs": legs,
        "roofline": {"bound": "mfma", "kernel": kname,
                     "achieved": kern[dom]["tflops"], "peak": PEAK[mprec], "unit": "TFLOP/s",
                     "frac": kern[dom]["tflops"] / PEAK[mprec],
                     "avg_launch_us": kern[dom]["avg_launch_us"],
                     "algorithmic_flop_per_launch": 2.0 * p.N * p.c * p.d * p.s /
                     max(kern[dom]["launches_per_product"], 1),
                     "traffic": read_traffic(traffic_file),
                     "hbm_frac": hbm_frac(read_traffic(traffic_file), kern[dom]["avg_launch_us"])},
    }
    if rounds:
        res["round_step"] = rounds
    if not args.no_cpu_baseline:
        log("cpu baseline: oracle products on a 1% row sample")
        res["cpu_baseline"] = cpu_baseline_products(p)
    print(json.dumps(res), flush=True)


# --------------------------------------------------------------- configuration 2

def cpu_baseline_relax(p, beta0, project, budget_s=10.0, max_iters=8):
    """Time the FP64 oracle on full-size Relax iterations of configuration 2: iterations
    t = 1, 2, ... until about budget_s seconds of CPU work (at most max_iters)."""
    import numpy as np

    from oracle import relax as orc
    w = np.full(p.n_pool, 1.0 / p.n_pool)
    t0 = time.perf_counter()
    it = 0
    while it < max_iters and (it == 0 or time.perf_counter() - t0 < budget_s):
        it += 1
        w, _ = orc.relax_iteration(p.X, p.H, p.n_pool, w, p.b, p.lam, beta0, p.probe_seed, it,
                                   p.s, p.tol, 1000, project=project)
    dt = time.perf_counter() - t0
    return {"value": it / dt, "unit": "relax_iter/s", "cores": int(host_threads()),
            "kind": "oracle",
            "sample": f"Relax iterations t=1..{it} of the same full-size workload in FP64 NumPy "
                      f"on the host, {dt:.1f} s"}


def run_leg(p, prec, steps, warmup, project, hvp_reps):
    """Time `steps` Relax iterations and the Hessian product in one precision."""
    import numpy as np
    import torch

    from paper_2409_07392_amd import RelaxContext, default_beta0
    dt = torch.float64 if prec == "f64" else torch.float32
    dev = torch.device("cuda:0")
    X = torch.as_tensor(p.X, dtype=dt, device=dev).contiguous()
    H = torch.as_tensor(p.H, dtype=dt, device=dev).contiguous()
    ctx = RelaxContext(X, H, p.n_pool, p.s, prec)
    beta0 = default_beta0(p.n_pool, p.T)
    wtmp = torch.full((p.n_pool,), 1.0 / p.n_pool, dtype=torch.float64, device=dev)
    for t in range(1, warmup + 1):
        ctx.relax_step(wtmp, p.b, p.lam, beta0, p.probe_seed, t, p.s, p.tol, 1000, project)
    w = torch.full((p.n_pool,), 1.0 / p.n_pool, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = [ctx.relax_step(w, p.b, p.lam, beta0, p.probe_seed, t, p.s, p.tol, 1000, project)
             for t in range(1, steps + 1)]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    B = ctx.probes(p.probe_seed, 1, p.s)
    out = torch.empty_like(B)
    om = torch.full((p.N,), 1.0, dtype=torch.float64, device=dev)
    om[:p.n_pool] = p.b / p.n_pool
    for _ in range(3):
        ctx.hvp(B, omega=om, shift=p.lam, out=out)
    # whole product call (main kernel + split-sum reduction), events on the call's stream
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(hvp_reps):
        ctx.hvp(B, omega=om, shift=p.lam, out=out)
    ev1.record(stream)
    torch.cuda.synchronize()
    t_hvp = ev0.elapsed_time(ev1) / 1e3 / hvp_reps
    # the main product kernel alone: the library's event pairs around each launch
    ctx.profile_begin()
    for _ in range(hvp_reps):
        ctx.hvp(B, omega=om, shift=p.lam, out=out)
    k_ms, k_n = ctx.profile_end()
    t_kern = k_ms / 1e3 / max(k_n, 1)
    flops = 4.0 * p.N * p.c * p.d * p.s
    ctx.close()
    return dict(w=w, elapsed=elapsed, ms=1e3 * elapsed / steps, value=steps / elapsed,
                cg=float(np.mean([i["cg_iters"][0] + i["cg_iters"][1] for i in infos])),
                t_hvp=t_hvp, hvp_tflops=flops / t_hvp / 1e12, t_kern=t_kern,
                kern_tflops=flops / t_kern / 1e12, f_hat_last=infos[-1]["f_hat"])



def grad_errors(p, project, n_cg=15):
    """Relative gradient error of FP32 and bf16x3 against the GPU FP64 mode (same probes,
    same fixed number of CG iterations, so only arithmetic precision differs)."""
    import numpy as np
    import torch

    from paper_2409_07392_amd import RelaxContext, default_beta0
    dev = torch.device("cuda:0")
    beta0 = default_beta0(p.n_pool, p.T)
    Xf = np.asarray(p.X, dtype=np.float32)
    Hf = np.asarray(p.H, dtype=np.float32)
    g = {}
    for prec in ("f64", "f32", "bf16x3"):
        dt = torch.float64 if prec == "f64" else torch.float32
        ctx = RelaxContext(torch.as_tensor(Xf, dtype=dt, device=dev),
                           torch.as_tensor(Hf, dtype=dt, device=dev), p.n_pool, p.s, prec)
        w = torch.full((p.n_pool,), 1.0 / p.n_pool, dtype=torch.float64, device=dev)
        gt = torch.empty_like(w)
        ctx.relax_step(w, p.b, p.lam, beta0, p.probe_seed, 1, p.s, 0.0, n_cg, project, g_out=gt)
        g[prec] = gt.cpu().numpy()
        ctx.close()
    ref = np.linalg.norm(g["f64"])
    return {k: float(np.linalg.norm(g[k] - g["f64"]) / ref) for k in ("f32", "bf16x3")}



def round_leg(p, w, eta, fp32, cpu_rounds=2):
    """The Round step (Algorithm 3) at the same workload: all b rounds from z = b w (the
    Relax leg's final weights).  fp32: the per-point objective and its argmax in FP32 (the
    paper's precision), else FP64; the block state is FP64 either way.  Reports ms per selected
    point, the scoring kernel's time and MFMA rate, and the oracle's time per round on the host
    (same decision precision)."""
    import numpy as np
    import torch

    from paper_2409_07392_amd import RelaxContext, RoundSolver
    dev = torch.device("cuda:0")
    X = torch.as_tensor(p.X, dtype=torch.float32, device=dev).contiguous()
    H = torch.as_tensor(p.H, dtype=torch.float32, device=dev).contiguous()
    ctx = RelaxContext(X, H, p.n_pool, 1, "f32")
    z = (p.b * w).contiguous()
    b = int(p.b)
    warm = RoundSolver(ctx, z, p.lam, eta, b, fp32=fp32)
    warm.step(2)
    warm.result()
    warm.close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rs = RoundSolver(ctx, z, p.lam, eta, b, fp32=fp32)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    ctx.profile_begin("round_score")
    t0 = time.perf_counter()
    rs.step(b)
    res = rs.result()
    elapsed = time.perf_counter() - t0
    k_ms, k_n = ctx.profile_end()
    flops = 2.0 * p.n_pool * p.c * p.d * p.d     # algorithmic: one d x d product per class
    t_kern = k_ms / 1e3 / b                      # the round's scoring launches
    rs.close()
    ctx.close()
    # the oracle on the host: the first rounds of the same solve
    from oracle import round as orr
    Xo = X.cpu().numpy().astype(np.float64)
    Ho = H.cpu().numpy().astype(np.float64)
    zo = z.cpu().numpy()
    tc = time.perf_counter()
    st = orr.DiagonalRound(Xo, Ho, p.n_pool, zo, p.lam, eta, b, fp32=fp32)
    for _ in range(cpu_rounds):
        st.step()
    t_cpu = (time.perf_counter() - tc) / cpu_rounds
    same = [int(i) for i in st.selected] == [int(i) for i in res["selected"][:cpu_rounds]]
    pk = PEAK["f32" if fp32 else "f64"]
    kname = ("k_round_score<float, float> (per-point objective, FP32 MFMA; achieved counts "
             "2 n c d^2 per round)" if fp32 else
             "k_round_score<float, double> (per-point objective, FP64 MFMA; achieved counts "
             "2 n c d^2 per round)")
    return {"decision": "fp32" if fp32 else "fp64", "rounds": res["t"], "eta": eta,
            "ms_per_point": 1e3 * elapsed / b,
            "points_per_s": b / elapsed, "setup_ms": 1e3 * t_setup,
            "first_selected": [int(i) for i in res["selected"][:8]],
            "roofline": {"bound": "mfma", "kernel": kname,
                         "achieved": flops / t_kern / 1e12, "peak": pk,
                         "unit": "TFLOP/s", "frac": flops / t_kern / 1e12 / pk,
                         "kernel_us": t_kern * 1e6, "traffic": read_traffic("round_score_fp32_cfg2_traffic.md" if fp32 else "round_score_fp64_cfg2_traffic.md"),
                         "executed_tflops": 1.5 * flops / t_kern / 1e12},
            "cpu_oracle": {"s_per_round": t_cpu, "rounds_timed": cpu_rounds,
                           "same_first_selections": same}}




def round_large(p, z, eta, rounds, fp32):
    """The Round step on a large workload: set-up, then `rounds` rounds after one untimed
    round, from the relaxed weights z (FP32 context; decision precision FP32 or FP64)."""
    import torch

    from paper_2409_07392_amd import RelaxContext, RoundSolver
    ctx = RelaxContext(p.X.contiguous(), p.H.contiguous(), p.n_pool, 1, "f32")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rs = RoundSolver(ctx, z, p.lam, eta, int(p.b), fp32=fp32)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    rs.step(1)
    rs.result()
    ctx.profile_begin("round_score")
    t0 = time.perf_counter()
    rs.step(rounds)
    res = rs.result()
    elapsed = time.perf_counter() - t0
    k_ms, k_n = ctx.profile_end()
    t_kern = k_ms / 1e3 / rounds               # the round's scoring launches (row chunks)
    flops = 2.0 * p.n_pool * p.c * p.d * p.d   # algorithmic: one d x d product per class
    executed = 1.5 * flops                     # u = L^-1 x (triangular) and v = D^-1 L^-1 x
    pk = PEAK["f32" if fp32 else "f64"]
    rs.close()
    ctx.close()
    return {"decision": "fp32" if fp32 else "fp64", "eta": eta, "rounds_timed": rounds,
            "setup_s": t_setup, "s_per_point": elapsed / rounds,
            "score_s_per_round": t_kern, "score_launches_per_round": k_n // rounds,
            "score_tflops": flops / t_kern / 1e12,
            "score_frac_of_peak": flops / t_kern / 1e12 / pk,
            "score_executed_tflops": executed / t_kern / 1e12,
            "selected": [int(i) for i in res["selected"]]}



def studies_workload(args):
    """Relax and Round studies on synthetic data, analogues of the paper's figures:
    fig1 - CG against block-Jacobi PCG (literal and projected) in the first mirror-descent
           iteration: relative residual after k iterations, and iterations to 1e-6;
    fig4 - the objective f(z_t) = Tr(Sigma^-1 H_p) (exact: all dc unit probes) along the
           Relax iterations for several probe counts s and CG tolerances;
    fig5 - Relax (preconditioner, 50 fixed CG iterations) and Round (one round: scoring
           and the rest) times as d and c grow."""
    import numpy as np
    import torch

    from paper_2409_07392_amd import RelaxContext, RoundSolver, default_beta0
    from synthdata import make_problem
    from synthdata.device import draw_device
    dev = torch.device("cuda:0")
    res = {}
    parts = args.study.split(",")

    def ctx_for(p, s_max):
        X = torch.as_tensor(p.X, dtype=torch.float32, device=dev).contiguous()
        H = torch.as_tensor(p.H, dtype=torch.float32, device=dev).contiguous()
        return RelaxContext(X, H, p.n_pool, s_max, "f32")

    # CIFAR-10 shape of the accuracy experiments (Table 4): n = 3000, d = 20, c = 10, n_o = 10
    small = make_problem(2, n=3000, n_lab=10, d=20, c=10, s=10, b=10.0, K=10, seed=7010)
    if "fig1" in parts:
        log("fig1: CG and PCG residuals")
        p = small
        ctx = ctx_for(p, p.s)
        om = torch.full((p.N,), 1.0, dtype=torch.float64, device=dev)
        om[:p.n_pool] = p.b / p.n_pool
        V = ctx.probes(p.probe_seed, 1, p.s)
        _, Pinv, _ = ctx.build_precond(om, p.lam, want_L=False)
        eye = torch.eye(p.d, dtype=torch.float64, device=dev).expand(p.c, p.d, p.d).contiguous()
        variants = {"cg": (eye, False), "cg_projected": (eye, True),
                    "pcg": (Pinv, False), "pcg_projected": (Pinv, True)}
        fig1 = {}
        for name, (P, proj) in variants.items():
            curve = []
            for k in range(1, 61):
                _, info = ctx.pcg_solve(V, P, om, p.lam, tol=0.0, max_iter=k, project=proj)
                curve.append(info["relres_max"])
            _, info = ctx.pcg_solve(V, P, om, p.lam, tol=1e-6, max_iter=5000, project=proj)
            fig1[name] = {"relres_after_k": curve, "iters_to_1e-6": info["cg_iters"][0]}
        ctx.close()
        res["fig1"] = {"problem": "n = 3000 + 10, d = 20, c = 10, s = 10, z = b/n (first "
                                  "mirror-descent iteration), lambda = 1e-3",
                       "variants": fig1}
    if "fig4" in parts:
        log("fig4: objective trajectories")
        p = small
        dc = p.d * p.c
        ctx = ctx_for(p, dc)
        U = torch.zeros((p.d, dc, p.c), dtype=torch.float32, device=dev)   # all unit probes
        for k in range(p.c):
            for a in range(p.d):
                U[a, k * p.d + a, k] = 1.0

        def exact_f(w):
            f, _, _ = ctx.sampled_objective((p.b * w).contiguous(), p.lam, U, tol=1e-9,
                                            max_iter=5000, project=False, grad=False)
            return f * dc
        T = 30
        beta0 = default_beta0(p.n_pool, T)
        runs = {}
        for s_, tol in ((2, 1e-3), (10, 1e-3), (50, 1e-3), (10, 1e-1), (10, 1e-6)):
            w = torch.full((p.n_pool,), 1.0 / p.n_pool, dtype=torch.float64, device=dev)
            traj = {0: exact_f(w)}
            for t in range(1, T + 1):
                ctx.relax_step(w, p.b, p.lam, beta0, p.probe_seed, t, s_, tol, 5000, True)
                if t in (1, 2, 5, 10, 20, 30):
                    traj[t] = exact_f(w)
            runs[f"s={s_},cg_tol={tol:g}"] = traj
        ctx.close()
        res["fig4"] = {"problem": "n = 3000 + 10, d = 20, c = 10, b = 10, T = 30, projected "
                                  "PCG; f exact (all dc unit probes, PCG to 1e-9)",
                       "objective_at_iteration": runs}
    if "fig5" in parts:
        fig5 = {"d_sweep": {}, "c_sweep": {}}

        def one(name, n, n_lab, d, c, key, store):
            log(f"fig5: {name}")
            pr = dict(n=n, n_lab=n_lab, d=d, c=c, s=10, b=float(c), lam=1e-3, tol=1e-6, T=1,
                      K=c, whiten=False, probs="maxprob")
            q = draw_device(name, pr, 9000 + d + c, 9500 + d + c, dev, torch.float32)
            ctx = RelaxContext(q.X, q.H, q.n_pool, 10, "f32")
            om = torch.full((q.N,), 1.0, dtype=torch.float64, device=dev)
            om[:q.n_pool] = q.b / q.n_pool
            ctx.build_precond(om, q.lam, want_L=False)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, Pinv, _ = ctx.build_precond(om, q.lam, want_L=False)
            torch.cuda.synchronize()
            t_pre = time.perf_counter() - t0
            V = ctx.probes(q.probe_seed, 1, 10)
            t0 = time.perf_counter()
            ctx.pcg_solve(V, Pinv, om, q.lam, tol=0.0, max_iter=50, project=True)
            torch.cuda.synchronize()
            t_cg = time.perf_counter() - t0
            z = om[:q.n_pool].contiguous()
            rs = RoundSolver(ctx, z, q.lam, 8.0 * (d * c) ** 0.5, 2, fp32=True)
            ctx.profile_begin("round_score")
            t0 = time.perf_counter()
            rs.step(1)
            rs.result()
            t_round = time.perf_counter() - t0
            k_ms, _ = ctx.profile_end()
            rs.close()
            ctx.close()
            del q, ctx, Pinv, V
            torch.cuda.empty_cache()
            store[key] = {"n": n, "d": d, "c": c, "precond_s": t_pre, "cg50_s": t_cg,
                          "round_s": t_round, "round_score_s": k_ms / 1e3,
                          "round_other_s": t_round - k_ms / 1e3}
        for d in (383, 766, 1022):
            one(f"d{d}", 100000, 1000, d, 1000, d, fig5["d_sweep"])
        for c in (100, 200, 400, 800, 1000):
            one(f"c{c}", 1280000, 2000, 383, c, c, fig5["c_sweep"])
        res["fig5"] = dict(fig5, problem="d sweep: n = 1e5, c = 1000; c sweep: n = 1.28e6, "
                                         "d = 383; s = 10, 50 fixed CG iterations, FP32; one "
                                         "Round round with the FP32 decision")
    print(json.dumps({"workload": "studies", "data": "synthetic", "results": res}))



def batch_workload(args):
    """Configuration 5: 64 independent problems (uneven n, d, c) for 30 Relax iterations, as
    one captured graph replayed 30 times and as the same iterations one call at a time."""
    import torch

    from paper_2409_07392_amd import RelaxBatch, RelaxContext, default_beta0
    from synthdata.device import batch_problems_device
    prec = args.prec if args.prec != "f64" else "f32"
    log("drawing the 64 problems on the GPU")
    plist = batch_problems_device(64, device="cuda:0")
    iters = 30
    max_iter = 100

    def contexts():
        out = []
        for p in plist:
            ctx = RelaxContext(p.X, p.H, p.n_pool, p.s, prec)
            w = torch.full((p.n_pool,), 1.0 / p.n_pool, dtype=torch.float64, device="cuda:0")
            out.append((p, ctx, w))
        return out

    log("batch: tune, warm up, capture")
    A = contexts()
    probs = [dict(ctx=ctx, w=w, b=p.b, lam=p.lam, beta0=default_beta0(p.n_pool, p.T),
                  seed=p.probe_seed, t0=1, s=p.s, tol=p.tol, max_iter=max_iter, project=True)
             for p, ctx, w in A]
    t0 = time.perf_counter()
    batch = RelaxBatch(probs)
    t_create = time.perf_counter() - t0
    log("batch: 30 replays")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    batch.run(iters)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    cg = [batch.info(i)["cg_iters"] for i in range(len(A))]
    log("one call at a time")
    B = contexts()
    for (p, ctx, w), (_, ca, _) in zip(B, A):
        ctx.autotune(p.s)   # the batch's variants (same bucket)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    by_bucket = {}   # (d, c) -> [problems, seconds, rows]: where the sequential time goes
    for p, ctx, w in B:
        beta0 = default_beta0(p.n_pool, p.T)
        tp = time.perf_counter()
        for t in range(1, iters + 1):
            ctx.relax_step(w, p.b, p.lam, beta0, p.probe_seed, t, p.s, p.tol, max_iter, True)
        torch.cuda.synchronize()
        e = by_bucket.setdefault("d%d_c%d" % (p.d, p.c), [0, 0.0, 0])
        e[0] += 1
        e[1] += time.perf_counter() - tp
        e[2] += p.n_pool + p.n_lab
    t_seq = time.perf_counter() - t0
    maxdiff = max(float((a[2] - b[2]).abs().max()) for a, b in zip(A, B))
    flops = sum(4.0 * (p.n_pool + p.n_lab) * p.c * p.d * p.s for p in plist)
    res = {
        "metric": METRIC,
        "workload": "configuration 5: 64 problems, n in [5k, 100k], d in {64,128,256}, "
                    "c in {10,50,100}, s = 16, 30 iterations each",
        "dtype": prec,
        "problem_iters_per_s_batched": len(plist) * iters / t_batch,
        "problem_iters_per_s_one_at_a_time": len(plist) * iters / t_seq,
        "batched_s": t_batch, "one_at_a_time_s": t_seq, "speedup": t_seq / t_batch,
        "capture_and_tune_s": t_create,
        "max_abs_weight_difference_batched_vs_one_at_a_time": maxdiff,
        "mean_cg_iters_last_iteration": float(sum(a + b for a, b in cg) / (2 * len(cg))),
        "sum_product_gflop_per_iteration_all_problems": flops / 1e9,
        "one_at_a_time_by_bucket": {k: {"problems": v[0], "seconds": v[1], "rows": v[2]}
                                    for k, v in sorted(by_bucket.items())},
    }
    batch.close()
    print(json.dumps(res))



def calibrate_copy(mib):
    """A plain device copy of `mib` MiB (for scaling the FETCH_SIZE / WRITE_SIZE counters)."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n * 4}))



def workload2(args):
    """Configuration 2: whole Relax iterations per step (FP32, then bf16x3), the Round step on
    the Relax leg's weights, and the oracle's Relax iterations on the host."""
    from paper_2409_07392_amd import default_beta0
    from synthdata import make_problem

    p = make_problem(2)
    if args.eta is None:
        args.eta = 8.0 * (p.d * p.c) ** 0.5
    project = not args.literal
    main_leg = run_leg(p, args.prec, args.steps, args.warmup, project, args.hvp_reps)
    legs = {args.prec: main_leg}
    if args.prec != "bf16x3" and not args.no_bf16x3:
        legs["bf16x3"] = run_leg(p, "bf16x3", args.steps, args.warmup, project, args.hvp_reps)
    errs = grad_errors(p, project)
    rnd = None if args.no_round else {
        "fp32_decision": round_leg(p, main_leg["w"], args.eta, True),
        "fp64_decision": round_leg(p, main_leg["w"], args.eta, False)}
    peak = PEAK[args.prec]
    kname = {"f32": "k_hvp_fused (fused Lemma 1 product, FP32)",
             "bf16x3": "k_hvp_fused_bf3 (fused Lemma 1 product, bf16x3)",
             "f64": "k_xv (row-tiled first contraction, FP64)"}[args.prec]
    tfile = {"f32": "k_hvp_fused_cfg2_traffic.md", "bf16x3": "k_hvp_fused_bf3_cfg2_traffic.md",
             "f64": ""}[args.prec]
    res = {
        "metric": METRIC,
        "value": main_leg["value"],
        "unit": "relax_iter/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": main_leg["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.prec,
        "data": "synthetic",
        "config": {"workload": "relax cfg2: n=50000+10 labeled, d=100, c=10, s=20, tol=1e-6, b=100",
                   "pcg": "projected" if project else "literal",
                   "mean_cg_iters_per_step": main_leg["cg"],
                   "hvp_ms": main_leg["t_hvp"] * 1e3, "hvp_tflops": main_leg["hvp_tflops"],
                   "f_hat_last": main_leg["f_hat_last"]},
        "precision_legs": {k: {"ms_per_step": v["ms"], "relax_iter_per_s": v["value"],
                               "hvp_ms": v["t_hvp"] * 1e3, "hvp_tflops": v["hvp_tflops"],
                               "kernel_us": v["t_kern"] * 1e6, "kernel_tflops": v["kern_tflops"],
                               "mean_cg_iters_per_step": v["cg"],
                               "rel_grad_err_vs_f64": errs.get(k)}
                           for k, v in legs.items()},
        "roofline": {"bound": "mfma", "kernel": kname,
                     "achieved": main_leg["kern_tflops"], "peak": peak, "unit": "TFLOP/s",
                     "frac": main_leg["kern_tflops"] / peak,
                     "kernel_us": main_leg["t_kern"] * 1e6,
                     "traffic": read_traffic(tfile) if tfile else None,
                     "hbm_frac": hbm_frac(read_traffic(tfile) if tfile else None,
                                          main_leg["t_kern"] * 1e6)},
    }
    if rnd is not None:
        res["round_step"] = rnd
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline_relax(p, default_beta0(p.n_pool, p.T), project)
    print(json.dumps(res))


def workload3(args):
    """Configuration 3: the sampled objective and its adjoint gradient (extension 3) at a
    Dirichlet z, FP32 and bf16x3, with the gradient error against the GPU FP64 mode at a fixed CG
    count; optionally the Round step."""
    import numpy as np
    import torch

    from paper_2409_07392_amd import RelaxContext
    from synthdata.device import make_problem_device
    log("drawing configuration 3 on the GPU")
    p = make_problem_device(3, device="cuda:0")
    flops = 4.0 * p.N * p.c * p.d * p.s
    z = dirichlet_weights_device(p, 3003)
    rounds = round_legs(p, args, 3003) if args.round_rounds > 0 else {}
    if args.round_only:
        print(json.dumps({"workload": "configuration 3", "round_step": rounds}))
        return
    legs, grads = {}, {}
    n_cg = 20
    for prec in ("f32", "bf16x3") if args.no_adjoint else ("f32", "bf16x3", "f64"):
        dt = torch.float64 if prec == "f64" else torch.float32
        ctx = RelaxContext(p.X.to(dt).contiguous(), p.H.to(dt).contiguous(), p.n_pool, p.s, prec)
        V = ctx.probes(p.probe_seed, 1, p.s)
        if prec != "f64":
            log(f"{prec}: products" + ("" if args.no_adjoint else " and the objective with its adjoint"))
            leg, _ = product_leg(ctx, p, prec, args.steps, args.warmup, args.prof_reps)
            legs[prec] = leg
            if args.no_adjoint:
                ctx.close()
                del ctx
                torch.cuda.empty_cache()
                continue
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            f, _, info = ctx.sampled_objective(z, p.lam, V, tol=p.tol, max_iter=1000, project=True)
            torch.cuda.synchronize()
            leg["objective_and_adjoint_ms"] = (time.perf_counter() - t0) * 1e3
            leg["cg_iters"] = list(info["cg_iters"])
            leg["f"] = f
        log(f"{prec}: adjoint gradient at {n_cg} fixed CG iterations")
        _, gv, _ = ctx.sampled_objective(z, p.lam, V, tol=0.0, max_iter=n_cg, project=True)
        grads[prec] = gv.cpu().numpy()
        ctx.close()
        del ctx
        torch.cuda.empty_cache()
    if not args.no_adjoint:
        ref = np.linalg.norm(grads["f64"])
        for prec in ("f32", "bf16x3"):
            legs[prec]["rel_grad_err_vs_f64"] = float(np.linalg.norm(grads[prec] - grads["f64"]) / ref)
    res = {"metric": METRIC, "workload": "configuration 3",
           "config": {"n_pool": p.n_pool, "n_lab": p.n_lab, "d": p.d, "c": p.c, "s": p.s,
                      "b": p.b, "tol": p.tol, "z": "b x Dirichlet(1), drawn on the GPU",
                      "step_flop": flops},
           "precision_legs": legs}
    if rounds:
        res["round_step"] = rounds
    print(json.dumps(res))


def al_workload(args):
    """A synthetic active-learning loop (ImageNet-50 shape of the accuracy experiments: c = 50,
    d = 50, pool 5000, 20,000 evaluation points, one labeled point per class to start, 6 rounds
    of 50): each round a multinomial logistic regression (scikit-learn, host) is trained on the
    labeled points and FIRAL selects the next 50 on the GPU: Relax (s = 10, CG relative residual
    0.1, the relative-change stop at 1e-4, at most 100 iterations) then the Round step with the
    eta choice over 5 values around 8 sqrt(dc), FP32 decision.  Reports the evaluation accuracy
    after every round and the GPU seconds per round."""
    import torch

    from paper_2409_07392_amd import RelaxContext, round_eta_sweep
    from synthdata.al import al_loop
    c, d, n_pool, n_eval, rounds, b = 50, 50, 5000, 20000, 6, 50
    lam, s, eta0 = 1e-3, 10, 8.0 * (d * c) ** 0.5
    times = []

    def select(X, H, n_unl, t):
        dev = torch.device("cuda:0")
        ctx = RelaxContext(torch.as_tensor(X, dtype=torch.float32, device=dev).contiguous(),
                           torch.as_tensor(H, dtype=torch.float32, device=dev).contiguous(),
                           n_unl, s, "f32")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        z, info = ctx.relax(float(b), lam, 9000 + t, 100, s, 0.1, 1000, project=True,
                            stop_rel=1e-4)
        torch.cuda.synchronize()
        t_relax = time.perf_counter() - t0
        t0 = time.perf_counter()
        sw = round_eta_sweep(ctx, z, lam, [eta0 / 8, eta0 / 2, eta0, 2 * eta0, 8 * eta0], b,
                             fp32=True)
        t_round = time.perf_counter() - t0
        ctx.close()
        times.append({"round": t + 1, "relax_s": t_relax, "relax_iters": info["iters"],
                      "round_and_eta_choice_s": t_round, "eta": sw["best"]})
        log(f"round {t + 1}: Relax {t_relax:.3f} s ({info['iters']} iterations), "
            f"Round {t_round:.3f} s")
        return sw["selected"]

    res = al_loop(select, c, d, n_pool, n_eval, rounds, seed=8000)
    print(json.dumps({"workload": "synthetic active learning, ImageNet-50 shape",
                      "data": "labeled Gaussian mixture: 50 classes, d = 50, cluster means "
                              "N(0, 0.25 I), unit noise; pool 5000, evaluation 20,000",
                      "classifier": "scikit-learn LogisticRegression (multinomial, C = 1)",
                      "eval_accuracy_after_round": res["accuracy"], "firal_gpu_seconds": times}))


def main():
    args = parse()
    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the library's "
              "Relax and Round paths are single-GPU.", file=sys.stderr)
        sys.exit(2)
    {"4": headline, "2": workload2, "3": workload3, "5": batch_workload,
     "studies": studies_workload, "al": al_workload}[args.workload](args)


if __name__ == "__main__":
    main()
