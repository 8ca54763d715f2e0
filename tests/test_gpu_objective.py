"""The sampled objective f_V(z) and its adjoint gradient (firal_sampled_objective,
RelaxObjective) against the FP64 oracle, finite differences and gradcheck.

Tolerances: FP64 results at PCG tol 1e-13 are compared at the FP64 bar 1e-10 normwise
(the two solves meet 1e-13 on the recurrence residual; kappa of the projected operator is
O(10-100)); FP32 against FP64 at the same fixed CG count at the FP32 bar 1e-5.
"""
import numpy as np
import pytest
import torch

from oracle import relax as orc
from paper_2409_07392_amd import RelaxContext, RelaxObjective
from synthdata import dirichlet_weights, make_problem, make_small

pytestmark = pytest.mark.gpu


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def relerr(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("shape", [(900, 6, 10, 4, 6), (1500, 20, 40, 7, 5)])
@pytest.mark.parametrize("project", [True, False])
def test_objective_and_adjoint_match_oracle(project, shape):
    n, n_lab, d, c, s = shape
    p = make_small(n=n, n_lab=n_lab, d=d, c=c, s=s, seed=21)
    ctx = RelaxContext(dev(p.X), dev(p.H), p.n_pool, p.s, "f64")
    z = dirichlet_weights(np.random.default_rng(3), p.n_pool, 20.0)
    V = orc.probes(31, 1, p.d, p.s, p.c)
    f, g, info = ctx.sampled_objective(dev(z), 1e-3, dev(V), tol=1e-13, max_iter=5000,
                                       project=project)
    fr, gr = orc.sampled_objective_grad(p.X, p.H, p.n_pool, z, 1e-3, V, 1e-13, 5000, project)
    assert info["rc"] == 0
    ef, eg = abs(f - fr) / abs(fr), relerr(g.cpu().numpy(), gr)
    print(f"objective {shape} project={project}: f {ef:.2e}, gradient {eg:.2e}")
    assert ef <= 1e-10, ef
    assert eg <= 1e-10, eg


def test_autograd_gradcheck_tiny():
    p = make_small(n=12, n_lab=3, d=3, c=3, s=4, seed=23)
    ctx = RelaxContext(dev(p.X), dev(p.H), p.n_pool, p.s, "f64")
    V = dev(orc.probes(5, 1, p.d, p.s, p.c))
    z = dev(np.random.default_rng(4).uniform(0.3, 1.0, p.n_pool)).requires_grad_(True)

    def fn(zz):
        return RelaxObjective.apply(zz, ctx, V, 1e-2, 1e-14, 2000, True)

    assert torch.autograd.gradcheck(fn, (z,), eps=1e-6, atol=1e-6, rtol=1e-4)


def test_directional_finite_difference_configuration_2_shape():
    # d = 100, c = 10 with configuration 2's recipe on a 4000-point pool, FP64.  The step is
    # relative (u_i = z_i r_i, r_i = +-1), so the second-order term is ~h^2 f while
    # g^T u ~ f / sqrt(n); with PCG at 1e-12 both error terms stay below 1e-6 of g^T u.
    p = make_problem(2, n=4000)
    ctx = RelaxContext(dev(p.X), dev(p.H), p.n_pool, p.s, "f64")
    rng = np.random.default_rng(2002)
    z = dirichlet_weights(rng, p.n_pool, 10.0 * p.b)
    V = ctx.probes(p.probe_seed, 1, p.s)
    zt = dev(z).requires_grad_(True)
    f = RelaxObjective.apply(zt, ctx, V, p.lam, 1e-12, 5000, True)
    f.backward()
    g = zt.grad.cpu().numpy()
    u = z * rng.choice([-1.0, 1.0], size=p.n_pool)
    h = 1e-4
    fp, _, ip = ctx.sampled_objective(dev(z + h * u), p.lam, V, 1e-12, 5000, True, grad=False)
    fm, _, im = ctx.sampled_objective(dev(z - h * u), p.lam, V, 1e-12, 5000, True, grad=False)
    assert ip["converged"] and im["converged"]
    fd = (fp - fm) / (2 * h)
    assert abs(fd - g @ u) <= 1e-5 * abs(g @ u), (fd, g @ u)


def test_objective_fp32_against_fp64_fixed_iterations():
    p = make_problem(2, n=4000)
    z = dev(np.full(p.n_pool, p.b / p.n_pool))
    out = {}
    for prec, dt in (("f64", torch.float64), ("f32", torch.float32)):
        Xr = np.asarray(p.X, np.float32)
        Hr = np.asarray(p.H, np.float32)
        ctx = RelaxContext(dev(Xr, dt), dev(Hr, dt), p.n_pool, p.s, prec)
        V = ctx.probes(p.probe_seed, 1, p.s)
        f, g, info = ctx.sampled_objective(z, p.lam, V, tol=0.0, max_iter=20, project=True)
        assert info["cg_iters"] == (20, 20)
        out[prec] = (f, g.cpu().numpy())
    assert abs(out["f32"][0] - out["f64"][0]) <= 1e-5 * abs(out["f64"][0])
    assert relerr(out["f32"][1], out["f64"][1]) <= 1e-5
