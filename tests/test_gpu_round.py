"""Parity of the GPU diagonal Round step (Algorithm 3) with the FP64 oracle.

Default mode: both sides decide the argmax in FP64 (the GPU reads FP32 storage exactly; the
oracle gets the same FP32 values).  FP32 mode (FIRAL_ROUND_FP32, the precision of the paper's
implementation): both sides evaluate the objective and take the argmax in FP32 while the block
state stays FP64; the two FP32 evaluations round differently (each rounds its own d-term
products and its FP32 copy of B^-1 or W: about u32 kappa sqrt(d), u32 = 6e-8), so objectives
agree to 1e-4 normwise and a pick may differ from the oracle's only in a round whose two best
objectives are within 1e-4 of each other (either row is then a valid maximiser).  Per case:
* teacher forcing: the oracle is advanced with the GPU's picks; in FP64 each pick must be the
  oracle's own argmax (index work: exact, so the whole sequence equals the oracle's run), in
  FP32 it must attain the oracle's maximum within 1e-4; nu_{t+1} (FP64 state in both modes)
  to 1e-9 and the winning objective to the mode's tolerance;
* the objective of every pool row (firal_round_scores) against the oracle's, normwise 1e-9
  (FP32 mode: 1e-4), before the first round and after the last checked one;
* the eta criterion min_k lambda_min((H)_k) to 1e-8.
Shapes span several scoring tiles and a ragged tail, odd d, no labeled rows, c = 2, d = 1
and the whole pool selected; configuration 2 at its full size (n = 50,000, d = 100, c = 10,
the bench's launch configuration) over its first rounds; a reduced configuration-3 shape
(d = 256, c = 100) for the global-memory tridiagonalisation and several column tiles per
class.
"""
import numpy as np
import pytest
import torch

from oracle import round as orr
from paper_2409_07392_amd import FiralError, RelaxContext, RoundSolver, round_eta_sweep
from synthdata import dirichlet_weights, make_problem, make_small

pytestmark = pytest.mark.gpu

TOL = 1e-9


def setup(p, prec, b, seed=3):
    dt = torch.float64 if prec == "f64" else torch.float32
    X = torch.tensor(p.X, dtype=dt, device="cuda")
    H = torch.tensor(p.H, dtype=dt, device="cuda")
    zn = dirichlet_weights(np.random.default_rng(seed), p.n_pool, float(b))
    z = torch.tensor(zn, dtype=torch.float64, device="cuda")
    Xo = X.cpu().numpy().astype(np.float64)
    Ho = H.cpu().numpy().astype(np.float64)
    ctx = RelaxContext(X, H, p.n_pool, 1, prec)
    return ctx, z, zn, Xo, Ho


def relerr(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


TOL32 = 1e-4


def check_run(p, prec, b, eta, rounds=None, lam=1e-3, fp32=False):
    ctx, z, zn, Xo, Ho = setup(p, prec, b)
    rs = RoundSolver(ctx, z, lam, eta, b, fp32=fp32)
    st = orr.DiagonalRound(Xo, Ho, p.n_pool, zn, lam, eta, b, fp32=fp32)
    tol = TOL32 if fp32 else TOL
    nr = b if rounds is None else rounds
    g0 = rs.scores().cpu().numpy()
    assert relerr(g0, st.scores()) <= tol
    rs.step(nr)
    res = rs.result()
    assert res["t"] == nr
    sel = res["selected"]
    assert len(set(sel.tolist())) == nr and sel.min() >= 0 and sel.max() < p.n_pool
    # teacher-forced validity, nu and the winning objective
    for t in range(nr):
        r = st.scores()
        i_or = st.argmax(r)
        i = int(sel[t])
        best = r[i_or]
        assert r[i] >= best - tol * abs(best), (t, i, i_or, r[i], best)
        if i != i_or:
            # only a near-tie may resolve differently, and never in FP64
            assert fp32, ("selection", t, i, i_or)
        assert abs(res["score_max"][t] - r[i]) <= tol * abs(r[i]), t
        st.step(i)
        # the block state is FP64 in both modes
        assert abs(res["nu"][t + 1] - st.nu) <= TOL * abs(st.nu), (t, res["nu"][t + 1], st.nu)
    assert res["nu"][0] == pytest.approx(np.sqrt(p.d * p.c), rel=1e-15)
    if nr < b:
        g1 = rs.scores().cpu().numpy()
        r1 = st.scores()
        m = st.available
        assert np.all(np.isneginf(g1[~m]))
        assert relerr(g1[m], r1[m]) <= tol
    crit = rs.criterion()
    assert crit == pytest.approx(st.criterion(), rel=1e-8, abs=1e-12)
    rs.close()
    ctx.close()
    return sel


SMALL = [
    # (n, n_lab, d, c, seed)
    (300, 5, 7, 3, 11),       # odd d
    (500, 10, 20, 5, 12),     # configuration-1 shape
    (1000, 0, 16, 4, 13),     # no labeled rows
    (700, 10, 33, 6, 14),     # ragged: three column tiles of 16, odd d
    (257, 4, 64, 2, 15),      # c = 2, one full column tile, ragged row tail
    (200, 3, 1, 3, 16),       # d = 1
]


@pytest.mark.parametrize("shape", SMALL)
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_round_small_matches_oracle(shape, prec):
    n, nl, d, c, seed = shape
    p = make_small(n=n, n_lab=nl, d=d, c=c, s=1, seed=seed)
    check_run(p, prec, b=12, eta=10.0)


@pytest.mark.parametrize("eta", [0.5, 300.0])
def test_round_eta_extremes(eta):
    p = make_small(n=400, n_lab=6, d=12, c=4, s=1, seed=21)
    check_run(p, "f32", b=10, eta=eta)


def test_round_selects_whole_pool():
    p = make_small(n=40, n_lab=3, d=5, c=3, s=1, seed=22)
    sel = check_run(p, "f64", b=40, eta=5.0)
    assert sorted(sel.tolist()) == list(range(40))


def test_round_configuration_2_full_size():
    p = make_problem(2)
    check_run(p, "f32", b=100, eta=50.0, rounds=4)


@pytest.mark.parametrize("shape", [SMALL[1], SMALL[3], SMALL[5]])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_round_fp32_decision_matches_oracle(shape, prec):
    n, nl, d, c, seed = shape
    p = make_small(n=n, n_lab=nl, d=d, c=c, s=1, seed=seed)
    check_run(p, prec, b=12, eta=10.0, fp32=True)


def test_round_fp32_decision_configuration_2_full_size():
    p = make_problem(2)
    check_run(p, "f32", b=100, eta=50.0, rounds=4, fp32=True)


def test_round_reduced_configuration_3_shape():
    p = make_problem(3, n=6000, n_lab=100)
    check_run(p, "f32", b=1000, eta=50.0, rounds=2)


def test_round_wide_features():
    # d = 600: the global-memory tridiagonalisation, factor and inverse of D (d > 256), ten
    # column tiles per class
    p = make_small(n=1500, n_lab=10, d=600, c=3, s=1, seed=25)
    check_run(p, "f32", b=20, eta=30.0, rounds=3)


def test_round_eta_sweep_matches_oracle():
    p = make_small(n=300, n_lab=5, d=10, c=4, s=1, seed=23)
    ctx, z, zn, Xo, Ho = setup(p, "f64", 8)
    etas = [1.0, 10.0, 100.0]
    got = round_eta_sweep(ctx, z, 1e-3, etas, 8)
    want = orr.eta_sweep(Xo, Ho, p.n_pool, zn, 1e-3, etas, 8)
    np.testing.assert_allclose(got["criterion"], want["criterion"], rtol=1e-8)
    assert got["best"] == want["best"]
    ctx.close()


def test_round_argument_errors():
    p = make_small(n=50, n_lab=2, d=4, c=3, s=1, seed=24)
    ctx, z, zn, Xo, Ho = setup(p, "f32", 5)
    with pytest.raises(FiralError):
        RoundSolver(ctx, z, 1e-3, 0.0, 5)          # eta must be positive
    with pytest.raises(FiralError):
        RoundSolver(ctx, z, 1e-3, 1.0, 51)         # b above n_pool
    rs = RoundSolver(ctx, z, 1e-3, 1.0, 5)
    rs.step(5)
    with pytest.raises(FiralError):
        rs.step(1)                                  # no rounds left
    rs.close()
    ctx.close()
