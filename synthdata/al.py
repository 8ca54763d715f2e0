"""A synthetic active-learning loop around a point-selection routine.

Labeled Gaussian-mixture data (one cluster per class), a pool and an
evaluation set; each round a multinomial logistic regression (scikit-learn)
is trained on the labeled points, its class probabilities on the pool and the
labeled rows become the inputs h_i of the selection routine (eq. 1: the
model's probabilities), and the routine's picks are labeled.  The routine is
passed in by the caller, so the same loop drives the GPU library and the CPU
oracle; this module holds none of the selection arithmetic.
"""
from __future__ import annotations

import numpy as np

from . import labeled_mixture


def al_loop(select, c: int, d: int, n_pool: int, n_eval: int, rounds: int, seed: int,
            mean_std: float = 0.5) -> dict:
    """Run `rounds` rounds of selection.

    select(X, H, n_unl, t) -> indices into the n_unl unlabeled rows: X and H are
    (n_unl + n_labeled) x d and x c float64, the unlabeled pool rows first, then the labeled
    rows (the row order of the Relax and Round calls); t is the 0-based round.  Starts from one
    labeled point per class.  Returns the evaluation accuracy after each round (rounds + 1
    values) and the pool indices picked in each round.
    """
    from sklearn.linear_model import LogisticRegression
    rng = np.random.default_rng(seed)
    X, y = labeled_mixture(rng, n_pool + n_eval, d, c, mean_std)
    Xp, yp, Xe, ye = X[:n_pool], y[:n_pool], X[n_pool:], y[n_pool:]
    labeled = np.array([rng.choice(np.flatnonzero(yp == k)) for k in range(c)])
    acc, picks = [], []
    for t in range(rounds + 1):
        clf = LogisticRegression(C=1.0, max_iter=2000).fit(Xp[labeled], yp[labeled])
        acc.append(float(clf.score(Xe, ye)))
        if t == rounds:
            break
        unl = np.setdiff1d(np.arange(n_pool), labeled)
        Xr = np.ascontiguousarray(np.concatenate([Xp[unl], Xp[labeled]]))
        Hr = np.ascontiguousarray(clf.predict_proba(Xr))
        sel = np.asarray(select(Xr, Hr, len(unl), t), dtype=np.int64)
        pick = unl[sel]
        picks.append(pick)
        labeled = np.concatenate([labeled, pick])
    return dict(accuracy=acc, picks=picks)
