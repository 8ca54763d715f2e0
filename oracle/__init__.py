"""FP64 CPU oracle for the Approx-FIRAL Relax and Round steps (Chen, Wen & Biros, SC24).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package: only the tests, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the
HIP library (no kernels, headers, helpers or tables); it takes its inputs from
``synthdata`` like the GPU path does, and derives the Rademacher probes from
the published SplitMix64 definition on its own.

Modules
-------
``relax``  the matrix-free method in the paper's order: Lemma 1 Hessian
           products, the eq. 12 block-diagonal preconditioner, block-Jacobi
           PCG, the eq. 11 Hutchinson gradient and the entropic
           mirror-descent update of Algorithm 2.
``round``  the diagonal Round step of Algorithm 3: the per-point objective of
           the Section 3.2 proposition, the (H)_k update, the eigenvalues of
           Sigma^-1/2 (H)_k Sigma^-1/2, nu by bisection and the next
           B^-1 blocks, plus the eta sweep of the experiments section.
``dense``  brute force for tiny problems: H_i = Gamma_i (x) x_i x_i^T formed
           with ``np.kron`` (eq. 2), Sigma_z = H_o + H_z + lam*I (eq. 3, 7),
           the objective Tr(Sigma_z^-1 H_p) (eq. 4-5) and its exact gradient
           (eq. 6); and Algorithm 1's Round step on dense dc x dc matrices
           with block-diagonal Fisher matrices (the pin of ``round``).

Parity status: every function of ``relax`` is pinned by the tests in
``tests/test_oracle_*.py`` against ``dense`` (which is itself pinned by
finite differences and closed forms) or against published values; see the
module docstrings for the pin of each function.
"""
