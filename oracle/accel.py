"""Accelerated inner solver: an accelerated proximal-point loop around the
minibatch SVRG epochs, for (lambda I - A) W = S.

TEST INFRASTRUCTURE ONLY (see the package header).

The paper uses an accelerated variant of its stochastic solver for the
n^{3/4} regime of Theorem "mainResult" and of Theorem "svrgSolve" (AccSVRG,
cited, not spelled out).  The reading implemented here is the standard
acceleration of a linearly convergent solver by an outer proximal-point loop:

  kappa = max(0, sqrt(8 ||X||_F^2 theta_1 / n) - mu)   (the inner solver's
          epoch of m = 8 sigma_b^2 / (mu + kappa)^2 steps then samples about
          n columns, the work of one pass)
  q = mu / (mu + kappa),  beta = (1 - sqrt(q)) / (1 + sqrt(q))
  W_0 = S (lambda I - S^T A S)^{-1} (the same warm start), Y_0 = W_0
  repeat:  one SVRG epoch on ((lambda + kappa) I - A) W = S + kappa Y_{k-1},
           started at W_{k-1}  ->  W_k
           residual of the original system:
             S - (lambda I - A) W_k = kappa (W_k - Y_{k-1}) - G_k
           with G_k the epoch's closing full gradient
           stop when its norm <= tau ||S||
           Y_k = W_k + beta (W_k - W_{k-1})
The next epoch's starting gradient follows from the last one without a pass:
G <- G - kappa (Y_k - Y_{k-1}).  Epoch e of the solve uses sample stream
(solve, epoch e), as the plain solver does.

Budget: an outer step gains a factor of about 1 - sqrt(q) where a plain epoch
gains a constant factor, so the solve may take max_epochs * ceil(1 / sqrt(q))
outer steps, 1 / sqrt(q) = (1 + beta) / (1 - beta).
"""
import math

import numpy as np

from .lowrank import (LR_ENOCONV, LR_ESHIFT, LowRankError, apply_A, deflate, solver_constants,
                      svrg_step)
from .sampling import step_indices


def accel_constants(fro2, theta1, lam, mu_hat, n, batch=0, eta_scale=1.0):
    """(kappa, beta, b, eta, m) of the accelerated solver; b, eta and m are
    the plain solver's constants for the shift lambda + kappa."""
    kappa = max(0.0, math.sqrt(8.0 * fro2 * theta1 / n) - mu_hat)
    q = mu_hat / (mu_hat + kappa)
    beta = (1.0 - math.sqrt(q)) / (1.0 + math.sqrt(q))
    b, eta, m = solver_constants(fro2, theta1, lam + kappa, mu_hat + kappa, n, batch, eta_scale)
    return kappa, beta, b, eta, m


def acc_svrg_solve(X, qc, S, lam, kappa, beta, eta, m, b, tau, seed, solve, max_epochs,
                   fixed_epochs=None, Ud=None):
    """Approximately solve (lam I - XX^T) W = S.  Returns (W, epochs, residual
    norms of the original system after the warm start and after each epoch)."""
    Y0 = apply_A(X, S, Ud)
    H = S.T @ Y0
    H = 0.5 * (H + H.T)
    p = S.shape[1]
    Mi = np.linalg.inv(lam * np.eye(p) - H)
    W = S @ Mi
    G0 = (lam * S - Y0) @ Mi - S                    # gradient of the original system at W
    sn = np.linalg.norm(S)
    res = [np.linalg.norm(G0)]
    lam2 = lam + kappa
    Yk = W.copy()
    Wprev = W.copy()
    G = G0 + kappa * W - kappa * Yk                  # inner gradient at W for S + kappa Y_0
    budget = max_epochs * math.ceil((1.0 + beta) / (1.0 - beta))
    e = 0
    while True:
        if fixed_epochs is None:
            if res[-1] <= tau * sn:
                break
            if e >= budget:
                raise LowRankError(LR_ENOCONV, "inner solver did not converge")
        elif e >= fixed_epochs:
            break
        Wt = Wprev
        Wc = Wt.copy()
        for t in range(m):
            idx, sc = step_indices(seed, solve, e, t, b, qc)
            Wc = svrg_step(X, Wc, Wt, G, lam2, eta, idx, sc, Ud)
        Wk = Wc
        G = lam2 * Wk - apply_A(X, Wk, Ud) - (S + kappa * Yk)
        r = np.linalg.norm(kappa * (Wk - Yk) - G)
        e += 1
        res.append(r)
        if not np.isfinite(r) or r > 1e3 * res[0]:
            raise LowRankError(LR_ESHIFT, "inner solver diverged: shift not above lambda_1")
        Ynew = Wk + beta * (Wk - Wprev)
        G = G - kappa * (Ynew - Yk)
        Yk, Wprev = Ynew, Wk
    return Wprev, e, res
