"""Adaptive gap-based partitioning: the interval loop of Algorithm "main"
(Section 3.2), in FP64 on the CPU.

TEST INFRASTRUCTURE ONLY (see the package header).

While directions s..k remain, for the deflated matrix A_{-(s-1)} = P A P with
P = I - U U^T (U the directions found so far, Section 3.1):

1. Algorithm "musco" on A_{-(s-1)} with a block of p - (s-1) columns (the same
   estimate phase as the q = k branch) gives estimates theta_s, theta_{s+1}, ...
2. Algorithm "largeDetect": if some q in {s..k-1} has
   theta_{q+1} <= theta_q (1 - p^-2), the interval s..q is found by plain
   subspace iteration (Algorithm "subspace iteration") on A_{-(s-1)} with
   q - s + 1 columns and no oversampling.
3. Otherwise Algorithm "shiftTune" places lambda for the deflated problem, the
   Ritz values nu_i of its last round estimate (lambda - lambda_i)^{-1}, and
   Algorithm "deltaDetect" returns the smallest q with
   nu_{q+1}^{-1} - nu_q^{-1} >= 5 Delta / 9, else q = k.  The interval is
   found by shift-and-invert subspace iteration on
   D_{-(s-1)} = P (lambda I - A)^{-1} P (eq. deflatedShift) with p' columns:
   p' = p - (s-1) when q = k (oversampling), else q - s + 1.
4. s = q + 1.

The found blocks form a d x p' orthonormal basis on which Algorithm "second
stage" (Rayleigh-Ritz with XX^T) gives U_k, as in the last step of Algorithm
"main".

Readings (the paper leaves them open):
  * "any q" of largeDetect: the largest such q (fewest intervals);
  * the estimates of Algorithm "musco" on D_{-(s-1)} are the Ritz values of the
    last shiftTune round (the same p - (s-1) block and the same solves);
  * the gap budget Delta_hat = (theta_k - theta_p) / 1.5 and the stopping
    threshold eps / (k mu_F) come from the first interval's estimates and hold
    for every interval; every iteration (plain or shift-and-invert) stops when
    the subspace it targets moves by at most that threshold;
  * the inner solver samples columns of the deflated matrix with the weights of
    the undeflated columns (pi_i ~ ||x_i||^2): still unbiased, and the sampling
    table stays that of X;
  * random streams: the estimate block of interval t uses stream (tag 1, t),
    the plain-iteration start (tag 4, t); shift-and-invert starts and inner
    solves use a solve counter that runs across intervals.
"""
from dataclasses import dataclass, field
import math

import numpy as np

from .philox import gaussian_block, TAG_EST_INIT, TAG_SI_INIT
from .sampling import column_sq_norms, build_table
from .linalg import cholqr2, eigh_desc, sign_fix
from .lowrank import (LR_OK, LR_ENOCONV, LR_ENOGAP, LR_EINVAL, LowRankError, Options, Schedule,
                      decode, deflate, apply_A, solver_constants, svrg_solve, tune_shift,
                      final_rr, validate, stop_scale, inner_schedule, inner_solve)

TAG_POWER_INIT = 4


def large_detect(theta_I, p):
    """Algorithm largeDetect on the estimates of I = {s..k} (theta_I[0] is
    theta_s): the largest local q < |I| - 1 with
    theta_I[q+1] <= theta_I[q] (1 - p^-2), else -1."""
    J = [q for q in range(len(theta_I) - 1) if theta_I[q + 1] <= theta_I[q] * (1.0 - p ** -2)]
    return max(J) if J else -1


def delta_detect(inv_I, delta):
    """Algorithm deltaDetect on the estimates of (lambda - lambda_i) for i in I
    (inv_I[0] for i = s): the smallest local q < |I| - 1 with
    inv_I[q+1] - inv_I[q] >= 5 delta / 9, else |I| - 1 (that is, q = k)."""
    J = [q for q in range(len(inv_I) - 1) if inv_I[q + 1] - inv_I[q] >= 5.0 * delta / 9.0]
    return min(J) if J else len(inv_I) - 1


def estimate_deflated(X, Ud, cols, seed, interval, iters):
    """Algorithm musco on A_{-(s-1)}: `iters` plain steps with `cols` columns,
    then Rayleigh-Ritz.  Returns (S, theta, residual norms)."""
    d = X.shape[0]
    S = cholqr2(deflate(Ud, gaussian_block(seed, TAG_EST_INIT, interval, d, cols)))[0]
    for _ in range(iters):
        S = cholqr2(apply_A(X, S, Ud))[0]
    Y = apply_A(X, S, Ud)
    theta, Q = eigh_desc(S.T @ Y)
    R = Y @ Q - (S @ Q) * theta[None, :]
    return S, theta, np.linalg.norm(R, axis=0)


def _change(V_prev, V):
    sv = np.linalg.svd(V_prev.T @ V, compute_uv=False)
    return math.sqrt(max(0.0, 1.0 - float(sv[-1]) ** 2))


def power_deflated(X, Ud, cols, seed, interval, eps_stop, max_outer):
    """Plain subspace iteration on A_{-(s-1)} with `cols` columns; stops when
    the block's span moves by at most eps_stop.  Returns (S, iterations,
    changes, converged)."""
    d = X.shape[0]
    S = cholqr2(deflate(Ud, gaussian_block(seed, TAG_POWER_INIT, interval, d, cols)))[0]
    changes = []
    for it in range(max_outer):
        S_new = cholqr2(apply_A(X, S, Ud))[0]
        ch = _change(S, S_new)
        changes.append(ch)
        S = S_new
        if ch <= eps_stop:
            return S, it + 1, changes, True
    return S, max_outer, changes, False


def si_deflated(X, qc, Ud, sched, target, cols, seed, max_outer, max_epochs):
    """Shift-and-invert subspace iteration on D_{-(s-1)} with `cols` columns;
    stops when the top-`target` Ritz subspace moves by at most sched.eps_stop.
    Returns (S, epochs per solve, changes, converged)."""
    d = X.shape[0]
    S = cholqr2(deflate(Ud, gaussian_block(seed, TAG_SI_INIT, sched.first_solve, d, cols)))[0]
    epochs, changes = [], []
    V_prev = None
    for ell in range(max_outer):
        W, e, _ = inner_solve(X, qc, S, sched, sched.tau, seed, sched.first_solve + ell,
                              max_epochs, Ud=Ud)
        epochs.append(e)
        K = S.T @ W
        _, Q = eigh_desc(0.5 * (K + K.T))
        V = S @ Q[:, :target]
        S = cholqr2(W)[0]
        if V_prev is not None:
            ch = _change(V_prev, V)
            changes.append(ch)
            if ch <= sched.eps_stop:
                return S, epochs, changes, True
        V_prev = V
    return S, epochs, changes, False


@dataclass
class Interval:
    s: int                 # first direction (1-based)
    q: int                 # last direction (1-based)
    branch: str            # "power" or "shift-invert"
    cols: int              # block width
    iterations: int        # plain iterations, or outer shift-and-invert iterations
    theta_est: np.ndarray = None
    lam: float = 0.0
    shift_rounds: int = 0
    epochs: list = field(default_factory=list)
    b: int = 0
    m: int = 0
    eta: float = 0.0


@dataclass
class AdaptiveResult:
    status: int
    U: np.ndarray
    theta: np.ndarray
    intervals: list
    delta_hat: float
    eps_stop: float
    solves: int


def solve_adaptive(xt, storage, k, p, eps, opt=None):
    """Algorithm main with adaptive partitioning (see the module docstring)."""
    opt = opt or Options()
    X = decode(xt, storage)
    d, n = X.shape
    validate(d, n, k, p)
    w = column_sq_norms(X)
    if not np.all(np.isfinite(w)):
        raise LowRankError(LR_EINVAL, "non-finite entries in X")
    _, qc = build_table(w)
    fro2 = float(np.sum(w))
    Ud = np.zeros((d, 0))
    s, t, solve_ctr = 0, 0, 0
    delta = eps_stop = tau = None
    intervals = []
    converged = True
    while s < k:
        kk, pc = k - s, p - s
        S_est, theta, res = estimate_deflated(X, Ud, pc, opt.seed, t, opt.est_iters)
        if t == 0:
            delta = (theta[k - 1] - theta[p - 1]) / 1.5
            if not delta > 1e-12 * theta[0]:
                raise LowRankError(LR_ENOGAP, "no gap between theta_k and theta_p")
            eps_stop = eps / (k * stop_scale(theta, fro2, k, opt.norm))
            tau = min(1e-2, 0.1 * eps_stop)
        q = large_detect(theta[:kk], p)
        if q >= 0:
            B, its, _, ok = power_deflated(X, Ud, q + 1, opt.seed, t, eps_stop, opt.max_outer)
            iv = Interval(s=s + 1, q=s + q + 1, branch="power", cols=q + 1, iterations=its,
                          theta_est=theta[:kk].copy())
        else:
            out = {}
            lam, mu, rounds, _ = tune_shift(X, qc, S_est, theta, res, delta, fro2, opt.seed,
                                            opt, n, Ud=Ud, solve0=solve_ctr, out=out)
            solve_ctr += rounds
            q = delta_detect(1.0 / out["nu"][:kk], delta)
            cols = pc if q == kk - 1 else q + 1
            sched = inner_schedule(fro2, theta[0], lam, mu, n, opt)
            sched.delta_hat, sched.tau, sched.eps_stop = delta, tau, eps_stop
            sched.first_solve = solve_ctr
            b, eta, m = sched.b, sched.eta, sched.m
            B, epochs, _, ok = si_deflated(X, qc, Ud, sched, q + 1, cols, opt.seed,
                                           opt.max_outer, opt.max_epochs)
            solve_ctr += len(epochs)
            if q < kk - 1:     # keep the interval's own directions: top Ritz vectors of A_{-(s-1)}
                Hm = B.T @ apply_A(X, B, Ud)
                _, Q = eigh_desc(0.5 * (Hm + Hm.T))
                B = B @ Q[:, :q + 1]
            iv = Interval(s=s + 1, q=s + q + 1, branch="shift-invert", cols=cols,
                          iterations=len(epochs), theta_est=theta[:kk].copy(), lam=lam,
                          shift_rounds=rounds, epochs=epochs, b=b, m=m, eta=eta)
        converged = converged and ok
        intervals.append(iv)
        Ud = np.hstack([Ud, cholqr2(deflate(Ud, B))[0]])
        s += q + 1
        t += 1
    U, th = final_rr(X, Ud, k, opt.polish)
    return AdaptiveResult(status=LR_OK if converged else LR_ENOCONV, U=U, theta=th,
                          intervals=intervals, delta_hat=delta, eps_stop=eps_stop,
                          solves=solve_ctr)
