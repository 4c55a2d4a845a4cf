"""Plain FP64 CPU implementation of the shift-and-invert block power iteration
with oversampling, with every inverse application done by a minibatch SVRG
solver (the q = k branch of Algorithm "main", Section 3.2).

Steps, in the paper's order:

1. Estimate phase -- Algorithm "musco" (Section 2.4) run on C = A = XX^T with
   a block of p columns: subspace iteration (Algorithm "subspace iteration",
   Section 2.2.1) followed by Rayleigh-Ritz (Algorithm "second stage",
   Section 2.2.2).  Gives Ritz values theta_1 >= ... >= theta_p of A and their
   residual norms.
2. Gap budget -- Section 3 assumes Delta <= lambda_k - lambda_{p+1} <= 2 Delta
   and says it can be found cheaply without giving a procedure; the reading
   here is Delta_hat = (theta_k - theta_p) / 1.5.
3. Shift -- Algorithm "shiftTune" (Appendix B) with the target interval of
   eq. (shiftClose): estimate lambda - lambda_1 by 1/nu_1, nu_1 the top Ritz
   value of (lambda I - A)^{-1} on the estimate-phase block; while it lies
   above Delta/5 lower lambda by (1 - 1/9)/2 times the estimate.
4. Shift-and-invert subspace iteration -- Algorithm "subspace iteration" with
   C = (lambda I - A)^{-1} and p' = p (Algorithm "main", q = k branch), each
   product C S computed by ``svrg_solve``; orthonormalisation by Cholesky-QR
   applied twice; stops when the top-k Ritz subspace moves by less than
   eps / (k mu_F) between iterations (Theorem "mainResultW": tan theta <= eps/k
   per interval, with the Frobenius rescaling of Corollary "mainResult").
5. Final Rayleigh-Ritz -- Algorithm "second stage" with C = XX^T on the last
   block, returning U_k = S U_hat_k and the top-k Ritz values (Algorithm
   "main", last step).

``svrg_solve`` is the stochastic solver of Theorem "svrgSolve" (Section 2.3):
SVRG on F(W) = 1/2 tr(W^T B W) - tr(W^T S), B = lambda I - XX^T, with the
unbiased minibatch estimate lambda I - (1/b) sum_j x_j x_j^T / pi_j.

This module is test infrastructure: a slow, obviously correct reference that
the GPU library is checked against.  It shares no code with the library.
"""
from dataclasses import dataclass, field
import math

import numpy as np

from .philox import gaussian_block, TAG_EST_INIT, TAG_SI_INIT
from .sampling import column_sq_norms, build_table, step_indices
from .linalg import cholqr2, eigh_desc, sign_fix, NotSPD

LR_OK, LR_EINVAL, LR_ENOMEM, LR_ENOGAP, LR_ENOCONV, LR_ESHIFT, LR_ENOTSPD = 0, 1, 2, 3, 4, 5, 6


class LowRankError(Exception):
    def __init__(self, code, msg):
        super().__init__(msg)
        self.code = code


@dataclass
class Options:
    seed: int = 0
    shift_mode: str = "fast"        # "fast": theta_1 + ||r_1|| + Delta/10 ; "literal": 1.5 theta_1
    shift_start: float = 0.0        # > 0: shift tuning starts from this lambda instead
    est_iters: int = 4
    max_outer: int = 2000
    max_epochs: int = 60
    max_shift_rounds: int = 30
    polish: int = 0
    batch: int = 0                  # 0 = automatic
    eta_scale: float = 1.0
    tau_shift: float = 1e-2
    norm: str = "fro"               # "fro" or "spectral": the norm of the (1 + eps) guarantee
    accel: bool = False             # accelerated inner solver (oracle.accel)


@dataclass
class Schedule:
    lam: float = 0.0
    mu_hat: float = 0.0
    delta_hat: float = 0.0
    eta: float = 0.0
    m: int = 0
    b: int = 0
    tau: float = 0.0
    eps_stop: float = 0.0
    first_solve: int = 0
    outer: int = 0
    epochs: list = field(default_factory=list)
    accel: bool = False
    kappa: float = 0.0
    beta: float = 0.0


def decode(xt, storage):
    """X (d x n, float64) from its stored form.

    Dense storage ("f64", "f32", "bf16"): xt is the column-major array (n x d).
    Compressed-column storage ("csc-f64", "csc-f32", "csc-bf16"): xt is a dict
    with d, n, col_ptr, row_idx, values; X becomes a scipy.sparse CSC matrix
    whose stored values are upcast exactly.  The paper allows sparse X with the
    per-pass cost nnz(X) in place of dn (Section 1 footnote; Theorem
    "svrgSolve").  Row indices must be sorted within each column, so that the
    stored order of a column is its row order."""
    if storage.startswith("csc-"):
        import scipy.sparse as sps
        vals = np.asarray(xt["values"])
        if storage == "csc-bf16":
            vals = (vals.astype(np.uint32) << np.uint32(16)).view(np.float32)
        cp = np.asarray(xt["col_ptr"], dtype=np.int64)
        ri = np.asarray(xt["row_idx"], dtype=np.int64)
        X = sps.csc_matrix((vals.astype(np.float64), ri, cp), shape=(xt["d"], xt["n"]))
        if not X.has_sorted_indices:
            raise LowRankError(LR_EINVAL, "row indices must be sorted within each column")
        return X
    if storage == "bf16":
        bits = np.asarray(xt, dtype=np.uint16).astype(np.uint32) << np.uint32(16)
        return bits.view(np.float32).astype(np.float64).T
    return np.asarray(xt).astype(np.float64).T


def deflate(Ud, W):
    """(I - Ud Ud^T) W: the projection that removes the directions already
    found (Section 3.1, the deflated matrices A_{-(s-1)} and D_{-(s-1)})."""
    if Ud is None or Ud.shape[1] == 0:
        return W
    return W - Ud @ (Ud.T @ W)


def apply_A(X, W, Ud=None):
    """A W = X (X^T W); A = XX^T is never formed (Section 2.2.1 footnote).
    With a deflation basis Ud: the deflated A_{-(s-1)} = P A P, P = I - Ud Ud^T."""
    if Ud is None:
        return X @ (X.T @ W)
    return deflate(Ud, X @ (X.T @ deflate(Ud, W)))


def estimate_phase(X, k, p, seed, est_iters):
    d = X.shape[0]
    S = cholqr2(gaussian_block(seed, TAG_EST_INIT, 0, d, p))[0]
    for _ in range(est_iters):
        S = cholqr2(apply_A(X, S))[0]
    Y = apply_A(X, S)
    theta, Q = eigh_desc(S.T @ Y)
    R = Y @ Q - (S @ Q) * theta[None, :]
    return S, theta, np.linalg.norm(R, axis=0)


def solver_constants(fro2, theta1, lam, mu_hat, n, batch=0, eta_scale=1.0):
    """Minibatch size b, step size eta and epoch length m of the inner solver.

    The per-sample variance of the importance-sampled estimate is bounded by
    ||X||_F^2 lambda_1 ||Delta||^2, so sigma_b^2 = ||X||_F^2 theta_1 / b;
    eta = min(1/lambda, mu/(4 sigma_b^2)), m = ceil(2 / (eta mu)) with mu the
    estimate of lambda - lambda_1 (the strong convexity of B)."""
    if batch:
        b = int(batch)
    else:
        bstar = 4.0 * fro2 * theta1 / (lam * mu_hat)
        b = 1 << max(0, math.ceil(math.log2(max(bstar, 1.0))))
        b = min(max(b, 256), 8192)
    b = min(b, n)
    sig2 = fro2 * theta1 / b
    eta = eta_scale * min(1.0 / lam, mu_hat / (4.0 * sig2))
    m = int(math.ceil(2.0 / (eta * mu_hat)))
    return b, eta, m


def svrg_step(X, W, Wt, G, lam, eta, idx, scale, Ud=None):
    """One minibatch step: with Delta = W - W~ and the sampled columns X_B,
    W <- W - eta (G~ + lam Delta - X_B diag(scale) X_B^T Delta), where
    G~ = lam W~ - XX^T W~ - S is the full gradient at the epoch's anchor W~ and
    scale_j = 1 / (b pi_j).  Deflated (Ud given): the sampled columns are those
    of P X, P = I - Ud Ud^T; Delta stays in the range of P, so only the product
    X_B C is projected."""
    Xb = X[:, idx]
    Dl = W - Wt
    C = (Xb.T @ Dl) * scale[:, None]
    return W - eta * (G + lam * Dl - deflate(Ud, Xb @ C))


def svrg_solve(X, qc, S, lam, eta, m, b, tau, seed, solve, max_epochs,
               fixed_epochs=None, Ud=None):
    """Approximately solve (lam I - XX^T) W = S.  Returns (W, epochs, residual
    norms per epoch).  Warm start W0 = S (lam I - S^T A S)^{-1}, whose gradient
    (lam S - AS) M - S needs no extra pass."""
    Y = apply_A(X, S, Ud)
    H = S.T @ Y
    H = 0.5 * (H + H.T)
    p = S.shape[1]
    Mi = np.linalg.inv(lam * np.eye(p) - H)
    Wt = S @ Mi
    G = (lam * S - Y) @ Mi - S
    W = Wt.copy()
    sn = np.linalg.norm(S)
    res = [np.linalg.norm(G)]
    e = 0
    while True:
        if fixed_epochs is None:
            if res[-1] <= tau * sn:
                break
            if e >= max_epochs:
                raise LowRankError(LR_ENOCONV, "inner solver did not converge")
        elif e >= fixed_epochs:
            break
        for t in range(m):
            idx, sc = step_indices(seed, solve, e, t, b, qc)
            W = svrg_step(X, W, Wt, G, lam, eta, idx, sc, Ud)
        Wt = W
        G = lam * Wt - apply_A(X, Wt, Ud) - S
        e += 1
        res.append(np.linalg.norm(G))
        if not np.isfinite(res[-1]) or res[-1] > 1e3 * res[0]:
            raise LowRankError(LR_ESHIFT, "inner solver diverged: shift not above lambda_1")
    return Wt, e, res


def inner_schedule(fro2, theta1, lam, mu, n, opt):
    """The inner solver's constants for shift lam and strong-convexity
    estimate mu: plain SVRG (solver_constants) or, with opt.accel, the
    accelerated loop (oracle.accel)."""
    if opt.accel:
        from .accel import accel_constants
        kappa, beta, b, eta, m = accel_constants(fro2, theta1, lam, mu, n, opt.batch,
                                                 opt.eta_scale)
        return Schedule(lam=lam, mu_hat=mu, eta=eta, m=m, b=b, accel=True, kappa=kappa,
                        beta=beta)
    b, eta, m = solver_constants(fro2, theta1, lam, mu, n, opt.batch, opt.eta_scale)
    return Schedule(lam=lam, mu_hat=mu, eta=eta, m=m, b=b)


def inner_solve(X, qc, S, sched, tau, seed, solve, max_epochs, fixed_epochs=None, Ud=None):
    """(lam I - A) W = S by the solver the schedule names."""
    if sched.accel:
        from .accel import acc_svrg_solve
        return acc_svrg_solve(X, qc, S, sched.lam, sched.kappa, sched.beta, sched.eta, sched.m,
                              sched.b, tau, seed, solve, max_epochs, fixed_epochs, Ud)
    return svrg_solve(X, qc, S, sched.lam, sched.eta, sched.m, sched.b, tau, seed, solve,
                      max_epochs, fixed_epochs, Ud)


def tune_shift(X, qc, S_est, theta, res, delta, fro2, seed, opt, n, Ud=None, solve0=0,
               out=None):
    """Alg. shiftTune on the estimate-phase block.  Returns (lam, mu_hat,
    rounds, history).  Ud: deflation basis; solve0: solve index of the first
    round; out (dict): receives "nu", the Ritz values of the last round."""
    t1, r1 = theta[0], res[0]
    if opt.shift_start > 0:
        lam = opt.shift_start
        mu = max(lam - t1 - r1, delta / 30.0)
    elif opt.shift_mode == "literal":
        lam = 1.5 * t1
        mu = max(lam - t1 - r1, delta / 30.0)
    else:
        lam = t1 + r1 + delta / 10.0
        mu = delta / 10.0
    hist = []
    for r in range(opt.max_shift_rounds):
        sched = inner_schedule(fro2, t1, lam, mu, n, opt)
        W, _, _ = inner_solve(X, qc, S_est, sched, opt.tau_shift, seed, solve0 + r,
                              opt.max_epochs, Ud=Ud)
        K = S_est.T @ W
        nu = eigh_desc(0.5 * (K + K.T))[0]
        if out is not None:
            out["nu"] = nu
        nu1 = nu[0]
        if not nu1 > 0:
            raise LowRankError(LR_ESHIFT, "shift estimate not positive")
        g = 1.0 / nu1
        hist.append((lam, g))
        if delta / 27.0 <= g <= delta / 5.0:
            return lam, g, r + 1, hist
        if g > delta / 5.0:
            lam = lam - (4.0 / 9.0) * g
            mu = (5.0 / 9.0) * g
        else:
            lam = lam + delta / 10.0
            mu = g + delta / 10.0
    raise LowRankError(LR_ESHIFT, "shift tuning did not reach the target interval")


def si_iterate(X, qc, sched, k, p, seed, max_outer, max_epochs, replay=False, solver=None):
    """Shift-and-invert subspace iteration.  With ``replay`` the number of
    outer iterations and the epochs of each solve are taken from ``sched``.
    ``solver(S, solve_index, fixed_epochs) -> (W, epochs)`` replaces the SVRG
    solve (used by tests with an exact solve)."""
    d = X.shape[0]
    S = cholqr2(gaussian_block(seed, TAG_SI_INIT, sched.first_solve, d, p))[0]
    changes = []
    epochs = []
    V_prev = None
    L = sched.outer if replay else max_outer
    for ell in range(L):
        solve = sched.first_solve + ell
        fixed = sched.epochs[ell] if replay else None
        if solver is None:
            W, e, _ = inner_solve(X, qc, S, sched, sched.tau, seed, solve, max_epochs,
                                  fixed_epochs=fixed)
        else:
            W, e = solver(S, solve, fixed)
        epochs.append(e)
        K = S.T @ W
        _, Q = eigh_desc(0.5 * (K + K.T))
        V = S @ Q[:, :k]
        S = cholqr2(W)[0]
        if V_prev is not None:
            sv = np.linalg.svd(V_prev.T @ V, compute_uv=False)
            ch = math.sqrt(max(0.0, 1.0 - float(sv[-1]) ** 2))
            changes.append(ch)
            if not replay and ch <= sched.eps_stop:
                return S, epochs, changes, True
        V_prev = V
    return S, epochs, changes, replay


def final_rr(X, S, k, polish=0):
    for _ in range(polish):
        S = cholqr2(apply_A(X, S))[0]
    Z = X.T @ S
    theta, Q = eigh_desc(Z.T @ Z)
    return sign_fix(S @ Q[:, :k]), theta[:k]


@dataclass
class Result:
    status: int
    U: np.ndarray
    theta: np.ndarray
    schedule: Schedule
    theta_est: np.ndarray = None
    res_est: np.ndarray = None
    mu_F: float = 0.0
    fro2: float = 0.0
    shift_rounds: int = 0
    shift_history: list = None
    changes: list = None


def stop_scale(theta, fro2, k, norm="fro"):
    """The rough upper bound mu on ||X|| / ||X - X_k|| by which eps is rescaled
    (Corollary "mainResult"; Algorithm "main", first line), from the estimate
    phase: Frobenius ||X||_F / sqrt(||X||_F^2 - sum_{i<=k} theta_i), spectral
    sqrt(theta_1 / theta_{k+1})."""
    if norm == "spectral":
        return math.sqrt(theta[0] / max(theta[k], 1e-300))
    if norm != "fro":
        raise LowRankError(LR_EINVAL, "norm must be fro or spectral")
    tail = max(fro2 - float(np.sum(theta[:k])), 1e-300)
    return math.sqrt(fro2 / tail)


def validate(d, n, k, p):
    if not (1 <= k < p < d) or p > n:
        raise LowRankError(LR_EINVAL, "need 1 <= k < p < d and p <= n")


def solve(xt, storage, k, p, eps, opt=None, replay=None):
    """Full oracle run.  ``replay``: a Schedule whose lam, mu_hat, eta, m, b,
    first_solve, outer and epochs are used instead of the estimate, shift and
    stopping decisions.  A block that loses rank (Cholesky-QR meets a Gram
    matrix that is not positive definite, e.g. rank(X) < p, against the full
    column rank the QR step of Algorithm "subspace iteration" needs) is
    reported as LR_ENOTSPD."""
    try:
        return _solve(xt, storage, k, p, eps, opt, replay)
    except NotSPD as e:
        raise LowRankError(LR_ENOTSPD, "Cholesky-QR: Gram matrix not positive definite (%s)" % e)


def _solve(xt, storage, k, p, eps, opt=None, replay=None):
    opt = opt or Options()
    X = decode(xt, storage)
    d, n = X.shape
    validate(d, n, k, p)
    w = column_sq_norms(X)
    if not np.all(np.isfinite(w)):
        raise LowRankError(LR_EINVAL, "non-finite entries in X")
    _, qc = build_table(w)
    fro2 = float(np.sum(w))
    S_est, theta, res = estimate_phase(X, k, p, opt.seed, opt.est_iters)
    delta = (theta[k - 1] - theta[p - 1]) / 1.5
    if not delta > 1e-12 * theta[0]:
        raise LowRankError(LR_ENOGAP, "no gap between theta_k and theta_p")
    mu_F = stop_scale(theta, fro2, k, opt.norm)
    eps_stop = eps / (k * mu_F)
    tau = min(1e-2, 0.1 * eps_stop)
    if replay is None:
        lam, mu, rounds, hist = tune_shift(X, qc, S_est, theta, res, delta, fro2, opt.seed,
                                           opt, n)
        sched = inner_schedule(fro2, theta[0], lam, mu, n, opt)
        sched.delta_hat, sched.tau, sched.eps_stop, sched.first_solve = delta, tau, eps_stop, rounds
    else:
        rounds, hist = replay.first_solve, []
        sched = Schedule(lam=replay.lam, mu_hat=replay.mu_hat, delta_hat=delta,
                         eta=replay.eta, m=replay.m, b=replay.b, tau=tau, eps_stop=eps_stop,
                         first_solve=replay.first_solve, outer=replay.outer,
                         epochs=list(replay.epochs))
    S, epochs, changes, converged = si_iterate(X, qc, sched, k, p, opt.seed, opt.max_outer,
                                               opt.max_epochs, replay=replay is not None)
    sched.outer = len(epochs)
    sched.epochs = epochs
    U, th = final_rr(X, S, k, opt.polish)
    return Result(status=LR_OK if converged else LR_ENOCONV, U=U, theta=th, schedule=sched,
                  theta_est=theta, res_est=res, mu_F=mu_F, fro2=fro2, shift_rounds=rounds,
                  shift_history=hist, changes=changes)
