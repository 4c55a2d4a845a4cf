"""Pins of the oracle's method against what the paper and the mathematics fix.

* Inner solver: one minibatch step that sees every column once with unit
  weight is exactly a gradient step on F(W) = 1/2 tr W^T B W - tr W^T S (so a
  dropped term or a wrong sign fails); averaged exactly over the sampling
  distribution the minibatch step is that gradient step (the importance
  weights make X_B diag(1/(b pi)) X_B^T unbiased for A); the solve converges
  to the direct solution of (lambda I - XX^T) W = S (Theorem "svrgSolve"); a
  shift below lambda_1 is detected.
* Subspace iteration with exact solves converges at the rate
  (lambda - lambda_k)/(lambda - lambda_{p+1}) (Theorem "zhang" applied to
  C = (lambda I - A)^{-1}).
* Estimate phase: Ritz values within the accuracy Algorithm "main" requests
  from Algorithm "musco" (1/(9p^2)), Theorem "musco".
* Shift tuning from the literal start 1.5 theta_1: terminates in
  O(log(lambda_1/Delta)) rounds with lambda - lambda_1 in [Delta/30, 2Delta/9]
  (Lemma "shiftTune", eq. shiftClose).
* End to end: the planted closed form (X = U Sigma V^T, so U_k is the answer),
  an SVD written out by hand (one-sided Jacobi), orthonormality, the
  (1 + eps) Frobenius bound of Theorem "mainResult" and Eckart-Young
  optimality of Pi* (Section 1).
"""
import math

import numpy as np
import pytest

import oracle
from oracle.lowrank import (LowRankError, LR_ESHIFT, LR_EINVAL, LR_ENOGAP, LR_ENOTSPD, Options,
                            Schedule,
                            svrg_step, svrg_solve, si_iterate, estimate_phase, tune_shift, solve,
                            decode)
from oracle.sampling import column_sq_norms, build_table
from oracle.linalg import cholqr2, jacobi_svd, sin_theta
import workloads


def planted(d, n, sigma, seed):
    rng = np.random.default_rng(seed)
    U = np.linalg.qr(rng.standard_normal((d, d)))[0]
    V = np.linalg.qr(rng.standard_normal((n, d)))[0]
    return (U * sigma) @ V.T, U


def test_svrg_step_full_batch_is_gradient_step():
    rng = np.random.default_rng(0)
    d, n, p = 12, 40, 3
    X = rng.standard_normal((d, n))
    S = rng.standard_normal((d, p))
    lam = 1.3 * np.linalg.norm(X, 2) ** 2
    B = lam * np.eye(d) - X @ X.T
    Wt = rng.standard_normal((d, p))
    W = Wt + 0.1 * rng.standard_normal((d, p))
    G = B @ Wt - S
    eta = 0.37 / lam
    got = svrg_step(X, W, Wt, G, lam, eta, np.arange(n), np.ones(n))
    want = W - eta * (B @ W - S)
    assert np.linalg.norm(got - want) < 1e-12 * np.linalg.norm(want)


@pytest.mark.parametrize("b", [1, 2])
def test_svrg_step_expectation_is_gradient_step(b):
    """Averaged exactly over the sampling distribution (every ordered b-tuple of
    i.i.d. draws from pi_i = q_i / Q of the quantised table, weights 1/(b pi_i)),
    the minibatch step equals the full gradient step W - eta (B W - S): the
    sampled X_B diag(1/(b pi)) X_B^T is an unbiased estimate of A = XX^T
    (Section 2.3).  A wrong weight, a missing 1/b or a dropped term fails."""
    import itertools
    rng = np.random.default_rng(3)
    d, n, p = 6, 9, 2
    X = rng.standard_normal((d, n)) * rng.uniform(0.3, 2.0, size=n)[None, :]
    X[:, 4] = 0.0   # a zero column: weight 0, never drawn
    S = rng.standard_normal((d, p))
    lam = 1.4 * np.linalg.norm(X, 2) ** 2
    B = lam * np.eye(d) - X @ X.T
    Wt = rng.standard_normal((d, p))
    W = Wt + 0.2 * rng.standard_normal((d, p))
    G = B @ Wt - S
    eta = 0.3 / lam
    q, qc = build_table(column_sq_norms(X))
    pi = q.astype(np.float64) / float(qc[n])
    cols = [i for i in range(n) if q[i] > 0]
    assert 4 not in cols
    mean = np.zeros_like(W)
    for tup in itertools.product(cols, repeat=b):
        idx = np.array(tup)
        prob = float(np.prod(pi[idx]))
        mean += prob * svrg_step(X, W, Wt, G, lam, eta, idx, 1.0 / (b * pi[idx]))
    want = W - eta * (B @ W - S)
    assert np.linalg.norm(mean - want) < 1e-12 * np.linalg.norm(want)


def test_svrg_solve_matches_direct_solve():
    sig = np.concatenate([[3.0, 2.5, 2.2], np.linspace(1.0, 0.1, 37)])
    X, _ = planted(40, 600, sig, 1)
    d = 40
    _, qc = build_table(column_sq_norms(X))
    fro2 = float(np.sum(sig ** 2))
    lam = sig[0] ** 2 + 0.5
    S = cholqr2(np.random.default_rng(2).standard_normal((d, 5)))[0]
    b, eta, m = oracle.solver_constants(fro2, sig[0] ** 2, lam, lam - sig[0] ** 2, 600)
    W, e, res = svrg_solve(X, qc, S, lam, eta, m, b, 1e-11, 77, 0, 200)
    Wd = np.linalg.solve(lam * np.eye(d) - X @ X.T, S)
    assert np.linalg.norm(W - Wd) / np.linalg.norm(Wd) < 1e-9
    # linear convergence: geometric-mean residual contraction per epoch
    rate = (res[-1] / res[0]) ** (1.0 / e)
    assert rate < 0.7


def test_svrg_detects_shift_below_lambda1():
    sig = np.concatenate([[3.0, 2.0], np.linspace(1.0, 0.1, 18)])
    X, _ = planted(20, 200, sig, 3)
    _, qc = build_table(column_sq_norms(X))
    S = cholqr2(np.random.default_rng(4).standard_normal((20, 3)))[0]
    lam = 0.9 * sig[0] ** 2
    with pytest.raises(LowRankError) as ei:
        svrg_solve(X, qc, S, lam, 0.5 / lam, 200, 64, 1e-10, 5, 0, 60)
    assert ei.value.code == LR_ESHIFT


def test_shift_and_invert_rate_with_exact_solves():
    d, n, k, p = 60, 300, 3, 6
    lam_i = np.concatenate([[10.0, 9.0, 8.5, 7.0, 6.8, 6.6, 6.0], np.linspace(3.0, 0.1, d - 7)])
    X, U = planted(d, n, np.sqrt(lam_i), 5)
    lam = 10.4
    B = lam * np.eye(d) - X @ X.T

    def exact(S, solve, fixed):
        return np.linalg.solve(B, S), 0

    sched = Schedule(lam=lam, first_solve=0, eps_stop=0.0, outer=14, epochs=[0] * 14)
    _, _, changes, _ = si_iterate(X, None, sched, k, p, 9, 14, 1, replay=True, solver=exact)
    rate = (lam - lam_i[k - 1]) / (lam - lam_i[p])
    ratios = np.array(changes[4:]) / np.array(changes[3:-1])
    assert abs(np.median(ratios) / rate - 1.0) < 0.1
    # plain power iteration on A would contract at lambda_{p+1}/lambda_k instead
    assert abs(lam_i[p] / lam_i[k - 1] - rate) > 0.2


def test_estimate_phase_meets_musco_accuracy():
    w = workloads.workload("planted-256x2048-f64")
    X = decode(w["Xt"], "f64")
    k, p = w["k"], w["p"]
    _, theta, res = estimate_phase(X, k, p, w["solver_seed"], 4)
    lam = w["sigma"][:k] ** 2
    eps1 = 1.0 / (9 * p * p)
    assert np.all(theta[:k] <= lam * (1 + 1e-13))
    assert np.all(theta[:k] >= (1 - eps1) * lam)
    assert res[0] < 1e-3


def test_shift_tuning_literal_start_lemma():
    w = workloads.workload("planted-256x2048-f64")
    X = decode(w["Xt"], "f64")
    k, p = w["k"], w["p"]
    opt = Options(seed=w["solver_seed"], shift_mode="literal")
    S_est, theta, res = estimate_phase(X, k, p, opt.seed, opt.est_iters)
    wn = column_sq_norms(X)
    _, qc = build_table(wn)
    delta = (theta[k - 1] - theta[p - 1]) / 1.5
    lam1 = w["sigma"][0] ** 2
    lamp1 = w["sigma"][p] ** 2
    assert delta <= lam1 - lamp1 <= 2 * delta   # the gap budget assumption of Section 3
    lam, mu, rounds, hist = tune_shift(X, qc, S_est, theta, res, delta, float(wn.sum()),
                                       opt.seed, opt, X.shape[1])
    assert delta / 30 <= lam - lam1 <= 2 * delta / 9
    assert rounds >= 2
    assert rounds <= 1 + math.ceil(math.log(2.78 * lam1 / delta, 4.0 / 3.0))
    # each update shrinks lambda - lambda_1 by a factor in [1/2, 3/4]
    gaps = [h[0] - lam1 for h in hist]
    for a, b in zip(gaps, gaps[1:]):
        assert 0.5 * a - 1e-12 <= b <= 0.75 * a + 1e-12


@pytest.fixture(scope="module")
def cfg1_result():
    w = workloads.workload("planted-256x2048-f64")
    r = solve(w["Xt"], w["storage"], w["k"], w["p"], w["eps"], Options(seed=w["solver_seed"]))
    return w, r


def test_end_to_end_planted_closed_form(cfg1_result):
    w, r = cfg1_result
    k = w["k"]
    X = decode(w["Xt"], "f64")
    assert r.status == 0
    assert np.linalg.norm(r.U.T @ r.U - np.eye(k)) < 1e-13
    assert sin_theta(w["U"][:, :k], r.U) < 1e-8
    np.testing.assert_allclose(r.theta, w["sigma"][:k] ** 2, rtol=1e-10)
    # Theorem mainResult, Frobenius norm: ||X - Pi X||_F <= (1 + eps) ||X - X_k||_F
    err = np.linalg.norm(X - r.U @ (r.U.T @ X))
    opt = math.sqrt(np.sum(w["sigma"][k:] ** 2))
    assert err <= (1 + w["eps"]) * opt
    # Eckart-Young: no rank-k projector does better than the optimum
    assert err >= opt * (1 - 1e-12)


def test_end_to_end_vs_handwritten_svd():
    d, n, k, p = 48, 400, 4, 8
    i = np.arange(1, d + 1, dtype=float)
    sig = np.where(i <= 4, 3.0 - 0.3 * i, 1.2 * i ** -0.6)
    X, _ = planted(d, n, sig, 12)
    # one-sided Jacobi on X^T = P diag(s) Q^T, so X = Q diag(s) P^T and the left
    # singular vectors of X are the columns of Q
    _, s, Q = jacobi_svd(X.T)
    np.testing.assert_allclose(s, sig, rtol=1e-12)
    r = solve(np.ascontiguousarray(X.T), "f64", k, p, 1e-8, Options(seed=4))
    assert sin_theta(Q[:, :k], r.U) < 1e-7
    np.testing.assert_allclose(r.theta, s[:k] ** 2, rtol=1e-10)


def test_replay_reproduces_auto_run(cfg1_result):
    w, r = cfg1_result
    s = r.schedule
    rep = Schedule(lam=s.lam, mu_hat=s.mu_hat, eta=s.eta, m=s.m, b=s.b,
                   first_solve=s.first_solve, outer=s.outer, epochs=list(s.epochs))
    r2 = solve(w["Xt"], w["storage"], w["k"], w["p"], w["eps"], Options(seed=w["solver_seed"]),
               replay=rep)
    assert np.array_equal(r2.U, r.U) and np.array_equal(r2.theta, r.theta)


def test_error_paths():
    rng = np.random.default_rng(0)
    xt = rng.standard_normal((100, 20))
    for k, p in [(3, 3), (0, 4), (3, 20), (5, 200)]:
        with pytest.raises(LowRankError) as ei:
            solve(xt, "f64", k, p, 1e-3, Options(seed=1))
        assert ei.value.code == LR_EINVAL
    bad = xt.copy()
    bad[7, 3] = np.nan
    with pytest.raises(LowRankError) as ei:
        solve(bad, "f64", 2, 4, 1e-3, Options(seed=1))
    assert ei.value.code == LR_EINVAL
    # a flat spectrum below the top direction: theta_k == theta_p, no gap budget
    sig = np.ones(20)
    sig[0] = 2.0
    X, _ = planted(20, 100, sig, 3)
    with pytest.raises(LowRankError) as ei:
        solve(np.ascontiguousarray(X.T), "f64", 2, 4, 1e-3, Options(seed=1))
    assert ei.value.code == LR_ENOGAP


def test_shift_tuning_from_below_the_interval():
    """A start inside (lambda_1, lambda_1 + Delta/27): the first estimate of
    lambda - lambda_1 lies below the interval of eq. (shiftClose), so lambda is
    raised by Delta/10 once and then lands in the interval (exact eigenvalue
    from the planted spectrum)."""
    w = workloads.workload("planted-256x2048-f64")
    X = decode(w["Xt"], "f64")
    k, p = w["k"], w["p"]
    S_est, theta, res = estimate_phase(X, k, p, w["solver_seed"], 4)
    wn = column_sq_norms(X)
    _, qc = build_table(wn)
    delta = (theta[k - 1] - theta[p - 1]) / 1.5
    lam1 = w["sigma"][0] ** 2
    opt = Options(seed=w["solver_seed"], shift_start=lam1 + delta / 50)
    lam, mu, rounds, hist = tune_shift(X, qc, S_est, theta, res, delta, float(wn.sum()),
                                       opt.seed, opt, X.shape[1])
    assert rounds == 2
    assert hist[0][1] < delta / 27
    assert abs(hist[0][1] - delta / 50) <= 0.05 * delta / 50
    assert hist[1][0] == hist[0][0] + delta / 10
    assert delta / 27 <= hist[1][1] <= delta / 5
    assert delta / 30 <= lam - lam1 <= 2 * delta / 9


def test_rank_deficient_block_is_reported():
    """rank(X) = 3 < p = 8: the estimate block loses rank and Cholesky-QR meets
    a Gram matrix that is not positive definite."""
    sig = np.zeros(64)
    sig[:3] = [3.0, 2.0, 1.0]
    X, _ = planted(64, 500, sig, 5)
    with pytest.raises(LowRankError) as ei:
        solve(np.ascontiguousarray(X.T), "f64", 2, 8, 1e-4, Options(seed=1))
    assert ei.value.code == LR_ENOTSPD
