"""Pins of the adaptive partitioning oracle (Algorithm "main" with
largeDetect / deltaDetect and deflation) against the rules as the paper states
them and against the exact SVD."""
import numpy as np
import pytest

import oracle
import workloads


def test_large_detect_rule():
    p = 10                                  # threshold ratio 1 - 1/100
    th = np.array([10.0, 9.95, 9.0, 8.99, 5.0])
    # consecutive ratios: 0.995 (no), 0.9045 (yes, q=1), 0.9989 (no), 0.556 (yes, q=3)
    assert oracle.large_detect(th, p) == 3          # the largest qualifying q
    assert oracle.large_detect(th[:3], p) == 1
    assert oracle.large_detect(np.array([1.0, 0.995, 0.991]), p) == -1
    assert oracle.large_detect(np.array([3.0]), p) == -1      # I = {k}: nothing to split
    # the boundary itself qualifies (<=)
    assert oracle.large_detect(np.array([1.0, 0.99]), p) == 0


def test_delta_detect_rule():
    delta = 0.9                              # 5 delta / 9 = 0.5
    inv = np.array([0.1, 0.2, 0.75, 0.8, 1.4])
    # consecutive differences 0.1, 0.55 (yes, q=1), 0.05, 0.6 (yes, q=3)
    assert oracle.delta_detect(inv, delta) == 1      # the smallest qualifying q
    assert oracle.delta_detect(np.array([0.1, 0.2, 0.3]), delta) == 2   # none: q = k
    assert oracle.delta_detect(np.array([0.5]), delta) == 0


def test_deflated_inner_solve_matches_direct_solve():
    """On the range of P = I - U U^T the deflated solver converges to the
    solution of (lambda I - P A P) W = S, checked against a dense solve."""
    rng = np.random.default_rng(4)
    d, n, p = 60, 400, 5
    sig = np.where(np.arange(1, d + 1) <= 3, 3.0, 1.0 / np.sqrt(np.arange(1, d + 1)))
    X = workloads.planted_dense(d, n, sig, 9, "f64")["Xt"].T
    u = np.linalg.svd(X, full_matrices=False)[0]
    Ud = u[:, :3]                            # deflate the three top directions
    P = np.eye(d) - Ud @ Ud.T
    A = X @ X.T
    lam = np.linalg.eigvalsh(P @ A @ P)[-1] * 1.3
    S = oracle.cholqr2(oracle.deflate(Ud, rng.standard_normal((d, p))))[0]
    _, qc = oracle.build_table(oracle.column_sq_norms(X))
    fro2 = float(np.sum(X * X))
    b, eta, m = oracle.solver_constants(fro2, lam / 1.3, lam, 0.3 * lam / 1.3, n, batch=64)
    W, e, res = oracle.svrg_solve(X, qc, S, lam, eta, m, b, 1e-12, 1, 0, 200, Ud=Ud)
    Wd = np.linalg.solve(lam * np.eye(d) - P @ A @ P, S)
    assert np.linalg.norm(W - Wd) <= 1e-9 * np.linalg.norm(Wd)
    assert np.linalg.norm(Ud.T @ W) <= 1e-9 * np.linalg.norm(W)


def _exact(X, k):
    u, s, _ = np.linalg.svd(X, full_matrices=False)
    return u[:, :k], s


def test_adaptive_geometric_spectrum_uses_both_branches():
    """sigma_1..10 geometric (10 -> 5), sigma_11 = 4.95: consecutive ratios of
    the top ten lambda are 0.857, so largeDetect splits off 1..9 for plain
    subspace iteration; lambda_11 / lambda_10 = 0.98 leaves 10 to
    shift-and-invert with oversampling.  The result is the exact top-10
    subspace (tan theta <= eps / k of Theorem "mainResultW") and meets the
    (1 + eps) Frobenius bound of the problem statement."""
    d, n, k, p, eps = 200, 3000, 10, 20, 1e-4
    data = workloads.planted_dense(d, n, workloads.spectrum("geometric", d), 7, "f64", 1e-4)
    r = oracle.solve_adaptive(data["Xt"], "f64", k, p, eps, oracle.Options(seed=3))
    assert r.status == 0
    br = [(iv.s, iv.q, iv.branch, iv.cols) for iv in r.intervals]
    assert br[0] == (1, 9, "power", 9)
    assert br[-1][1:] == (10, "shift-invert", p - 9)
    X = data["Xt"].T
    uk, s = _exact(X, k)
    assert oracle.sin_theta(uk, r.U) <= eps / k
    np.testing.assert_allclose(r.theta, s[:k] ** 2, rtol=1e-10)
    err = np.linalg.norm(X - r.U @ (r.U.T @ X))
    assert err <= (1 + eps) * np.sqrt(np.sum(s[k:] ** 2))
    assert np.linalg.norm(r.U.T @ r.U - np.eye(k)) <= 1e-13


def test_adaptive_clustered_spectrum_is_one_interval():
    """sigma_1..4 = 1: no gap of either kind inside I, so the whole problem is
    the q = k interval with oversampling."""
    d, n, k, p, eps = 200, 3000, 4, 8, 1e-4
    data = workloads.planted_dense(d, n, workloads.spectrum("clustered", d), 7, "f64")
    r = oracle.solve_adaptive(data["Xt"], "f64", k, p, eps, oracle.Options(seed=3))
    assert [(iv.s, iv.q, iv.branch, iv.cols) for iv in r.intervals] == \
        [(1, 4, "shift-invert", 8)]
    uk, s = _exact(data["Xt"].T, k)
    assert oracle.sin_theta(uk, r.U) <= eps / k
    np.testing.assert_allclose(r.theta, s[:k] ** 2, rtol=1e-10)


def test_spectral_norm_guarantee():
    """Corollary "mainResult" for the spectral norm: with eps rescaled by
    mu_2 = sqrt(theta_1 / theta_{k+1}), ||X - U U^T X||_2 <= (1 + eps) sigma_{k+1}
    (the exact rank-k error), checked with LAPACK's SVD; both the q = k branch
    and the adaptive loop."""
    d, n, k, p, eps = 160, 2500, 6, 12, 1e-3
    i = np.arange(1, d + 1, dtype=float)
    sig = np.where(i <= k, 1.0 + 0.02 * (k - i), 0.8 * i ** -0.5)
    data = workloads.planted_dense(d, n, sig, 21, "f64")
    X = data["Xt"].T
    s = np.linalg.svd(X, compute_uv=False)
    for fn in (oracle.solve, oracle.solve_adaptive):
        r = fn(data["Xt"], "f64", k, p, eps, oracle.Options(seed=4, norm="spectral"))
        assert r.status == 0
        R = X - r.U @ (r.U.T @ X)
        assert np.linalg.norm(R, 2) <= (1 + eps) * s[k]
    th = oracle.estimate_phase(X, k, p, 4, 4)[1]
    assert oracle.lowrank.stop_scale(th, float(np.sum(X * X)), k, "spectral") == \
        pytest.approx(np.sqrt(th[0] / th[k]))
