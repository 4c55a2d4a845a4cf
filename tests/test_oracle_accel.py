"""Pins of the accelerated inner solver (oracle.accel): the plain solver as
its kappa = 0 special case, the exact solution as its fixed point, and the
accuracy guarantee of the whole method when it replaces the plain solver."""
import numpy as np

import oracle
import workloads


def _problem(seed=3):
    d, n, p = 80, 1500, 6
    i = np.arange(1, d + 1, dtype=float)
    sig = np.where(i <= 3, 2.0, 1.2 * i ** -0.5)
    X = workloads.planted_dense(d, n, sig, seed, "f64")["Xt"].T
    w = oracle.column_sq_norms(X)
    _, qc = oracle.build_table(w)
    S = oracle.cholqr2(np.random.default_rng(seed).standard_normal((d, p)))[0]
    lam1 = np.linalg.eigvalsh(X @ X.T)[-1]
    return X, qc, S, float(np.sum(w)), lam1


def test_kappa_zero_is_the_plain_solver():
    X, qc, S, fro2, lam1 = _problem()
    lam, mu = 1.05 * lam1, 0.05 * lam1
    b, eta, m = oracle.solver_constants(fro2, lam1, lam, mu, X.shape[1], batch=128)
    Wp, ep, rp = oracle.svrg_solve(X, qc, S, lam, eta, m, b, 0.0, 11, 2, 60, fixed_epochs=3)
    Wa, ea, ra = oracle.acc_svrg_solve(X, qc, S, lam, 0.0, 0.0, eta, m, b, 0.0, 11, 2, 60,
                                       fixed_epochs=3)
    assert ep == ea == 3
    assert np.array_equal(Wp, Wa)
    assert np.array_equal(np.array(rp), np.array(ra))


def test_converges_to_the_direct_solution():
    X, qc, S, fro2, lam1 = _problem()
    lam, mu = 1.02 * lam1, 0.02 * lam1
    kappa, beta, b, eta, m = oracle.accel_constants(fro2, lam1, lam, mu, X.shape[1])
    assert kappa > 0 and 0 < beta < 1
    W, e, res = oracle.acc_svrg_solve(X, qc, S, lam, kappa, beta, eta, m, b, 1e-11, 5, 0, 2000)
    Wd = np.linalg.solve(lam * np.eye(X.shape[0]) - X @ X.T, S)
    assert np.linalg.norm(W - Wd) <= 1e-8 * np.linalg.norm(Wd)
    # the reported residual is that of the original system
    assert abs(res[-1] - np.linalg.norm(S - (lam * W - X @ (X.T @ W)))) <= 1e-12 + 1e-6 * res[-1]


def test_whole_method_with_accelerated_solver():
    d, n, k, p, eps = 200, 3000, 4, 8, 1e-4
    data = workloads.planted_dense(d, n, workloads.spectrum("clustered", d), 7, "f64")
    r = oracle.solve(data["Xt"], "f64", k, p, eps, oracle.Options(seed=3, accel=True))
    assert r.status == 0 and r.schedule.accel and r.schedule.kappa >= 0
    X = data["Xt"].T
    u, s, _ = np.linalg.svd(X, full_matrices=False)
    assert oracle.sin_theta(u[:, :k], r.U) <= eps / k
    np.testing.assert_allclose(r.theta, s[:k] ** 2, rtol=1e-10)
