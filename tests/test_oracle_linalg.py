"""Pins of the oracle's small linear algebra against LAPACK and SciPy."""
import numpy as np
import scipy.linalg as sla

from oracle.linalg import cholqr2, eigh_desc, jacobi_svd, sin_theta


def test_cholqr2_is_a_qr():
    rng = np.random.default_rng(0)
    W = rng.standard_normal((300, 12)) @ np.diag(np.logspace(0, 4, 12))
    S, R = cholqr2(W)
    assert np.linalg.norm(S.T @ S - np.eye(12)) < 1e-14
    assert np.allclose(np.tril(R, -1), 0.0)
    assert np.linalg.norm(S @ R - W) / np.linalg.norm(W) < 1e-14
    Q, _ = np.linalg.qr(W)
    assert sin_theta(Q, S) < 1e-12


def test_eigh_desc():
    rng = np.random.default_rng(1)
    B = rng.standard_normal((9, 9))
    H = B + B.T
    v, Q = eigh_desc(H)
    assert np.all(np.diff(v) <= 0)
    assert np.linalg.norm(Q @ np.diag(v) @ Q.T - H) < 1e-12
    big = np.argmax(np.abs(Q), axis=0)
    assert np.all(Q[big, np.arange(9)] > 0)


def test_jacobi_svd_matches_lapack():
    rng = np.random.default_rng(2)
    for m, n in [(40, 12), (64, 64), (200, 30)]:
        A = rng.standard_normal((m, n)) @ np.diag(np.linspace(1, 10, n))
        U, s, V = jacobi_svd(A)
        s_ref = np.linalg.svd(A, compute_uv=False)
        np.testing.assert_allclose(s, s_ref, rtol=1e-12)
        assert np.linalg.norm(U @ np.diag(s) @ V.T - A) / np.linalg.norm(A) < 1e-13
        assert np.linalg.norm(U.T @ U - np.eye(n)) < 1e-12


def test_sin_theta_matches_scipy_subspace_angles():
    rng = np.random.default_rng(3)
    for k in (1, 3, 8):
        A = np.linalg.qr(rng.standard_normal((50, k)))[0]
        B = np.linalg.qr(A + 0.1 * rng.standard_normal((50, k)))[0]
        ang = sla.subspace_angles(A, B)
        assert abs(sin_theta(A, B) - np.sin(ang.max())) < 1e-13


def test_tan_theta_non_recursive_form():
    """Appendix C, Lemma nonRecursiveAngle with p = k: tan theta_k(U_k, S) =
    || (U_-k^T S)(U_k^T S)^{-1} ||_2, cross-checked against SciPy's angles."""
    rng = np.random.default_rng(4)
    d, k = 30, 4
    U = np.linalg.qr(rng.standard_normal((d, d)))[0]
    S = U[:, :k] + 0.2 * rng.standard_normal((d, k))
    tan = np.linalg.norm((U[:, k:].T @ S) @ np.linalg.inv(U[:, :k].T @ S), 2)
    ang = sla.subspace_angles(U[:, :k], S).max()
    assert abs(tan - np.tan(ang)) < 1e-12
    Sq = np.linalg.qr(S)[0]
    assert abs(sin_theta(U[:, :k], Sq) - np.sin(ang)) < 1e-13
