"""Small dense linear algebra used by the oracle and by its pins.

* ``cholqr2``: the QR step of the subspace iteration (Algorithm "subspace
  iteration", Section 2.2.1: Y = S R), realised as Cholesky-QR applied twice.
* ``eigh_desc``: the symmetric eigendecomposition of the p x p projected matrix
  S^T C S (Algorithm "low-rank approximation restricted to a subspace",
  Section 2.2.2), eigenvalues in descending order, each eigenvector's
  largest-magnitude entry made positive.
* ``jacobi_svd``: one-sided (Hestenes) Jacobi SVD, an SVD written out by hand
  for small inputs, used only to pin the exact answer Pi* = sum_{i<=k} u_i u_i^T
  (Section 1) independently of LAPACK.
* ``sin_theta``: sine of the largest principal angle between two subspaces
  (Appendix C, Definition "principalAngle").
"""
import numpy as np
import scipy.linalg as sla


class NotSPD(Exception):
    pass


# A Cholesky pivot below this fraction of its diagonal entry marks the block
# as numerically rank deficient (its Gram matrix is then treated as not
# positive definite).
PIVOT_REL = 1e-14


def cholqr(w):
    g = w.T @ w
    g = 0.5 * (g + g.T)
    try:
        lower = np.linalg.cholesky(g)
    except np.linalg.LinAlgError as e:
        raise NotSPD(str(e))
    piv = np.diag(lower) ** 2
    if not np.all(piv > PIVOT_REL * np.diag(g)):
        raise NotSPD("pivot below %g of its diagonal" % PIVOT_REL)
    # S = W R^{-1} with R = L^T, i.e. S^T = L^{-1} W^T
    s = sla.solve_triangular(lower, w.T, lower=True).T
    return s, lower.T


def cholqr2(w):
    s1, r1 = cholqr(w)
    s2, r2 = cholqr(s1)
    return s2, r2 @ r1


def sign_fix(v):
    """Make the largest-magnitude entry of each column positive (first such
    entry on ties)."""
    idx = np.argmax(np.abs(v), axis=0)
    sgn = np.sign(v[idx, np.arange(v.shape[1])])
    sgn[sgn == 0] = 1.0
    return v * sgn[None, :]


def eigh_desc(h):
    h = 0.5 * (h + h.T)
    vals, vecs = np.linalg.eigh(h)
    order = np.argsort(-vals, kind="stable")
    return vals[order], sign_fix(vecs[:, order])


def jacobi_svd(a, tol=1e-15, max_sweeps=60):
    """One-sided Jacobi SVD of a (m x n, m >= n would not be required): rotates
    pairs of columns of a until they are mutually orthogonal.  Returns U (m x r),
    s (r,), V (n x r) with a = U diag(s) V^T, s descending, r = n."""
    a = np.array(a, dtype=np.float64, copy=True)
    m, n = a.shape
    v = np.eye(n)
    for _ in range(max_sweeps):
        off = 0.0
        for i in range(n - 1):
            for j in range(i + 1, n):
                ai, aj = a[:, i], a[:, j]
                alpha = ai @ ai
                beta = aj @ aj
                gamma = ai @ aj
                if alpha == 0.0 or beta == 0.0 or gamma == 0.0:
                    continue
                c_ij = abs(gamma) / np.sqrt(alpha * beta)
                off = max(off, c_ij)
                if c_ij < tol:
                    continue
                zeta = (beta - alpha) / (2.0 * gamma)
                t = np.sign(zeta) / (abs(zeta) + np.sqrt(1.0 + zeta * zeta)) if zeta != 0 else 1.0
                c = 1.0 / np.sqrt(1.0 + t * t)
                s = c * t
                a[:, i], a[:, j] = c * ai - s * aj, s * ai + c * aj
                vi, vj = v[:, i].copy(), v[:, j].copy()
                v[:, i], v[:, j] = c * vi - s * vj, s * vi + c * vj
        if off < tol:
            break
    s = np.linalg.norm(a, axis=0)
    order = np.argsort(-s, kind="stable")
    s = s[order]
    a = a[:, order]
    v = v[:, order]
    u = np.zeros_like(a)
    nz = s > 0
    u[:, nz] = a[:, nz] / s[nz]
    return u, s, v


def sin_theta(u1, u2):
    """sin of the largest principal angle between span(u1) and span(u2), both
    with orthonormal columns and the same number of columns:
    || u2 - u1 (u1^T u2) ||_2."""
    return float(np.linalg.norm(u2 - u1 @ (u1.T @ u2), 2))
