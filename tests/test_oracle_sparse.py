"""Pins of the oracle on compressed-column (CSC) input and of the sparse
generator, against what the mathematics fixes: the dense definition of every
quantity (a CSC matrix is the same linear map as its dense copy), the exact
SVD from LAPACK, and the accuracy guarantee of the method."""
import numpy as np
import pytest

import oracle
from workloads import sparse


@pytest.fixture(scope="module")
def small():
    sp = sparse.zipf_csc(600, 5000, 16, seed=11)
    return sp, sparse.to_dense_xt(sp)


def test_generator_structure(small):
    sp, xt = small
    d, n, kk = 600, 5000, 16
    cp, ri = sp["col_ptr"], sp["row_idx"]
    assert cp.dtype == np.int32 and ri.dtype == np.int32 and sp["values"].dtype == np.float32
    assert np.array_equal(cp, np.arange(n + 1) * kk)
    rows = ri.reshape(n, kk)
    assert np.all(np.diff(rows, axis=1) > 0)          # distinct and sorted in each column
    assert rows.min() >= 0 and rows.max() < d
    w = np.sum(sp["values"].astype(np.float64).reshape(n, kk) ** 2, axis=1)
    assert np.max(np.abs(w - 1.0)) < 1e-6              # unit columns (up to FP32 rounding)
    assert np.all(sp["values"] > 0)                    # lognormal values are positive


def test_generator_zipf_marginals():
    """With one draw per column the row frequencies follow the truncated Zipf
    law P(rank j) ~ j^-1.1; the most frequent row (rank 1) has probability
    1 / H_{d,1.1}.  Checked by a chi-square statistic over the top ranks."""
    d, n = 200, 200000
    sp = sparse.zipf_csc(d, n, 1, seed=5)
    cnt = np.bincount(sp["row_idx"], minlength=d)
    pmf = np.arange(1, d + 1, dtype=float) ** -1.1
    pmf /= pmf.sum()
    obs = np.sort(cnt)[::-1][:20]
    exp = n * pmf[:20]
    chi2 = np.sum((obs - exp) ** 2 / exp)
    assert chi2 < 60, chi2                              # 20 dof; p < 1e-5 beyond ~50
    assert abs(obs[0] / n - pmf[0]) < 0.01


def test_csc_decode_and_norms_equal_dense(small):
    sp, xt = small
    X = oracle.decode(sp, "csc-f32")
    Xd = oracle.decode(xt, "f64")
    assert X.shape == Xd.shape
    assert np.array_equal(X.toarray(), Xd)
    # the sampler's norms follow the same (row-order) roundings as the dense definition
    assert np.array_equal(oracle.column_sq_norms(X), oracle.column_sq_norms(Xd))
    W = np.random.default_rng(0).standard_normal((600, 7))
    np.testing.assert_allclose(oracle.apply_A(X, W), Xd @ (Xd.T @ W), rtol=1e-12, atol=1e-12)


def test_csc_bf16_decode():
    sp = sparse.zipf_csc(50, 300, 5, seed=2, storage="csc-bf16")
    X = oracle.decode(sp, "csc-bf16").toarray()
    xt = sparse.to_dense_xt(sp)
    assert np.array_equal(X, xt.T)
    # BF16 keeps 8 significant bits: the columns stay unit within 2^-7
    assert np.max(np.abs(np.sum(X * X, axis=0) - 1.0)) < 2 ** -6


def test_unsorted_rows_rejected():
    sp = sparse.zipf_csc(40, 30, 4, seed=1)
    bad = dict(sp, row_idx=sp["row_idx"].copy())
    bad["row_idx"][0], bad["row_idx"][1] = bad["row_idx"][1], bad["row_idx"][0]
    with pytest.raises(oracle.LowRankError) as e:
        oracle.decode(bad, "csc-f32")
    assert e.value.code == oracle.LR_EINVAL


def test_sparse_solve_against_exact_svd(small):
    """Top singular vector of a Zipf CSC matrix: the method's result against the
    LAPACK SVD of the dense copy (tan theta <= eps / k is the per-interval
    target of Theorem "mainResultW"), the (1 + eps) Frobenius bound of the
    problem statement, and the same decisions as on the dense copy."""
    sp, xt = small
    k, p, eps = 1, 4, 1e-4
    r = oracle.solve(sp, "csc-f32", k, p, eps, oracle.Options(seed=7))
    assert r.status == 0
    Xd = xt.T
    u, s, _ = np.linalg.svd(Xd, full_matrices=False)
    sin = oracle.sin_theta(u[:, :k], r.U)
    assert sin <= eps / k, sin
    np.testing.assert_allclose(r.theta, s[:k] ** 2, rtol=1e-10)
    err = np.linalg.norm(Xd - r.U @ (r.U.T @ Xd))
    best = np.sqrt(np.sum(s[k:] ** 2))
    assert err <= (1 + eps) * best
    rd = oracle.solve(xt, "f64", k, p, eps, oracle.Options(seed=7))
    assert rd.schedule.epochs == r.schedule.epochs and rd.schedule.b == r.schedule.b
    assert oracle.sin_theta(rd.U, r.U) <= 1e-12
