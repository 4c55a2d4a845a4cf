"""Sparse X in compressed-column (CSC) storage with Zipf-distributed rows.

Recipe (one column = one data point x_i of X, d x n):
  * rows: `nnz_col` distinct rows per column; candidates are drawn i.i.d. from
    the truncated Zipf law P(rank j) ~ j^-s on ranks 1..d (inverse CDF of a
    uniform) and the first `nnz_col` distinct ones are kept (rejection of
    repeats); ranks map to row ids through a seeded random permutation; row ids
    are sorted within each column;
  * values: lognormal(0, 1), then each column divided by its Euclidean norm
    (computed in FP64) before rounding to the storage type.
All randomness comes from one NumPy PCG64 generator with the given seed.

Storage dict: d, n, nnz, col_ptr (int32, n + 1), row_idx (int32, nnz), values
(float32 / float64, or uint16 BF16 bit patterns), storage ("csc-f32", ...).
"""
import numpy as np

from .planted import f64_to_bf16_bits


def _distinct_draws(rng, cdf, m, kk):
    """(m, kk) int64 ranks (0-based): the first kk distinct values of i.i.d.
    Zipf draws in each row."""
    out = np.empty((m, kk), dtype=np.int64)
    todo = np.arange(m)
    K = 2 * kk + 32
    while todo.size:
        cand = np.searchsorted(cdf, rng.random((todo.size, K)), side="right")
        order = np.argsort(cand, axis=1, kind="stable")
        sc = np.take_along_axis(cand, order, axis=1)
        first = np.ones_like(sc, dtype=bool)
        first[:, 1:] = sc[:, 1:] != sc[:, :-1]
        pos = np.where(first, order, K)               # first occurrence of each value
        pick = np.argsort(pos, axis=1, kind="stable")[:, :kk]
        ok = np.take_along_axis(pos, pick, axis=1)[:, -1] < K
        out[todo[ok]] = np.take_along_axis(sc, pick, axis=1)[ok]
        todo = todo[~ok]
        K *= 4
    return out


def zipf_csc(d, n, nnz_col, s=1.1, seed=1003, storage="csc-f32", chunk=1 << 16):
    assert 1 <= nnz_col <= d
    rng = np.random.default_rng(seed)
    pmf = np.arange(1, d + 1, dtype=np.float64) ** -s
    cdf = np.cumsum(pmf)
    cdf /= cdf[-1]
    cdf[-1] = 1.0
    perm = rng.permutation(d).astype(np.int32)
    rows = np.empty((n, nnz_col), dtype=np.int32)
    vals = np.empty((n, nnz_col), dtype=np.float64)
    for c0 in range(0, n, chunk):
        m = min(chunk, n - c0)
        r = perm[_distinct_draws(rng, cdf, m, nnz_col)]
        rows[c0:c0 + m] = np.sort(r, axis=1)
        v = rng.lognormal(0.0, 1.0, size=(m, nnz_col))
        vals[c0:c0 + m] = v / np.sqrt(np.sum(v * v, axis=1))[:, None]
    if storage == "csc-f32":
        values = vals.astype(np.float32).ravel()
    elif storage == "csc-f64":
        values = vals.ravel()
    elif storage == "csc-bf16":
        values = f64_to_bf16_bits(vals.ravel())
    else:
        raise ValueError(storage)
    nnz = n * nnz_col
    assert nnz < 2 ** 31
    return {"d": d, "n": n, "nnz": nnz, "storage": storage,
            "col_ptr": (np.arange(n + 1, dtype=np.int64) * nnz_col).astype(np.int32),
            "row_idx": rows.ravel(), "values": values}


def to_dense_xt(sp):
    """Dense (n, d) float64 copy (column-major X) of a small CSC matrix, for
    checks only."""
    xt = np.zeros((sp["n"], sp["d"]), dtype=np.float64)
    cp = sp["col_ptr"].astype(np.int64)
    v = sp["values"]
    if sp["storage"] == "csc-bf16":
        v = (v.astype(np.uint32) << np.uint32(16)).view(np.float32)
    v = v.astype(np.float64)
    cols = np.repeat(np.arange(sp["n"]), np.diff(cp))
    xt[cols, sp["row_idx"]] = v
    return xt
