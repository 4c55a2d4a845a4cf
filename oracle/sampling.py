"""Importance-sampling table and exact inverse-CDF column draws for the
stochastic inner solver.

The paper invokes a variance-reduced stochastic solver for (lambda I - XX^T)
(Section 2.3, Theorem "svrgSolve", cost O~(nnz + d sr(X) lambda_1^2 /
(lambda - lambda_1)^2)) and notes in Section 1.2 that, for a random column x_j,
x_j x_j^T is an unbiased estimate of A = XX^T.  The stable-rank term sr(X) =
||X||_F^2 / sigma_1^2 in that bound is what sampling column i with probability
proportional to ||x_i||^2 gives.  The paper does not spell the sampler out; the
reading implemented here:

  w_i = sum_j X_ji^2, summed in FP64 in row order j = 0, 1, ..., d-1
  q_i = floor(2^24 w_i / max_j w_j) + 1   (q_i = 0 when w_i = 0)
  Q_i = q_0 + ... + q_{i-1}  (uint64, Q_0 = 0),  Q = Q_n,  pi_i = q_i / Q

A draw takes one Philox block (o0, o1, o2, o3), forms u = o0 * 2^32 + o1,
r = floor(u Q / 2^64) (exact 128-bit product) and returns the largest i with
Q_i <= r.  Draw j of step t in epoch e of solve s uses counter
(j, t, e, (3 << 28) | s).  Its importance weight is 1 / (b pi_i) = Q / (b q_i).
"""
import numpy as np

from .philox import philox4x32_10, key_of, stream_word, TAG_SAMPLES

MASK32 = np.uint64(0xFFFFFFFF)
QBITS = 24


def column_sq_norms(X):
    """w_i = ||x_i||^2 for the columns of X (d x n, float64), accumulated in
    row order so that every implementation performs the same roundings.  For a
    CSC matrix with sorted row indices the stored entries of a column are
    visited in that same row order (the skipped zeros would add exactly 0)."""
    d, n = X.shape
    w = np.zeros(n, dtype=np.float64)
    if hasattr(X, "indptr"):
        ptr = X.indptr.astype(np.int64)
        length = np.diff(ptr)
        for t in range(int(length.max()) if n else 0):
            has = length > t
            v = X.data[ptr[:-1][has] + t]
            w[has] += v * v
        return w
    for j in range(d):
        row = X[j, :]
        w += row * row
    return w


def build_table(w):
    """Quantised weights q (uint64) and cumulative table Qc of length n+1."""
    w = np.asarray(w, dtype=np.float64)
    if not np.all(np.isfinite(w)):
        raise ValueError("non-finite column norm")
    wmax = w.max()
    if not wmax > 0:
        raise ValueError("X is zero")
    q = np.where(w > 0, np.floor((w / wmax) * float(1 << QBITS)) + 1.0, 0.0).astype(np.uint64)
    qc = np.zeros(len(w) + 1, dtype=np.uint64)
    np.cumsum(q, out=qc[1:])
    return q, qc


def mulhi64(u, q):
    """floor(u * q / 2^64) for uint64 arrays u and q, exactly, via 32-bit limbs."""
    u = np.asarray(u, dtype=np.uint64)
    q = np.asarray(q, dtype=np.uint64)
    a1, a0 = u >> np.uint64(32), u & MASK32
    b1, b0 = q >> np.uint64(32), q & MASK32
    p00 = a0 * b0
    p01 = a0 * b1
    p10 = a1 * b0
    p11 = a1 * b1
    mid = (p00 >> np.uint64(32)) + (p01 & MASK32) + (p10 & MASK32)
    return p11 + (p01 >> np.uint64(32)) + (p10 >> np.uint64(32)) + (mid >> np.uint64(32))


def draw(qc, u):
    """Largest i with Qc[i] <= floor(u Q / 2^64)."""
    n = len(qc) - 1
    r = mulhi64(u, qc[n])
    return np.searchsorted(qc[:n], r, side="right").astype(np.int64) - 1


def step_indices(seed, solve, epoch, step, b, qc):
    """The b column indices of one inner step, and their weights 1/(b pi_i)."""
    k0, k1 = key_of(seed)
    j = np.arange(b, dtype=np.uint64)
    o0, o1, _, _ = philox4x32_10(j, step, epoch, stream_word(TAG_SAMPLES, solve), k0, k1)
    u = (o0 << np.uint64(32)) | o1
    idx = draw(qc, u)
    n = len(qc) - 1
    q = qc[idx + 1] - qc[idx]
    scale = float(qc[n]) / (float(b) * q.astype(np.float64))
    return idx, scale
