"""Pins of the oracle's Philox generator, Gaussian block and column sampler.

Philox is pinned by the published known-answer vectors and by rocRAND's own
engine (an independent implementation) run on the host.  The sampler is pinned
by exact big-integer arithmetic, by the inverse-CDF property, by a chi-square
test of draw frequencies, and by unbiasedness of the minibatch estimate of
A = XX^T that the inner solver relies on (Section 1.2 notes x_j x_j^T is an
unbiased estimate of A)."""
import os
import shutil
import subprocess

import numpy as np
import pytest
import scipy.stats

from oracle.philox import philox4x32_10, gaussian_block, key_of, stream_word
from oracle.sampling import mulhi64, draw, build_table, step_indices, column_sq_norms

HERE = os.path.dirname(os.path.abspath(__file__))


def test_philox_known_answers():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            rows.append([int(t, 16) for t in line.split()])
    assert len(rows) == 3
    for r in rows:
        out = philox4x32_10(r[0], r[1], r[2], r[3], r[4], r[5])
        assert [int(x) for x in out] == r[6:10]


@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand"):
        pytest.skip("hipcc / rocRAND headers not available")
    exe = str(tmp_path_factory.mktemp("philox") / "philox_ref")
    subprocess.run([hipcc, "-x", "c++", "-O1", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                    "-o", exe, os.path.join(HERE, "philox_ref.cpp")],
                   check=True, capture_output=True)
    return exe


def test_philox_matches_rocrand(rocrand_ref):
    rng = np.random.default_rng(7)
    cases = []
    for _ in range(200):
        seed = int(rng.integers(0, 2 ** 63)) * 2 + int(rng.integers(0, 2))
        c = [int(x) for x in rng.integers(0, 2 ** 32, size=4)]
        c[1] &= (1 << 30) - 1      # rocRAND's offset argument is 4 * (c0 | c1 << 32) in 64 bits
        cases.append((seed, *c))
    # the counter layout used by the method: draw j, step t, epoch e, tag|solve
    for j, t, e, s in [(0, 0, 0, 0), (2047, 123, 5, 40), (5, 1, 0, 3)]:
        cases.append((0x1607029250000002, j, t, e, stream_word(3, s)))
    inp = "".join("%d %d %d %d %d\n" % c for c in cases)
    out = subprocess.run([rocrand_ref], input=inp, capture_output=True, text=True, check=True)
    got = [list(map(int, line.split())) for line in out.stdout.strip().splitlines()]
    assert len(got) == len(cases)
    for c, g in zip(cases, got):
        k0, k1 = key_of(c[0])
        mine = [int(x) for x in philox4x32_10(c[1], c[2], c[3], c[4], k0, k1)]
        assert mine == g, c


def test_gaussian_block_distribution():
    z = gaussian_block(1234, 2, 0, 4096, 64).ravel()
    ks = scipy.stats.kstest(z, "norm")
    assert ks.pvalue > 1e-3
    assert abs(z.mean()) < 0.01 and abs(z.std() - 1.0) < 0.01
    # different tags / solve indices give unrelated blocks
    z2 = gaussian_block(1234, 1, 0, 4096, 64).ravel()
    z3 = gaussian_block(1234, 2, 1, 4096, 64).ravel()
    assert abs(np.corrcoef(z, z2)[0, 1]) < 0.01
    assert abs(np.corrcoef(z, z3)[0, 1]) < 0.01


def test_mulhi64_exact():
    rng = np.random.default_rng(3)
    u = rng.integers(0, 2 ** 63, size=5000, dtype=np.uint64) * np.uint64(2) + \
        rng.integers(0, 2, size=5000, dtype=np.uint64)
    q = rng.integers(1, 2 ** 50, size=5000, dtype=np.uint64)
    got = mulhi64(u, q)
    for a, b, g in zip(u[:500], q[:500], got[:500]):
        assert int(g) == (int(a) * int(b)) >> 64
    assert int(mulhi64(np.uint64(2 ** 64 - 1), np.uint64(2 ** 64 - 1))) == \
        ((2 ** 64 - 1) ** 2) >> 64


def test_inverse_cdf_property_and_zero_weights():
    w = np.array([0.0, 1.0, 4.0, 0.0, 0.25, 9.0, 0.0])
    q, qc = build_table(w)
    assert int(q.max()) == (1 << 24) + 1
    assert list(q[[0, 3, 6]]) == [0, 0, 0]
    rng = np.random.default_rng(11)
    u = rng.integers(0, 2 ** 63, size=20000, dtype=np.uint64) * np.uint64(2)
    idx = draw(qc, u)
    total = int(qc[-1])
    for a, i in zip(u[:2000], idx[:2000]):
        r = (int(a) * total) >> 64
        assert int(qc[i]) <= r < int(qc[i + 1])
    assert not np.isin(idx, [0, 3, 6]).any()
    # the extreme draws land on the first and last positive-weight columns
    assert int(draw(qc, np.array([0], dtype=np.uint64))[0]) == 1
    assert int(draw(qc, np.array([2 ** 64 - 1], dtype=np.uint64))[0]) == 5


def test_draw_frequencies_chi_square():
    rng = np.random.default_rng(5)
    X = rng.standard_normal((6, 40)) * rng.uniform(0.1, 3.0, size=40)[None, :]
    q, qc = build_table(column_sq_norms(X))
    counts = np.zeros(40)
    for t in range(100):
        idx, _ = step_indices(99, 0, 0, t, 2000, qc)
        counts += np.bincount(idx, minlength=40)
    expected = q.astype(np.float64) / float(qc[-1]) * counts.sum()
    chi = scipy.stats.chisquare(counts, expected)
    assert chi.pvalue > 1e-3


def test_weights_give_unbiased_estimate_of_A():
    rng = np.random.default_rng(8)
    X = rng.standard_normal((5, 30)) * rng.uniform(0.2, 2.0, size=30)[None, :]
    A = X @ X.T
    _, qc = build_table(column_sq_norms(X))
    acc = np.zeros_like(A)
    T = 400
    b = 500
    for t in range(T):
        idx, sc = step_indices(1, 0, 0, t, b, qc)
        Xb = X[:, idx]
        acc += (Xb * sc[None, :]) @ Xb.T
    est = acc / T
    assert np.linalg.norm(est - A) / np.linalg.norm(A) < 0.02


def test_column_norms_match_definition():
    rng = np.random.default_rng(2)
    X = rng.standard_normal((100, 37))
    w = column_sq_norms(X)
    np.testing.assert_allclose(w, np.linalg.norm(X, axis=0) ** 2, rtol=1e-14)
