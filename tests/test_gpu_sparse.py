"""Compressed-column (CSC) X on the GPU against the CPU oracle.

Bit-exact: the structure checks, column norms and sampling table.  Within
rounding (different summation orders): passes, inner solves and whole solves.
The inner-step update adds each row's contributions in a fixed order (sorted by
row, then by sample), so repeated runs are bitwise equal; a plan whose
minibatch times its largest column passes the sorted form's cap adds with FP64
atomics instead, whose rounding order varies (tested against the oracle only).
"""
import numpy as np
import pytest

import oracle
import workloads
from workloads import sparse

pytestmark = pytest.mark.gpu

def ragged_csc(d, n, seed, storage="csc-f32", max_nnz=12):
    """Columns with 0..max_nnz distinct sorted rows (empty columns included),
    Gaussian values."""
    rng = np.random.default_rng(seed)
    counts = rng.integers(0, max_nnz + 1, size=n)
    counts[:3] = [0, max_nnz, 1]
    rows = [np.sort(rng.choice(d, size=c, replace=False)) for c in counts]
    vals = rng.standard_normal(int(counts.sum()))
    cp = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    ri = (np.concatenate(rows) if counts.sum() else np.zeros(0)).astype(np.int32)
    if storage == "csc-f32":
        v = vals.astype(np.float32)
    elif storage == "csc-f64":
        v = vals
    else:
        v = workloads.f64_to_bf16_bits(vals)
    return {"d": d, "n": n, "nnz": int(counts.sum()), "storage": storage, "col_ptr": cp,
            "row_idx": ri, "values": v}


def dev(sp):
    from paper_1607_02925_amd import lowrank
    return lowrank.CscMatrix.from_arrays(sp["d"], sp["n"], sp["col_ptr"], sp["row_idx"],
                                         sp["values"])


def plan(sp, k, p, eps=1e-4, **kw):
    from paper_1607_02925_amd import lowrank
    return lowrank.Plan(dev(sp), k, p, eps, **kw)


def test_structure_checks(torch_cuda):
    from paper_1607_02925_amd import lowrank
    sp = ragged_csc(50, 40, 1)
    bad_ptr = dict(sp, col_ptr=sp["col_ptr"].copy())
    bad_ptr["col_ptr"][5] = bad_ptr["col_ptr"][6] + 1
    unsorted = dict(sp, row_idx=sp["row_idx"].copy())
    c = int(np.argmax(np.diff(sp["col_ptr"]) >= 2))
    a = sp["col_ptr"][c]
    unsorted["row_idx"][a], unsorted["row_idx"][a + 1] = sp["row_idx"][a + 1], sp["row_idx"][a]
    out_of_range = dict(sp, row_idx=sp["row_idx"].copy())
    out_of_range["row_idx"][-1] = 50
    for bad in (bad_ptr, unsorted, out_of_range):
        print("structure case", flush=True)
        with pytest.raises(lowrank.LowRankError) as e:
            plan(bad, 2, 4)
        assert e.value.code == lowrank.LR_EINVAL
    plan(sp, 2, 4).close()


@pytest.mark.parametrize("storage", ["csc-f64", "csc-f32", "csc-bf16"])
def test_norms_and_table_bit_exact(torch_cuda, storage):
    sp = ragged_csc(300, 2500, 3, storage)
    pl = plan(sp, 2, 5)
    w, cdf, fro2 = pl.prepare()
    X = oracle.decode(sp, storage)
    wo = oracle.column_sq_norms(X)
    _, qc = oracle.build_table(wo)
    assert np.array_equal(w.cpu().numpy(), wo)
    assert np.array_equal(cdf.cpu().numpy().astype(np.uint64), qc)
    assert fro2 == pytest.approx(float(np.sum(wo)), rel=1e-14)
    # the draws of a step are the oracle's, index for index
    for (solve, epoch, step) in [(0, 0, 0), (3, 2, 17)]:
        idx, sc = pl.sample(solve, epoch, step, 700)
        io, so = oracle.step_indices(0, solve, epoch, step, 700, qc)
        assert np.array_equal(idx.cpu().numpy(), io)
        assert np.array_equal(sc.cpu().numpy(), so)


@pytest.mark.parametrize("case", [("ragged", "csc-f32", 3), ("ragged", "csc-f64", 17),
                                  ("zipf", "csc-f32", 32), ("zipf", "csc-bf16", 40),
                                  ("ragged", "csc-bf16", 64)])
def test_apply_A(torch_cuda, case):
    """X (X^T W) for every padded width (16, 32, 48, 64 columns), empty columns,
    and rows long enough to span several chunks."""
    import torch
    kind, storage, p = case
    if kind == "zipf":
        sp = sparse.zipf_csc(600, 5000, 16, seed=11, storage=storage)
        assert np.max(np.bincount(sp["row_idx"])) > 2 * 2048
    else:
        sp = ragged_csc(333, 4097, 5, storage)
    pl = plan(sp, 1, p)
    W = np.random.default_rng(p).standard_normal((sp["d"], p))
    Y = pl.apply_A(torch.from_numpy(W).cuda()).cpu().numpy()
    Yo = oracle.apply_A(oracle.decode(sp, storage), W)
    scale = np.max(np.abs(Yo))
    assert np.max(np.abs(Y - Yo)) <= 1e-13 * scale * np.sqrt(sp["n"])


@pytest.mark.parametrize("storage", ["csc-f32", "csc-bf16"])
def test_svrg_solve_fixed_epochs(torch_cuda, storage):
    import torch
    sp = sparse.zipf_csc(600, 5000, 16, seed=11, storage=storage)
    X = oracle.decode(sp, storage)
    p = 8
    pl = plan(sp, 2, p, seed=99)
    pl.prepare()
    _, qc = oracle.build_table(oracle.column_sq_norms(X))
    S = oracle.cholqr2(np.random.default_rng(1).standard_normal((600, p)))[0]
    lam1 = np.linalg.eigvalsh((X @ X.T).toarray())[-1]
    lam, b = 1.1 * lam1, 512
    fro2 = float(X.multiply(X).sum())
    b, eta, m = oracle.solver_constants(fro2, lam1, lam, 0.1 * lam1, sp["n"], batch=b)
    Wg, res_g = pl.svrg_solve(torch.from_numpy(S).cuda(), lam, eta, m, b, 4, 3)
    Wo, e, res_o = oracle.svrg_solve(X, qc, S, lam, eta, m, b, 0.0, 99, 4, 60, fixed_epochs=3)
    Wg = Wg.cpu().numpy()
    print("m=%d b=%d eta=%.3e residuals gpu %s oracle %s" % (m, b, eta, res_g, res_o), flush=True)
    assert np.max(np.abs(Wg - Wo)) <= 1e-9 * np.max(np.abs(Wo))
    np.testing.assert_allclose(res_g, res_o, rtol=1e-7)


def test_solve_auto_matches_oracle(torch_cuda):
    sp = sparse.zipf_csc(600, 5000, 16, seed=11)
    k, p, eps = 1, 4, 1e-4
    ref = oracle.solve(sp, "csc-f32", k, p, eps, oracle.Options(seed=7))
    pl = plan(sp, k, p, eps, seed=7)
    st, U, theta, rep = pl.solve()
    assert st == ref.status == 0
    assert pl.schedule().epochs == ref.schedule.epochs
    assert oracle.sin_theta(ref.U, U.cpu().numpy()) <= 1e-6
    np.testing.assert_allclose(theta, ref.theta, rtol=1e-9)


def test_replay_prefix_p32(torch_cuda):
    """k = 16, p = 32 on the reduced Zipf workload, three outer iterations of a
    fixed schedule: the whole trajectory (estimate phase, passes, 2-epoch
    inner solves, CholQR2, final Rayleigh-Ritz) against the oracle."""
    from paper_1607_02925_amd import lowrank
    w = workloads.workload("zipf-2000x20000-csc-f32")
    X = oracle.decode(w["Xt"], w["storage"])
    lam1 = np.linalg.eigvalsh((X @ X.T).toarray())[-1]
    lam, mu = 1.05 * lam1, 0.05 * lam1
    b, eta, m = oracle.solver_constants(w["n"] * 1.0, lam1, lam, mu, w["n"], batch=1024)
    m = min(m, 40)
    sched = oracle.Schedule(lam=lam, mu_hat=mu, eta=eta, m=m, b=b, first_solve=0, outer=3,
                            epochs=[2, 2, 2])
    ref = oracle.solve(w["Xt"], w["storage"], w["k"], w["p"], w["eps"],
                       oracle.Options(seed=w["solver_seed"]), replay=sched)
    rs = lowrank.Schedule(lam, mu, eta, m, b, 0, 3, [2, 2, 2])
    pl = plan(w["Xt"], w["k"], w["p"], w["eps"], seed=w["solver_seed"], replay=rs)
    st, U, theta, _ = pl.solve()
    assert st == 0
    sin = oracle.sin_theta(ref.U, U.cpu().numpy())
    print("p32 replay prefix: sin=%.2e" % sin, flush=True)
    assert sin <= 1e-8
    np.testing.assert_allclose(theta, ref.theta, rtol=1e-10)


@pytest.mark.slow
def test_full_size_pass_table_and_epoch(torch_cuda):
    """The 50000 x 1000000 Zipf workload at full size: the sampling table bit
    for bit, one whole pass X (X^T W) for p = 32, and one inner-solver epoch
    (m = 3 steps of b = 8192 samples) against the oracle."""
    import torch
    w = workloads.workload("zipf-50000x1000000-csc-f32")
    X = oracle.decode(w["Xt"], w["storage"])
    print("full-size CSC generated", flush=True)
    pl = plan(w["Xt"], w["k"], w["p"], w["eps"], seed=w["solver_seed"])
    wg, cdf, fro2 = pl.prepare()
    wo = oracle.column_sq_norms(X)
    _, qc = oracle.build_table(wo)
    assert np.array_equal(wg.cpu().numpy(), wo)
    assert np.array_equal(cdf.cpu().numpy().astype(np.uint64), qc)
    W = np.random.default_rng(3).standard_normal((w["d"], w["p"]))
    Y = pl.apply_A(torch.from_numpy(W).cuda()).cpu().numpy()
    Yo = oracle.apply_A(X, W)
    rel = np.linalg.norm(Y - Yo) / np.linalg.norm(Yo)
    print("full-size pass rel err %.2e" % rel, flush=True)
    assert rel <= 1e-13
    S = oracle.cholqr2(W)[0]
    lam = 1.01 * fro2            # above lambda_1 (<= ||X||_F^2)
    eta = 0.5 / lam
    Wg, res_g = pl.svrg_solve(torch.from_numpy(S).cuda(), lam, eta, 3, 8192, 0, 1)
    Wo, _, res_o = oracle.svrg_solve(X, qc, S, lam, eta, 3, 8192, 0.0, w["solver_seed"], 0, 60,
                                     fixed_epochs=1)
    Wg = Wg.cpu().numpy()
    assert np.max(np.abs(Wg - Wo)) <= 1e-10 * np.max(np.abs(Wo))
    np.testing.assert_allclose(res_g, res_o, rtol=1e-8)


def _fixed_epochs(sp, storage, p, b_req, seed, epochs=2):
    """Inner solves under fixed epochs on the GPU (twice) and in the oracle."""
    import torch
    X = oracle.decode(sp, storage)
    d = sp["d"]
    pl = plan(sp, 2, p, seed=seed)
    pl.prepare()
    _, qc = oracle.build_table(oracle.column_sq_norms(X))
    S = oracle.cholqr2(np.random.default_rng(3).standard_normal((d, p)))[0]
    lam1 = np.linalg.eigvalsh((X @ X.T).toarray())[-1]
    lam = 1.1 * lam1
    fro2 = float(X.multiply(X).sum())
    b, eta, m = oracle.solver_constants(fro2, lam1, lam, 0.1 * lam1, sp["n"], batch=b_req)
    runs = [pl.svrg_solve(torch.from_numpy(S).cuda(), lam, eta, m, b, 5, epochs)
            for _ in range(2)]
    Wo, _, res_o = oracle.svrg_solve(X, qc, S, lam, eta, m, b, 0.0, seed, 5, 60,
                                     fixed_epochs=epochs)
    return runs, Wo, res_o, (m, b)


def test_inner_steps_bitwise_repeatable(torch_cuda):
    """The same inner solve twice on a Zipf-row matrix (rows shared by many
    sampled columns, the sorted scatter's long runs): bitwise equal, and
    against the oracle."""
    import torch
    sp = sparse.zipf_csc(600, 5000, 16, seed=11)
    runs, Wo, res_o, mb = _fixed_epochs(sp, "csc-f32", 8, 512, 99)
    (W1, r1), (W2, r2) = runs
    print("m, b =", mb, "residuals", r1, res_o, flush=True)
    assert torch.equal(W1, W2)
    assert np.array_equal(np.asarray(r1), np.asarray(r2))
    W = W1.cpu().numpy()
    assert np.max(np.abs(W - Wo)) <= 1e-9 * np.max(np.abs(Wo))
    np.testing.assert_allclose(r1, res_o, rtol=1e-7)


@pytest.mark.parametrize("p", [5, 33])
def test_ragged_columns_inner_steps(torch_cuda, p):
    """Columns of 0..12 entries (empty ones included), so the sorted scatter
    pads the short columns' slots: bitwise repeatable and against the oracle,
    for p in one and in three 16-column slices."""
    import torch
    sp = ragged_csc(300, 4000, 21, max_nnz=12)
    runs, Wo, res_o, mb = _fixed_epochs(sp, "csc-f32", p, 1024, 17)
    (W1, r1), (W2, r2) = runs
    print("p %d m, b = %s residuals %s %s" % (p, mb, r1, res_o), flush=True)
    assert torch.equal(W1, W2)
    W = W1.cpu().numpy()
    assert np.max(np.abs(W - Wo)) <= 1e-9 * np.max(np.abs(Wo))
    np.testing.assert_allclose(r1, res_o, rtol=1e-7)


def test_wide_column_atomic_scatter(torch_cuda):
    """One column holding every row makes minibatch x largest column pass the
    sorted scatter's cap (4000 x 1500 > 2^22), so the plan adds with atomics:
    against the oracle within rounding."""
    sp = ragged_csc(1500, 4000, 23, max_nnz=8)
    cp = sp["col_ptr"].astype(np.int64)
    # replace column 5 by a column with all 1500 rows
    rows = [sp["row_idx"][cp[i]:cp[i + 1]] for i in range(sp["n"])]
    vals = [sp["values"][cp[i]:cp[i + 1]] for i in range(sp["n"])]
    rows[5] = np.arange(1500, dtype=np.int32)
    vals[5] = (np.random.default_rng(5).standard_normal(1500) * 0.05).astype(np.float32)
    counts = np.array([len(r) for r in rows])
    sp = dict(sp, nnz=int(counts.sum()), row_idx=np.concatenate(rows).astype(np.int32),
              values=np.concatenate(vals).astype(np.float32),
              col_ptr=np.concatenate([[0], np.cumsum(counts)]).astype(np.int32))
    runs, Wo, res_o, mb = _fixed_epochs(sp, "csc-f32", 8, 2048, 29, epochs=1)
    W = runs[0][0].cpu().numpy()
    print("m, b =", mb, "residuals", runs[0][1], res_o, flush=True)
    assert np.max(np.abs(W - Wo)) <= 1e-9 * np.max(np.abs(Wo))
    np.testing.assert_allclose(runs[0][1], res_o, rtol=1e-7)
