"""The dense workloads at full size, in the launch configuration the benchmark
times, against the oracle:

* 2048 x 200000 f32 (the benchmark workload): the sampling table bit for bit,
  one whole pass X (X^T W) at p = 20, and one whole inner-solver epoch with the
  schedule a solve of this workload uses (m = 124 steps of b = 2048 samples),
  with FP64 and with FP32 matrix-core steps;
* 4096 x 500000 bf16: the sampling table bit for bit and one whole pass at
  p = 48, and a whole adaptive solve against the exact top-k subspace;
* whole solves of the 2048 x 200000 f32 workload (as the NumPy generator makes
  it) against the stored full oracle run on the same bytes, in the FP64 form
  and with matrix-core passes and steps;
* the matrix-core pass elementwise on both workloads.

The oracle works on column chunks of X (FP64 copies of 1-2 GB), so its memory
stays bounded; the chunk sums of the pass reorder FP64 additions only.
"""
import os

import numpy as np
import pytest

import oracle
import workloads

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

CHUNK = 50000
HERE = os.path.dirname(os.path.abspath(__file__))


def host_columns(Xt, storage, c0, c1):
    """X[:, c0:c1] in FP64 from the device tensor Xt (n x d)."""
    import torch
    part = Xt[c0:c1]
    if storage == "bf16":
        part = part.view(torch.int16)
    return oracle.decode(part.cpu().numpy(), storage)


def chunked_norms_and_pass(Xt, storage, n, W):
    """Column squared norms (each column in row order, as the oracle defines
    them) and X (X^T W), over column chunks."""
    w = np.empty(n)
    Y = np.zeros((W.shape[0], W.shape[1]))
    for c0 in range(0, n, CHUNK):
        c1 = min(n, c0 + CHUNK)
        Xc = host_columns(Xt, storage, c0, c1)
        w[c0:c1] = oracle.column_sq_norms(Xc)
        Y += oracle.apply_A(Xc, W)
        del Xc
    return w, Y


@pytest.mark.parametrize("name", ["planted-2048x200000-f32", "planted-4096x500000-bf16"])
def test_full_size_table_and_pass(torch_cuda, name):
    import torch
    from paper_1607_02925_amd import lowrank
    w = workloads.workload(name, device="cuda")
    print("%s generated on the GPU" % name, flush=True)
    plan = lowrank.Plan(w["Xt"], w["k"], w["p"], w["eps"], seed=w["solver_seed"])
    wg, cdf, fro2 = plan.prepare()
    W = np.random.default_rng(11).standard_normal((w["d"], w["p"]))
    Y = plan.apply_A(torch.from_numpy(W).cuda()).cpu().numpy()
    wo, Yo = chunked_norms_and_pass(w["Xt"], w["storage"], w["n"], W)
    _, qc = oracle.build_table(wo)
    assert np.array_equal(wg.cpu().numpy(), wo)
    assert np.array_equal(cdf.cpu().numpy().astype(np.uint64), qc)
    assert fro2 == pytest.approx(float(np.sum(wo)), rel=1e-12)
    rel = np.linalg.norm(Y - Yo) / np.linalg.norm(Yo)
    print("%s: table bit-exact, pass rel err %.2e" % (name, rel), flush=True)
    assert rel <= 1e-13
    # elementwise against each entry's own scale: the pass in FP64 errs by a few
    # (n + d) 2^-53 of |X| (|X|^T |W|); here bounded through |Y_r| sums of
    # column magnitudes, sampled rows (the full |X| product is a pass itself)
    Wa = np.abs(W)
    Yb = np.zeros_like(Y)
    for c0 in range(0, w["n"], CHUNK):
        Xc = np.abs(host_columns(w["Xt"], w["storage"], c0, min(w["n"], c0 + CHUNK)))
        Yb += Xc @ (Xc.T @ Wa)
        del Xc
    assert np.all(np.abs(Y - Yo) <= 4 * (w["n"] + w["d"]) * 2.0 ** -53 * Yb)
    # the matrix-core pass on the same X and W, elementwise against the same bound
    plan_mc = lowrank.Plan(w["Xt"], w["k"], w["p"], w["eps"], seed=w["solver_seed"],
                           precision=lowrank.LR_PREC_MC_PASS)
    Ym = plan_mc.apply_A(torch.from_numpy(W).cuda()).cpu().numpy()
    err_mc = np.abs(Ym - Yo)
    rel_mc = np.linalg.norm(Ym - Yo) / np.linalg.norm(Yo)
    print("%s: matrix-core pass rel err %.2e, max err / bound %.2e" %
          (name, rel_mc, float(np.max(err_mc / Yb))), flush=True)
    assert np.all(err_mc <= 2e-5 * Yb)
    assert rel_mc <= 1e-6


@pytest.mark.parametrize("precision", [0, 2])
def test_full_size_epoch_bench_schedule(torch_cuda, precision):
    """One inner-solver epoch on 2048 x 200000 f32 with the schedule of this
    workload's solve (shift 101.647, eta 9.838e-3, m = 124, b = 2048): the
    iterate and the residuals agree with the oracle's.  With FP32 matrix-core
    steps (precision 2) the bar is 1e-4 of the correction W - W_0 the steps
    made, as for the smaller FP32-step solves."""
    import torch
    from paper_1607_02925_amd import lowrank
    name = "planted-2048x200000-f32"
    w = workloads.workload(name, device="cuda")
    plan = lowrank.Plan(w["Xt"], w["k"], w["p"], w["eps"], seed=w["solver_seed"],
                        precision=precision)
    wg, _, _ = plan.prepare()
    X = host_columns(w["Xt"], w["storage"], 0, w["n"])      # 2048 x 200000 FP64
    wo = oracle.column_sq_norms(X)
    assert np.array_equal(wg.cpu().numpy(), wo)
    _, qc = oracle.build_table(wo)
    S = oracle.cholqr2(np.random.default_rng(5).standard_normal((w["d"], w["p"])))[0]
    lam, eta, m, b = 101.64710238615051, 0.009837925024862453, 124, 2048
    Wg, res_g = plan.svrg_solve(torch.from_numpy(S).cuda(), lam, eta, m, b, 3, 1)
    Wo, _, res_o = oracle.svrg_solve(X, qc, S, lam, eta, m, b, 0.0, w["solver_seed"], 3, 60,
                                     fixed_epochs=1)
    Wg = Wg.cpu().numpy()
    rel = np.linalg.norm(Wg - Wo) / np.linalg.norm(Wo)
    print("epoch (precision %d): W rel err %.2e, residuals gpu %s oracle %s" %
          (precision, rel, res_g, res_o), flush=True)
    if precision == 0:
        assert rel <= 1e-11
        np.testing.assert_allclose(res_g, res_o, rtol=1e-8)
    else:
        W0 = oracle.svrg_solve(X, qc, S, lam, eta, m, b, 0.0, w["solver_seed"], 3, 60,
                               fixed_epochs=0)[0]
        err = np.linalg.norm(Wg - Wo) / np.linalg.norm(Wo - W0)
        print("|W_f32 - W_oracle| / |W - W_0| = %.2e" % err, flush=True)
        assert err <= 1e-4
        np.testing.assert_allclose(res_g, res_o, rtol=1e-3)
    assert res_o[-1] < res_o[0]


def test_full_size_adaptive_bf16_exact_subspace(torch_cuda):
    """A whole solve of 4096 x 500000 bf16 (k = 32, p = 48, eps = 1e-4) by the
    adaptive partitioning of Algorithm "main", against the definition of the
    answer: the top-k eigenvectors of X X^T for the stored X, from an FP64 Gram
    summed over column chunks on the CPU and LAPACK's eigh.  (The q = k branch
    needs about 300 outer iterations on this spectrum; its trajectory is
    checked on the oracle-sized 512 x 16384 version.)"""
    import time
    import torch
    from paper_1607_02925_amd import lowrank
    w = workloads.workload("planted-4096x500000-bf16", device="cuda")
    k, p = w["k"], w["p"]
    plan = lowrank.Plan(w["Xt"], k, p, w["eps"], seed=w["solver_seed"], adaptive=1)
    t = time.time()
    st, U, theta, rep = plan.solve()
    torch.cuda.synchronize()
    print("adaptive solve: status %d in %.2f s, %d passes, %d inner steps, intervals %s" %
          (st, time.time() - t, rep["passes"], rep["steps"],
           [(iv["s"], iv["q"], iv["branch"], iv["iters"]) for iv in rep["intervals"]]),
          flush=True)
    assert st == 0
    d, n = w["d"], w["n"]
    gram = np.zeros((d, d))
    for c0 in range(0, n, CHUNK):
        xc = host_columns(w["Xt"], w["storage"], c0, min(n, c0 + CHUNK))
        gram += xc @ xc.T
        del xc
    ev, V = np.linalg.eigh(gram)
    ev, V = ev[::-1], V[:, ::-1]
    Ug = U.cpu().numpy()
    sin = oracle.sin_theta(V[:, :k], Ug)
    rel = np.max(np.abs(theta - ev[:k]) / ev[:k])
    print("sin vs exact top-%d subspace %.2e, Ritz values rel err %.2e, sin vs planted %.2e" %
          (k, sin, rel, oracle.sin_theta(w["U"][:, :k], Ug)), flush=True)
    assert sin <= 1e-6
    assert rel <= 1e-10


@pytest.fixture(scope="module")
def cfg2_oracle():
    """The 2048 x 200000 FP32 workload from the NumPy generator and the stored
    full oracle run on it (tests/golden, written by make_oracle_fixtures.py);
    skipped when the fixture is absent or was made from other bytes."""
    import sys
    sys.path.insert(0, os.path.join(HERE, "golden"))
    import make_oracle_fixtures as mk
    name = "planted-2048x200000-f32"
    path = mk.fixture_path(name, None)
    if not os.path.exists(path):
        pytest.skip("no stored oracle run for %s" % name)
    w = workloads.workload(name)
    z = np.load(path)
    if str(z["input_sha256"]) != mk.input_hash(w["Xt"]):
        pytest.skip("stored oracle run was made from other input bytes")
    return w, z


@pytest.mark.parametrize("precision", [0, 4])
def test_full_size_solve_against_oracle(torch_cuda, cfg2_oracle, precision):
    """A whole solve of the 2048 x 200000 FP32 workload (FP64 form, and
    matrix-core passes and steps) against the stored full oracle run: subspace
    sine <= 1e-6, Ritz values, the relative Frobenius error to 1e-8 and the
    (1 + eps) bound of Theorem "mainResult"."""
    import torch
    from paper_1607_02925_amd import lowrank
    from oracle.linalg import sin_theta
    w, z = cfg2_oracle
    Uo, tho = z["U"], z["theta"]
    Xt = torch.from_numpy(w["Xt"]).cuda()
    plan = lowrank.Plan(Xt, w["k"], w["p"], w["eps"], seed=w["solver_seed"], precision=precision)
    st, U, theta, rep = plan.solve()
    Ug = U.cpu().numpy()
    del plan, Xt
    torch.cuda.empty_cache()
    sin = sin_theta(Uo, Ug)
    # ||X - U U^T X||_F^2 = ||X||_F^2 - ||U^T X||_F^2 (U orthonormal); X X^T for X_k
    fro2, proj_g, proj_o = 0.0, 0.0, 0.0
    G = np.zeros((w["d"], w["d"]))
    for c0 in range(0, w["n"], CHUNK):
        Xc = host_columns_np(w["Xt"], c0, min(w["n"], c0 + CHUNK))
        fro2 += float(np.sum(Xc * Xc))
        proj_g += float(np.sum((Ug.T @ Xc) ** 2))
        proj_o += float(np.sum((Uo.T @ Xc) ** 2))
        G += Xc @ Xc.T
        del Xc
    e_g, e_o = np.sqrt(fro2 - proj_g), np.sqrt(fro2 - proj_o)
    lam = np.linalg.eigvalsh(G)[::-1]
    e_k = np.sqrt(max(fro2 - float(np.sum(lam[:w["k"]])), 0.0))
    print("full-size solve (precision %d): status %d outer %d/%d epochs %d/%d sin %.2e "
          "||X - PX||_F gpu %.10e oracle %.10e best %.10e" %
          (precision, st, rep["outer"], int(z["outer"]), rep["total_epochs"],
           int(np.sum(z["epochs"])), sin, e_g, e_o, e_k), flush=True)
    assert st == 0
    assert sin <= 1e-6
    np.testing.assert_allclose(theta, tho, rtol=1e-9)
    assert abs(e_g - e_o) <= 1e-8 * e_o
    assert e_g <= (1 + w["eps"]) * e_k


def host_columns_np(xt, c0, c1):
    """Columns c0..c1 of the NumPy-stored X (n x d rows) as a d x (c1 - c0) FP64 block."""
    return np.ascontiguousarray(xt[c0:c1].astype(np.float64).T)
