"""The accelerated inner solver (lr_options.accel = 1) on the GPU against the
oracle's accel module: one solve with a fixed number of outer steps, and whole
solves (dense q = k, adaptive, compressed-column) taking the oracle's
decisions."""
import numpy as np
import pytest

import oracle
import workloads
from oracle.linalg import sin_theta
from workloads import sparse

pytestmark = pytest.mark.gpu


def to_dev(torch, xt, storage):
    if storage == "bf16":
        return torch.from_numpy(np.ascontiguousarray(xt).view(np.int16)).cuda().view(
            torch.bfloat16)
    return torch.from_numpy(np.ascontiguousarray(xt)).cuda()


def _problem(storage):
    d, n, p = 70, 1500, 6
    sig = np.concatenate([[3.0, 2.9, 2.3], np.linspace(1.2, 0.05, d - 3)])
    rng = np.random.default_rng(17)
    U = np.linalg.qr(rng.standard_normal((d, d)))[0]
    V = np.linalg.qr(rng.standard_normal((n, d)))[0]
    xt = (V * sig) @ U.T
    if storage == "f32":
        xt = xt.astype(np.float32)
    elif storage == "bf16":
        xt = workloads.f64_to_bf16_bits(xt)
    S = oracle.cholqr2(rng.standard_normal((d, p)))[0]
    return xt, S, p


@pytest.mark.parametrize("storage,precision", [("f64", 0), ("f32", 0), ("bf16", 0),
                                               ("bf16", 1), ("f32", 2), ("bf16", 2)])
def test_acc_solve_fixed_outer_steps(torch_cuda, storage, precision):
    """Three outer steps from the same warm start: iterate and the residuals
    of the original system agree with the oracle within rounding."""
    from paper_1607_02925_amd import lowrank
    torch = torch_cuda
    xt, S, p = _problem(storage)
    X = oracle.decode(xt, storage)
    plan = lowrank.Plan(to_dev(torch, xt, storage), 2, p, 1e-4, seed=31, accel=1,
                        precision=precision)
    plan.prepare()
    w = oracle.column_sq_norms(X)
    _, qc = oracle.build_table(w)
    lam1 = np.linalg.norm(X, 2) ** 2
    lam, mu = 1.01 * lam1, 0.01 * lam1
    kappa, beta, b, eta, m = oracle.accel_constants(w.sum(), lam1, lam, mu, X.shape[1])
    assert kappa > 0
    print("storage %s precision %d kappa %.3e beta %.3f b %d m %d" %
          (storage, precision, kappa, beta, b, m), flush=True)
    Wg, res_g = plan.acc_svrg_solve(torch.from_numpy(S).cuda(), lam, kappa, beta, eta, m, b, 5, 3)
    Wo, e, res_o = oracle.acc_svrg_solve(X, qc, S, lam, kappa, beta, eta, m, b, 0.0, 31, 5, 60,
                                         fixed_epochs=3)
    Wg = Wg.cpu().numpy()
    if precision == 0:
        assert np.linalg.norm(Wg - Wo) <= 1e-10 * np.linalg.norm(Wo)
        np.testing.assert_allclose(res_g, res_o, rtol=1e-7)
    else:
        # the BF16 step form rounds the step operands to hi/lo BF16 pairs, the
        # FP32 form to FP32: each differs by a small fraction of the correction
        # W - W_0 the steps made
        W0 = oracle.acc_svrg_solve(X, qc, S, lam, kappa, beta, eta, m, b, 0.0, 31, 5, 60,
                                   fixed_epochs=0)[0]
        err = np.linalg.norm(Wg - Wo) / np.linalg.norm(Wo - W0)
        print("|W - W_oracle| / |W - W_0| = %.2e" % err, flush=True)
        assert err <= (1e-3 if precision == 1 else 1e-4)
        np.testing.assert_allclose(res_g, res_o, rtol=1e-2)
    assert res_o[-1] < 0.8 * res_o[0]


def test_kappa_zero_matches_plain_op(torch_cuda):
    from paper_1607_02925_amd import lowrank
    torch = torch_cuda
    xt, S, p = _problem("f64")
    X = oracle.decode(xt, "f64")
    plan = lowrank.Plan(to_dev(torch, xt, "f64"), 2, p, 1e-4, seed=31, accel=1)
    plan.prepare()
    w = oracle.column_sq_norms(X)
    lam1 = np.linalg.norm(X, 2) ** 2
    b, eta, m = oracle.solver_constants(w.sum(), lam1, 1.05 * lam1, 0.05 * lam1, X.shape[1],
                                        batch=128)
    Sd = torch.from_numpy(S).cuda()
    Wa, ra = plan.acc_svrg_solve(Sd, 1.05 * lam1, 0.0, 0.0, eta, m, b, 2, 3)
    Wp, rp = plan.svrg_solve(Sd, 1.05 * lam1, eta, m, b, 2, 3)
    assert torch.equal(Wa, Wp)
    np.testing.assert_array_equal(ra, rp)


def test_accel_solve_matches_oracle(torch_cuda):
    """q = k branch with the accelerated solver: the same kappa, beta, b, m,
    outer iterations and outer steps per solve; the same subspace."""
    from paper_1607_02925_amd import lowrank
    w = workloads.workload("planted-256x2048-f64")
    ref = oracle.solve(w["Xt"], w["storage"], w["k"], w["p"], w["eps"],
                       oracle.Options(seed=w["solver_seed"], accel=True))
    plan = lowrank.Plan(to_dev(torch_cuda, w["Xt"], w["storage"]), w["k"], w["p"], w["eps"],
                        seed=w["solver_seed"], accel=1)
    st, U, theta, rep = plan.solve()
    sc, rs = plan.schedule(), ref.schedule
    print("gpu b %d m %d outer %d epochs %s; oracle b %d m %d outer %d epochs %s" %
          (sc.b, sc.m, sc.outer, sc.epochs, rs.b, rs.m, rs.outer, rs.epochs), flush=True)
    assert st == ref.status == 0
    assert rep["shift_rounds"] == ref.shift_rounds
    assert (sc.b, sc.m, sc.outer) == (rs.b, rs.m, rs.outer)
    assert sc.epochs == rs.epochs
    assert rep["accel_kappa"] == pytest.approx(rs.kappa, rel=1e-9)
    assert rep["accel_beta"] == pytest.approx(rs.beta, rel=1e-9)
    Ug = U.cpu().numpy()
    assert sin_theta(ref.U, Ug) <= 1e-6
    assert sin_theta(w["U"][:, :w["k"]], Ug) < 1e-8
    np.testing.assert_allclose(theta, ref.theta, rtol=1e-10)


def test_accel_adaptive_matches_oracle(torch_cuda):
    from paper_1607_02925_amd import lowrank
    w = workloads.workload("planted-256x8192-f32")
    ref = oracle.solve_adaptive(w["Xt"], w["storage"], w["k"], w["p"], w["eps"],
                                oracle.Options(seed=w["solver_seed"], accel=True))
    plan = lowrank.Plan(to_dev(torch_cuda, w["Xt"], w["storage"]), w["k"], w["p"], w["eps"],
                        seed=w["solver_seed"], adaptive=1, accel=1)
    st, U, theta, rep = plan.solve()
    got = [(iv["s"], iv["q"], iv["branch"], iv["cols"], iv["iters"]) for iv in rep["intervals"]]
    want = [(iv.s, iv.q, iv.branch, iv.cols, iv.iterations) for iv in ref.intervals]
    print("intervals gpu %s oracle %s" % (got, want), flush=True)
    assert st == ref.status == 0
    assert got == want
    assert sin_theta(ref.U, U.cpu().numpy()) <= 1e-6
    np.testing.assert_allclose(theta, ref.theta, rtol=1e-9)


def test_accel_sparse_matches_oracle(torch_cuda):
    from paper_1607_02925_amd import lowrank
    sp = sparse.zipf_csc(600, 5000, 16, seed=11)
    k, p, eps = 1, 4, 1e-4
    ref = oracle.solve(sp, "csc-f32", k, p, eps, oracle.Options(seed=7, accel=True))
    X = lowrank.CscMatrix.from_arrays(sp["d"], sp["n"], sp["col_ptr"], sp["row_idx"],
                                      sp["values"])
    pl = lowrank.Plan(X, k, p, eps, seed=7, accel=1)
    st, U, theta, rep = pl.solve()
    print("epochs gpu %s oracle %s" % (pl.schedule().epochs, ref.schedule.epochs), flush=True)
    assert st == ref.status == 0
    assert pl.schedule().epochs == ref.schedule.epochs
    assert sin_theta(ref.U, U.cpu().numpy()) <= 1e-6
    np.testing.assert_allclose(theta, ref.theta, rtol=1e-9)


def test_accel_option_checks(torch_cuda):
    from paper_1607_02925_amd import lowrank
    xt, S, p = _problem("f64")
    X = to_dev(torch_cuda, xt, "f64")
    for kw in ({"accel": 2}, {"accel": 1, "replay": lowrank.Schedule(1.0, 0.1, 1e-3, 4, 64, 0, 1,
                                                                       [1])}):
        with pytest.raises(lowrank.LowRankError) as e:
            lowrank.Plan(X, 2, p, 1e-4, **kw)
        assert e.value.code == lowrank.LR_EINVAL
    plan = lowrank.Plan(X, 2, p, 1e-4)
    plan.prepare()
    with pytest.raises(lowrank.LowRankError) as e:   # the plan has no momentum buffers
        plan.acc_svrg_solve(torch_cuda.from_numpy(S).cuda(), 10.0, 1.0, 0.5, 1e-3, 4, 64, 0, 1)
    assert e.value.code == lowrank.LR_EINVAL
