"""FP32 matrix-core inner steps (precision LR_PREC_F32_STEPS) against the FP64
oracle, for dense FP32 and BF16 X.

The steps round the step difference to FP32 (relative 2^-24) and accumulate
each wave's share of a product in FP32 (a few hundred terms, relative error
about sqrt(terms) 2^-24 < 1e-6 of the sum of magnitudes); the waves' partial
sums, the FP64 master copy of the difference and everything outside the steps
stay FP64.  Each epoch restarts from an exactly computed residual, so an inner
solve's result differs from the oracle's by about 1e-6 of the correction the
steps made (bound used: 1e-4), and whole solves reach the oracle's subspace to
within the FP64 tolerances of the other solve tests, widened tenfold.
"""
import numpy as np
import pytest

import oracle
import workloads
from oracle.linalg import sin_theta

pytestmark = pytest.mark.gpu


def to_dev(torch, xt, storage):
    if storage == "bf16":
        return torch.from_numpy(np.ascontiguousarray(xt).view(np.int16)).cuda().view(
            torch.bfloat16)
    return torch.from_numpy(np.ascontiguousarray(xt)).cuda()


def planted(d, n, k, seed, storage):
    i = np.arange(1, min(d, n) + 1, dtype=float)
    sig = np.where(i <= k, 1.0, 0.7 * i ** -0.5)
    return workloads.planted_dense(d, n, sig, seed, storage)["Xt"]


@pytest.mark.parametrize("d,n,p,b,storage", [(256, 8192, 12, 512, "f32"),
                                             (130, 3001, 9, 256, "bf16"),
                                             (520, 6000, 48, 1024, "f32"),
                                             (333, 4097, 64, 300, "bf16"),
                                             (47, 900, 3, 33, "f32")])
def test_inner_solve_against_oracle(torch_cuda, d, n, p, b, storage):
    """Fixed epochs of the inner solver on ragged shapes (d, b and p off the
    16-tiles): the FP32-step result differs from the oracle by a small fraction
    of the correction W - W_0 the steps computed; the residuals, computed by
    FP64 passes, agree closely."""
    from paper_1607_02925_amd import lowrank
    torch = torch_cuda
    xt = planted(d, n, 4, 60 + d, storage)
    X = oracle.decode(xt, storage)
    S = oracle.cholqr2(np.random.default_rng(d).standard_normal((d, p)))[0]
    lam1 = np.linalg.eigvalsh(X @ X.T)[-1]
    lam, mu = 1.1 * lam1, 0.1 * lam1
    fro2 = float(np.sum(X * X))
    b, eta, m = oracle.solver_constants(fro2, lam1, lam, mu, n, batch=b)
    m = min(m, 24)
    plan = lowrank.Plan(to_dev(torch, xt, storage), 2, p, 1e-4, seed=77,
                        precision=lowrank.LR_PREC_F32_STEPS)
    plan.prepare()
    _, qc = oracle.build_table(oracle.column_sq_norms(X))
    Wg, res_g = plan.svrg_solve(torch.from_numpy(S).cuda(), lam, eta, m, b, 3, 2)
    Wo, _, res_o = oracle.svrg_solve(X, qc, S, lam, eta, m, b, 0.0, 77, 3, 60, fixed_epochs=2)
    W0, _, _ = oracle.svrg_solve(X, qc, S, lam, eta, m, b, 0.0, 77, 3, 60, fixed_epochs=0)
    Wg = Wg.cpu().numpy()
    err = np.linalg.norm(Wg - Wo) / np.linalg.norm(Wo - W0)
    print("%s d=%d p=%d b=%d m=%d: |W_f32 - W_oracle| / |W - W_0| = %.2e, residuals %s vs %s" %
          (storage, d, p, b, m, err, np.array(res_g), np.array(res_o)), flush=True)
    assert err <= 1e-4
    np.testing.assert_allclose(res_g, res_o, rtol=1e-3)
    assert res_o[-1] < res_o[0]


def test_solve_auto_f32(torch_cuda):
    """A whole solve (shift tuning, stopping rules) with FP32 steps on FP32 X:
    the oracle's subspace and Ritz values."""
    from paper_1607_02925_amd import lowrank
    w = workloads.workload("planted-256x8192-f32")
    ref = oracle.solve(w["Xt"], w["storage"], w["k"], w["p"], w["eps"],
                       oracle.Options(seed=w["solver_seed"]))
    plan = lowrank.Plan(to_dev(torch_cuda, w["Xt"], w["storage"]), w["k"], w["p"], w["eps"],
                        seed=w["solver_seed"], precision=lowrank.LR_PREC_F32_STEPS)
    st, U, theta, rep = plan.solve()
    Ug = U.cpu().numpy()
    sin = sin_theta(ref.U, Ug)
    print("f32 steps auto: sin=%.2e outer %d/%d epochs %s / %s" %
          (sin, rep["outer"], ref.schedule.outer, plan.schedule().epochs, ref.schedule.epochs),
          flush=True)
    assert st == ref.status == 0
    assert sin <= 1e-5
    np.testing.assert_allclose(theta, ref.theta, rtol=1e-8)


def test_powerlaw_prefix_replay_bf16(torch_cuda):
    """k = 32, p = 48 on the oracle-sized power-law BF16 workload, replaying
    the oracle's schedule for three outer iterations."""
    import test_gpu_parity as tp
    from paper_1607_02925_amd import lowrank
    torch = torch_cuda
    w, Uo, tho, sched, _ = tp._fixture_or_oracle("planted-512x16384-bf16", 3)
    plan = lowrank.Plan(to_dev(torch, w["Xt"], "bf16"), w["k"], w["p"], w["eps"],
                        seed=w["solver_seed"], replay=sched,
                        precision=lowrank.LR_PREC_F32_STEPS)
    st, U, theta, _ = plan.solve()
    sin = sin_theta(Uo, U.cpu().numpy())
    print("power-law f32 steps replay prefix: sin=%.2e" % sin, flush=True)
    assert st == 0
    assert sin <= 1e-5
    np.testing.assert_allclose(theta, tho, rtol=1e-8)


def test_deterministic_repeat(torch_cuda):
    """The FP32-step kernels reduce in a fixed order: two solves of one plan
    are bitwise equal."""
    from paper_1607_02925_amd import lowrank
    torch = torch_cuda
    X = to_dev(torch, planted(384, 5000, 5, 321, "f32"), "f32")
    plan = lowrank.Plan(X, 5, 13, 1e-4, seed=5, precision=lowrank.LR_PREC_F32_STEPS)
    a = plan.solve()
    b = plan.solve()
    assert a[0] == b[0] == 0
    assert torch.equal(a[1], b[1])
    assert np.array_equal(a[2], b[2])


def test_served_bitwise_alone(torch_cuda):
    """FP32-step requests of mixed shapes and storage are bitwise the same alone
    and in a mix through the server (fixed-order reductions, per-request
    workspaces)."""
    from paper_1607_02925_amd import lowrank
    torch = torch_cuda
    specs = [(256, 6000, 3, "f32"), (512, 5000, 6, "bf16"), (192, 7000, 2, "f32"),
             (384, 4500, 5, "bf16")]
    xs = [to_dev(torch, planted(d, n, k, 700 + d, st), st) for d, n, k, st in specs]
    ks = [k for _, _, k, _ in specs]
    alone = []
    for X, k in zip(xs, ks):
        st, U, th, _ = lowrank.Plan(X, k, k + 8, 1e-4, seed=5,
                                    precision=lowrank.LR_PREC_F32_STEPS).solve()
        alone.append((st, U.clone(), th))
    srv = lowrank.Server(1 << 30, slots=4)
    tickets = [srv.submit(X, k, k + 8, 1e-4, seed=5, precision=lowrank.LR_PREC_F32_STEPS)
               for X, k in zip(xs, ks)]
    outs = [srv.wait(t) for t in tickets]
    srv.close()
    for a, o in zip(alone, outs):
        assert a[0] == o[0] == 0
        assert torch.equal(a[1], o[1])
        assert np.array_equal(a[2], o[2])
