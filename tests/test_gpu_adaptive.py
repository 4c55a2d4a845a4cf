"""Adaptive partitioning (lr_options.adaptive = 1) on the GPU against the
oracle's adaptive module: the same intervals, branches and iteration counts,
and the same subspace within rounding."""
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


@pytest.mark.parametrize("name", ["planted-256x8192-f32"])
def test_adaptive_matches_oracle(torch_cuda, name):
    """Geometric top spectrum: plain subspace iteration for 1..9, then
    shift-and-invert for 10 on the deflated operator."""
    from paper_1607_02925_amd import lowrank
    w = workloads.workload(name)
    ref = oracle.solve_adaptive(w["Xt"], w["storage"], w["k"], w["p"], w["eps"],
                                oracle.Options(seed=w["solver_seed"]))
    plan = lowrank.Plan(to_dev(torch_cuda, w["Xt"], w["storage"]), w["k"], w["p"], w["eps"],
                        seed=w["solver_seed"], adaptive=1)
    st, U, theta, rep = plan.solve()
    got = [(iv["s"], iv["q"], iv["branch"], iv["cols"], iv["iters"]) for iv in rep["intervals"]]
    want = [(iv.s, iv.q, iv.branch, iv.cols, iv.iterations) for iv in ref.intervals]
    sin = sin_theta(ref.U, U.cpu().numpy())
    print("intervals gpu %s oracle %s sin %.2e" % (got, want, sin), flush=True)
    assert st == ref.status == 0
    assert got == want
    assert sin <= 1e-6
    np.testing.assert_allclose(theta, ref.theta, rtol=1e-9)


def test_adaptive_single_interval_equals_q_equals_k(torch_cuda):
    """Clustered top spectrum: one shift-and-invert interval with
    oversampling, the q = k branch itself."""
    from paper_1607_02925_amd import lowrank
    w = workloads.workload("planted-256x2048-f64")
    X = to_dev(torch_cuda, w["Xt"], w["storage"])
    st0, U0, th0, rep0 = lowrank.Plan(X, w["k"], w["p"], w["eps"], seed=w["solver_seed"]).solve()
    st1, U1, th1, rep1 = lowrank.Plan(X, w["k"], w["p"], w["eps"], seed=w["solver_seed"],
                                      adaptive=1).solve()
    assert st0 == st1 == 0
    assert [(iv["s"], iv["q"], iv["branch"]) for iv in rep1["intervals"]] == \
        [(1, w["k"], "shift-invert")]
    assert rep1["outer"] == rep0["outer"]
    assert sin_theta(U0.cpu().numpy(), U1.cpu().numpy()) <= 1e-12
    np.testing.assert_allclose(th1, th0, rtol=1e-12)


def test_adaptive_option_checks(torch_cuda):
    from paper_1607_02925_amd import lowrank
    xt = workloads.planted_dense(100, 400, np.linspace(2, 0.1, 100), 3, "bf16")["Xt"]
    with pytest.raises(lowrank.LowRankError) as e:
        lowrank.Plan(to_dev(torch_cuda, xt, "bf16"), 2, 6, 1e-4, adaptive=1, precision=1)
    assert e.value.code == lowrank.LR_EINVAL


@pytest.mark.parametrize("name,adaptive", [("planted-256x2048-f64", 0),
                                           ("planted-256x8192-f32", 1)])
def test_spectral_norm_option(torch_cuda, name, adaptive):
    """norm = 1 rescales eps by sqrt(theta_1 / theta_{k+1}); the GPU takes the
    oracle's decisions and reaches its subspace."""
    from paper_1607_02925_amd import lowrank
    w = workloads.workload(name)
    opt = oracle.Options(seed=w["solver_seed"], norm="spectral")
    fn = oracle.solve_adaptive if adaptive else oracle.solve
    ref = fn(w["Xt"], w["storage"], w["k"], w["p"], w["eps"], opt)
    plan = lowrank.Plan(to_dev(torch_cuda, w["Xt"], w["storage"]), w["k"], w["p"], w["eps"],
                        seed=w["solver_seed"], adaptive=adaptive, norm=1)
    st, U, theta, rep = plan.solve()
    assert st == ref.status == 0
    assert sin_theta(ref.U, U.cpu().numpy()) <= 1e-6
    np.testing.assert_allclose(theta, ref.theta, rtol=1e-9)
