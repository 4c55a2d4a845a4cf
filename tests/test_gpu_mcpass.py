"""Matrix-core full-gradient passes (precision LR_PREC_MC_PASS / LR_PREC_MC)
against the FP64 oracle, for dense FP32 and BF16 X.

Error model of one pass Y = X (X^T W).  W and T = X^T W are carried as three
BF16 parts (relative residue below 2^-24); FP32 X is split exactly, BF16 X is
exact.  The matrix cores accumulate in FP32 over at most 256 terms before the
sum is added into FP64, so each partial sum carries at most 256 * 2^-24 of the
sum of its terms' magnitudes.  With both halves of the pass the elementwise
error is below about 3e-5 (|X| (|X|^T |W|)) in the worst case and around 1e-6
of it in practice; the bound asserted is 2e-5.

Whole solves: the passes of the shift-and-invert solves run on matrix cores,
everything that decides the schedule (estimate phase, shift tuning) and the
final Rayleigh-Ritz stay FP64.  Bars: sin <= 1e-6 against the oracle for FP32
X, <= 1e-3 for BF16 X (the per-path tolerances of the method's parity
requirement), Ritz values to 1e-8 relative.
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


# d and n off the 32-row, 128-row and 256-column tiles, p off and on the
# 16-column slices, up to the 64-column maximum
SHAPES = [(200, 1000, 20, "f32"), (256, 4133, 48, "bf16"), (520, 3000, 64, "f32"),
          (64, 50, 3, "bf16"), (1000, 7001, 16, "f32"), (136, 2050, 33, "bf16"),
          (2048, 9000, 20, "f32"), (4096, 2000, 48, "bf16")]


@pytest.mark.parametrize("d,n,p,storage", SHAPES)
def test_mc_apply_A_elementwise(torch_cuda, d, n, p, storage):
    from paper_1607_02925_amd import lowrank
    torch = torch_cuda
    print("mc apply_A", d, n, p, storage, flush=True)
    xt = planted(d, n, 4, 300 + d + n, storage)
    X = oracle.decode(xt, storage)
    W = np.random.default_rng(d * 7 + p).standard_normal((d, p))
    plan = lowrank.Plan(to_dev(torch, xt, storage), 1, p if p < d else d - 1, 1e-4,
                        precision=lowrank.LR_PREC_MC_PASS)
    Yg = plan.apply_A(torch.from_numpy(W).cuda()).cpu().numpy()
    Yo = oracle.apply_A(X, W)
    bound = np.abs(X) @ (np.abs(X).T @ np.abs(W))
    err = np.abs(Yg - Yo)
    assert np.all(np.isfinite(Yg))
    assert np.all(err <= 2e-5 * bound + 1e-300), float(np.max(err / bound))
    rel = np.linalg.norm(Yg - Yo) / np.linalg.norm(Yo)
    print("  max err/bound %.2e  relative Frobenius %.2e" % (np.max(err / bound), rel),
          flush=True)
    assert rel <= 1e-6


def test_mc_rejects_fp64_x(torch_cuda):
    from paper_1607_02925_amd import lowrank
    torch = torch_cuda
    X = torch.zeros((300, 64), dtype=torch.float64, device="cuda")
    for prec in (lowrank.LR_PREC_MC_PASS, lowrank.LR_PREC_MC):
        with pytest.raises(lowrank.LowRankError) as e:
            lowrank.Plan(X, 2, 8, 1e-4, precision=prec)
        assert e.value.code == lowrank.LR_EINVAL


@pytest.mark.parametrize("prec", ["MC_PASS", "MC"])
def test_mc_solve_f32_against_oracle(torch_cuda, prec):
    """The 256 x 8192 FP32 geometric-spectrum workload (k = 10, p = 20) solved
    with matrix-core passes against the stored full oracle run."""
    import test_gpu_parity as tp
    from paper_1607_02925_amd import lowrank
    torch = torch_cuda
    w, Uo, tho, sched, _ = tp._fixture_or_oracle("planted-256x8192-f32", None)
    plan = lowrank.Plan(to_dev(torch, w["Xt"], "f32"), w["k"], w["p"], w["eps"],
                        seed=w["solver_seed"], precision=getattr(lowrank, "LR_PREC_" + prec))
    st, U, theta, rep = plan.solve()
    sin = sin_theta(Uo, U.cpu().numpy())
    print("mc f32 %s: status %d outer %d/%d epochs %d (oracle %d) mc passes %d/%d sin %.2e" %
          (prec, st, rep["outer"], sched.outer, rep["total_epochs"], sum(sched.epochs),
           rep["mc_passes"], rep["passes"], sin), flush=True)
    assert st == 0
    assert rep["mc_passes"] > 0
    assert sin <= 1e-6, sin
    np.testing.assert_allclose(theta, tho, rtol=1e-8)


@pytest.mark.parametrize("prec", ["MC_PASS", "MC"])
def test_mc_solve_bf16_against_oracle(torch_cuda, prec):
    """A clustered-spectrum BF16 X (256 x 8192, k = 4, p = 12) solved with
    matrix-core passes against a live oracle run."""
    from paper_1607_02925_amd import lowrank
    torch = torch_cuda
    xt = planted(256, 8192, 4, 123, "bf16")
    ref = oracle.solve(xt, "bf16", 4, 12, 1e-4, oracle.Options(seed=9))
    plan = lowrank.Plan(to_dev(torch, xt, "bf16"), 4, 12, 1e-4, seed=9,
                        precision=getattr(lowrank, "LR_PREC_" + prec))
    st, U, theta, rep = plan.solve()
    sin = sin_theta(ref.U, U.cpu().numpy())
    print("mc bf16 %s: status %d outer %d/%d mc passes %d/%d sin %.2e" %
          (prec, st, rep["outer"], ref.schedule.outer, rep["mc_passes"], rep["passes"], sin),
          flush=True)
    assert st == 0
    assert rep["mc_passes"] > 0
    assert sin <= 1e-3, sin
    np.testing.assert_allclose(theta, ref.theta, rtol=1e-6)


def test_mc_powerlaw_prefix_replay(torch_cuda):
    """k = 32, p = 48 on the oracle-sized power-law BF16 workload, replaying the
    oracle's schedule for three outer iterations with matrix-core passes and
    steps."""
    import test_gpu_parity as tp
    from paper_1607_02925_amd import lowrank
    torch = torch_cuda
    w, Uo, tho, sched, _ = tp._fixture_or_oracle("planted-512x16384-bf16", 3)
    plan = lowrank.Plan(to_dev(torch, w["Xt"], "bf16"), w["k"], w["p"], w["eps"],
                        seed=w["solver_seed"], replay=sched, precision=lowrank.LR_PREC_MC)
    st, U, theta, rep = plan.solve()
    sin = sin_theta(Uo, U.cpu().numpy())
    print("mc power-law bf16 replay prefix: sin=%.2e mc passes %d/%d" %
          (sin, rep["mc_passes"], rep["passes"]), flush=True)
    assert st == 0
    assert sin <= 1e-3
    np.testing.assert_allclose(theta, tho, rtol=1e-5)


def test_mc_served_bitwise_alone(torch_cuda):
    """Matrix-core-form requests (LR_PREC_MC) of mixed shapes and storage types
    are bitwise the same solved alone and served concurrently in a mix: the
    pass kernels reduce in a fixed order and each request has its own
    workspace."""
    from paper_1607_02925_amd import lowrank
    torch = torch_cuda
    shapes = [(256, 6000, 3, "f32"), (512, 5000, 6, "bf16"), (192, 7000, 2, "f32"),
              (384, 4500, 5, "bf16"), (1024, 9000, 8, "f32"), (136, 4100, 4, "bf16")]
    xs = [to_dev(torch, planted(d, n, k, 900 + d, st), st) for d, n, k, st in shapes]
    ks = [k for _, _, k, _ in shapes]
    alone = []
    for X, k in zip(xs, ks):
        st, U, th, rep = lowrank.Plan(X, k, k + 8, 1e-4, seed=5,
                                      precision=lowrank.LR_PREC_MC).solve()
        assert st == 0 and rep["mc_passes"] > 0
        alone.append((st, U.clone(), th))
    srv = lowrank.Server(1 << 30, slots=4)
    tickets = [srv.submit(X, k, k + 8, 1e-4, seed=5, precision=lowrank.LR_PREC_MC)
               for X, k in zip(xs, ks)]
    outs = [srv.wait(t) for t in tickets]
    stats = srv.stats()
    srv.close()
    assert stats["peak_running"] >= 2
    for a, o in zip(alone, outs):
        assert a[0] == o[0] == 0
        assert torch.equal(a[1], o[1])
        assert np.array_equal(a[2], o[2])
