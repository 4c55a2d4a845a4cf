"""Reads of unwritten workspace, and results that depend on what else runs.

With lr_options.fill_workspace = 1 the library fills a plan's whole device
workspace with the byte 0xFF (a NaN in every floating-point type it uses)
before the first kernel.  A solve that read any workspace memory before
writing it would then change, so every form of the path must give bitwise the
same U_k and theta with and without the fill: dense FP64/FP32/BF16 storage,
the FP32 and BF16 matrix-core steps, the adaptive partitioning, the
accelerated inner solver, and (within the rounding of its atomic scatter)
compressed-column X.  Served requests run on arena slices that other requests
have used; a mixed trace of 24 requests on 8 slots, every one filled, must be
bitwise equal to the same requests solved alone.
"""
import numpy as np
import pytest

import oracle
import workloads
from workloads import serving, sparse

pytestmark = pytest.mark.gpu


def _dev(torch, xt):
    t = torch.from_numpy(np.ascontiguousarray(xt)).cuda()
    return t.view(torch.bfloat16) if xt.dtype == np.uint16 else t


def _solve_pair(torch, X, k, p, eps, **kw):
    from paper_1607_02925_amd import lowrank
    out = []
    for fill in (0, 1):
        plan = lowrank.Plan(X, k, p, eps, fill_workspace=fill, **kw)
        st, U, theta, rep = plan.solve()
        torch.cuda.synchronize()
        out.append((st, U.clone(), theta, rep))
        plan.close()
    return out


CASES = [
    ("planted-256x2048-f64", {}),
    ("planted-256x8192-f32", {}),
    ("planted-256x8192-f32", {"precision": 2}),
    ("planted-256x8192-f32", {"adaptive": 1}),
    ("planted-256x8192-f32", {"accel": 1}),
    ("planted-512x16384-bf16", {"precision": 1, "max_outer": 3}),
    ("planted-512x16384-bf16", {"precision": 2, "max_outer": 3}),
]


@pytest.mark.parametrize("name,kw", CASES)
def test_fill_does_not_change_dense_results(torch_cuda, name, kw):
    torch = torch_cuda
    w = workloads.workload(name)
    X = _dev(torch, w["Xt"])
    print("fill case", name, kw, flush=True)
    a, b = _solve_pair(torch, X, w["k"], w["p"], w["eps"], seed=w["solver_seed"], **kw)
    assert a[0] == b[0] and a[0] in (0, 4)
    assert torch.equal(a[1], b[1])
    assert np.array_equal(a[2], b[2])
    assert a[3]["total_epochs"] == b[3]["total_epochs"] and a[3]["outer"] == b[3]["outer"]


def test_fill_does_not_change_csc_results(torch_cuda):
    from paper_1607_02925_amd import lowrank
    torch = torch_cuda
    sp = sparse.zipf_csc(600, 5000, 16, seed=11, storage="csc-f32")
    X = lowrank.CscMatrix.from_arrays(sp["d"], sp["n"], sp["col_ptr"], sp["row_idx"],
                                      sp["values"])
    a, b = _solve_pair(torch, X, 2, 8, 1e-3, seed=7, max_outer=3)
    assert a[0] == b[0] and a[0] in (0, 4)
    # the inner-step scatter adds in a fixed order: bitwise equal
    assert torch.equal(a[1], b[1])
    assert np.array_equal(a[2], b[2])
    assert a[3]["total_epochs"] == b[3]["total_epochs"] and a[3]["outer"] == b[3]["outer"]


def _mixed_requests(count):
    rng = np.random.default_rng(2024)
    reqs = []
    for i in range(count):
        d = int(rng.choice([64, 128, 256, 384, 512]))
        n = int(rng.integers(4096, 12000))
        k = int(rng.integers(1, 9))
        p = min(k + int(rng.integers(4, 13)), d - 1)
        reqs.append(dict(id=i, d=d, n=n, k=k, p=p, eps=1e-4,
                         storage="f32" if i % 2 == 0 else "bf16", data_seed=9100 + i,
                         solver_seed=serving.SOLVER_SEED_BASE + 5000 + i))
    return reqs


def test_served_mix_bitwise_equal_alone_with_fill(torch_cuda):
    """24 requests of mixed shape and storage type, 8 slots, a budget that
    holds about half of them at once; each request's workspace is filled with
    NaN bytes when admitted.  Each result is bitwise the one its own plan
    gives alone without the fill, and the matrix-core step forms agree the
    same way."""
    from paper_1607_02925_amd import lowrank
    torch = torch_cuda
    reqs = _mixed_requests(24)
    X = [_dev(torch, serving.request_data(r)) for r in reqs]
    torch.cuda.synchronize()
    for prec_of in (lambda x: 0, lambda x: 1 if x.dtype == torch.bfloat16 else 2):
        alone = []
        for r, x in zip(reqs, X):
            plan = lowrank.Plan(x, r["k"], r["p"], r["eps"], seed=r["solver_seed"],
                                precision=prec_of(x))
            st, U, theta, rep = plan.solve()
            alone.append((st, U.clone(), theta))
            plan.close()
        sizes = [lowrank.plan_bytes(x, r["k"], r["p"], precision=prec_of(x))
                 for r, x in zip(reqs, X)]
        budget = sum(sorted(sizes)[-12:])
        srv = lowrank.Server(budget, slots=8)
        tickets = [srv.submit(x, r["k"], r["p"], r["eps"], seed=r["solver_seed"],
                              precision=prec_of(x), fill_workspace=1)
                   for r, x in zip(reqs, X)]
        outs = [srv.wait(t) for t in tickets]
        stats = srv.stats()
        srv.close()
        print("mix stats:", stats, flush=True)
        assert stats["peak_running"] >= 4
        for r, a, o in zip(reqs, alone, outs):
            assert o[0] == a[0] == 0, (r, o[0], a[0])
            assert torch.equal(o[1], a[1]), r
            assert np.array_equal(o[2], a[2]), r
