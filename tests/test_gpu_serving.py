"""Serving form on the GPU: requests of mixed shape and storage type solved
concurrently by the library's request server.

Each request's result must be bitwise the same alone (its own plan, nothing
else on the device) and in the mix (admitted by HBM budget among others that
run at the same time); a sample per storage type is checked against the CPU
oracle.  Requests follow the serving-trace recipe at reduced sizes so the
oracle finishes in seconds.
"""
import time

import numpy as np
import pytest

import oracle
import workloads
from workloads import serving

pytestmark = pytest.mark.gpu

# reduced-size requests: same spectrum recipe as the serving trace
REQS = [
    dict(d=256, n=6000, k=4, p=12, storage="f32"),
    dict(d=128, n=4096, k=1, p=6, storage="bf16"),
    dict(d=512, n=9000, k=9, p=17, storage="f32"),
    dict(d=256, n=5000, k=6, p=20, storage="bf16"),
    dict(d=64, n=4096, k=3, p=9, storage="f32"),
    dict(d=384, n=7000, k=12, p=24, storage="bf16"),
    dict(d=256, n=4500, k=2, p=8, storage="f32"),
    dict(d=192, n=6100, k=5, p=13, storage="bf16"),
]
for i, r in enumerate(REQS):
    r.update(id=i, eps=1e-4, data_seed=7000 + i, solver_seed=serving.SOLVER_SEED_BASE + 900 + i)


def _host(req):
    return serving.request_data(req)


def _device(xt):
    import torch
    t = torch.from_numpy(xt).to("cuda:0")
    return t.view(torch.bfloat16) if xt.dtype == np.uint16 else t


@pytest.fixture(scope="module")
def data():
    out = []
    for r in REQS:
        xt = _host(r)
        out.append((xt, _device(xt)))
    return out


@pytest.fixture(scope="module")
def alone(data):
    from paper_1607_02925_amd import lowrank
    res = []
    for r, (_xt, X) in zip(REQS, data):
        print("alone: request", r["id"], r, flush=True)
        plan = lowrank.Plan(X, r["k"], r["p"], r["eps"], seed=r["solver_seed"])
        st, U, theta, rep = plan.solve()
        res.append((st, U.clone(), theta, rep))
        plan.close()
    return res


def test_mix_is_bitwise_alone(data, alone):
    import torch
    from paper_1607_02925_amd import lowrank
    sizes = [lowrank.plan_bytes(X, r["k"], r["p"]) for r, (_x, X) in zip(REQS, data)]
    # room for the two largest at once: forces queueing behind the HBM budget
    budget = sum(sorted(sizes)[-2:]) + 4096
    srv = lowrank.Server(budget, slots=4)
    tickets = [srv.submit(X, r["k"], r["p"], r["eps"], seed=r["solver_seed"])
               for r, (_x, X) in zip(REQS, data)]
    outs = [srv.wait(t) for t in tickets]
    stats = srv.stats()
    srv.close()
    print("server stats:", stats, flush=True)
    assert stats["completed"] == len(REQS)
    assert stats["peak_bytes"] <= budget
    assert 2 <= stats["peak_running"] <= 4
    for r, a, o in zip(REQS, alone, outs):
        st, U, theta, rep, info = o
        assert st == a[0] == 0, (r, st, a[0])
        assert torch.equal(U, a[1]), r
        assert np.array_equal(theta, a[2]), r
        assert rep["outer"] == a[3]["outer"] and rep["total_epochs"] == a[3]["total_epochs"]
        assert info["t_submit"] <= info["t_admit"] <= info["t_done"]
        assert info["workspace_bytes"] == sizes[r["id"]]


def test_requests_against_oracle(data, alone):
    """Three requests per storage type against the FP64 oracle on the same
    stored X: subspace sine <= 1e-6 and Ritz values to 1e-10."""
    picked = {"f32": [], "bf16": []}
    for r in REQS:
        if len(picked[r["storage"]]) < 3:
            picked[r["storage"]].append(r)
    for st_name, rs in picked.items():
        for r in rs:
            xt = data[r["id"]][0]
            ref = oracle.solve(xt, r["storage"], r["k"], r["p"], r["eps"],
                               oracle.Options(seed=r["solver_seed"]))
            st, U, theta, rep = alone[r["id"]]
            sin = oracle.sin_theta(ref.U, U.cpu().numpy())
            print("request %d (%s): sin=%.2e outer gpu/oracle %d/%d" %
                  (r["id"], st_name, sin, rep["outer"], ref.schedule.outer), flush=True)
            assert st == 0
            assert sin <= 1e-6, (r, sin)
            np.testing.assert_allclose(theta, ref.theta, rtol=1e-10, atol=0)


def test_server_errors_and_polling(data):
    import torch
    from paper_1607_02925_amd import lowrank
    r0, X0 = REQS[0], data[0][1]
    need = lowrank.plan_bytes(X0, r0["k"], r0["p"])
    srv = lowrank.Server(need + 256, slots=2)
    # a request whose workspace alone exceeds the budget is refused at submit
    big = REQS[2]
    with pytest.raises(lowrank.LowRankError) as ei:
        srv.submit(data[2][1], big["k"], big["p"], big["eps"])
    assert ei.value.code == lowrank.LR_ENOMEM
    # a failing request reports its own status; the next one is unaffected
    bad = X0.clone()
    bad[17, 3] = float("nan")
    tb = srv.submit(bad, r0["k"], r0["p"], r0["eps"], seed=r0["solver_seed"])
    tg = srv.submit(X0, r0["k"], r0["p"], r0["eps"], seed=r0["solver_seed"])
    st_b = srv.wait(tb)[0]
    assert st_b == lowrank.LR_EINVAL
    deadline = time.time() + 60
    out = None
    while out is None and time.time() < deadline:
        out = srv.poll(tg)
        if out is None:
            time.sleep(0.002)
    assert out is not None and out[0] == 0
    with pytest.raises(lowrank.LowRankError):
        srv.poll(tg)          # ticket already collected
    srv.close()
    torch.cuda.synchronize()


def test_trace_mix_bitwise_alone():
    """A 64-request slice of the serving trace (its d, n, k, p and storage mix,
    with d capped at 1024 and n at 32768 to keep the test short), every other
    request in the matrix-core form: each result is bitwise the same solved
    alone and served by 8 slots with all 64 submitted at once, where at least
    four run together."""
    import torch
    from paper_1607_02925_amd import lowrank
    reqs = serving.trace(count=64, seed=11, d_choices=(256, 512, 1024), n_range=(4096, 32768))
    xs = [serving.request_data(r, device="cuda") for r in reqs]   # FP32 or BF16 tensors
    torch.cuda.synchronize()
    prec = [lowrank.LR_PREC_MC if i % 2 else 0 for i in range(len(reqs))]
    alone = []
    for r, X, pr in zip(reqs, xs, prec):
        plan = lowrank.Plan(X, r["k"], r["p"], r["eps"], seed=r["solver_seed"], precision=pr)
        st, U, theta, rep = plan.solve()
        plan.close()
        alone.append((st, U.clone(), theta, rep["outer"]))
    print("alone: %d solves, %d matrix-core" % (len(reqs), sum(1 for p_ in prec if p_)),
          flush=True)
    srv = lowrank.Server(1 << 31, slots=8)
    tickets = [srv.submit(X, r["k"], r["p"], r["eps"], seed=r["solver_seed"], precision=pr)
               for r, X, pr in zip(reqs, xs, prec)]
    outs = [srv.wait(t) for t in tickets]
    stats = srv.stats()
    srv.close()
    print("server stats:", stats, flush=True)
    assert stats["peak_running"] >= 4
    same = 0
    for r, a, o in zip(reqs, alone, outs):
        assert a[0] == o[0] == 0, (r, a[0], o[0])
        same += int(torch.equal(a[1], o[1]) and np.array_equal(a[2], o[2]) and
                    a[3] == o[3]["outer"])
    assert same == len(reqs), "%d of %d bitwise equal" % (same, len(reqs))
