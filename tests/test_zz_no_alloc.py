"""lowrank_solve_noalloc (no device allocation; workspace in the library's fixed
device array) against lowrank_plan + lowrank_solve on the same inputs.

Both run the same kernels in the same order and neither depends on what its
workspace held before, so U_k and the Ritz values must be bitwise equal.  Two
calls in a row, the second on a smaller problem, so the second reads an array
the first left dirty.
"""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

CASES = ["planted-256x8192-f32", "planted-256x2048-f64"]   # second one smaller


def _dev(xt):
    import torch
    t = torch.from_numpy(xt).to("cuda:0")
    return t.view(torch.bfloat16) if xt.dtype == np.uint16 else t


def test_noalloc_equals_plan_solve_twice(torch_cuda):
    import torch
    from paper_1607_02925_amd import lowrank
    for name in CASES:
        w = workloads.workload(name)
        X = _dev(w["Xt"])
        need = lowrank.plan_bytes(X, w["k"], w["p"])
        print("noalloc case", name, "workspace bytes", need, flush=True)
        assert need <= lowrank.NOALLOC_MAX_BYTES
        st_a, U_a, th_a, rep_a = lowrank.solve_noalloc(X, w["k"], w["p"], w["eps"],
                                                       seed=w["solver_seed"])
        plan = lowrank.Plan(X, w["k"], w["p"], w["eps"], seed=w["solver_seed"])
        st_b, U_b, th_b, rep_b = plan.solve()
        plan.close()
        torch.cuda.synchronize()
        assert st_a == st_b == 0, (name, st_a, st_b)
        assert torch.equal(U_a, U_b), name
        assert np.array_equal(th_a, th_b), name
        assert rep_a["outer"] == rep_b["outer"]
        assert rep_a["total_epochs"] == rep_b["total_epochs"]


def test_noalloc_rejections(torch_cuda):
    """Sizes beyond the fixed array and compressed-column X are refused before
    anything runs."""
    import torch
    from paper_1607_02925_amd import lowrank
    # 4096 x 40000 f32 with p = 32: the n x 32 FP64 block alone is 10 MB, the
    # whole workspace over 64 MiB
    X = torch.zeros((300000, 64), dtype=torch.float32, device="cuda:0")
    need = lowrank.plan_bytes(X, 4, 32)
    assert need > lowrank.NOALLOC_MAX_BYTES
    with pytest.raises(lowrank.LowRankError) as e:
        lowrank.solve_noalloc(X, 4, 32, 1e-4)
    assert e.value.code == lowrank.LR_ENOMEM
