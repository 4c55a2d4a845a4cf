"""Edge shapes of the dense inner solver in each step precision, against the
oracle: the largest minibatch (b = 8192, the plan's cap) with the largest block
(p = 64) on a ragged d, and the smallest shapes (d a few rows, inside one
partial 16-row tile; b below one 16-sample block).

Bars: FP64 steps 1e-10 relative (rounding order only); matrix-core steps a
small fraction of the correction W - W_0 the steps made (FP32 steps 1e-4, BF16
steps 1e-3), as in the precision-specific tests.
"""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

# (storage of X, precision of the steps)
FORMS = [("f64", 0), ("f32", 0), ("bf16", 0), ("bf16", 1), ("f32", 2), ("bf16", 2)]


def to_dev(torch, xt, storage):
    if storage == "bf16":
        return torch.from_numpy(np.ascontiguousarray(xt).view(np.int16)).cuda().view(
            torch.bfloat16)
    return torch.from_numpy(np.ascontiguousarray(xt)).cuda()


def _planted(d, n, seed, storage):
    i = np.arange(1, min(d, n) + 1, dtype=float)
    sig = np.where(i <= 2, 1.0, 0.6 * i ** -0.5)
    return workloads.planted_dense(d, n, sig, seed, storage)["Xt"]


def _check(torch_cuda, xt, storage, precision, k, p, b, m, epochs, seed):
    from paper_1607_02925_amd import lowrank
    X = oracle.decode(xt, storage)
    d, n = X.shape
    S = oracle.cholqr2(np.random.default_rng(seed).standard_normal((d, p)))[0]
    lam1 = np.linalg.eigvalsh(X @ X.T)[-1]
    lam = 1.1 * lam1
    fro2 = float(np.sum(X * X))
    eta = min(1.0 / lam, 0.1 * lam1 * b / (4.0 * fro2 * lam1))
    plan = lowrank.Plan(to_dev(torch_cuda, xt, storage), k, p, 1e-4, seed=seed,
                        precision=precision)
    plan.prepare()
    _, qc = oracle.build_table(oracle.column_sq_norms(X))
    Wg, res_g = plan.svrg_solve(torch_cuda.from_numpy(S).cuda(), lam, eta, m, b, 1, epochs)
    Wo, _, res_o = oracle.svrg_solve(X, qc, S, lam, eta, m, b, 0.0, seed, 1, 60,
                                     fixed_epochs=epochs)
    Wg = Wg.cpu().numpy()
    if precision == 0:
        err = np.linalg.norm(Wg - Wo) / np.linalg.norm(Wo)
        bar = 1e-10
        np.testing.assert_allclose(res_g, res_o, rtol=1e-7)
    else:
        W0 = oracle.svrg_solve(X, qc, S, lam, eta, m, b, 0.0, seed, 1, 60, fixed_epochs=0)[0]
        err = np.linalg.norm(Wg - Wo) / np.linalg.norm(Wo - W0)
        bar = 1e-3 if precision == 1 else 1e-4
        np.testing.assert_allclose(res_g, res_o, rtol=1e-2 if precision == 1 else 1e-3)
    print("%s precision %d d=%d n=%d p=%d b=%d m=%d: err %.2e (bar %.0e)" %
          (storage, precision, d, n, p, b, m, err, bar), flush=True)
    assert err <= bar


@pytest.mark.parametrize("storage,precision", FORMS)
def test_max_batch_max_block(torch_cuda, storage, precision):
    """b = 8192 samples (the largest minibatch) and p = 64 columns (the largest
    block) on d = 300 (not a multiple of 16 or 32), three steps, one epoch."""
    xt = _planted(300, 9000, 31, storage)
    _check(torch_cuda, xt, storage, precision, k=2, p=64, b=8192, m=3, epochs=1, seed=13)


@pytest.mark.parametrize("storage,precision", FORMS)
@pytest.mark.parametrize("d,n,p,b", [(5, 7, 2, 3), (11, 40, 3, 17), (17, 33, 9, 1)])
def test_tiny_shapes(torch_cuda, storage, precision, d, n, p, b):
    """d inside one partial 16-row tile (or just past it), b from 1 sample to
    just past one 16-sample block, p from 2 to 9: two epochs of 6 steps."""
    xt = _planted(d, n, 100 + d, storage)
    _check(torch_cuda, xt, storage, precision, k=1, p=p, b=b, m=6, epochs=2, seed=7)
