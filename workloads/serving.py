"""Request traces for the serving form: many independent low-rank problems of
mixed shape and storage type arriving as a Poisson process.

Recipe of the default trace (512 requests): inter-arrival gaps Exp(mean 1/rate)
from NumPy PCG64 seed 5; per request r, d uniform over {256, 512, 1024, 2048,
4096}, n = floor(exp(U(ln 4096, ln 131072))), k uniform on 1..16,
p = k + uniform on 4..16, storage FP32 or BF16 with probability 1/2 each,
epsilon 1e-4.  The data of request r is a planted-spectrum matrix with data
seed 5000000 + r and the clustered spectrum sigma_i = 1 for i <= k, then
0.7 i^-1/2, which puts the top k singular values in one cluster above a clear
gap (the regime shift-and-invert is built for).
"""
import numpy as np

from .planted import planted_dense, planted_dense_torch, spectrum

SOLVER_SEED_BASE = 0x1607029250000100


def trace(count=512, rate=50.0, seed=5, d_choices=(256, 512, 1024, 2048, 4096),
          n_range=(4096, 131072), k_range=(1, 16), extra_range=(4, 16), eps=1e-4):
    """List of request dicts: arrival (s), d, n, k, p, storage, eps, data_seed,
    solver_seed."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, count)
    arrival = np.cumsum(gaps)
    out = []
    for r in range(count):
        d = int(rng.choice(np.asarray(d_choices)))
        n = int(np.floor(np.exp(rng.uniform(np.log(n_range[0]), np.log(n_range[1])))))
        k = int(rng.integers(k_range[0], k_range[1] + 1))
        p = k + int(rng.integers(extra_range[0], extra_range[1] + 1))
        storage = "f32" if rng.random() < 0.5 else "bf16"
        out.append(dict(id=r, arrival=float(arrival[r]), d=d, n=max(n, d), k=k, p=p,
                        storage=storage, eps=eps, data_seed=5000000 + r,
                        solver_seed=SOLVER_SEED_BASE + r))
    return out


def request_data(req, device=None, storage=None):
    """X of one request (Xt, n x d, in the request's storage type unless
    `storage` overrides it): NumPy generator without ``device``, else the
    device generator (U drawn on the device too; a different but equally
    seeded sample of the same distribution)."""
    st = storage or req["storage"]
    sig = spectrum("clustered", min(req["d"], req["n"]), k=req["k"])
    if device is None:
        return planted_dense(req["d"], req["n"], sig, req["data_seed"], st)["Xt"]
    return planted_dense_torch(req["d"], req["n"], sig, req["data_seed"], st,
                               device=device, u_on_device=True)["Xt"]
