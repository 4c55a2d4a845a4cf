"""Planted-spectrum dense matrices X = U diag(sigma) V^T.

Storage convention shared by every consumer: X is d x n with data points as
columns (the paper's main convention, Section 1), stored column-major, i.e. as a
C-contiguous array ``Xt`` of shape (n, d) whose row i is the data point x_i.

U is Haar-distributed (QR of a Gaussian square matrix with the diagonal of R
made positive).  V has orthonormal columns drawn the same way (QR of an n x d
Gaussian, or, for large n, G R^{-1} with R the Cholesky factor of G^T G, which
has the same distribution).  Optional i.i.d. Gaussian noise of the given
standard deviation is added before rounding to the storage type.

BF16 storage is produced as FP64 -> FP32 (round to nearest even) -> BF16 (round
to nearest even), and held as raw uint16 bit patterns.
"""
import numpy as np


def _clustered(d, k=4):
    i = np.arange(1, d + 1, dtype=np.float64)
    s = 0.7 * i ** -0.5
    s[:k] = 1.0
    return s


def _geometric(d):
    i = np.arange(1, d + 1, dtype=np.float64)
    s = np.empty(d)
    top = i <= 10
    s[top] = 10.0 * 2.0 ** (-(i[top] - 1) / 9.0)
    if d > 10:
        s[10] = 4.95
    rest = i >= 12
    s[rest] = 4.0 * (i[rest] - 10.0) ** -0.8
    return s


def _powerlaw(d):
    i = np.arange(1, d + 1, dtype=np.float64)
    return np.where(i <= 32, i ** -0.5, 0.6 / i)


SPECTRA = {
    # sigma_i = 1 for i <= k, then 0.7 i^-1/2 (clustered top singular values)
    "clustered": _clustered,
    # 10 .. 5 geometric over the first ten, sigma_11 = 4.95, then 4 (i-10)^-0.8
    "geometric": _geometric,
    # sigma_i = i^-1/2 up to 32, then 0.6 / i
    "powerlaw": _powerlaw,
}


def spectrum(name, d, **kw):
    return SPECTRA[name](d, **kw)


def haar_orthogonal(d, rng):
    g = rng.standard_normal((d, d))
    q, r = np.linalg.qr(g)
    return q * np.sign(np.diag(r))[None, :]


def _orthonormal_columns(n, d, rng):
    g = rng.standard_normal((n, d))
    q, r = np.linalg.qr(g)
    return q * np.sign(np.diag(r))[None, :]


def f64_to_bf16_bits(x):
    """FP64 -> FP32 (RNE) -> BF16 (RNE) bit patterns as uint16."""
    b = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32)).view(np.uint32)
    lsb = (b >> np.uint32(16)) & np.uint32(1)
    return ((b + np.uint32(0x7FFF) + lsb) >> np.uint32(16)).astype(np.uint16)


def _store(xt, storage):
    if storage == "f64":
        return np.ascontiguousarray(xt, dtype=np.float64)
    if storage == "f32":
        return np.ascontiguousarray(xt.astype(np.float32))
    if storage == "bf16":
        return f64_to_bf16_bits(xt)
    raise ValueError(storage)


# BLAS threads of the generator: the QR factorisations and the product that
# build X are blocked by thread count, so their rounding (and the stored bytes)
# depends on it; a fixed count makes X the same on every host with at least
# this many cores
GEN_BLAS_THREADS = 8


def planted_dense(d, n, sigma, seed, storage="f64", noise_std=0.0):
    """CPU (NumPy PCG64) generator.  Returns dict with Xt (n x d, storage
    type), U (d x d, planted left singular vectors), sigma (d,)."""
    from threadpoolctl import threadpool_limits
    sigma = np.asarray(sigma, dtype=np.float64)
    assert sigma.shape == (min(d, n),)
    rng = np.random.default_rng(seed)
    r = min(d, n)
    with threadpool_limits(limits=GEN_BLAS_THREADS, user_api="blas"):
        u = haar_orthogonal(d, rng)
        v = _orthonormal_columns(n, r, rng)
        xt = (v * sigma[None, :]) @ u[:, :r].T
    if noise_std:
        xt += noise_std * rng.standard_normal((n, d))
    return {"Xt": _store(xt, storage), "U": u, "sigma": sigma, "storage": storage,
            "d": d, "n": n}


def planted_dense_torch(d, n, sigma, seed, storage="f32", noise_std=0.0,
                        device="cuda", chunk=65536, u_on_device=False):
    """Large-size generator: U from NumPy (seeded), V and noise from a seeded
    torch generator on ``device``.  Returns dict with Xt as a device tensor of
    the storage dtype (torch.float64 / float32 / bfloat16), plus U and sigma.
    X is formed as Xt = G (R^{-1} diag(sigma) U^T), with G^T G = R^T R.
    With ``u_on_device`` U is drawn by the same torch generator (QR of a
    Gaussian on the device, diagonal of R made positive) instead of NumPy,
    which avoids a host QR per matrix when many are generated."""
    import torch
    sigma = np.asarray(sigma, dtype=np.float64)
    assert n >= d and sigma.shape == (d,)
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    if u_on_device:
        gq = torch.randn((d, d), generator=gen, dtype=torch.float64, device=device)
        q, r = torch.linalg.qr(gq)
        u_dev = q * torch.sign(torch.diagonal(r))[None, :]
        u = u_dev.cpu().numpy()
    else:
        rng = np.random.default_rng(seed)
        u = haar_orthogonal(d, rng)
    g = torch.randn((n, d), generator=gen, dtype=torch.float64, device=device)
    gram = torch.zeros((d, d), dtype=torch.float64, device=device)
    for c0 in range(0, n, chunk):
        blk = g[c0:c0 + chunk]
        gram += blk.T @ blk
    lower = torch.linalg.cholesky(gram)                       # gram = L L^T, R = L^T
    su = torch.from_numpy(sigma[:, None] * u.T).to(device)     # diag(sigma) U^T
    m = torch.linalg.solve_triangular(lower.T, su, upper=True)  # R^{-1} diag(sigma) U^T
    dt = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[storage]
    out = torch.empty((n, d), dtype=dt, device=device)
    for c0 in range(0, n, chunk):
        blk = g[c0:c0 + chunk] @ m
        if noise_std:
            blk += noise_std * torch.randn(blk.shape, generator=gen, dtype=torch.float64,
                                           device=device)
        if storage == "bf16":
            out[c0:c0 + chunk] = blk.to(torch.float32).to(torch.bfloat16)
        else:
            out[c0:c0 + chunk] = blk.to(dt)
    del g
    return {"Xt": out, "U": u, "sigma": sigma, "storage": storage, "d": d, "n": n}


# Named workloads: the configurations the method is measured and checked on.
# ``solver_seed`` keys the method's own Philox streams.
WORKLOADS = {
    "planted-256x2048-f64": dict(d=256, n=2048, spectrum="clustered", storage="f64",
                                 noise_std=0.0, k=4, p=8, eps=1e-6, data_seed=1001,
                                 solver_seed=0x1607029250000001),
    "planted-2048x200000-f32": dict(d=2048, n=200000, spectrum="geometric", storage="f32",
                                    noise_std=1e-4, k=10, p=20, eps=1e-4, data_seed=1002,
                                    solver_seed=0x1607029250000002),
    "planted-4096x500000-bf16": dict(d=4096, n=500000, spectrum="powerlaw", storage="bf16",
                                     noise_std=0.0, k=32, p=48, eps=1e-4, data_seed=1004,
                                     solver_seed=0x1607029250000004),
    # reduced-size versions with the same spectral shape, for CPU-oracle parity
    "planted-256x8192-f32": dict(d=256, n=8192, spectrum="geometric", storage="f32",
                                 noise_std=1e-4, k=10, p=20, eps=1e-4, data_seed=2002,
                                 solver_seed=0x1607029250000012),
    "planted-512x16384-bf16": dict(d=512, n=16384, spectrum="powerlaw", storage="bf16",
                                   noise_std=0.0, k=32, p=48, eps=1e-4, data_seed=2004,
                                   solver_seed=0x1607029250000014),
    # compressed-column sparse X with Zipf(1.1) rows (workloads/sparse.py)
    "zipf-50000x1000000-csc-f32": dict(d=50000, n=1000000, nnz_col=32, storage="csc-f32",
                                       k=16, p=32, eps=1e-3, data_seed=1003,
                                       solver_seed=0x1607029250000003),
    "zipf-2000x20000-csc-f32": dict(d=2000, n=20000, nnz_col=32, storage="csc-f32",
                                    k=16, p=32, eps=1e-3, data_seed=2003,
                                    solver_seed=0x1607029250000013),
}


def workload(name, device=None):
    """Build a named workload.  With ``device`` (e.g. "cuda") the large-size
    torch generator is used and Xt is a device tensor; otherwise NumPy.  For
    compressed-column workloads Xt is the CSC dict of workloads.sparse (NumPy,
    whatever ``device`` says)."""
    w = dict(WORKLOADS[name])
    if w["storage"].startswith("csc-"):
        from .sparse import zipf_csc
        sp = zipf_csc(w["d"], w["n"], w["nnz_col"], seed=w["data_seed"], storage=w["storage"])
        w.update(sp)
        w["Xt"] = sp
        w["name"] = name
        return w
    sig = spectrum(w["spectrum"], min(w["d"], w["n"]))
    if device is None:
        data = planted_dense(w["d"], w["n"], sig, w["data_seed"], w["storage"], w["noise_std"])
    else:
        data = planted_dense_torch(w["d"], w["n"], sig, w["data_seed"], w["storage"],
                                   w["noise_std"], device=device)
    w.update(data)
    w["name"] = name
    return w
