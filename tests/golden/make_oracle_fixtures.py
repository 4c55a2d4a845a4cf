"""Write the oracle's results for the workloads whose oracle run is too slow to
repeat inside every GPU test.  Calls only ``oracle`` (and ``workloads`` to build
the inputs).  Each fixture records a SHA-256 of the input bytes; tests use the
fixture only when the regenerated input hashes the same, and otherwise rerun
the oracle.

Usage: python tests/golden/make_oracle_fixtures.py [name ...]
"""
import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads  # noqa: E402

# name -> max_outer (None: run to convergence; an integer gives a trajectory prefix)
FIXTURES = {
    "planted-256x8192-f32": None,
    "planted-512x16384-bf16": 3,
    "planted-2048x200000-f32": None,
}


def input_hash(xt):
    return hashlib.sha256(np.ascontiguousarray(xt).tobytes()).hexdigest()


def fixture_path(name, max_outer):
    tag = "full" if max_outer is None else "prefix%d" % max_outer
    return os.path.join(HERE, "oracle_%s_%s.npz" % (name, tag))


def run(name, max_outer):
    w = workloads.workload(name)
    opt = oracle.Options(seed=w["solver_seed"])
    if max_outer is not None:
        opt.max_outer = max_outer
    t0 = time.time()
    r = oracle.solve(w["Xt"], w["storage"], w["k"], w["p"], w["eps"], opt)
    s = r.schedule
    np.savez(fixture_path(name, max_outer), U=r.U, theta=r.theta, status=r.status,
             lam=s.lam, mu_hat=s.mu_hat, delta_hat=s.delta_hat, eta=s.eta, m=s.m, b=s.b,
             tau=s.tau, eps_stop=s.eps_stop, first_solve=s.first_solve, outer=s.outer,
             epochs=np.array(s.epochs, dtype=np.int32), theta_est=r.theta_est,
             input_sha256=input_hash(w["Xt"]))
    print("%s: %.1f s, status %d, outer %d" % (name, time.time() - t0, r.status, s.outer))


if __name__ == "__main__":
    names = sys.argv[1:] or list(FIXTURES)
    for nm in names:
        run(nm, FIXTURES[nm])
