"""Seeded synthetic inputs shaped like the paper's workloads.

This package only builds input matrices (planted-spectrum dense X, sparse X) and
their known ground truth.  It holds none of the low-rank method's arithmetic and
is imported both by the CPU oracle's tests and by the GPU tests and benchmark,
so that both sides read identical bytes.
"""
from .planted import (  # noqa: F401
    SPECTRA, spectrum, haar_orthogonal, planted_dense, planted_dense_torch,
    f64_to_bf16_bits, workload, WORKLOADS,
)
from . import serving  # noqa: F401
from . import sparse  # noqa: F401
