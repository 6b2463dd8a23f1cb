"""Seeded synthetic inputs shared by the oracle-side tests and the GPU library's callers."""
from .gen import CSR, Workload, make_small, make_splade_like, make_batch, sparse_rows  # noqa: F401
