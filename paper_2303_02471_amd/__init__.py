"""Column-wise sparse matrix product C = A x B (CSC) for MI355X (gfx950).

The compute path is the HIP library libspgemm.so behind the C ABI of
include/spgemm.h; `api` only marshals arguments (torch tensors as device
memory). The library is loaded on first use and a missing build raises.
"""
from . import inputs  # noqa: F401

__all__ = ["inputs", "api"]
