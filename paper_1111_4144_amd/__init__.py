"""MI355X-native Cholesky/LDL inversion of Hermitian positive-definite matrices
(Krishnamoorthy & Menon, arXiv:1111.4144), behind the C-ABI library libcholinv.

The torch-facing functions live in :mod:`paper_1111_4144_amd.api`; they are
imported lazily so that ``paper_1111_4144_amd.inputs`` (the seeded synthetic
input generators) can be used without loading the GPU library.
"""

__all__ = ["inverse", "inverse_varlen", "factor", "ldl", "inverse_backward", "CholInverse"]


def __getattr__(name):
    if name in __all__:
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
