"""Transpose-free tensor contraction on AMD MI355X (gfx950).

``C[idx_C] = alpha * sum A[idx_A] * B[idx_B] + beta * C`` computed as a matrix
multiply whose operands are addressed in place through block-scatter-matrix
layouts (scatter-offset vectors plus block strides), so no transposed copy of
any tensor is ever formed.

The compute path is the C-ABI library ``libtc.so`` built from ``csrc/``; this
package is its thin binding.  Importing the package loads nothing; the library
is opened on first use and a missing library is an error, never a fallback.
"""

__all__ = ["contract", "Plan", "Contract", "Batch"]


def __getattr__(name):
    if name in ("contract", "Plan", "Batch", "describe", "lib", "TCError"):
        from . import tc
        return getattr(tc, name)
    if name == "Contract":
        from .autograd import Contract
        return Contract
    raise AttributeError(name)
