"""dwp: MI355X-native dry/wet generalized-Poisson solver.

The compute path lives in the HIP library ``libdwp.so`` (built from
``csrc/``); :mod:`.binding` marshals arguments to its C ABI and
:mod:`.autograd` wraps a solve as a ``torch.autograd.Function``.  Nothing is
loaded at import time, so the seeded input generators in :mod:`.workloads`
can be used without a GPU or a built library.
"""
__all__ = ["workloads"]
