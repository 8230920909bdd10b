"""MI355X-native hot path of CNN variational Monte Carlo for the J1-J2 model.

The compute path is the C-ABI library ``libnqs.so`` (hand-written HIP for
gfx950, built from ``csrc/``); ``nqs`` is its thin ctypes binding.  The
binding is imported lazily so that CPU-only tooling can import the package.
"""
__all__ = ["inputs", "nqs"]
