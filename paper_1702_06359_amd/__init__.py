"""MI355X-native Kalman-filter track building (barrel, combinatorial KF).

The compute path lives in the HIP library ``libmkf.so`` (built from ``csrc/``)
behind the C ABI declared in ``include/mkf.h``; ``abi`` is its thin ctypes
binding.  Nothing is loaded at import time so that the synthetic-event
generator can be used on hosts without the GPU library.
"""
__all__ = ["abi", "synth"]
