"""MI355X-native locally entropy-stable relaxation Runge-Kutta hot path.

The compute path is the HIP library ``libesrk.so`` (built from ``csrc/``)
behind the C-ABI declared in ``include/esrk.h``; ``esrk`` is its thin ctypes
binding.  Importing this package loads nothing; ``esrk.load()`` does, and
raises if the HIP library is missing.
"""

__all__ = ["esrk", "inputs"]
