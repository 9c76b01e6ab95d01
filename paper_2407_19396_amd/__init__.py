"""MI355X-native batched gridworld environment step (NAVIX, arXiv 2407.19396).

The compute path is the HIP library ``libgridenv.so`` (built from ``csrc/``)
behind the C-ABI declared in ``include/gridenv.h``; ``gridenv`` is its thin
ctypes binding.  Importing this package does not load the library; the first
use of ``gridenv`` does, and fails loudly when it is missing.
"""
__all__ = ["gridenv", "workloads"]
