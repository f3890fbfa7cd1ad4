"""tanTRG one-site tangent-space sweep on MI355X (gfx950).

The compute lives in the C-ABI library ``libtantrg.so`` (HIP kernels for
gfx950, declared in ``include/tantrg.h``); ``paper_2212_11973_amd.tantrg``
is its thin ctypes binding.  Importing this package does not load the
library; the binding loads it on first use and raises if it is missing.
"""
__all__ = ["tantrg", "workloads"]
