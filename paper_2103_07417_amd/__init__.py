"""Adaptive black-hole ray tracing on MI355X (gfx950).

The product path is the HIP library ``libart.so`` (C ABI in include/art.h);
``art`` is a thin ctypes binding that marshals arguments and uses PyTorch only
for device memory and streams.  Importing this package does not load the
library; the first call does, and fails loudly if it is missing.
"""
from . import art  # noqa: F401
