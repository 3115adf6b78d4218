"""MI355X (gfx950) hot path of concurrent GPU checkpoint/restore with validated
speculation (PhoenixOS, arXiv 2405.12079).

The product is libphos.so (C ABI in include/phos.h, HIP kernels in csrc/);
``phos`` is its thin ctypes binding.  Importing this package loads the
library and fails if it has not been built: there is no CPU fallback.
"""
from . import phos  # noqa: F401
from .phos import PhosError  # noqa: F401

phos.lib()
