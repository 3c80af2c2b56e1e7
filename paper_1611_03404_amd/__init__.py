"""MI355X-native Celeste ELBO / trust-region Newton hot path (HIP for gfx950).

The compute lives in libceleste.so (C ABI declared in include/celeste.h); the
Python module `celeste` is its binding.
"""
from .celeste import Batch, Context, default_opts, load  # noqa: F401
