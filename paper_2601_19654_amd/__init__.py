"""MI355X hot path of a Mercury-style hybrid symplectic N-body step (arXiv 2601.19654).

The compute lives in ``libnbody.so`` (hand-written HIP for gfx950 behind the C
ABI of ``include/nb.h``); ``nb`` is its ctypes binding.
"""
from . import nb  # noqa: F401

__all__ = ["nb"]
