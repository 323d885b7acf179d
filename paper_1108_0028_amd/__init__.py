"""MI355X-native recursive coordinate bisection (RCB) tree for neighbour
search and self-gravity (Gafton & Rosswog, MNRAS 2011).

The work runs in librcb.so (hand-written HIP kernels for gfx950 behind the C
ABI of include/rcb.h); this package only marshals torch tensors into it.
"""
from ._lib import RCBGravity, RcbError, Tree, gravity, lib, release_cache  # noqa: F401

__all__ = ["Tree", "RCBGravity", "gravity", "lib", "RcbError", "release_cache"]
