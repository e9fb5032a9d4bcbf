"""MI355X-native nonlinear time-history ensemble solver (arXiv 2604.02755).

The compute path lives in the C-ABI library ``libnlth.so`` (hand-written HIP
for gfx950); :mod:`.nlth` is its thin ctypes binding and :mod:`.inputs` builds
seeded synthetic meshes, spring tables and input waves.  Importing the package
does not load the library; the first call into :mod:`.nlth` does, and raises if
it has not been built.
"""
from . import inputs  # noqa: F401

__all__ = ["inputs"]
