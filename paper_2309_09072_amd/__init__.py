"""MI355X (gfx950) engine for the LCS hot path of arXiv 2309.09072.

The compute lives in ``liblcs.so`` (HIP kernels + C ABI, include/lcs.h); this
package holds its ctypes binding (``lcs``), the build script (``build``) and
the seeded synthetic input generators (``synth``).
"""
from . import synth  # noqa: F401
