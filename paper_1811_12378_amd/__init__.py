"""MI355X-native contour-integral Helmholtz solver (hot path of arXiv 1811.12378).

The compute path lives in libhfci.so (HIP for gfx950, C ABI in include/hfci.h);
`hfci` is its thin ctypes binding.
"""
from .hfci import (Context, Contour, HfciError, Net, Operator, SolveOpts, Stats, apply, default_opts,  # noqa: F401
                   fci_apply, load_library, medium_channel, shifted_solve, solve, LIB_PATH, EXPORTED)
