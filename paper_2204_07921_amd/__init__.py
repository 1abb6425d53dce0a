"""MI355X-native multigrid minimisation of curvature energies (arXiv 2204.07921).

The compute path is libmgcurv.so (hand-written HIP for gfx950, C ABI in
include/mgcurv.h); this package only marshals torch device tensors into it.
Import the binding explicitly: ``from paper_2204_07921_amd import mgcurv``.
"""
__all__ = ["mgcurv", "build"]
