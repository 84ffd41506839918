"""MI355X (gfx950) differentiable Gaussian rasterizer for Gaussian-splatting
SLAM mapping: EWA projection, tile binning, depth-keyed radix sort,
front-to-back compositing and its backward, as hand-written HIP behind the C
ABI in include/gsr.h. Python is a thin ctypes binding plus a
torch.autograd.Function."""
from ._lib import GsrError, load  # noqa: F401

__all__ = ["GsrError", "load"]
