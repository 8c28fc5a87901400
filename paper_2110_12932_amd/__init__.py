"""MI355X (gfx950) implementation of the fine-level hot path of the
spatiotemporal two-level thermal method for laser powder-bed fusion
(arXiv 2110.12932): HIP kernels and a C++ runtime behind the C interface in
include/tl.h, with a ctypes binding in `tl`."""
from . import tl  # noqa: F401
