"""MI355X-native masked differentiable Gaussian-splatting rasterizer (the
per-sub-region rendering step of PG-SAG, arXiv 2501.01677).

The compute lives in libpgsag.so (hand-written HIP for gfx950, C ABI in
include/pgsag.h); this package only marshals arguments.  Importing it does
not load the library; the first use does, and fails if it is not built.
"""
from .raster import (Batch, MaskedRasterizer, RenderConfig, CapacityError, adam_step,  # noqa: F401
                     gaussians_to_device, make_camera)
