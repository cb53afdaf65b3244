"""FP64 CPU oracle for the masked, tile-based differentiable Gaussian rasterizer.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link anything here; only the test-suite, the smoke check and the benchmark's
CPU-baseline leg use it.  It shares no code with the HIP library: the only
module both sides use is ``scenes`` (seeded inputs, none of the method's
arithmetic).

What it computes is the plain definition the tiled method reaches: for every
masked pixel, depth-sorted front-to-back alpha compositing over every
surviving Gaussian (3DGS projection and blending, Sec. 3.1 Eq. 1), of colour,
camera-frame normal (Eq. 2) and plane distance (Eq. 3), followed by the
ray/plane unbiased depth (Eq. 4).  Tiles, binning and sorting only decide
which Gaussians a pixel looks at; here every pixel looks at every Gaussian
(``mode="brute"``) or at every Gaussian whose exact FP64 support box holds it
(``mode="culled"``, identical results by construction).

Modules
  sh         real spherical harmonics from the associated-Legendre definition
  project    per-Gaussian activation, EWA projection, colour, normal, distance
  composite  per-pixel compositing, depth, near-threshold allowances, gradients
  binning    tile-mask reduce, key emission, stable sort and tile ranges
  adam       the Adam update from its definition
  losses     masked L1, boundary-aware normal loss, balance-load statistics

Readings of points the paper leaves open (pixel centres, cut-offs, the
sort key, the distance term) are listed in ``oracle.config``.
"""
from .config import OracleConfig  # noqa: F401
