"""CPU reference (oracle) for the reduced-Gaussian-blendshape rendering path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports this
package; only the tests, the smoke check and the CPU-baseline leg of the
benchmark may use it.  It is written from the paper's equations in plain
double precision and shares no code with the GPU library:

* ``oracle.blendshape`` -- linear blending (Eq. 1) and its adjoint, the
  weight MLP psi = F(theta) (Eq. 2), the L1/L2 photometric losses (Sec. 3.2,
  "Loss Function") and the Adam update (Sec. A.3), in numpy float64;
* ``oracle.raster`` -- post-blend activation, EWA projection, per-pixel
  depth-ordered alpha compositing and its exact adjoint (the 3DGS renderer
  the paper builds on, Sec. A.3), in C (``gs_ref.c``) called through ctypes,
  plus the tile binning / sort reference (Sec. 3.2: the rasterize stage needs
  the per-tile lists that preprocess determines).
"""
from . import blendshape, raster  # noqa: F401
