"""Constants of the rasterizer and the readings the oracle takes.

The paper (Sec. 3.1) names the operations -- project each 3D Gaussian to a
2D Gaussian, assign it to image tiles, sort, alpha-blend (Eq. 1), blend
normals (Eq. 2) and plane distances (Eq. 3), intersect rays with the blended
plane (Eq. 4) -- but fixes none of the numeric constants.  The readings:

* Eq. 1's transmittance is T_i = prod_{j<i} (1 - alpha_j) (the printed index
  is garbled).
* A fragment with alpha < 1/255 is skipped; blending stops *before* the
  fragment whose updated transmittance would fall below 1e-4.
* alpha = min(0.99, o * exp(-q/2)).
* The projected covariance gets +0.3 px^2 on its diagonal (no opacity
  compensation).
* The projection Jacobian uses the lateral coordinate clamped to
  +-1.3 * (half image size / focal length) * depth; the gradient is the exact
  derivative of that clamped function.
* Gaussians with FP32 camera depth <= 0.2 are culled, and so are Gaussians
  whose FP32 opacity logit is below float32(-ln 254) (opacity < 1/255).
* Pixel (u, v) samples the image plane at (u + 0.5, v + 0.5).
* The depth order key is the FP32 camera depth of the mean computed as
  ((R20*x + R21*y) + R22*z) + t2 with every operation rounded to FP32 and no
  fused multiply-add; ties go to the lower Gaussian index.
* Background is 0.  Pixels outside the building mask output 0 everywhere and
  receive no gradient.
* The Gaussian normal is the rotation axis of the smallest scale (lowest axis
  on ties, decided on the FP32 log-scales), rotated into the camera frame and
  flipped to face the camera.  The plane distance is d = n_c . t (signed,
  negative for a camera-facing plane); Eq. 4 is then D / (N . K^-1 p~), set to
  0 unless N . K^-1 p~ < -1e-6.
* SH: real orthonormal basis with the Condon-Shortley phase, index l^2+l+m,
  theta from +z, phi from +x toward +y, evaluated on the world-frame
  direction from the camera centre to the mean; colour = sum + 0.5 clamped
  at 0.
"""
from dataclasses import dataclass
import math

import numpy as np


@dataclass(frozen=True)
class OracleConfig:
    alpha_min: float = 1.0 / 255.0
    t_min: float = 1e-4
    alpha_max: float = 0.99
    dilation: float = 0.3
    z_near: float = 0.2
    fov_clamp: float = 1.3
    logit_min: float = float(np.float32(-math.log(254.0)))
    bg: tuple = (0.0, 0.0, 0.0)
    depth_guard: float = 1e-6
