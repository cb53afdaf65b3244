"""Real spherical harmonics from the associated-Legendre definition.

Colour in 3DGS is a sum of SH coefficients times the basis evaluated on the
viewing direction (Sec. 3.1: "multi-order spherical harmonics to represent
color").  The basis here is the real orthonormal one with the
Condon-Shortley phase, written out from its textbook definition:

  Y_l^m  = sqrt(2) K_l^m  P_l^m(cos th) cos(m ph)      m > 0
  Y_l^0  =         K_l^0  P_l^0(cos th)
  Y_l^-m = sqrt(2) K_l^m  P_l^m(cos th) sin(m ph)      m > 0
  K_l^m  = sqrt((2l+1)/(4 pi) * (l-m)!/(l+m)!)

with P_l^m carrying the (-1)^m phase.  To stay differentiable at the poles
the factor sin^m(th) is folded into the azimuthal part:
sin^m(th) cos(m ph) = Re((x + i y)^m) and sin^m(th) sin(m ph) = Im((x+iy)^m)
for a unit direction, and Q_l^m(z) = P_l^m(z) / sin^m(th) is a polynomial
obeying the same three-term recurrence in l as P_l^m.

Index of (l, m) in a coefficient array: l*l + l + m.
"""
import math

import torch


def legendre_q(lmax, z):
    """Q_l^m(z) = P_l^m(z) / (1 - z^2)^(m/2) for 0 <= m <= l <= lmax.

    Returns a dict (l, m) -> tensor shaped like z.
    """
    q = {}
    for m in range(lmax + 1):
        # P_m^m = (-1)^m (2m-1)!! (1-z^2)^(m/2)
        dfact = 1.0
        for k in range(1, 2 * m, 2):
            dfact *= k
        q[(m, m)] = torch.full_like(z, ((-1.0) ** m) * dfact)
        if m + 1 <= lmax:
            q[(m + 1, m)] = z * (2 * m + 1) * q[(m, m)]
        for l in range(m + 2, lmax + 1):
            q[(l, m)] = (z * (2 * l - 1) * q[(l - 1, m)] - (l + m - 1) * q[(l - 2, m)]) / (l - m)
    return q


def sh_basis(degree, dirs):
    """Y_lm on unit directions ``dirs`` [..., 3] -> [(degree+1)^2, ...]."""
    x, y, z = dirs[..., 0], dirs[..., 1], dirs[..., 2]
    q = legendre_q(degree, z)
    # (x + i y)^m as (re, im), built by repeated complex multiplication
    re = [torch.ones_like(x)]
    im = [torch.zeros_like(x)]
    for m in range(1, degree + 1):
        re.append(re[-1] * x - im[-1] * y)
        im.append(re[-2] * y + im[-1] * x)
    out = [None] * ((degree + 1) ** 2)
    for l in range(degree + 1):
        for m in range(0, l + 1):
            k = math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - m) / math.factorial(l + m))
            if m == 0:
                out[l * l + l] = k * q[(l, 0)]
            else:
                out[l * l + l + m] = math.sqrt(2.0) * k * q[(l, m)] * re[m]
                out[l * l + l - m] = math.sqrt(2.0) * k * q[(l, m)] * im[m]
    return torch.stack(out, dim=0)
