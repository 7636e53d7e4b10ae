"""Imaginary-frequency quadrature grid (oracle; test infrastructure only).

The paper integrates the imaginary-axis term I_nn(omega) numerically on a
"modified Gauss-Legendre" grid (Implementation, Contour Deformation; it cites
Ren et al. 2012 and uses 200 points) without printing the map.  Reading used
here: Gauss-Legendre nodes t_g and weights w_g on [-1, 1] mapped to [0, inf)
by xi = x0 (1 + t) / (1 - t), so that d xi = 2 x0 / (1 - t)^2 dt, with
x0 = 0.5 Ha.  The weights returned are the d-xi weights z_g (no 1/pi).
"""
import numpy as np


def gauss_legendre(n: int, x0: float = 0.5):
    """Return (xi[n], z[n]) with sum_g z_g h(xi_g) ~ int_0^inf h(xi) d xi."""
    if n < 1 or not (x0 > 0):
        raise ValueError("need n >= 1 and x0 > 0")
    t, w = np.polynomial.legendre.leggauss(n)
    xi = x0 * (1.0 + t) / (1.0 - t)
    z = w * 2.0 * x0 / (1.0 - t) ** 2
    return xi.astype(np.float64), z.astype(np.float64)
