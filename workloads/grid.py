"""Imaginary-frequency quadrature grid handed to the method as an input.

The energy is an integral over imaginary frequency from 0 to infinity (Sec. II.B,
the MBD energy expression).  The paper does not fix a quadrature; the workloads
use an n-point Gauss-Legendre rule on x in (-1, 1) mapped to (0, inf) by
omega = s (1 + x) / (1 - x), with weights w_GL * 2 s / (1 - x)^2 and s = 0.5 Ha.
The returned weights integrate d(omega) only; the 1/(2 pi) factor of the energy
is applied by the method itself.
"""
import numpy as np


def frequency_grid(n: int = 12, scale: float = 0.5):
    """Return (omega [Ha], weight) as float64 arrays of length n."""
    if n < 1:
        raise ValueError("need at least one quadrature point")
    x, w = np.polynomial.legendre.leggauss(n)
    omega = scale * (1.0 + x) / (1.0 - x)
    weight = w * 2.0 * scale / (1.0 - x) ** 2
    return omega.astype(np.float64), weight.astype(np.float64)
