"""Kaiser-Bessel (KB) interpolation kernel of the NUFFT measurement operator (FP64).

The paper writes the measurement as y = Phi x + n with Phi a discretisation of
the interferometric measurement (measurement-model paragraph).  Its continuous
visibilities are realised, as in the authors' toolbox, by a non-uniform FFT:
deapodise, zero-pad, FFT, then interpolate the oversampled grid with a compact
kernel.  The kernel here is the KB window with the Beatty et al. (2005) shape
parameter, written from its definition.
"""
from __future__ import annotations

import numpy as np
import scipy.special


def beta(J: int, alpha: float) -> float:
    """KB shape parameter for width J and oversampling alpha (Beatty et al. 2005)."""
    return float(np.pi * np.sqrt((J / alpha) ** 2 * (alpha - 0.5) ** 2 - 0.8))


def psi(t, J: int, b: float) -> np.ndarray:
    """KB window psi(t) = I0(b sqrt(1 - (2t/J)^2)) / I0(b) for |t| <= J/2, else 0."""
    t = np.asarray(t, dtype=np.float64)
    arg = 1.0 - (2.0 * t / J) ** 2
    inside = arg >= 0.0
    out = np.zeros_like(t)
    out[inside] = scipy.special.i0(b * np.sqrt(arg[inside])) / scipy.special.i0(b)
    return out


def psi_hat(xi, J: int, b: float) -> np.ndarray:
    """Continuous Fourier transform  int psi(t) exp(-2 pi i xi t) dt  in closed form.

    J sinh(sqrt(b^2 - (pi J xi)^2)) / (sqrt(b^2 - (pi J xi)^2) I0(b)); past
    pi J |xi| = b the square root turns imaginary and sinh(z)/z becomes sin(w)/w.
    """
    xi = np.asarray(xi, dtype=np.float64)
    z2 = b * b - (np.pi * J * xi) ** 2
    out = np.empty_like(xi)
    pos = z2 > 0
    neg = z2 < 0
    zero = ~(pos | neg)
    z = np.sqrt(z2[pos])
    out[pos] = np.sinh(z) / z
    w = np.sqrt(-z2[neg])
    out[neg] = np.sin(w) / w
    out[zero] = 1.0
    return J * out / scipy.special.i0(b)
