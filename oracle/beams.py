"""Focused Gaussian input beam (Sec. 2.1, Eqs. 5-6), FP64.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Reading of the printed sign: the coupled-wave equations and Appendix A use the
paraxial operator -(i/2k) lap, whose Gaussian solution is
    A(r, z) = A0 / (1 - i tau) exp[-r^2 / (w0^2 (1 - i tau))],  tau = (z - f)/z_R,
with z_R = k_F w0^2 / 2.  At z = 0 and f = L/2 this is A0/(1 + i xi) ...; the
printed Eq. 6 has the conjugate, which in this convention diverges from a
virtual focus at z = -L/2.  The amplitude follows from P = int I dA with
I = eps0 c n |A|^2 / 2 (Sec. 2.2): A0 = sqrt(4 P / (pi w0^2 eps0 c n_F)).
"""
from __future__ import annotations

import math

import numpy as np

from .ssfm import EPS0, C_LIGHT, coordinates


def gaussian_field(p: dict, power: float, w0: float, focus: float, z: float = 0.0,
                   n: float = None, lam: float = None) -> np.ndarray:
    """Free-space Gaussian beam of the -(i/2k) lap convention at plane z."""
    n = p["n_f"] if n is None else n
    lam = p["lambda_f"] if lam is None else lam
    k = 2.0 * math.pi * n / lam
    z_r = k * w0 * w0 / 2.0
    tau = (z - focus) / z_r
    a0 = math.sqrt(4.0 * power / (math.pi * w0 * w0 * EPS0 * C_LIGHT * n))
    x, y = coordinates(p)
    r2 = y[:, None] ** 2 + x[None, :] ** 2
    q = 1.0 - 1j * tau
    return a0 / q * np.exp(-r2 / (w0 * w0 * q))


def input_pump(p: dict, power: float, w0: float, focus: float, theta=None) -> np.ndarray:
    """Pump at the crystal entrance, optionally times a phase mask exp(i theta)."""
    a = gaussian_field(p, power, w0, focus, 0.0)
    if theta is not None:
        a = a * np.exp(1j * np.asarray(theta, dtype=np.float64))
    return a
