"""Closed forms and quadratures that pin the oracle to the physics.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

  bk_h, bk_sigma_opt, bk_efficiency   Boyd-Kleinman focusing function and the
        efficiency of Eq. 17 (Sec. 5.1), by Gauss-Legendre quadrature.
  undepleted_sh_power                 low-conversion SH power of a focused
        Gaussian pump when k_SH != 2 k_F, by a 2-D quadrature derived from the
        coupled-wave equations (Eqs. 1-2) and the Gaussian solution of Eq. 5.
  plane-wave laws                     tanh^2 depletion, TPA decay, sinc^2.
  grin_gaussian                       Gaussian beam in a quadratic-index medium
        via the ABCD law (thermal-lens pin).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.optimize import minimize_scalar

from .ssfm import EPS0, C_LIGHT


def _gl(n, a, b):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (b - a) * x + 0.5 * (b + a), 0.5 * (b - a) * w


def bk_h(sigma: float, xi: float, nodes: int = 400) -> float:
    """h(sigma, xi) = (1 / 4 xi) |int_{-xi}^{xi} e^{i sigma tau} / (1 + i tau) dtau|^2
    (Boyd-Kleinman focusing function with no walk-off, the h of Eq. 17)."""
    t, w = _gl(nodes, -xi, xi)
    val = np.sum(w * np.exp(1j * sigma * t) / (1.0 + 1j * t))
    return float(abs(val) ** 2 / (4.0 * xi))


def bk_sigma_opt(xi: float) -> float:
    """sigma that maximises h(sigma, xi)."""
    res = minimize_scalar(lambda s: -bk_h(s, xi), bounds=(0.0, 2.0), method="bounded",
                          options={"xatol": 1e-12})
    return float(res.x)


def bk_efficiency(p: dict, power: float, h: float) -> float:
    """eta_BK of Eq. 17: 16 pi^2 d^2 P L h / (eps0 c n_F n_SH lambda_F^3)."""
    return (16.0 * math.pi ** 2 * p["d_eff"] ** 2 * power * p["lcr"] * h
            / (EPS0 * C_LIGHT * p["n_f"] * p["n_sh"] * p["lambda_f"] ** 3))


def undepleted_sh_power(p: dict, power: float, w0: float, focus: float, dk: float,
                        nodes: int = 240) -> float:
    """SH power at z = L for an undepleted, lossless Gaussian pump (Eq. 5 form,
    -(i/2k) lap convention) and the SH equation of Eq. 2 with coupling
    kSH = 2 pi d / (n_SH lambda_F) and phase e^{i dk z}.

    Each slab dz' launches the Gaussian source i kSH e^{i dk z'} A_F(z')^2 which
    then diffracts freely at k_SH to z = L; integrating |A_SH(L)|^2 over the plane
    gives P_SH = 2 pi d^2 P^2 Re J / (eps0 c n_SH n_F^2 lambda_F^2) with
      J = int int e^{i dk (z - z')} / [(1 - i tau)(1 + i tau')(w0^2/4 - i eps (z - z'))] dz dz',
      tau = (z - f)/z_R, eps = 1/(4 k_F) - 1/(2 k_SH).
    For k_SH = 2 k_F this reduces to Eq. 17."""
    lam = p["lambda_f"]
    k_f = 2.0 * math.pi * p["n_f"] / lam
    k_sh = 2.0 * math.pi * p["n_sh"] / (lam / 2.0)
    z_r = k_f * w0 * w0 / 2.0
    eps = 1.0 / (4.0 * k_f) - 1.0 / (2.0 * k_sh)
    z, w = _gl(nodes, 0.0, p["lcr"])
    tau = (z - focus) / z_r
    dzz = z[:, None] - z[None, :]
    kern = (np.exp(1j * dk * dzz)
            / ((1.0 - 1j * tau)[:, None] * (1.0 + 1j * tau)[None, :] * (w0 * w0 / 4.0 - 1j * eps * dzz)))
    j = np.sum(w[:, None] * w[None, :] * kern)
    return float(2.0 * math.pi * p["d_eff"] ** 2 * power ** 2 * j.real
                 / (EPS0 * C_LIGHT * p["n_sh"] * p["n_f"] ** 2 * lam ** 2))


def tanh2_gain(p: dict, intensity: float) -> float:
    """Plane-wave depletion rate Gamma with eta(z) = tanh^2(Gamma z):
    Gamma^2 = 8 pi^2 d^2 I / (eps0 c n_F^2 n_SH lambda_F^2)."""
    return math.sqrt(8.0 * math.pi ** 2 * p["d_eff"] ** 2 * intensity
                     / (EPS0 * C_LIGHT * p["n_f"] ** 2 * p["n_sh"] * p["lambda_f"] ** 2))


def tpa_intensity(i0: float, beta: float, z: float) -> float:
    """dI/dz = -beta I^2  ->  I(z) = I0 / (1 + beta I0 z)."""
    return i0 / (1.0 + beta * i0 * z)


def undepleted_plane_wave_sh(p: dict, a0: complex, dk: float, length: float) -> complex:
    """A_SH(L) for a constant pump a0, no loss:
    i kSH a0^2 int_0^L e^{i dk z} dz = i kSH a0^2 L e^{i dk L/2} sinc(dk L / 2)."""
    kappa_sh = 2.0 * math.pi * p["d_eff"] / (p["n_sh"] * p["lambda_f"])
    x = dk * length / 2.0
    sinc = 1.0 if x == 0.0 else math.sin(x) / x
    return 1j * kappa_sh * a0 * a0 * length * np.exp(1j * x) * sinc


def grin_gaussian(p: dict, power: float, w0: float, focus: float, curvature: float,
                  z: float, nodes: int = 400) -> np.ndarray:
    """Gaussian beam after distance z in the index profile n = n_F + dn/dT * dT(r),
    dT(r) = -curvature * r^2 (thermal lens term of the oracle RHS with only
    the F wave present).  The field keeps the form u(z) exp(-r^2 / Q(z)); with
    q = i k Q / 2 the beam parameter follows the GRIN ABCD law
    [[cos gz, sin gz / g], [-g sin gz, cos gz]], g^2 = 2 g_F curvature / k_F,
    and u' / u = 2 i / (k_F Q(z)) fixes the complex amplitude."""
    from .ssfm import coordinates
    lam = p["lambda_f"]
    n = p["n_f"]
    k = 2.0 * math.pi * n / lam
    g_f = 2.0 * math.pi * p["dn_dT"] / lam
    gam = math.sqrt(2.0 * g_f * curvature / k)
    z_r = k * w0 * w0 / 2.0
    tau0 = -focus / z_r
    q_cap0 = w0 * w0 * (1.0 - 1j * tau0)
    qq0 = 1j * k * q_cap0 / 2.0

    def q_of(zz):
        c, s = np.cos(gam * zz), np.sin(gam * zz)
        qq = (c * qq0 + s / gam) / (-gam * s * qq0 + c)
        return -2j * qq / k

    a0 = math.sqrt(4.0 * power / (math.pi * w0 * w0 * EPS0 * C_LIGHT * n))
    u0 = a0 / (1.0 - 1j * tau0)
    zs, ws = _gl(nodes, 0.0, z)
    log_u = np.log(u0) + np.sum(ws * 2j / (k * q_of(zs)))
    x, y = coordinates(p)
    r2 = y[:, None] ** 2 + x[None, :] ** 2
    return np.exp(log_u) * np.exp(-r2 / q_of(z))
