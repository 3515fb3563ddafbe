"""Plan parameters of the temperature-dependent phase mismatch of Eq. 4.

    dk(T) = (4 pi / lambda_F) [n_SH(T) - n_F(T)] - 2 pi / Lambda(T),
    Lambda(T) = Lambda(25 C) [1 + a (T - 25 C) + b (T - 25 C)^2].

The march takes dk at the reference temperature (dk0, or a per-step profile)
plus, per cell, dk(T) - dk(T_ref): the grating part exactly as above, and the
dispersion part as a cubic c1 dT + c2 dT^2 + c3 dT^3 in dT = T - T_ref.  These
helpers turn a caller's temperature-dependent index model (for instance a
Sellmeier fit of the crystal, evaluated at lambda_F and lambda_F / 2) into
those parameters.  Host-side arithmetic only.
"""
from __future__ import annotations

import math
from typing import Callable, Dict

import numpy as np

T_25C = 298.15


def grating_period(T, period_25c: float, a: float, b: float):
    """Lambda(T) of Eq. 4 [m]."""
    x = np.asarray(T, dtype=np.float64) - T_25C
    return period_25c * (1.0 + x * (a + x * b))


def mismatch(T, lambda_f: float, n_f: Callable, n_sh: Callable, period_25c: float = 0.0,
             a: float = 0.0, b: float = 0.0):
    """dk(T) of Eq. 4 [rad/m]; period_25c = 0 leaves out the grating term."""
    T = np.asarray(T, dtype=np.float64)
    out = 4.0 * math.pi / lambda_f * (np.asarray(n_sh(T), np.float64) - np.asarray(n_f(T), np.float64))
    if period_25c > 0.0:
        out = out - 2.0 * math.pi / grating_period(T, period_25c, a, b)
    return out


def dispersion_cubic(lambda_f: float, n_f: Callable, n_sh: Callable, t_ref: float,
                     span: float = 5.0, samples: int = 41) -> Dict[str, float]:
    """Least-squares cubic of the dispersion part of dk(T) - dk(T_ref) on
    |T - t_ref| <= span [K]: returns {"ddk_dT", "ddk_dT2", "ddk_dT3"}.  Exact
    when n_SH - n_F is a polynomial of degree <= 3 in T."""
    if not (span > 0.0) or samples < 4:
        raise ValueError("span must be > 0 and samples >= 4")
    dT = np.linspace(-span, span, samples)
    y = mismatch(t_ref + dT, lambda_f, n_f, n_sh) - mismatch(t_ref, lambda_f, n_f, n_sh)
    A = np.stack([dT, dT * dT, dT * dT * dT], axis=1)
    c = np.linalg.lstsq(A, y, rcond=None)[0]
    return {"ddk_dT": float(c[0]), "ddk_dT2": float(c[1]), "ddk_dT3": float(c[2])}


def plan_parameters(lambda_f: float, n_f: Callable, n_sh: Callable, t_ref: float,
                    period_25c: float = 0.0, a: float = 0.0, b: float = 0.0,
                    span: float = 5.0) -> Dict[str, float]:
    """Every dk(T) parameter of a plan: dk0 = dk(t_ref), the dispersion cubic,
    the grating period and its expansion, and t_ref."""
    out = {"dk0": float(mismatch(t_ref, lambda_f, n_f, n_sh, period_25c, a, b)), "t_ref": t_ref,
           "grating_period": period_25c, "grating_a": a, "grating_b": b}
    out.update(dispersion_cubic(lambda_f, n_f, n_sh, t_ref, span))
    return out
