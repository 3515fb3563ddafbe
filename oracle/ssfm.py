"""Forward SSFM march in FP64 (complex128), written from the paper's equations.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Model (Sec. 2.1, Eqs. 1-4; Sec. 3, Eqs. 11-15; Appendix A, Eqs. A.1-A.5):

  dA_F/dz  = i kF e^{-i phi} A_SH conj(A_F) - (i/2k_F) lap A_F - (alpha_F/2) A_F
             - (beta~_F/2)|A_F|^2 A_F - i g_F dT A_F
  dA_SH/dz = i kSH e^{+i phi} A_F^2       - (i/2k_SH) lap A_SH - (alpha_SH/2) A_SH
             - (beta~_SH/2)|A_SH|^2 A_SH - i g_SH dT A_SH

Readings of the printed equations (each is pinned by a test in
tests/test_oracle_pins.py):
  * coupling: kF = 2 pi d/(n_F lambda_F); kSH = 2 pi d/(n_SH lambda_F).  The
    printed SH coefficient uses lambda_SH, which breaks Manley-Rowe energy
    conservation with the intensity I = eps0 c n |A|^2 / 2 of Sec. 2.2 and gives
    four times the Boyd-Kleinman efficiency of Eq. 17.
  * two-photon absorption acts on intensity: beta~_j = beta_j eps0 c n_j / 2,
    so that dI/dz = -beta I^2.
  * linear absorption alpha_j is part of the linear operator L (Eq. 11), i.e.
    it is applied exactly inside the Fourier-space propagator.
  * the accumulated mismatch phase phi(z) = int_0^z dk dz' (Eq. 3) is exact for
    a mismatch that is constant within each z-step (per step, or per cell when
    a temperature field is given).
  * temperature (optional): dk = dk_s + [dk(T) - dk(T_ref)] per cell, dk(T)
    of Eq. 4 with a cubic in dT = T - T_ref standing in for the Sellmeier part
    and the printed grating period Lambda(T) (see thermal_mismatch), and a
    thermal-lens term -i (2 pi/lambda_j)(dn/dT) dT A_j, with T sampled at the
    step mid-plane.
  * undepleted pump (Sec. 5.1): the nonlinear part of dA_F/dz is zero.
  * spatial walk-off (optional; Sec. 4, the propagator set-up of the package
    description): dA_j/dz gains -tan(rho_j) dA_j/dx, a linear term that moves the
    beam of wave j towards +x by tan(rho_j) per unit length.  It is part of L,
    i.e. a factor exp(-2 i pi qx tan(rho_j) dz) of the propagator.  rho_j comes
    from params "walkoff_f" / "walkoff_sh" (rad, default 0).

Discrete scheme, one z-step s on [z_s, z_s + dz] (Eq. 14, order N/2 - L - N/2,
the order the paper implements; params "split" = "NLN", the default):
  y <- RK4 over [z_s, z_s + dz/2] of the pointwise nonlinear system
  A_j <- IFFT2( M_j * FFT2(A_j) ),
         M_j = exp[(2 i pi^2 (qx^2 + qy^2)/k_j - alpha_j/2 - 2 i pi qx tan(rho_j)) dz]
  y <- RK4 over [z_s + dz/2, z_s + dz]
The other Strang order that Sec. 3 calls equivalent (params "split" = "LNL"):
  A_j <- L(dz/2) A_j;  y <- RK4 over [z_s, z_s + dz];  A_j <- L(dz/2) A_j
with the same per-step mismatch and temperature sample.
Grid: x_m = (m - Nx/2) dx, dx = Lx/Nx (periodic window); q = fftfreq(N, dx)
in cycles per metre, which is the transform pair of Eq. A.2.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Optional

import numpy as np

EPS0 = 8.8541878128e-12      # vacuum permittivity [F/m] (CODATA 2018)
C_LIGHT = 299792458.0        # speed of light [m/s]


@dataclass
class Coefficients:
    k_f: float
    k_sh: float
    kappa_f: float
    kappa_sh: float
    tpa_f: float      # beta~_F
    tpa_sh: float     # beta~_SH
    lens_f: float     # g_F = (2 pi / lambda_F) dn/dT
    lens_sh: float    # g_SH = (2 pi / lambda_SH) dn/dT
    dx: float
    dy: float
    dz: float


def coefficients(p: dict) -> Coefficients:
    """Constants of Eqs. 1-2 under the readings listed in the module header."""
    lam_f = p["lambda_f"]
    lam_sh = lam_f / 2.0
    k_f = 2.0 * math.pi * p["n_f"] / lam_f
    k_sh = 2.0 * math.pi * p["n_sh"] / lam_sh
    kappa_f = 2.0 * math.pi * p["d_eff"] / (p["n_f"] * lam_f)
    kappa_sh = 2.0 * math.pi * p["d_eff"] / (p["n_sh"] * lam_f)
    tpa_f = p["beta_f"] * EPS0 * C_LIGHT * p["n_f"] / 2.0
    tpa_sh = p["beta_sh"] * EPS0 * C_LIGHT * p["n_sh"] / 2.0
    lens_f = 2.0 * math.pi * p["dn_dT"] / lam_f
    lens_sh = 2.0 * math.pi * p["dn_dT"] / lam_sh
    return Coefficients(k_f, k_sh, kappa_f, kappa_sh, tpa_f, tpa_sh, lens_f, lens_sh,
                        p["lx"] / p["nx"], p["ly"] / p["ny"], p["lcr"] / p["nz"])


def coordinates(p: dict):
    """Transverse sample positions x[m], y[n] (periodic window centred on 0)."""
    dx, dy = p["lx"] / p["nx"], p["ly"] / p["ny"]
    x = (np.arange(p["nx"]) - p["nx"] // 2) * dx
    y = (np.arange(p["ny"]) - p["ny"] // 2) * dy
    return x, y


def propagator(p: dict, k: float, alpha: float, dz: float, walkoff: float = 0.0) -> np.ndarray:
    """Fourier-space propagator of the linear operator over dz (Eqs. A.3-A.5 with
    the linear loss of Eq. 11 and the walk-off term):
    exp[(2 i pi^2 (qx^2+qy^2)/k - alpha/2 - 2 i pi qx tan(walkoff)) dz]."""
    qx = np.fft.fftfreq(p["nx"], p["lx"] / p["nx"])
    qy = np.fft.fftfreq(p["ny"], p["ly"] / p["ny"])
    q2 = qy[:, None] ** 2 + qx[None, :] ** 2
    drift = 2j * math.pi * math.tan(walkoff) * qx[None, :]
    return np.exp((2j * math.pi ** 2 * q2 / k - alpha / 2.0 - drift) * dz)


T_25C = 298.15    # the reference temperature of the grating-period expansion (Eq. 4)


def grating_period(p: dict, T):
    """Lambda(T) = Lambda(25 C) [1 + a (T - 25 C) + b (T - 25 C)^2] (Eq. 4)."""
    d = T - T_25C
    return p["grating_period"] * (1.0 + p.get("grating_a", 0.0) * d + p.get("grating_b", 0.0) * d * d)


def thermal_mismatch(p: dict, dT):
    """dk(T) - dk(T_ref) per cell, dT = T - T_ref, following Eq. 4:
      dispersion part (4 pi/lambda_F)(n_SH(T) - n_F(T)): c1 dT + c2 dT^2 + c3 dT^3
        (c1 = "ddk_dT", c2 = "ddk_dT2", c3 = "ddk_dT3"), a polynomial stand-in
        for the Sellmeier indices, which the paper only cites;
      grating part -2 pi / Lambda(T): exactly as printed, with Lambda(25 C) =
        "grating_period" (0 = no grating term), a = "grating_a", b = "grating_b"."""
    c2, c3 = p.get("ddk_dT2", 0.0), p.get("ddk_dT3", 0.0)
    out = dT * (p["ddk_dT"] + dT * (c2 + dT * c3))
    if p.get("grating_period", 0.0) > 0.0:
        t_ref = p["t_ref"]
        out = out + (2.0 * math.pi / grating_period(p, t_ref)
                     - 2.0 * math.pi / grating_period(p, t_ref + dT))
    return out


def thermal_mismatch_slope(p: dict, dT):
    """d(dk)/dT at the cell's temperature."""
    c2, c3 = p.get("ddk_dT2", 0.0), p.get("ddk_dT3", 0.0)
    out = p["ddk_dT"] + dT * (2.0 * c2 + 3.0 * c3 * dT)
    if p.get("grating_period", 0.0) > 0.0:
        T = p["t_ref"] + dT
        lam = grating_period(p, T)
        dlam = p["grating_period"] * (p.get("grating_a", 0.0) + 2.0 * p.get("grating_b", 0.0) * (T - T_25C))
        out = out + 2.0 * math.pi * dlam / (lam * lam)
    return out


def split_order(p: dict) -> str:
    """"NLN" (N/2 - L - N/2, default) or "LNL" (L/2 - N - L/2)."""
    order = p.get("split", "NLN")
    if order not in ("NLN", "LNL"):
        raise ValueError(f"unknown split order {order!r}")
    return order


def walkoff_angles(p: dict):
    """(rho_F, rho_SH) in rad; zero when the parameters do not set them."""
    return p.get("walkoff_f", 0.0), p.get("walkoff_sh", 0.0)


def linear_step(a: np.ndarray, m: np.ndarray) -> np.ndarray:
    """Diffraction + linear loss over one full step, solved in Fourier space."""
    return np.fft.ifft2(m * np.fft.fft2(a))


def rhs(a, b, e_mphi, dT, c: Coefficients, undepleted: bool):
    """Nonlinear operator N of Eq. 11 applied pointwise (with the readings above).

    e_mphi = exp(-i phi) at the evaluation point (scalar or per cell);
    dT = T - T_ref at the step mid-plane (None when no temperature field)."""
    fb = 1j * c.kappa_sh * np.conj(e_mphi) * a * a - 0.5 * c.tpa_sh * (np.abs(b) ** 2) * b
    if undepleted:
        fa = np.zeros_like(a)
    else:
        fa = 1j * c.kappa_f * e_mphi * b * np.conj(a) - 0.5 * c.tpa_f * (np.abs(a) ** 2) * a
    if dT is not None:
        if not undepleted:
            fa = fa - 1j * c.lens_f * dT * a
        fb = fb - 1j * c.lens_sh * dT * b
    return fa, fb


def rk4(a, b, phi0, dk, t0, h, dT, c: Coefficients, undepleted: bool):
    """Classical RK4 over [t0, t0 + h] (t measured from the start of the step);
    the mismatch phase is phi(t) = phi0 + dk * t, exact for a piecewise-constant
    mismatch (Eq. 3)."""
    def f(t, ya, yb):
        return rhs(ya, yb, np.exp(-1j * (phi0 + dk * t)), dT, c, undepleted)

    k1a, k1b = f(t0, a, b)
    k2a, k2b = f(t0 + h / 2, a + h / 2 * k1a, b + h / 2 * k1b)
    k3a, k3b = f(t0 + h / 2, a + h / 2 * k2a, b + h / 2 * k2b)
    k4a, k4b = f(t0 + h, a + h * k3a, b + h * k3b)
    a = a + h / 6 * (k1a + 2 * k2a + 2 * k3a + k4a)
    b = b + h / 6 * (k1b + 2 * k2b + 2 * k3b + k4b)
    return a, b


def step_mismatch(p: dict, s: int, dk_z: Optional[np.ndarray], temp: Optional[np.ndarray]):
    """Mismatch on step s: dk_z[s] (or dk0), plus (d dk/dT)(T_s - T_ref) per cell.
    Returns (dk_s, dT_s) where dk_s is a scalar or a [ny, nx] array."""
    base = float(dk_z[s]) if dk_z is not None else float(p["dk0"])
    if temp is None:
        return base, None
    dT = np.asarray(temp[s], dtype=np.float64) - p["t_ref"]
    return base + thermal_mismatch(p, dT), dT


def power(a: np.ndarray, n: float, dx: float, dy: float) -> float:
    """Beam power P = int I dA with I = eps0 c n |A|^2 / 2 (Sec. 2.2)."""
    return float(EPS0 * C_LIGHT * n / 2.0 * dx * dy * np.sum(np.abs(np.asarray(a, np.complex128)) ** 2))


def propagate(p: dict, a_f: np.ndarray, a_sh: np.ndarray, dk_z: Optional[np.ndarray] = None,
              temp: Optional[np.ndarray] = None, s_begin: int = 0, s_end: Optional[int] = None,
              trace: bool = False, return_states: bool = False) -> dict:
    """March steps [s_begin, s_end) of the crystal.

    a_f, a_sh : [ny, nx] complex fields at z = s_begin * dz (not modified)
    dk_z      : optional [nz] per-step mismatch (rad/m), replaces dk0
    temp      : optional [nz, ny, nx] mid-plane temperature samples (K)
    Returns a dict with the exit fields, powers, and optionally the power trace
    after every step and the list of step-input states."""
    nz = p["nz"]
    s_end = nz if s_end is None else s_end
    c = coefficients(p)
    dz = c.dz
    undepleted = bool(p.get("undepleted", False))
    rho_f, rho_sh = walkoff_angles(p)
    lnl = split_order(p) == "LNL"
    hstep = dz / 2 if lnl else dz
    m_f = propagator(p, c.k_f, p["alpha_f"], hstep, rho_f)
    m_sh = propagator(p, c.k_sh, p["alpha_sh"], hstep, rho_sh)
    a = np.array(a_f, dtype=np.complex128)
    b = np.array(a_sh, dtype=np.complex128)

    # accumulated phase Phi at the start of step s_begin (Eq. 3)
    phi = 0.0
    for s in range(s_begin):
        dk_s, _ = step_mismatch(p, s, dk_z, temp)
        phi = phi + dk_s * dz

    tr_f, tr_sh, states = [], [], []
    for s in range(s_begin, s_end):
        if return_states:
            states.append((a.copy(), b.copy()))
        dk_s, dT = step_mismatch(p, s, dk_z, temp)
        if lnl:
            a = linear_step(a, m_f)
            b = linear_step(b, m_sh)
            a, b = rk4(a, b, phi, dk_s, 0.0, dz, dT, c, undepleted)
            a = linear_step(a, m_f)
            b = linear_step(b, m_sh)
        else:
            a, b = rk4(a, b, phi, dk_s, 0.0, dz / 2, dT, c, undepleted)
            a = linear_step(a, m_f)
            b = linear_step(b, m_sh)
            a, b = rk4(a, b, phi, dk_s, dz / 2, dz / 2, dT, c, undepleted)
        phi = phi + dk_s * dz
        if trace:
            tr_f.append(power(a, p["n_f"], c.dx, c.dy))
            tr_sh.append(power(b, p["n_sh"], c.dx, c.dy))
    out = {
        "a_f": a, "a_sh": b,
        "p_f": power(a, p["n_f"], c.dx, c.dy),
        "p_sh": power(b, p["n_sh"], c.dx, c.dy),
    }
    if trace:
        out["trace_f"] = np.array(tr_f)
        out["trace_sh"] = np.array(tr_sh)
    if return_states:
        out["states"] = states
    return out


def efficiency(p: dict, a_f0: np.ndarray, result: dict) -> float:
    """eta = P_SH(L) / P_F(0), with P_F(0) from the discrete input field."""
    c = coefficients(p)
    return result["p_sh"] / power(a_f0, p["n_f"], c.dx, c.dy)
