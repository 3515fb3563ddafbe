"""Reverse-mode derivative of the discrete FP64 SSFM march of oracle.ssfm.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The loss L is real.  Gradients with respect to complex fields follow the
torch convention g = dL/dRe + i dL/dIm.  The pointwise nonlinear step is
differentiated with the state of each cell written as the real 4-vector
y = (Re A_F, Im A_F, Re A_SH, Im A_SH), so the Jacobian of the right-hand side is
a real 4x4 matrix per cell and its adjoint is the transpose.  The linear step
A <- IFFT2(M FFT2 A) is complex-linear; its adjoint is IFFT2(conj(M) FFT2 .).

Parameters differentiated: the input fields, the per-step mismatch dk_s and,
with a temperature field, every mid-plane temperature sample T_s(x, y) (through
dk = dk_s + (d dk/dT)(T - T_ref) and the thermal-lens term).  The mismatch phase
on step s is phi(t) = Phi_s + dk_s t with Phi_s = sum_{s' < s} dk_s' dz (Eq. 3), so
dL/d dk_s = (direct part at the stage times) + dz * sum_{s > s'} dL/dPhi_s.
"""
from __future__ import annotations

from typing import Optional

import numpy as np

from . import ssfm


def rhs_real(y, e_mphi, dT, c, undepleted):
    a = y[0] + 1j * y[1]
    b = y[2] + 1j * y[3]
    fa, fb = ssfm.rhs(a, b, e_mphi, dT, c, undepleted)
    return np.stack([fa.real, fa.imag, fb.real, fb.imag])


def rhs_jacobian(y, e_mphi, dT, c, undepleted):
    """J[i, j] = d f_i / d y_j of the nonlinear right-hand side (real form)."""
    ar, ai, br, bi = y
    cf = 1j * c.kappa_f * e_mphi
    cs = 1j * c.kappa_sh * np.conj(e_mphi)
    pf, qf = np.real(cf) + 0 * ar, np.imag(cf) + 0 * ar
    ps, qs = np.real(cs) + 0 * ar, np.imag(cs) + 0 * ar
    tf, ts = c.tpa_f, c.tpa_sh
    gf = c.lens_f * dT if dT is not None else 0.0 * ar
    gs = c.lens_sh * dT if dT is not None else 0.0 * ar
    z = 0.0 * ar
    J = np.empty((4, 4) + ar.shape)
    if undepleted:
        J[0, :] = z
        J[1, :] = z
    else:
        J[0, 0] = pf * br - qf * bi - 0.5 * tf * (3 * ar * ar + ai * ai)
        J[0, 1] = pf * bi + qf * br - tf * ar * ai + gf
        J[0, 2] = pf * ar + qf * ai
        J[0, 3] = pf * ai - qf * ar
        J[1, 0] = pf * bi + qf * br - tf * ar * ai - gf
        J[1, 1] = -pf * br + qf * bi - 0.5 * tf * (ar * ar + 3 * ai * ai)
        J[1, 2] = -pf * ai + qf * ar
        J[1, 3] = pf * ar + qf * ai
    J[2, 0] = 2 * ps * ar - 2 * qs * ai
    J[2, 1] = -2 * ps * ai - 2 * qs * ar
    J[2, 2] = -0.5 * ts * (3 * br * br + bi * bi)
    J[2, 3] = -ts * br * bi + gs
    J[3, 0] = 2 * ps * ai + 2 * qs * ar
    J[3, 1] = 2 * ps * ar - 2 * qs * ai
    J[3, 2] = -ts * br * bi - gs
    J[3, 3] = -0.5 * ts * (br * br + 3 * bi * bi)
    return J


def rhs_dphi(y, e_mphi, c, undepleted):
    """d f / d phi: the coupling factors are i kF e^{-i phi} and i kSH e^{+i phi}."""
    a = y[0] + 1j * y[1]
    b = y[2] + 1j * y[3]
    if undepleted:
        dfa = np.zeros_like(a)
    else:
        dfa = -1j * (1j * c.kappa_f * e_mphi * b * np.conj(a))
    dfb = 1j * (1j * c.kappa_sh * np.conj(e_mphi) * a * a)
    return np.stack([dfa.real, dfa.imag, dfb.real, dfb.imag])


def rhs_ddT(y, c, undepleted):
    """d f / d (T - T_ref) through the thermal-lens term -i g_j (T - T_ref) A_j."""
    a = y[0] + 1j * y[1]
    b = y[2] + 1j * y[3]
    dfa = np.zeros_like(a) if undepleted else -1j * c.lens_f * a
    dfb = -1j * c.lens_sh * b
    return np.stack([dfa.real, dfa.imag, dfb.real, dfb.imag])


def _vjp(J, lam):
    return np.einsum("ji...,j...->i...", J, lam)


def rk4_forward_stages(y, phi0, dk, t0, h, dT, c, undepleted):
    """Stage times and stage inputs of one RK4 step (same formulas as ssfm.rk4)."""
    def f(t, u):
        return rhs_real(u, np.exp(-1j * (phi0 + dk * t)), dT, c, undepleted)
    t1, t2, t3, t4 = t0, t0 + h / 2, t0 + h / 2, t0 + h
    u1 = y
    k1 = f(t1, u1)
    u2 = y + h / 2 * k1
    k2 = f(t2, u2)
    u3 = y + h / 2 * k2
    k3 = f(t3, u3)
    u4 = y + h * k3
    k4 = f(t4, u4)
    y_new = y + h / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
    return y_new, [(t1, u1), (t2, u2), (t3, u3), (t4, u4)]


def rk4_reverse(y, lam, phi0, dk, t0, h, dT, c, undepleted):
    """Pull lam = dL/dy_new back through one RK4 step.  Returns dL/dy,
    dL/dPhi (per cell), sum over stages of dL/dphi * t (per cell) and dL/d(T-T_ref)."""
    _, stages = rk4_forward_stages(y, phi0, dk, t0, h, dT, c, undepleted)
    weights = [h / 6, h / 3, h / 3, h / 6]
    # cotangent of k_i: kbar_i = w_i lam + (coefficient of k_i in u_{i+1}) * ubar_{i+1}
    next_coef = [h / 2, h / 2, h, None]
    ubar_next = None
    y_bar = lam.copy()
    g_phi = 0.0
    g_phi_t = 0.0
    g_dT = 0.0
    for i in (3, 2, 1, 0):
        t_i, u_i = stages[i]
        kbar = weights[i] * lam
        if ubar_next is not None:
            kbar = kbar + next_coef[i] * ubar_next
        e = np.exp(-1j * (phi0 + dk * t_i))
        ubar = _vjp(rhs_jacobian(u_i, e, dT, c, undepleted), kbar)
        dphi = np.sum(kbar * rhs_dphi(u_i, e, c, undepleted), axis=0)
        g_phi = g_phi + dphi
        g_phi_t = g_phi_t + dphi * t_i
        if dT is not None:
            g_dT = g_dT + np.sum(kbar * rhs_ddT(u_i, c, undepleted), axis=0)
        y_bar = y_bar + ubar
        ubar_next = ubar
    return y_bar, g_phi, g_phi_t, g_dT


def _to_real(a, b):
    return np.stack([a.real, a.imag, b.real, b.imag])


def adjoint(p: dict, a_f0: np.ndarray, a_sh0: np.ndarray, g_f_out: np.ndarray,
            g_sh_out: np.ndarray, dk_z: Optional[np.ndarray] = None,
            temp: Optional[np.ndarray] = None, power_weights=(0.0, 0.0)) -> dict:
    """Gradient of L = Re<g_out, A(L)> + w_F P_F(L) + w_SH P_SH(L) (first-order
    terms) with respect to the inputs of ssfm.propagate over the whole crystal.

    g_f_out, g_sh_out : seeds dL/dA(L) (torch convention), may be zero arrays
    power_weights     : (w_F, w_SH) multiplying the exit powers in L
    Returns g_f, g_sh (gradients at z = 0), g_dk [nz] (per-step mismatch),
    g_temp [nz, ny, nx] when a temperature field is given, and the forward result."""
    c = ssfm.coefficients(p)
    dz = c.dz
    nz = p["nz"]
    und = bool(p.get("undepleted", False))
    lnl = ssfm.split_order(p) == "LNL"
    fwd = ssfm.propagate(p, a_f0, a_sh0, dk_z, temp, return_states=True)
    rho_f, rho_sh = ssfm.walkoff_angles(p)
    # the linear step of the split: L(dz) between the half-steps, or L(dz/2)
    # on both sides of one RK4 over dz in the L/2 - N - L/2 order
    hstep = dz / 2 if lnl else dz
    m_f = ssfm.propagator(p, c.k_f, p["alpha_f"], hstep, rho_f)
    m_sh = ssfm.propagator(p, c.k_sh, p["alpha_sh"], hstep, rho_sh)

    def linear_adjoint(lam):
        la = ssfm.linear_step(lam[0] + 1j * lam[1], np.conj(m_f))
        lb = ssfm.linear_step(lam[2] + 1j * lam[3], np.conj(m_sh))
        return _to_real(la, lb)

    cf = ssfm.EPS0 * ssfm.C_LIGHT * p["n_f"] / 2 * c.dx * c.dy
    cs = ssfm.EPS0 * ssfm.C_LIGHT * p["n_sh"] / 2 * c.dx * c.dy
    gF = np.asarray(g_f_out, np.complex128) + 2 * cf * power_weights[0] * fwd["a_f"]
    gS = np.asarray(g_sh_out, np.complex128) + 2 * cs * power_weights[1] * fwd["a_sh"]
    lam = _to_real(gF, gS)

    # Phi_s at the start of every step
    phis = []
    phi = 0.0
    for s in range(nz):
        phis.append(phi)
        dk_s, _ = ssfm.step_mismatch(p, s, dk_z, temp)
        phi = phi + dk_s * dz

    g_dk_cells = []          # dL/d dk_s per cell (or scalar), filled backwards
    g_temp = np.zeros((nz, p["ny"], p["nx"])) if temp is not None else None
    acc_phi = 0.0            # sum over later steps of dL/dPhi
    for s in range(nz - 1, -1, -1):
        a, b = fwd["states"][s]
        dk_s, dT = ssfm.step_mismatch(p, s, dk_z, temp)
        phi0 = phis[s]
        if lnl:
            # step s: y0 -> L(dz/2) -> RK4 over [z_s, z_s + dz] -> L(dz/2)
            v = _to_real(ssfm.linear_step(a, m_f), ssfm.linear_step(b, m_sh))
            lam = linear_adjoint(lam)
            lam, gp1, gpt1, gT1 = rk4_reverse(v, lam, phi0, dk_s, 0.0, dz, dT, c, und)
            lam = linear_adjoint(lam)
            gp2 = gpt2 = 0.0
            gT2 = 0.0
        else:
            # recompute the forward stages of step s
            y0 = _to_real(a, b)
            y1, _ = rk4_forward_stages(y0, phi0, dk_s, 0.0, dz / 2, dT, c, und)
            a1 = ssfm.linear_step(y1[0] + 1j * y1[1], m_f)
            b1 = ssfm.linear_step(y1[2] + 1j * y1[3], m_sh)
            y2 = _to_real(a1, b1)
            # second half-step
            lam, gp2, gpt2, gT2 = rk4_reverse(y2, lam, phi0, dk_s, dz / 2, dz / 2, dT, c, und)
            # linear step (complex-linear, adjoint uses conj(M))
            lam = linear_adjoint(lam)
            # first half-step
            lam, gp1, gpt1, gT1 = rk4_reverse(y0, lam, phi0, dk_s, 0.0, dz / 2, dT, c, und)
        g_phi_s = gp1 + gp2
        g_dk_direct = gpt1 + gpt2
        g_dk_s = g_dk_direct + dz * acc_phi
        acc_phi = acc_phi + g_phi_s
        g_dk_cells.append(g_dk_s)
        if temp is not None:
            g_temp[s] = ssfm.thermal_mismatch_slope(p, dT) * g_dk_s + (gT1 + gT2)
    g_dk_cells.reverse()
    g_dk = np.array([float(np.sum(g)) for g in g_dk_cells])
    out = {
        "g_f": lam[0] + 1j * lam[1],
        "g_sh": lam[2] + 1j * lam[3],
        "g_dk": g_dk,
        "forward": fwd,
    }
    if temp is not None:
        out["g_temp"] = g_temp
        dTs = np.asarray(temp, np.float64) - p["t_ref"]
        out["g_t_moments"] = np.array([float(np.sum(g_temp * dTs)), float(np.sum(g_temp))])
    return out
