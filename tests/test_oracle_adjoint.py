"""Pins of the oracle's reverse-mode derivative (CPU only).

The adjoint is checked against central finite differences of the forward
oracle, against the adjoint identity of the linear step, and against the
derivative of the independent focusing-integral quadrature.
"""
import math

import numpy as np
import pytest

from oracle import ssfm, adjoint, beams, pins

LAM = 1064e-9


def params(n=8, nz=6, **kw):
    p = dict(nx=n, ny=n, nz=nz, lx=0.12e-3, ly=0.12e-3, lcr=2e-3, lambda_f=LAM, n_f=2.14,
             n_sh=2.18, d_eff=10e-12, alpha_f=5.0, alpha_sh=9.0, beta_f=2e-11, beta_sh=3e-11,
             dk0=900.0, ddk_dT=300.0, dn_dT=3e-5, t_ref=300.0, undepleted=False)
    p.update(kw)
    return p


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def crand(r, shape, scale):
    return (r.normal(size=shape) + 1j * r.normal(size=shape)) * scale


def loss(p, a, b, g_f, g_sh, w, dk_z=None, temp=None):
    out = ssfm.propagate(p, a, b, dk_z=dk_z, temp=temp)
    return (np.real(np.vdot(g_f, out["a_f"])) + np.real(np.vdot(g_sh, out["a_sh"]))
            + w[0] * out["p_f"] + w[1] * out["p_sh"])


@pytest.mark.parametrize("with_temp,undepleted,walkoff,cubic,split", [
    (False, False, 0.0, False, "NLN"), (True, False, 0.0, False, "NLN"),
    (True, True, 0.0, False, "NLN"), (False, False, 0.02, False, "NLN"),
    (True, False, 0.0, True, "NLN"), (False, False, 0.02, False, "LNL"),
    (True, False, 0.0, True, "LNL")])
def test_adjoint_matches_central_differences(with_temp, undepleted, walkoff, cubic, split):
    p = params(undepleted=undepleted, walkoff_sh=walkoff, walkoff_f=-0.5 * walkoff, split=split)
    if cubic:
        # cubic dispersion part and a grating period with an exaggerated expansion
        p.update(ddk_dT2=-120.0, ddk_dT3=45.0, grating_period=8e-6, grating_a=2e-3, grating_b=-4e-5)
    r = rng(21)
    shape = (p["ny"], p["nx"])
    a = crand(r, shape, 5e7)
    b = crand(r, shape, 2e7)
    g_f = crand(r, shape, 1.0)
    g_sh = crand(r, shape, 1.0)
    w = (0.3, 1.7)
    dk_z = 900.0 + 200.0 * r.normal(size=p["nz"])
    temp = 300.0 + 2.0 * r.normal(size=(p["nz"],) + shape) if with_temp else None
    adj = adjoint.adjoint(p, a, b, g_f * 1e-9, g_sh * 1e-9, dk_z=dk_z, temp=temp, power_weights=w)
    L = lambda **kw: loss(p, kw.get("a", a), kw.get("b", b), g_f * 1e-9, g_sh * 1e-9, w,
                          kw.get("dk_z", dk_z), kw.get("temp", temp))
    # directional derivatives along random directions
    va, vb = crand(r, shape, 5e7), crand(r, shape, 2e7)
    eps = 1e-6
    fd = (L(a=a + eps * va, b=b + eps * vb) - L(a=a - eps * va, b=b - eps * vb)) / (2 * eps)
    an = np.real(np.vdot(adj["g_f"], va)) + np.real(np.vdot(adj["g_sh"], vb))
    assert abs(fd - an) <= 1e-6 * abs(an)
    vk = r.normal(size=p["nz"]) * 100.0
    fd = (L(dk_z=dk_z + eps * vk) - L(dk_z=dk_z - eps * vk)) / (2 * eps)
    an = float(np.dot(adj["g_dk"], vk))
    assert abs(fd - an) <= 1e-6 * abs(an)
    if with_temp:
        vt = r.normal(size=temp.shape)
        fd = (L(temp=temp + eps * vt) - L(temp=temp - eps * vt)) / (2 * eps)
        an = float(np.sum(adj["g_temp"] * vt))
        assert abs(fd - an) <= 1e-6 * abs(an)
        # the moments are the derivatives along (T - T_ref) and along a uniform shift
        dTs = temp - p["t_ref"]
        for k, v in enumerate((dTs, np.ones_like(temp))):
            fd = (L(temp=temp + eps * v) - L(temp=temp - eps * v)) / (2 * eps)
            assert abs(fd - adj["g_t_moments"][k]) <= 1e-6 * abs(fd)


def test_linear_step_adjoint_identity():
    p = params(n=16)
    c = ssfm.coefficients(p)
    m = ssfm.propagator(p, c.k_sh, p["alpha_sh"], c.dz)
    r = rng(3)
    x, y = crand(r, (16, 16), 1.0), crand(r, (16, 16), 1.0)
    lhs = np.vdot(y, ssfm.linear_step(x, m))
    rhs = np.vdot(ssfm.linear_step(y, np.conj(m)), x)
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)


def test_rhs_jacobian_against_differences():
    p = params()
    c = ssfm.coefficients(p)
    r = rng(9)
    y = r.normal(size=(4, 3, 3)) * 4e7
    e = np.exp(-1j * r.normal(size=(3, 3)))
    dT = r.normal(size=(3, 3))
    J = adjoint.rhs_jacobian(y, e, dT, c, False)
    for j in range(4):
        h = np.zeros_like(y)
        h[j] = 1e-3 * 4e7
        fd = (adjoint.rhs_real(y + h, e, dT, c, False) - adjoint.rhs_real(y - h, e, dT, c, False)) / (2 * h[j])
        assert np.max(np.abs(fd - J[:, j])) <= 1e-7 * np.max(np.abs(J[:, j]))


def test_mismatch_gradient_matches_focusing_integral():
    """Undepleted, lossless Gaussian: sum_s dP_SH/d dk_s from the adjoint equals
    d/d dk of the focusing-integral SH power (independent quadrature)."""
    lcr, xi = 10e-3, 1.0
    w0 = math.sqrt(lcr / (xi * 2 * math.pi * 2.14 / LAM))
    dk = -150.0
    base = dict(nx=64, ny=64, lx=12 * w0 * math.sqrt(2), ly=12 * w0 * math.sqrt(2), lcr=lcr,
                lambda_f=LAM, n_f=2.14, n_sh=2.18, d_eff=10e-12, alpha_f=0.0, alpha_sh=0.0,
                beta_f=0.0, beta_sh=0.0, dk0=dk, ddk_dT=0.0, dn_dT=0.0, t_ref=0.0, undepleted=True)
    grads = []
    for nz in (60, 120):
        p = dict(base, nz=nz)
        a0 = beams.input_pump(p, 1.0, w0, lcr / 2)
        zero = np.zeros_like(a0)
        adj = adjoint.adjoint(p, a0, zero, zero, zero, power_weights=(0.0, 1.0))
        grads.append(float(np.sum(adj["g_dk"])))
    g = (4 * grads[1] - grads[0]) / 3
    h = 1.0
    q = (pins.undepleted_sh_power(base, 1.0, w0, lcr / 2, dk + h)
         - pins.undepleted_sh_power(base, 1.0, w0, lcr / 2, dk - h)) / (2 * h)
    assert abs(g / q - 1) < 1e-5
