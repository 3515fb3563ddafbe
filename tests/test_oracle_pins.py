"""Pins of the FP64 oracle to what the paper and the physics fix (CPU only).

Each test names the reading of the paper it protects.  None of them compares
the oracle with itself: the expected values are closed forms, quadratures of
independent integrals, conservation laws, the paper's printed optimum, or a
brute-force re-implementation with naive DFT matrices and scalar loops.
"""
import json
import math
import os

import numpy as np
import pytest

import workloads
from oracle import ssfm, beams, pins

LAM = 1064e-9
NF, NSH = 2.14, 2.18
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")


def base_params(n=64, nz=100, lcr=10e-3, width=1e-3, **kw):
    p = dict(nx=n, ny=n, nz=nz, lx=width, ly=width, lcr=lcr, lambda_f=LAM, n_f=NF, n_sh=NSH,
             d_eff=10e-12, alpha_f=0.0, alpha_sh=0.0, beta_f=0.0, beta_sh=0.0, dk0=0.0,
             ddk_dT=0.0, dn_dT=0.0, t_ref=0.0, undepleted=False)
    p.update(kw)
    return p


def waist(lcr, xi, n=NF):
    return math.sqrt(lcr / (xi * 2 * math.pi * n / LAM))


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


# --------------------------------------------------------------------- P1
def test_free_gaussian_diffraction_matches_closed_form():
    """d = 0: the march must reproduce the Gaussian beam of the -(i/2k) lap
    convention (input sign reading of Eq. 6), waist at z = f and Gouy phase."""
    lcr, xi = 10e-3, 1.5
    w0 = waist(lcr, xi)
    wmax = w0 * math.sqrt(1 + xi * xi)
    p = base_params(n=128, nz=7, lcr=lcr, width=12 * wmax, d_eff=0.0)
    a0 = beams.input_pump(p, 2.0, w0, lcr / 2)
    out = ssfm.propagate(p, a0, np.zeros_like(a0))
    exact = beams.gaussian_field(p, 2.0, w0, lcr / 2, z=lcr)
    assert rel(out["a_f"], exact) < 1e-10
    # beam width at the focus equals w0: propagate to z = f
    pf = dict(p, nz=7, lcr=lcr / 2)
    outf = ssfm.propagate(pf, a0, np.zeros_like(a0))
    x, y = ssfm.coordinates(p)
    r2 = y[:, None] ** 2 + x[None, :] ** 2
    inten = np.abs(outf["a_f"]) ** 2
    w_meas = math.sqrt(2 * np.sum(r2 * inten) / np.sum(inten))
    assert abs(w_meas / w0 - 1) < 1e-10
    # the on-axis Gouy phase advances by arctan(tau) as 1/(1 - i tau) prescribes
    c = p["ny"] // 2, p["nx"] // 2
    dphase = np.angle(out["a_f"][c] / a0[c])
    assert abs(dphase - (math.atan(xi) - math.atan(-xi))) < 1e-9
    # the power of the discrete input equals the requested power on a wide window
    cf = ssfm.coefficients(p)
    assert abs(ssfm.power(a0, NF, cf.dx, cf.dy) / 2.0 - 1) < 1e-12


def test_printed_input_sign_diverges():
    """The literal Eq. 6 (1 - i xi) input is the conjugate beam: in the
    propagation convention of Eqs. 1-2 it widens monotonically instead of
    focusing at the crystal centre.  Guards against silently adopting it."""
    lcr, xi = 10e-3, 1.0
    w0 = waist(lcr, xi)
    p = base_params(n=128, nz=5, lcr=lcr / 2, width=20 * w0, d_eff=0.0)
    literal = np.conj(beams.input_pump(p, 1.0, w0, lcr / 2))
    out = ssfm.propagate(p, literal, np.zeros_like(literal))
    x, y = ssfm.coordinates(p)
    r2 = y[:, None] ** 2 + x[None, :] ** 2
    inten = np.abs(out["a_f"]) ** 2
    w_mid = math.sqrt(2 * np.sum(r2 * inten) / np.sum(inten))
    assert w_mid > 2.0 * w0      # literal: sqrt(5) w0 at z = L/2; corrected: w0


# --------------------------------------------------------------------- P2
def test_linear_absorption_exact():
    """alpha sits in the linear operator (Eq. 11): P(L) = P(0) exp(-alpha L)."""
    p = base_params(n=32, nz=13, width=0.4e-3, d_eff=0.0, alpha_f=7.0, alpha_sh=19.0)
    rng = np.random.Generator(np.random.PCG64(11))
    a = rng.normal(size=(32, 32)) + 1j * rng.normal(size=(32, 32))
    b = rng.normal(size=(32, 32)) + 1j * rng.normal(size=(32, 32))
    c = ssfm.coefficients(p)
    out = ssfm.propagate(p, a, b)
    assert abs(out["p_f"] / ssfm.power(a, NF, c.dx, c.dy) - math.exp(-7.0 * p["lcr"])) < 1e-13
    assert abs(out["p_sh"] / ssfm.power(b, NSH, c.dx, c.dy) - math.exp(-19.0 * p["lcr"])) < 1e-13


def uniform_amplitude(intensity, n):
    return math.sqrt(2 * intensity / (ssfm.EPS0 * ssfm.C_LIGHT * n))


# --------------------------------------------------------------------- P3
def test_two_photon_absorption_law():
    """TPA acts on intensity: dI/dz = -beta I^2 -> I0 / (1 + beta I0 z)."""
    beta, i0, lcr = 1e-12, 2e11, 20e-3   # beta I0 L = 4
    p = base_params(n=4, nz=400, lcr=lcr, d_eff=0.0, beta_f=beta, beta_sh=beta)
    a = np.full((4, 4), uniform_amplitude(i0, NF), complex)
    b = np.full((4, 4), uniform_amplitude(i0, NSH) * 1j, complex)
    out = ssfm.propagate(p, a, b)
    expect = pins.tpa_intensity(i0, beta, lcr)
    i_f = ssfm.EPS0 * ssfm.C_LIGHT * NF / 2 * abs(out["a_f"][0, 0]) ** 2
    i_sh = ssfm.EPS0 * ssfm.C_LIGHT * NSH / 2 * abs(out["a_sh"][0, 0]) ** 2
    assert abs(i_f / expect - 1) < 1e-10
    assert abs(i_sh / expect - 1) < 1e-10


# --------------------------------------------------------------------- P4
def test_plane_wave_tanh2_depletion():
    """Uniform pump, dk = 0, lossless: eta(L) = tanh^2(Gamma L) with
    Gamma^2 = 8 pi^2 d^2 I / (eps0 c n_F^2 n_SH lambda_F^2) (coupling reading)."""
    inten, lcr = 1e9, 0.1
    p = base_params(n=4, nz=200, lcr=lcr)
    a = np.full((4, 4), uniform_amplitude(inten, NF), complex)
    out = ssfm.propagate(p, a, np.zeros_like(a))
    eta = ssfm.efficiency(p, a, out)
    gam = pins.tanh2_gain(p, inten)
    assert abs(gam - 16.2228) < 1e-4
    assert abs(eta - math.tanh(gam * lcr) ** 2) < 1e-9
    assert eta > 0.8   # strongly depleted


# --------------------------------------------------------------------- P5
def manley_rowe_drift(monkeypatch=None, printed=False):
    lcr, xi = 10e-3, 1.0
    w0 = waist(lcr, xi)
    p = base_params(n=64, nz=800, lcr=lcr, width=12 * w0 * math.sqrt(2))
    a0 = beams.input_pump(p, 3e3, w0, lcr / 2)
    out = ssfm.propagate(p, a0, np.zeros_like(a0), trace=True)
    tot = out["trace_f"] + out["trace_sh"]
    c = ssfm.coefficients(p)
    p0 = ssfm.power(a0, NF, c.dx, c.dy)
    return float(np.max(np.abs(tot / p0 - 1))), float(out["trace_sh"][-1] / p0)


def test_manley_rowe_conservation():
    """Lossless depleted Gaussian: P_F + P_SH is conserved (up to RK4 truncation)."""
    drift, eta = manley_rowe_drift()
    assert eta > 0.3
    assert drift < 1e-10


def test_manley_rowe_detects_printed_sh_coupling(monkeypatch):
    """Planted mistake in the oracle (printed kSH with lambda_SH): conservation
    fails at the level of the efficiency, so the pin above has teeth."""
    orig = ssfm.coefficients

    def printed(p):
        c = orig(p)
        c.kappa_sh = 2 * math.pi * p["d_eff"] / (p["n_sh"] * p["lambda_f"] / 2)
        return c
    monkeypatch.setattr(ssfm, "coefficients", printed)
    drift, eta = manley_rowe_drift()
    assert drift > 0.1


# --------------------------------------------------------------------- P6/P7
def richardson_eta(p, power, w0, focus, nz):
    etas = []
    for k in (nz, 2 * nz):
        pp = dict(p, nz=k)
        a0 = beams.input_pump(pp, power, w0, focus)
        etas.append(ssfm.efficiency(pp, a0, ssfm.propagate(pp, a0, np.zeros_like(a0))))
    return (4 * etas[1] - etas[0]) / 3, etas


def test_boyd_kleinman_closed_form_sigma0():
    """Undepleted, lossless, n_SH = n_F, dk = 0: Eq. 17 with h = arctan^2(xi)/xi."""
    lcr, xi = 10e-3, 1.0
    w0 = waist(lcr, xi)
    p = base_params(n=64, lcr=lcr, width=12 * w0 * math.sqrt(1 + xi * xi), n_sh=NF,
                    undepleted=True)
    eta, etas = richardson_eta(p, 1.0, w0, lcr / 2, 100)
    bk = pins.bk_efficiency(p, 1.0, math.atan(xi) ** 2 / xi)
    assert abs(pins.bk_h(0.0, xi) - math.atan(xi) ** 2 / xi) < 1e-13
    assert abs(eta / bk - 1) < 1e-5
    # second-order convergence in dz
    assert abs(etas[1] / bk - 1) < abs(etas[0] / bk - 1) / 3.5


def test_boyd_kleinman_optimum_focusing():
    """Eq. 17 at the paper's optimum xi = 2.84 (Sec. 5.1): the focusing function
    peaks there, its maximum is BK's 1.068, and the march at dk = -sigma_m / z_R
    reproduces it; a mismatch of the opposite sign gives far less (sign reading
    of the mismatch)."""
    gold = json.load(open(GOLDEN))
    xs = np.linspace(2.6, 3.1, 51)
    hm = [pins.bk_h(pins.bk_sigma_opt(x), x) for x in xs]
    x_best = xs[int(np.argmax(hm))]
    assert abs(x_best - gold["xi_opt"]["value"]) <= gold["xi_opt"]["tolerance"]
    assert abs(max(hm) - gold["h_max"]["value"]) <= gold["h_max"]["tolerance"]
    xi, lcr = 2.84, 10e-3
    w0 = waist(lcr, xi)
    z_r = lcr / (2 * xi)
    sig = pins.bk_sigma_opt(xi)
    p = base_params(n=64, lcr=lcr, width=8 * w0 * math.sqrt(1 + xi * xi), n_sh=NF,
                    undepleted=True, dk0=-sig / z_r)
    eta, _ = richardson_eta(p, 1.0, w0, lcr / 2, 100)
    bk = pins.bk_efficiency(p, 1.0, pins.bk_h(sig, xi))
    assert abs(eta / bk - 1) < 1e-5
    p_wrong = dict(p, dk0=+sig / z_r, nz=100)
    a0 = beams.input_pump(p_wrong, 1.0, w0, lcr / 2)
    eta_wrong = ssfm.efficiency(p_wrong, a0, ssfm.propagate(p_wrong, a0, np.zeros_like(a0)))
    assert eta_wrong < 0.7 * bk


# --------------------------------------------------------------------- P8
def test_plane_wave_sinc2_phase():
    """Undepleted plane wave with dk != 0: A_SH(L) = i kSH a0^2 L e^{i dk L/2} sinc(dk L/2),
    which fixes the sign and integration of the mismatch phase (Eq. 3)."""
    lcr, dk = 10e-3, 700.0
    p = base_params(n=4, nz=300, lcr=lcr, dk0=dk, undepleted=True)
    a0 = uniform_amplitude(1e9, NF)
    a = np.full((4, 4), a0, complex)
    out = ssfm.propagate(p, a, np.zeros_like(a))
    expect = pins.undepleted_plane_wave_sh(p, a0, dk, lcr)
    assert abs(out["a_sh"][1, 2] / expect - 1) < 1e-9


def test_per_step_mismatch_equals_uniform():
    """A per-step dk profile equal to dk0 everywhere reproduces the uniform run."""
    lcr, dk = 10e-3, 300.0
    p = base_params(n=8, nz=30, width=0.3e-3, lcr=lcr, dk0=dk)
    rng = np.random.Generator(np.random.PCG64(5))
    a = (rng.normal(size=(8, 8)) + 1j * rng.normal(size=(8, 8))) * 3e6
    b = (rng.normal(size=(8, 8)) + 1j * rng.normal(size=(8, 8))) * 1e6
    u = ssfm.propagate(p, a, b)
    v = ssfm.propagate(dict(p, dk0=-5.0), a, b, dk_z=np.full(30, dk))
    assert rel(v["a_sh"], u["a_sh"]) < 1e-14


# --------------------------------------------------------------------- P9
def test_undepleted_focused_sh_with_dispersion():
    """k_SH != 2 k_F (every workload here): the march matches the 2-D focusing
    integral derived from Eqs. 1-2 and the Gaussian of Eq. 5 (config-1 beam)."""
    lcr, xi = 10e-3, 1.0
    w0 = waist(lcr, xi)
    p = base_params(n=64, lcr=lcr, width=12 * w0 * math.sqrt(1 + xi * xi), undepleted=True)
    eta, _ = richardson_eta(p, 1.0, w0, lcr / 2, 100)
    expect = pins.undepleted_sh_power(p, 1.0, w0, lcr / 2, 0.0)
    assert abs(expect - 6.4974e-3) < 1e-7
    assert abs(eta / expect - 1) < 1e-5


# --------------------------------------------------------------------- P10
def test_uniform_temperature_offset_only_rotates_phases():
    """Uniform T offset with d(dk)/dT = 0: the thermal-lens phases cancel in the
    coupling (g_SH = 2 g_F), so P_SH is unchanged and each field picks up
    exp(-i g_j dT L).  The residual is the RK4 truncation of the rotation, so it
    must fall as dz^4."""
    lcr, xi, dT = 10e-3, 1.0, 0.7
    w0 = waist(lcr, xi)
    errs = []
    for nz in (80, 160):
        p = base_params(n=32, nz=nz, lcr=lcr, width=10 * w0, dn_dT=1e-5, t_ref=300.0)
        a0 = beams.input_pump(p, 1.0, w0, lcr / 2)
        ref = ssfm.propagate(p, a0, np.zeros_like(a0))
        out = ssfm.propagate(p, a0, np.zeros_like(a0), temp=np.full((nz, 32, 32), 300.0 + dT))
        c = ssfm.coefficients(p)
        errs.append(abs(out["p_sh"] / ref["p_sh"] - 1))
        assert rel(out["a_f"], ref["a_f"] * np.exp(-1j * c.lens_f * dT * lcr)) < 1e-12
        assert rel(out["a_sh"], ref["a_sh"] * np.exp(-1j * c.lens_sh * dT * lcr)) < 2e-11
    assert errs[1] < 1e-11
    assert errs[0] / errs[1] > 12.0


# --------------------------------------------------------------------- P11
def test_quadratic_temperature_focuses_like_grin_lens():
    """T = T_ref - C r^2 with dn/dT > 0 is a graded-index lens: the beam follows
    the ABCD law of a quadratic medium (direction and strength of the thermal lens)."""
    lcr, xi = 20e-3, 0.5
    w0 = waist(lcr, xi)
    curv = 1e8                     # K / m^2
    p = base_params(n=128, nz=200, lcr=lcr, width=14 * w0 * math.sqrt(1 + xi * xi),
                    d_eff=0.0, dn_dT=1e-5, t_ref=300.0)
    x, y = ssfm.coordinates(p)
    r2 = y[:, None] ** 2 + x[None, :] ** 2
    temp = np.broadcast_to(300.0 - curv * r2, (200,) + r2.shape)
    a0 = beams.input_pump(p, 1.0, w0, lcr / 2)
    out = ssfm.propagate(p, a0, np.zeros_like(a0), temp=temp)
    expect = pins.grin_gaussian(p, 1.0, w0, lcr / 2, curv, lcr)
    free = beams.gaussian_field(p, 1.0, w0, lcr / 2, z=lcr)
    assert rel(out["a_f"], expect) < 1e-4
    assert rel(free, expect) > 0.1     # the lens is strong enough to matter


# --------------------------------------------------------------------- P12
def naive_dft2(a, inverse=False):
    ny, nx = a.shape
    sgn = 1 if inverse else -1
    fy = np.array([[np.exp(sgn * 2j * math.pi * j * k / ny) for k in range(ny)] for j in range(ny)])
    fx = np.array([[np.exp(sgn * 2j * math.pi * j * k / nx) for k in range(nx)] for j in range(nx)])
    out = fy @ a @ fx.T
    return out / (nx * ny) if inverse else out


def brute_force_march(p, a, b, temp=None):
    """Scalar re-implementation of the march from Eqs. 1-3, 11-14 and A.5."""
    lam_f = p["lambda_f"]
    k_f = 2 * math.pi * p["n_f"] / lam_f
    k_sh = 4 * math.pi * p["n_sh"] / lam_f
    kf = 2 * math.pi * p["d_eff"] / (p["n_f"] * lam_f)
    ksh = 2 * math.pi * p["d_eff"] / (p["n_sh"] * lam_f)
    e0c = ssfm.EPS0 * ssfm.C_LIGHT
    bf, bsh = p["beta_f"] * e0c * p["n_f"] / 2, p["beta_sh"] * e0c * p["n_sh"] / 2
    gf, gsh = 2 * math.pi * p["dn_dT"] / lam_f, 4 * math.pi * p["dn_dT"] / lam_f
    ny, nx, nz = p["ny"], p["nx"], p["nz"]
    dz = p["lcr"] / nz
    dx, dy = p["lx"] / nx, p["ly"] / ny

    def freq(m, n, d):
        return (m if m < (n + 1) // 2 else m - n) / (n * d)

    mf = np.empty((ny, nx), complex)
    msh = np.empty((ny, nx), complex)
    for j in range(ny):
        for i in range(nx):
            q2 = freq(i, nx, dx) ** 2 + freq(j, ny, dy) ** 2
            mf[j, i] = complex(math.cos(2 * math.pi ** 2 * q2 / k_f * dz),
                               math.sin(2 * math.pi ** 2 * q2 / k_f * dz)) * math.exp(-p["alpha_f"] * dz / 2)
            msh[j, i] = complex(math.cos(2 * math.pi ** 2 * q2 / k_sh * dz),
                                math.sin(2 * math.pi ** 2 * q2 / k_sh * dz)) * math.exp(-p["alpha_sh"] * dz / 2)
    a = a.astype(complex).copy()
    b = b.astype(complex).copy()
    phi = np.zeros((ny, nx))
    for s in range(nz):
        for j in range(ny):
            for i in range(nx):
                dT = 0.0 if temp is None else temp[s][j][i] - p["t_ref"]
                dk = (p["dk0"] + p["ddk_dT"] * dT + p.get("ddk_dT2", 0.0) * dT ** 2
                      + p.get("ddk_dT3", 0.0) * dT ** 3)

                def f(t, u, v):
                    ph = phi[j, i] + dk * t
                    e = complex(math.cos(ph), -math.sin(ph))
                    fu = 1j * kf * e * v * u.conjugate() - 0.5 * bf * abs(u) ** 2 * u - 1j * gf * dT * u
                    fv = 1j * ksh * e.conjugate() * u * u - 0.5 * bsh * abs(v) ** 2 * v - 1j * gsh * dT * v
                    return fu, fv

                def rk(t0, h, u, v):
                    k1 = f(t0, u, v)
                    k2 = f(t0 + h / 2, u + h / 2 * k1[0], v + h / 2 * k1[1])
                    k3 = f(t0 + h / 2, u + h / 2 * k2[0], v + h / 2 * k2[1])
                    k4 = f(t0 + h, u + h * k3[0], v + h * k3[1])
                    return (u + h / 6 * (k1[0] + 2 * k2[0] + 2 * k3[0] + k4[0]),
                            v + h / 6 * (k1[1] + 2 * k2[1] + 2 * k3[1] + k4[1]))
                a[j, i], b[j, i] = rk(0.0, dz / 2, a[j, i], b[j, i])
        a = naive_dft2(mf * naive_dft2(a), inverse=True)
        b = naive_dft2(msh * naive_dft2(b), inverse=True)
        for j in range(ny):
            for i in range(nx):
                dT = 0.0 if temp is None else temp[s][j][i] - p["t_ref"]
                dk = (p["dk0"] + p["ddk_dT"] * dT + p.get("ddk_dT2", 0.0) * dT ** 2
                      + p.get("ddk_dT3", 0.0) * dT ** 3)

                def f(t, u, v):
                    ph = phi[j, i] + dk * t
                    e = complex(math.cos(ph), -math.sin(ph))
                    fu = 1j * kf * e * v * u.conjugate() - 0.5 * bf * abs(u) ** 2 * u - 1j * gf * dT * u
                    fv = 1j * ksh * e.conjugate() * u * u - 0.5 * bsh * abs(v) ** 2 * v - 1j * gsh * dT * v
                    return fu, fv

                def rk(t0, h, u, v):
                    k1 = f(t0, u, v)
                    k2 = f(t0 + h / 2, u + h / 2 * k1[0], v + h / 2 * k1[1])
                    k3 = f(t0 + h / 2, u + h / 2 * k2[0], v + h / 2 * k2[1])
                    k4 = f(t0 + h, u + h * k3[0], v + h * k3[1])
                    return (u + h / 6 * (k1[0] + 2 * k2[0] + 2 * k3[0] + k4[0]),
                            v + h / 6 * (k1[1] + 2 * k2[1] + 2 * k3[1] + k4[1]))
                a[j, i], b[j, i] = rk(dz / 2, dz / 2, a[j, i], b[j, i])
                phi[j, i] += dk * dz
    return a, b


@pytest.mark.parametrize("shape,with_temp,cubic", [((4, 4), False, False), ((8, 4), False, False),
                                                  ((4, 8), True, False), ((4, 4), True, True)])
def test_tiny_grid_brute_force(shape, with_temp, cubic):
    ny, nx = shape
    p = base_params(n=4, nz=3, width=0.05e-3, lcr=1e-3, dk0=500.0, alpha_f=3.0, alpha_sh=5.0,
                    beta_f=1e-11, beta_sh=2e-11, ddk_dT=40.0, dn_dT=2e-4, t_ref=300.0)
    if cubic:
        p.update(ddk_dT2=-150.0, ddk_dT3=60.0)
    p.update(nx=nx, ny=ny, lx=0.05e-3 * nx / 4, ly=0.05e-3 * ny / 4)
    rng = np.random.Generator(np.random.PCG64(17))
    a = (rng.normal(size=shape) + 1j * rng.normal(size=shape)) * 4e7
    b = (rng.normal(size=shape) + 1j * rng.normal(size=shape)) * 2e7
    temp = 300.0 + rng.normal(size=(3,) + shape) if with_temp else None
    ba, bb = brute_force_march(p, a, b, temp)
    out = ssfm.propagate(p, a, b, temp=temp)
    assert rel(out["a_f"], ba) < 1e-13
    assert rel(out["a_sh"], bb) < 1e-13
    # the nonlinear terms matter at this amplitude
    lin = ssfm.propagate(dict(p, d_eff=0.0, beta_f=0.0, beta_sh=0.0), a, b, temp=temp)
    assert rel(lin["a_sh"], bb) > 1e-3


def test_grating_term_derivatives_at_25C_match_the_expansion():
    """-2 pi/Lambda(T) with Lambda = Lambda25 (1 + a u + b u^2), u = T - 25 C,
    has first derivative (2 pi/Lambda25) a and second derivative
    (2 pi/Lambda25)(2 b - 2 a^2) at u = 0 (calculus on Eq. 4).  The oracle's
    mismatch shift is checked by differences against both, with T_ref away
    from 25 C so that a wrong reference temperature fails, and its slope
    against differences of the shift over a range of temperatures."""
    a, b, lam = workloads.GRATING_A, workloads.GRATING_B, workloads.GRATING_PERIOD
    p = dict(ddk_dT=0.0, grating_period=lam, grating_a=a, grating_b=b, t_ref=330.0)
    g = 2 * math.pi / lam
    h = 0.5
    dT25 = ssfm.T_25C - p["t_ref"]
    f = lambda x: ssfm.thermal_mismatch(p, dT25 + x)
    d1 = (f(h) - f(-h)) / (2 * h)
    d2 = (f(h) - 2 * f(0.0) + f(-h)) / (h * h)
    assert abs(d1 / (g * a) - 1) < 1e-6
    assert abs(d2 / (g * (2 * b - 2 * a * a)) - 1) < 1e-4
    assert ssfm.thermal_mismatch(p, 3.0) > 0.0       # heating lengthens the period
    pc = dict(p, ddk_dT=40.0, ddk_dT2=-3.0, ddk_dT3=0.7)
    for dT in (-20.0, -1.0, 0.0, 2.5, 30.0):
        e = 1e-3
        fd = (ssfm.thermal_mismatch(pc, dT + e) - ssfm.thermal_mismatch(pc, dT - e)) / (2 * e)
        assert abs(fd - ssfm.thermal_mismatch_slope(pc, dT)) < 1e-6 * abs(fd)
    assert ssfm.thermal_mismatch(pc, 0.0) == 0.0


@pytest.mark.parametrize("dT,grating", [(-1.5, False), (0.8, False), (2.6, False), (2.6, True)])
def test_polynomial_mismatch_with_uniform_offset_equals_shifted_dk0(dT, grating):
    """A uniform temperature offset with no thermal lens (dn/dT = 0) only moves
    the phase mismatch, so the march with the cubic dk(T) must equal the
    temperature-free march at dk0 + c1 dT + c2 dT^2 + c3 dT^3.  The third case
    is chosen so that the shift cancels dk0 (phase matching restored by
    temperature tuning): there P_SH must reach the dk = 0 value, far above the
    mismatched one."""
    lcr, xi = 10e-3, 1.0
    w0 = waist(lcr, xi)
    c1, c2, c3 = 3000.0, -40.0, 9.0
    shift = lambda x: c1 * x + c2 * x * x + c3 * x * x * x
    extra = {}
    if grating:
        # a period 1 % too short at 25 C, tuned by temperature; the expansion
        # coefficients are scaled up so that the grating term dominates
        lam25, a, b = 8e-6, 3e-3, -2e-5
        extra = dict(grating_period=lam25, grating_a=a, grating_b=b)
        period = lambda T: lam25 * (1 + a * (T - 298.15) + b * (T - 298.15) ** 2)
        shift = lambda x, s0=shift: s0(x) + 2 * math.pi / period(300.0) - 2 * math.pi / period(300.0 + x)
    dk0 = -shift(2.6)
    p = base_params(n=32, nz=40, lcr=lcr, width=10 * w0, dk0=dk0, alpha_f=2.0, alpha_sh=4.0,
                    ddk_dT=c1, ddk_dT2=c2, ddk_dT3=c3, dn_dT=0.0, t_ref=300.0, **extra)
    a0 = beams.input_pump(p, 200.0, w0, lcr / 2)
    out = ssfm.propagate(p, a0, np.zeros_like(a0), temp=np.full((40, 32, 32), 300.0 + dT))
    shifted = dict(p, dk0=dk0 + shift(dT))
    ref = ssfm.propagate(shifted, a0, np.zeros_like(a0))
    assert rel(out["a_f"], ref["a_f"]) < 1e-12
    assert rel(out["a_sh"], ref["a_sh"]) < 1e-12
    if dT == 2.6:
        mismatched = ssfm.propagate(p, a0, np.zeros_like(a0))
        assert abs(shifted["dk0"]) < 1e-9
        assert out["p_sh"] > 20.0 * mismatched["p_sh"]


def test_resume_from_midpoint():
    """march(0 -> L) equals march(0 -> z_k) followed by march(z_k -> L)."""
    p = base_params(n=8, nz=20, width=0.3e-3, dk0=400.0, alpha_f=1.0)
    rng = np.random.Generator(np.random.PCG64(8))
    a = (rng.normal(size=(8, 8)) + 1j * rng.normal(size=(8, 8))) * 3e6
    b = np.zeros_like(a)
    full = ssfm.propagate(p, a, b)
    half = ssfm.propagate(p, a, b, s_end=9)
    rest = ssfm.propagate(p, half["a_f"], half["a_sh"], s_begin=9)
    assert rel(rest["a_sh"], full["a_sh"]) < 1e-14


# --------------------------------------------------------------------- walk-off
def test_walkoff_on_both_waves_is_an_exact_translation():
    """Spatial walk-off (the tan(rho) dA/dx term of the propagators, Sec. 4).
    With the same angle on both waves the coupled march is the rho = 0 march
    translated by tan(rho) z, since every other term is pointwise or
    translation invariant.  With tan(rho) dz = dx the translation is one sample
    per step, so the result must equal np.roll of the rho = 0 result, on a
    depleted march with mismatch, loss, TPA and a random input phase."""
    lcr, xi, n, nz = 10e-3, 2.0, 64, 24
    w0 = waist(lcr, xi)
    p0 = base_params(n=n, nz=nz, lcr=lcr, width=10 * w0 * math.sqrt(1 + xi * xi),
                     dk0=-150.0, alpha_f=0.5, alpha_sh=1.0, beta_f=1e-11, beta_sh=1e-11)
    rng = np.random.Generator(np.random.PCG64(21))
    a0 = beams.input_pump(p0, 2e3, w0, lcr / 2, 0.2 * rng.normal(size=(n, n)))
    b0 = 1e-3 * np.abs(a0).max() * (rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n)))
    ref = ssfm.propagate(p0, a0, b0)
    assert np.abs(ref["a_sh"]).max() > 1e-2 * np.abs(ref["a_f"]).max()   # real coupling
    dx, dz = p0["lx"] / n, lcr / nz
    rho = math.atan(dx / dz)
    out = ssfm.propagate(dict(p0, walkoff_f=rho, walkoff_sh=rho), a0, b0)
    for key in ("a_f", "a_sh"):
        assert rel(out[key], np.roll(ref[key], nz, axis=1)) < 1e-12, key
        # the opposite sign or a missing wave is far off
        assert rel(out[key], np.roll(ref[key], -nz, axis=1)) > 1e-2
    only_sh = ssfm.propagate(dict(p0, walkoff_sh=rho), a0, b0)
    assert rel(only_sh["a_sh"], out["a_sh"]) > 1e-2


def test_walkoff_moves_the_centroid_by_tan_rho_z():
    """One wave with walk-off, linear propagation (d = 0): its intensity centroid
    moves by tan(rho) L along +x (a non-integer number of samples); the other
    wave and the y centroid stay put; power is unchanged."""
    lcr, xi, n, nz = 10e-3, 1.0, 128, 10
    w0 = waist(lcr, xi)
    width = 16 * w0 * math.sqrt(1 + xi * xi)
    rho = math.atan(7.37 * (width / n) / lcr)          # 7.37 samples over the crystal
    p = base_params(n=n, nz=nz, lcr=lcr, width=width, d_eff=0.0, walkoff_sh=rho)
    a0 = beams.input_pump(p, 1.0, w0, lcr / 2)
    out = ssfm.propagate(p, a0, a0.copy())
    x, y = ssfm.coordinates(p)

    def centroid(f):
        i = np.abs(f) ** 2
        return float(np.sum(i * x[None, :]) / np.sum(i)), float(np.sum(i * y[:, None]) / np.sum(i))

    cx0, cy0 = centroid(a0)
    cxs, cys = centroid(out["a_sh"])
    cxf, cyf = centroid(out["a_f"])
    shift = math.tan(rho) * lcr
    assert 0.2 < (shift / (p["lx"] / n)) % 1.0 < 0.8    # not a whole number of samples
    assert abs((cxs - cx0) / shift - 1) < 1e-9
    assert abs(cys - cy0) < 1e-12 * p["ly"] and abs(cxf - cx0) < 1e-12 * p["lx"]
    c = ssfm.coefficients(p)
    assert abs(ssfm.power(out["a_sh"], 1.0, c.dx, c.dy) / ssfm.power(a0, 1.0, c.dx, c.dy) - 1) < 1e-12


# --------------------------------------------------------------------- split order
def lnl_case(nz, split, **kw):
    lcr, xi = 10e-3, 2.0
    w0 = waist(lcr, xi)
    p = base_params(n=32, nz=nz, lcr=lcr, width=10 * w0 * math.sqrt(1 + xi * xi), dk0=-120.0,
                    alpha_f=2.0, alpha_sh=5.0, beta_f=2e-11, beta_sh=2e-11, split=split)
    p.update(kw)
    a0 = beams.input_pump(p, 2e3, w0, lcr / 2)
    return p, a0


def test_split_orders_agree_to_second_order():
    """Sec. 3 calls L/2 - N - L/2 equivalent to the implemented N/2 - L - N/2:
    both are second-order Strang splittings of the same flow, so on a depleted,
    lossy march they differ by O(dz^2) (ratio ~4 per halving of dz), and each
    converges to the same limit."""
    diffs = []
    for nz in (50, 100):
        p, a0 = lnl_case(nz, "NLN")
        nln = ssfm.propagate(p, a0, np.zeros_like(a0))
        lnl = ssfm.propagate(dict(p, split="LNL"), a0, np.zeros_like(a0))
        c = ssfm.coefficients(p)
        assert nln["p_sh"] > 0.05 * ssfm.power(a0, NF, c.dx, c.dy)
        diffs.append(rel(lnl["a_sh"], nln["a_sh"]))
    assert 1e-5 < diffs[1] < 1e-2               # a real O(dz^2) splitting difference
    assert 3.8 < diffs[0] / diffs[1] < 4.2


def test_split_orders_coincide_without_nonlinearity():
    """With d = 0, no TPA and no temperature, N is the identity and both orders
    reduce to L^nz exactly."""
    p, a0 = lnl_case(12, "NLN", d_eff=0.0, beta_f=0.0, beta_sh=0.0)
    b0 = 0.3 * a0
    nln = ssfm.propagate(p, a0, b0)
    lnl = ssfm.propagate(dict(p, split="LNL"), a0, b0)
    assert rel(lnl["a_f"], nln["a_f"]) < 1e-13 and rel(lnl["a_sh"], nln["a_sh"]) < 1e-13


def test_lnl_conserves_energy_without_loss():
    """Manley-Rowe conservation for the L/2 - N - L/2 order (lossless, no TPA):
    the drift is RK4 truncation over the full step."""
    lcr, xi = 10e-3, 1.0
    w0 = waist(lcr, xi)
    p = base_params(n=64, nz=400, lcr=lcr, width=12 * w0 * math.sqrt(2), split="LNL")
    a0 = beams.input_pump(p, 3e3, w0, lcr / 2)
    out = ssfm.propagate(p, a0, np.zeros_like(a0), trace=True)
    c = ssfm.coefficients(p)
    p0 = ssfm.power(a0, NF, c.dx, c.dy)
    assert out["trace_sh"][-1] / p0 > 0.3
    assert np.max(np.abs((out["trace_f"] + out["trace_sh"]) / p0 - 1)) < 1e-9
