"""Pins of the FP64 heat-equation oracle and the self-consistent loop (CPU only).

Expected values are closed forms that the second-order finite-difference scheme
reproduces exactly (quadratic profiles), the discrete energy balance, the
second-order convergence to a manufactured solution, energy conservation of the
field march (absorbed = lost power), and fixed-point properties of the loop.
"""
import math

import numpy as np
import pytest

from oracle import beams, ssfm, thermal

LAM = 1064e-9


def grid(n=16, nz=12, lx=1e-3, ly=0.8e-3, lcr=5e-3):
    return dict(nx=n, ny=n, nz=nz, lx=lx, ly=ly, lcr=lcr)


def xs(p):
    x, y = ssfm.coordinates(dict(p, nx=p["nx"], ny=p["ny"]))
    z = np.arange(p["nz"] + 1) * p["lcr"] / p["nz"]
    return x, y, z


def test_slab_between_two_ovens_is_the_exact_parabola():
    """Uniform source, x faces on the oven, other faces insulated: T depends on x
    only and is q/(2k) (x - x0)(x1 - x) above T_oven, which a second-order
    scheme reproduces exactly."""
    p = grid()
    tp = thermal.ThermalParams(4.0, 0.0, 290.0, 330.0,
                               {"x-": "oven", "x+": "oven", "y-": "insulated", "y+": "insulated",
                                "z-": "insulated", "z+": "insulated"})
    q0 = 3e8
    t = thermal.solve(p, tp, np.full(thermal.grid_shape(p), q0))
    x, _, _ = xs(p)
    exact = tp.t_oven + q0 / (2 * tp.k_th) * (x - x[0]) * (x[-1] - x)
    rise = exact.max() - tp.t_oven
    assert rise > 1.0
    assert np.max(np.abs(t - exact[None, None, :])) < 1e-9 * rise


def test_convective_face_is_the_exact_parabola():
    """Oven at x-, convection to T_inf at x+, other faces insulated, uniform
    source: the quadratic T = T_oven + a s - q s^2 / (2k), s = x - x0, with
    -k T'(S) = h (T(S) - T_inf) at s = S, is exact for the scheme."""
    p = grid(n=32)
    k, h, t_inf, t_oven, q0 = 3.0, 4e3, 300.0, 340.0, 2e8
    tp = thermal.ThermalParams(k, h, t_inf, t_oven,
                               {"x-": "oven", "x+": "air", "y-": "insulated", "y+": "insulated",
                                "z-": "insulated", "z+": "insulated"})
    t = thermal.solve(p, tp, np.full(thermal.grid_shape(p), q0))
    x, _, _ = xs(p)
    s_face = x[-1] - x[0]
    # -k (a - q S / k) = h (t_oven + a S - q S^2 / (2k) - t_inf)
    a = (q0 * s_face - h * (t_oven - q0 * s_face ** 2 / (2 * k) - t_inf)) / (k + h * s_face)
    s = x - x[0]
    exact = t_oven + a * s - q0 * s ** 2 / (2 * k)
    assert np.ptp(exact) > 1.0
    assert np.max(np.abs(t - exact[None, None, :])) < 1e-9 * np.ptp(exact)
    # the opposite sign of the convective term would heat the face instead
    wrong = thermal.ThermalParams(k, -h, t_inf, t_oven, tp.faces)
    tw = thermal.solve(p, wrong, np.full(thermal.grid_shape(p), q0))
    assert np.max(np.abs(tw - exact[None, None, :])) > 1e-2 * np.ptp(exact)


@pytest.mark.parametrize("preset", ["bottom", "surrounding"])
def test_discrete_energy_balance(preset):
    """Heat generated inside equals the heat leaving through the air faces plus
    the heat conducted into the oven, for a random source."""
    p = grid(n=16, nz=10)
    make = thermal.bottom_oven if preset == "bottom" else thermal.surrounding_oven
    tp = make(5.0, 25.0, 295.0, 330.0)
    rng = np.random.Generator(np.random.PCG64(5))
    q = np.abs(rng.normal(size=thermal.grid_shape(p))) * 1e7
    t = thermal.solve(p, tp, q)
    src, loss = thermal.energy_balance(p, tp, t, q)
    assert abs(loss / src - 1) < 1e-9
    # with no source the oven feeds exactly what the air faces take away
    t0 = thermal.solve(p, tp, np.zeros_like(q))
    src0, loss0 = thermal.energy_balance(p, tp, t0, np.zeros_like(q))
    area = 2 * (p["lx"] * p["ly"] + (p["lx"] + p["ly"]) * p["lcr"])
    scale = tp.h_conv * (tp.t_oven - tp.t_inf) * area
    assert src0 == 0.0 and abs(loss0) < 1e-9 * scale


def test_second_order_convergence_to_a_manufactured_solution():
    """All faces on the oven; T = T_oven + A sin(pi s_x/Sx) sin(pi s_y/Sy)
    sin(pi z/L) with the matching source.  The error falls ~4x per halving."""
    k, amp, t_oven = 2.0, 1.5, 320.0
    errs = []
    box = 1e-3
    for n, nz in ((16, 8), (32, 16)):
        # the same physical box: the nodes span (n - 1) dx = box
        p = grid(n=n, nz=nz, lx=box * n / (n - 1), ly=box * n / (n - 1), lcr=2e-3)
        x, y, z = xs(p)
        sx, sy = x[-1] - x[0], y[-1] - y[0]
        tp = thermal.ThermalParams(k, 0.0, 300.0, t_oven, {f: "oven" for f in thermal.FACES})
        X = (x - x[0])[None, None, :]
        Y = (y - y[0])[None, :, None]
        Z = z[:, None, None]
        shape = np.sin(math.pi * X / sx) * np.sin(math.pi * Y / sy) * np.sin(math.pi * Z / p["lcr"])
        exact = t_oven + amp * shape
        q = k * amp * math.pi ** 2 * (1 / sx ** 2 + 1 / sy ** 2 + 1 / p["lcr"] ** 2) * shape
        t = thermal.solve(p, tp, q)
        errs.append(np.max(np.abs(t - exact)))
    assert errs[0] < 0.05 * amp
    assert 3.5 < errs[0] / errs[1] < 4.8        # spacings shrink by 31/15 (x, y) and 2 (z)


def field_case(n=32, nz=40, power=300.0, **kw):
    lcr, xi = 8e-3, 1.5
    w0 = math.sqrt(lcr / (xi * 2 * math.pi * 2.14 / LAM))
    width = 8 * w0 * math.sqrt(1 + xi * xi)
    p = dict(nx=n, ny=n, nz=nz, lx=width, ly=width, lcr=lcr, lambda_f=LAM, n_f=2.14, n_sh=2.18,
             d_eff=10e-12, alpha_f=3.0, alpha_sh=8.0, beta_f=5e-11, beta_sh=8e-11, dk0=-100.0,
             ddk_dT=0.0, dn_dT=0.0, t_ref=330.0, undepleted=False)
    p.update(kw)
    a0 = beams.input_pump(p, power, w0, lcr / 2)
    return p, a0, np.zeros_like(a0)


def test_heat_source_integrates_to_the_absorbed_power():
    """With loss the total power P_F + P_SH falls only by absorption, so the
    z-integral (trapezoid) of the deposited heat equals that fall to O(dz^2)."""
    p, a0, b0 = field_case()
    m = thermal.march_heat(p, a0, b0)
    c = ssfm.coefficients(p)
    p_in = ssfm.power(a0, p["n_f"], c.dx, c.dy)
    lost = p_in - (m["p_f"] + m["p_sh"])
    per_plane = m["q"].sum(axis=(1, 2)) * c.dx * c.dy
    absorbed = np.trapezoid(per_plane, dx=c.dz)
    assert m["p_sh"] > 1e-3 * p_in                       # SHG is active
    assert abs(absorbed / lost - 1) < 1e-3
    # the two-photon part matters at this intensity
    lin = thermal.heat_source(dict(p, beta_f=0.0, beta_sh=0.0), m["a_f"], m["a_sh"])
    assert np.max(np.abs(m["q"][-1] - lin)) > 1e-3 * np.max(lin)


def test_self_consistent_loop_stops_after_one_update_without_coupling():
    """If T does not act on the fields (no dk(T), no thermal lens), the second
    solve repeats the first exactly."""
    p, a0, b0 = field_case(n=16, nz=12)
    tp = thermal.bottom_oven(5.0, 20.0, 295.0, 330.0)
    t, _, hist = thermal.self_consistent(p, tp, a0, b0, tol=1e-12)
    assert len(hist) == 2 and hist[1] <= 1e-12 and hist[0] > 1e-3


def test_self_consistent_loop_reaches_a_fixed_point():
    """With dk(T) and the thermal lens on, the loop contracts and its result
    reproduces itself: solving with the heat of a march at T gives T back."""
    p, a0, b0 = field_case(n=16, nz=12, power=30.0, alpha_f=0.5, alpha_sh=3.0, ddk_dT=300.0,
                           dn_dT=1e-5)
    tp = thermal.bottom_oven(2.0, 20.0, 295.0, 330.0)
    t, march, hist = thermal.self_consistent(p, tp, a0, b0, tol=1e-9)
    assert hist[-1] <= 1e-9 and len(hist) >= 3
    assert all(b < a for a, b in zip(hist[1:], hist[2:]))
    again = thermal.solve(p, tp, thermal.march_heat(p, a0, b0, temp=thermal.midplanes(t))["q"])
    assert np.max(np.abs(again - t)) < 1e-8
    # the heat changed the march: compare with the march at the q = 0 field
    t0 = thermal.solve(p, tp, np.zeros(thermal.grid_shape(p)))
    m0 = thermal.march_heat(p, a0, b0, temp=thermal.midplanes(t0))
    assert abs(march["p_sh"] / m0["p_sh"] - 1) > 1e-6
