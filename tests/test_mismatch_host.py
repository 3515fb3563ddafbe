"""Host helpers that turn a temperature-dependent index model into the dk(T)
parameters of a plan (Eq. 4), checked against the oracle's per-cell mismatch."""
import math

import numpy as np
import pytest

import workloads
from oracle import ssfm
from paper_2410_04994_amd import mismatch

LAM = 1064e-9


def poly_indices(t_ref):
    # n_SH - n_F = 0.04 + 2e-5 u - 3e-8 u^2 + 4e-10 u^3, u = T - t_ref
    n_f = lambda T: 2.14 + 1e-5 * (T - t_ref) + 1e-8 * (T - t_ref) ** 2
    n_sh = lambda T: 2.18 + 3e-5 * (T - t_ref) - 2e-8 * (T - t_ref) ** 2 + 4e-10 * (T - t_ref) ** 3
    return n_f, n_sh


def test_cubic_is_exact_for_cubic_indices():
    t_ref = 330.0
    n_f, n_sh = poly_indices(t_ref)
    c = mismatch.dispersion_cubic(LAM, n_f, n_sh, t_ref)
    k = 4 * math.pi / LAM
    assert c["ddk_dT"] == pytest.approx(k * 2e-5, rel=1e-9)
    assert c["ddk_dT2"] == pytest.approx(k * -3e-8, rel=1e-7)
    assert c["ddk_dT3"] == pytest.approx(k * 4e-10, rel=1e-6)


def test_plan_parameters_reproduce_eq4_in_the_oracle():
    """dk0 + the oracle's per-cell shift with the fitted parameters equals
    dk(T) of Eq. 4 evaluated directly, grating term included."""
    t_ref = 329.65
    n_f, n_sh = poly_indices(t_ref)
    per = dict(period_25c=workloads.GRATING_PERIOD, a=workloads.GRATING_A, b=workloads.GRATING_B)
    p = mismatch.plan_parameters(LAM, n_f, n_sh, t_ref, **per)
    T = t_ref + np.linspace(-4.0, 4.0, 17)
    direct = mismatch.mismatch(T, LAM, n_f, n_sh, **per)
    cells = p["dk0"] + ssfm.thermal_mismatch(p, T - t_ref)
    assert np.max(np.abs(cells - direct)) < 1e-9 * np.max(np.abs(direct))
    # the grating term is there: without it dk(T) moves differently
    no_grating = mismatch.mismatch(T, LAM, n_f, n_sh)
    assert np.ptp(direct - no_grating) > 1.0


def test_smooth_index_model_is_fitted_within_its_span():
    """A non-polynomial index model: the cubic's error stays at the size of the
    fourth-order Taylor term over the fitted span."""
    t_ref = 330.0
    n_f = lambda T: 2.14 + 2e-5 * np.tanh((T - 300.0) / 40.0)
    n_sh = lambda T: 2.18 + 6e-5 * np.tanh((T - 300.0) / 40.0)
    c = mismatch.dispersion_cubic(LAM, n_f, n_sh, t_ref, span=5.0)
    T = t_ref + np.linspace(-5.0, 5.0, 101)
    exact = mismatch.mismatch(T, LAM, n_f, n_sh) - mismatch.mismatch(t_ref, LAM, n_f, n_sh)
    dT = T - t_ref
    fit = dT * (c["ddk_dT"] + dT * (c["ddk_dT2"] + dT * c["ddk_dT3"]))
    assert np.max(np.abs(fit - exact)) < 1e-3 * np.max(np.abs(exact))


def test_bad_span_rejected():
    n_f, n_sh = poly_indices(300.0)
    with pytest.raises(ValueError):
        mismatch.dispersion_cubic(LAM, n_f, n_sh, 300.0, span=0.0)
