"""Seeded synthetic workloads for the SSFM hot path.

This module defines the physical parameter sets of the benchmark workloads and
draws every random number they need (input phase noise, batch instance
parameters).  It contains none of the method's arithmetic: no beam formula, no
propagator, no coupled-wave right-hand side.  Both the FP64 oracle and the HIP
path consume what it returns, so it is the only code the two sides share.

Units are SI throughout (m, W, rad/m, 1/m, m/W, K).

Workload shapes follow the paper's illustrative examples (Sec. 5.1, Example 1:
30 W pump, xi = 2.84, waist about 29 um, 30 mm crystal, 1064 nm -> 532 nm).
Material constants are the stated synthetic values (n_F = 2.14, n_SH = 2.18,
d_eff = 10 pm/V); the MgO:sPPLT dispersion data the paper cites are not used.
"""
from __future__ import annotations

import json
import math
import os
from dataclasses import dataclass, field, asdict, replace
from typing import List, Optional

import numpy as np

LAMBDA_F = 1064e-9      # fundamental vacuum wavelength [m]
N_F = 2.14              # refractive index at the fundamental
N_SH = 2.18             # refractive index at the second harmonic
D_EFF = 10e-12          # effective nonlinear coefficient [m/V]
ALPHA_F = 0.05          # 0.0005 /cm  -> 1/m (intensity absorption)
ALPHA_SH = 0.2          # 0.002 /cm   -> 1/m
BETA_TPA = 1e-12        # 0.1 cm/GW   -> m/W (two-photon absorption)
T_OVEN = 329.65         # 56.5 C, the oven temperature of the paper's Example 1 [K]
GRATING_A = 2.2e-6      # thermal expansion of the MgO:sPPLT poling period, Eq. 4 [1/K]
GRATING_B = -5.9e-9     # [1/K^2]
GRATING_PERIOD = 7.97e-6  # first-order period for 1064 -> 532 nm in PPLT at 25 C [m]; a
                          # stand-in, the paper gives no value

_HERE = os.path.dirname(os.path.abspath(__file__))


@dataclass
class Workload:
    """One SSFM instance: grid, crystal, beam and material parameters."""
    name: str
    nx: int
    ny: int
    nz: int
    lx: float
    ly: float
    lcr: float
    power: float            # pump power at z = 0 [W]
    xi: float               # focusing parameter L / (2 z_R)
    w0: float               # pump waist radius [m]
    focus: float            # focal position inside the crystal [m]
    lambda_f: float = LAMBDA_F
    n_f: float = N_F
    n_sh: float = N_SH
    d_eff: float = D_EFF
    alpha_f: float = 0.0
    alpha_sh: float = 0.0
    beta_f: float = 0.0
    beta_sh: float = 0.0
    dk0: float = 0.0
    ddk_dT: float = 0.0
    ddk_dT2: float = 0.0           # d2(dk)/dT2 / 2 [rad/(m K^2)]
    ddk_dT3: float = 0.0           # d3(dk)/dT3 / 6 [rad/(m K^3)]
    grating_period: float = 0.0    # poling period at 25 C [m]; 0 = no grating term in dk(T)
    grating_a: float = 0.0         # linear thermal expansion of the period [1/K]
    grating_b: float = 0.0         # quadratic thermal expansion of the period [1/K^2]
    dn_dT: float = 0.0
    t_ref: float = 0.0
    walkoff_f: float = 0.0         # spatial walk-off angle of the fundamental [rad]
    walkoff_sh: float = 0.0        # spatial walk-off angle of the SH [rad]
    split: str = "NLN"             # Strang order: "NLN" (the paper's) or "LNL"
    undepleted: bool = False
    phase_noise_std: float = 0.0   # std of the i.i.d. input phase mask [rad]
    seed: int = 0
    dtype: str = "c64"             # "c64" or "c128"
    detuning_K: float = 0.0        # batch: temperature detuning mapped onto dk0
    extra: dict = field(default_factory=dict)

    def params(self) -> dict:
        """Plain parameter dict understood by both the oracle and the binding."""
        keys = ("nx", "ny", "nz", "lx", "ly", "lcr", "lambda_f", "n_f", "n_sh", "d_eff",
                "alpha_f", "alpha_sh", "beta_f", "beta_sh", "dk0", "ddk_dT", "ddk_dT2", "ddk_dT3", "grating_period", "grating_a", "grating_b", "dn_dT",
                "t_ref", "walkoff_f", "walkoff_sh", "split", "undepleted")
        return {k: getattr(self, k) for k in keys}

    @property
    def cells(self) -> int:
        return self.nx * self.ny

    @property
    def cell_steps(self) -> int:
        return self.nx * self.ny * self.nz

    def with_(self, **kw) -> "Workload":
        return replace(self, **kw)


def waist_from_xi(lcr: float, xi: float, n_f: float = N_F, lambda_f: float = LAMBDA_F) -> float:
    """Waist that gives focusing parameter xi = L/(2 z_R) with z_R = k_F w0^2 / 2
    (definitions under Eqs. 5-6, Sec. 2.1).  Workload definition only."""
    k_f = 2.0 * math.pi * n_f / lambda_f
    return math.sqrt(lcr / (xi * k_f))


def rayleigh_range(lcr: float, xi: float) -> float:
    return lcr / (2.0 * xi)


def window_rule(w0: float, xi: float) -> float:
    """Full transverse window width: +-3 beam radii at the crystal faces."""
    return 6.0 * w0 * math.sqrt(1.0 + xi * xi)


_SIGMA_TABLE = None


def sigma_opt(xi: float) -> float:
    """Boyd-Kleinman optimum phase-mismatch parameter sigma_m(xi), linearly
    interpolated from the stored table sigma_opt_table.json (written by
    make_sigma_table.py from the oracle's focusing-function quadrature)."""
    global _SIGMA_TABLE
    if _SIGMA_TABLE is None:
        with open(os.path.join(_HERE, "sigma_opt_table.json")) as fh:
            tab = json.load(fh)
        _SIGMA_TABLE = (np.asarray(tab["xi"], float), np.asarray(tab["sigma_m"], float))
    xs, ss = _SIGMA_TABLE
    if not (xs[0] <= xi <= xs[-1]):
        raise ValueError(f"xi={xi} outside the tabulated range [{xs[0]}, {xs[-1]}]")
    return float(np.interp(xi, xs, ss))


def dk_optimum(lcr: float, xi: float) -> float:
    """Phase mismatch at the focusing-function optimum, in the sign convention of
    Eqs. 1-4 (phase e^{+i phi} drives the SH): dk = -sigma_m / z_R."""
    return -sigma_opt(xi) / rayleigh_range(lcr, xi)


def _base(name, n, nz, lcr, power, xi, window_factor=None, **kw) -> Workload:
    w0 = waist_from_xi(lcr, xi)
    width = window_rule(w0, xi) if window_factor is None else window_factor * w0
    return Workload(name=name, nx=n, ny=n, nz=nz, lx=width, ly=width, lcr=lcr,
                    power=power, xi=xi, w0=w0, focus=lcr / 2.0, **kw)


def c1_plain_fp64() -> Workload:
    """64x64 grid over a 4 w0 window, 200 steps, 10 mm, 1 W, xi = 1, dk = 0,
    lossless, SH zero at input; complex128 arithmetic."""
    return _base("c1_plain_fp64_64x64x200", 64, 200, 10e-3, 1.0, 1.0, window_factor=4.0,
                 dtype="c128")


def c2_plain_c64() -> Workload:
    """256x256, 1000 steps, 30 mm, 30 W, xi = 2.84, dk at the focusing optimum,
    depleted pump, linear + two-photon absorption, input phase noise N(0, 0.01 rad)."""
    lcr, xi = 30e-3, 2.84
    return _base("c2_plain_c64_256x256x1000", 256, 1000, lcr, 30.0, xi,
                 alpha_f=ALPHA_F, alpha_sh=ALPHA_SH, beta_f=BETA_TPA, beta_sh=BETA_TPA,
                 dk0=dk_optimum(lcr, xi), phase_noise_std=0.01, seed=2)


def c4_diff_c64() -> Workload:
    """256x256, 1000 steps, 20 mm, 10 W, xi = 2.84; gradient workload (phase mask
    N(0, 0.1 rad), per-step dk profile, checkpoints every 32 steps)."""
    lcr, xi = 20e-3, 2.84
    return _base("c4_diff_c64_256x256x1000", 256, 1000, lcr, 10.0, xi,
                 alpha_f=ALPHA_F, alpha_sh=ALPHA_SH, beta_f=BETA_TPA, beta_sh=BETA_TPA,
                 dk0=dk_optimum(lcr, xi), phase_noise_std=0.1, seed=4,
                 extra={"checkpoint_every": 32, "fd_directions": 64, "fd_seed": 40, "fd_h": 1e-3})


def c5_thermal_c64() -> Workload:
    """512x512, 2000 steps, 30 mm, 50 W, xi = 2.84, absorption as c2; synthetic
    temperature field T0 + dT(z) exp(-2 r^2 / w_T^2), dT(z) = 3 K exp(-alpha_SH z),
    w_T = 1.5 w0; d(dk)/dT = 2 rad/(m K), dn/dT = 1e-5 /K on both waves."""
    lcr, xi = 30e-3, 2.84
    return _base("c5_thermal_c64_512x512x2000", 512, 2000, lcr, 50.0, xi,
                 alpha_f=ALPHA_F, alpha_sh=ALPHA_SH, beta_f=BETA_TPA, beta_sh=BETA_TPA,
                 dk0=dk_optimum(lcr, xi), ddk_dT=2.0, dn_dT=1e-5, t_ref=T_OVEN,
                 extra={"t0": T_OVEN, "dT_peak": 3.0, "wT_over_w0": 1.5})


def open_top_oven() -> dict:
    """Thermal set-up of the paper's experiment (Sec. 2: the crystal's base on an
    oven at T_oven, the other faces in ambient air).  The paper gives neither
    the conductivity nor the convection coefficient; these are stand-ins of the
    right order for MgO:sPPLT in still air."""
    return dict(k_th=8.4, h_conv=10.0, t_inf=298.15, t_oven=T_OVEN, faces={"y-": "oven"})


def c3_batch(n_instances: int = 512, seed: int = 3) -> List[Workload]:
    """Batched sweep: sizes 64/128/256 in the ratio 1:2:1 (shuffled), per-instance
    nz ~ U{200..1000}, xi ~ U[0.5, 5], detuning ~ U[-2, 2] K mapped to
    dk = dk_opt(xi) + 2 rad/(m K) * detuning, power ~ U[1, 30] W; 30 mm crystal,
    absorption as c2, window rule as c2."""
    rng = np.random.Generator(np.random.PCG64(seed))
    q = n_instances // 4
    sizes = np.array([64] * q + [128] * (n_instances - 2 * q) + [256] * q)
    rng.shuffle(sizes)
    nzs = rng.integers(200, 1001, size=n_instances)
    xis = rng.uniform(0.5, 5.0, size=n_instances)
    dts = rng.uniform(-2.0, 2.0, size=n_instances)
    pws = rng.uniform(1.0, 30.0, size=n_instances)
    lcr = 30e-3
    out = []
    for i in range(n_instances):
        xi = float(xis[i])
        out.append(_base(f"c3_inst{i:03d}_{int(sizes[i])}", int(sizes[i]), int(nzs[i]), lcr,
                         float(pws[i]), xi, alpha_f=ALPHA_F, alpha_sh=ALPHA_SH,
                         beta_f=BETA_TPA, beta_sh=BETA_TPA,
                         dk0=dk_optimum(lcr, xi) + 2.0 * float(dts[i]),
                         detuning_K=float(dts[i]), seed=1000 + i))
    return out


def phase_noise(wl: Workload, std: Optional[float] = None, seed: Optional[int] = None) -> np.ndarray:
    """I.i.d. Gaussian phase mask theta[y, x] ~ N(0, std^2), float64, PCG64(seed)."""
    std = wl.phase_noise_std if std is None else std
    seed = wl.seed if seed is None else seed
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.normal(0.0, 1.0, size=(wl.ny, wl.nx)) * std


def random_complex(shape, seed: int, scale: float = 1.0) -> np.ndarray:
    """Complex128 array with i.i.d. N(0, scale^2) real and imaginary parts."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return (rng.normal(size=shape) + 1j * rng.normal(size=shape)) * scale


def random_real(shape, seed: int, scale: float = 1.0) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.normal(size=shape) * scale


def _radial_temperature_parts(wl: Workload):
    ex = wl.extra
    t0, peak, wt = ex["t0"], ex["dT_peak"], ex["wT_over_w0"] * wl.w0
    dx, dy, dz = wl.lx / wl.nx, wl.ly / wl.ny, wl.lcr / wl.nz
    x = (np.arange(wl.nx) - wl.nx // 2) * dx
    y = (np.arange(wl.ny) - wl.ny // 2) * dy
    r2 = y[:, None] ** 2 + x[None, :] ** 2
    zmid = (np.arange(wl.nz) + 0.5) * dz
    dT = peak * np.exp(-wl.alpha_sh * zmid)
    return t0, dT, np.exp(-2.0 * r2 / wt ** 2)


def radial_temperature_profile(wl: Workload) -> np.ndarray:
    """Synthetic midplane temperature samples T[s, y, x] (float64) for the
    thermal-lens workload: T0 + dT(z_s + dz/2) exp(-2 r^2 / w_T^2)."""
    t0, dT, g = _radial_temperature_parts(wl)
    return t0 + dT[:, None, None] * g[None, :, :]


class RadialTemperature:
    """The same samples as radial_temperature_profile, built one step plane at a
    time (T[s] is bitwise the plane s of the whole array), rounded to `dtype`
    when given: the [nz][ny][nx] field of the 512 x 512 x 2000 workload is
    2.1 GB in float32 and need not be held in float64."""

    def __init__(self, wl: Workload, dtype=None):
        self.t0, self.dT, self.g = _radial_temperature_parts(wl)
        self.dtype = dtype
        self.shape = (wl.nz, wl.ny, wl.nx)

    def __len__(self):
        return self.shape[0]

    def __getitem__(self, s: int) -> np.ndarray:
        plane = self.t0 + self.dT[s] * self.g
        return plane if self.dtype is None else plane.astype(self.dtype)

    def materialise(self, dtype=np.float32) -> np.ndarray:
        out = np.empty(self.shape, dtype)
        for s in range(self.shape[0]):
            out[s] = self[s]
        return out


CONFIGS = {
    "c1": c1_plain_fp64,
    "c2": c2_plain_c64,
    "c4": c4_diff_c64,
    "c5": c5_thermal_c64,
}
