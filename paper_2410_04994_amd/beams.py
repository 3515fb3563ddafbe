"""Input-beam builder on the GPU (torch), differentiable in power, waist and
focus so that gradients of the SH power reach the focusing through autograd.

Focused Gaussian pump at the crystal entrance (Sec. 2.1, Eqs. 5-6), written in
the propagation convention of the coupled-wave equations (-(i/2k) lap):
    A_F(x, y, 0) = A0 / q exp(-r^2 / (w0^2 q)),  q = 1 + i f / z_R,
    z_R = k_F w0^2 / 2,  k_F = 2 pi n_F / lambda_F,
    A0 = sqrt(4 P / (pi w0^2 eps0 c n_F))   (so that int eps0 c n |A|^2 / 2 dA = P).
The printed Eq. 6 carries the conjugate q, which in this convention is a beam
diverging from a virtual focus in front of the crystal.
"""
from __future__ import annotations

import math

EPS0 = 8.8541878128e-12
C_LIGHT = 299792458.0


def grid_coords(n: int, width: float, torch, device, dtype):
    d = width / n
    return (torch.arange(n, device=device, dtype=dtype) - n // 2) * d


def gaussian_pump(nx: int, ny: int, lx: float, ly: float, power, w0, focus, n_f: float,
                  lambda_f: float, theta=None, dtype=None, device="cuda"):
    """Complex [ny, nx] pump field; power, w0 and focus may be 0-d tensors with
    requires_grad.  theta: optional [ny, nx] phase mask (radians)."""
    import torch
    dtype = torch.complex64 if dtype is None else dtype
    rdt = torch.float64
    x = grid_coords(nx, lx, torch, device, rdt)
    y = grid_coords(ny, ly, torch, device, rdt)
    r2 = y[:, None] ** 2 + x[None, :] ** 2
    power = torch.as_tensor(power, dtype=rdt, device=device)
    w0 = torch.as_tensor(w0, dtype=rdt, device=device)
    focus = torch.as_tensor(focus, dtype=rdt, device=device)
    k = 2.0 * math.pi * n_f / lambda_f
    z_r = k * w0 * w0 / 2.0
    q = torch.complex(torch.ones_like(z_r), focus / z_r)
    a0 = torch.sqrt(4.0 * power / (math.pi * w0 * w0 * EPS0 * C_LIGHT * n_f))
    field = (a0 / q) * torch.exp(-r2.to(torch.complex128) / (w0 * w0 * q))
    if theta is not None:
        th = torch.as_tensor(theta, device=device).to(rdt)
        field = field * torch.polar(torch.ones_like(th), th)
    return field.to(dtype)


def pump_for(wl, theta=None, dtype=None, device="cuda", power=None, w0=None, focus=None):
    """Pump of a workloads.Workload (optionally overriding power/w0/focus)."""
    return gaussian_pump(wl.nx, wl.ny, wl.lx, wl.ly, wl.power if power is None else power,
                         wl.w0 if w0 is None else w0, wl.focus if focus is None else focus,
                         wl.n_f, wl.lambda_f, theta=theta, dtype=dtype, device=device)
