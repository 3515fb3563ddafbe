"""torch.autograd wrapper of the HIP march and its hand-written adjoint.

    a_L, sh_L, powers = march(plan, a_f0, a_sh0, dk_z=None, temp=None)

Forward runs shg_propagate on copies of the inputs; backward runs
shg_propagate_adjoint (checkpointed forward + reverse march in the library)
seeded with the incoming gradients of the exit fields and of the exit powers.
Complex gradients follow torch's convention g = dL/dRe + i dL/dIm, the same as
the library's.  Gradients flow to a_f0, a_sh0, the per-step mismatch dk_z and,
through torch, to whatever built a_f0 (phase mask, waist, focus).
"""
from __future__ import annotations

import torch


class _March(torch.autograd.Function):
    @staticmethod
    def forward(ctx, plan, a_f, a_sh, dk_z, temp):
        a = a_f.detach().contiguous().clone()
        b = a_sh.detach().contiguous().clone()
        dk = dk_z.detach().contiguous() if dk_z is not None else None
        tt = temp.detach().contiguous() if temp is not None else None
        pw = plan.propagate(a, b, dk_z=dk, temp=tt)
        ctx.plan = plan
        ctx.has_dk = dk is not None
        ctx.has_t = tt is not None
        ctx.save_for_backward(a_f.detach().contiguous(), a_sh.detach().contiguous(),
                              dk if dk is not None else torch.empty(0),
                              tt if tt is not None else torch.empty(0))
        return a, b, pw

    @staticmethod
    def backward(ctx, g_a, g_b, g_pw):
        a_f, a_sh, dk, tt = ctx.saved_tensors
        dk = dk if ctx.has_dk else None
        tt = tt if ctx.has_t else None
        want_dk = ctx.has_dk and ctx.needs_input_grad[3]
        res = ctx.plan.adjoint(
            a_f, a_sh,
            g_f_out=g_a.contiguous() if g_a is not None else None,
            g_sh_out=g_b.contiguous() if g_b is not None else None,
            power_weights=g_pw.to(torch.float64).contiguous() if g_pw is not None else None,
            dk_z=dk, temp=tt, want_dk=want_dk)
        return None, res["g_f"], res["g_sh"], res.get("g_dk") if want_dk else None, None


def march(plan, a_f, a_sh, dk_z=None, temp=None):
    """Differentiable march over the whole crystal: (A_F(L), A_SH(L), powers[2])."""
    return _March.apply(plan, a_f, a_sh, dk_z, temp)


class _ThermalMarch(torch.autograd.Function):
    """Exit powers as a function of the scalars of T = t0 + scale * profile."""

    @staticmethod
    def forward(ctx, plan, a_f, a_sh, t0, scale, profile):
        temp = (t0.detach() + scale.detach() * profile).to(plan.real_dtype).contiguous()
        a = a_f.detach().contiguous().clone()
        b = a_sh.detach().contiguous().clone()
        pw = plan.propagate(a, b, temp=temp)
        ctx.plan = plan
        ctx.save_for_backward(a_f.detach().contiguous(), a_sh.detach().contiguous(), temp,
                              t0.detach(), scale.detach())
        return pw

    @staticmethod
    def backward(ctx, g_pw):
        a_f, a_sh, temp, t0, scale = ctx.saved_tensors
        plan = ctx.plan
        res = plan.adjoint(a_f, a_sh, power_weights=g_pw.to(torch.float64).contiguous(),
                           temp=temp, want_t=True)
        m1, m2 = res["g_t_moments"][0], res["g_t_moments"][1]
        t_ref = plan.params["t_ref"]
        # T - t_ref = (t0 - t_ref) + scale * profile
        g_scale = (m1 - (t0 - t_ref) * m2) / scale
        return None, res["g_f"], res["g_sh"], m2.to(t0.dtype), g_scale.to(scale.dtype), None


def thermal_powers(plan, a_f, a_sh, t0, scale, profile):
    """Exit powers [2] for the temperature field T = t0 + scale * profile
    ([nz, ny, nx] float64 profile); differentiable in a_f, a_sh, t0 and scale
    (scale must be non-zero)."""
    return _ThermalMarch.apply(plan, a_f, a_sh, t0, scale, profile)
