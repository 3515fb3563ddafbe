"""Power trace along the crystal: P_F(z) and P_SH(z) at every k-th step
boundary, for conversion-efficiency curves eta(z) = P_SH(z) / P_F(0) and
Manley-Rowe checks (Sec. 2.2 powers).

The march runs in chunks of k steps through shg_propagate's step ranges; each
chunk returns the powers at its end.  A chunk boundary splits one row pass
between its two half-steps without changing any arithmetic, so the fields
after the last chunk are those of the one-shot march bit for bit.  The cost is
one extra row pass per chunk.
"""
from __future__ import annotations

from typing import Optional


def power_trace(plan, a_f, a_sh, every: int = 1, dk_z=None, temp=None, workspace=None,
                stream=None):
    """March a_f, a_sh (in place) over the whole crystal and return
    (z [m], powers [n, 2]) as device float64 tensors at z = k dz, 2k dz, ...,
    L (the last point is always L)."""
    from .binding import _torch
    torch = _torch()
    nz = int(plan.params["nz"])
    if every < 1:
        raise ValueError("every must be >= 1")
    ends = list(range(every, nz, every)) + [nz]
    dev = a_f.device
    out = torch.empty((len(ends), 2), dtype=torch.float64, device=dev)
    s0 = 0
    for i, s1 in enumerate(ends):
        plan.propagate(a_f, a_sh, dk_z=dk_z, temp=temp, s_begin=s0, s_end=s1, workspace=workspace,
                       powers=out[i], stream=stream)
        s0 = s1
    dz = float(plan.params["lcr"]) / nz
    z = torch.tensor([s * dz for s in ends], dtype=torch.float64, device=dev)
    return z, out
