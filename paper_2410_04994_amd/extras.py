"""Secondary benchmark lines reported beside the single-instance forward march:
the batched sweep (512 instances, sizes 64/128/256 in 1:2:1, nz in [200, 1000])
and forward + adjoint on the 256 x 256 x 1000 differentiation workload."""
from __future__ import annotations

import time


def _timed(fn, reps, torch):
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t) / reps


def batched(device, reps=3):
    import torch
    import workloads
    from paper_2410_04994_amd import Plan, propagate_batch, beams, autotune
    wls = workloads.c3_batch()
    plans = [Plan(w.params(), "c64") for w in wls]
    autotune.tune_batch(plans)
    a_in = [beams.pump_for(w, dtype=torch.complex64, device=device) for w in wls]
    a = [x.clone() for x in a_in]
    b = [torch.zeros_like(x) for x in a_in]
    powers = torch.empty((len(wls), 2), dtype=torch.float64, device=device)

    def run():
        for x, y, z in zip(a, a_in, b):
            x.copy_(y)
            z.zero_()
        propagate_batch(plans, a, b, powers=powers)

    run()                      # direct run + graph capture
    run()
    sec = _timed(run, reps, torch)
    cells = sum(w.cell_steps for w in wls)
    scheds = sorted({p.describe().split("batch(")[1].split(")")[0] for p in plans})
    return {"workload": "c3_batch_512_mixed_64_128_256", "instances": len(wls), "schedules": scheds,
            "cell_steps": cells, "ms_per_sweep": round(sec * 1e3, 3),
            "cell_steps_per_s": round(cells / sec, 1),
            "frac_hbm_at_64B": round(cells / sec * 64 / 8e12, 4)}


def fwd_adj(device, reps=2):
    import torch
    import workloads
    from paper_2410_04994_amd import Plan, beams, autotune
    wl = workloads.c4_diff_c64()
    plan = Plan(wl.params(), "c64")     # default K: every step staged when it fits
    autotune.tune_single(plan)
    theta = torch.from_numpy(workloads.phase_noise(wl)).to(device)
    a0 = beams.pump_for(wl, theta=theta, dtype=torch.complex64, device=device)
    b0 = torch.zeros_like(a0)
    dk = torch.full((wl.nz,), wl.dk0, dtype=torch.float64, device=device)
    w = torch.tensor([0.0, 1.0], dtype=torch.float64, device=device)
    ws = plan.workspace(adjoint=True, device=device)

    def run():
        plan.adjoint(a0, b0, power_weights=w, dk_z=dk, want_dk=True, workspace=ws)

    run()
    sec = _timed(run, reps, torch)
    return {"workload": wl.name, "schedule": plan.describe(), "workspace_MB": round(ws.numel() / 2**20, 1),
            "cell_steps": wl.cell_steps, "ms_per_fwd_adj": round(sec * 1e3, 3),
            "cell_steps_per_s": round(wl.cell_steps / sec, 1),
            "frac_hbm_at_224B": round(wl.cell_steps / sec * 224 / 8e12, 4)}


def run_all(device) -> dict:
    out = {}
    for name, fn in (("batched", batched), ("fwd_adj", fwd_adj)):
        try:
            out[name] = fn(device)
        except Exception as exc:
            out[name] = {"error": f"{type(exc).__name__}: {exc}"}
    return out
