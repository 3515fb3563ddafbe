"""Secondary benchmark lines reported beside the single-instance forward march:
the batched sweep (512 instances, sizes 64/128/256 in 1:2:1, nz in [200, 1000]),
forward + adjoint on the 256 x 256 x 1000 differentiation workload, the
512 x 512 x 2000 temperature-field march, the 64 x 64 x 200 complex128 march, the heat
equation for the heat of the 256 x 256 x 1000 march, and the self-consistent
field <-> temperature loop of the 50 W workload (512 x 512 x 2000)."""
from __future__ import annotations

import sys
import time

# When set, each finished repetition and line prints a line to stderr (for runs
# under a profiler, where a line can take minutes).
PROGRESS = False


def _progress(msg: str) -> None:
    if PROGRESS:
        print(f"extras: {msg}", file=sys.stderr, flush=True)


def _timed(fn, reps, torch):
    torch.cuda.synchronize()
    t = time.perf_counter()
    for i in range(reps):
        fn()
        if PROGRESS:
            torch.cuda.synchronize()
            _progress(f"repetition {i + 1}/{reps}")
    torch.cuda.synchronize()
    return (time.perf_counter() - t) / reps


def _adjoint_outputs(a, nz, torch):
    """Output buffers kept across timed adjoint calls (no allocation in the
    timed region)."""
    return {"g_f": torch.empty_like(a), "g_sh": torch.empty_like(a), "a_f": torch.empty_like(a),
            "a_sh": torch.empty_like(a), "powers": torch.empty(2, dtype=torch.float64, device=a.device),
            "g_dk": torch.empty(nz, dtype=torch.float64, device=a.device),
            "g_t_moments": torch.empty(2, dtype=torch.float64, device=a.device)}


def batched(device, reps=3, split="NLN"):
    import torch
    import workloads
    from paper_2410_04994_amd import Plan, propagate_batch, beams, autotune
    wls = [w.with_(split=split) for w in workloads.c3_batch()]
    plans = [Plan(w.params(), "c64") for w in wls]
    autotune.tune_batch(plans)
    # every instance's fields are views of one buffer per field, so that the
    # reset before each sweep is two launches rather than one per instance
    sizes = [w.nx * w.ny for w in wls]
    offs = [0]
    for n in sizes:
        offs.append(offs[-1] + n)
    a_in = torch.empty(offs[-1], dtype=torch.complex64, device=device)
    for w, o, n in zip(wls, offs, sizes):
        a_in[o:o + n].copy_(beams.pump_for(w, dtype=torch.complex64, device=device).reshape(-1))
    a_all = a_in.clone()
    b_all = torch.zeros_like(a_in)
    a = [a_all[o:o + n].view(w.ny, w.nx) for w, o, n in zip(wls, offs, sizes)]
    b = [b_all[o:o + n].view(w.ny, w.nx) for w, o, n in zip(wls, offs, sizes)]
    powers = torch.empty((len(wls), 2), dtype=torch.float64, device=device)

    def run():
        a_all.copy_(a_in)
        b_all.zero_()
        propagate_batch(plans, a, b, powers=powers)

    run()                      # direct run + graph capture
    run()
    _progress("batch warm-up done")
    sec = _timed(run, reps, torch)
    cells = sum(w.cell_steps for w in wls)
    scheds = sorted({p.describe().split("batch(")[1].split(")")[0] for p in plans})
    return {"workload": "c3_batch_512_mixed_64_128_256", "instances": len(wls), "schedules": scheds,
            "cell_steps": cells, "ms_per_sweep": round(sec * 1e3, 3),
            "cell_steps_per_s": round(cells / sec, 1),
            "frac_hbm_at_64B": round(cells / sec * 64 / 8e12, 4)}


def adjoint_bytes_per_cell_step(nz: int, k: int) -> float:
    """Algorithmic HBM bytes per cell-step of a complex64 forward + adjoint with
    checkpoints every k steps: forward 64 (two passes reading and writing both
    fields), staged state written once per step 16, the recomputed fraction of
    the forward 64 (every segment but the last, which the forward sweep stages
    itself), adjoint row pass (cotangent in and out 32, staged state in 16) and
    adjoint column pass 32, and a checkpoint of both fields per segment."""
    segs = -(-nz // k)
    last = nz - (segs - 1) * k
    recomputed = (nz - last) / nz
    return 64 + 16 + 64 * recomputed + 48 + 32 + 16 * segs / nz


def c5_forward(device, reps=3):
    """The 512 x 512 x 2000 temperature-field march (forward only): reported at
    the 68 B/cell-step convention (64 B of fields plus one 4 B read of T per
    step) and at the bytes this implementation moves (each T plane is read by
    the two row passes around its step, 8 B, and the per-cell phase Psi is read
    and written once per step, 8 B: 80 B)."""
    import torch
    import workloads
    from paper_2410_04994_amd import Plan, beams, autotune
    wl = workloads.c5_thermal_c64()
    plan = Plan(wl.params(), "c64")
    autotune.tune_single(plan)
    temp = torch.from_numpy(workloads.RadialTemperature(wl, "float32").materialise()).to(device)
    a_in = beams.pump_for(wl, dtype=torch.complex64, device=device)
    a = torch.empty_like(a_in)
    b = torch.zeros_like(a_in)
    ws = plan.workspace(device=device)
    pw = torch.empty(2, dtype=torch.float64, device=device)

    def run():
        a.copy_(a_in)
        b.zero_()
        plan.propagate(a, b, temp=temp, workspace=ws, powers=pw)

    run()
    sec = _timed(run, reps, torch)
    rate = wl.cell_steps / sec
    return {"workload": wl.name, "schedule": plan.describe(), "ms": round(sec * 1e3, 3),
            "cell_steps_per_s": round(rate, 1), "frac_hbm_at_68B": round(rate * 68 / 8e12, 4),
            "frac_hbm_at_80B": round(rate * 80 / 8e12, 4)}


def c1_complex128(device, reps=20):
    """The 64 x 64 x 200 lossless march in complex128 (FP64 arithmetic),
    reported at 128 B/cell-step (the 64 B convention with 16-byte values)."""
    import torch
    import workloads
    from paper_2410_04994_amd import Plan, beams
    wl = workloads.c1_plain_fp64()
    plan = Plan(wl.params(), "c128")
    a_in = beams.pump_for(wl, dtype=torch.complex128, device=device)
    a = torch.empty_like(a_in)
    b = torch.zeros_like(a_in)
    ws = plan.workspace(device=device)
    pw = torch.empty(2, dtype=torch.float64, device=device)

    def run():
        a.copy_(a_in)
        b.zero_()
        plan.propagate(a, b, workspace=ws, powers=pw)

    run()
    sec = _timed(run, reps, torch)
    rate = wl.cell_steps / sec
    return {"workload": wl.name, "schedule": plan.describe(), "ms": round(sec * 1e3, 4),
            "cell_steps_per_s": round(rate, 1), "frac_hbm_at_128B": round(rate * 128 / 8e12, 5)}


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

    out = _adjoint_outputs(a0, wl.nz, torch)

    def run():
        plan.adjoint(a0, b0, power_weights=w, dk_z=dk, want_dk=True, workspace=ws, out=out)

    run()
    sec = _timed(run, reps, torch)
    k = int(plan.describe().split(" K=")[1].split(")")[0])
    nbytes = adjoint_bytes_per_cell_step(wl.nz, k)
    out = {"workload": wl.name, "schedule": plan.describe(), "workspace_MB": round(ws.numel() / 2**20, 1),
           "cell_steps": wl.cell_steps, "ms_per_fwd_adj": round(sec * 1e3, 3),
           "cell_steps_per_s": round(wl.cell_steps / sec, 1),
           "bytes_per_cell_step": round(nbytes, 2),
           "frac_hbm": round(wl.cell_steps / sec * nbytes / 8e12, 4),
           "frac_hbm_at_224B": round(wl.cell_steps / sec * 224 / 8e12, 4)}
    # checkpoints every 32 steps, each segment recomputed in the reverse sweep
    plan32 = Plan(wl.params(), "c64", checkpoint_every=32)
    autotune.tune_single(plan32)
    ws32 = plan32.workspace(adjoint=True, device=device)

    def run32():
        plan32.adjoint(a0, b0, power_weights=w, dk_z=dk, want_dk=True, workspace=ws32, out=out)

    run32()
    sec32 = _timed(run32, reps, torch)
    nb32 = adjoint_bytes_per_cell_step(wl.nz, 32)
    out["k32"] = {"schedule": plan32.describe(), "workspace_MB": round(ws32.numel() / 2**20, 1),
                  "ms_per_fwd_adj": round(sec32 * 1e3, 3),
                  "cell_steps_per_s": round(wl.cell_steps / sec32, 1),
                  "bytes_per_cell_step": round(nb32, 2),
                  "frac_hbm": round(wl.cell_steps / sec32 * nb32 / 8e12, 4),
                  "frac_hbm_at_224B": round(wl.cell_steps / sec32 * 224 / 8e12, 4)}
    return out


def thermal_fwd_adj(device, reps=2):
    """Forward + adjoint of the 512 x 512 x 2000 temperature-field workload
    with the temperature moments (the gradients in dT scale and T0), automatic
    checkpoint interval."""
    import torch
    import workloads
    from paper_2410_04994_amd import Plan, beams, autotune
    wl = workloads.c5_thermal_c64()
    plan = Plan(wl.params(), "c64")
    autotune.tune_single(plan)
    temp = torch.from_numpy(workloads.radial_temperature_profile(wl).astype("float32")).to(device)
    a0 = beams.pump_for(wl, dtype=torch.complex64, device=device)
    b0 = torch.zeros_like(a0)
    w = torch.tensor([0.0, 1.0], dtype=torch.float64, device=device)
    ws = plan.workspace(adjoint=True, device=device)

    out = _adjoint_outputs(a0, wl.nz, torch)

    def run():
        plan.adjoint(a0, b0, power_weights=w, temp=temp, want_t=True, workspace=ws, out=out)

    run()
    sec = _timed(run, reps, torch)
    return {"workload": wl.name, "schedule": plan.describe(), "workspace_MB": round(ws.numel() / 2**20, 1),
            "cell_steps": wl.cell_steps, "ms_per_fwd_adj": round(sec * 1e3, 3),
            "cell_steps_per_s": round(wl.cell_steps / sec, 1)}


FP64_MFMA_PEAK = 78.6e12
HBM_PEAK = 8.0e12


TRI_BYTES_PER_NODE = 48    # z sweep: read f; write d', c'; read d', c'; write u (FP64)


def _direct_work(nx, ny, nzn, faces):
    """Algorithmic work of one direct solve: flops of the four FP64 GEMM mode
    products (x and y, forward and backward) and bytes of the tridiagonal
    sweep along z, over the packed free nodes."""
    def free(n, lo, hi):
        return n - (faces.get(lo) == "oven") - (faces.get(hi) == "oven")
    m = [free(nx, "x-", "x+"), free(ny, "y-", "y+"), free(nzn, "z-", "z+")]
    prod = m[0] * m[1] * m[2]
    return 2 * 2 * (m[0] + m[1]) * prod, TRI_BYTES_PER_NODE * prod


def _heat_of_march(wl, device):
    import torch
    import workloads
    from paper_2410_04994_amd import Plan, beams, autotune
    plan = Plan(wl.params(), "c64")
    autotune.tune_single(plan)
    theta = torch.from_numpy(workloads.phase_noise(wl)).to(device) if wl.phase_noise_std else None
    a = beams.pump_for(wl, theta=theta, dtype=torch.complex64, device=device)
    b = torch.zeros_like(a)
    heat, _ = plan.propagate_heat(a, b)
    return heat


def thermal(device, reps=3):
    """Heat equation (open-top oven) for the heat source of a march.
      direct  diagonalisation in x and y (FP64 GEMM mode products on MFMA) and
              tridiagonal solves along z (HBM-bound); its bound is the GEMM flops
              at the FP64 MFMA peak plus the sweep's bytes at the HBM peak (the
              set-up, once per plan, is timed apart)
      cg      Jacobi-PCG to a relative residual of 1e-6 from a cold start;
              convention 40 B per node and iteration"""
    import torch
    import workloads
    from paper_2410_04994_amd import Thermal
    setup = workloads.open_top_oven()
    out = {}
    for wl in (workloads.c2_plain_c64(), workloads.c5_thermal_c64()):
        heat = _heat_of_march(wl, device)
        nodes = wl.nx * wl.ny * (wl.nz + 1)
        th = Thermal(wl.params(), dtype="c64", method="direct", **setup)
        th.workspace(device)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        t, _, _, res = th.solve(heat)
        torch.cuda.synchronize()
        first = time.perf_counter() - t0
        t0 = time.perf_counter()
        for _ in range(reps):
            t, _, _, res = th.solve(heat)
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / reps
        flops, tri_bytes = _direct_work(wl.nx, wl.ny, wl.nz + 1, setup["faces"])
        bound = flops / FP64_MFMA_PEAK + tri_bytes / HBM_PEAK
        out[f"direct_{wl.nx}x{wl.ny}x{wl.nz + 1}"] = {
            "nodes": nodes, "ms": round(sec * 1e3, 3), "first_solve_ms": round(first * 1e3, 2),
            "residual": res, "gemm_flops": flops, "tri_bytes": tri_bytes,
            "bound_ms": round(bound * 1e3, 3), "frac_of_bound": round(bound / sec, 4),
            "t_max_rise_K": round(float(t.max()) - workloads.T_OVEN, 4)}
        del th, t
    wl = workloads.c2_plain_c64()
    heat = _heat_of_march(wl, device)
    th = Thermal(wl.params(), dtype="c64", method="cg", **setup)
    th.workspace(device)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, iters, res = th.solve(heat, tol=1e-6, max_iter=40000)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    nodes = wl.nx * wl.ny * (wl.nz + 1)
    out[f"cg_{wl.nx}x{wl.ny}x{wl.nz + 1}"] = {
        "iterations": iters, "residual": res, "ms": round(sec * 1e3, 2),
        "node_iterations_per_s": round(nodes * iters / sec, 1),
        "frac_hbm_at_40B": round(nodes * iters / sec * 40 / 8e12, 4)}
    return out


def self_consistent_loop(device):
    """Self-consistent loop of the 50 W temperature-field workload (512 x 512 x
    2000, dk(T), thermal lens, open-top oven, direct solver) until the largest
    change of T is below 1 mK."""
    import torch
    import workloads
    from paper_2410_04994_amd import Plan, Thermal, beams, autotune, self_consistent
    wl = workloads.c5_thermal_c64()
    plan = Plan(wl.params(), "c64")
    autotune.tune_single(plan)
    a0 = beams.pump_for(wl, dtype=torch.complex64, device=device)
    b0 = torch.zeros_like(a0)
    th = Thermal(wl.params(), dtype="c64", **workloads.open_top_oven())
    th.workspace(device)
    # the same march at the uniform oven temperature, for comparison
    a_u, b_u = a0.clone(), b0.clone()
    p_u = plan.propagate(a_u, b_u)
    # the first loop includes the solver set-up (x and y eigendecompositions,
    # first BLAS use) and the capture of the temperature-field march; the
    # second shows the steady cost
    times = []
    for _ in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = self_consistent(plan, th, a0, b0, tol_t=1e-3, max_outer=20, solve_tol=1e-6,
                              max_iter=40000)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    sec = times[1]
    # exit powers of a march at the converged temperature field
    p_sc = plan.propagate(a0.clone(), b0.clone(), temp=out["t_mid"])
    return {"workload": wl.name, "marches": out["outer"], "last_change_K": out["change"],
            "ms": round(sec * 1e3, 1), "first_loop_ms": round(times[0] * 1e3, 1), "t_max_rise_K": round(float(out["t_nodes"].max()) - workloads.T_OVEN, 4),
            "p_sh_uniform_oven_W": round(float(p_u[1]), 5), "p_sh_self_consistent_W": round(float(p_sc[1]), 5)}


def lnl(device, steps=5):
    """The L/2 - N - L/2 order (one RK4 over dz per step): the 256 x 256 x 1000
    march, the batched sweep and the forward + adjoint of the differentiation
    workload, to compare with the N/2 - L - N/2 lines."""
    import torch
    import workloads
    from paper_2410_04994_amd import Plan, beams, autotune
    wl = workloads.c2_plain_c64().with_(split="LNL")
    plan = Plan(wl.params(), "c64")
    autotune.tune_single(plan)
    theta = torch.from_numpy(workloads.phase_noise(wl)).to(device)
    a_in = beams.pump_for(wl, theta=theta, dtype=torch.complex64, device=device)
    a = torch.empty_like(a_in)
    b = torch.zeros_like(a_in)
    ws = plan.workspace(device=device)

    def run():
        a.copy_(a_in)
        b.zero_()
        plan.propagate(a, b, workspace=ws)

    run()
    sec = _timed(run, steps, torch)
    out = {"single": {"workload": wl.name + "_lnl", "ms": round(sec * 1e3, 3),
                      "cell_steps_per_s": round(wl.cell_steps / sec, 1)}}
    res = batched(device, split="LNL")
    out["batched"] = {k: res[k] for k in ("ms_per_sweep", "cell_steps_per_s", "frac_hbm_at_64B")}
    # forward + adjoint of the differentiation workload in this order
    wd = workloads.c4_diff_c64().with_(split="LNL")
    pd = Plan(wd.params(), "c64")
    autotune.tune_single(pd)
    a0 = beams.pump_for(wd, theta=torch.from_numpy(workloads.phase_noise(wd)).to(device),
                        dtype=torch.complex64, device=device)
    b0 = torch.zeros_like(a0)
    dk = torch.full((wd.nz,), wd.dk0, dtype=torch.float64, device=device)
    w = torch.tensor([0.0, 1.0], dtype=torch.float64, device=device)
    wsa = pd.workspace(adjoint=True, device=device)

    out_adj = _adjoint_outputs(a0, wd.nz, torch)

    def run_adj():
        pd.adjoint(a0, b0, power_weights=w, dk_z=dk, want_dk=True, workspace=wsa, out=out_adj)

    run_adj()
    sec = _timed(run_adj, 2, torch)
    out["fwd_adj"] = {"workload": wd.name + "_lnl", "ms_per_fwd_adj": round(sec * 1e3, 3),
                      "cell_steps_per_s": round(wd.cell_steps / sec, 1)}
    return out


def latency_floor(device, launches=2000, reps=3):
    """A measured floor for the 256 x 256 single-instance march: any design
    with two device-wide exchanges per z-step launches (at least) two kernels
    per step, each of which reads and writes the whole state (both complex64
    fields, 1 MiB) once.  Timed with plain library kernels replayed from a
    HIP graph, like the march: a launch that touches one element (the launch
    gap alone) and a launch that adds a constant to the whole state in place
    (the gap plus one read and one write of the state from the Infinity Cache,
    where the march's state lives between passes)."""
    import torch
    state = torch.zeros(2 * 256 * 256 * 2, dtype=torch.float32, device=device)
    tiny = torch.zeros(1, dtype=torch.float32, device=device)

    def per_launch_us(t):
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            for _ in range(3):
                t.add_(1.0)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            for _ in range(launches):
                t.add_(1.0)
        g.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            g.replay()
        torch.cuda.synchronize()
        us = (time.perf_counter() - t0) / (reps * launches) * 1e6
        del g
        return us

    gap = per_launch_us(tiny)
    rw = per_launch_us(state)
    return {"graph_launch_one_element_us": round(gap, 3), "graph_launch_state_rw_us": round(rw, 3),
            "two_pass_step_floor_us": round(2 * rw, 3),
            "note": ("floor of a z-step with two device-wide exchanges at 256 x 256: two "
                     "graph-replayed launches that each read and write the 1 MiB state once")}


def run_all(device, only=None) -> dict:
    """Every extra line, or those named in `only`."""
    lines = (("batched", batched), ("fwd_adj", fwd_adj), ("c5_forward", c5_forward),
             ("c1_complex128", c1_complex128), ("thermal_fwd_adj", thermal_fwd_adj),
             ("lnl", lnl), ("thermal", thermal), ("self_consistent", self_consistent_loop),
             ("latency_floor", latency_floor))
    known = [name for name, _ in lines]
    unknown = [x for x in (only or []) if x not in known]
    if unknown:
        raise ValueError(f"unknown extra lines {unknown}; known: {known}")
    out = {}
    for name, fn in lines:
        if only is not None and name not in only:
            continue
        try:
            out[name] = fn(device)
        except Exception as exc:
            out[name] = {"error": f"{type(exc).__name__}: {exc}"}
        _progress(f"{name} done")
    return out
