#!/usr/bin/env python3
"""Benchmark of the SSFM march on one MI355X.

Workload: the 256 x 256 grid, 1000 z-step, 30 mm, 30 W, xi = 2.84 march with
depleted pump, linear and two-photon absorption and input phase noise
(complex64).  One benchmark step is one whole march of that crystal (all
passes of every z-step, the mismatch-phase table and the exit powers), started
from the seeded input field that is resident in HBM.

Printed JSON line:
  value        cell-steps/s = nx * ny * nz * steps / wall time of the timed steps
  roofline     dominant kernel: algorithmic bytes per launch (both complex64
               fields read and written once, 32 B per cell) / its average launch
               duration in the timed march (the timed region per step, split
               between the row and column launches in the ratio of their
               kernel durations, which timing mode measures with a HIP event
               pair around every launch), against 8 TB/s
  cpu_baseline the FP64 oracle on a bounded sample of the same workload, one
               process per host core (and one process alone), with the CPU model
  extras       batched and forward+adjoint throughput when those paths run

    python bench.py [--gpus 1] [--steps 10] [--warmup 2]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "SSFM cell-steps/s (Nx·Ny·Nz/s) fwd, fwd+adjoint, batched; % HBM roofline"


# Sources that define the benchmarked kernels (row and column passes, their
# FFTs) and the host code that chooses and launches them; the committed HBM
# counters are valid while these are unchanged.
MARCH_SOURCES = ("fft.hpp", "kernels.hpp", "shg.hip")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2410_04994_amd", "csrc")
    for f in MARCH_SOURCES:
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, launch_bytes: float):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
    except ValueError:
        return None
    if rec.get("source_hash") != kernel_source_hash():
        return None
    ent = rec.get("kernels", {}).get(kernel)
    return None if ent is None else ent.get("bytes_per_launch")


# One oracle process of the CPU baseline.  argv: kind, steps, rank, processes.
# It times the oracle on its share of a bounded sample of one config and prints
# "<seconds> <cell-steps>" (imports and input set-up are not timed):
#   c2  the benchmark workload, first `steps` z-steps
#   c1  the 64 x 64 x 200 complex128 workload, whole crystal
#   c5  the 512 x 512 x 2000 temperature-field workload, first `steps` z-steps
#   c4  forward + adjoint (loss P_SH, per-step mismatch gradient) of the
#       differentiation workload's grid over a crystal of `steps` z-steps
#   c3  every `processes`-th instance of the first 64 of the batch sweep,
#       starting at `rank`, first `steps` z-steps each
_ORACLE_SAMPLE = """
import sys, time
sys.path.insert(0, {root!r})
import numpy as np
import workloads
from oracle import beams, ssfm, adjoint
kind, steps, rank, procs = sys.argv[1], int(sys.argv[2]), int(sys.argv[3]), int(sys.argv[4])
def inputs(wl):
    p = wl.params()
    th = workloads.phase_noise(wl) if wl.phase_noise_std else None
    a0 = beams.input_pump(p, wl.power, wl.w0, wl.focus, th)
    return p, a0, np.zeros_like(a0)
if kind == "c3":
    cases = [inputs(w) + (w.nx * w.ny * steps,) for w in workloads.c3_batch()[:64][rank::procs]]
    t = time.perf_counter()
    for p, a0, b0, _ in cases:
        ssfm.propagate(p, a0, b0, s_end=steps)
    print(time.perf_counter() - t, sum(c[3] for c in cases))
else:
    wl = {{"c1": workloads.c1_plain_fp64, "c2": workloads.c2_plain_c64,
           "c4": workloads.c4_diff_c64, "c5": workloads.c5_thermal_c64}}[kind]()
    if kind == "c4":
        wl = wl.with_(nz=steps)
    p, a0, b0 = inputs(wl)
    if kind == "c2":
        a0 = a0.astype(np.complex64)
    temp = workloads.RadialTemperature(wl) if kind == "c5" else None
    n = wl.nz if kind in ("c1", "c4") else steps
    t = time.perf_counter()
    if kind == "c4":
        adjoint.adjoint(p, a0, b0, np.zeros_like(a0), np.zeros_like(a0),
                        dk_z=np.full(n, wl.dk0), power_weights=(0.0, 1.0))
    else:
        ssfm.propagate(p, a0, b0, temp=temp, s_end=n)
    print(time.perf_counter() - t, wl.nx * wl.ny * n)
"""


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_cores() -> int:
    """Cores this process may run on, capped at the 16 a one-GPU share holds."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _oracle_runs(kind: str, steps: int, n: int):
    """n child processes of the oracle sample at once (ranks 0..n-1); returns
    [(seconds, cell_steps)] per process.  The children touch no GPU."""
    import subprocess
    code = _ORACLE_SAMPLE.format(root=ROOT)
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    procs = [subprocess.Popen([sys.executable, "-c", code, kind, str(steps), str(r), str(n)],
                              stdout=subprocess.PIPE, env=env, text=True) for r in range(n)]
    res = []
    for pr in procs:
        out, _ = pr.communicate()
        if pr.returncode != 0:
            raise RuntimeError(f"oracle sample process failed ({pr.returncode})")
        sec, cells = out.strip().splitlines()[-1].split()
        res.append((float(sec), int(cells)))
    return res


def _rate(runs):
    return round(sum(c for _, c in runs) / max(s for s, _ in runs), 1)


def cpu_baseline(wl, sample_steps: int, other_configs: bool = True):
    """Time the FP64 oracle (as it stands) on the first `sample_steps` z-steps
    of the workload: one process on one core, then one independent copy per
    host core at once (the oracle's FFTs and pointwise steps are single
    threaded, so independent marches are how it uses more cores).  With
    `other_configs`, bounded samples of the other configs as well: the batch
    sweep as a pool of processes over its instances, and the others on one
    core (and, for the temperature-field march, on every core)."""
    cores = host_cores()
    one = _oracle_runs("c2", sample_steps, 1)
    many = _oracle_runs("c2", sample_steps, cores)
    out = {"value": _rate(many), "unit": "cell-steps/s", "cores": cores, "kind": "oracle",
           "sample": (f"{wl.name}: first {sample_steps} of {wl.nz} z-steps per process, numpy "
                      f"FP64; {cores} independent processes at once (value: total cell-steps / "
                      f"slowest process)"),
           "single_core": {"value": _rate(one), "cores": 1, "seconds": round(one[0][0], 3)},
           "cpu_model": cpu_model(), "host_cpus_visible": os.cpu_count()}
    if other_configs:
        oc = {}
        r = _oracle_runs("c1", 0, 1)
        oc["c1_plain_fp64_64x64x200"] = {"value": _rate(r), "cores": 1, "sample": "whole crystal"}
        r = _oracle_runs("c3", 40, cores)
        oc["c3_batch"] = {"value": _rate(r), "cores": cores,
                          "sample": (f"first 64 of the 512 instances, first 40 z-steps each, over "
                                     f"{cores} processes (total cell-steps / slowest process)")}
        r = _oracle_runs("c4", 20, 1)
        oc["c4_diff_c64_fwd_adj"] = {"value": _rate(r), "cores": 1,
                                     "sample": ("forward + adjoint on the 256 x 256 grid over a "
                                                "20-step crystal")}
        r1 = _oracle_runs("c5", 10, 1)
        rn = _oracle_runs("c5", 10, cores)
        oc["c5_thermal_c64_512x512x2000"] = {
            "value": _rate(rn), "cores": cores, "single_core": _rate(r1),
            "sample": (f"first 10 of 2000 z-steps with the temperature field, one process and "
                       f"{cores} processes at once")}
        out["other_configs"] = oc
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-sample-steps", type=int, default=300)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-baseline-main-only", action="store_true",
                    help="time the oracle on the benchmark workload only")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--extras", default="",
                    help="comma-separated extra lines to run (default: all of "
                         "batched, fwd_adj, c5_forward, c1_complex128, thermal_fwd_adj, lnl, thermal, "
                         "self_consistent, latency_floor)")
    ap.add_argument("--progress", action="store_true",
                    help="print a line to stderr after each step of the extra lines "
                         "(for runs under a profiler)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 64 MiB device copy from a cache-cold source "
                         "(reference for the HBM byte counters)")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported: a single march "
              "does not shard (two all-to-alls per z-step would outweigh the step), and "
              "independent instances would shard by instance with no exchange",
              file=sys.stderr)
        return 2

    import torch
    import workloads
    from paper_2410_04994_amd import Plan, beams

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    from paper_2410_04994_amd import autotune
    dev = torch.device("cuda:0")
    wl = workloads.c2_plain_c64()
    plan = Plan(wl.params(), "c64")
    autotune.tune_single(plan)
    theta = torch.from_numpy(workloads.phase_noise(wl)).to(dev)
    a_in = beams.pump_for(wl, theta=theta, dtype=torch.complex64, device=dev)
    b_in = torch.zeros_like(a_in)
    a = torch.empty_like(a_in)
    b = torch.empty_like(b_in)
    ws = plan.workspace(device=dev)
    powers = torch.empty(2, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()

    def step():
        a.copy_(a_in)
        b.copy_(b_in)
        plan.propagate(a, b, workspace=ws, powers=powers, stream=stream)

    if args.calibrate_copy:
        src = torch.ones(16 << 20, dtype=torch.float32, device=dev)      # 64 MiB
        dst = torch.empty_like(src)
        evict = torch.ones(128 << 20, dtype=torch.float32, device=dev)   # 512 MiB > L2 + MALL
        evict.add_(1.0)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst, evict
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    ms_per_step = ms / args.steps
    value = wl.cell_steps * args.steps / (ms / 1e3)

    # per-kernel durations: timing mode brackets every launch of the same
    # march (same kernels and arguments, no graph) with a HIP event pair on
    # this stream; one march first, discarded, while the event pool fills
    plan.set_timing(True)
    step()
    plan.kernel_times()
    for _ in range(args.steps):
        step()
    kt = plan.kernel_times()
    plan.set_timing(False)
    row_k = kt["row_ms"] / max(1, kt["row_n"])
    col_k = kt["col_ms"] / max(1, kt["col_n"])
    # the graph-replayed march runs one row and one column launch per z-step
    # (plus one row launch): its per-launch time is the timed region per step,
    # split between the two kernels in the ratio of their kernel durations
    # (the two input copies, the phase table and the power reduction, about
    # 0.2 % of a march, are charged to the passes)
    launches = wl.nz + 1
    ratio = row_k / col_k
    col_avg = ms_per_step / (ratio * launches + wl.nz)
    row_avg = ratio * col_avg
    dom, avg_ms = ("row_pass", row_avg) if row_avg * launches >= col_avg * wl.nz else ("col_pass", col_avg)
    launch_bytes = 32.0 * wl.nx * wl.ny
    achieved = launch_bytes / (avg_ms * 1e-3) / 1e9
    traffic = measured_traffic(dom, launch_bytes)
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic, "kernel": dom, "avg_launch_us": round(avg_ms * 1e3, 3),
                "algorithmic_bytes_per_launch": int(launch_bytes),
                "row_pass_avg_us": round(row_avg * 1e3, 3), "col_pass_avg_us": round(col_avg * 1e3, 3),
                "launch_timing": ("timed graph-replayed march per step, split between the row and "
                                  "column launches in the ratio of their event-bracketed kernel "
                                  "durations"),
                "row_pass_kernel_us": round(row_k * 1e3, 3), "col_pass_kernel_us": round(col_k * 1e3, 3),
                "whole_march_frac_at_64B": round(value * 64.0 / (HBM_PEAK_GBS * 1e9), 4),
                "whole_march_frac_at_32B": round(value * 32.0 / (HBM_PEAK_GBS * 1e9), 4)}

    out = {"metric": METRIC, "value": round(value, 1), "unit": "cell-steps/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": wl.name, "grid": [wl.nx, wl.ny], "nz": wl.nz,
                      "crystal_m": wl.lcr, "power_W": wl.power, "xi": wl.xi,
                      "schedule": plan.describe()},
           "roofline": roofline}
    if not args.no_extras:
        try:
            from paper_2410_04994_amd import extras
            extras.PROGRESS = args.progress
            only = [x for x in args.extras.split(",") if x] or None
            out["extras"] = extras.run_all(dev, only)
            lf = out["extras"].get("latency_floor")
            if isinstance(lf, dict) and "two_pass_step_floor_us" in lf:
                step_us = ms_per_step * 1e3 / wl.nz
                lf["march_step_us"] = round(step_us, 3)
                lf["march_fraction_of_floor"] = round(lf["two_pass_step_floor_us"] / step_us, 4)
        except Exception as exc:  # extras must never hide the main line
            out["extras"] = {"error": f"{type(exc).__name__}: {exc}"}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_sample_steps,
                                           not args.cpu_baseline_main_only)
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
