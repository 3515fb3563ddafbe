"""Launch-schedule autotuner.

A schedule is (row_e, row_wg, col_e, col_tc): elements per thread of the row
transforms (row_e = 1 selects the wide row pass), threads per row block,
elements per thread of the column transforms and columns per column block.
The tuner times the candidates that the library has built for a grid on short
probe marches and keeps the fastest:

  single instance  wall time of a probe march (min(nz, probe_steps) steps)
  batch            throughput of a probe batch of the same grid (up to 32
                   instances, probe_steps steps each)

Results are cached in a JSON file ($SHG_AUTOTUNE_CACHE, default
~/.cache/shg_autotune.json) keyed by device architecture, dtype, mode and grid,
so a tuned grid is timed once per machine.  A table tuned on MI355X for the
standard grids ships with the package (tuned_mi355x.json) and is consulted
after the user cache; regenerate it on the device with

    python -m paper_2410_04994_amd.autotune --write-packaged
"""
from __future__ import annotations

import json
import os
import time
from typing import Callable, Dict, List, Optional, Sequence, Tuple

Sched = Tuple[int, int, int, int]

ROW_CANDIDATES = [(1, 256), (1, 512), (4, 64), (4, 256), (8, 64), (8, 256), (16, 64)]
COL_CANDIDATES = [(e, tc) for e in (4, 8, 16) for tc in (1, 2, 4, 8, 16)]


PACKAGED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_mi355x.json")


def cache_path() -> str:
    return os.environ.get("SHG_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "shg_autotune.json"))


def load_cache(path: Optional[str] = None) -> Dict[str, list]:
    path = path or cache_path()
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def lookup(key: str) -> Optional[list]:
    """User cache first, then the packaged table."""
    user = load_cache()
    if key in user:
        return user[key]
    return load_cache(PACKAGED).get(key)


def store_cache(cache: Dict[str, list], path: Optional[str] = None) -> None:
    path = path or cache_path()
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(cache, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def cache_key(arch: str, dtype: str, mode: str, nx: int, ny: int) -> str:
    return f"{arch}|{dtype}|{mode}|{nx}x{ny}"


def device_arch() -> str:
    import torch
    return getattr(torch.cuda.get_device_properties(0), "gcnArchName", "unknown").split(":")[0]


def candidates(try_set: Callable[[Sched], bool]) -> List[Sched]:
    """Schedules accepted by the library (try_set returns False when the
    library reports SHG_EUNSUPPORTED)."""
    out = []
    for re_, rw in ROW_CANDIDATES:
        for ce, ct in COL_CANDIDATES:
            s = (re_, rw, ce, ct)
            if try_set(s):
                out.append(s)
    return out


def pick_fastest(scheds: Sequence[Sched], measure: Callable[[Sched], float]) -> Tuple[Sched, float]:
    """Lowest measured cost; ties keep the earlier candidate."""
    best, best_t = None, float("inf")
    for s in scheds:
        t = measure(s)
        if t < best_t:
            best, best_t = s, t
    if best is None:
        raise RuntimeError("no schedule could be measured")
    return best, best_t


def _set_ok(fn, s: Sched) -> bool:
    from .binding import ShgError
    try:
        fn(*s)
        return True
    except ShgError:
        return False


def tune_single(plan, probe_steps: int = 48, reps: int = 3, cache: bool = True) -> Sched:
    """Choose and set the fastest single-instance schedule of `plan`."""
    import torch
    p = plan.params
    key = cache_key(device_arch(), plan.dtype, "single", p["nx"], p["ny"])
    hit = lookup(key) if cache else None
    if hit is not None and _set_ok(plan.set_schedule, tuple(hit)):
        return tuple(hit)
    steps = min(p["nz"], probe_steps)
    a = torch.zeros((p["ny"], p["nx"]), dtype=plan.complex_dtype, device="cuda")
    a.fill_(1.0e6)
    b = torch.zeros_like(a)

    def measure(s: Sched) -> float:
        plan.set_schedule(*s)
        plan.propagate(a, b, s_end=steps)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            plan.propagate(a, b, s_end=steps)
        torch.cuda.synchronize()
        return time.perf_counter() - t

    best, _ = pick_fastest(candidates(lambda s: _set_ok(plan.set_schedule, s)), measure)
    plan.set_schedule(*best)
    if cache:
        table = load_cache()
        table[key] = list(best)
        store_cache(table)
    return best


def tune_batch(plans, probe_steps: int = 40, probe_count: int = 32, reps: int = 2,
               cache: bool = True) -> Dict[Tuple[int, int], Sched]:
    """Choose and set the fastest in-batch schedule for every grid of `plans`."""
    import torch
    from .binding import Plan, propagate_batch
    chosen: Dict[Tuple[int, int], Sched] = {}
    groups: Dict[Tuple[int, int], list] = {}
    for pl in plans:
        groups.setdefault((pl.params["nx"], pl.params["ny"]), []).append(pl)
    arch = device_arch()
    for (nx, ny), members in groups.items():
        dtype = members[0].dtype
        key = cache_key(arch, dtype, "batch", nx, ny)
        hit = lookup(key) if cache else None
        if hit is not None and all(_set_ok(pl.set_batch_schedule, tuple(hit)) for pl in members):
            chosen[(nx, ny)] = tuple(hit)
            continue
        probe = [Plan(dict(pl.params, nz=min(pl.params["nz"], probe_steps)), dtype)
                 for pl in members[:probe_count]]
        a = [torch.full((ny, nx), 1.0e6, dtype=probe[0].complex_dtype, device="cuda") for _ in probe]
        b = [torch.zeros_like(x) for x in a]

        def measure(s: Sched) -> float:
            for pl in probe:
                pl.set_batch_schedule(*s)
            propagate_batch(probe, a, b)
            propagate_batch(probe, a, b)
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(reps):
                propagate_batch(probe, a, b)
            torch.cuda.synchronize()
            return time.perf_counter() - t

        best, _ = pick_fastest(candidates(lambda s: _set_ok(probe[0].set_batch_schedule, s)), measure)
        for pl in members:
            pl.set_batch_schedule(*best)
        chosen[(nx, ny)] = best
        if cache:
            table = load_cache()
            table[key] = list(best)
            store_cache(table)
    return chosen


def write_packaged(sizes=(16, 32, 64, 128, 256, 512), dtypes=("c64",),
                   path: Optional[str] = None) -> Dict[str, list]:
    """Tune every standard grid on this device (no caches consulted) and write
    the table (default: the packaged one)."""
    import workloads
    from .binding import Plan
    out: Dict[str, list] = {}
    arch = device_arch()
    base = workloads.c2_plain_c64()
    for dt in dtypes:
        for n in sizes:
            wl = base.with_(nx=n, ny=n, nz=200, lx=base.lx * n / 256, ly=base.ly * n / 256)
            plan = Plan(wl.params(), dt)
            out[cache_key(arch, dt, "single", n, n)] = list(tune_single(plan, cache=False))
            plans = [Plan(wl.params(), dt) for _ in range(max(8, min(64, 2 ** 20 // (n * n))))]
            best = tune_batch(plans, cache=False)[(n, n)]
            out[cache_key(arch, dt, "batch", n, n)] = list(best)
            print(dt, n, out[cache_key(arch, dt, "single", n, n)], best, flush=True)
    store_cache(out, path or PACKAGED)
    return out


if __name__ == "__main__":
    import sys
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    if "--write-packaged" in sys.argv:
        i = sys.argv.index("--write-packaged")
        dest = sys.argv[i + 1] if len(sys.argv) > i + 1 else None
        write_packaged(path=dest)
