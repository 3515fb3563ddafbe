"""Write the FP64 oracle references of the full-size parity tests.

    python tests/golden/make_full_size_refs.py [--jobs N] [--only NAME ...]

Imports only `oracle/` (the FP64 CPU oracle) and `workloads/` (seeded inputs);
nothing here comes from the HIP path.  Each output file under
tests/golden/full_size/ holds the oracle's results at the workload's full size
together with a fingerprint of its inputs, so a test can tell that it fed the
same seeded inputs to the GPU.

Inputs follow the tests' recipe: the pump from the oracle's beam builder (the
seeded phase mask where the workload has one), rounded to complex64; the
oracle consumes the rounded values.  Temperature samples are rounded to
float32 the same way.  Fields are stored rounded to complex64 (a relative
rounding of 6e-8, far below the 1e-4 parity bound); powers, gradients and
derivatives in float64.

References (name: workload, what is stored):
  c5_forward    512 x 512 x 2000 with the synthetic temperature field: exit
                fields and powers.
  c4_adjoint    256 x 256 x 1000, phase mask N(0, 0.1^2), dk(z) = dk_opt for
                every step: the oracle's reverse-mode gradient of P_SH(L) with
                respect to the input fields and to dk(z).
  c4_fd         the same workload: central differences (h = 1e-3) of the
                oracle's P_SH(L) along 64 random directions of (theta, dk(z))
                (seed 40; a dk direction is scaled by 1/(dz sqrt(nz)) so that
                it moves the accumulated phase by about h rad).
  c3_longest    the longest instance of each grid size of the 512-instance
                sweep: exit fields and powers.
  c5_adjoint    512 x 512 x 2000 with the temperature field: the oracle's
                temperature moments of dP_SH/dT (sum g_T (T - T_ref), sum g_T).
                About 25 GB of memory and two hours of one core.
"""
from __future__ import annotations

import argparse
import math
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads  # noqa: E402
from oracle import adjoint as oadj, beams, ssfm  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "full_size")


def pump(wl, theta=None) -> np.ndarray:
    """Seeded input pump rounded to complex64 (returned as complex128)."""
    th = workloads.phase_noise(wl) if (theta is None and wl.phase_noise_std) else theta
    a = beams.input_pump(wl.params(), wl.power, wl.w0, wl.focus, th)
    return a.astype(np.complex64).astype(np.complex128)


def fingerprint(a: np.ndarray) -> np.ndarray:
    """sum |a|^2 and the centre sample, to recognise the same inputs."""
    ny, nx = a.shape
    return np.array([float(np.sum(np.abs(a) ** 2)), a[ny // 2, nx // 2].real,
                     a[ny // 2, nx // 2].imag])


class RoundedTemperature:
    """Temperature planes rounded to float32, consumed by the oracle in FP64."""

    def __init__(self, wl):
        self.src = workloads.RadialTemperature(wl, np.float32)

    def __len__(self):
        return len(self.src)

    def __getitem__(self, s):
        return self.src[s].astype(np.float64)


def save(name: str, **arrays):
    os.makedirs(OUT, exist_ok=True)
    path = os.path.join(OUT, name + ".npz")
    np.savez_compressed(path, **arrays)
    print(f"wrote {path} ({os.path.getsize(path) / 1e6:.2f} MB)", flush=True)


def c5_forward():
    wl = workloads.c5_thermal_c64()
    a0 = pump(wl)
    t = time.time()
    ref = ssfm.propagate(wl.params(), a0, np.zeros_like(a0), temp=RoundedTemperature(wl))
    save("c5_forward", a_f=ref["a_f"].astype(np.complex64), a_sh=ref["a_sh"].astype(np.complex64),
         powers=np.array([ref["p_f"], ref["p_sh"]]), input=fingerprint(a0),
         seconds=np.array(time.time() - t))


def c4_adjoint():
    wl = workloads.c4_diff_c64()
    a0 = pump(wl)
    dk = np.full(wl.nz, wl.dk0)
    zero = np.zeros_like(a0)
    t = time.time()
    ref = oadj.adjoint(wl.params(), a0, zero, zero, zero, dk_z=dk, power_weights=(0.0, 1.0))
    fwd = ref["forward"]
    save("c4_adjoint", g_f=ref["g_f"].astype(np.complex64), g_sh=ref["g_sh"].astype(np.complex64),
         g_dk=ref["g_dk"], powers=np.array([fwd["p_f"], fwd["p_sh"]]), input=fingerprint(a0),
         seconds=np.array(time.time() - t))


def _c4_fd_one(j: int) -> float:
    """Central difference of the oracle's P_SH along direction j."""
    wl = workloads.c4_diff_c64()
    theta0 = workloads.phase_noise(wl)
    rng = np.random.Generator(np.random.PCG64(40))
    dz = wl.lcr / wl.nz
    h = 1e-3
    for _ in range(j + 1):
        v = rng.normal(size=(wl.ny, wl.nx))
        vk = rng.normal(size=wl.nz) / (dz * math.sqrt(wl.nz))
    dk0 = np.full(wl.nz, wl.dk0)
    p = wl.params()

    def p_sh(theta, dk):
        a = beams.input_pump(p, wl.power, wl.w0, wl.focus, theta)
        return ssfm.propagate(p, a, np.zeros_like(a), dk_z=dk)["p_sh"]

    return (p_sh(theta0 + h * v, dk0 + h * vk) - p_sh(theta0 - h * v, dk0 - h * vk)) / (2 * h)


def c4_fd(jobs: int):
    t = time.time()
    with ProcessPoolExecutor(jobs) as ex:
        fd = np.array(list(ex.map(_c4_fd_one, range(64))))
    save("c4_fd", fd=fd, h=np.array(1e-3), seed=np.array(40), seconds=np.array(time.time() - t))


def c3_longest():
    wls = workloads.c3_batch()
    out = {}
    t = time.time()
    for size in (64, 128, 256):
        idx = max((i for i, w in enumerate(wls) if w.nx == size), key=lambda i: (wls[i].nz, -i))
        w = wls[idx]
        a0 = pump(w)
        ref = ssfm.propagate(w.params(), a0, np.zeros_like(a0))
        out[f"index_{size}"] = np.array(idx)
        out[f"nz_{size}"] = np.array(w.nz)
        out[f"a_f_{size}"] = ref["a_f"].astype(np.complex64)
        out[f"a_sh_{size}"] = ref["a_sh"].astype(np.complex64)
        out[f"powers_{size}"] = np.array([ref["p_f"], ref["p_sh"]])
        out[f"input_{size}"] = fingerprint(a0)
        print(f"c3 instance {idx}: {size}x{size}x{w.nz}", flush=True)
    save("c3_longest", seconds=np.array(time.time() - t), **out)


def c5_adjoint():
    wl = workloads.c5_thermal_c64()
    a0 = pump(wl)
    temp = workloads.RadialTemperature(wl, np.float32).materialise(np.float32).astype(np.float64)
    zero = np.zeros_like(a0)
    t = time.time()
    ref = oadj.adjoint(wl.params(), a0, zero, zero, zero, temp=temp, power_weights=(0.0, 1.0))
    fwd = ref["forward"]
    save("c5_adjoint", g_t_moments=ref["g_t_moments"], g_dk=ref["g_dk"],
         powers=np.array([fwd["p_f"], fwd["p_sh"]]), input=fingerprint(a0),
         seconds=np.array(time.time() - t))


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--jobs", type=int, default=max(1, (os.cpu_count() or 2) - 1))
    ap.add_argument("--only", nargs="*", default=None,
                    help="subset of: c5_forward c4_adjoint c4_fd c3_longest c5_adjoint")
    args = ap.parse_args(argv)
    todo = args.only or ["c3_longest", "c5_forward", "c4_adjoint", "c4_fd"]
    for name in todo:
        print(f"== {name}", flush=True)
        if name == "c4_fd":
            c4_fd(args.jobs)
        else:
            globals()[name]()


if __name__ == "__main__":
    main()
