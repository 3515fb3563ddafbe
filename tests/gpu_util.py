"""Helpers shared by the GPU tests: run the HIP path and the oracle on the same
seeded inputs and compare them."""
import numpy as np

import workloads
from oracle import ssfm, beams

TOL_FIELD_C64 = 1e-4     # relative L2 field error, complex64 path vs FP64 oracle
TOL_ETA_C64 = 1e-5       # relative error of the conversion efficiency / powers
TOL_FIELD_C128 = 1e-12   # complex128 path: same algorithm, FP64 arithmetic
TOL_ETA_C128 = 1e-12


def rel(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))


def inputs(wl: workloads.Workload, dtype="c64", theta=True):
    """Seeded input fields, rounded to the GPU precision (the oracle consumes the
    rounded values, so input rounding is not charged to parity)."""
    p = wl.params()
    th = workloads.phase_noise(wl) if (theta and wl.phase_noise_std) else None
    a0 = beams.input_pump(p, wl.power, wl.w0, wl.focus, th)
    b0 = np.zeros_like(a0)
    npdt = np.complex64 if dtype == "c64" else np.complex128
    return a0.astype(npdt), b0.astype(npdt)


def run_gpu(plan, a0, b0, dk_z=None, temp=None, s_begin=0, s_end=None):
    import torch
    a = torch.from_numpy(np.ascontiguousarray(a0)).cuda()
    b = torch.from_numpy(np.ascontiguousarray(b0)).cuda()
    dk = torch.from_numpy(np.asarray(dk_z, np.float64)).cuda() if dk_z is not None else None
    tt = None
    if temp is not None:
        rdt = np.float32 if plan.dtype == "c64" else np.float64
        tt = torch.from_numpy(np.ascontiguousarray(temp, rdt)).cuda()
    pw = plan.propagate(a, b, dk_z=dk, temp=tt, s_begin=s_begin, s_end=s_end)
    torch.cuda.synchronize()
    return a.cpu().numpy(), b.cpu().numpy(), pw.cpu().numpy()


def run_oracle(wl, a0, b0, dk_z=None, temp=None, s_begin=0, s_end=None):
    p = wl.params()
    t = None if temp is None else np.asarray(temp, np.float64)
    return ssfm.propagate(p, np.asarray(a0, np.complex128), np.asarray(b0, np.complex128),
                          dk_z=dk_z, temp=t, s_begin=s_begin, s_end=s_end)


def compare(wl, gpu, ref, dtype="c64", label=""):
    A, B, pw = gpu
    tf, te = (TOL_FIELD_C64, TOL_ETA_C64) if dtype == "c64" else (TOL_FIELD_C128, TOL_ETA_C128)
    ef, es = rel(A, ref["a_f"]), rel(B, ref["a_sh"])
    epf = abs(pw[0] / ref["p_f"] - 1)
    eps = abs(pw[1] / ref["p_sh"] - 1) if ref["p_sh"] > 0 else abs(pw[1])
    msg = f"{label}: F={ef:.2e} SH={es:.2e} P_F={epf:.2e} P_SH={eps:.2e}"
    print(msg)
    assert ef <= tf and (es <= tf or ref["p_sh"] == 0), msg
    assert epf <= te and eps <= te, msg
    return ef, es, epf, eps
