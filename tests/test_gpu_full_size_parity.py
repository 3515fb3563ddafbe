"""Full-size parity of the complex64 HIP path against the FP64 oracle.

The oracle's results at these sizes take minutes to hours of CPU, so they are
stored under tests/golden/full_size/ by tests/golden/make_full_size_refs.py,
which calls only the oracle and the seeded input generators.  Each test feeds
the GPU the same seeded inputs (checked against the fingerprint stored with
the reference) in the schedule the benchmark uses, and compares element by
element at the stated tolerances: relative L2 field error <= 1e-4, relative
power / efficiency error <= 1e-5, relative L2 gradient error <= 1e-4.
"""
import math
import os

import numpy as np
import pytest

import workloads
from gpu_util import inputs, rel, TOL_FIELD_C64, TOL_ETA_C64

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "full_size")
TOL_GRAD_C64 = 1e-4


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def golden(name):
    return np.load(os.path.join(GOLDEN, name + ".npz"))


def same_inputs(a0, stored):
    a = np.asarray(a0, np.complex128)
    ny, nx = a.shape
    fp = np.array([float(np.sum(np.abs(a) ** 2)), a[ny // 2, nx // 2].real, a[ny // 2, nx // 2].imag])
    assert np.allclose(fp, stored, rtol=1e-12, atol=0), (fp, stored)


def test_temperature_field_workload_full_size_against_oracle():
    """512 x 512 x 2000, 50 W, xi = 2.84, the synthetic T field over all 2000
    step planes (float32), absorption and TPA: exit fields and powers against
    the oracle's march of the whole crystal."""
    from paper_2410_04994_amd import Plan, autotune
    ref = golden("c5_forward")
    wl = workloads.c5_thermal_c64()
    print(f"case: {wl.name} full length against the oracle", flush=True)
    a0, b0 = inputs(wl)
    same_inputs(a0, ref["input"])
    temp = torch.from_numpy(workloads.RadialTemperature(wl, np.float32).materialise()).cuda()
    plan = Plan(wl.params(), "c64")
    autotune.tune_single(plan)
    a = torch.from_numpy(a0).cuda()
    b = torch.from_numpy(b0).cuda()
    pw = plan.propagate(a, b, temp=temp)
    torch.cuda.synchronize()
    del temp
    A, B, P = a.cpu().numpy(), b.cpu().numpy(), pw.cpu().numpy()
    ef, es = rel(A, ref["a_f"]), rel(B, ref["a_sh"])
    epf, eps = abs(P[0] / ref["powers"][0] - 1), abs(P[1] / ref["powers"][1] - 1)
    print(f"{plan.describe()}: F={ef:.2e} SH={es:.2e} P_F={epf:.2e} P_SH={eps:.2e}", flush=True)
    assert ef <= TOL_FIELD_C64 and es <= TOL_FIELD_C64
    assert epf <= TOL_ETA_C64 and eps <= TOL_ETA_C64


def test_differentiation_workload_full_size_against_oracle_adjoint_and_differences():
    """256 x 256 x 1000, 20 mm, 10 W, phase mask N(0, 0.1^2), dk(z) = dk_opt on
    every step, checkpoints every 32 steps (recomputed segments), loss P_SH(L):
    the gradient in the input field, in theta (a = |a| e^{i theta}) and in
    dk(z) against the oracle's reverse-mode gradient; the directional
    derivatives along 64 random directions of (theta, dk(z)) against central
    differences (h = 1e-3) of the oracle's march."""
    from paper_2410_04994_amd import Plan
    ref = golden("c4_adjoint")
    fd = golden("c4_fd")["fd"]
    wl = workloads.c4_diff_c64()
    print(f"case: {wl.name} K=32 against the oracle adjoint", flush=True)
    a0, b0 = inputs(wl)
    same_inputs(a0, ref["input"])
    plan = Plan(wl.params(), "c64", checkpoint_every=32)
    a = torch.from_numpy(a0).cuda()
    dk = torch.full((wl.nz,), wl.dk0, dtype=torch.float64, device="cuda")
    w = torch.tensor([0.0, 1.0], dtype=torch.float64, device="cuda")
    res = plan.adjoint(a, torch.from_numpy(b0).cuda(), power_weights=w, dk_z=dk, want_dk=True)
    torch.cuda.synchronize()
    g_f = res["g_f"].cpu().numpy().astype(np.complex128)
    g_dk = res["g_dk"].cpu().numpy()
    p_sh = float(res["powers"][1])
    a0d = a0.astype(np.complex128)
    g_th = np.real(np.conj(g_f) * 1j * a0d)
    g_th_ref = np.real(np.conj(ref["g_f"].astype(np.complex128)) * 1j * a0d)
    e_f, e_th, e_dk = rel(g_f, ref["g_f"]), rel(g_th, g_th_ref), rel(g_dk, ref["g_dk"])
    e_p = abs(p_sh / ref["powers"][1] - 1)
    # directional derivatives along the oracle's 64 difference directions
    rng = np.random.Generator(np.random.PCG64(40))
    dz = wl.lcr / wl.nz
    an = []
    for _ in range(len(fd)):
        v = rng.normal(size=(wl.ny, wl.nx))
        vk = rng.normal(size=wl.nz) / (dz * math.sqrt(wl.nz))
        an.append(float(np.sum(g_th * v) + np.sum(g_dk * vk)))
    e_fd = float(np.linalg.norm(np.array(an) - fd) / np.linalg.norm(fd))
    print(f"{plan.describe()}: g_f={e_f:.2e} g_theta={e_th:.2e} g_dk={e_dk:.2e} P_SH={e_p:.2e} "
          f"FD(64 directions)={e_fd:.2e}", flush=True)
    assert e_f <= TOL_GRAD_C64 and e_th <= TOL_GRAD_C64 and e_dk <= TOL_GRAD_C64
    assert e_p <= TOL_ETA_C64
    assert e_fd <= TOL_GRAD_C64


def test_temperature_field_workload_full_size_adjoint_against_oracle():
    """512 x 512 x 2000 with the temperature field, loss P_SH(L): the complex64
    adjoint (automatic checkpoint interval) gives the temperature moments
    sum dP/dT (T - T_ref) and sum dP/dT (the gradients in the dT scale and in
    T0) and the per-step mismatch gradient; all against the oracle's
    reverse-mode gradient of the same march."""
    from paper_2410_04994_amd import Plan, autotune
    ref = golden("c5_adjoint")
    wl = workloads.c5_thermal_c64()
    print(f"case: {wl.name} adjoint against the oracle", flush=True)
    a0, b0 = inputs(wl)
    same_inputs(a0, ref["input"])
    temp = torch.from_numpy(workloads.RadialTemperature(wl, np.float32).materialise()).cuda()
    plan = Plan(wl.params(), "c64")
    autotune.tune_single(plan)
    w = torch.tensor([0.0, 1.0], dtype=torch.float64, device="cuda")
    res = plan.adjoint(torch.from_numpy(a0).cuda(), torch.from_numpy(b0).cuda(), power_weights=w,
                       temp=temp, want_dk=True, want_t=True)
    torch.cuda.synchronize()
    del temp
    gm = res["g_t_moments"].cpu().numpy()
    g_dk = res["g_dk"].cpu().numpy()
    p_sh = float(res["powers"][1])
    e_m = np.abs(gm / ref["g_t_moments"] - 1)
    e_dk = rel(g_dk, ref["g_dk"])
    e_p = abs(p_sh / ref["powers"][1] - 1)
    print(f"{plan.describe()}: moments {gm} vs {ref['g_t_moments']} (rel {e_m}), g_dk={e_dk:.2e} "
          f"P_SH={e_p:.2e}", flush=True)
    assert np.all(e_m <= TOL_GRAD_C64) and e_dk <= TOL_GRAD_C64
    assert e_p <= TOL_ETA_C64
