"""Hand-written adjoint of the HIP march against the oracle's reverse-mode
derivative and against finite differences (needs the GPU)."""
import math

import numpy as np
import pytest

import workloads
from oracle import adjoint as oadj
from gpu_util import inputs, rel

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def cuda(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def gpu_adjoint(wl, dtype, a0, b0, gf, gs, w, dk=None, ckpt=0):
    from paper_2410_04994_amd import Plan
    plan = Plan(wl.params(), dtype, checkpoint_every=ckpt)
    npdt = np.complex64 if dtype == "c64" else np.complex128
    res = plan.adjoint(cuda(a0.astype(npdt)), cuda(b0.astype(npdt)),
                       g_f_out=cuda(gf.astype(npdt)) if gf is not None else None,
                       g_sh_out=cuda(gs.astype(npdt)) if gs is not None else None,
                       power_weights=cuda(np.asarray(w, np.float64)),
                       dk_z=cuda(dk) if dk is not None else None, want_dk=True)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in res.items()}


def small_case(n=32, nz=20, seed=3, undepleted=False):
    wl = workloads.c2_plain_c64().with_(nx=n, ny=n, nz=nz, lcr=4e-3, undepleted=undepleted,
                                        lx=workloads.c2_plain_c64().lx * n / 256 * 2,
                                        ly=workloads.c2_plain_c64().ly * n / 256 * 2)
    rng = np.random.Generator(np.random.PCG64(seed))
    a0, b0 = inputs(wl, "c128")
    b0 = (0.05 * np.abs(a0).max() * (rng.normal(size=a0.shape) + 1j * rng.normal(size=a0.shape)))
    gf = rng.normal(size=a0.shape) + 1j * rng.normal(size=a0.shape)
    gs = rng.normal(size=a0.shape) + 1j * rng.normal(size=a0.shape)
    scale = 1.0 / np.abs(a0).max()
    dk = wl.dk0 + 500.0 * rng.normal(size=nz)
    return wl, a0, b0, gf * scale, gs * scale, (0.3, 2.0), dk


def oracle_adjoint(wl, a0, b0, gf, gs, w, dk):
    return oadj.adjoint(wl.params(), a0, b0, gf, gs, dk_z=dk, power_weights=w)


@pytest.mark.parametrize("undepleted", [False, True])
def test_complex128_adjoint_matches_oracle(undepleted):
    wl, a0, b0, gf, gs, w, dk = small_case(undepleted=undepleted)
    ref = oracle_adjoint(wl, a0, b0, gf, gs, w, dk)
    got = gpu_adjoint(wl, "c128", a0, b0, gf, gs, w, dk, ckpt=6)
    assert rel(got["g_f"], ref["g_f"]) < 1e-10
    assert rel(got["g_sh"], ref["g_sh"]) < 1e-10
    assert rel(got["g_dk"], ref["g_dk"]) < 1e-10
    assert rel(got["a_sh"], ref["forward"]["a_sh"]) < 1e-12


def test_walkoff_adjoint_matches_oracle():
    """The adjoint of the walk-off factor is its conjugate, like the rest of L."""
    wl, a0, b0, gf, gs, w, dk = small_case()
    wl = wl.with_(walkoff_sh=0.05 * wl.lx / wl.lcr, walkoff_f=0.02 * wl.lx / wl.lcr)
    ref = oracle_adjoint(wl, a0, b0, gf, gs, w, dk)
    got = gpu_adjoint(wl, "c128", a0, b0, gf, gs, w, dk, ckpt=6)
    for key in ("g_f", "g_sh", "g_dk"):
        assert rel(got[key], ref[key]) < 1e-10, key


def test_complex64_adjoint_matches_oracle():
    wl, a0, b0, gf, gs, w, dk = small_case(n=64, nz=40)
    ref = oracle_adjoint(wl, a0, b0, gf, gs, w, dk)
    got = gpu_adjoint(wl, "c64", a0.astype(np.complex64).astype(complex),
                      b0.astype(np.complex64).astype(complex), gf, gs, w, dk, ckpt=7)
    assert rel(got["g_f"], ref["g_f"]) < 1e-4
    assert rel(got["g_sh"], ref["g_sh"]) < 1e-4
    assert rel(got["g_dk"], ref["g_dk"]) < 1e-4


def test_checkpoint_interval_does_not_change_the_result():
    """The recompute replays the same passes, so fields, powers and input
    gradients are bitwise independent of K.  The mismatch gradient sums stage
    values recomputed inside the adjoint kernel, whose code generation (FMA
    contraction) may differ from the forward kernel's by an ulp per cell, so it
    is compared to 1e-6."""
    wl, a0, b0, gf, gs, w, dk = small_case(n=32, nz=13)
    base = gpu_adjoint(wl, "c64", a0, b0, gf, gs, w, dk, ckpt=1)
    for k in (2, 5, 13, 64, 0):     # 0: the library's default (all 13 steps staged)
        got = gpu_adjoint(wl, "c64", a0, b0, gf, gs, w, dk, ckpt=k)
        for key in ("g_f", "g_sh", "a_f", "a_sh", "powers"):
            assert np.array_equal(got[key], base[key]), (k, key)
        assert rel(got["g_dk"], base["g_dk"]) < 1e-6


def test_full_grid_power_gradient_matches_oracle():
    """256 x 256 differentiation workload (20 mm, 10 W, xi = 2.84, phase mask
    0.1 rad), shortened to 100 steps so the FP64 oracle adjoint stays quick."""
    wl = workloads.c4_diff_c64().with_(nz=100)
    a0, b0 = inputs(wl, "c64")
    a0 = a0.astype(complex)
    b0 = b0.astype(complex)
    dk = np.full(wl.nz, wl.dk0)
    zero = np.zeros_like(a0)
    ref = oracle_adjoint(wl, a0, b0, zero, zero, (0.0, 1.0), dk)
    got = gpu_adjoint(wl, "c64", a0, b0, None, None, (0.0, 1.0), dk, ckpt=32)
    assert rel(got["g_f"], ref["g_f"]) < 1e-4
    assert rel(got["g_dk"], ref["g_dk"]) < 1e-4


def test_autograd_power_gradient_finite_differences():
    """d P_SH / d(theta, dk_z, focus) through torch: phase mask -> beam builder ->
    march; checked by central differences of the complex128 march."""
    from paper_2410_04994_amd import Plan, beams
    from paper_2410_04994_amd.autograd import march
    wl = workloads.c4_diff_c64().with_(nx=64, ny=64, nz=60,
                                       lx=workloads.c4_diff_c64().lx * 0.5,
                                       ly=workloads.c4_diff_c64().ly * 0.5)
    plan = Plan(wl.params(), "c128")
    theta0 = torch.from_numpy(workloads.phase_noise(wl)).cuda()
    dk0 = torch.full((wl.nz,), wl.dk0, dtype=torch.float64, device="cuda")
    focus0 = torch.tensor(wl.focus, dtype=torch.float64, device="cuda")

    def psh(theta, dk, focus):
        a = beams.pump_for(wl, theta=theta, dtype=torch.complex128, focus=focus)
        _, _, pw = march(plan, a, torch.zeros_like(a), dk_z=dk)
        return pw[1]

    th = theta0.clone().requires_grad_(True)
    dk = dk0.clone().requires_grad_(True)
    fo = focus0.clone().requires_grad_(True)
    p = psh(th, dk, fo)
    p.backward()
    rng = np.random.Generator(np.random.PCG64(40))
    dz = wl.lcr / wl.nz
    for _ in range(4):
        v = torch.from_numpy(rng.normal(size=theta0.shape)).cuda()
        vk = torch.from_numpy(rng.normal(size=wl.nz)).cuda() / (dz * math.sqrt(wl.nz))
        h = 1e-3
        with torch.no_grad():
            fd = (psh(theta0 + h * v, dk0 + h * vk, focus0) - psh(theta0 - h * v, dk0 - h * vk, focus0)) / (2 * h)
        an = (th.grad * v).sum() + (dk.grad * vk).sum()
        assert abs(fd.item() - an.item()) <= 1e-5 * abs(fd.item()), (fd.item(), an.item())
    hf = 1e-6
    with torch.no_grad():
        fd = (psh(theta0, dk0, focus0 + hf) - psh(theta0, dk0, focus0 - hf)) / (2 * hf)
    assert abs(fd.item() - fo.grad.item()) <= 1e-4 * abs(fd.item())


def test_adjoint_rejects_missing_workspace_and_outputs():
    from paper_2410_04994_amd import Plan, ShgError
    from paper_2410_04994_amd import binding
    wl = workloads.c2_plain_c64().with_(nx=32, ny=32, nz=4)
    plan = Plan(wl.params(), "c64")
    a = torch.zeros((32, 32), dtype=torch.complex64, device="cuda")
    lib = binding.load_library()
    rc = lib.shg_propagate_adjoint(plan.handle, a.data_ptr(), a.data_ptr(), None, None, None, None,
                                   None, a.data_ptr(), a.data_ptr(), None, None, None, None, None,
                                   None, None)
    assert rc == binding.SHG_EINVAL and b"workspace" in lib.shg_last_error()


def thermal_small(n=32, nz=18, undepleted=False):
    base = workloads.c5_thermal_c64()
    wl = base.with_(nx=n, ny=n, nz=nz, lcr=6e-3, lx=base.lx * n / 512 * 4, ly=base.ly * n / 512 * 4,
                    undepleted=undepleted)
    temp = workloads.radial_temperature_profile(wl)
    rng = np.random.Generator(np.random.PCG64(8))
    temp = temp + 0.5 * rng.normal(size=temp.shape)
    return wl, temp


# cubic dispersion part and the printed MgO:sPPLT grating expansion (Eq. 4)
CUBIC_DK = dict(ddk_dT=60.0, ddk_dT2=-15.0, ddk_dT3=4.0, grating_period=workloads.GRATING_PERIOD,
                grating_a=workloads.GRATING_A, grating_b=workloads.GRATING_B)


@pytest.mark.parametrize("dtype,tol,cubic", [("c128", 1e-10, False), ("c64", 1e-4, False),
                                             ("c128", 1e-10, True), ("c64", 1e-4, True)])
def test_thermal_adjoint_matches_oracle(dtype, tol, cubic):
    """Per-cell mismatch and lens; with cubic, dk(T) carries quadratic and
    cubic terms, so the temperature moments go through the slope c1 + 2 c2 dT
    + 3 c3 dT^2 of each cell."""
    from paper_2410_04994_amd import Plan
    wl, temp = thermal_small()
    if cubic:
        wl = wl.with_(**CUBIC_DK)
    npdt = np.complex64 if dtype == "c64" else np.complex128
    rdt = np.float32 if dtype == "c64" else np.float64
    temp = temp.astype(rdt)
    a0, b0 = inputs(wl, dtype)
    rng = np.random.Generator(np.random.PCG64(5))
    dk = wl.dk0 + 300 * rng.normal(size=wl.nz)
    w = (0.2, 1.0)
    ref = oadj.adjoint(wl.params(), a0.astype(complex), b0.astype(complex), np.zeros(a0.shape, complex),
                       np.zeros(a0.shape, complex), dk_z=dk, temp=temp.astype(np.float64),
                       power_weights=w)
    plan = Plan(wl.params(), dtype, checkpoint_every=5)
    res = plan.adjoint(cuda(a0), cuda(b0), power_weights=cuda(np.asarray(w)), dk_z=cuda(dk),
                       temp=cuda(temp), want_dk=True, want_t=True)
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy() for k, v in res.items()}
    assert rel(got["g_f"], ref["g_f"]) < tol
    assert rel(got["g_dk"], ref["g_dk"]) < tol
    assert rel(got["g_t_moments"], ref["g_t_moments"]) < tol


@pytest.mark.parametrize("dtype,tol", [("c128", 1e-10), ("c64", 1e-4)])
def test_thermal_adjoint_on_narrow_row_schedules(dtype, tol):
    """The temperature-field adjoint row pass with several cells per thread
    (schedules the defaults do not pick), with the cubic and grating dk(T),
    against the oracle's reverse-mode gradient."""
    from paper_2410_04994_amd import Plan
    wl, temp = thermal_small()
    wl = wl.with_(**CUBIC_DK)
    rdt = np.float32 if dtype == "c64" else np.float64
    temp = temp.astype(rdt)
    a0, b0 = inputs(wl, dtype)
    w = (0.2, 1.0)
    ref = oadj.adjoint(wl.params(), a0.astype(complex), b0.astype(complex), np.zeros(a0.shape, complex),
                       np.zeros(a0.shape, complex), temp=temp.astype(np.float64), power_weights=w)
    plan = Plan(wl.params(), dtype, checkpoint_every=5)
    tried = 0
    for re_, rw in ((4, 64), (8, 64), (4, 256)):
        try:
            plan.set_schedule(re_, rw, 0, 0)
        except Exception:
            continue
        res = plan.adjoint(cuda(a0), cuda(b0), power_weights=cuda(np.asarray(w)), temp=cuda(temp),
                           want_dk=True, want_t=True)
        torch.cuda.synchronize()
        got = {k: v.cpu().numpy() for k, v in res.items()}
        msg = plan.describe()
        assert rel(got["g_f"], ref["g_f"]) < tol, msg
        assert rel(got["g_dk"], ref["g_dk"]) < tol, msg
        assert rel(got["g_t_moments"], ref["g_t_moments"]) < tol, msg
        tried += 1
    assert tried >= 1


def test_thermal_scalar_gradients_by_finite_differences():
    """dP_SH/d(dT scale) and dP_SH/dT0 of the thermal-lens workload shape,
    through torch, against central differences of the complex128 march."""
    from paper_2410_04994_amd import Plan, beams
    from paper_2410_04994_amd.autograd import thermal_powers
    base = workloads.c5_thermal_c64()
    wl = base.with_(nx=64, ny=64, nz=40, lx=base.lx * 0.5, ly=base.ly * 0.5)
    plan = Plan(wl.params(), "c128")
    prof = workloads.radial_temperature_profile(wl) - wl.extra["t0"]
    prof = torch.from_numpy(prof).cuda()
    a = beams.pump_for(wl, dtype=torch.complex128)
    b = torch.zeros_like(a)
    t0 = torch.tensor(wl.extra["t0"], dtype=torch.float64, device="cuda", requires_grad=True)
    sc = torch.tensor(1.0, dtype=torch.float64, device="cuda", requires_grad=True)
    thermal_powers(plan, a, b, t0, sc, prof)[1].backward()
    with torch.no_grad():
        f = lambda tt, ss: thermal_powers(plan, a, b, tt, ss, prof)[1].item()
        h = 1e-3
        fd_t0 = (f(t0 + h, sc) - f(t0 - h, sc)) / (2 * h)
        fd_sc = (f(t0, sc + h) - f(t0, sc - h)) / (2 * h)
    assert abs(t0.grad.item() - fd_t0) <= 1e-5 * abs(fd_t0) + 1e-12
    assert abs(sc.grad.item() - fd_sc) <= 1e-5 * abs(fd_sc) + 1e-12


def test_full_size_differentiation_config_against_central_differences():
    """The differentiation workload at its full size and as stated (256 x 256 x
    1000, 20 mm, 10 W, xi = 2.84, phase mask N(0, 0.1^2), checkpoints every 32
    steps, recomputed): the complex64 adjoint's derivative of P_SH along 64
    random directions of (theta, dk_z) against central differences (h = 1e-3)
    of the complex128 march.  A dk direction moves the accumulated phase by
    about h rad: delta dk_s = h v_s / (dz sqrt(nz))."""
    from paper_2410_04994_amd import Plan, beams
    wl = workloads.c4_diff_c64()
    print(f"case: {wl.name} K=32", flush=True)
    theta0 = torch.from_numpy(workloads.phase_noise(wl)).cuda()
    dk0 = torch.full((wl.nz,), wl.dk0, dtype=torch.float64, device="cuda")
    w = torch.tensor([0.0, 1.0], dtype=torch.float64, device="cuda")
    plan = Plan(wl.params(), "c64", checkpoint_every=32)
    a0 = beams.pump_for(wl, theta=theta0, dtype=torch.complex64)
    res = plan.adjoint(a0, torch.zeros_like(a0), power_weights=w, dk_z=dk0, want_dk=True)
    # dP/dtheta: a = |a| e^{i theta}, da/dtheta = i a, g = dP/dRe + i dP/dIm
    g_theta = (torch.conj(res["g_f"]) * (1j * a0)).real.double()
    g_dk = res["g_dk"]
    ref = Plan(wl.params(), "c128")

    def p_sh(theta, dk):
        a = beams.pump_for(wl, theta=theta, dtype=torch.complex128)
        pw = ref.propagate(a, torch.zeros_like(a), dk_z=dk)
        return float(pw[1])

    rng = np.random.Generator(np.random.PCG64(40))
    dz = wl.lcr / wl.nz
    h = 1e-3
    fd, an = [], []
    for _ in range(64):
        v = torch.from_numpy(rng.normal(size=(wl.ny, wl.nx))).cuda()
        vk = torch.from_numpy(rng.normal(size=wl.nz)).cuda() / (dz * math.sqrt(wl.nz))
        fd.append((p_sh(theta0 + h * v, dk0 + h * vk) - p_sh(theta0 - h * v, dk0 - h * vk)) / (2 * h))
        an.append(float((g_theta * v).sum() + (g_dk * vk).sum()))
    fd, an = np.array(fd), np.array(an)
    # relative L2 over the 64 directions (a single direction can have a
    # derivative near zero, so per-direction ratios are not used)
    err = float(np.linalg.norm(fd - an) / np.linalg.norm(fd))
    print(f"relative L2 difference over 64 directions: {err:.2e}", flush=True)
    assert err < 1e-4


def test_full_size_thermal_scalar_gradients_against_central_differences():
    """The temperature-field workload at its full size (512 x 512 x 2000, 50 W,
    the synthetic T field): dP_SH/d(dT scale) and dP_SH/dT0 from the complex64
    adjoint (temperature moments, automatic K) against central differences of
    the complex128 march."""
    from paper_2410_04994_amd import Plan, beams
    from paper_2410_04994_amd.autograd import thermal_powers
    wl = workloads.c5_thermal_c64()
    print(f"case: {wl.name}", flush=True)
    prof = torch.from_numpy(workloads.radial_temperature_profile(wl) - wl.extra["t0"]).cuda()
    t0 = torch.tensor(wl.extra["t0"], dtype=torch.float64, device="cuda", requires_grad=True)
    sc = torch.tensor(1.0, dtype=torch.float64, device="cuda", requires_grad=True)
    plan = Plan(wl.params(), "c64")
    a = beams.pump_for(wl, dtype=torch.complex64)
    thermal_powers(plan, a, torch.zeros_like(a), t0, sc, prof)[1].backward()
    ref = Plan(wl.params(), "c128")
    a128 = beams.pump_for(wl, dtype=torch.complex128)
    with torch.no_grad():
        f = lambda tt, ss: thermal_powers(ref, a128, torch.zeros_like(a128), tt, ss, prof)[1].item()
        h = 1e-3
        fd_t0 = (f(t0 + h, sc) - f(t0 - h, sc)) / (2 * h)
        fd_sc = (f(t0, sc + h) - f(t0, sc - h)) / (2 * h)
    print(f"dP/dT0 {t0.grad.item():.6e} vs {fd_t0:.6e}; dP/dscale {sc.grad.item():.6e} vs {fd_sc:.6e}",
          flush=True)
    assert abs(t0.grad.item() - fd_t0) <= 1e-3 * abs(fd_t0)
    assert abs(sc.grad.item() - fd_sc) <= 1e-3 * abs(fd_sc)


@pytest.mark.parametrize("dtype,tol,ckpt,thermal", [("c128", 1e-10, 0, False), ("c128", 1e-10, 4, False),
                                                   ("c64", 1e-4, 5, False), ("c128", 1e-10, 5, True),
                                                   ("c64", 1e-4, 0, True)])
def test_lnl_adjoint_matches_oracle(dtype, tol, ckpt, thermal):
    """The L/2 - N - L/2 order: reverse of L(dz/2), one RK4 over dz, L(dz/2)
    per step, with walk-off, a per-step mismatch profile and (thermal) a
    temperature field with the full dk(T); ckpt > 0 recomputes segments from
    checkpoints, whose boundaries split a merged column pass into two halves."""
    from paper_2410_04994_amd import Plan
    if thermal:
        wl, temp = thermal_small(nz=18)
        wl = wl.with_(split="LNL", **CUBIC_DK)
    else:
        wl, a0, b0, gf, gs, w, dk = small_case(nz=17)
        base = workloads.c2_plain_c64()
        wl = wl.with_(split="LNL", walkoff_sh=0.05 * base.lx / base.lcr)
        temp = None
    rng = np.random.Generator(np.random.PCG64(12))
    a0, b0 = inputs(wl, "c128")
    a0 = a0.astype(complex)
    b0 = (0.05 * np.abs(a0).max() * (rng.normal(size=a0.shape) + 1j * rng.normal(size=a0.shape)))
    scale = 1.0 / np.abs(a0).max()
    gf = (rng.normal(size=a0.shape) + 1j * rng.normal(size=a0.shape)) * scale
    gs = (rng.normal(size=a0.shape) + 1j * rng.normal(size=a0.shape)) * scale
    dk = wl.dk0 + 300.0 * rng.normal(size=wl.nz)
    w = (0.3, 2.0)
    rdt = np.float32 if dtype == "c64" else np.float64
    npdt = np.complex64 if dtype == "c64" else np.complex128
    if temp is not None:
        temp = temp.astype(rdt)
    a0, b0, gf, gs = (x.astype(npdt).astype(complex) for x in (a0, b0, gf, gs))
    ref = oadj.adjoint(wl.params(), a0, b0, gf, gs, dk_z=dk,
                       temp=None if temp is None else temp.astype(np.float64), power_weights=w)
    plan = Plan(wl.params(), dtype, checkpoint_every=ckpt)
    res = plan.adjoint(cuda(a0.astype(npdt)), cuda(b0.astype(npdt)), g_f_out=cuda(gf.astype(npdt)),
                       g_sh_out=cuda(gs.astype(npdt)), power_weights=cuda(np.asarray(w)),
                       dk_z=cuda(dk), temp=None if temp is None else cuda(temp), want_dk=True,
                       want_t=temp is not None)
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy() for k, v in res.items()}
    assert rel(got["g_f"], ref["g_f"]) < tol
    assert rel(got["g_sh"], ref["g_sh"]) < tol
    assert rel(got["g_dk"], ref["g_dk"]) < tol
    assert rel(got["a_sh"], ref["forward"]["a_sh"]) < tol
    if temp is not None:
        assert rel(got["g_t_moments"], ref["g_t_moments"]) < tol



def test_adjoint_into_caller_buffers():
    """Outputs written into caller-provided buffers equal those of a call that
    allocates them."""
    from paper_2410_04994_amd import Plan
    wl = small_case(nz=8)[0]
    plan = Plan(wl.params(), "c64")
    a0, b0 = inputs(wl, "c64")
    a, b = cuda(a0), cuda(b0)
    w = cuda(np.array([0.2, 1.0]))
    ref = plan.adjoint(a, b, power_weights=w, want_dk=True)
    out = {k: torch.empty_like(v) for k, v in ref.items()}
    got = plan.adjoint(a, b, power_weights=w, want_dk=True, out=out)
    torch.cuda.synchronize()
    for k in ref:
        assert got[k].data_ptr() == out[k].data_ptr()
        assert torch.equal(got[k], ref[k]), k


@pytest.mark.parametrize("split,thermal", [("NLN", False), ("NLN", True), ("LNL", False)])
def test_overlapped_recompute_graph_equals_serial_launches(split, thermal):
    """With checkpoints every 4 of 18 steps, the recompute of each segment runs
    on a second stream beside the reverse sweep of the segment after it (double
    buffered staging), inside a graph the plan caches and replays.  Three calls
    equal the serial one-stream launches of an SHG_NO_GRAPH plan bit for bit."""
    from paper_2410_04994_amd import Plan
    from paper_2410_04994_amd.binding import SHG_NO_GRAPH
    if thermal:
        wl, temp = thermal_small()
        tt = cuda(temp.astype(np.float32))
    else:
        wl, tt = small_case(n=32, nz=18)[0], None
    wl = wl.with_(split=split)
    a0, b0 = inputs(wl, "c64")
    a, b = cuda(a0), cuda(b0)
    w = cuda(np.array([0.3, 1.0]))
    gs = cuda((np.ones_like(a0) * 0.01).astype(np.complex64))
    kw = dict(g_sh_out=gs, power_weights=w, temp=tt, want_dk=True, want_t=thermal)
    serial = Plan(wl.params(), "c64", flags=SHG_NO_GRAPH, checkpoint_every=4)
    ref = serial.adjoint(a, b, **kw)
    torch.cuda.synchronize()
    plan = Plan(wl.params(), "c64", checkpoint_every=4)
    ws = plan.workspace(adjoint=True)
    out = {k: torch.empty_like(v) for k, v in ref.items()}
    for rep in range(3):
        got = plan.adjoint(a, b, workspace=ws, out=out, **kw)
        torch.cuda.synchronize()
        for k in ref:
            assert torch.equal(got[k], ref[k]), (rep, k)


def test_adjoint_graph_cache_keeps_several_output_sets():
    """Adjoint calls with two sets of output buffers, alternating, equal the
    serial launches of an SHG_NO_GRAPH plan bit for bit."""
    from paper_2410_04994_amd import Plan
    from paper_2410_04994_amd.binding import SHG_NO_GRAPH
    wl = small_case(n=32, nz=12)[0]
    a0, b0 = inputs(wl, "c64")
    a, b = cuda(a0), cuda(b0)
    w = cuda(np.array([0.3, 1.0]))
    ref = Plan(wl.params(), "c64", flags=SHG_NO_GRAPH, checkpoint_every=5).adjoint(
        a, b, power_weights=w, want_dk=True)
    torch.cuda.synchronize()
    plan = Plan(wl.params(), "c64", checkpoint_every=5)
    ws = plan.workspace(adjoint=True)
    outs = [{k: torch.empty_like(v) for k, v in ref.items()} for _ in range(2)]
    for rnd in range(3):
        for out in outs:
            got = plan.adjoint(a, b, power_weights=w, want_dk=True, workspace=ws, out=out)
            torch.cuda.synchronize()
            for k in ref:
                assert torch.equal(got[k], ref[k]), (rnd, k)
