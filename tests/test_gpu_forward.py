"""Parity of the HIP forward march with the FP64 oracle (needs the GPU).

Tolerances: complex64 path field relative L2 <= 1e-4 and efficiency / power
relative error <= 1e-5; complex128 path (same kernels in FP64) <= 1e-12.
"""
import numpy as np
import pytest

import workloads
from oracle import beams, ssfm
from gpu_util import inputs, run_gpu, run_oracle, compare, rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def make_plan(wl, dtype="c64", **kw):
    from paper_2410_04994_amd import Plan
    return Plan(wl.params(), dtype, **kw)


def parity(wl, dtype="c64", label="", dk_z=None, sched=None, flags=0):
    plan = make_plan(wl, dtype, flags=flags)
    if sched:
        plan.set_schedule(*sched)
    a0, b0 = inputs(wl, dtype)
    gpu = run_gpu(plan, a0, b0, dk_z=dk_z)
    ref = run_oracle(wl, a0, b0, dk_z=dk_z)
    return compare(wl, gpu, ref, dtype, label or plan.describe())


def test_config1_complex128_algorithmic_parity():
    """64x64 x 200 steps, 4 w0 window, FP64: the kernels compute the oracle's scheme."""
    parity(workloads.c1_plain_fp64(), "c128")


def test_config1_complex64():
    parity(workloads.c1_plain_fp64().with_(dtype="c64"), "c64")


def test_config2_physics_small_grid():
    """Depleted pump, linear + two-photon absorption, dk at the optimum, phase noise."""
    parity(workloads.c2_plain_c64().with_(nx=64, ny=64, nz=120), "c64")


def test_config2_full_size():
    """256x256 x 1000 steps, 30 W, xi = 2.84, with the schedule the benchmark
    uses (autotuner, packaged table)."""
    from paper_2410_04994_amd import autotune
    wl = workloads.c2_plain_c64()
    plan = make_plan(wl)
    autotune.tune_single(plan)
    a0, b0 = inputs(wl)
    ef, es, epf, eps = compare(wl, run_gpu(plan, a0, b0), run_oracle(wl, a0, b0), "c64",
                               plan.describe())
    assert es < 5e-5 and eps < 5e-6


def test_config2_full_size_in_the_lnl_order():
    """The benchmark workload (256 x 256 x 1000) in the L/2 - N - L/2 order,
    whole crystal, against the oracle's march in the same order."""
    from paper_2410_04994_amd import autotune
    wl = workloads.c2_plain_c64().with_(split="LNL")
    plan = make_plan(wl)
    autotune.tune_single(plan)
    a0, b0 = inputs(wl)
    compare(wl, run_gpu(plan, a0, b0), run_oracle(wl, a0, b0), "c64", "LNL " + plan.describe())


def test_autotuner_picks_a_correct_schedule(tmp_path, monkeypatch):
    from paper_2410_04994_amd import autotune
    monkeypatch.setenv("SHG_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    wl = workloads.c2_plain_c64().with_(nx=64, ny=64, nz=30)
    plan = make_plan(wl)
    best = autotune.tune_single(plan, probe_steps=8, reps=1, cache=False)
    assert best in autotune.candidates(lambda s: autotune._set_ok(plan.set_schedule, s))
    plan.set_schedule(*best)
    a0, b0 = inputs(wl)
    compare(wl, run_gpu(plan, a0, b0), run_oracle(wl, a0, b0), "c64", plan.describe())


def test_config2_full_grid_complex128():
    parity(workloads.c2_plain_c64().with_(nz=40), "c128")


@pytest.mark.parametrize("nx,ny,nz", [(16, 16, 9), (512, 16, 3), (16, 512, 3), (128, 32, 7),
                                      (32, 256, 5), (512, 512, 2)])
def test_grid_shapes(nx, ny, nz):
    base = workloads.c2_plain_c64()
    wl = base.with_(nx=nx, ny=ny, nz=nz, lx=base.lx * nx / 256, ly=base.ly * ny / 256)
    parity(wl, "c64")
    parity(wl.with_(nz=2), "c128")


def test_single_step():
    parity(workloads.c2_plain_c64().with_(nx=64, ny=64, nz=1), "c64")
    parity(workloads.c2_plain_c64().with_(nx=64, ny=64, nz=1), "c128")


def test_undepleted_pump():
    wl = workloads.c2_plain_c64().with_(nx=64, ny=64, nz=60, undepleted=True)
    parity(wl, "c64")
    parity(wl, "c128")


def test_per_step_mismatch_profile():
    wl = workloads.c4_diff_c64().with_(nx=64, ny=64, nz=80)
    rng = np.random.Generator(np.random.PCG64(12))
    dk = wl.dk0 + 300.0 * rng.normal(size=wl.nz)
    parity(wl, "c64", dk_z=dk)
    parity(wl, "c128", dk_z=dk)


def test_step_ranges_resume_bitwise():
    wl = workloads.c2_plain_c64().with_(nx=64, ny=64, nz=30)
    plan = make_plan(wl)
    a0, b0 = inputs(wl)
    full = run_gpu(plan, a0, b0)
    part = run_gpu(plan, a0, b0, s_end=11)
    rest = run_gpu(plan, part[0], part[1], s_begin=11)
    assert np.array_equal(rest[0], full[0]) and np.array_equal(rest[1], full[1])
    ref = run_oracle(wl, a0, b0, s_end=11)
    assert rel(part[1], ref["a_sh"]) < 1e-4


def test_graph_replay_equals_plain_launches_and_is_deterministic():
    from paper_2410_04994_amd import SHG_NO_GRAPH
    wl = workloads.c2_plain_c64().with_(nx=128, ny=128, nz=25)
    a0, b0 = inputs(wl)
    g = make_plan(wl)
    r1 = run_gpu(g, a0, b0)
    r2 = run_gpu(g, a0, b0)       # replays the cached graph
    s = run_gpu(make_plan(wl, flags=SHG_NO_GRAPH), a0, b0)
    for x, y in ((r1, r2), (r1, s)):
        assert all(np.array_equal(u, v) for u, v in zip(x, y))


def test_every_built_schedule_matches_the_oracle():
    wl = workloads.c2_plain_c64().with_(nx=256, ny=256, nz=6)
    plan = make_plan(wl)
    a0, b0 = inputs(wl)
    ref = run_oracle(wl, a0, b0)
    tried = 0
    for re_ in (1, 4, 8, 16):
        for rw in (64, 256):
            for ce in (4, 8, 16):
                for ct in (1, 2, 4, 8, 16):
                    try:
                        plan.set_schedule(re_, rw, ce, ct)
                    except Exception:
                        continue
                    compare(wl, run_gpu(plan, a0, b0), ref, "c64", plan.describe())
                    tried += 1
    assert tried >= 10


@pytest.mark.parametrize("n", [32, 128, 512])
def test_narrow_row_schedules_on_other_row_lengths(n):
    """The narrow row passes run their Stockham passes in place in one LDS
    buffer when a transform has one butterfly per thread in every pass but the
    last: every built narrow row schedule on 32-, 128- and 512-point rows."""
    base = workloads.c2_plain_c64()
    wl = base.with_(nx=n, ny=64, nz=5, lx=base.lx * n / 256, ly=base.ly * 64 / 256)
    plan = make_plan(wl)
    a0, b0 = inputs(wl)
    ref = run_oracle(wl, a0, b0)
    tried = 0
    for re_ in (4, 8, 16):
        for rw in (64, 256):
            try:
                plan.set_schedule(re_, rw, 0, 0)
            except Exception:
                continue
            compare(wl, run_gpu(plan, a0, b0), ref, "c64", plan.describe())
            tried += 1
    assert tried >= 3


def test_invalid_step_range_and_fields():
    from paper_2410_04994_amd import ShgError
    wl = workloads.c2_plain_c64().with_(nx=64, ny=64, nz=10)
    plan = make_plan(wl)
    a = torch.zeros((64, 64), dtype=torch.complex64, device="cuda")
    b = torch.zeros_like(a)
    for s0, s1 in ((0, 11), (5, 5), (-1, 3), (7, 2)):
        with pytest.raises(ShgError, match="SHG_EINVAL"):
            plan.propagate(a, b, s_begin=s0, s_end=s1)
    with pytest.raises(ValueError):
        plan.propagate(a.to(torch.complex128), b)
    # buffers smaller than the kernels address are refused before any launch
    small = torch.zeros((64, 32), dtype=torch.complex64, device="cuda")
    with pytest.raises(ValueError, match="a_sh holds"):
        plan.propagate(a, small)
    with pytest.raises(ValueError, match="dk_z holds"):
        plan.propagate(a, b, dk_z=torch.zeros(9, dtype=torch.float64, device="cuda"))
    with pytest.raises(ValueError, match="temp holds"):
        plan.propagate(a, b, temp=torch.zeros((9, 64, 64), dtype=torch.float32, device="cuda"))
    with pytest.raises(ValueError, match="workspace holds"):
        plan.propagate(a, b, workspace=torch.zeros(plan.workspace_bytes() - 1, dtype=torch.uint8,
                                                   device="cuda"))
    with pytest.raises(ValueError, match="heat holds"):
        plan.propagate_heat(a, b, heat=torch.zeros((10, 64, 64), dtype=torch.float32, device="cuda"))
    with pytest.raises(ValueError, match="powers holds"):
        plan.propagate(a, b, powers=torch.zeros(1, dtype=torch.float64, device="cuda"))


def test_explicit_workspace_and_no_powers():
    wl = workloads.c2_plain_c64().with_(nx=64, ny=64, nz=12)
    plan = make_plan(wl)
    a0, b0 = inputs(wl)
    ws = torch.empty(plan.workspace_bytes(), dtype=torch.uint8, device="cuda")
    a = torch.from_numpy(a0).cuda()
    b = torch.from_numpy(b0).cuda()
    pw = plan.propagate(a, b, workspace=ws)
    ref = run_oracle(wl, a0, b0)
    compare(wl, (a.cpu().numpy(), b.cpu().numpy(), pw.cpu().numpy()), ref)


def test_gpu_beam_builder_matches_oracle_builder():
    from paper_2410_04994_amd import beams as gb
    wl = workloads.c2_plain_c64()
    th = workloads.phase_noise(wl)
    g = gb.pump_for(wl, theta=torch.from_numpy(th).cuda(), dtype=torch.complex128).cpu().numpy()
    o = beams.input_pump(wl.params(), wl.power, wl.w0, wl.focus, th)
    assert rel(g, o) < 1e-12
    c = ssfm.coefficients(wl.params())
    assert abs(ssfm.power(g, wl.n_f, c.dx, c.dy) / wl.power - 1) < 1e-6


def thermal_case(n=64, nz=60):
    base = workloads.c5_thermal_c64()
    wl = base.with_(nx=n, ny=n, nz=nz, lx=base.lx * n / 512 * 4, ly=base.ly * n / 512 * 4)
    temp = workloads.radial_temperature_profile(wl).astype(np.float32)
    return wl, temp


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_temperature_field_forward(dtype):
    """Synthetic thermal-lens field T0 + 3 K exp(-alpha_SH z) exp(-2 r^2 / w_T^2):
    per-cell mismatch and lens phases."""
    wl, temp = thermal_case()
    plan = make_plan(wl, dtype)
    a0, b0 = inputs(wl, dtype)
    gpu = run_gpu(plan, a0, b0, temp=temp)
    ref = run_oracle(wl, a0, b0, temp=temp.astype(np.float64))
    compare(wl, gpu, ref, dtype, "thermal " + plan.describe())
    # the field matters: without it the result differs well beyond the tolerance
    cold = run_oracle(wl, a0, b0)
    assert rel(ref["a_sh"], cold["a_sh"]) > 1e-2


@pytest.mark.parametrize("dtype,grating", [("c64", False), ("c128", False), ("c64", True),
                                           ("c128", True)])
def test_temperature_field_cubic_mismatch(dtype, grating):
    """dk(T) of Eq. 4: the cubic dispersion part (stand-in for the Sellmeier
    indices) and, with grating, the printed Lambda(T) of MgO:sPPLT, split at a
    resume point so that the carried thermal phase is rebuilt from the samples."""
    wl, temp = thermal_case(n=64, nz=40)
    wl = wl.with_(ddk_dT=60.0, ddk_dT2=-15.0, ddk_dT3=4.0)
    if grating:
        wl = wl.with_(grating_period=workloads.GRATING_PERIOD, grating_a=workloads.GRATING_A,
                      grating_b=workloads.GRATING_B)
    plan = make_plan(wl, dtype)
    a0, b0 = inputs(wl, dtype)
    gpu = run_gpu(plan, a0, b0, temp=temp)
    ref = run_oracle(wl, a0, b0, temp=temp.astype(np.float64))
    compare(wl, gpu, ref, dtype, "cubic dk(T) " + plan.describe())
    part = run_gpu(plan, a0, b0, temp=temp, s_end=17)
    rest = run_gpu(plan, part[0], part[1], temp=temp, s_begin=17)
    compare(wl, rest, ref, dtype, "cubic dk(T) resume")
    # the higher terms matter
    lin = run_oracle(wl.with_(ddk_dT2=0.0, ddk_dT3=0.0, grating_period=0.0), a0, b0,
                     temp=temp.astype(np.float64))
    assert rel(ref["a_sh"], lin["a_sh"]) > 1e-2
    if grating:
        nog = run_oracle(wl.with_(grating_period=0.0), a0, b0, temp=temp.astype(np.float64))
        assert rel(ref["a_sh"], nog["a_sh"]) > 1e-3


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_temperature_field_on_every_row_schedule(dtype):
    """The temperature-field row pass in every built row schedule, the narrow
    ones (several cells per thread) included, which the default schedules do
    not pick: dk(T) with the cubic and the grating term, against the oracle."""
    wl, temp = thermal_case(n=64, nz=24)
    wl = wl.with_(ddk_dT=60.0, ddk_dT2=-15.0, ddk_dT3=4.0, grating_period=workloads.GRATING_PERIOD,
                  grating_a=workloads.GRATING_A, grating_b=workloads.GRATING_B)
    plan = make_plan(wl, dtype)
    a0, b0 = inputs(wl, dtype)
    ref = run_oracle(wl, a0, b0, temp=temp.astype(np.float64))
    tried = []
    for re_, rw in ((1, 256), (4, 64), (4, 256), (8, 64), (8, 256), (16, 64)):
        try:
            plan.set_schedule(re_, rw, 0, 0)
        except Exception:
            continue
        compare(wl, run_gpu(plan, a0, b0, temp=temp), ref, dtype, "T field " + plan.describe())
        tried.append(re_)
    assert 1 in tried and any(e > 1 for e in tried)


def test_temperature_field_resume_and_profile():
    wl, temp = thermal_case(n=32, nz=24)
    rng = np.random.Generator(np.random.PCG64(3))
    dk = wl.dk0 + 100 * rng.normal(size=wl.nz)
    plan = make_plan(wl)
    a0, b0 = inputs(wl)
    part = run_gpu(plan, a0, b0, dk_z=dk, temp=temp, s_end=10)
    rest = run_gpu(plan, part[0], part[1], dk_z=dk, temp=temp, s_begin=10)
    ref = run_oracle(wl, a0, b0, dk_z=dk, temp=temp.astype(np.float64))
    compare(wl, rest, ref, "c64", "thermal resume")


def test_temperature_field_full_grid():
    """512 x 512 thermal-lens workload (50 W, xi = 2.84), shortened to 40 steps
    for the oracle, with the default schedule."""
    base = workloads.c5_thermal_c64()
    wl = base.with_(nz=40)
    temp = workloads.radial_temperature_profile(base)[:40].astype(np.float32)
    plan = make_plan(wl)
    a0, b0 = inputs(wl)
    gpu = run_gpu(plan, a0, b0, temp=temp)
    ref = run_oracle(wl, a0, b0, temp=temp.astype(np.float64))
    compare(wl, gpu, ref, "c64", "thermal 512 " + plan.describe())


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_spatial_walkoff(dtype):
    """Walk-off on the SH (type-I birefringent matching) and a smaller one on
    the fundamental: the tan(rho) dA/dx term rides in the x propagator factor."""
    base = workloads.c2_plain_c64()
    wl = base.with_(nx=64, ny=64, nz=120, walkoff_sh=0.1 * base.lx / base.lcr,
                    walkoff_f=-0.03 * base.lx / base.lcr)
    parity(wl, dtype)
    a0, b0 = inputs(wl, dtype)
    plain = run_oracle(wl.with_(walkoff_sh=0.0, walkoff_f=0.0), a0, b0)
    walk = run_oracle(wl, a0, b0)
    assert rel(walk["a_sh"], plain["a_sh"]) > 1e-2


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_lnl_split_order(dtype):
    """The L/2 - N - L/2 order (SHG_SPLIT_LNL): one RK4 over dz per step between
    half-step propagators, with a per-step mismatch profile and walk-off."""
    base = workloads.c2_plain_c64()
    wl = base.with_(nx=64, ny=64, nz=50, split="LNL", walkoff_sh=0.05 * base.lx / base.lcr)
    rng = np.random.Generator(np.random.PCG64(5))
    dk = wl.dk0 + 200.0 * rng.normal(size=wl.nz)
    parity(wl, dtype, dk_z=dk)
    # it is a different discrete scheme: the N/2 - L - N/2 result differs
    a0, b0 = inputs(wl, dtype)
    lnl = run_oracle(wl, a0, b0, dk_z=dk)
    nln = run_oracle(wl.with_(split="NLN"), a0, b0, dk_z=dk)
    assert rel(lnl["a_sh"], nln["a_sh"]) > 1e-6


@pytest.mark.parametrize("dtype,dk_t", [("c64", False), ("c128", False), ("c64", True)])
def test_lnl_with_temperature_field_and_resume(dtype, dk_t):
    """L/2 - N - L/2 with per-cell mismatch and lens; dk_t adds the cubic
    dispersion part and the grating-period expansion of dk(T)."""
    wl, temp = thermal_case(n=32, nz=24)
    wl = wl.with_(split="LNL")
    if dk_t:
        wl = wl.with_(ddk_dT=60.0, ddk_dT2=-15.0, ddk_dT3=4.0,
                      grating_period=workloads.GRATING_PERIOD, grating_a=workloads.GRATING_A,
                      grating_b=workloads.GRATING_B)
    plan = make_plan(wl, dtype)
    a0, b0 = inputs(wl, dtype)
    full = run_gpu(plan, a0, b0, temp=temp)
    ref = run_oracle(wl, a0, b0, temp=temp.astype(np.float64))
    compare(wl, full, ref, dtype, "lnl thermal")
    part = run_gpu(plan, a0, b0, temp=temp, s_end=10)
    rest = run_gpu(plan, part[0], part[1], temp=temp, s_begin=10)
    # L/2 L/2 across the split point equals one L up to rounding
    assert rel(rest[1], full[1]) < (1e-5 if dtype == "c64" else 1e-12)


def test_lnl_refuses_heat_output():
    """The heat source is written between the half-steps of the N/2 - L - N/2
    order; in the L/2 - N - L/2 order no pass holds a step boundary in real space."""
    from paper_2410_04994_amd import ShgError
    wl = workloads.c2_plain_c64().with_(nx=32, ny=32, nz=4, split="LNL")
    plan = make_plan(wl)
    a = torch.ones((32, 32), dtype=torch.complex64, device="cuda")
    b = torch.zeros_like(a)
    with pytest.raises(ShgError, match="SHG_EUNSUPPORTED"):
        plan.propagate_heat(a, b)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_lnl_single_step_and_undepleted(dtype):
    base = workloads.c2_plain_c64()
    parity(base.with_(nx=64, ny=64, nz=1, split="LNL"), dtype)
    parity(base.with_(nx=64, ny=64, nz=30, split="LNL", undepleted=True), dtype)
    parity(base.with_(nx=128, ny=32, nz=7, split="LNL", lx=base.lx / 2, ly=base.ly / 8), dtype)


def test_power_trace_matches_oracle_and_one_shot_march():
    """P(z) every 7 steps: the exit fields equal the one-shot march bit for bit,
    every point matches the oracle's powers at that z, and without loss the
    total P_F + P_SH is conserved along z (Manley-Rowe)."""
    from paper_2410_04994_amd.trace import power_trace
    wl = workloads.c2_plain_c64().with_(nx=64, ny=64, nz=40)
    plan = make_plan(wl)
    a0, b0 = inputs(wl)
    a = torch.from_numpy(a0).cuda()
    b = torch.from_numpy(b0).cuda()
    z, pw = power_trace(plan, a, b, every=7)
    full = run_gpu(plan, a0, b0)
    assert np.array_equal(a.cpu().numpy(), full[0]) and np.array_equal(b.cpu().numpy(), full[1])
    assert np.array_equal(pw[-1].cpu().numpy(), full[2])
    ends = [7, 14, 21, 28, 35, 40]
    assert np.allclose(z.cpu().numpy(), np.array(ends) * wl.lcr / wl.nz, rtol=0, atol=1e-15)
    for i, s in enumerate(ends):
        ref = run_oracle(wl, a0, b0, s_end=s)
        got = pw[i].cpu().numpy()
        assert abs(got[0] / ref["p_f"] - 1) < 1e-5 and abs(got[1] / ref["p_sh"] - 1) < 1e-5, s
    lossless = wl.with_(alpha_f=0.0, alpha_sh=0.0, beta_f=0.0, beta_sh=0.0)
    plan = make_plan(lossless)
    a = torch.from_numpy(a0).cuda()
    b = torch.from_numpy(b0).cuda()
    _, pw = power_trace(plan, a, b, every=5)
    tot = pw.sum(dim=1).cpu().numpy()
    c = ssfm.coefficients(lossless.params())
    p_in = ssfm.power(a0.astype(complex), lossless.n_f, c.dx, c.dy)
    assert pw[-1, 1].item() > 1e-3 * p_in
    assert np.max(np.abs(tot / p_in - 1)) < 1e-5


def test_check_finite_flag_names_the_bad_array():
    """SHG_CHECK_FINITE: NaN or Inf in an input is reported before the march
    (naming the array), a march that overflows is reported after it, and clean
    inputs give the same result as without the flag, bit for bit."""
    from paper_2410_04994_amd import Plan, ShgError, propagate_batch
    from paper_2410_04994_amd.binding import SHG_CHECK_FINITE
    wl = workloads.c2_plain_c64().with_(nx=64, ny=64, nz=12)
    plan = Plan(wl.params(), "c64", flags=SHG_CHECK_FINITE)
    a0, b0 = inputs(wl)
    dev = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()
    a, b = dev(a0), dev(b0)
    pw = plan.propagate(a, b)
    ref = run_gpu(make_plan(wl), a0, b0)
    assert np.array_equal(a.cpu().numpy(), ref[0]) and np.array_equal(b.cpu().numpy(), ref[1])
    assert np.array_equal(pw.cpu().numpy(), ref[2])
    bad = a0.copy()
    bad[5, 7] = np.nan
    with pytest.raises(ShgError, match="SHG_ENONFINITE.*input a_f"):
        plan.propagate(dev(bad), dev(b0))
    dk = np.full(wl.nz, wl.dk0)
    dk[3] = np.inf
    with pytest.raises(ShgError, match="SHG_ENONFINITE.*dk_z"):
        plan.propagate(dev(a0), dev(b0), dk_z=dev(dk))
    temp = np.full((wl.nz, 64, 64), wl.t_ref, np.float32)
    temp[2, 1, 1] = np.nan
    with pytest.raises(ShgError, match="SHG_ENONFINITE.*temp"):
        plan.propagate(dev(a0), dev(b0), temp=dev(temp))
    # a finite input so large that two-photon absorption overflows float
    with pytest.raises(ShgError, match="SHG_ENONFINITE.*output"):
        plan.propagate(dev(a0 * np.float32(1e19 / np.abs(a0).max())), dev(b0))
    # the adjoint checks its cotangents, the batch each instance
    g = np.zeros_like(a0)
    g[0, 0] = np.inf
    with pytest.raises(ShgError, match="SHG_ENONFINITE.*g_f_out"):
        plan.adjoint(dev(a0), dev(b0), g_f_out=dev(g))
    plans = [plan, Plan(wl.params(), "c64", flags=SHG_CHECK_FINITE)]
    with pytest.raises(ShgError, match=r"SHG_ENONFINITE.*a_f\[1\]"):
        propagate_batch(plans, [dev(a0), dev(bad)], [dev(b0), dev(b0)])


@pytest.mark.parametrize("n", [16, 32, 64, 128, 256, 512])
@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_transforms_on_white_noise(n, dtype):
    """The linear step alone (d_eff = 0, no two-photon absorption) on white-noise
    fields, which fill every frequency bin: two steps are IFFT(M FFT(.)) twice
    with the row and column transforms of every pass, against NumPy's FP64
    FFT in the oracle.  Loss keeps M off unit modulus."""
    wl = workloads.c2_plain_c64().with_(nx=n, ny=n, nz=2, d_eff=0.0, beta_f=0.0, beta_sh=0.0,
                                        lx=2e-4 * n / 64, ly=2e-4 * n / 64, lcr=2e-3)
    rng = np.random.Generator(np.random.PCG64(n))
    npdt = np.complex64 if dtype == "c64" else np.complex128
    a0 = ((rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))) * 1e6).astype(npdt)
    b0 = ((rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))) * 3e5).astype(npdt)
    plan = make_plan(wl, dtype)
    gpu = run_gpu(plan, a0, b0)
    ref = run_oracle(wl, a0, b0)
    tol = 2e-6 if dtype == "c64" else 1e-13
    assert rel(gpu[0], ref["a_f"]) < tol and rel(gpu[1], ref["a_sh"]) < tol
    # diffraction acted: the output differs from the input well beyond rounding
    assert rel(ref["a_sh"], b0.astype(complex)) > 1e-2


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_pointwise_nonlinear_step_on_random_states(dtype):
    """The nonlinear step alone on random states: a 1 m window makes the
    propagator the identity to ~1e-6 rad, so every cell runs the RK4 of its
    own state (coupling, two-photon absorption, a per-step mismatch profile),
    against the oracle's RK4."""
    n = 64
    wl = workloads.c2_plain_c64().with_(nx=n, ny=n, nz=30, lx=1.0, ly=1.0, alpha_f=0.0,
                                        alpha_sh=0.0, beta_f=1e-10, beta_sh=2e-10)
    rng = np.random.Generator(np.random.PCG64(5))
    npdt = np.complex64 if dtype == "c64" else np.complex128
    scale = 3e6
    a0 = ((rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))) * scale).astype(npdt)
    b0 = ((rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))) * 0.3 * scale).astype(npdt)
    dk = wl.dk0 + 2000.0 * rng.normal(size=wl.nz)
    plan = make_plan(wl, dtype)
    gpu = run_gpu(plan, a0, b0, dk_z=dk)
    ref = run_oracle(wl, a0, b0, dk_z=dk)
    tol = 1e-5 if dtype == "c64" else 1e-12
    assert rel(gpu[0], ref["a_f"]) < tol and rel(gpu[1], ref["a_sh"]) < tol
    # the nonlinearity acted on every cell
    lin = run_oracle(wl.with_(d_eff=0.0, beta_f=0.0, beta_sh=0.0), a0, b0, dk_z=dk)
    assert rel(ref["a_sh"], lin["a_sh"]) > 1e-2


def test_march_without_workspace_records_under_stream_capture():
    """shg_propagate without a workspace allocates nothing: the plan allocated
    its forward workspace when it was created.  So the call can be recorded
    into a caller's HIP graph (any allocation would end the capture with an
    error).  Every replay, with eager work and synchronisations between the
    replays, equals the eager march bit for bit."""
    from paper_2410_04994_amd import Plan
    wl = workloads.c2_plain_c64().with_(nx=64, ny=64, nz=24)
    plan = Plan(wl.params(), "c64")
    a0, b0 = inputs(wl)
    ae, be = torch.from_numpy(a0).cuda(), torch.from_numpy(b0).cuda()
    pe = plan.propagate(ae, be)
    torch.cuda.synchronize()
    a, b = torch.from_numpy(a0).cuda(), torch.from_numpy(b0).cuda()
    pw = torch.empty(2, dtype=torch.float64, device="cuda")
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        plan.propagate(a, b, powers=pw)
    for rep in range(3):
        a.copy_(torch.from_numpy(a0).cuda())
        b.copy_(torch.from_numpy(b0).cuda())
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(a, ae) and torch.equal(b, be) and torch.equal(pw, pe), rep


def test_graph_cache_keeps_several_argument_sets():
    """A plan keeps the graphs of its last few argument sets: marches on two
    sets of buffers, called alternately (as with fresh output tensors from an
    allocator), replay their own graphs and equal the one-by-one launches of
    an SHG_NO_GRAPH plan bit for bit."""
    from paper_2410_04994_amd import Plan
    from paper_2410_04994_amd.binding import SHG_NO_GRAPH
    wl = workloads.c2_plain_c64().with_(nx=64, ny=64, nz=20)
    a0, b0 = inputs(wl)
    ref = Plan(wl.params(), "c64", flags=SHG_NO_GRAPH)
    ra, rb = torch.from_numpy(a0).cuda(), torch.from_numpy(b0).cuda()
    rp = ref.propagate(ra, rb)
    plan = Plan(wl.params(), "c64")
    sets = [(torch.empty_like(ra), torch.empty_like(rb), torch.empty(2, dtype=torch.float64, device="cuda"))
            for _ in range(2)]
    for rnd in range(3):
        for a, b, pw in sets:
            a.copy_(torch.from_numpy(a0).cuda())
            b.copy_(torch.from_numpy(b0).cuda())
            plan.propagate(a, b, powers=pw)
            torch.cuda.synchronize()
            assert torch.equal(a, ra) and torch.equal(b, rb) and torch.equal(pw, rp), rnd
