"""Parity of the HIP heat source, heat-equation solver and self-consistent loop
with the FP64 oracle (needs the GPU).

Tolerances: complex128 plans (FP64 solver) agree to ~1e-9 of the temperature
rise; complex64 plans (FP32 vectors, FP64 reductions) to 2e-4 of the rise; heat
sources follow the field tolerances of the march (|A|^2 doubles the relative
error of the field)."""
import math

import numpy as np
import pytest

from oracle import beams, ssfm, thermal

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

LAM = 1064e-9


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def field_case(n=32, nz=24, power=300.0, **kw):
    lcr, xi = 8e-3, 1.5
    w0 = math.sqrt(lcr / (xi * 2 * math.pi * 2.14 / LAM))
    width = 8 * w0 * math.sqrt(1 + xi * xi)
    p = dict(nx=n, ny=n, nz=nz, lx=width, ly=width, lcr=lcr, lambda_f=LAM, n_f=2.14, n_sh=2.18,
             d_eff=10e-12, alpha_f=3.0, alpha_sh=8.0, beta_f=5e-11, beta_sh=8e-11, dk0=-100.0,
             ddk_dT=0.0, dn_dT=0.0, t_ref=330.0, undepleted=False)
    p.update(kw)
    a0 = beams.input_pump(p, power, w0, lcr / 2)
    return p, a0, np.zeros_like(a0)


def cdt(dtype):
    return (np.complex64, torch.complex64) if dtype == "c64" else (np.complex128, torch.complex128)


def presets(name):
    return {"bottom": {"y-": "oven"},
            "surrounding": {"x-": "oven", "x+": "oven", "y-": "oven", "y+": "oven"}}[name]


def oracle_tp(name, k_th, h_conv, t_inf, t_oven):
    return thermal.ThermalParams(k_th, h_conv, t_inf, t_oven, presets(name))


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_heat_source_of_the_march(dtype):
    from paper_2410_04994_amd import Plan
    p, a0, b0 = field_case()
    npdt, tdt = cdt(dtype)
    a0 = a0.astype(npdt)
    ref = thermal.march_heat(p, a0.astype(complex), b0)
    plan = Plan(p, dtype)
    a = torch.from_numpy(a0).cuda()
    b = torch.zeros_like(a)
    heat, powers = plan.propagate_heat(a, b)
    got = heat.cpu().numpy()
    tol = 3e-4 if dtype == "c64" else 1e-10
    assert rel(got, ref["q"]) < tol
    for l in (0, p["nz"] // 2, p["nz"]):
        assert rel(got[l], ref["q"][l]) < tol, l
    # the fields are those of the plain march, bit for bit
    a2 = torch.from_numpy(a0).cuda()
    b2 = torch.zeros_like(a2)
    plan.propagate(a2, b2)
    assert torch.equal(a, a2) and torch.equal(b, b2)


@pytest.mark.parametrize("method", ["direct", "cg"])
@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("preset", ["bottom", "surrounding"])
def test_heat_equation_solve(dtype, preset, method):
    from paper_2410_04994_amd import Thermal
    p = dict(nx=32, ny=32, nz=16, lx=0.9e-3, ly=0.7e-3, lcr=6e-3)
    k_th, h_conv, t_inf, t_oven = 4.6, 2e3, 295.0, 330.0
    rng = np.random.Generator(np.random.PCG64(17))
    shape = thermal.grid_shape(p)
    q = 1e8 * np.exp(rng.normal(size=shape) * 0.5)
    ref = thermal.solve(p, oracle_tp(preset, k_th, h_conv, t_inf, t_oven), q)
    rise = np.ptp(ref)
    th = Thermal(p, k_th, h_conv, t_inf, t_oven, presets(preset), dtype, method=method)
    rdt = torch.float32 if dtype == "c64" else torch.float64
    qd = torch.from_numpy(q).to(rdt).cuda()
    tol = 1e-6 if dtype == "c64" else 1e-13
    t_nodes, t_mid, it, res = th.solve(qd, tol=tol, max_iter=20000)
    got = t_nodes.cpu().numpy()
    bound = 2e-4 if dtype == "c64" else 1e-9
    if method == "cg":
        assert res <= tol and 0 < it < 20000
    else:
        # exact up to FP64 GEMM rounding (the residual is that of the FP64
        # solution; T is then rounded to the plan's precision)
        assert it == 0 and res < 1e-11
    assert np.max(np.abs(got - ref)) < bound * rise
    assert np.max(np.abs(t_mid.cpu().numpy() - thermal.midplanes(ref))) < bound * rise
    # a second solve (warm start for CG, cached factors for the direct solver)
    t2, _, it2, _ = th.solve(qd, t_nodes=t_nodes.clone(), tol=max(tol, 1e-5), max_iter=20000)
    assert it2 <= 16
    assert np.max(np.abs(t2.cpu().numpy() - ref)) < bound * rise


@pytest.mark.parametrize("method", ["direct", "cg"])
def test_no_drive_gives_the_oven_temperature(method):
    """No source and air at the oven temperature: T = T_oven exactly."""
    from paper_2410_04994_amd import Thermal
    p = dict(nx=16, ny=16, nz=6, lx=1e-3, ly=1e-3, lcr=2e-3)
    th = Thermal(p, 5.0, 50.0, 330.0, 330.0, presets("bottom"), "c64", method=method)
    q = torch.zeros(thermal.grid_shape(p), dtype=torch.float32, device="cuda")
    start = torch.full(thermal.grid_shape(p), 400.0, dtype=torch.float32, device="cuda")
    t, t_mid, it, res = th.solve(q, t_nodes=start)
    assert it == 0 and torch.all(t == 330.0) and torch.all(t_mid == 330.0)


@pytest.mark.parametrize("method", ["direct", "cg"])
def test_energy_balance_at_a_large_grid(method):
    """256 x 256 x 201 nodes (13 M), too many for the oracle's sparse solve: the
    FP32 solution must still balance the generated heat against the heat leaving
    through the air faces and into the oven."""
    from paper_2410_04994_amd import Thermal
    p = dict(nx=256, ny=256, nz=200, lx=0.9e-3, ly=0.9e-3, lcr=30e-3)
    k_th, h_conv, t_inf, t_oven = 4.6, 20.0, 295.0, 330.0
    shape = thermal.grid_shape(p)
    x, y = ssfm.coordinates(p)
    z = np.arange(p["nz"] + 1) * p["lcr"] / p["nz"]
    w = 60e-6
    q = (5e8 * np.exp(-0.2 * z)[:, None, None]
         * np.exp(-2 * (x[None, None, :] ** 2 + y[None, :, None] ** 2) / w ** 2)).astype(np.float32)
    th = Thermal(p, k_th, h_conv, t_inf, t_oven, presets("bottom"), "c64", method=method)
    t, _, it, res = th.solve(torch.from_numpy(q).cuda(), tol=1e-6, max_iter=40000)
    assert res <= (1e-9 if method == "direct" else 1e-6)
    src, loss = thermal.energy_balance(p, oracle_tp("bottom", k_th, h_conv, t_inf, t_oven),
                                       t.cpu().numpy().astype(np.float64), q.astype(np.float64))
    assert abs(loss / src - 1) < 1e-3


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_self_consistent_loop(dtype):
    from paper_2410_04994_amd import Plan, Thermal, self_consistent
    p, a0, b0 = field_case(n=16, nz=12, power=30.0, alpha_f=0.5, alpha_sh=3.0, ddk_dT=300.0,
                           dn_dT=1e-5)
    npdt, tdt = cdt(dtype)
    a0 = a0.astype(npdt)
    k_th, h_conv, t_inf, t_oven = 2.0, 20.0, 295.0, 330.0
    tol_t = 1e-7 if dtype == "c128" else 1e-3
    ref_t, ref_m, hist = thermal.self_consistent(p, oracle_tp("bottom", k_th, h_conv, t_inf, t_oven),
                                                 a0.astype(complex), b0, tol=tol_t)
    plan = Plan(p, dtype)
    th = Thermal(p, k_th, h_conv, t_inf, t_oven, presets("bottom"), dtype)
    out = self_consistent(plan, th, torch.from_numpy(a0).cuda(), torch.zeros(a0.shape, dtype=tdt,
                                                                               device="cuda"),
                          tol_t=tol_t, solve_tol=1e-13 if dtype == "c128" else 1e-6, max_iter=20000)
    rise = np.ptp(ref_t)
    assert rise > 1.0
    got_t = out["t_nodes"].cpu().numpy()
    if dtype == "c128":
        assert abs(out["outer"] - len(hist)) <= 1
        assert np.max(np.abs(got_t - ref_t)) < 1e-7 * rise
        assert rel(out["a_sh"].cpu().numpy(), ref_m["a_sh"]) < 1e-7
    else:
        assert out["change"] <= tol_t
        assert np.max(np.abs(got_t - ref_t)) < 2e-3 * rise
        assert rel(out["a_sh"].cpu().numpy(), ref_m["a_sh"]) < 1e-3


@pytest.mark.parametrize("method", ["direct", "cg"])
def test_non_square_grid_and_single_step(method):
    """64 x 16 nodes per plane and a single z-step (two planes of nodes), with
    the oven on the x+ face and an insulated z- face."""
    from paper_2410_04994_amd import Thermal
    p = dict(nx=64, ny=16, nz=1, lx=1.2e-3, ly=0.3e-3, lcr=0.2e-3)
    faces = {"x+": "oven", "z-": "insulated"}
    k_th, h_conv, t_inf, t_oven = 3.0, 5e3, 300.0, 340.0
    rng = np.random.Generator(np.random.PCG64(23))
    q = 1e9 * np.exp(rng.normal(size=thermal.grid_shape(p)))
    ref = thermal.solve(p, thermal.ThermalParams(k_th, h_conv, t_inf, t_oven, faces), q)
    th = Thermal(p, k_th, h_conv, t_inf, t_oven, faces, "c128", method=method)
    t, t_mid, it, res = th.solve(torch.from_numpy(q).cuda(), tol=1e-13, max_iter=50000)
    assert np.max(np.abs(t.cpu().numpy() - ref)) < 1e-9 * np.ptp(ref)
    assert t_mid.shape == (1, 16, 64)


@pytest.mark.parametrize("faces,nz", [
    ({"z-": "oven"}, 8),                                   # oven on a z face
    ({"z-": "oven", "z+": "oven"}, 2),                     # one free plane along z
    ({"x-": "insulated", "x+": "insulated", "y-": "insulated", "y+": "insulated",
      "z+": "oven"}, 12),                                  # zero shift for the (0, 0) mode
    ({}, 5),                                               # convective faces only
    ({"x-": "insulated", "x+": "insulated", "y-": "insulated", "y+": "insulated",
      "z-": "insulated"}, 7),                              # one convective face, no oven
])
def test_direct_solve_z_lines(faces, nz):
    """The direct solver diagonalises x and y and eliminates along z, one
    tridiagonal system per (x, y) mode pair.  Face layouts that change the z
    system: ovens on z faces (fewer free planes, down to one), insulated x and
    y faces (the (0, 0) mode adds nothing to the z diagonal, so the z system
    alone must be regular), and convective faces only."""
    from paper_2410_04994_amd import Thermal
    p = dict(nx=16, ny=32, nz=nz, lx=0.5e-3, ly=0.8e-3, lcr=1.5e-3)
    k_th, h_conv, t_inf, t_oven = 6.0, 3e3, 297.0, 335.0
    rng = np.random.Generator(np.random.PCG64(31 + nz))
    q = 1e9 * np.exp(rng.normal(size=thermal.grid_shape(p)))
    ref = thermal.solve(p, thermal.ThermalParams(k_th, h_conv, t_inf, t_oven, faces), q)
    th = Thermal(p, k_th, h_conv, t_inf, t_oven, faces, "c128", method="direct")
    t, _, it, res = th.solve(torch.from_numpy(q).cuda())
    assert it == 0 and res < 1e-11
    assert np.max(np.abs(t.cpu().numpy() - ref)) < 1e-9 * np.ptp(ref)


def test_every_node_on_an_oven():
    """Ovens on both z faces of a single step: no free node, T = T_oven."""
    from paper_2410_04994_amd import Thermal
    p = dict(nx=16, ny=16, nz=1, lx=1e-3, ly=1e-3, lcr=1e-4)
    th = Thermal(p, 5.0, 10.0, 300.0, 330.0, {"z-": "oven", "z+": "oven"}, "c64")
    q = torch.full(thermal.grid_shape(p), 1e9, dtype=torch.float32, device="cuda")
    t, t_mid, it, res = th.solve(q)
    assert torch.all(t == 330.0) and torch.all(t_mid == 330.0)


def test_self_consistent_loop_with_cg():
    from paper_2410_04994_amd import Plan, Thermal, self_consistent
    p, a0, b0 = field_case(n=16, nz=12, power=30.0, alpha_f=0.5, alpha_sh=3.0, ddk_dT=300.0,
                           dn_dT=1e-5)
    k_th, h_conv, t_inf, t_oven = 2.0, 20.0, 295.0, 330.0
    ref_t, _, _ = thermal.self_consistent(p, oracle_tp("bottom", k_th, h_conv, t_inf, t_oven),
                                          a0, b0, tol=1e-7)
    plan = Plan(p, "c128")
    th = Thermal(p, k_th, h_conv, t_inf, t_oven, presets("bottom"), "c128", method="cg")
    out = self_consistent(plan, th, torch.from_numpy(a0).cuda(),
                          torch.zeros(a0.shape, dtype=torch.complex128, device="cuda"),
                          tol_t=1e-7, solve_tol=1e-13, max_iter=20000)
    assert np.max(np.abs(out["t_nodes"].cpu().numpy() - ref_t)) < 1e-7 * np.ptp(ref_t)


def test_full_size_temperature_field_march_deposits_the_lost_power():
    """The 50 W temperature-field workload at its full size (512 x 512 x 2000,
    the synthetic T field), in the schedule the benchmark uses: the heat source
    written at the 2001 step boundaries, integrated over the crystal
    (trapezoid in z), equals the power the two fields lose.  The lens and the
    mismatch only rotate phases, so this holds at any size; the residual is
    the O(dz^2) of the trapezoid and the FP32 rounding of the powers."""
    import workloads
    from paper_2410_04994_amd import Plan, autotune, beams as gbeams
    wl = workloads.c5_thermal_c64()
    print(f"case: {wl.name}", flush=True)
    temp = torch.from_numpy(workloads.radial_temperature_profile(wl).astype(np.float32)).cuda()
    plan = Plan(wl.params(), "c64")
    autotune.tune_single(plan)
    a = gbeams.pump_for(wl, dtype=torch.complex64, device="cuda")
    c = ssfm.coefficients(wl.params())
    p_in = ssfm.power(a.cpu().numpy().astype(complex), wl.n_f, c.dx, c.dy)
    b = torch.zeros_like(a)
    heat, powers = plan.propagate_heat(a, b, temp=temp)
    torch.cuda.synchronize()
    del temp
    per_plane = heat.double().sum(dim=(1, 2)).cpu().numpy() * c.dx * c.dy
    absorbed = float(np.trapezoid(per_plane, dx=c.dz))
    p_f, p_sh = powers.cpu().numpy()
    lost = p_in - (p_f + p_sh)
    assert p_sh > 0.1 * p_in                              # strong conversion
    assert lost > 0.0
    assert abs(absorbed / lost - 1) < 1e-3, (absorbed, lost)
