"""Batched march: every instance equals its own single-instance march, sampled
instances match the oracle, graph replays are deterministic (needs the GPU)."""
import os

import numpy as np
import pytest

import workloads
from gpu_util import inputs, run_oracle, compare, rel

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def small_batch(n=24, seed=9, max_nz=30):
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    base = workloads.c3_batch(n_instances=n, seed=seed)
    for i, w in enumerate(base):
        size = [32, 64, 128][i % 3]
        out.append(w.with_(nx=size, ny=size, nz=int(rng.integers(3, max_nz + 1)),
                           lx=w.lx * size / w.nx, ly=w.ly * size / w.nx))
    return out


def run_batch(wls, dtype="c64", dk=None):
    from paper_2410_04994_amd import Plan, propagate_batch
    plans = [Plan(w.params(), dtype) for w in wls]
    ins = [inputs(w, dtype) for w in wls]
    a = [torch.from_numpy(x[0]).cuda() for x in ins]
    b = [torch.from_numpy(x[1]).cuda() for x in ins]
    dks = [torch.from_numpy(d).cuda() for d in dk] if dk is not None else None
    pw = propagate_batch(plans, a, b, dk_z=dks)
    torch.cuda.synchronize()
    return plans, ins, [x.cpu().numpy() for x in a], [x.cpu().numpy() for x in b], pw.cpu().numpy()


def test_wide_batch_schedule_matches_narrow():
    """The wide row pass inside batches gives the same instances as the
    narrow one to rounding."""
    wls = small_batch(n=6, seed=11, max_nz=12)
    from paper_2410_04994_amd import Plan, propagate_batch
    outs = []
    for sched in ((1, 256, 4, 4), None):
        plans = [Plan(w.params(), "c64") for w in wls]
        if sched:
            for p in plans:
                p.set_batch_schedule(*sched)
        ins = [inputs(w) for w in wls]
        a = [torch.from_numpy(x[0]).cuda() for x in ins]
        b = [torch.from_numpy(x[1]).cuda() for x in ins]
        propagate_batch(plans, a, b)
        torch.cuda.synchronize()
        outs.append([x.cpu().numpy() for x in b])
    for x, y in zip(*outs):
        assert rel(x, y) < 1e-5


def batch_schedule(plan):
    """(row_e, row_wg, col_e, col_tc) the plan uses inside batches."""
    import re
    m = re.search(r"batch\(row e=(\d+) wg=(\d+) col e=(\d+) tc=(\d+)\)", plan.describe())
    return tuple(int(x) for x in m.groups())


def test_batch_equals_single_instance_runs_bitwise():
    from paper_2410_04994_amd import Plan
    wls = small_batch()
    plans, ins, A, B, pw = run_batch(wls)
    for i, w in enumerate(wls):
        p = Plan(w.params(), "c64")
        p.set_schedule(*batch_schedule(plans[i]))
        a = torch.from_numpy(ins[i][0]).cuda()
        b = torch.from_numpy(ins[i][1]).cuda()
        pp = p.propagate(a, b)
        torch.cuda.synchronize()
        assert np.array_equal(a.cpu().numpy(), A[i]), i
        assert np.array_equal(b.cpu().numpy(), B[i]), i
        assert np.array_equal(pp.cpu().numpy(), pw[i]), i


def test_batch_matches_oracle_and_replays_deterministically():
    from paper_2410_04994_amd import Plan, propagate_batch
    wls = small_batch(n=9, seed=4, max_nz=20)
    rng = np.random.Generator(np.random.PCG64(2))
    dk = [w.dk0 + 200 * rng.normal(size=w.nz) for w in wls]
    plans = [Plan(w.params(), "c64") for w in wls]
    ins = [inputs(w) for w in wls]
    dks = [torch.from_numpy(d).cuda() for d in dk]
    results = []
    for rep in range(3):      # first call runs directly, later calls replay the graph
        a = [torch.from_numpy(x[0]).cuda() for x in ins]
        b = [torch.from_numpy(x[1]).cuda() for x in ins]
        if rep == 0:
            keep = (a, b)
        else:
            for x, y in zip(keep[0], a):
                x.copy_(y)
            for x, y in zip(keep[1], b):
                x.copy_(y)
            a, b = keep
        pw = propagate_batch(plans, a, b, dk_z=dks)
        torch.cuda.synchronize()
        results.append(([x.cpu().numpy() for x in a], [x.cpu().numpy() for x in b], pw.cpu().numpy()))
    for r in results[1:]:
        assert all(np.array_equal(x, y) for x, y in zip(r[0], results[0][0]))
        assert all(np.array_equal(x, y) for x, y in zip(r[1], results[0][1]))
        assert np.array_equal(r[2], results[0][2])
    A, B, pw = results[0]
    for i, w in enumerate(wls):
        ref = run_oracle(w, ins[i][0], ins[i][1], dk_z=dk[i])
        compare(w, (A[i], B[i], pw[i]), ref, "c64", f"batch[{i}] {w.nx}x{w.ny}x{w.nz}")


def test_mixed_size_sweep_sampled_against_oracle():
    """The 512-instance sweep (64/128/256 in 1:2:1, nz in [200, 1000]) with its
    steps cut by 8 so the oracle check stays quick; every instance is checked
    against its own single-instance march, the smallest of each size against
    the oracle."""
    from paper_2410_04994_amd import Plan
    wls = [w.with_(nz=max(1, w.nz // 8)) for w in workloads.c3_batch()]
    plans, ins, A, B, pw = run_batch(wls)
    rng = np.random.Generator(np.random.PCG64(77))
    for i in rng.choice(len(wls), size=24, replace=False):
        w = wls[i]
        p = Plan(w.params(), "c64")
        p.set_schedule(*batch_schedule(plans[i]))
        a = torch.from_numpy(ins[i][0]).cuda()
        b = torch.from_numpy(ins[i][1]).cuda()
        p.propagate(a, b)
        torch.cuda.synchronize()
        assert np.array_equal(b.cpu().numpy(), B[i]), i
    for size in (64, 128, 256):
        idx = min((i for i, w in enumerate(wls) if w.nx == size), key=lambda i: wls[i].nz)
        w = wls[idx]
        ref = run_oracle(w, ins[idx][0], ins[idx][1])
        compare(w, (A[idx], B[idx], pw[idx]), ref, "c64", f"sweep[{idx}] {size}x{size}x{w.nz}")


def test_batch_argument_errors():
    from paper_2410_04994_amd import Plan, ShgError, propagate_batch
    w = small_batch(n=2)
    p64 = Plan(w[0].params(), "c64")
    p128 = Plan(w[1].params(), "c128")
    a = torch.zeros((w[0].ny, w[0].nx), dtype=torch.complex64, device="cuda")
    b = torch.zeros((w[1].ny, w[1].nx), dtype=torch.complex128, device="cuda")
    with pytest.raises(ShgError, match="dtype"):
        propagate_batch([p64, p128], [a, b], [a, b])
    with pytest.raises(ShgError, match="SHG_EINVAL"):
        propagate_batch([], [], [])


def test_lnl_batch_matches_single_marches_and_oracle():
    """A mixed-size batch in the L/2 - N - L/2 order: every instance equals its
    single-instance march (same schedule) bit for bit, and matches the oracle."""
    from paper_2410_04994_amd import Plan
    wls = [w.with_(split="LNL") for w in small_batch(n=9, seed=13, max_nz=20)]
    plans, ins, a_out, b_out, pw = run_batch(wls)
    for i, w in enumerate(wls):
        single = Plan(w.params(), "c64")
        single.set_schedule(*batch_schedule(plans[i]))
        a = torch.from_numpy(ins[i][0]).cuda()
        b = torch.from_numpy(ins[i][1]).cuda()
        single.propagate(a, b)
        assert np.array_equal(a.cpu().numpy(), a_out[i]) and np.array_equal(b.cpu().numpy(), b_out[i])
    for i in (0, 4, 8):
        ref = run_oracle(wls[i], ins[i][0], ins[i][1])
        compare(wls[i], (a_out[i], b_out[i], pw[i]), ref, "c64", f"lnl batch {i}")


def test_batch_rejects_mixed_split_orders():
    from paper_2410_04994_amd import Plan, ShgError, propagate_batch
    wls = small_batch(n=2, seed=3, max_nz=5)
    plans = [Plan(wls[0].params(), "c64"), Plan(wls[1].with_(split="LNL").params(), "c64")]
    a = [torch.ones((w.ny, w.nx), dtype=torch.complex64, device="cuda") for w in wls]
    b = [torch.zeros_like(x) for x in a]
    with pytest.raises(ShgError, match="split"):
        propagate_batch(plans, a, b)


def test_full_size_sweep_against_single_marches_and_oracle():
    """The 512-instance sweep at its full step counts (64/128/256 in 1:2:1, nz
    in [200, 1000]) with the schedules the benchmark uses: 16 sampled
    instances equal their own single-instance marches bit for bit, the
    shortest instance of each size matches the oracle, and so does the longest
    (the oracle's results for those are stored by
    tests/golden/make_full_size_refs.py)."""
    from paper_2410_04994_amd import Plan
    wls = workloads.c3_batch()
    print(f"case: c3 sweep, {len(wls)} instances, full nz", flush=True)
    plans, ins, A, B, pw = run_batch(wls)
    rng = np.random.Generator(np.random.PCG64(78))
    for i in rng.choice(len(wls), size=16, replace=False):
        w = wls[i]
        p = Plan(w.params(), "c64")
        p.set_schedule(*batch_schedule(plans[i]))
        a = torch.from_numpy(ins[i][0]).cuda()
        b = torch.from_numpy(ins[i][1]).cuda()
        p.propagate(a, b)
        torch.cuda.synchronize()
        assert np.array_equal(a.cpu().numpy(), A[i]) and np.array_equal(b.cpu().numpy(), B[i]), i
    for size in (64, 128, 256):
        idx = min((i for i, w in enumerate(wls) if w.nx == size), key=lambda i: wls[i].nz)
        w = wls[idx]
        ref = run_oracle(w, ins[idx][0], ins[idx][1])
        compare(w, (A[idx], B[idx], pw[idx]), ref, "c64", f"sweep[{idx}] {size}x{size}x{w.nz}")
    longest = np.load(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                                   "full_size", "c3_longest.npz"))
    for size in (64, 128, 256):
        idx = int(longest[f"index_{size}"])
        w = wls[idx]
        assert w.nx == size and w.nz == int(longest[f"nz_{size}"])
        assert w.nz == max(x.nz for x in wls if x.nx == size)
        a_in = ins[idx][0].astype(np.complex128)
        fp = np.array([float(np.sum(np.abs(a_in) ** 2)), a_in[size // 2, size // 2].real,
                       a_in[size // 2, size // 2].imag])
        assert np.allclose(fp, longest[f"input_{size}"], rtol=1e-12, atol=0)
        pr = longest[f"powers_{size}"]
        ref = {"a_f": longest[f"a_f_{size}"].astype(np.complex128),
               "a_sh": longest[f"a_sh_{size}"].astype(np.complex128), "p_f": pr[0], "p_sh": pr[1]}
        compare(w, (A[idx], B[idx], pw[idx]), ref, "c64", f"longest sweep[{idx}] {size}x{size}x{w.nz}")


def test_two_batches_alternating_through_one_caller_workspace():
    """Two different batches share one caller workspace and alternate.  Each
    batch's cached graph reads its descriptors from a table the library owns,
    so a replay never sees the other batch's descriptors: every instance stays
    bit for bit equal to its single-instance march."""
    from paper_2410_04994_amd import Plan, propagate_batch, batch_workspace_bytes
    batches = [small_batch(n=5, seed=21, max_nz=10), small_batch(n=7, seed=22, max_nz=12)]
    plans = [[Plan(w.params(), "c64") for w in wls] for wls in batches]
    ins = [[inputs(w) for w in wls] for wls in batches]
    singles = []
    for wls, ps, xs in zip(batches, plans, ins):
        out = []
        for w, p, (a0, b0) in zip(wls, ps, xs):
            single = Plan(w.params(), "c64")
            single.set_schedule(*batch_schedule(p))
            a, b = torch.from_numpy(a0).cuda(), torch.from_numpy(b0).cuda()
            pw = single.propagate(a, b)
            torch.cuda.synchronize()
            out.append((a.cpu().numpy(), b.cpu().numpy(), pw.cpu().numpy()))
        singles.append(out)
    nbytes = max(batch_workspace_bytes(ps) for ps in plans)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    for rnd in range(3):
        for k in (0, 1):
            a = [torch.from_numpy(x[0]).cuda() for x in ins[k]]
            b = [torch.from_numpy(x[1]).cuda() for x in ins[k]]
            pw = propagate_batch(plans[k], a, b, workspace=ws)
            torch.cuda.synchronize()
            for i, (sa, sb, sp) in enumerate(singles[k]):
                assert np.array_equal(a[i].cpu().numpy(), sa), (rnd, k, i)
                assert np.array_equal(b[i].cpu().numpy(), sb), (rnd, k, i)
                assert np.array_equal(pw[i].cpu().numpy(), sp), (rnd, k, i)


def test_batch_without_workspace_is_refused_under_capture_before_its_first_run():
    """A batch whose library-owned workspace does not exist yet would have to
    allocate it: under stream capture that is refused with SHG_EINVAL instead."""
    from paper_2410_04994_amd import Plan, ShgError, propagate_batch
    wls = small_batch(n=3, seed=23, max_nz=6)
    plans = [Plan(w.params(), "c64") for w in wls]
    a = [torch.from_numpy(inputs(w)[0]).cuda() for w in wls]
    b = [torch.zeros_like(x) for x in a]
    pw = torch.empty((3, 2), dtype=torch.float64, device="cuda")
    s = torch.cuda.Stream()
    graph = torch.cuda.CUDAGraph()
    with pytest.raises(ShgError, match="SHG_EINVAL.*capture"):
        with torch.cuda.graph(graph, stream=s, capture_error_mode="relaxed"):
            propagate_batch(plans, a, b, powers=pw, stream=s)
    torch.cuda.synchronize()
