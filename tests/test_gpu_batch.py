"""GPU parity of the persistent batch sweep (ge_batch_plan / ge_solve_batch)
against the CPU oracle rod by rod, bitwise agreement with the single-rod
path, and graph replay."""
import numpy as np
import pytest

import oracle
from paper_1310_3422_amd import ge, inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    ge.lib()


def rel_l2(x, y):
    return float(np.linalg.norm(x - y) / max(np.linalg.norm(y), 1e-300))


def run_batch(rb, precision, nsteps, step0=0, tune=False, sync=0):
    b = ge.Batch.from_inputs(rb, precision, tune=tune, sync=sync)
    u = ge.pack_batch_state(rb.u0, rb.offsets, rb.n, precision)
    ws = b.new_workspace()
    b.solve(u, step0, nsteps, ws)
    torch.cuda.synchronize()
    return b, u.cpu().numpy()


def start_rod(rb, i, precision):
    u = ge.pack_batch_state(rb.u0, rb.offsets, rb.n, precision).cpu().numpy()
    return ge.unpack_batch_rod(u, rb.offsets, rb.n, i, precision)


@pytest.mark.parametrize("sync", [1, 2, 3])
@pytest.mark.parametrize("precision", ["fp32", "fp64", "fp32c"])
def test_small_batch_parity(precision, sync):
    rb = inputs.rod_batch(seed=11, nrods=48, nmin=1, nmax=20000, align=4)
    nsteps = 120
    b, got = run_batch(rb, precision, nsteps, step0=1, sync=sync)
    tol = {"fp64": 1e-12, "fp32": 2e-5, "fp32c": 1e-6}[precision]
    for i in range(rb.nrods):
        v0 = start_rod(rb, i, precision)
        want = oracle.step_n(v0, rb.r[i], nsteps, step0=1, gl=rb.g_left[i], gr=rb.g_right[i],
                             extended=(precision == "fp32c"))
        g = ge.unpack_batch_rod(got, rb.offsets, rb.n, i, precision)
        assert rel_l2(g, want) < tol, (i, int(rb.n[i]))


@pytest.mark.parametrize("sync", [1, 2, 3])
@pytest.mark.parametrize("precision", ["fp32", "fp64", "fp32c"])
def test_batch_matches_single_rod_bitwise(precision, sync):
    rb = inputs.rod_batch(seed=12, nrods=24, nmin=3, nmax=30000, align=4)
    nsteps = 57
    b, got = run_batch(rb, precision, nsteps, step0=2, sync=sync)
    ks = b.info()["rod_k"]
    assert len(set(ks.tolist())) >= 2   # several points-per-lane choices in play
    for i in range(rb.nrods):
        n = int(rb.n[i])
        plan = ge.Plan(n, rb.r[i], precision, g_left=rb.g_left[i], g_right=rb.g_right[i])
        u = ge.pack_state(start_rod(rb, i, precision), precision)
        plan.step_n(u, 2, nsteps)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(ge.unpack_batch_rod(got, rb.offsets, rb.n, i, precision),
                                      ge.unpack_state(u, n, precision))


def _sized_batch(sizes, seed):
    rng = np.random.default_rng(seed)
    n = np.array(sizes, dtype=np.int64)
    padded = (n + 3) // 4 * 4
    offsets = np.zeros(n.size + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(padded)
    u0 = np.zeros(int(offsets[-1]))
    for i, m in enumerate(sizes):
        u0[offsets[i]:offsets[i] + m] = inputs.sine_modes(int(m), rng.standard_normal(16)) + \
            0.01 * rng.standard_normal(m)
    return inputs.RodBatch(n=n, r=rng.uniform(0.25, 4.0, n.size), g_left=rng.uniform(-1, 1, n.size),
                           g_right=rng.uniform(-1, 1, n.size), offsets=offsets, u0=u0)


@pytest.mark.parametrize("precision", ["fp32", "fp64", "fp32c"])
def test_halo_lane_tasks_at_wave_boundaries(precision):
    """Rods whose lengths sit at the edges of the overlapping-wave layout
    (one wave of 64k points, 62k more per further wave, the largest rod that
    fits 16 waves and the next one, which falls back to the per-level
    exchange) for k = 4..64: bit-identical to the single-rod sweep over a
    level count that is no multiple of any block length (k - 1)."""
    cap = 65536 if precision == "fp32" else 32768
    sizes = [1, 2, 3, 5, 6]
    for k in (4, 8, 16, 32, 64):
        for m in (64 * k, 64 * k + 62 * k, 64 * k + 15 * 62 * k):
            sizes += [m - 1, m, m + 1]
    sizes = sorted(set(x for x in sizes if x <= cap)) + [cap]
    rb = _sized_batch(sizes, seed=21)
    nsteps = 131
    b, got = run_batch(rb, precision, nsteps, step0=1, sync=3)
    for i in range(rb.nrods):
        n = int(rb.n[i])
        plan = ge.Plan(n, rb.r[i], precision, g_left=rb.g_left[i], g_right=rb.g_right[i])
        u = ge.pack_state(start_rod(rb, i, precision), precision)
        plan.step_n(u, 1, nsteps)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(ge.unpack_batch_rod(got, rb.offsets, rb.n, i, precision),
                                      ge.unpack_state(u, n, precision), err_msg=f"rod {i}, n={n}")


@pytest.mark.parametrize("precision", ["fp32", "fp64", "fp32c"])
def test_long_rods_match_single_rod_bitwise(precision):
    """Rods above the on-chip limit (65536 points FP32, 32768 FP64 and the
    pair) run as long-rod tasks (passes of up to 32 levels over single-wave
    windows with halos, in the same launch as on-chip rods): bit-identical to
    ge_step_n for level counts below, at and above one pass, even and odd,
    from both parities."""
    cap = 65536 if precision == "fp32" else 32768
    sizes = [cap + 1, cap + 3, cap + 1000, 2 * cap + 77, 100, 5000, cap, 1]
    rb = _sized_batch(sizes, seed=22)
    b = ge.Batch.from_inputs(rb, precision)
    ks = b.info()["rod_k"]
    assert b.workspace_bytes > 256   # the second level buffer of the long rods
    ws = b.new_workspace()
    u0 = ge.pack_batch_state(rb.u0, rb.offsets, rb.n, precision)
    for step0, nsteps in [(0, 1), (1, 2), (1, 33), (0, 64), (3, 131)]:
        u = u0.clone()
        b.solve(u, step0, nsteps, ws)
        b.check()
        got = u.cpu().numpy()
        for i in range(rb.nrods):
            n = int(rb.n[i])
            plan = ge.Plan(n, rb.r[i], precision, g_left=rb.g_left[i], g_right=rb.g_right[i])
            v = ge.pack_state(start_rod(rb, i, precision), precision)
            plan.step_n(v, step0, nsteps)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(ge.unpack_batch_rod(got, rb.offsets, rb.n, i, precision),
                                          ge.unpack_state(v, n, precision),
                                          err_msg=f"rod {i}, n={n}, k={ks[i]}, levels {step0}+{nsteps}")


def test_graph_replays_match_eager_result():
    """The first call captures the graph, later calls replay it; eager work
    and synchronisations run between replays, and every replay must give
    the same result."""
    rb = inputs.rod_batch(seed=13, nrods=64, nmin=64, nmax=40000, align=4)
    b = ge.Batch.from_inputs(rb, "fp32")
    u0 = ge.pack_batch_state(rb.u0, rb.offsets, rb.n, "fp32")
    ws = b.new_workspace()
    results = []
    for rep in range(4):
        u = u0.clone()
        junk = torch.randn(1 << 20, device="cuda").sum()   # eager work between replays
        b.solve(u, 0, 40, ws)
        torch.cuda.synchronize()
        results.append(u.cpu().numpy())
        float(junk)
    for r_ in results[1:]:
        np.testing.assert_array_equal(r_, results[0])
    # a different level count re-captures and still composes: 40 = 17 + 23
    u = u0.clone()
    b.solve(u, 0, 17, ws)
    b.solve(u, 17, 23, ws)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(u.cpu().numpy(), results[0])


def test_tuned_plan_gives_identical_results(tmp_path, monkeypatch):
    monkeypatch.setenv("GE_TUNE_CACHE", str(tmp_path / "tune.txt"))
    rb = inputs.rod_batch(seed=14, nrods=40, nmin=256, nmax=65536, align=4)
    b0, got0 = run_batch(rb, "fp32", 30)
    b1, got1 = run_batch(rb, "fp32", 30, tune=True)
    np.testing.assert_array_equal(got0, got1)
    assert (tmp_path / "tune.txt").exists()
    info = b1.info()
    assert info["ntasks"] >= 1 and info["est_us_per_level"] > 0


def _sampled_errors(rb, got, precision, nsteps, extra=()):
    rng = np.random.default_rng(0)
    pick = sorted(set([int(np.argmax(rb.n)), int(np.argmin(rb.n)), *extra] +
                      rng.choice(rb.nrods, 10, replace=False).tolist()))
    errs = []
    for i in pick:
        v0 = start_rod(rb, i, precision)
        want = oracle.step_n(v0, rb.r[i], nsteps, gl=rb.g_left[i], gr=rb.g_right[i],
                             extended=(precision == "fp32c"))
        errs.append(rel_l2(ge.unpack_batch_rod(got, rb.offsets, rb.n, i, precision), want))
    return pick, np.array(errs)


# rod 1103 of the seed-3 draw (n = 11694, r = 0.650): the plain-FP32 rod
# furthest from the oracle among the sampled ones
PLAIN_FP32_WORST = 1103


def _report(tag, rb, pick, errs):
    j = int(np.argmax(errs))
    i = pick[j]
    print("%s per-rod rel-L2 max %.3e (rod %d, n=%d, r=%.3f, gL=%+.3f, gR=%+.3f) median %.3e"
          % (tag, errs[j], i, rb.n[i], rb.r[i], rb.g_left[i], rb.g_right[i], np.median(errs)))


def test_rod_batch_4096_sampled_fp32():
    """4096 rods, N log-uniform in [256, 65536], r in [0.25, 4], walls in
    [-1, 1], 2000 levels, plain FP32: sampled rods against the oracle started
    from the same FP32-rounded values.  Plain FP32 rounds u once per level;
    where a level's increment is below half an FP32 unit of u (long rods,
    small r: the smooth modes change by about r pi^2 k^2 h^2 u per level) it
    is lost, so those rods lag the oracle: up to 2.14e-5 on rod 1103 (n =
    11694, r = 0.65), which a float32 emulation of the same arithmetic on the
    CPU reproduces to three digits.  The bar is that drift with a margin; the
    compensated pair takes the same draw to 1e-6 (next test)."""
    rb = inputs.rod_batch(seed=3, nrods=4096, align=4)
    b, got = run_batch(rb, "fp32", 2000)
    pick, errs = _sampled_errors(rb, got, "fp32", 2000, extra=(PLAIN_FP32_WORST,))
    _report("fp32", rb, pick, errs)
    assert errs.max() < 5e-5
    assert np.median(errs) < 5e-6


def test_rod_batch_4096_compensated_full_draw():
    """The whole seed-3 draw (N up to 65536: the rods above 32768 points run
    as long-rod tasks) in the compensated pair against the extended-precision
    oracle: the largest rods, the shortest, plain FP32's worst and ten
    random ones, every one within 1e-6."""
    rb = inputs.rod_batch(seed=3, nrods=4096, align=4)
    b, got = run_batch(rb, "fp32c", 2000)
    b.check()
    big = np.argsort(rb.n)[-3:].tolist()
    pick, errs = _sampled_errors(rb, got, "fp32c", 2000, extra=(PLAIN_FP32_WORST, *big))
    _report("fp32c", rb, pick, errs)
    assert max(rb.n[i] for i in pick) > 65000
    assert errs.max() < 1e-6


def test_rod_batch_4096_compensated_within_on_chip_range():
    """The same draw with N capped at 32768 (the compensated pair's on-chip
    limit), compensated FP32 against the extended oracle."""
    rb = inputs.rod_batch(seed=3, nrods=4096, nmax=32768, align=4)
    b, got = run_batch(rb, "fp32c", 2000)
    pick, errs = _sampled_errors(rb, got, "fp32c", 2000)
    _report("fp32c (on-chip)", rb, pick, errs)
    assert errs.max() < 1e-6
