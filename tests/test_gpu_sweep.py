"""GPU parity of the HIP sweep (called through the C ABI) against the CPU
oracle, element by element on the same seeded inputs.

Bars: FP64 within 1e-12 relative L2 of the FP64 oracle; FP32 within 1e-5 of
the oracle started from the same FP32-rounded values; the compensated FP32
pair judged on the increment u(T) - u(0) against the extended-precision
oracle (at large n the FP64 oracle's own rounding, about sqrt(S) ulps of u,
exceeds what the increment metric must resolve).
"""
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
    ge.lib()   # raises if libge.so is missing


def rel_l2(x, y):
    return float(np.linalg.norm(x - y) / max(np.linalg.norm(y), 1e-300))


def run_gpu(u0, r, nsteps, precision="fp64", step0=0, gl=0.0, gr=0.0, src_b=None,
            src_a=None, flux=False, **cfg):
    n = len(u0)
    dev_b = None
    if src_b is not None:
        dt = ge.state_dtype(precision)
        dev_b = torch.from_numpy(np.asarray(src_b)).to(dt).cuda()
    scalar_l, scalar_r = np.ndim(gl) == 0, np.ndim(gr) == 0
    plan = ge.Plan(n, r, precision, g_left=gl if scalar_l else 0.0,
                   g_right=gr if scalar_r else 0.0, src_b=dev_b, **cfg)
    u = ge.pack_state(u0, precision)
    d = lambda a: None if a is None else torch.from_numpy(np.asarray(a, dtype=np.float64)).cuda()
    fl = torch.zeros(2, dtype=torch.float64, device="cuda") if flux else None
    plan.step_n(u, step0, nsteps, g_left_t=None if scalar_l else d(gl),
                g_right_t=None if scalar_r else d(gr), src_a_t=d(src_a), flux=fl)
    torch.cuda.synchronize()
    out = ge.unpack_state(u, n, precision)
    if flux:
        return out, fl.cpu().numpy()
    return out


def start_values(u0, precision):
    """The FP64 values the GPU state actually starts from."""
    return ge.unpack_state(ge.pack_state(u0, precision), len(u0), precision)


# ---------------------------------------------------------------- C1 ------
def test_sine_decay_closed_form_fp64():
    """N = 1024, r = 1 (twice the explicit limit), 1000 levels, u0 = sin(pi x)."""
    n, r, s = 1024, 1.0, 1000
    u0 = inputs.sine_pulse(n)
    got = run_gpu(u0, r, s)
    want = oracle.step_n(u0, r, s)
    assert rel_l2(got, want) < 1e-12
    h, x = oracle.grid(n)
    exact = np.exp(-np.pi ** 2 * s * r * h * h) * np.sin(np.pi * x)
    assert rel_l2(got, exact) < 2e-7


def test_max_norm_never_grows_at_r_one():
    rng = np.random.default_rng(21)
    n = 3000
    u0 = rng.uniform(-1, 1, n)
    plan = ge.Plan(n, 1.0, "fp64", tile=8, waves=1, depth=4)
    u = ge.pack_state(u0, "fp64")
    prev = float(u.abs().max())
    for m in range(60):
        plan.step_n(u, m, 1)
        cur = float(u.abs().max())
        assert cur <= prev * (1 + 1e-15)
        prev = cur


# ------------------------------------------------------- multi-tile ------
CONFIGS_FP64 = [dict(tile=8, waves=1, depth=1), dict(tile=8, waves=1, depth=8),
                dict(tile=16, waves=1, depth=13), dict(tile=16, waves=4, depth=32),
                dict(tile=8, waves=4, depth=64), dict(tile=32, waves=1, depth=48),
                dict(tile=32, waves=4, depth=96)]


@pytest.mark.parametrize("cfg", CONFIGS_FP64, ids=lambda c: f"k{c['tile']}w{c['waves']}d{c['depth']}")
@pytest.mark.parametrize("n", [5000, 4099, 12289])
@pytest.mark.parametrize("step0", [0, 1])
def test_fp64_multi_tile_parity(cfg, n, step0):
    u0 = inputs.sine_rod(n, seed=n) + 0.3 * np.random.default_rng(n).standard_normal(n)
    s = 37
    got = run_gpu(u0, 2.0, s, step0=step0, gl=0.25, gr=-0.6, **cfg)
    want = oracle.step_n(u0, 2.0, s, step0=step0, gl=0.25, gr=-0.6)
    assert rel_l2(got, want) < 1e-12


@pytest.mark.parametrize("precision,cfg", [
    ("fp64", dict(tile=16, waves=4, depth=16)), ("fp64", dict(tile=8, waves=1, depth=5)),
    ("fp32", dict(tile=32, waves=4, depth=16)), ("fp32", dict(tile=16, waves=1, depth=7)),
    ("fp32c", dict(tile=16, waves=4, depth=16)), ("fp32c", dict(tile=8, waves=1, depth=9)),
])
def test_moving_walls_source_and_flux(precision, cfg):
    n, r, s = 20000, 4.0, 150
    w = inputs.moving_wall_rod(n, r=r, nsteps=s)
    rng = np.random.default_rng(5)
    u0 = 0.1 * rng.standard_normal(n)
    v0 = start_values(u0, precision)
    got, fl = run_gpu(u0, r, s, precision, gl=w.g_left, gr=w.g_right + 0.5,
                      src_b=w.src_b, src_a=w.src_a, flux=True, **cfg)
    src_b = w.src_b if precision == "fp64" else w.src_b.astype(np.float32).astype(np.float64)
    want_fl = np.zeros(2)
    want = oracle.step_n(v0, r, s, gl=w.g_left, gr=w.g_right + 0.5, src_b=src_b,
                         src_a=w.src_a, flux=want_fl)
    # rough data: every level's increment is O(u), so both FP32 forms carry
    # FP32 rounding of the increment itself
    tol = {"fp64": 1e-12, "fp32": 1e-5, "fp32c": 1e-5}[precision]
    assert rel_l2(got, want) < tol
    np.testing.assert_allclose(fl, want_fl, rtol=tol * 10)


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp32c"])
def test_bitwise_invariance_across_tiling_depth_and_calls(precision):
    n, s = 30011, 40
    rng = np.random.default_rng(17)
    u0 = inputs.sine_rod(n, 17) + 0.05 * rng.standard_normal(n)
    tiles = {"fp64": (2, 4, 8, 16, 20, 24, 28, 32, 64), "fp32": (4, 8, 16, 32), "fp32c": (4, 8, 16)}[precision]
    results = []
    for tile in tiles:
        for waves in (1, 4):
            for depth in (1, 6, 17, 40):
                try:
                    results.append(run_gpu(u0, 3.0, s, precision, step0=3, gl=0.1, gr=0.2,
                                           tile=tile, waves=waves, depth=depth))
                except ge.GEError as err:   # halo too wide for this window
                    assert err.status == ge.GE_ERR_INVALID
    assert len(results) >= 3 * len(tiles)
    for r_ in results[1:]:
        np.testing.assert_array_equal(r_, results[0])
    # split into calls
    plan = ge.Plan(n, 3.0, precision, g_left=0.1, g_right=0.2, tile=tiles[0], waves=4, depth=9)
    u = ge.pack_state(u0, precision)
    ws = plan.new_workspace()
    for a, b in ((3, 5), (8, 1), (9, 20), (29, 14)):
        plan.step_n(u, a, b, workspace=ws)
    np.testing.assert_array_equal(ge.unpack_state(u, n, precision), results[0])


@pytest.mark.parametrize("precision", ["fp32", "fp32c"])
def test_fp32_parity(precision):
    n, r, s = 7001, 2.0, 300
    u0 = inputs.sine_rod(n, 9) + 0.2
    v0 = start_values(u0, precision)
    got = run_gpu(u0, r, s, precision, gl=0.2, gr=0.2)
    want = oracle.step_n(v0, r, s, gl=0.2, gr=0.2, extended=(precision == "fp32c"))
    assert rel_l2(got, want) < 1e-5
    inc = rel_l2(got - v0, want - v0)
    if precision == "fp32c":
        assert inc < 1e-6, inc


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp32c"])
@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 63, 64, 65, 1023, 1024, 1025, 4095, 4096,
                               4097, 4098, 8191, 8193])
def test_edge_sizes(precision, n):
    rng = np.random.default_rng(n)
    u0 = rng.uniform(-1, 1, n)
    v0 = start_values(u0, precision)
    tol = 1e-12 if precision == "fp64" else 2e-5
    for step0, s in ((0, 1), (1, 1), (0, 2), (1, 7), (0, 33)):
        got = run_gpu(u0, 1.7, s, precision, step0=step0, gl=0.4, gr=-0.9,
                      tile=16, waves=4, depth=8)
        want = oracle.step_n(v0, 1.7, s, step0=step0, gl=0.4, gr=-0.9,
                             extended=(precision == "fp32c"))
        assert rel_l2(got, want) < tol, (step0, s)


def test_zero_steps_is_a_no_op():
    u0 = np.arange(10000, dtype=np.float64)
    np.testing.assert_array_equal(run_gpu(u0, 2.0, 0), u0)


def test_comp_checkpoint_round_trip():
    rng = np.random.default_rng(2)
    x = torch.from_numpy(rng.standard_normal(1000)).cuda()
    pair = ge.comp_from_fp64(x)
    y = ge.comp_to_fp64(pair, 1000)
    torch.cuda.synchronize()
    err = (x - y).abs().max().item()
    assert err <= 1e-14 * x.abs().max().item()


# ----------------------------------------------- full-size, sampled ------
def _samples(n, width=64):
    return [(0, width), (n // 2 - width // 2, n // 2 + width // 2),
            (int(0.3137 * n) // 2 * 2, int(0.3137 * n) // 2 * 2 + width), (n - width, n)]


def test_single_rod_2p24_fp64_sampled():
    """N = 2^24, r = 2, 10^4 levels, seeded sine modes: sampled blocks against
    the oracle evaluated on each block's dependence window."""
    n, r, s = 1 << 24, 2.0, 10000
    u0 = inputs.sine_rod(n, seed=2)
    plan = ge.Plan(n, r, "fp64")
    u = ge.pack_state(u0, "fp64")
    plan.step_n(u, 0, s)
    torch.cuda.synchronize()
    got = u.cpu().numpy()
    for lo, hi in _samples(n):
        want = oracle.window_step_n(u0, lo, hi, r, s)
        err = np.linalg.norm(got[lo:hi] - want)
        assert err <= 1e-12 * np.linalg.norm(want) + 1e-300, (lo, hi, err)


def test_single_rod_2p24_increment_vs_extended_oracle():
    """FP64 and the compensated pair on the N = 2^24 rod, judged on the
    increment u(T) - u(0) against the extended-precision oracle.  Over 10^4
    levels u changes by ~1e-9 relative, and each level's second difference
    is ~1e-13 of u: the FP64 state resolves it to ~1e-16 of u, the float pair
    (about 48 significant bits) to ~2^5 times that."""
    n, r, s = 1 << 24, 2.0, 10000
    u0 = inputs.sine_rod(n, seed=2)
    for precision, bar in (("fp64", 2e-6), ("fp32c", 5e-5)):
        v0 = start_values(u0, precision)
        plan = ge.Plan(n, r, precision)
        u = ge.pack_state(u0, precision)
        plan.step_n(u, 0, s)
        torch.cuda.synchronize()
        got = ge.unpack_state(u, n, precision)
        for lo, hi in _samples(n)[1:3]:
            want = oracle.window_step_n(v0, lo, hi, r, s, extended=True)
            inc = rel_l2(got[lo:hi] - v0[lo:hi], want - v0[lo:hi])
            assert inc < bar, (precision, lo, hi, inc)
            assert rel_l2(got[lo:hi], want) < 1e-12


def test_compensated_increment_at_2p20():
    """At N = 2^20 (second differences 256x larger than at 2^24) the pair
    resolves the increment to better than 1e-6."""
    n, r, s = 1 << 20, 2.0, 2000
    u0 = inputs.sine_rod(n, seed=2)
    v0 = start_values(u0, "fp32c")
    plan = ge.Plan(n, r, "fp32c")
    u = ge.pack_state(u0, "fp32c")
    plan.step_n(u, 0, s)
    torch.cuda.synchronize()
    got = ge.unpack_state(u, n, "fp32c")
    for lo, hi in _samples(n)[1:3]:
        want = oracle.window_step_n(v0, lo, hi, r, s, extended=True)
        inc = rel_l2(got[lo:hi] - v0[lo:hi], want - v0[lo:hi])
        assert inc < 1e-6, (lo, hi, inc)


@pytest.mark.parametrize("precision", ["fp64", "fp32c", "fp32"])
def test_single_rod_2p27_moving_walls_sampled(precision):
    """N = 2^27, r = 4, 5000 levels, g_L = sin(2 pi t), source exp(-t) x(1-x),
    u0 = 0.  Plain FP32 rounds u once per level, so over 5000 levels of a
    field that grows from zero it drifts by ~sqrt(5000) float roundings; the
    compensated pair is the FP32 form held to 1e-5."""
    n, r, s = 1 << 27, 4.0, 5000
    w = inputs.moving_wall_rod(n, r=r, nsteps=s)
    got = run_gpu(w.u0, r, s, precision, gl=w.g_left, gr=w.g_right, src_b=w.src_b,
                  src_a=w.src_a)
    src_b = w.src_b if precision == "fp64" else w.src_b.astype(np.float32).astype(np.float64)
    tol = {"fp64": 1e-12, "fp32c": 1e-5, "fp32": 5e-5}[precision]
    for lo, hi in ((0, 256), (n // 2, n // 2 + 64), (n - 256, n)):
        want = oracle.window_step_n(w.u0, lo, hi, r, s, gl=w.g_left, gr=w.g_right,
                                    src_b=src_b, src_a=w.src_a)
        assert rel_l2(got[lo:hi], want) < tol, (lo, hi)


# ------------------------------------------------- persistent schedule ----
@pytest.mark.parametrize("precision,tile", [("fp64", 16), ("fp64", 32), ("fp64", 64), ("fp32", 16),
                                            ("fp32", 32), ("fp32c", 16)])
def test_persistent_schedule_is_bitwise_the_per_tile_schedule(precision, tile):
    """The persistent kernel sweeps the same tiles with the same arithmetic:
    same bits, with walls, a source, per-level walls and the flux; rods whose
    last tile is short put two tiles on the wall path."""
    rng = np.random.default_rng(tile)
    for n, depth in ((200003, 17), (64 * tile * 7 + 5, 40), (64 * tile * 3 - 1, 9)):
        w = inputs.moving_wall_rod(n, r=3.0, nsteps=53, step0=1)
        u0 = inputs.sine_rod(n, n) + 0.05 * rng.standard_normal(n)
        runs = []
        for schedule in (1, 2):
            got, fl = run_gpu(u0, 3.0, 53, precision, step0=1, gl=w.g_left, gr=0.3,
                              src_b=w.src_b, src_a=w.src_a, flux=True, tile=tile, waves=1,
                              depth=depth, schedule=schedule)
            runs.append((got, fl))
        np.testing.assert_array_equal(runs[0][0], runs[1][0])
        np.testing.assert_array_equal(runs[0][1], runs[1][1])
    plan = ge.Plan(200003, 3.0, precision, tile=tile, waves=1, depth=17, schedule=2)
    assert plan.config()["schedule"] == 2


def test_persistent_schedule_fp64_parity():
    n, s = 300007, 97
    u0 = inputs.sine_rod(n, 3) + 0.1 * np.random.default_rng(3).standard_normal(n)
    got = run_gpu(u0, 2.0, s, "fp64", step0=0, gl=0.5, gr=-0.25, tile=16, waves=1, depth=48,
                  schedule=2)
    want = oracle.step_n(u0, 2.0, s, gl=0.5, gr=-0.25)
    assert rel_l2(got, want) < 1e-12


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp32c"])
def test_split_wall_launch_is_bitwise_the_single_launch(precision):
    """Launches of very many tiles (here more than 128 per CU: 2^23 points at
    2 or 4 points per lane, one level per launch) run the wall tiles and the
    interior tiles as two kernels; a plan of few large tiles runs one.  Same
    bits, with moving walls, a source and the flux."""
    n, s = (1 << 23) + 5, 7
    w = inputs.moving_wall_rod(n, r=3.0, nsteps=s, step0=3)
    u0 = inputs.sine_rod(n, 7) + 0.05 * np.random.default_rng(7).standard_normal(n)
    tile = 2 if precision == "fp64" else 4
    runs = []
    for cfg in (dict(tile=tile, waves=1, depth=1, schedule=1),
                dict(tile=16, waves=4, depth=s, schedule=1)):
        runs.append(run_gpu(u0, 3.0, s, precision, step0=3, gl=w.g_left, gr=0.2, src_b=w.src_b,
                            src_a=w.src_a, flux=True, **cfg))
    np.testing.assert_array_equal(runs[0][0], runs[1][0])
    np.testing.assert_array_equal(runs[0][1], runs[1][1])


@pytest.mark.parametrize("tile,waves,depth", [(20, 1, 64), (20, 4, 23), (16, 1, 64), (24, 1, 64),
                                              (28, 1, 80), (28, 4, 31)])
def test_source_tiles_bitwise(tile, waves, depth):
    """FP64 with moving walls and a source: every tile, wave count and depth
    gives the bits of a reference plan (8 points per lane, 9 levels)."""
    n, s = 300007, 130
    w = inputs.moving_wall_rod(n, r=4.0, nsteps=s, step0=2)
    u0 = inputs.sine_rod(n, 3) + 0.05 * np.random.default_rng(3).standard_normal(n)
    ref, fref = run_gpu(u0, 4.0, s, "fp64", step0=2, gl=w.g_left, gr=-0.3, src_b=w.src_b,
                        src_a=w.src_a, flux=True, tile=8, waves=1, depth=9)
    got, fgot = run_gpu(u0, 4.0, s, "fp64", step0=2, gl=w.g_left, gr=-0.3, src_b=w.src_b,
                        src_a=w.src_a, flux=True, tile=tile, waves=waves, depth=depth)
    np.testing.assert_array_equal(got, ref)
    np.testing.assert_array_equal(fgot, fref)


def test_split_launch_captured_in_a_graph():
    """A plan whose launches split off their wall tiles (the wall kernel on
    the plan's second stream, forked from and joined back into the caller's
    stream) can be captured: every replay equals an eager call, with eager
    work and synchronisations between the replays."""
    n, s = (1 << 23) + 5, 6
    u0 = inputs.sine_rod(n, 7) + 0.05 * np.random.default_rng(11).standard_normal(n)
    plan = ge.Plan(n, 3.0, "fp64", g_left=0.2, g_right=-0.1, tile=2, waves=1, depth=1, schedule=1)
    ws = plan.new_workspace()
    ref = ge.pack_state(u0, "fp64")
    plan.step_n(ref, 0, s, workspace=ws)            # eager warm-up, and the first reference
    torch.cuda.synchronize()
    u = ge.pack_state(u0, "fp64")
    g = torch.cuda.CUDAGraph()
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(stream):
        with torch.cuda.graph(g, stream=stream):
            plan.step_n(u, 0, s, workspace=ws)
    torch.cuda.synchronize()
    u.copy_(ge.pack_state(u0, "fp64"))
    torch.cuda.synchronize()
    for rep in range(3):
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(u, ref), f"replay {rep}"
        # eager work between replays: the next reference, from the same state
        nxt = ref.clone()
        plan.step_n(nxt, 0, s, workspace=ws)
        torch.cuda.synchronize()
        ref = nxt
