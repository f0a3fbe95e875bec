"""GPU parity of the sub-domain scheme (Section 2, sub-domains of k nodes;
ge_plan with desc.k >= 2, called through the C ABI) against the CPU oracle
oracle.sdc_step_n, element by element on the same seeded inputs.

Bars: FP64 within 1e-12 relative L2 of the FP64 oracle; FP32 within 1e-5 of
the oracle started from the same FP32-rounded values.  Sizes span single
windows (64 sub-domain couples or fewer, advanced in place), several tiles
and a ragged last tile."""
import numpy as np
import pytest

import oracle
from paper_1310_3422_amd import ge

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    ge.lib()


def rel_l2(x, y):
    return float(np.linalg.norm(x - y) / max(np.linalg.norm(y), 1e-300))


def run(u0, r, k, nsteps, precision="fp64", step0=0, gl=0.0, gr=0.0, depth=0, schedule=0,
        waves=0):
    n = len(u0)
    scalar_l, scalar_r = np.ndim(gl) == 0, np.ndim(gr) == 0
    plan = ge.Plan(n, r, precision, g_left=gl if scalar_l else 0.0,
                   g_right=gr if scalar_r else 0.0, depth=depth, k=k, schedule=schedule,
                   waves=waves)
    u = ge.pack_state(u0, precision)
    d = lambda a: torch.from_numpy(np.asarray(a, dtype=np.float64)).cuda()
    plan.step_n(u, step0, nsteps, g_left_t=None if scalar_l else d(gl),
                g_right_t=None if scalar_r else d(gr))
    torch.cuda.synchronize()
    return ge.unpack_state(u, n, precision), plan.config()


def rough(n, seed):
    rng = np.random.default_rng(seed)
    x = np.arange(1, n + 1) / (n + 1)
    return np.sin(np.pi * x) + 0.3 * np.sin(7 * np.pi * x) + 0.05 * rng.standard_normal(n)


@pytest.mark.parametrize("k", [2, 4, 8, 16])
@pytest.mark.parametrize("couples", [1, 3, 64, 65, 64 * 5 + 17])
@pytest.mark.parametrize("step0", [0, 1])
def test_fp64_matches_the_oracle(k, couples, step0):
    n = 2 * k * couples - 1
    u0 = rough(n, k * 1000 + couples)
    got, cfg = run(u0, 2.3, k, 41, step0=step0, gl=0.4, gr=-0.25)
    want = oracle.sdc_step_n(u0, 2.3, k, 41, step0=step0, gl=0.4, gr=-0.25)
    assert rel_l2(got, want) < 1e-12, cfg


@pytest.mark.parametrize("k,depth", [(2, 1), (4, 3), (8, 5), (16, 2), (16, 7), (16, 12), (8, 20)])
def test_depths_give_the_same_bits(k, depth):
    """The depth only moves launch boundaries (each value is computed by the
    same operations in every window that holds it)."""
    n = 2 * k * 700 - 1
    u0 = rough(n, 7)
    ref, _ = run(u0, 1.6, k, 45, depth=1, gl=0.1, gr=0.2)
    got, cfg = run(u0, 1.6, k, 45, depth=depth, gl=0.1, gr=0.2)
    np.testing.assert_array_equal(got, ref, err_msg=str(cfg))
    want = oracle.sdc_step_n(u0, 1.6, k, 45, gl=0.1, gr=0.2)
    assert rel_l2(got, want) < 1e-12


def test_time_dependent_walls_and_split_calls():
    k, n, s = 16, 32 * 300 - 1, 60
    rng = np.random.default_rng(3)
    u0 = rough(n, 3)
    gl = np.sin(np.linspace(0, 3, s + 1))
    gr = rng.uniform(-1, 1, s + 1)
    want = oracle.sdc_step_n(u0, 4.0, k, s, step0=5, gl=gl, gr=gr)
    got, _ = run(u0, 4.0, k, s, step0=5, gl=gl, gr=gr)
    assert rel_l2(got, want) < 1e-12
    # two calls compose bit for bit with one
    plan = ge.Plan(n, 4.0, "fp64", k=k)
    u = ge.pack_state(u0, "fp64")
    d = lambda a: torch.from_numpy(np.asarray(a, dtype=np.float64)).cuda()
    plan.step_n(u, 5, 23, g_left_t=d(gl[:24]), g_right_t=d(gr[:24]))
    plan.step_n(u, 28, s - 23, g_left_t=d(gl[23:]), g_right_t=d(gr[23:]))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(ge.unpack_state(u, n, "fp64"), got)


@pytest.mark.parametrize("k", [4, 16])
def test_fp32_matches_the_oracle(k):
    n = 2 * k * 400 - 1
    u0 = rough(n, 11)
    v0 = ge.unpack_state(ge.pack_state(u0, "fp32"), n, "fp32")
    got, _ = run(u0, 2.0, k, 100, precision="fp32", gl=0.3)
    want = oracle.sdc_step_n(v0, 2.0, k, 100, gl=float(np.float32(0.3)))
    assert rel_l2(got, want) < 1e-5


def test_large_rod_fp64():
    """2^20 points (k = 16: 32768 couples, many tiles), 120 levels."""
    k, n = 16, (1 << 20) - 1
    u0 = rough(n, 5)
    got, _ = run(u0, 2.0, k, 120)
    want = oracle.sdc_step_n(u0, 2.0, k, 120)
    assert rel_l2(got, want) < 1e-12


# The persistent schedule (resident waves, the next window copied into LDS
# during the levels) runs the same operations on the same windows as one
# workgroup per tile: same bits.  Rods of 2^22 - 1 points give thousands of
# tiles, so every wave takes several in turn; 45 levels at depth 20 make
# launches of 20, 20 and 5 levels, the third starting on an odd level.
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("k", [2, 4, 8, 16])
def test_persistent_schedule_gives_the_same_bits(k, precision):
    n = (1 << 22) - 1
    u0 = rough(n, 40 + k)
    ref, c1 = run(u0, 1.9, k, 45, precision=precision, gl=0.2, gr=-0.6, schedule=1)
    got, c2 = run(u0, 1.9, k, 45, precision=precision, gl=0.2, gr=-0.6, schedule=2)
    assert (c1["schedule"], c2["schedule"]) == (1, 2)
    np.testing.assert_array_equal(got, ref)


@pytest.mark.parametrize("k", [2, 16])
@pytest.mark.parametrize("couples", [3 * 42 - 5, 2 * 42 + 1, 42 * 9 + 40, 5000])
@pytest.mark.parametrize("step0", [0, 1])
def test_persistent_schedule_matches_the_oracle(k, couples, step0):
    """Ragged last tiles whose window reaches past the rod (the tail loads),
    down to three tiles, against the oracle."""
    n = 2 * k * couples - 1
    u0 = rough(n, couples + k)
    got, cfg = run(u0, 2.3, k, 33, step0=step0, gl=0.4, gr=-0.25, schedule=2)
    want = oracle.sdc_step_n(u0, 2.3, k, 33, step0=step0, gl=0.4, gr=-0.25)
    assert rel_l2(got, want) < 1e-12, cfg


def test_persistent_schedule_time_dependent_walls():
    k, n, s = 16, 32 * 3000 - 1, 70
    rng = np.random.default_rng(9)
    u0 = rough(n, 9)
    gl = np.cos(np.linspace(0, 2, s + 1))
    gr = rng.uniform(-1, 1, s + 1)
    want = oracle.sdc_step_n(u0, 3.0, k, s, step0=3, gl=gl, gr=gr)
    got, cfg = run(u0, 3.0, k, s, step0=3, gl=gl, gr=gr, schedule=2)
    assert cfg["schedule"] == 2
    assert rel_l2(got, want) < 1e-12
    ref, _ = run(u0, 3.0, k, s, step0=3, gl=gl, gr=gr, schedule=1)
    np.testing.assert_array_equal(got, ref)


# Windows of two, four or eight waves exchange their edge lanes' values
# through LDS once per level; every value is still computed by the same
# operations as in a single-wave window (the halo per side is the same), so
# the bits agree.
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("k", [2, 4, 8, 16])
@pytest.mark.parametrize("waves,schedule", [(2, 1), (4, 1), (8, 1), (2, 2), (4, 2), (8, 2)])
def test_wave_counts_give_the_same_bits(k, precision, waves, schedule):
    n = 2 * k * (64 * 4 * 37 + 19) - 1
    u0 = rough(n, 70 + k)
    ref, c1 = run(u0, 1.9, k, 45, precision=precision, gl=0.2, gr=-0.6, schedule=1, waves=1,
                  depth=20)
    got, c2 = run(u0, 1.9, k, 45, precision=precision, gl=0.2, gr=-0.6, schedule=schedule,
                  waves=waves, depth=20)
    assert (c1["waves"], c2["waves"], c2["schedule"]) == (1, waves, schedule)
    np.testing.assert_array_equal(got, ref)


@pytest.mark.parametrize("k", [2, 16])
@pytest.mark.parametrize("couples", [3, 200, 256, 257, 256 * 3 + 41, 4000])
@pytest.mark.parametrize("step0", [0, 1])
def test_four_wave_windows_match_the_oracle(k, couples, step0):
    """Single four-wave windows (up to 256 couples, advanced in place), a
    window and a ragged second one, and many tiles, per tile and (from three
    tiles on) persistent, against the oracle."""
    n = 2 * k * couples - 1
    u0 = rough(n, couples + 3 * k)
    want = oracle.sdc_step_n(u0, 2.3, k, 33, step0=step0, gl=0.4, gr=-0.25)
    got, cfg = run(u0, 2.3, k, 33, step0=step0, gl=0.4, gr=-0.25, waves=4, schedule=1)
    assert cfg["waves"] == 4
    assert rel_l2(got, want) < 1e-12, cfg
    got2, cfg2 = run(u0, 2.3, k, 33, step0=step0, gl=0.4, gr=-0.25, waves=4, schedule=2)
    np.testing.assert_array_equal(got2, got, err_msg=str(cfg2))


def test_four_wave_windows_time_dependent_walls():
    k, n, s = 16, 32 * 3000 - 1, 70
    rng = np.random.default_rng(19)
    u0 = rough(n, 19)
    gl = np.cos(np.linspace(0, 2, s + 1))
    gr = rng.uniform(-1, 1, s + 1)
    want = oracle.sdc_step_n(u0, 3.0, k, s, step0=3, gl=gl, gr=gr)
    for sched in (1, 2):
        got, cfg = run(u0, 3.0, k, s, step0=3, gl=gl, gr=gr, schedule=sched, waves=4)
        assert (cfg["waves"], cfg["schedule"]) == (4, sched)
        assert rel_l2(got, want) < 1e-12


@pytest.mark.parametrize("k", [4, 16])
def test_wide_windows_fp32_time_dependent_walls(k):
    """FP32 in windows of eight waves (the library's FP32 choice on long
    rods), per tile and persistent, with walls that change every level,
    against the oracle started from the same FP32-rounded values."""
    n, s = 2 * k * 9000 - 1, 61
    rng = np.random.default_rng(23)
    u0 = rough(n, 23)
    v0 = ge.unpack_state(ge.pack_state(u0, "fp32"), n, "fp32")
    gl = np.sin(np.linspace(0, 2.5, s + 1)).astype(np.float32).astype(np.float64)
    gr = rng.uniform(-1, 1, s + 1).astype(np.float32).astype(np.float64)
    want = oracle.sdc_step_n(v0, 2.6, k, s, step0=1, gl=gl, gr=gr)
    outs = []
    for sched in (1, 2):
        got, cfg = run(u0, 2.6, k, s, precision="fp32", step0=1, gl=gl, gr=gr, schedule=sched,
                       waves=8, depth=24)
        assert (cfg["waves"], cfg["schedule"]) == (8, sched)
        assert rel_l2(got, want) < 1e-5, cfg
        outs.append(got)
    np.testing.assert_array_equal(outs[1], outs[0])
