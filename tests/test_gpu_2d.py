"""GPU parity of the two-dimensional extension (ge_2d_step_n through the C
ABI) against the CPU oracle oracle.step2d_n, element by element on the same
seeded grids.  FP64 within 1e-12 relative L2; FP32 within 1e-5 of the
oracle started from the FP32-rounded grid.  Shapes cover single points and
lines, exact 64 x 16 tiles, ragged tiles in both directions and a grid of
several thousand tiles."""
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


def grid(nx, ny, seed):
    rng = np.random.default_rng(seed)
    x = np.arange(1, nx + 1) / (nx + 1)
    y = np.arange(1, ny + 1) / (ny + 1)
    return (np.outer(np.sin(np.pi * y), np.sin(2 * np.pi * x))
            + 0.2 * rng.standard_normal((ny, nx)))


def run(u0, rx, ry, nsteps, step0=0, walls=(0.0, 0.0, 0.0, 0.0), precision="fp64"):
    ny, nx = u0.shape
    dt = torch.float64 if precision == "fp64" else torch.float32
    u = torch.from_numpy(np.ascontiguousarray(u0)).to(dt).cuda()
    ge.step2d_n(u, nx, ny, rx, ry, step0, nsteps, precision=precision, walls=walls)
    torch.cuda.synchronize()
    return u.double().cpu().numpy()


WALLS = (0.3, -0.5, 0.8, 0.1)


@pytest.mark.parametrize("nx,ny", [(1, 1), (1, 9), (9, 1), (2, 3), (64, 16), (65, 17),
                                   (130, 37), (37, 130), (200, 300)])
@pytest.mark.parametrize("step0", [0, 1])
@pytest.mark.parametrize("nsteps", [1, 2, 7])
def test_fp64_matches_the_oracle(nx, ny, step0, nsteps):
    u0 = grid(nx, ny, nx * 7 + ny)
    got = run(u0, 1.7, 0.6, nsteps, step0=step0, walls=WALLS)
    want = oracle.step2d_n(u0, 1.7, 0.6, nsteps, step0=step0, walls=WALLS)
    assert rel_l2(got, want) < 1e-12


@pytest.mark.parametrize("nx,ny", [(33, 70), (256, 64)])
def test_fp32_matches_the_oracle(nx, ny):
    u0 = grid(nx, ny, 3)
    v0 = u0.astype(np.float32).astype(np.float64)
    w = tuple(float(np.float32(g)) for g in WALLS)
    got = run(u0, 3.0, 2.2, 9, walls=WALLS, precision="fp32")
    want = oracle.step2d_n(v0, 3.0, 2.2, 9, walls=w)
    assert rel_l2(got, want) < 1e-5


def test_large_grid_fp64():
    """2048 x 1536 points (3072 tiles), 6 levels."""
    nx, ny = 2048, 1536
    u0 = grid(nx, ny, 11)
    got = run(u0, 2.0, 1.125, 6, step0=3, walls=WALLS)
    want = oracle.step2d_n(u0, 2.0, 1.125, 6, step0=3, walls=WALLS)
    assert rel_l2(got, want) < 1e-12


def test_split_calls_compose_bit_for_bit():
    nx, ny = 150, 90
    u0 = grid(nx, ny, 4)
    one = run(u0, 0.9, 1.4, 9, step0=2, walls=WALLS)
    u = torch.from_numpy(u0.copy()).cuda()
    ge.step2d_n(u, nx, ny, 0.9, 1.4, 2, 5, walls=WALLS)
    ge.step2d_n(u, nx, ny, 0.9, 1.4, 7, 4, walls=WALLS)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(u.cpu().numpy(), one)


def test_zero_levels_leave_the_grid():
    u0 = grid(20, 30, 1)
    np.testing.assert_array_equal(run(u0, 1.0, 1.0, 0), u0)


def test_unit_square_sine_decays():
    """sin(pi x) sin(pi y), r = 1 in both directions on the unit square:
    the GPU result tracks exp(-2 pi^2 t) as the oracle does."""
    n = 127
    h = 1.0 / (n + 1)
    x = np.arange(1, n + 1) * h
    u0 = np.outer(np.sin(np.pi * x), np.sin(np.pi * x))
    steps = 200
    t = steps * h * h
    got = run(u0, 1.0, 1.0, steps)
    exact = np.exp(-2 * np.pi ** 2 * t) * u0
    assert np.abs(got - exact).max() < 0.05 * (1 - np.exp(-2 * np.pi ** 2 * t))


@pytest.mark.parametrize("nx,ny", [(50001, 1), (1, 3001), (3, 2500)])
def test_long_thin_grids(nx, ny):
    """One long row (hundreds of tiles side by side, every column a single
    point between the south and north walls), one long column, and a
    three-column strip."""
    u0 = grid(nx, ny, nx + ny)
    got = run(u0, 2.2, 0.9, 3, step0=1, walls=WALLS)
    want = oracle.step2d_n(u0, 2.2, 0.9, 3, step0=1, walls=WALLS)
    assert rel_l2(got, want) < 1e-12


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("nx,ny", [(1, 1), (5, 3), (129, 17), (300, 70), (1000, 1)])
@pytest.mark.parametrize("nsteps", [1, 5, 8])
def test_depths_give_the_same_bits(precision, nx, ny, nsteps):
    """Fusing 2 or 4 levels per launch recomputes the halo with the same
    operations: every depth, with a remainder of single levels, gives the
    bits of one level per launch."""
    u0 = grid(nx, ny, 17)
    dt = torch.float64 if precision == "fp64" else torch.float32
    outs = []
    for depth in (1, 2, 4):
        u = torch.from_numpy(u0.copy()).to(dt).cuda()
        ge.step2d_n(u, nx, ny, 1.4, 2.6, 3, nsteps, precision=precision, walls=WALLS, depth=depth)
        torch.cuda.synchronize()
        outs.append(u.cpu().numpy())
    np.testing.assert_array_equal(outs[1], outs[0])
    np.testing.assert_array_equal(outs[2], outs[0])
    if precision == "fp64":
        want = oracle.step2d_n(u0, 1.4, 2.6, nsteps, step0=3, walls=WALLS)
        assert rel_l2(outs[0].astype(np.float64), want) < 1e-12


def test_fp32_interior_tiles_four_levels_per_launch():
    """A grid large enough for tiles that touch no wall (the path without
    per-point tests), FP32 at four levels per launch, against the oracle."""
    nx, ny = 700, 300
    u0 = grid(nx, ny, 29)
    v0 = u0.astype(np.float32).astype(np.float64)
    w = tuple(float(np.float32(g)) for g in WALLS)
    got = run(u0, 1.3, 2.1, 12, step0=1, walls=WALLS, precision="fp32")
    want = oracle.step2d_n(v0, 1.3, 2.1, 12, step0=1, walls=w)
    assert rel_l2(got, want) < 1e-5


def test_large_grid_every_depth():
    """A grid of thousands of tiles per launch (most of them touching no
    wall): every depth gives the same bits, and they match the oracle."""
    nx, ny = 4096, 2048
    u0 = grid(nx, ny, 31)
    want = oracle.step2d_n(u0, 1.9, 0.7, 9, step0=1, walls=WALLS)
    outs = []
    for depth in (1, 2, 4):
        u = torch.from_numpy(u0.copy()).cuda()
        ge.step2d_n(u, nx, ny, 1.9, 0.7, 1, 9, walls=WALLS, depth=depth)
        torch.cuda.synchronize()
        outs.append(u.cpu().numpy())
    np.testing.assert_array_equal(outs[1], outs[0])
    np.testing.assert_array_equal(outs[2], outs[0])
    assert rel_l2(outs[0], want) < 1e-12
