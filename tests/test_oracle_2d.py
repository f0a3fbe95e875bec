"""Pins of the two-dimensional oracle (oracle.step2d_n): the one-dimensional
scheme of Section 2 along every row, then every column, in every level.
The checks do not re-state the composition: a Kronecker-product form of
the level built from the one-dimensional oracle's response to unit vectors,
the exact factorisation of separable data, constants, the closed-form decay
of sin(pi x) sin(pi y), and boundedness far above the explicit limit."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.filterwarnings("ignore")


def level_matrix(n, r, m, gl, gr):
    """The one-dimensional level m as u' = L u + w, read off the 1D oracle's
    answers to the zero vector (w, the walls' part) and to unit vectors."""
    w = oracle.step_n(np.zeros(n), r, 1, step0=m, gl=gl, gr=gr)
    L = np.empty((n, n))
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        L[:, i] = oracle.step_n(e, r, 1, step0=m, gl=gl, gr=gr) - w
    return L, w


@pytest.mark.parametrize("nx,ny", [(1, 1), (1, 6), (5, 1), (7, 4), (6, 9), (10, 10)])
@pytest.mark.parametrize("step0", [0, 1])
def test_level_is_the_kronecker_form(nx, ny, step0):
    """vec(U') = (Ly (x) I)((I (x) Lx) vec(U) + 1 (x) wx) + wy (x) 1, with
    row-major vec: rows take Lx, then columns take Ly."""
    rx, ry = 1.3, 0.7
    walls = (0.4, -0.3, 0.9, 0.2)
    rng = np.random.default_rng(nx * 31 + ny)
    u = rng.standard_normal((ny, nx))
    got = oracle.step2d_n(u, rx, ry, 3, step0=step0, walls=walls)
    v = u.ravel()
    for m in range(step0, step0 + 3):
        Lx, wx = level_matrix(nx, rx, m, walls[0], walls[1])
        Ly, wy = level_matrix(ny, ry, m, walls[2], walls[3])
        v = np.kron(np.eye(ny), Lx) @ v + np.tile(wx, ny)
        v = np.kron(Ly, np.eye(nx)) @ v + np.repeat(wy, nx)
    np.testing.assert_allclose(got.ravel(), v, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("nx,ny", [(9, 14), (32, 17)])
def test_separable_data_factorises(nx, ny):
    """Zero walls, u0 = g(y) f(x): every row is a multiple of f and every
    column a multiple of the x-advanced column, so the result is the outer
    product of the two one-dimensional runs."""
    rng = np.random.default_rng(5)
    f, g = rng.standard_normal(nx), rng.standard_normal(ny)
    got = oracle.step2d_n(np.outer(g, f), 2.5, 0.8, 11, step0=1)
    want = np.outer(oracle.step_n(g, 0.8, 11, step0=1), oracle.step_n(f, 2.5, 11, step0=1))
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-13)


def test_constants_are_kept():
    out = oracle.step2d_n(np.full((8, 13), 0.35), 4.0, 1.5, 20, walls=(0.35,) * 4)
    np.testing.assert_allclose(out, 0.35, rtol=0, atol=1e-14)


def test_sine_decays_as_the_closed_form():
    """u0 = sin(pi x) sin(pi y), zero walls: u(T) -> exp(-2 pi^2 T) u0.  At
    fixed r the error falls with h and stays well below the change of u."""
    errs = []
    T = 0.02
    for n in (15, 31, 63):
        h = 1.0 / (n + 1)
        x = np.arange(1, n + 1) * h
        r = 1.0
        nsteps = int(round(T / (r * h * h)))
        t = nsteps * r * h * h
        u0 = np.outer(np.sin(np.pi * x), np.sin(np.pi * x))
        got = oracle.step2d_n(u0, r, r, nsteps)
        errs.append(np.abs(got - np.exp(-2 * np.pi ** 2 * t) * u0).max())
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 0.05 * (1 - np.exp(-2 * np.pi ** 2 * T))


def test_large_r_stays_bounded():
    u = np.random.default_rng(2).standard_normal((12, 17))
    out = oracle.step2d_n(u, 40.0, 25.0, 400)
    assert np.all(np.isfinite(out))
    assert np.linalg.norm(out) < np.linalg.norm(u)


def test_rejects_bad_shapes():
    with pytest.raises(ValueError):
        oracle.step2d_n(np.zeros(5), 1.0, 1.0, 1)
    with pytest.raises(ValueError):
        oracle.step2d_n(np.zeros((0, 3)), 1.0, 1.0, 1)
