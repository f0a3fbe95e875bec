"""Pins of the sub-domain oracle (oracle/sdc_ref.c): the scheme of Section 2
with sub-domains of k nodes (Eq. (3)/(4) where sub-domains meet, Saul'yev
sweeps Eq. (1)/(2) inside them).  Each check is independent of the C code:
the two-point-group oracle for k = 1, a dense solve of the level's split
form, invariants and the closed-form decay of sin(pi x)."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.filterwarnings("ignore")


def dense_level(w_in, r, k, m, gl_old, gl_new, gr_old, gr_new):
    """One level as a linear solve.  Every interior node j takes scheme A
    ((1+r) v_j - r v_{j-1} = (1-r) w_j + r w_{j+1}) or scheme B ((1+r) v_j -
    r v_{j+1} = (1-r) w_j + r w_{j-1}): on levels of even index A in odd
    sub-domains [2ik, 2ik+k-1] and B in even ones, the reverse on odd
    levels.  Where a B node meets an A node to its right the two unknowns
    couple (the confluence pair); the solve never sees the sweep order."""
    n = w_in.size
    M = n + 1
    w = np.concatenate([[gl_old], w_in, [gr_old]])
    L = np.zeros((n, n))
    rhs = np.zeros(n)
    for j in range(1, M):
        odd_sub = (j // k) % 2 == 0
        a_node = odd_sub if m % 2 == 0 else not odd_sub
        row = j - 1
        L[row, row] = 1 + r
        rhs[row] = (1 - r) * w[j]
        if a_node:
            rhs[row] += r * w[j + 1]
            if j - 1 == 0:
                rhs[row] += r * gl_new
            else:
                L[row, row - 1] = -r
        else:
            rhs[row] += r * w[j - 1]
            if j + 1 == M:
                rhs[row] += r * gr_new
            else:
                L[row, row + 1] = -r
    return np.linalg.solve(L, rhs)


@pytest.mark.parametrize("n", [1, 3, 7, 63, 255])
def test_k1_is_the_two_point_group_sweep(n):
    u = np.random.default_rng(n).standard_normal(n)
    for step0 in (0, 1):
        a = oracle.sdc_step_n(u, 1.7, 1, 13, step0=step0, gl=0.3, gr=-0.2)
        b = oracle.step_n(u, 1.7, 13, step0=step0, gl=0.3, gr=-0.2)
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-14)


@pytest.mark.parametrize("k,e", [(2, 1), (2, 3), (3, 2), (4, 4), (16, 2), (5, 3)])
@pytest.mark.parametrize("r", [0.4, 2.0, 9.0])
def test_each_level_is_the_dense_split_solve(k, e, r):
    n = 2 * e * k - 1
    rng = np.random.default_rng(k * 100 + e)
    u = rng.standard_normal(n)
    nsteps = 6
    gl = rng.standard_normal(nsteps + 1)
    gr = rng.standard_normal(nsteps + 1)
    got = oracle.sdc_step_n(u, r, k, nsteps, step0=3, gl=gl, gr=gr)
    want = u.copy()
    for s in range(nsteps):
        want = dense_level(want, r, k, 3 + s, gl[s], gl[s + 1], gr[s], gr[s + 1])
    np.testing.assert_allclose(got, want, rtol=1e-11, atol=1e-12)


@pytest.mark.parametrize("k", [2, 4, 16])
def test_constants_and_linear_profiles_are_kept(k):
    n = 2 * 5 * k - 1
    x = np.arange(1, n + 1) / (n + 1)
    c = oracle.sdc_step_n(np.full(n, 0.7), 3.0, k, 40, gl=0.7, gr=0.7)
    np.testing.assert_allclose(c, 0.7, rtol=0, atol=1e-14)
    lin = 0.2 + 1.5 * x
    out = oracle.sdc_step_n(lin, 3.0, k, 40, gl=0.2, gr=1.7)
    np.testing.assert_allclose(out, lin, rtol=0, atol=1e-13)


@pytest.mark.parametrize("k", [2, 8, 16])
def test_sine_decays_as_the_closed_form(k):
    """u0 = sin(pi x), zero walls: u(T) -> exp(-pi^2 T) sin(pi x).  At a
    fixed r the error shrinks with h (first order in tau is second order in
    h at fixed r), and sits well below the change of u itself."""
    errs = []
    for e in (4, 8, 16):
        n = 2 * e * k - 1
        h = 1.0 / (n + 1)
        x = np.arange(1, n + 1) * h
        r = 1.0
        T = 0.02
        nsteps = int(round(T / (r * h * h)))
        T = nsteps * r * h * h
        got = oracle.sdc_step_n(np.sin(np.pi * x), r, k, nsteps)
        want = np.exp(-np.pi ** 2 * T) * np.sin(np.pi * x)
        errs.append(np.abs(got - want).max())
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 0.1 * (1 - np.exp(-np.pi ** 2 * 0.02))


@pytest.mark.parametrize("r", [5.0, 50.0])
def test_large_r_stays_bounded(r):
    """Unconditional stability: far above the explicit limit, 2000 levels of
    rough data stay bounded by their start (the decay of every mode)."""
    k = 8
    n = 2 * 6 * k - 1
    u = np.random.default_rng(3).standard_normal(n)
    out = oracle.sdc_step_n(u, r, k, 2000)
    assert np.all(np.isfinite(out))
    assert np.linalg.norm(out) < np.linalg.norm(u)


def test_rejects_a_grid_that_does_not_split():
    with pytest.raises(ValueError):
        oracle.sdc_step_n(np.zeros(10), 1.0, 4, 1)     # n + 1 = 11, not a multiple of 8
