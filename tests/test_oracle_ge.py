"""Pins of the CPU oracle for the GE sweep against what the paper and the
mathematics fix, independently of the oracle's own formulas.

Section 2 defines the scheme: every node takes one of Saul'yev's formulas,
scheme A (Eq. 1, implicit in the left neighbour) or scheme B (Eq. 2,
implicit in the right neighbour), chosen so that within a coupled pair the
left node uses B and the right node uses A; the pair is solved in closed
form by Eq. (3)/(4).  The dense pins below assemble the per-node Saul'yev
equations directly and solve them with a library routine (or with exact
rationals), so the closed form, the denominator, the pairing and the wall
treatment are each checked against the definition, not against a retyped
copy of Eq. (3)/(4).
"""
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def partner(i, n, p):
    """1-based partner of node i at a level of parity p (two-point groups:
    even levels couple (1,2),(3,4),..., odd levels couple (2,3),(4,5),...)."""
    return i + 1 if (i + p) % 2 == 1 else i - 1


def saulyev_system(n, r, tau, p, u, gl_old, gl_new, gr_old, gr_new, f):
    """Assemble M u' = rhs from the node-wise Saul'yev equations.

    Node i with partner i+1 (B, Eq. 2): (1+r)u_i' - r u_{i+1}' = (1-r)u_i + r u_{i-1}
    Node i with partner i-1 (A, Eq. 1): (1+r)u_i' - r u_{i-1}' = (1-r)u_i + r u_{i+1}
    plus tau*f_i on the right; wall values enter at the new level on the
    implicit side and at the old level on the explicit side.
    """
    M = np.zeros((n, n))
    rhs = np.zeros(n)
    uu = np.concatenate([[gl_old], u, [gr_old]])  # uu[i] = u_i, i = 0..n+1
    for i in range(1, n + 1):
        q = partner(i, n, p)
        M[i - 1, i - 1] = 1 + r
        rhs[i - 1] = (1 - r) * uu[i] + tau * f[i - 1]
        expl = i - 1 if q == i + 1 else i + 1  # explicit neighbour
        rhs[i - 1] += r * uu[expl]
        if 1 <= q <= n:
            M[i - 1, q - 1] = -r
        elif q == 0:
            rhs[i - 1] += r * gl_new
        else:
            rhs[i - 1] += r * gr_new
    return M, rhs


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 8])
@pytest.mark.parametrize("r", [0.3, 1.0, 2.5])
@pytest.mark.parametrize("step0", [0, 1])
def test_single_level_equals_dense_saulyev_solve(n, r, step0):
    rng = np.random.default_rng(100 + n)
    u = rng.standard_normal(n)
    gl = np.array([0.3, -0.7])          # g_L(t_m), g_L(t_{m+1})
    gr = np.array([1.1, 0.4])
    b = rng.standard_normal(n)
    a = np.array([0.8])
    h = 1.0 / (n + 1)
    tau = r * h * h
    got = oracle.step_n(u, r, 1, step0=step0, gl=gl, gr=gr, src_b=b, src_a=a)
    M, rhs = saulyev_system(n, r, tau, step0 % 2, u, gl[0], gl[1], gr[0],
                            gr[1], a[0] * b)
    want = np.linalg.solve(M, rhs)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-13 * max(1, np.abs(want).max()))


def test_several_levels_equal_exact_rational_solve():
    """Brute force in exact arithmetic: Gauss-Jordan on Fractions."""
    n, r_f, nsteps = 7, Fraction(5, 2), 4
    u = [Fraction(k * k - 3 * k + 1, 7) for k in range(1, n + 1)]
    gl = [Fraction(1, 3), Fraction(-1, 2), Fraction(2, 5), Fraction(0), Fraction(1, 7)]
    gr = [Fraction(-2, 3), Fraction(1, 4), Fraction(3, 5), Fraction(1, 9), Fraction(0)]
    cur = list(u)
    for m in range(nsteps):
        p = m % 2
        A = [[Fraction(0)] * n + [Fraction(0)] for _ in range(n)]
        uu = [gl[m]] + cur + [gr[m]]
        for i in range(1, n + 1):
            q = partner(i, n, p)
            row = A[i - 1]
            row[i - 1] = 1 + r_f
            expl = i - 1 if q == i + 1 else i + 1
            row[n] = (1 - r_f) * uu[i] + r_f * uu[expl]
            if 1 <= q <= n:
                row[q - 1] = -r_f
            elif q == 0:
                row[n] += r_f * gl[m + 1]
            else:
                row[n] += r_f * gr[m + 1]
        for c in range(n):  # exact Gauss-Jordan
            piv = next(k for k in range(c, n) if A[k][c] != 0)
            A[c], A[piv] = A[piv], A[c]
            inv = 1 / A[c][c]
            A[c] = [x * inv for x in A[c]]
            for k in range(n):
                if k != c and A[k][c] != 0:
                    fac = A[k][c]
                    A[k] = [x - fac * y for x, y in zip(A[k], A[c])]
        cur = [A[i][n] for i in range(n)]
    got = oracle.step_n(np.array([float(x) for x in u]), float(r_f), nsteps,
                        gl=np.array([float(x) for x in gl]),
                        gr=np.array([float(x) for x in gr]))
    want = np.array([float(x) for x in cur])
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-14)


def _read_numerators():
    rows = {}
    with open(os.path.join(GOLDEN, "eq3_eq4_numerators.txt")) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            eq, node, c0, c1, c2 = line.split()
            rows[(eq, node)] = (float(c0), float(c1), float(c2))
    return rows


@pytest.mark.parametrize("r", [0.25, 1.0, 3.0])
def test_printed_numerators_of_eq3_eq4(r):
    """The response of a pair to a unit value at u_{j-1}..u_{j+2} is the
    printed numerator over (1+2r)."""
    rows = _read_numerators()
    poly = lambda c: c[0] + c[1] * r + c[2] * r * r
    den = poly(rows[("den", "den")])
    n, j = 8, 5          # pair (5,6) is coupled on even levels
    for off, node in enumerate(["jm1", "j", "jp1", "jp2"]):
        e = np.zeros(n)
        e[j - 2 + off] = 1.0         # u_{j-1+off}, 0-based index j-2+off
        out = oracle.step_n(e, r, 1, step0=0)
        assert out[j - 1] == pytest.approx(poly(rows[("eq3", node)]) / den, abs=1e-15)
        assert out[j] == pytest.approx(poly(rows[("eq4", node)]) / den, abs=1e-15)


@pytest.mark.parametrize("n", [1, 2, 9, 64])
@pytest.mark.parametrize("r", [0.4, 2.0, 50.0])
def test_constants_preserved(n, r):
    c = 0.7
    out = oracle.step_n(np.full(n, c), r, 37, gl=c, gr=c)
    # the printed numerators carry terms of size r^2 that cancel
    np.testing.assert_allclose(out, c, rtol=0, atol=1e-14 * (1 + r) ** 2)


@pytest.mark.parametrize("n", [3, 10, 33])
@pytest.mark.parametrize("r", [0.5, 4.0])
def test_linear_profile_is_fixed_point(n, r):
    gl, gr = -0.4, 1.3
    h, x = oracle.grid(n)
    lin = gl + (gr - gl) * x
    out = oracle.step_n(lin, r, 25, gl=gl, gr=gr)
    np.testing.assert_allclose(out, lin, rtol=0, atol=1e-13)


@pytest.mark.parametrize("n", [2, 8, 30, 31])
@pytest.mark.parametrize("step0", [0, 1])
def test_mirror_symmetry(n, step0):
    """Mirroring x -> 1-x maps the pairing of parity p to itself for even n
    and to the other parity for odd n; scheme A at the left wall mirrors to
    scheme B at the right wall."""
    rng = np.random.default_rng(n)
    u = rng.standard_normal(n)
    gl = rng.standard_normal(12)
    gr = rng.standard_normal(12)
    a = oracle.step_n(u, 1.7, 11, step0=step0, gl=gl, gr=gr)
    mstep0 = step0 if n % 2 == 0 else step0 + 1
    b = oracle.step_n(u[::-1], 1.7, 11, step0=mstep0, gl=gr, gr=gl)
    np.testing.assert_allclose(a, b[::-1], rtol=0, atol=1e-14)


def test_superposition():
    rng = np.random.default_rng(5)
    n = 21
    u, v = rng.standard_normal(n), rng.standard_normal(n)
    f = lambda w: oracle.step_n(w, 2.2, 13)
    np.testing.assert_allclose(f(2.0 * u - 3.0 * v), 2.0 * f(u) - 3.0 * f(v),
                               rtol=0, atol=1e-13)


def _G(n, p):
    G = np.zeros((n, n))
    for i in range(1, n + 1):
        q = partner(i, n, p)
        G[i - 1, i - 1] = 1
        if 1 <= q <= n:
            G[i - 1, q - 1] = -1
    return G


def test_split_operators_sum_to_the_laplacian():
    for n in (1, 2, 5, 8):
        A = _G(n, 0) + _G(n, 1)
        T = 2 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
        np.testing.assert_array_equal(A, T)


@pytest.mark.parametrize("r", [0.6, 2.0, 4.0, 50.0])
def test_unconditional_stability_energy(r):
    """Two levels are a Peaceman-Rachford step for A = G_0 + G_1 with both
    G_p symmetric positive semi-definite, so with zero walls
    E = ||(I + r G_1) u^{2m}||_2 never increases, for any r > 0."""
    rng = np.random.default_rng(7)
    n = 40
    u = rng.standard_normal(n)
    W = np.eye(n) + r * _G(n, 1)
    E = [np.linalg.norm(W @ u)]
    for m in range(60):
        u = oracle.step_n(u, r, 2, step0=2 * m)
        E.append(np.linalg.norm(W @ u))
    E = np.array(E)
    assert np.all(np.diff(E) <= 1e-13 * E[:-1])
    assert E[-1] < E[0]


@pytest.mark.parametrize("r", [0.5, 0.75, 1.0])
def test_maximum_principle_for_r_at_most_one(r):
    """For r <= 1 every coefficient of Eq. (1)-(4) is >= 0 and they sum to
    one, so the max norm cannot grow (zero walls)."""
    rng = np.random.default_rng(11)
    u = rng.uniform(-1, 1, 50)
    for m in range(200):
        v = oracle.step_n(u, r, 1, step0=m)
        assert np.abs(v).max() <= np.abs(u).max() * (1 + 1e-15)
        u = v


def test_closed_form_sine_decay():
    """u0 = sin(pi x), zero walls: the exact solution is exp(-pi^2 t) sin(pi x);
    N = 1024 interior points, r = 1, 1000 levels."""
    n, r, s = 1024, 1.0, 1000
    h, x = oracle.grid(n)
    out = oracle.step_n(np.sin(np.pi * x), r, s)
    t = s * r * h * h
    exact = np.exp(-np.pi ** 2 * t) * np.sin(np.pi * x)
    err = np.linalg.norm(out - exact) / np.linalg.norm(exact)
    assert err < 2e-7
    assert err > 1e-9   # the scheme's own truncation error is visible


def _modes(x, t):
    a = {1: 1.0, 2: -0.5, 3: 0.3, 5: 0.2}
    return sum(c * np.exp(-(k * np.pi) ** 2 * t) * np.sin(k * np.pi * x)
               for k, c in a.items())


@pytest.mark.parametrize("r", [1.0, 4.0])
def test_second_order_convergence(r):
    errs = []
    for n, s in ((255, 64), (511, 256), (1023, 1024)):
        h, x = oracle.grid(n)
        t = s * r * h * h   # the same final time for all three grids
        out = oracle.step_n(_modes(x, 0.0), r, s)
        errs.append(np.abs(out - _modes(x, t)).max())
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all((orders > 1.8) & (orders < 2.4)), orders


def test_error_falls_with_mesh_ratio():
    n = 511
    h, x = oracle.grid(n)
    errs = []
    for r in (4.0, 2.0, 1.0, 0.5):
        s = int(round(512 / r))
        out = oracle.step_n(_modes(x, 0.0), r, s)
        errs.append(np.abs(out - _modes(x, s * r * h * h)).max())
    assert all(a > b for a, b in zip(errs, errs[1:])), errs


def test_manufactured_solution_with_source_and_moving_walls():
    """u = exp(-t) cos(pi x) solves u_t = u_xx + f with
    f = (pi^2 - 1) exp(-t) cos(pi x), g_L = exp(-t), g_R = -exp(-t).
    The source enters at t_m + tau/2 (a reading, pinned only by this
    convergence check)."""
    r = 2.0
    errs = []
    for n, s in ((63, 16), (127, 64), (255, 256)):
        h, x = oracle.grid(n)
        tau = r * h * h
        t = np.arange(s + 1) * tau
        out = oracle.step_n(np.cos(np.pi * x), r, s, gl=np.exp(-t), gr=-np.exp(-t),
                            src_b=(np.pi ** 2 - 1) * np.cos(np.pi * x),
                            src_a=np.exp(-(t[:-1] + 0.5 * tau)))
        errs.append(np.abs(out - np.exp(-t[-1]) * np.cos(np.pi * x)).max())
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(orders > 1.7), (errs, orders)
    assert errs[-1] < 1e-4


def test_composition_is_bitwise():
    rng = np.random.default_rng(3)
    u = rng.standard_normal(101)
    gl = rng.standard_normal(31)
    whole = oracle.step_n(u, 3.0, 30, gl=gl)
    a = oracle.step_n(u, 3.0, 13, gl=gl[:14])
    b = oracle.step_n(a, 3.0, 17, step0=13, gl=gl[13:])
    np.testing.assert_array_equal(whole, b)


def test_threads_are_bitwise_equal_to_serial():
    rng = np.random.default_rng(4)
    u = rng.standard_normal(1001)
    one = oracle.step_n(u, 2.0, 40, step0=3, gl=0.2, gr=-0.1)
    for t in (2, 3, 8):
        np.testing.assert_array_equal(
            oracle.step_n(u, 2.0, 40, step0=3, gl=0.2, gr=-0.1, nthreads=t), one)


def test_extended_precision_agrees():
    rng = np.random.default_rng(8)
    u = rng.standard_normal(300)
    a = oracle.step_n(u, 1.5, 200)
    b = oracle.step_n(u, 1.5, 200, extended=True)
    assert np.linalg.norm(a - b) / np.linalg.norm(b) < 1e-14


def test_window_evaluation_is_exact():
    rng = np.random.default_rng(9)
    n, s = 2000, 150
    u = rng.standard_normal(n)
    b = rng.standard_normal(n)
    a = rng.standard_normal(s)
    full = oracle.step_n(u, 2.0, s, step0=1, gl=0.5, gr=-0.5, src_b=b, src_a=a)
    for lo, hi in ((0, 40), (700, 777), (1960, 2000)):
        w = oracle.window_step_n(u, lo, hi, 2.0, s, step0=1, gl=0.5, gr=-0.5,
                                 src_b=b, src_a=a)
        np.testing.assert_array_equal(w, full[lo:hi])


def test_wall_flux_matches_the_exact_heat_flux():
    """sum_m tau (u_1^{m+1} - g_L)/h approximates int_0^T u_x(0, t) dt,
    which is (1 - exp(-pi^2 T))/pi for u0 = sin(pi x)."""
    n, r, s = 1023, 1.0, 4096
    h, x = oracle.grid(n)
    flux = np.zeros(2)
    oracle.step_n(np.sin(np.pi * x), r, s, flux=flux)
    t = s * r * h * h
    want = (1 - np.exp(-np.pi ** 2 * t)) / np.pi
    assert flux[0] == pytest.approx(want, rel=2e-3)
    assert flux[1] == pytest.approx(want, rel=2e-3)


def test_rejects_invalid_arguments():
    with pytest.raises(ValueError):
        oracle.step_n(np.zeros(0), 1.0, 1)
    with pytest.raises(ValueError):
        oracle.step_n(np.zeros(4), 1.0, -1)
    with pytest.raises(ValueError):
        oracle.step_n(np.zeros(4), 1.0, 2, gl=np.zeros(2))
