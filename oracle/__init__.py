"""CPU oracle for the group explicit (GE) sweep and for the surrogate network.

TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library imports this package;
only tests/, the smoke check and the benchmark's CPU-baseline leg use it.

* ``step_n``: the GE scheme of Section 2 (Eq. (1)-(4), two-point groups,
  alternating grouping) in plain C, FP64 or x87 extended precision
  (``ge_ref.c``).
* ``sdc_step_n``: the same scheme with sub-domains of k nodes (Section 2's
  complementary scheme: Eq. (3)/(4) where sub-domains meet, Saul'yev
  sweeps Eq. (1)/(2) inside them), FP64 (``sdc_ref.c``).
* ``step2d_n``: the two-dimensional extension on the unit square, the
  scheme applied along every grid line, x then y, in every level (a
  composition of ``step_n`` calls).
* ``conv_ref``: the FP64 forward/backward of the 1D convolutional propagator.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libge_ref.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    src = [os.path.join(_HERE, f) for f in ("ge_ref.c", "ge_ref_core.inc", "sdc_ref.c")]
    if not os.path.exists(_LIB_PATH) or any(
            os.path.getmtime(s) > os.path.getmtime(_LIB_PATH) for s in src):
        from . import build as _build
        _build.build()
    lib = ctypes.CDLL(_LIB_PATH)
    for name in ("ge_ref_step_n", "ge_ref_step_n_ext"):
        f = getattr(lib, name)
        f.restype = ctypes.c_int
        f.argtypes = [ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                      ctypes.c_double, ctypes.c_int64, ctypes.c_int64, _dp,
                      _dp, _dp, ctypes.c_double, ctypes.c_double, _dp, _dp,
                      _dp, ctypes.c_int]
    lib.sdc_ref_step_n.restype = ctypes.c_int
    lib.sdc_ref_step_n.argtypes = [ctypes.c_int64, ctypes.c_int, ctypes.c_double,
                                   ctypes.c_int64, ctypes.c_int64, _dp, _dp, _dp,
                                   ctypes.c_double, ctypes.c_double]
    _lib = lib
    return lib


def _ptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(_dp)


def _f64(a, n=None, name="array"):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    if n is not None and a.shape != (n,):
        raise ValueError(f"{name} must have shape ({n},), got {a.shape}")
    return a


def grid(n):
    """h = 1/(n+1) and the interior abscissae x_i = i h, i = 1..n."""
    h = 1.0 / (n + 1)
    return h, np.arange(1, n + 1, dtype=np.float64) * h


def step_n(u0, r, nsteps, step0=0, gl=0.0, gr=0.0, src_b=None, src_a=None,
           tau=None, h=None, flux=None, nthreads=1, extended=False, inplace=False):
    """Advance interior values ``u0`` (u_1..u_n at level ``step0``) by
    ``nsteps`` levels and return the new array (``u0`` is not modified,
    unless ``inplace``: then ``u0``, a contiguous float64 array, is advanced
    in place and returned).

    gl, gr: wall values, either scalars (constant) or arrays of length
    nsteps+1 holding g(t_m) for m = step0..step0+nsteps.
    src_b, src_a: the source f(x, t) = a(t) b(x) as b(x_i) (length n) and
    a(t_m + tau/2) for m = step0..step0+nsteps-1 (length nsteps).
    tau, h: default to the full rod's h = 1/(n+1), tau = r h^2; a sub-window
    of a longer rod passes the rod's own values.
    flux: None, or a length-2 float64 array updated in place with the wall
    first-difference sums (see ge_ref_core.inc).
    """
    lib = _load()
    if inplace:
        if not (isinstance(u0, np.ndarray) and u0.dtype == np.float64 and u0.ndim == 1
                and u0.flags.c_contiguous and u0.flags.writeable):
            raise ValueError("inplace needs a writeable contiguous 1-D float64 array")
        u = u0
    else:
        u = np.array(u0, dtype=np.float64, copy=True).ravel()
    n = u.size
    if h is None:
        h = 1.0 / (n + 1)
    if tau is None:
        tau = r * h * h
    gla = gra = None
    gl0 = gr0 = 0.0
    if np.ndim(gl) == 0:
        gl0 = float(gl)
    else:
        gla = _f64(gl, nsteps + 1, "gl")
    if np.ndim(gr) == 0:
        gr0 = float(gr)
    else:
        gra = _f64(gr, nsteps + 1, "gr")
    sb = _f64(src_b, n, "src_b")
    sa = _f64(src_a, nsteps, "src_a")
    if (sb is None) != (sa is None):
        raise ValueError("src_b and src_a go together")
    if flux is not None:
        if not (isinstance(flux, np.ndarray) and flux.dtype == np.float64
                and flux.shape == (2,)):
            raise ValueError("flux must be a float64 array of shape (2,)")
    fn = lib.ge_ref_step_n_ext if extended else lib.ge_ref_step_n
    rc = fn(n, float(r), float(tau), float(h), int(step0), int(nsteps),
            _ptr(u), _ptr(gla), _ptr(gra), gl0, gr0, _ptr(sb), _ptr(sa),
            _ptr(flux), int(nthreads))
    if rc != 0:
        raise ValueError("oracle rejected its arguments")
    return u


def window_step_n(u_full, lo, hi, r, nsteps, step0=0, gl=0.0, gr=0.0,
                  src_b=None, src_a=None, extended=False):
    """Values u_{lo+1}..u_{hi} (0-based slice [lo, hi)) of a long rod after
    ``nsteps`` levels, computed by the oracle on a sub-window only.

    A value at level m+1 depends on level-m values at most two places away,
    and the pairing of a window that starts at an even 0-based index is the
    rod's own; so running the window [lo - nsteps - 2, hi + nsteps + 2]
    (clipped at the rod's walls, which then keep their true wall values)
    leaves [lo, hi) exact.  A cut that is not a wall gets an arbitrary
    value, whose influence spreads one point per level and stays outside
    [lo, hi).
    """
    u_full = np.asarray(u_full, dtype=np.float64)
    n = u_full.size
    h = 1.0 / (n + 1)
    tau = r * h * h
    a = max(0, lo - nsteps - 2)
    a -= a % 2
    b = min(n, hi + nsteps + 2)
    if b - a < 1:
        return np.zeros(0)
    # cut edges that are not walls get a frozen value of 0
    gl_w = gl if a == 0 else 0.0
    gr_w = gr if b == n else 0.0
    sb = None if src_b is None else np.asarray(src_b, dtype=np.float64)[a:b]
    out = step_n(u_full[a:b], r, nsteps, step0=step0, gl=gl_w, gr=gr_w,
                 src_b=sb, src_a=src_a, tau=tau, h=h, extended=extended)
    return out[lo - a:hi - a]


def sdc_step_n(u0, r, k, nsteps, step0=0, gl=0.0, gr=0.0):
    """The sub-domain scheme with sub-domains of ``k`` nodes (``sdc_ref.c``):
    advance interior values ``u0`` (u_1..u_n, n + 1 a multiple of 2k) by
    ``nsteps`` levels from global level ``step0``; walls as in ``step_n``
    (no source).  Returns the new array."""
    lib = _load()
    u = np.array(u0, dtype=np.float64, copy=True).ravel()
    n = u.size
    gla = gra = None
    gl0 = gr0 = 0.0
    if np.ndim(gl) == 0:
        gl0 = float(gl)
    else:
        gla = _f64(gl, nsteps + 1, "gl")
    if np.ndim(gr) == 0:
        gr0 = float(gr)
    else:
        gra = _f64(gr, nsteps + 1, "gr")
    rc = lib.sdc_ref_step_n(n, int(k), float(r), int(step0), int(nsteps), _ptr(u),
                            _ptr(gla), _ptr(gra), gl0, gr0)
    if rc != 0:
        raise ValueError("oracle rejected its arguments (n + 1 must be a multiple of 2k)")
    return u


def step2d_n(u0, rx, ry, nsteps, step0=0, walls=(0.0, 0.0, 0.0, 0.0)):
    """u_t = u_xx + u_yy on the unit square (Section 2's scheme extended to
    two dimensions, which the paper claims without formulas).  Reading: in
    every level m the one-dimensional level m is applied along every row
    (r = rx = tau/hx^2, walls west/east) and then along every column
    (r = ry = tau/hy^2, walls south/north) -- first-order operator
    splitting, each line paired by the level's global index as in
    ``step_n``.

    u0: array (ny, nx); row j holds y_{j+1}, column i holds x_{i+1}, with
    hx = 1/(nx+1), hy = 1/(ny+1).  walls: constant (west, east, south,
    north) values.  Returns the new array (u0 is not modified)."""
    u = np.array(u0, dtype=np.float64, copy=True)
    if u.ndim != 2 or u.shape[0] < 1 or u.shape[1] < 1:
        raise ValueError("u0 must be a non-empty 2-D array (ny, nx)")
    ny, nx = u.shape
    gw, ge_, gs, gn = (float(w) for w in walls)
    for s in range(nsteps):
        m = step0 + s
        for j in range(ny):
            u[j, :] = step_n(u[j, :], rx, 1, step0=m, gl=gw, gr=ge_)
        for i in range(nx):
            u[:, i] = step_n(u[:, i], ry, 1, step0=m, gl=gs, gr=gn)
    return u
