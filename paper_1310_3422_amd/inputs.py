"""Seeded synthetic inputs for the GE sweep and its surrogate.

Shared by the tests, the benchmark and the oracle checks; it holds none of
the method's arithmetic, only the problem data of Section 2 (initial values,
wall values, source) drawn from NumPy's PCG64 (``default_rng``) in the order
stated in each function.  Everything is FP64 on the host; FP32 runs round
these same bytes.

Workloads (interior points N, h = 1/(N+1), time levels t_m = m*tau with
tau = r*h^2):

* ``sine_rod``: u0(x) = sum_{k=1..16} a_k sin(k pi x), a_k = z_k / k^2,
  z ~ N(0,1)^16, zero walls.
* ``rod_batch``: independent rods with N log-uniform in [nmin, nmax],
  r uniform in [rmin, rmax], constant walls uniform in [-1, 1], sine-mode
  initial values as above.
* ``moving_wall_rod``: u0 = 0, g_L(t) = sin(2 pi t), g_R = 0 and the source
  f(x, t) = exp(-t) x (1 - x), given as a(t) = exp(-t) sampled at
  t_m + tau/2 and b(x_i) = x_i (1 - x_i).
"""
from dataclasses import dataclass

import numpy as np

NMODES = 16


def abscissae(n):
    """x_i = i/(n+1), i = 1..n."""
    return np.arange(1, n + 1, dtype=np.float64) / (n + 1)


def sine_modes(n, z):
    """sum_k (z_k / k^2) sin(k pi x_i) over k = 1..len(z)."""
    x = abscissae(n)
    u = np.zeros(n)
    for k, zk in enumerate(np.asarray(z, dtype=np.float64), start=1):
        u += (zk / (k * k)) * np.sin(k * np.pi * x)
    return u


def sine_rod(n, seed):
    rng = np.random.default_rng(seed)
    z = rng.standard_normal(NMODES)
    return sine_modes(n, z)


def sine_pulse(n):
    """u0 = sin(pi x): its exact evolution is exp(-pi^2 t) sin(pi x)."""
    return np.sin(np.pi * abscissae(n))


@dataclass
class RodBatch:
    n: np.ndarray          # int64 [nrods]
    r: np.ndarray          # float64 [nrods]
    g_left: np.ndarray     # float64 [nrods]
    g_right: np.ndarray    # float64 [nrods]
    offsets: np.ndarray    # int64 [nrods + 1], CSR offsets into u
    u0: np.ndarray         # float64 [offsets[-1]], rods packed back to back

    @property
    def nrods(self):
        return int(self.n.size)

    def rod(self, i):
        return self.u0[self.offsets[i]:self.offsets[i + 1]]


def rod_batch(seed=3, nrods=4096, nmin=256, nmax=65536, rmin=0.25, rmax=4.0,
              align=1):
    """Draw, in this order: N (nrods), r (nrods), g_L (nrods), g_R (nrods),
    z (nrods x 16).  ``align`` pads each rod's start offset to a multiple of
    ``align`` values (the padding is never read as data)."""
    rng = np.random.default_rng(seed)
    n = np.rint(np.exp(rng.uniform(np.log(nmin), np.log(nmax), nrods))).astype(np.int64)
    r = rng.uniform(rmin, rmax, nrods)
    gl = rng.uniform(-1.0, 1.0, nrods)
    gr = rng.uniform(-1.0, 1.0, nrods)
    z = rng.standard_normal((nrods, NMODES))
    padded = (n + align - 1) // align * align
    offsets = np.zeros(nrods + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(padded)
    u0 = np.zeros(int(offsets[-1]))
    for i in range(nrods):
        u0[offsets[i]:offsets[i] + n[i]] = sine_modes(int(n[i]), z[i])
    return RodBatch(n=n, r=r, g_left=gl, g_right=gr, offsets=offsets, u0=u0)


@dataclass
class MovingWallRod:
    n: int
    r: float
    nsteps: int
    u0: np.ndarray        # [n]
    g_left: np.ndarray    # [nsteps + 1], g_L(t_m)
    g_right: np.ndarray   # [nsteps + 1], g_R(t_m)
    src_b: np.ndarray     # [n], b(x_i)
    src_a: np.ndarray     # [nsteps], a(t_m + tau/2)


def moving_wall_rod(n, r=4.0, nsteps=5000, step0=0):
    h = 1.0 / (n + 1)
    tau = r * h * h
    t = (step0 + np.arange(nsteps + 1, dtype=np.float64)) * tau
    x = abscissae(n)
    return MovingWallRod(
        n=n, r=r, nsteps=nsteps, u0=np.zeros(n),
        g_left=np.sin(2.0 * np.pi * t), g_right=np.zeros(nsteps + 1),
        src_b=x * (1.0 - x), src_a=np.exp(-(t[:-1] + 0.5 * tau)))


def surrogate_rods(seed, nrods, n=4096, rmin=0.5, rmax=2.0, noise=None, modes=None):
    """Initial values and mesh ratios for surrogate training/evaluation:
    draws r (nrods) then z (nrods x 16); zero walls.  ``seed`` may be an int
    or a sequence of ints (a data set split into seeded chunks).

    ``modes = (lo, hi)`` widens the spectrum: z is drawn as nrods x hi, then
    each rod's cutoff K, log-uniform in [lo, hi], keeps modes 1..K (the
    coefficients z_k / k^2 give every mode the same second-difference
    amplitude, so short waves weigh as much as long ones in the features).
    ``noise = (lo, hi)`` then adds white noise of relative size eps, eps
    log-uniform in [lo, hi] times the rod's RMS (eps, then the values)."""
    rng = np.random.default_rng(seed)
    r = rng.uniform(rmin, rmax, nrods)
    kmax = NMODES if modes is None else int(modes[1])
    z = rng.standard_normal((nrods, kmax))
    if modes is not None:
        cut = np.exp(rng.uniform(np.log(modes[0]), np.log(modes[1]), nrods))
        z = np.where(np.arange(1, kmax + 1)[None, :] <= cut[:, None], z, 0.0)
    x = abscissae(n)
    k = np.arange(1, kmax + 1, dtype=np.float64)
    basis = np.sin(np.pi * np.outer(k, x))          # [kmax, n]
    u0 = (z / (k * k)) @ basis                       # [nrods, n]
    if noise is not None:
        lo, hi = noise
        eps = np.exp(rng.uniform(np.log(lo), np.log(hi), nrods))
        rms = np.sqrt(np.mean(u0 * u0, axis=1))
        u0 = u0 + (eps * rms)[:, None] * rng.standard_normal((nrods, n))
    return r, u0
