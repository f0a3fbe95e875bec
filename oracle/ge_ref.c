/*
 * ge_ref.c -- plain CPU oracle of the group explicit (GE) sweep for the 1D
 * diffusion equation u_t = u_xx (Parand, Zafarvahedian, Hossayni,
 * "GPU-Acceleration of Parallel Unconditionally Stable Group Explicit
 * Finite Difference Method", Section 2, Eq. (1)-(4)).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the correctness reference for the
 * GPU library: only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark load it.  It shares no code, header, table or helper with the
 * GPU path, and the GPU path never calls it.
 *
 * What it computes: the Saul'yev-type alternating group scheme of Tavakoli
 * as restated in Section 2, with sub-domains of width k = 1 (two-point
 * groups).  Each level solves every coupled pair by the confluence formulas
 * Eq. (3)/(4) and each node left alone beside a wall by scheme A, Eq. (1),
 * or scheme B, Eq. (2).  The grouping alternates between levels.  Readings
 * of points the paper leaves open (denominator of Eq. (3)/(4), which pairing
 * comes first, wall treatment, unequal or time-dependent wall values, the
 * source term, the wall-flux diagnostic) are stated where they are used in
 * ge_ref_core.inc.
 *
 * Arithmetic: FP64 (ge_ref_step_n), or x87 extended precision
 * (ge_ref_step_n_ext) for checks whose tolerance is below what FP64
 * rounding over many levels can resolve.  Built with -O2
 * -ffp-contract=off, no explicit SIMD: every product and sum is rounded as
 * written.  The all-core form (nthreads > 1) splits the points into
 * contiguous ranges, one thread each, with a barrier per level, the same
 * arithmetic in the same order per point.
 *
 * Parity pins (tests/test_oracle_ge.py): a dense matrix solve of the split
 * form and an exact rational solve on tiny grids, the printed numerators of
 * Eq. (3)/(4), preservation of constants and linear profiles, mirror
 * symmetry, the closed-form decay of sin(pi x), second-order convergence,
 * the unconditional-stability energy bound, the maximum principle at r <= 1,
 * and composition of split runs.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

#define REAL double
#define FN(name) ge_ref64_##name
#include "ge_ref_core.inc"
#undef REAL
#undef FN

#define REAL long double
#define FN(name) ge_refext_##name
#include "ge_ref_core.inc"
#undef REAL
#undef FN

/* FP64 oracle.  See ge_ref_core.inc for the meaning of each argument. */
int ge_ref_step_n(int64_t n, double r, double tau, double h,
                  int64_t step0, int64_t nsteps, double *u,
                  const double *gl, const double *gr, double gl0, double gr0,
                  const double *src_b, const double *src_a,
                  double *flux, int nthreads)
{
    return ge_ref64_step_n(n, r, tau, h, step0, nsteps, u, gl, gr, gl0, gr0,
                           src_b, src_a, flux, nthreads);
}

/* Same scheme in x87 extended precision (64-bit significand). */
int ge_ref_step_n_ext(int64_t n, double r, double tau, double h,
                      int64_t step0, int64_t nsteps, double *u,
                      const double *gl, const double *gr, double gl0, double gr0,
                      const double *src_b, const double *src_a,
                      double *flux, int nthreads)
{
    return ge_refext_step_n(n, r, tau, h, step0, nsteps, u, gl, gr, gl0, gr0,
                            src_b, src_a, flux, nthreads);
}
