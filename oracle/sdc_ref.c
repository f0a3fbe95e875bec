/*
 * sdc_ref.c -- plain CPU oracle of the sub-domain form of the scheme
 * (Section 2, "complementary scheme" of Tavakoli with sub-domains of k
 * nodes; Eq. (1)-(4)).
 *
 * TEST INFRASTRUCTURE ONLY, like ge_ref.c: the tests load it; the GPU
 * library never calls it and shares nothing with it.
 *
 * Grid (Section 2): nodes x_0..x_M, h = 1/M, walls x_0 and x_M, interior
 * unknowns u_1..u_{M-1}; M an even multiple of k, M = 2ek.  The nodes
 * 0..M-1 split into odd sub-domains [x_{2ik}, x_{2ik+k-1}] and even
 * sub-domains [x_{2ik+k}, x_{2(i+1)k-1}], i = 0..e-1; an odd and the
 * following even sub-domain form a sub-domain couple (SDC) of 2k nodes.
 *
 * Two kinds of level alternate (reading: a level of global index m takes
 * the first kind when m is even):
 *
 *   first kind  -- the confluence pairs sit where two SDCs meet, nodes
 *     (2ik-1, 2ik), i = 1..e-1; they take Eq. (3)/(4) from level-m values.
 *     Then each odd sub-domain is swept left to right by scheme A, Eq. (1),
 *     from its first node (the left wall for i = 0, else the confluence
 *     value), and each even sub-domain right to left by scheme B, Eq. (2),
 *     from its last node (the confluence value, or for the last SDC node
 *     M-1 by scheme B against the right wall at the new level).
 *   second kind -- the confluence pairs sit inside each SDC, nodes
 *     (2ik+k-1, 2ik+k); then each odd sub-domain is swept right to left by
 *     scheme B down to its first node (down to x_1 for i = 0), and each even
 *     sub-domain left to right by scheme A up to its last node.  With k = 1
 *     the pair (x_0, x_1) of the first SDC meets the wall: x_1 alone takes
 *     scheme A against the wall at the new level.
 *
 * Eq. (3)/(4) are used with the denominator 1 + 2r (the determinant of the
 * pair system: scheme B at the left node and scheme A at the right one, each
 * with the other's new value), in the printed numerators.  A scheme-A/B node
 * reads its sweep predecessor at the new level and its other neighbour at
 * the old level; walls enter at the level being read.  With k = 1 the
 * scheme is the two-point-group sweep of ge_ref.c.
 *
 * FP64, -O2 -ffp-contract=off, serial.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Advance u (interior values u_1..u_{M-1}, n = M - 1 of them) by nsteps
 * levels starting at global level step0.  gl/gr: wall values per level
 * (nsteps + 1 of them, g(t_m) for m = step0..step0+nsteps) or NULL for the
 * constants gl0/gr0.  Returns 0, or -1 when (n + 1) is not a positive
 * multiple of 2k or an argument is out of range. */
int sdc_ref_step_n(int64_t n, int k, double r, int64_t step0, int64_t nsteps,
                   double *u, const double *gl, const double *gr, double gl0,
                   double gr0)
{
    if (n < 1 || k < 1 || nsteps < 0 || step0 < 0 || !u || !(r > 0))
        return -1;
    const int64_t M = n + 1;
    if (M % (2 * (int64_t)k) != 0)
        return -1;
    const int64_t e = M / (2 * (int64_t)k);
    double *w = malloc(sizeof(double) * (size_t)(M + 1));   /* level m   */
    double *v = malloc(sizeof(double) * (size_t)(M + 1));   /* level m+1 */
    if (!w || !v) {
        free(w);
        free(v);
        return -1;
    }
    for (int64_t i = 1; i < M; ++i)
        w[i] = u[i - 1];
    const double den = 1.0 + 2.0 * r;

    for (int64_t s = 0; s < nsteps; ++s) {
        const int64_t m = step0 + s;
        w[0] = gl ? gl[s] : gl0;
        w[M] = gr ? gr[s] : gr0;
        v[0] = gl ? gl[s + 1] : gl0;
        v[M] = gr ? gr[s + 1] : gr0;

        /* Eq. (3) and (4) for the pair (j, j+1) from level-m values */
#define PAIR(j)                                                              \
        do {                                                                 \
            const int64_t j_ = (j);                                          \
            v[j_] = ((r + r * r) * w[j_ - 1] + (1.0 - r * r) * w[j_] +       \
                     (r - r * r) * w[j_ + 1] + r * r * w[j_ + 2]) / den;     \
            v[j_ + 1] = (r * r * w[j_ - 1] + (r - r * r) * w[j_] +           \
                         (1.0 - r * r) * w[j_ + 1] + (r + r * r) * w[j_ + 2]) / den; \
        } while (0)
        /* scheme A, Eq. (1): predecessor on the left at the new level */
#define SCHEME_A(j) (v[(j)] = (r * v[(j) - 1] + (1.0 - r) * w[(j)] + r * w[(j) + 1]) / (1.0 + r))
        /* scheme B, Eq. (2): predecessor on the right at the new level */
#define SCHEME_B(j) (v[(j)] = (r * v[(j) + 1] + (1.0 - r) * w[(j)] + r * w[(j) - 1]) / (1.0 + r))

        if (m % 2 == 0) {
            for (int64_t i = 1; i < e; ++i)
                PAIR(2 * i * k - 1);
            for (int64_t i = 0; i < e; ++i) {
                const int64_t o0 = 2 * i * k;            /* odd sub-domain [o0, o0+k-1]  */
                const int64_t e1 = 2 * i * k + 2 * k - 1; /* even sub-domain [o0+k, e1] */
                for (int64_t j = o0 + 1; j <= o0 + k - 1; ++j)
                    SCHEME_A(j);
                if (i == e - 1)
                    SCHEME_B(e1);                        /* node M-1 against the wall */
                for (int64_t j = e1 - 1; j >= o0 + k; --j)
                    SCHEME_B(j);
            }
        } else {
            for (int64_t i = 0; i < e; ++i) {
                const int64_t o0 = 2 * i * k;
                const int64_t c = o0 + k - 1;            /* pair (c, c+1) */
                if (c == 0)
                    SCHEME_A(1);                         /* k = 1, first SDC */
                else
                    PAIR(c);
                for (int64_t j = c - 1; j >= (o0 > 0 ? o0 : 1); --j)
                    SCHEME_B(j);
                for (int64_t j = c + 2; j <= o0 + 2 * k - 1; ++j)
                    SCHEME_A(j);
            }
        }
#undef PAIR
#undef SCHEME_A
#undef SCHEME_B
        double *t = w;
        w = v;
        v = t;
    }
    for (int64_t i = 1; i < M; ++i)
        u[i - 1] = w[i];
    free(w);
    free(v);
    return 0;
}
