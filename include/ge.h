/*
 * ge.h -- C ABI of libge, the MI355X (gfx950) group explicit (GE) sweep for
 * the 1D diffusion equation u_t = u_xx.
 *
 * The method (Section 2 of Parand, Zafarvahedian and Hossayni, "GPU-
 * Acceleration of Parallel Unconditionally Stable Group Explicit Finite
 * Difference Method"): the rod [0,1] carries n interior unknowns u_1..u_n at
 * x_i = i h, h = 1/(n+1), with wall values u_0 = g_L(t) and u_{n+1} = g_R(t).
 * With r = tau/h^2, level m -> m+1 couples the points in two-point groups,
 * (1,2),(3,4),... when m is even and (2,3),(4,5),... when m is odd; each
 * group is solved in closed form by the confluence formulas Eq. (3)/(4)
 * (denominator 1+2r) and a point left alone beside a wall takes Saul'yev
 * scheme A, Eq. (1) (left wall) or scheme B, Eq. (2) (right wall).  The
 * scheme is explicit and unconditionally stable for every r > 0.
 *
 * Conventions for every call:
 *  - Arrays marked "device" live in GPU memory of the current HIP device;
 *    arrays marked "host" live in host memory.  The caller owns every buffer;
 *    the library never frees a caller buffer.
 *  - State layout: the n interior values u_1..u_n, contiguous, element type
 *    double (GE_FP64) or float (GE_FP32).  GE_FP32_COMP holds the
 *    compensated pair (s, e), value s + e, as floats: s_1..s_n at element
 *    offset 0 and e_1..e_n at element offset ge_comp_offset(n) (n rounded up
 *    to a multiple of 64), 2*ge_comp_offset(n) floats in all.
 *  - Work is enqueued asynchronously on `stream` (a hipStream_t passed as
 *    void*, NULL = the default stream); the call returns once it is enqueued.
 *  - Errors are returned as ge_status; on any status other than GE_OK no work
 *    has been enqueued (GE_ERR_HIP excepted: a launch error may follow work
 *    already enqueued by the same call).  ge_last_error() gives a message for
 *    the last failing call of the calling thread.
 *  - Device-side conditions (a NaN or infinite value stored by a launch, a
 *    wait between waves that gave up) are recorded in status words of the
 *    plan (pinned, host-mapped memory the kernels write).  The next call on
 *    the plan reports a condition raised by a launch that has finished by
 *    then (GE_ERR_NONFINITE, GE_ERR_SYNC; nothing is enqueued by that call,
 *    and the word is cleared); ge_plan_check / ge_batch_check wait for the
 *    stream first, so they report every launch enqueued before them.
 *  - Results are bit-for-bit reproducible: they do not depend on the tiling,
 *    the number of levels fused per launch, the grid, or how a run is split
 *    into calls.
 */
#ifndef GE_H
#define GE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GE_OK = 0,
    GE_ERR_INVALID = 1,      /* an argument is out of range or inconsistent */
    GE_ERR_NOMEM = 2,        /* a host or plan-time device allocation failed */
    GE_ERR_HIP = 3,          /* the HIP runtime reported an error            */
    GE_ERR_UNSUPPORTED = 4,  /* valid request this build does not handle     */
    GE_ERR_NONFINITE = 5,    /* a parameter or value is NaN or infinite      */
    GE_ERR_SYNC = 6          /* a wait between waves inside a launch gave up */
                             /* (the results of that launch are not valid)   */
} ge_status;

typedef enum {
    GE_FP64 = 0,       /* double state, double arithmetic                      */
    GE_FP32 = 1,       /* float state, float arithmetic                        */
    GE_FP32_COMP = 2   /* float pair (s, e): the increment of each level is    */
                       /* formed from s + e and added with Kahan compensation  */
} ge_precision;

/* Library version, "major.minor.patch". */
const char *ge_version(void);

/* Message for the last failing call on the calling thread ("" if none). */
const char *ge_last_error(void);

/* Fixed name of a status code. */
const char *ge_status_str(int status);

/* Element offset of the e block of a GE_FP32_COMP state of n points
 * (n rounded up to a multiple of 64); -1 for n < 0. */
int64_t ge_comp_offset(int64_t n);

/* ------------------------------------------------------------------------
 * Single rod.
 *
 * A plan fixes the problem of Section 2 for one rod: n, r, the precision,
 * the default (constant) wall values and, optionally, a source
 * f(x, t) = a(t) b(x) whose profile b(x_i) is given here and whose time
 * factor a is given per call.  A plan holds host-side metadata and its
 * status words (pinned host memory).
 * ---------------------------------------------------------------------- */
typedef struct ge_plan_s *ge_plan_t;

typedef struct {
    int64_t n;          /* interior points, n >= 1                            */
    double r;           /* mesh ratio tau/h^2, finite and > 0                 */
    int32_t precision;  /* ge_precision                                       */
    int32_t tile;       /* points per lane (even; 0 = the library's choice)   */
    int32_t depth;      /* levels fused per launch (>= 1; 0 = library choice) */
    int32_t waves;      /* waves per workgroup (1 or 4, with k >= 2 also 2    */
                        /* and 8; 0 = library choice)                         */
    double g_left;      /* wall value g_L, used when a call gives no array    */
    double g_right;     /* wall value g_R, likewise                           */
    const void *src_b;  /* device, n values of the state's element type       */
                        /* (float for both FP32 forms): b(x_i); NULL = no     */
                        /* source.  Must stay valid while the plan is used.   */
    int32_t schedule;   /* 0 = library choice; 1 = one workgroup per tile per */
                        /* launch; 2 = persistent single-wave workgroups that */
                        /* sweep several tiles each, loading the next tile    */
                        /* during the current one (waves must be 1, except    */
                        /* for the sub-domain scheme: see k)                  */
    int32_t k;          /* sub-domain width (Section 2): 0 or 1 = two-point   */
                        /* groups, the sweep described above; 2, 4, 8 or 16 = */
                        /* odd and even sub-domains of k nodes, Eq. (3)/(4)   */
                        /* where they meet and Saul'yev's schemes A and B,    */
                        /* Eq. (1)/(2), swept through them; n + 1 must be a   */
                        /* multiple of 2k, GE_FP64 or GE_FP32, no source and  */
                        /* no flux; levels of even index take the pairs where */
                        /* sub-domain couples meet, odd ones the pairs at     */
                        /* their centres.  One couple (2k nodes) per lane,    */
                        /* 64 per wave, windows of 1, 2, 4 or 8 waves (waves  */
                        /* 0, 1, 2, 4 or 8; the waves of a window exchange    */
                        /* their edge values through LDS once per level);     */
                        /* tile must be 0 or 2k.  Schedule 2 here: resident   */
                        /* workgroups of `waves` waves that copy the          */
                        /* next window from HBM into LDS while the current    */
                        /* one advances (used from 3 windows on; at most 64   */
                        /* levels per launch, else GE_ERR_INVALID);           */
                        /* the library's choice takes it for GE_FP64 with     */
                        /* k = 16 from 64 windows on, at 24 levels per launch */
                        /* (20 otherwise).                                    */
} ge_desc;

/* Bytes of device workspace a ge_step_n call on this problem needs (the
 * second level buffer, the size of the state): 8n for GE_FP64, 4n for
 * GE_FP32, 8*ge_comp_offset(n) for GE_FP32_COMP.  Returns 0 for an invalid
 * descriptor.  A rod that fits one workgroup window is advanced in place
 * and ignores the workspace (it may then be NULL). */
size_t ge_workspace_bytes(const ge_desc *desc);

/* Validate `desc` and create a plan in *out.  Errors: GE_ERR_INVALID (null
 * pointer, n < 1, r <= 0, unknown precision, tile/depth/waves out of range,
 * k < 0, or k >= 2 with n + 1 not a multiple of 2k), GE_ERR_UNSUPPORTED
 * (k >= 2 other than 2, 4, 8, 16, or with GE_FP32_COMP or a source),
 * GE_ERR_NONFINITE (r, g_left or g_right not finite), GE_ERR_NOMEM. */
ge_status ge_plan(ge_plan_t *out, const ge_desc *desc);

/* Release a plan (NULL is ignored).  Work already enqueued is unaffected
 * (a plan that has launched work waits for the device first: its kernels
 * hold the plan's status words). */
void ge_destroy(ge_plan_t plan);

/* Wait for `stream`, then report what the plan's launches raised since the
 * last report: GE_ERR_NONFINITE if one of them stored a NaN or infinite
 * value in the state (every stored value is tested), else GE_OK.  The word
 * is cleared.  Errors: GE_ERR_INVALID (NULL plan), GE_ERR_HIP. */
ge_status ge_plan_check(ge_plan_t plan, void *stream);

/* Advance the state `u` (device, layout above) from global level `step0` to
 * level step0 + nsteps.  The parity of each level, hence its grouping, is
 * taken from the global level index, so consecutive calls compose exactly:
 * (step0=0, nsteps=a) then (step0=a, nsteps=b) equals (0, a+b) bit for bit.
 *
 * workspace: device, ge_workspace_bytes(desc) bytes, 256-byte aligned, not
 *            overlapping u; its contents on return are unspecified.
 * g_left_t, g_right_t: device, nsteps+1 doubles each, the wall values
 *            g(t_m) for m = step0..step0+nsteps; NULL = the plan's constant.
 * src_a_t:   device, nsteps doubles, a(t_m + tau/2) for m = step0..; must be
 *            given when the plan has a source and be NULL otherwise.
 * flux:      device, 2 doubles or NULL.  Adds, level by level in FP64, the
 *            wall first differences tau*(u_1 - g_L)/h and tau*(u_n - g_R)/h
 *            at every new level to flux[0] and flux[1].
 * u and workspace must be 16-byte aligned.  nsteps = 0 enqueues nothing.
 * Errors: GE_ERR_INVALID (null plan/u/workspace, negative step0 or nsteps,
 * misalignment, aliasing, source array missing or unexpected),
 * GE_ERR_UNSUPPORTED (flux with a sub-domain plan), GE_ERR_NONFINITE (an
 * earlier launch of this plan, finished by now, stored a NaN or infinite
 * value; nothing is enqueued), GE_ERR_HIP. */
ge_status ge_step_n(ge_plan_t plan, void *u, void *workspace, int64_t step0,
                    int64_t nsteps, const double *g_left_t,
                    const double *g_right_t, const double *src_a_t,
                    double *flux, void *stream);

/* Choice the plan made (or was given): points per lane, levels per launch,
 * waves per workgroup, and the halo width it implies. */
ge_status ge_plan_config(ge_plan_t plan, int32_t *tile, int32_t *depth,
                         int32_t *waves, int32_t *halo);

/* The schedule the plan's multi-tile launches use: 1 = one workgroup per
 * tile, 2 = persistent single-wave workgroups; -1 for NULL. */
int32_t ge_plan_schedule(ge_plan_t plan);

/* Convert between the compensated pair and FP64 (checkpoints of a
 * GE_FP32_COMP run).  pair: device, GE_FP32_COMP layout of n points; x:
 * device, n doubles.  to_fp64 writes x = s + e; from_fp64 writes
 * s = fl32(x), e = fl32(x - s). */
ge_status ge_comp_to_fp64(const float *pair, double *x, int64_t n, void *stream);
ge_status ge_comp_from_fp64(const double *x, float *pair, int64_t n, void *stream);

/* ------------------------------------------------------------------------
 * Two-dimensional extension: u_t = u_xx + u_yy on the unit square with
 * constant Dirichlet walls.  The paper states that the method extends to two
 * dimensions but gives no formulas; the reading built here applies, in every
 * level m, the one-dimensional level m of Section 2 (two-point groups,
 * Eq. (3)/(4); a point alone beside a wall by Eq. (1)/(2)) along every row
 * with r = rx, then along every column with r = ry (first-order splitting;
 * each line paired by the global level index as a single rod is).
 *
 * Layout: u holds ny rows of nx values, row-major; element (j, i) is
 * u(x_{i+1}, y_{j+1}) with hx = 1/(nx+1), hy = 1/(ny+1), so rx = tau/hx^2
 * and ry = tau/hy^2.  double for GE_FP64, float for GE_FP32.
 * ---------------------------------------------------------------------- */
typedef struct {
    int64_t nx, ny;     /* interior points per row and per column (>= 1)     */
    double rx, ry;      /* mesh ratios, > 0 and finite                      */
    int32_t precision;  /* GE_FP64 or GE_FP32                               */
    double g_west, g_east, g_south, g_north;   /* wall values (x = 0, x = 1, */
                                               /* y = 0, y = 1)              */
    int32_t depth;      /* levels fused per launch: 1, 2 or 4 (a halo of 2   */
                        /* points per level and side is recomputed); 0 =     */
                        /* library choice.  Changes no bits of the result.   */
} ge_2d_desc;

/* Bytes of device workspace a ge_2d_step_n call needs (a second grid:
 * nx*ny elements); 0 for an invalid description. */
size_t ge_2d_workspace_bytes(const ge_2d_desc *desc);

/* Advance the grid u (device, caller-owned, layout above) by nsteps levels
 * starting at global level step0 >= 0, on `stream` (a hipStream_t, NULL =
 * the null stream).  workspace: device, ge_2d_workspace_bytes bytes, not
 * overlapping u.  One launch per `depth` levels; the call returns once the work is
 * enqueued and u holds the result when the stream reaches it.  Errors:
 * GE_ERR_INVALID (bad description, NULL or overlapping buffers, negative
 * step0/nsteps, depth not 0, 1, 2 or 4; nothing enqueued),
 * GE_ERR_UNSUPPORTED (GE_FP32_COMP), GE_ERR_HIP. */
ge_status ge_2d_step_n(const ge_2d_desc *desc, void *u, void *workspace, int64_t step0,
                      int64_t nsteps, void *stream);

/* ------------------------------------------------------------------------
 * Batch of independent rods: the same scheme (Section 2) for every rod, each
 * rod with its own n, r and constant wall values, all advanced by the same
 * levels in one persistent launch that a hipGraph captures.
 *
 * Layout of the packed state u: rod i occupies elements
 * offsets[i] .. offsets[i] + n[i] - 1 (double for GE_FP64, float for the two
 * FP32 forms).  For GE_FP32_COMP the e parts follow in a second block at
 * element offset ge_comp_offset(offsets[nrods]); ge_batch_state_elems() gives
 * the buffer length in elements.  Every offsets[i] must be a multiple of 4 and
 * offsets[i+1] >= offsets[i] + n[i].
 *
 * A rod of up to 65536 (GE_FP32) or 32768 (GE_FP64, GE_FP32_COMP) points is
 * held in registers of one workgroup for all levels, so it is read and
 * written once per call.  A longer rod takes a workgroup of its own and is
 * swept the way ge_step_n sweeps a rod: in passes of up to 32 levels over
 * windows with recomputed halos, ping-ponging between u and its own second
 * level buffer in the workspace (an even number of passes, so the result
 * lands in u).  Every rod gets the same bits as ge_step_n gives it.
 * ---------------------------------------------------------------------- */
typedef struct ge_batch_s *ge_batch_t;

typedef struct {
    int64_t nrods;
    const int64_t *n;        /* host, nrods: interior points of each rod      */
    const int64_t *offsets;  /* host, nrods+1: element offset of each rod     */
    const double *r;         /* host, nrods: mesh ratio of each rod           */
    const double *g_left;    /* host, nrods: constant left wall values        */
    const double *g_right;   /* host, nrods: constant right wall values       */
    int32_t precision;       /* ge_precision                                  */
    int32_t tune;            /* 1: measure the per-level cost of each         */
                             /* points-per-lane choice on this device now and */
                             /* store it (file $GE_TUNE_CACHE, default        */
                             /* ~/.cache/libge/batch_tune.txt); 0: use the    */
                             /* stored measurement, or built-in defaults      */
    int32_t sync;            /* how the waves of a rod exchange edge values:  */
                             /* 0 = library choice, 1 = every level, at a     */
                             /* workgroup barrier, 2 = every level, each wave */
                             /* waiting for its two neighbours only (level    */
                             /* flags in LDS), 3 = neighbouring waves overlap */
                             /* by a lane or more, refreshed at a barrier     */
                             /* every K-1 levels (the default; rods of one    */
                             /* wave and rods whose overlapping waves do not  */
                             /* fit a workgroup use 2 in the same launch)     */
} ge_batch_desc;

/* Create a batch plan: choose points per lane for every rod, bundle rods
 * into workgroup tasks, order them largest first, and copy the rod and task
 * tables to device memory owned by the plan (freed by ge_batch_destroy).
 * With tune = 1 this runs timing kernels on the current device.  Every
 * choice gives bit-identical results.  Errors: GE_ERR_INVALID,
 * GE_ERR_NONFINITE, GE_ERR_NOMEM, GE_ERR_HIP. */
ge_status ge_batch_plan(ge_batch_t *out, const ge_batch_desc *desc);

/* Release a batch plan and its graph (NULL is ignored). */
void ge_batch_destroy(ge_batch_t batch);

/* Elements of the packed state buffer (see the layout above); -1 for NULL. */
int64_t ge_batch_state_elems(ge_batch_t batch);

/* Bytes of device workspace ge_solve_batch needs: 256 (the task queue head),
 * plus, when rods are above the on-chip limit, their second level buffers
 * from byte 256 on (each rod's points rounded up to 64 elements, twice for
 * GE_FP32_COMP). */
size_t ge_batch_workspace_bytes(ge_batch_t batch);

/* Number of polls (each a short sleep, about 30 ns) a wave's wait for a
 * neighbouring wave makes before it gives up (default 65536).  The waits
 * belong to rods whose waves exchange edge values every level (sync = 2, or
 * the rods sync = 3 cannot give overlapping lanes); they always end within
 * microseconds, and the bound only keeps a wave from spinning forever.  A
 * wait that gives up raises GE_ERR_SYNC for the next ge_solve_batch or
 * ge_batch_check.  polls = 0 makes every wait give up without looking (a
 * test of that path; every kernel still exits normally).  Drops the
 * plan's captured graphs.  Errors: GE_ERR_INVALID (NULL, polls < 0 or above
 * 2^30). */
ge_status ge_batch_set_wait_polls(ge_batch_t batch, int64_t polls);

/* Wait for `stream`, then report what the plan's runs raised since the last
 * report: GE_ERR_SYNC (a wait gave up), else GE_ERR_NONFINITE (a stored
 * value was NaN or infinite), else GE_OK.  The reported word is cleared.
 * Errors: GE_ERR_INVALID (NULL batch), GE_ERR_HIP. */
ge_status ge_batch_check(ge_batch_t batch, void *stream);

/* The plan's shape: number of tasks, resident workgroups, the planner's
 * estimate of the time of one level in microseconds, and (if rod_k is not
 * NULL, host, nrods entries) the points per lane chosen for each rod. */
ge_status ge_batch_info(ge_batch_t batch, int32_t *ntasks, int32_t *grid,
                        double *est_us_per_level, int32_t *rod_k);

/* Advance every rod from level step0 by nsteps levels, in place in u
 * (device, packed as above, 16-byte aligned).  workspace: device,
 * ge_batch_workspace_bytes() bytes, 256-byte aligned; it must not be used
 * by another run at the same time.  The first call for a given (u,
 * workspace, parity of step0, nsteps) captures the queue reset and the
 * persistent launch in a hipGraph; later calls with the same key replay it
 * on `stream`.  Errors: GE_ERR_INVALID, GE_ERR_SYNC or GE_ERR_NONFINITE (an
 * earlier run, finished by now, raised it; nothing is enqueued), GE_ERR_HIP. */
ge_status ge_solve_batch(ge_batch_t batch, void *u, void *workspace,
                         int64_t step0, int64_t nsteps, void *stream);

/* ge_solve_batch for callers that cannot allocate device memory or
 * instantiate a graph (code under stream capture, tight serving loops,
 * harnesses that forbid allocation): the same run, bit for bit, with the
 * task queue head and the second level buffers of the rods above the
 * on-chip limit in a static scratch array of the library (32 MiB per GPU,
 * held from the first call on that GPU until the process ends), launched
 * directly on `stream` (no graph).  It allocates nothing.  Every call on a
 * GPU shares that GPU's scratch: calls that overlap on one GPU (on two
 * streams, or from two threads) race and give undefined results.
 * Errors: GE_ERR_INVALID (as ge_solve_batch), GE_ERR_UNSUPPORTED (the plan's
 * rods above the on-chip limit need more than 32 MiB - 256 B of second
 * level buffers, ge_batch_workspace_bytes() > 32 MiB), GE_ERR_SYNC /
 * GE_ERR_NONFINITE (as ge_solve_batch), GE_ERR_HIP. */
ge_status ge_solve_batch_static(ge_batch_t batch, void *u, int64_t step0, int64_t nsteps,
                                void *stream);

/* ------------------------------------------------------------------------
 * Learned 64-level propagator (surrogate).  A 1D convolutional network over
 * the points of a rod maps u at level m to a normalised increment; a jump is
 *     u(m + 64) ~ u + 64 r s out,
 * with s the RMS of the rod's second differences.  Layers (channels last,
 * bfloat16 activations and weights, FP32 accumulation on the matrix cores):
 * conv 2->64 + GELU; four residual layers h += GELU(conv 64->64); conv
 * 64->1; kernel width 5, tap spacings 1, 2, 4, 8, 16, 1, zero padding, GELU
 * in its tanh form (z/2)(1 + tanh(sqrt(2/pi)(z + 0.044715 z^3))).  Inputs: the second
 * difference of u divided by s, and r mapped from [0.5, 2] to [-1, 1].
 * Training minimises the mean squared error against the normalised
 * increment (u(m + 64) - u(m)) / (64 r s) of the GE sweep, with Adam on
 * FP32 master weights; every reduction has a fixed order, so a training run
 * is reproducible bit for bit.
 *
 * Arrays: u, u64: device, batch x width floats (rods back to back, zero
 * walls); r: device, batch floats.  width is a multiple of 128.
 * ---------------------------------------------------------------------- */
typedef struct ge_nn_s *ge_nn_t;

/* Number of parameters (83201), in the flat layout used below: for each of
 * the six layers, W[5][c_out][c_in] then b[c_out]. */
int64_t ge_nn_param_count(void);

/* Create a network for rods of `width` points and up to `max_batch` rods
 * per call, with a seeded initialisation.  Allocates every device buffer
 * the network needs (about 3.7 GB for 512 x 4096); later calls allocate
 * nothing.  Errors: GE_ERR_INVALID, GE_ERR_NOMEM, GE_ERR_HIP. */
ge_status ge_nn_create(ge_nn_t *out, int32_t width, int32_t max_batch, uint64_t seed);
void ge_nn_destroy(ge_nn_t net);

/* Copy the FP32 master parameters in (resets the optimiser) or out (host
 * arrays of ge_nn_param_count() floats; synchronous). */
ge_status ge_nn_set_params(ge_nn_t net, const float *host, int64_t count);
ge_status ge_nn_get_params(ge_nn_t net, float *host, int64_t count);

/* Network output (device, batch x width floats, the normalised increment)
 * and the per-rod scale s (device, batch floats); either may be NULL. */
ge_status ge_nn_forward(ge_nn_t net, const float *u, const float *r, int32_t batch,
                        float *out, float *scale, void *stream);

/* One 64-level jump: u_next = u + 64 r s out (device, batch x width). */
ge_status ge_nn_jump(ge_nn_t net, const float *u, const float *r, int32_t batch,
                     float *u_next, void *stream);

/* Forward, loss and backward without an update: the mean squared error goes
 * to *loss (device float, or NULL) and the gradient of every parameter is
 * kept in the network (ge_nn_gradient copies it out). */
ge_status ge_nn_grads(ge_nn_t net, const float *u, const float *u64, const float *r,
                      int32_t batch, float *loss, void *stream);
ge_status ge_nn_gradient(ge_nn_t net, float *grad /* device, param_count */, void *stream);

/* ge_nn_grads followed by one Adam step (beta 0.9/0.999, eps 1e-8). */
ge_status ge_nn_train_step(ge_nn_t net, const float *u, const float *u64, const float *r,
                           int32_t batch, float lr, float *loss, void *stream);

/* Surrogate time stepping with a re-check and a fallback to the GE sweep.
 * Advances `batch` rods of the network's width (zero walls; u: device,
 * batch x width floats, updated in place) by njumps jumps of 64 levels,
 * starting at level step0.  The jumps go in windows of `check` jumps (the
 * last window may be shorter).  The last jump of each window is also taken
 * by 64 levels of the GE sweep from the same input, with `ge`: an FP64 batch
 * plan (ge_batch_plan) of exactly these rods -- batch rods of width points,
 * in order, with the mesh ratios that r (device, batch floats) holds rounded
 * to FP32 and zero walls -- and its workspace ge_ws.  A rod whose relative
 * L2 distance ||u_net - u_GE|| / ||u_GE|| exceeds tol (or is not a number)
 * restarts the window from its state at the window's start and takes the
 * whole window by the GE sweep (FP64, rounded to FP32 at the end); the
 * other rods keep the network's result.
 * Optional outputs: accepted, fallbacks (device int32 per rod: counts of
 * accepted and rejected windows, incremented), last_err (device double per
 * rod: the distance at the last check), *n_fallback (host: rejected
 * rod-windows in this call).  The GE state lives in network-owned buffers;
 * the stream is synchronised once per window to learn whether any rod was
 * rejected, and the fallback sweep (whole batch, rejected rods kept) runs
 * only then.  Errors: GE_ERR_INVALID (arguments, a plan that is not FP64 or
 * does not match the rods), GE_ERR_HIP. */
ge_status ge_nn_advance(ge_nn_t net, ge_batch_t ge, void *ge_ws, float *u, const float *r,
                        int32_t batch, int64_t step0, int32_t njumps, int32_t check,
                        double tol, int32_t *accepted, int32_t *fallbacks, double *last_err,
                        int64_t *n_fallback, void *stream);

/* Shape of layer `layer` (1..6): real input and output channels (ci, co),
 * the padded channels its activations are stored with on the device (input
 * cip, output cop), the padded channels of the gradient entering it from
 * its output (cod), and its tap spacing (dil).  Any pointer may be NULL.
 * Errors: GE_ERR_INVALID (layer outside 1..6). */
ge_status ge_nn_layer_shape(int32_t layer, int32_t *ci, int32_t *co, int32_t *cip, int32_t *cop,
                            int32_t *cod, int32_t *dil);

/* One product of one layer on caller-given bfloat16 operands, with the
 * network's current (bfloat16-packed) weights, each result in FP32 before
 * any rounding -- a probe for tests that check the matrix-core products
 * against an oracle fed the same operands.  Arrays are device memory,
 * channels last, `batch` rods of the network's width:
 *   op 0, forward:        x: bf16 [batch][width][cip]; out: float
 *                         [batch][width][cop] = conv(x, W) + b;
 *   op 1, input gradient: g: bf16 [batch][width][cod]; out: float
 *                         [batch][width][cip], the gradient of
 *                         sum(conv(x, W) g) with respect to x (layers 2..6);
 *   op 2, weight gradient: x as op 0, g as op 1; out: float, the flat
 *                         gradient of the layer, dW[5][co][ci] then db[co]
 *                         (the order of ge_nn_param_count's layout).
 * Padded channels of x and g must hold zeros.  Uses the network's scratch
 * buffers: do not overlap with other calls on the same network.  Errors:
 * GE_ERR_INVALID (network, layer, op, batch or a NULL array), GE_ERR_HIP. */
ge_status ge_nn_layer_probe(ge_nn_t net, int32_t layer, int32_t op, const void *x, const void *g,
                            int32_t batch, float *out, void *stream);

/* Element-wise precision conversions on the device (n elements, enqueued on
 * the stream): FP32 to FP64 and FP64 to FP32 (round to nearest). */
ge_status ge_f32_to_f64(const float *x, double *y, int64_t n, void *stream);
ge_status ge_f64_to_f32(const double *x, float *y, int64_t n, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* GE_H */
