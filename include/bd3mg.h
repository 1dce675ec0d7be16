/*
 * bd3mg.h -- C interface of libbd3mg, the MI355X (gfx950) implementation of
 * the block distributed 3MG method (BD3MG) for restoring a 3D volume blurred
 * by a depth-variant PSF (Chalvidal & Chouzenoux, arXiv 2002.02328).
 *
 * Problem (Sec. 2, eq. "P"; Sec. 3.1, eqs. "model" and "eq_crit"):
 *   minimise over x in R^N, N = nx*ny*nz,
 *     f(x) = 1/2 ||H x - y||^2 + eta * d^2(x, [xmin, xmax]^N)
 *          + lambda * sum_n sqrt((V^X x)_n^2 + (V^Y x)_n^2 + delta^2)
 *          + kappa * ||V^Z x||^2
 *   where H is a depth-variant 3D blur and V^X, V^Y, V^Z are forward
 *   differences (last difference 0).  The variables are split into blocks of
 *   whole z-slices (Sec. 3.1), and each block update is one memory-gradient
 *   majorize-minimize step (Sec. 2.3, boxes "Master" and "Worker").
 *
 * Conventions
 *   - Volumes are [nz][ny][nx], x fastest, dense, no padding.
 *   - Element type of every volume crossing this interface is the problem's
 *     storage type: double for BD3MG_FP64, float for BD3MG_FP32.  Scalars
 *     (f, norms, PSF tables, parameters) are always double.
 *   - PSF: separable per output slice k,
 *       (H x)_{k,j,i} = sum_{c,b,a} gz_k[c] gy_k[b] gx_k[a] x_{k-c, j-b, i-a},
 *     zero padding; table rows are indexed [k][a + r], a in [-r, r].
 *   - "on_device" pointers are device memory of the calling process on the
 *     problem's HIP device; the library reads/writes them in order on the
 *     problem's stream (its own, or the caller's, see bd3mg_create) and
 *     synchronises that stream before returning.  Host pointers may be
 *     pageable.
 *   - Ownership: every input is copied before the call returns; the library
 *     keeps no caller pointer.  A problem handle owns all of its device
 *     memory and releases it in bd3mg_destroy.
 *   - Errors: every call returns a status; nothing aborts or throws across
 *     this interface.  bd3mg_last_error() returns a thread-local description
 *     of the last failure in the calling thread.
 *   - Calls on one handle must not overlap (no internal locking).
 */
#ifndef BD3MG_H
#define BD3MG_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bd3mg_problem_s *bd3mg_problem;

typedef enum {
    BD3MG_OK = 0,
    BD3MG_ERR_ARG = 1,           /* invalid argument (sizes, parameters, tables) */
    BD3MG_ERR_STATE = 2,         /* call made before the state it needs was set */
    BD3MG_ERR_NOMEM = 3,         /* device or host allocation failed */
    BD3MG_ERR_HIP = 4,           /* a HIP runtime call failed */
    BD3MG_ERR_NOT_CONVERGED = 5  /* run stopped at max_sweeps above the tolerance; x is valid */
} bd3mg_status;

typedef enum {
    BD3MG_FP64 = 0,  /* storage, stencils, reductions and solve in double */
    BD3MG_FP32 = 1   /* storage and stencils in float; inner products, the 2x2
                        majorant system, its solve and f in double */
} bd3mg_precision;

typedef enum {
    /* Blocks at least max(2*r_z, kappa > 0 or bd3mg_set_tv3d) slices apart
     * share a colour and are updated together; colours run in order.
     * Same-colour blocks read and write disjoint data, so this equals the
     * sequential (delay-free) rule of Sec. 3.1 applied in colour-major order
     * (Sec. 2.4, delta_k = 0). */
    BD3MG_SCHED_COLORED = 0,
    /* One block at a time in z order (the natural sequential rule). */
    BD3MG_SCHED_SEQUENTIAL = 1,
    /* Asynchronous rounds: every block computes its step from the same
     * snapshot of x, then all steps are applied (Sec. 2.4: block updates with
     * delays of at most tau = nblocks - 1, Assumption B).  Without inflation
     * of the majorant this can diverge when blocks interact through H (thin
     * blocks, wide z blur); Assumption C asks for curvature beyond
     * L sqrt(tau), see bd3mg_set_inflation and bd3mg_lipschitz_bound. */
    BD3MG_SCHED_ROUND = 2
} bd3mg_schedule;

typedef enum { BD3MG_OP_H = 0, BD3MG_OP_HT = 1, BD3MG_OP_GRAD = 2 } bd3mg_op;

typedef struct {
    int sweeps;           /* sweeps done by this call (a sweep updates every block once) */
    int converged;        /* 1 if ||grad f|| <= grad_rtol * grad_norm_ref was reached */
    double f;             /* f at the returned x (NaN when nothing was evaluated) */
    double grad_norm;     /* ||grad f(x)|| at the last check */
    double grad_norm_ref; /* ||grad f(y)||, the normaliser of the stop rule */
    double seconds;       /* device time of the call, from HIP events */
} bd3mg_result;

/* Library version, (major << 16) | minor. */
int bd3mg_version(void);

/* Thread-local text of the last failure ("" if none). */
const char *bd3mg_last_error(void);

/* PSF factor tables of a depth-variant Gaussian (Sec. 3.1: per-depth blur
 * widths).  table[z][a + r] = exp(-a^2 / (2 sigma[z]^2)) normalised to sum 1
 * over a in [-r, r], r = (k - 1) / 2.  Host arrays: sigma[nz], table[nz*k].
 * ERR_ARG: nz < 1, k < 1 or even, sigma <= 0 or not finite. */
bd3mg_status bd3mg_psf_gaussian(int nz, int k, const double *sigma, double *table);

/* Create a problem of nx*ny*nz voxels in the given precision (bd3mg_precision)
 * on the current HIP device (the problem statement of Sec. 2, eq. "P", on the
 * volume of Sec. 3.1).  hip_stream is the hipStream_t on which every pass,
 * copy and evaluation of this problem is enqueued: NULL gives the problem a
 * non-blocking stream of its own (created here, destroyed by bd3mg_destroy);
 * a caller's stream (for instance a torch stream's handle) is used as given,
 * is not destroyed, must outlive the problem and must belong to the current
 * device.  Work the caller enqueues on that stream before a call is ordered
 * before it, so device buffers written there may be passed with on_device = 1
 * without further synchronisation.  ERR_ARG: a dimension < 1, precision
 * unknown, or one slice (nx*ny elements) of 2 GiB or more. */
bd3mg_status bd3mg_create(int nx, int ny, int nz, int precision, void *hip_stream,
                          bd3mg_problem *out);

/* Release the handle and all its device memory.  NULL is accepted. */
bd3mg_status bd3mg_destroy(bd3mg_problem p);

/* Separable depth-variant PSF (Sec. 3.1).  Host tables gx[nz*kx], gy[nz*ky],
 * gz[nz*kz].  ERR_ARG: even or < 1 sizes, kx or ky > 9, kz > 9, or a
 * non-finite entry.  Marks the residual stale. */
bd3mg_status bd3mg_set_psf_separable(bd3mg_problem p, int kx, int ky, int kz,
                                     const double *gx, const double *gy, const double *gz);

/* Depth-variant Gaussian PSF built with bd3mg_psf_gaussian: kxy x kxy in-slice
 * with widths sigma_xy[nz], kz along z with widths sigma_z[nz]. */
bd3mg_status bd3mg_set_psf_gaussian(bd3mg_problem p, int kxy, int kz,
                                    const double *sigma_xy, const double *sigma_z);

/* Per-depth rotated anisotropic Gaussian kernels (Sec. 3.1: the blur of each
 * depth has its own variance and rotation, drawn at random): for slice z,
 *   P_z[t][b][a] = exp(-u^2 / (2 sx^2) - v^2 / (2 sy^2) - t^2 / (2 sz^2)) / Z_z,
 *   u = a cos(theta) + b sin(theta),  v = b cos(theta) - a sin(theta),
 * t, b, a centred (|t| <= kz/2, |b|, |a| <= kxy/2), each kernel summing to 1.
 * Host arrays sx, sy, theta, sz [nz]; out [nz][kz][kxy][kxy] (host, caller
 * owned).  ERR_ARG: even sizes, nz < 1, a width <= 0 or a non-finite
 * value. */
bd3mg_status bd3mg_psf_rotated_gaussian(int nz, int kxy, int kz, const double *sx, const double *sy,
                                        const double *theta, const double *sz, double *out);

/* General depth-variant PSF (Sec. 3.1, eq. "model"): the kernel of output
 * slice k is P[k] (host, [nz][kz][ky][kx], c, b, a centred) and
 *   (Hx)_k[j][i] = sum_{c,b,a} P_k[c][b][a] x_{k-c}[j-b][i-a]
 * with zero padding.  Replaces a separable PSF (and a separable PSF set later
 * replaces this one).  The passes then use the general kernels: the
 * maintained residual vector (the q of bd3mg_get_state / bd3mg_set_state) is
 * r = Hx - y itself.  ERR_ARG: even sizes, kx or ky > 11, kz > 21, or a
 * non-finite entry.  Marks the residual stale. */
bd3mg_status bd3mg_set_psf_dense(bd3mg_problem p, int kx, int ky, int kz, const double *P);

/* Parameters of f (Sec. 3.1, eq. "eq_crit").  ERR_ARG: delta <= 0, lambda,
 * eta or kappa < 0, xmin > xmax, or a non-finite value.  Defaults before the
 * first call: lambda = eta = kappa = 0, delta = 1, [xmin, xmax] = [0, 1]. */
bd3mg_status bd3mg_set_params(bd3mg_problem p, double lambda, double delta, double eta,
                              double kappa, double xmin, double xmax);

/* Total variation over the volume instead of per slice, an option beside the
 * criterion of Sec. 3.1 (eq. "eq_crit"), whose total variation takes only the
 * in-slice differences V^X, V^Y inside the root and leaves z to the separate
 * kappa ||V^Z x||^2.  on = 1 puts V^Z inside the root as well:
 *   lambda sum sqrt((V^X x)^2 + (V^Y x)^2 + (V^Z x)^2 + delta^2),
 * with the same forward differences (zero at the last slice), its gradient
 * term lambda V^Z^T(omega V^Z x) and the matching half-quadratic majorant
 * term lambda V^Z^T Diag(omega) V^Z; kappa still adds its own term.  on = 0
 * (the default) is the paper's criterion.  A block's gradient then reads x
 * on the slices next to the block, and same-colour blocks keep at least one
 * slice apart.  Async-MM and the fused launches of a batch do not take it.
 * ERR_ARG: on not 0 or 1.  ERR_STATE: the method is Async-MM. */
bd3mg_status bd3mg_set_tv3d(bd3mg_problem p, int on);

/* Restores the last run's guard of the asynchronous rounds made
 * (BD3MG_OPT_ROUND_GUARD), and the inflation mu now in use.  Either pointer
 * may be NULL. */
bd3mg_status bd3mg_round_guard_info(bd3mg_problem p, int *trips, double *mu);

/* Curvature inflation (Sec. 2.5, Assumption C): every block step uses the
 * majorant A_S(x) + mu Id instead of A_S(x), for every schedule.  mu = 0
 * (the default) is the paper's majorant.  ERR_ARG: mu < 0 or not finite. */
bd3mg_status bd3mg_set_inflation(bd3mg_problem p, double mu);

/* Block step of the ablation study (Sec. 3.2, "Ablation study and
 * comparative analysis"), each a change of the Worker's step:
 * BD3MG_METHOD_BD3MG (default): the memory-gradient subspace [-grad, d_prev]
 *   with the half-quadratic majorant (Sec. 2.3);
 * BD3MG_METHOD_ASYNC_GD: the subspace {-grad} with the metric L Id, so the
 *   step is -grad_S f / L;
 * BD3MG_METHOD_ASYNC_CG: BD3MG's subspace with the metric L Id (read
 *   literally: -grad lies in the subspace, so the step equals Async-GD's up to
 *   rounding);
 * BD3MG_METHOD_ASYNC_MM: no subspace, d' = -A_S(x)^{-1} grad_S f, the linear
 *   system solved by at most n_inner iterations of conjugate gradients from
 *   0 (for the symmetric A_S these are the linear biconjugate gradient
 *   iterates with the shadow residual started at the residual), stopping
 *   early once ||r|| <= tol_inner ||r_0|| (tol_inner = 0: n_inner
 *   iterations) or when a step is undefined; needs the separable PSF, the
 *   total variation of the slices (not bd3mg_set_tv3d) and the coloured or
 *   sequential schedule (ERR_STATE at run otherwise).
 * lip: L of the metric L Id (GD, CG); lip <= 0 takes bd3mg_lipschitz_bound
 * at each run.  The inflation mu (bd3mg_set_inflation) adds to every metric.
 * bd3mg_block_step's info for Async-MM is {iterations, ||r_end||^2, 0,
 * -||g||^2, 0, 0, 0, ||g||^2}; for GD and CG {B11, B12, B22, c1, c2, u1, u2,
 * ||g||^2} of the metric L Id.  ERR_ARG: unknown method, non-finite lip,
 * n_inner outside [1, 10000] for Async-MM, tol_inner < 0. */
typedef enum {
    BD3MG_METHOD_BD3MG = 0,
    BD3MG_METHOD_ASYNC_GD = 1,
    BD3MG_METHOD_ASYNC_CG = 2,
    BD3MG_METHOD_ASYNC_MM = 3
} bd3mg_method;
bd3mg_status bd3mg_set_method(bd3mg_problem p, int method, double lip, int n_inner, double tol_inner);

/* An upper bound L of the Lipschitz constant of grad f (Assumption A) from
 * the PSF tables and parameters: ||H||_1 ||H||_inf + 2 eta + 8 lambda / delta
 * + 8 kappa (the in-slice difference operators have ||D||^2 <= 8 and
 * omega <= 1 / delta; 12 lambda / delta with the total variation along z,
 * bd3mg_set_tv3d).  With tau = nblocks - 1, mu = L (2 sqrt(tau) + 1)
 * satisfies Assumption C for BD3MG_SCHED_ROUND whatever the point (a
 * sufficient, conservative reading).  ERR_STATE: PSF not set. */
bd3mg_status bd3mg_lipschitz_bound(bd3mg_problem p, double *L);

/* Observation y (eq. "model"), nz*ny*nx elements of the storage type. */
bd3mg_status bd3mg_set_data(bd3mg_problem p, const void *y, int on_device);

/* Block partition along z: nblocks blocks of nslices[b] consecutive slices,
 * in z order (Sec. 3.1; the sets are pairwise disjoint, Sec. 2.3 eq. "disj").
 * schedule is a bd3mg_schedule.  ERR_ARG: nblocks < 1, a count < 1, or the
 * counts not summing to nz.  Resets every block's previous step to 0.
 * The first run afterwards also allocates, besides the problem's volumes,
 * room for H d1 and H d2 on S +- r_z of every block updated together (the
 * direction pass stores them, the update pass combines them): at most 2 (n_c + 2 r_z
 * b_c) slices for the largest group of b_c blocks with n_c slices in all; for
 * BD3MG_SCHED_ROUND, 2 (nz + 2 r_z nblocks) slices.  ERR_NOMEM there if that
 * does not fit. */
bd3mg_status bd3mg_set_blocks(bd3mg_problem p, int nblocks, const int *nslices, int schedule);

/* The sweep order in use: *ncolors, order[nblocks] (block indices in update
 * order) and color[nblocks].  Arrays may be NULL.  ERR_STATE before set_blocks
 * (needs the PSF too, as the colouring depends on r_z). */
bd3mg_status bd3mg_get_schedule(bd3mg_problem p, int *ncolors, int *order, int *color);

/* Initial point x^0 (box "Master", initialisation).  x0 == NULL means x^0 = y.
 * Resets every block's previous step to 0. */
bd3mg_status bd3mg_set_x0(bd3mg_problem p, const void *x0, int on_device);

/* Run BD3MG sweeps from the current state (x, each block's previous step and
 * the maintained blurred residual q, q_m = XY^T_m (H x - y)_m: the residual of
 * slice m blurred by the adjoint of slice m's in-slice factors, from which
 * H^T (H x - y) is a z-stencil; with a general PSF, q = H x - y), so calls
 * can be chained: run(a) then run(b)
 * gives bitwise the same state as run(a + b).  Stops after max_sweeps
 * sweeps, or, when grad_rtol > 0, at the first check with ||grad f(x)|| <=
 * grad_rtol * ||grad f(y)||; a check happens every check_every sweeps and
 * after the last sweep.  A check runs on the device from the maintained q;
 * a check that passes is confirmed on a residual rebuilt from x (in scratch,
 * q untouched), and when the rebuilt gradient is above the threshold q is
 * replaced by the rebuilt residual and the run goes on.  res->f and
 * res->grad_norm are evaluated at the returned x from a rebuilt residual.
 * With grad_rtol <= 0 and check_every == 0 nothing is evaluated (res->f and
 * res->grad_norm are NaN) and the call only enqueues the sweeps and waits for
 * them.  res may be NULL.  check_every == BD3MG_CHECK_ADAPTIVE (grad_rtol >
 * 0 only): checks are spaced by the trend of ||grad f||: a check after the
 * first sweep, then, while the line through the last two checks (log
 * ||grad f|| against sweeps) meets the threshold more than 8 sweeps ahead,
 * one check after half that distance (at most 256 sweeps), else a check
 * after every sweep; the run stops at the first check that meets the
 * tolerance, as with check_every = 1 near the crossing, at the cost of far
 * fewer evaluations.  ERR_ARG: max_sweeps < 0, check_every < -1, or
 * adaptive checks without a tolerance.  ERR_STATE: PSF, data or blocks not
 * set.  ERR_NOT_CONVERGED: grad_rtol > 0 and not reached (state still
 * valid). */
#define BD3MG_CHECK_ADAPTIVE (-1)
bd3mg_status bd3mg_run(bd3mg_problem p, int max_sweeps, double grad_rtol, int check_every,
                       bd3mg_result *res);

/* bd3mg_run for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, hosts that forbid hipMalloc): the same
 * sweeps with the same kernels, but no call of hipMalloc, hipFree or any
 * allocating routine.  Its partial sums, per-block coefficients, stop-test
 * control block and stored directions H d1, H d2 come from a fixed scratch
 * array of 64 MiB per GPU, held from the library's first use on that GPU until
 * the process ends; the problem's own buffers of these are left untouched.
 * Needed: 2 (n_c + 2 r_z b_c) nx ny slices of the storage type for the
 * stored directions of the largest launch group (see bd3mg_set_blocks), plus
 * the partial sums (about 0.2 % of a slice each per work item); a problem
 * needing more than 64 MiB is refused with ERR_ARG and the needed size in
 * bd3mg_last_error().  Every call on one GPU shares that GPU's array: calls
 * that overlap in time on one GPU (any problems, any streams) race and must
 * be ordered by the caller.  The stop-test control block is cleared at the
 * start of every call; every other part is written before it is read.
 * Differences from bd3mg_run: both directions are blurred every sweep (no
 * H dp is kept, as with BD3MG_OPT_HDP_EVERY = 0, whose bd3mg_run it equals
 * bitwise); a passing check is confirmed on q rebuilt in place from x (then
 * kept), and res->f is formed from q rebuilt in place; profiling is not
 * recorded.  Needs the separable PSF and a built schedule
 * (bd3mg_get_schedule, bd3mg_run or bd3mg_eval after the last change of
 * blocks or PSF): ERR_STATE otherwise, as for a missing PSF, data or
 * blocks.  x^0 = y, the reference norm ||grad f(y)|| and q are formed in
 * place when not yet current. */
bd3mg_status bd3mg_run_noalloc(bd3mg_problem p, int max_sweeps, double grad_rtol, int check_every,
                               bd3mg_result *res);

/* Copy the current iterate out (storage type). */
bd3mg_status bd3mg_get_x(bd3mg_problem p, void *x, int on_device);

/* Copy the previous-step volume (each block's last step on its own slices). */
bd3mg_status bd3mg_get_dprev(bd3mg_problem p, void *d, int on_device);

/* Checkpoint: copy out the whole solver state -- iterate x, previous steps
 * dprev, maintained blurred residual q (see bd3mg_run; volumes of the storage
 * type, any may be NULL) and the number of sweeps done since x^0 (may be
 * NULL). */
bd3mg_status bd3mg_get_state(bd3mg_problem p, void *x, void *dprev, void *q, long long *sweeps,
                             int on_device);

/* Resume: restore a state saved with bd3mg_get_state.  With q == NULL the
 * blurred residual is recomputed from x (equal up to rounding, not bitwise).
 * H dp (BD3MG_OPT_HDP_EVERY) is not part of the state: the first sweep after
 * a resume blurs both directions, so the resumed run equals the uninterrupted
 * one bitwise only with BD3MG_OPT_HDP_EVERY = 0 (else up to rounding). */
bd3mg_status bd3mg_set_state(bd3mg_problem p, const void *x, const void *dprev, const void *q,
                             long long sweeps, int on_device);

/* f(x) and ||grad f(x)|| at the current iterate, recomputing the blurred
 * residual q from x first.  Either pointer may be NULL. */
bd3mg_status bd3mg_eval(bd3mg_problem p, double *f, double *grad_norm);

/* Apply one operator of the criterion to a volume: BD3MG_OP_H (H in),
 * BD3MG_OP_HT (H^T in), BD3MG_OP_GRAD (grad f at in; needs the data).  Uses
 * the kernels of the solver.  in and out must not overlap. */
bd3mg_status bd3mg_apply(bd3mg_problem p, int op, const void *in, void *out, int on_device);

/* One block update (worker step and master update, Sec. 2.3) of block b
 * alone, from the current state; info (may be NULL) receives
 * {B11, B12, B22, c1, c2, u1, u2, ||g_S||^2} of the 2x2 subspace system. */
bd3mg_status bd3mg_block_step(bd3mg_problem p, int block, double *info);

/* Tunables (bd3mg_option).  BD3MG_OPT_REFRESH_EVERY: recompute the blurred
 * residual q from x after every that many sweeps (counted from x^0; 0 =
 * never; default 0 for FP64, 64 for FP32), bounding the drift of the
 * incrementally updated q.  BD3MG_OPT_PROFILE: 1 records HIP events around
 * every kernel launch of bd3mg_run on the problem's stream (0 = off). */
typedef enum {
    BD3MG_OPT_REFRESH_EVERY = 0,
    BD3MG_OPT_PROFILE = 1,
    /* Tile height (rows of a 64-column workgroup tile: 16 or 32; FP64 takes 16
     * only) of the direction pass, the update pass, and the whole-volume H and
     * adjoint-blur passes.  Taller tiles recompute less halo; shorter tiles give
     * more workgroups.  Defaults: 32 for FP32, 16 for FP64.  Results are
     * bitwise reproducible for a fixed setting; changing it changes the order
     * of the partial sums (rounding only). */
    BD3MG_OPT_TILE_ROWS_DIRS = 2,
    BD3MG_OPT_TILE_ROWS_UPDATE = 3,
    BD3MG_OPT_TILE_ROWS_AUX = 4,
    /* Output slices per workgroup of the direction pass: 1, 2 (consecutive
     * slices of a block share the reads of their common source slices), or 0
     * (the default: 2 for a launch group with at least 2^20 direction output
     * voxels, else 1).  Results are bitwise the same for every setting. */
    BD3MG_OPT_DIRS_SLICES = 5,
    /* Keeping H dp (Sec. 2.3, Worker: the subspace is [-grad, d_prev], so its
     * second image H d2 = H d_prev is the H d' the block's previous visit
     * formed).  n >= 1 (default 64): the update pass stores each block's
     * H d' = u1 H d1 + u2 H d2 for the block's next visit, whose direction
     * pass then blurs d1 = -grad only; every n-th sweep blurs both directions
     * again, bounding the rounding the recurrence carries (n = 1: always).
     * 0: both directions every sweep, nothing kept.  Applies to bd3mg_run
     * and batches with the separable PSF and a method other than Async-MM;
     * bd3mg_run_noalloc and bd3mg_block_step blur both directions.  Costs two
     * volumes of sum over blocks of |S +- r_z| slices, allocated at the first
     * run (without them, both directions are blurred).  Results differ from
     * n = 0 by rounding only. */
    BD3MG_OPT_HDP_EVERY = 6,
    /* Guard of the asynchronous rounds (BD3MG_SCHED_ROUND), m >= 1 sweeps
     * (0, the default: none).  Rounds below the inflation of Assumption C
     * (Sec. 2.5) are not guaranteed to converge.  With the guard, bd3mg_run
     * evaluates f at its start and after every m sweeps (at the end of a
     * run's chunk of sweeps); when f rose above the last accepted value by
     * more than the storage precision's rounding (4e-9 relative in FP32,
     * 1e-13 in FP64), x, every block's previous step and q go back to the
     * last accepted state and the inflation mu is raised (doubled, at least
     * L / 16, at most L (2 sqrt(tau) + 1) with L from bd3mg_lipschitz_bound
     * and tau = nblocks - 1, where Assumption C holds); otherwise the state
     * is accepted.  At the largest inflation every state is accepted.  The
     * raised mu stays with the problem (bd3mg_round_guard_info,
     * bd3mg_set_inflation).  res->sweeps counts every sweep run, discarded
     * ones included; the state's sweep count (bd3mg_get_state) only those
     * kept.  Costs three volumes, an evaluation of f (the blur of x and an
     * evaluation pass) and a copy of the state every m sweeps.  Other
     * schedules, batches and bd3mg_run_noalloc ignore it. */
    BD3MG_OPT_ROUND_GUARD = 7,
    /* Stores of the gradient and update passes' volume outputs (g, unless
     * the total variation is taken along z as well; x, the steps, q and the
     * kept H d' of a coloured or sequential sweep) with the non-temporal
     * cache hint: 1 on, 0 off, -1 (the default) on when one volume of the
     * problem holds at least 64 MiB.  A cache hint only: results are
     * bitwise the same for every setting. */
    BD3MG_OPT_STREAM_STORES = 8
} bd3mg_option;
bd3mg_status bd3mg_set_option(bd3mg_problem p, int option, long long value);

/* Autotuner: after `sweeps` warm-up sweeps at the current tiles, times
 * `sweeps` sweeps (after one more warm-up sweep) for every combination of tile
 * heights of the direction and update passes on this problem, twice (forward,
 * then reverse order), keeps the combination with the fastest of its two
 * times, and restores the solver state it started from
 * (x, previous steps, q, sweep count), so the call does not advance the
 * method.  chosen (may be NULL) receives {rows of the direction pass, rows of
 * the update pass}; ms (may be NULL) the best time per sweep in milliseconds.
 * ERR_STATE: PSF, data or blocks not set. */
bd3mg_status bd3mg_autotune(bd3mg_problem p, int sweeps, int *chosen, double *ms);

/* Kernel kinds reported by bd3mg_get_profile. */
typedef enum {
    BD3MG_K_GRAD = 0,    /* gradient pass of a colour of blocks */
    BD3MG_K_DIRS = 1,    /* direction pass (H d1, H d2, inner products) and the 2x2 solve */
    BD3MG_K_SOLVE = 2,   /* per-block 2x2 solve */
    BD3MG_K_UPDATE = 3,  /* update pass (x, dprev, r) */
    BD3MG_K_EVAL = 4,    /* whole-volume refresh of q and ||grad f|| checks */
    BD3MG_K_COUNT = 5
} bd3mg_kernel_kind;

/* Profile of the bd3mg_run calls made since profiling was switched on (or
 * since the last reset == 1): per kernel kind, the number of launches, their
 * summed device time in milliseconds (HIP events on the problem's stream) and
 * the summed algorithmic bytes -- the bytes each launch must move to or from
 * device memory by the method's definition, counting every element it reads
 * or writes once.  Arrays of BD3MG_K_COUNT entries; any may be NULL. */
bd3mg_status bd3mg_get_profile(bd3mg_problem p, long long *launches, double *ms, double *bytes,
                               int reset);

/* Attainable device-memory bandwidth: copies a buffer of the given size
 * (rounded down to 16 B) with a streaming copy kernel in four launch shapes
 * (1, 4 or 8 loads of 16 B in flight per lane; 8 to 32 workgroups per
 * compute unit), iters times each on the current device, and reports the
 * best launch as read + write bytes per second (*gbps, GB/s) and its
 * duration (*ms).  Allocates and frees its two buffers.  ERR_ARG: bytes <
 * 1 MiB or iters < 1. */
bd3mg_status bd3mg_probe_copy(size_t bytes, int iters, double *gbps, double *ms);

/* ---------------------------------------------------------------------------
 * Batches: many independent problems (own sizes, PSF, data, parameters and
 * block partitions) advanced together, two sweeps per HIP graph launch.
 * Fused launches (when every problem has the same precision, z extent,
 * in-slice radius and tile heights, the separable PSF, BD3MG's step and a
 * coloured or sequential schedule; see bd3mg_batch_set_mode for when they
 * are used): each pass of a colour index runs
 * once for all problems, its grid the concatenation of every problem's
 * work list (each problem as many workgroups as its own launch would have),
 * so a sweep of the whole batch is 4 x (most colours) launches; results are
 * bitwise those of the problems run one by one (each problem's direction
 * pass keeps H dp, or not, on the same sweeps as its single run).  Branch mode (or a batch
 * that cannot be fused): each problem's sweep is captured on its own stream
 * into the graph (fork/join), problems as parallel branches.
 * ------------------------------------------------------------------------- */
typedef struct bd3mg_batch_s *bd3mg_batch;

/* Group n problems (each fully set up: PSF, data, blocks) into a batch.  The
 * batch keeps the handles, which must outlive it and must not be run on their
 * own while it exists.  ERR_ARG: n < 1 or a NULL or repeated handle;
 * ERR_STATE: a problem not set up. */
bd3mg_status bd3mg_batch_create(int n, const bd3mg_problem *probs, bd3mg_batch *out);
bd3mg_status bd3mg_batch_destroy(bd3mg_batch b);

/* Tile heights for the batch: when it runs fused launches, bd3mg_autotune on
 * the largest problem, whose choice every problem of its precision then
 * takes (a fused launch has one tile height); with graph branches,
 * bd3mg_autotune on every problem. */
bd3mg_status bd3mg_batch_tune(bd3mg_batch b);

/* Batch mode: BD3MG_BATCH_AUTO (default: fused launches when the batch can
 * be fused and its volumes total at most 64 MiB of storage, graph branches
 * otherwise), BD3MG_BATCH_FUSED (whenever the batch can be fused) or
 * BD3MG_BATCH_BRANCHES.  Measured on one MI355X: 48 volumes of 64x64x32 run
 * 3x faster fused (every problem's launch alone is a few dozen workgroups);
 * 16 volumes of 128..256 x 128..256 x 32..96 (146 MB) run 1.6x faster as
 * branches (4 hardware queues run 4 problems at a time, whose data stays in
 * the caches, where a fused launch streams every problem's colour slab).
 * *fused (may be NULL) receives 1 when the batch will run fused launches as
 * it stands.  ERR_ARG: unknown mode. */
typedef enum { BD3MG_BATCH_AUTO = 0, BD3MG_BATCH_FUSED = 1, BD3MG_BATCH_BRANCHES = 2 } bd3mg_batch_mode;
bd3mg_status bd3mg_batch_set_mode(bd3mg_batch b, int mode, int *fused);

/* Advance every problem by max_sweeps sweeps (graph launches of two sweeps,
 * then one direct sweep when max_sweeps is odd).  With grad_rtol > 0 the
 * problems are checked every check_every sweeps (rounded up to an even
 * number); a converged problem stops and the graph is rebuilt for the rest.
 * results[n] (may be NULL) receive per-problem outcomes, f and ||grad f||
 * evaluated at the end.  ERR_NOT_CONVERGED when some problem missed the
 * tolerance (states still valid). */
bd3mg_status bd3mg_batch_run(bd3mg_batch b, int max_sweeps, double grad_rtol, int check_every,
                             bd3mg_result *results);


/* ---------------------------------------------------------------------------
 * Learned warm start (an addition to the paper's method, which starts from a
 * given x^0; Sec. 2.3 leaves the start point free).  A three-level 3D U-Net
 * maps the observation y to a start point x^0 = y + net(y) that is close to
 * the minimiser, so that BD3MG needs fewer sweeps to reach a tolerance.
 *
 * Network (base width c = 16, one input channel; every convolution 3x3x3 with
 * zero padding and a bias, followed by ReLU, except the head):
 *   a1 = conv(y; 1->c)     s1 = conv(a1; c->c)      p1 = avgpool2(s1)
 *   a2 = conv(p1; c->2c)   s2 = conv(a2; 2c->2c)    p2 = avgpool2(s2)
 *   a3 = conv(p2; 2c->4c)  b3 = conv(a3; 4c->4c)
 *   c2 = conv(up2(b3); 4c->2c)   e2 = conv([c2, s2]; 4c->2c)
 *   c1 = conv(up2(e2); 2c->c)    e1 = conv([c1, s1]; 2c->c)
 *   x0 = y + conv1x1(e1; c->1)   (no ReLU)
 * avgpool2 averages 2x2x2 cells, up2 repeats every voxel over a 2x2x2 cell,
 * [a, b] stacks channels.  Volume sides must be multiples of 4.
 *
 * Parameters: one float array, layer by layer in the order above, each layer
 * its weights [cout][cin][kd][kh][kw] followed by its bias [cout] (353,281
 * values for c = 16).  Arithmetic: activations and weights are stored as
 * bfloat16 (round to nearest even) and multiplied on the matrix cores with
 * float accumulation; biases, the head and its residual add are float; the
 * input y of the first layer is rounded to bfloat16, the residual uses y as
 * given.  Training: mean squared error of x0 against a target x*, averaged
 * over every voxel of the batch, and Adam (beta1 0.9, beta2 0.999, eps 1e-8)
 * on float master parameters.
 *
 * Batches of nb volumes are float arrays [nb][nz][ny][nx].  The handle owns
 * device buffers sized for the last batch shape it saw and reallocates them
 * when the shape changes.
 * ------------------------------------------------------------------------- */
typedef struct bd3mg_net_s *bd3mg_net;

/* levels must be 3, base_channels 16 and in_channels 1 (ERR_ARG otherwise).
 * The parameters start at zero (x0 = y) until set or loaded. */
bd3mg_status bd3mg_net_create(int levels, int base_channels, int in_channels, bd3mg_net *out);
bd3mg_status bd3mg_net_destroy(bd3mg_net n);
bd3mg_status bd3mg_net_num_params(bd3mg_net n, size_t *count);

/* Host arrays of exactly num_params floats.  set_params resets Adam.
 * ERR_ARG: wrong count or a non-finite value. */
bd3mg_status bd3mg_net_set_params(bd3mg_net n, const float *params, size_t count);
bd3mg_status bd3mg_net_get_params(bd3mg_net n, float *params, size_t count);

/* Serialised parameters: six uint32 (magic "BD3N", version 1, levels, base
 * channels, input channels, parameter count) followed by the float
 * parameters, little endian.  save with blob == NULL stores the size in
 * *bytes; otherwise *bytes is the capacity on entry and the size written on
 * return.  load checks the header against the handle (ERR_ARG on mismatch)
 * and resets Adam. */
bd3mg_status bd3mg_net_save(bd3mg_net n, void *blob, size_t *bytes);
bd3mg_status bd3mg_net_load(bd3mg_net n, const void *blob, size_t bytes);

/* x0 = y + net(y) for a batch of nb volumes (float, host or device). */
bd3mg_status bd3mg_net_forward(bd3mg_net n, int nb, int nx, int ny, int nz, const float *y,
                               float *x0, int on_device);

/* Start a problem from the network: like bd3mg_set_x0 with x0 = y + net(y),
 * y the problem's data (FP64 problems are rounded to float for the network
 * and the result widened back).  ERR_STATE: the problem has no data;
 * ERR_ARG: sides not multiples of 4. */
bd3mg_status bd3mg_net_infer(bd3mg_net n, bd3mg_problem p);

/* Loss (mean squared error of x0 against xstar) and its gradient with respect
 * to the parameters (host array of num_params floats, same layout), without
 * changing the parameters. */
bd3mg_status bd3mg_net_grad(bd3mg_net n, int nb, int nx, int ny, int nz, const float *y,
                            const float *xstar, int on_device, float *grad, double *loss);

/* One Adam step with learning rate lr on the batch (y, xstar).  *loss (may
 * be NULL) receives the loss before the step. */
bd3mg_status bd3mg_net_train_step(bd3mg_net n, int nb, int nx, int ny, int nz, const float *y,
                                  const float *xstar, int on_device, float lr, double *loss);

#ifdef __cplusplus
}
#endif

#endif /* BD3MG_H */
