/*
 * parareal.h -- C ABI of an MI355X (gfx950) library for Parareal and
 * asynchronous Parareal time integration of the heat equation
 *     du/dt = nu * Laplace(u)  on (0,1)^d, d = 1, 2, 3, u = 0 on the boundary,
 * following Magoules & Gbikpi-Benissan, "Asynchronous parareal time
 * discretization for partial differential equations" (arXiv 2110.10762).
 *
 * Problem statement (Section 3.1, equation (pde) and the time decomposition
 * [T_{i-1}, T_i], i = 1..N): the caller gives the PDE data (nu, zero Dirichlet
 * boundary), the initial value u0, the end time T and the number of slices N,
 * the choice of fine and coarse propagators, and the stopping threshold eps of
 * equation (thresh).  The library returns the slice-boundary values
 * lambda_i ~ u(T_i), i = 0..N.
 *
 * Discretisation: n interior points per dimension, h = 1/(n+1), zero ghost
 * values.  F = m explicit-Euler steps of the (2d+1)-point Laplacian with
 * m = max(1, ceil(dT/dt_nominal - 1e-9)), dT = T/N, dt = dT/m.  G = one
 * backward-Euler step of length dT (Thomas in 1D, conjugate gradients in 2D/3D).
 *
 * Memory: every double* is DEVICE memory on the handle's device, contiguous
 * FP64, C order with x fastest ([z][y][x]).  A state has n^d values; an
 * iterate lambda has (N+1) states, slice 0 first.  For a batch of problems
 * (pr_create with nproblems > 1) the per-problem arrays are concatenated in
 * problem order.  The caller owns all pointers it passes; the library owns its
 * workspace (allocated by pr_create or lazily by the first solve of a kind,
 * freed by pr_destroy) and never keeps a caller pointer after a call returns.
 *
 * Streams: all work is queued on the stream given to pr_create (NULL = the
 * null stream).  Calls return after their work has completed, because the
 * stop decisions and statistics are needed on the host.
 *
 * Errors: every int-returning call returns PR_OK (0) or a negative PR_E* code
 * and leaves a message for pr_last_error() (per thread).  No C++ exception
 * crosses the ABI.  A handle is not thread-safe; calls on one handle must not
 * overlap.
 */
#ifndef PARAREAL_H
#define PARAREAL_H

#ifdef __cplusplus
extern "C" {
#endif

#define PR_OK            0
#define PR_EINVAL       -1   /* bad argument (dimension, size, null pointer...) */
#define PR_EUNSTABLE    -2   /* explicit Euler unstable: r = nu*dt/h^2 > 1/(2d) */
#define PR_ENOMEM       -3   /* device allocation failed */
#define PR_EHIP         -4   /* HIP runtime error (message holds the HIP string) */
#define PR_ENOTCONV     -5   /* kmax reached before the threshold; outputs written */
#define PR_ENORESIDENT  -6   /* persistent teams cannot all be resident at once */
#define PR_ETIMEOUT     -7   /* a bounded device-side wait ran out; outputs invalid */

#define PR_COARSE_AUTO    0  /* Thomas in 1D, CG otherwise */
#define PR_COARSE_THOMAS  1  /* 1D only */
#define PR_COARSE_CG      2

/* Fine propagator F: m steps of length dt per slice (Section 3.1 leaves F
 * abstract; the paper's experiments use implicit schemes, Section 5.1). */
#define PR_FINE_EXPLICIT        0  /* explicit Euler, r = nu dt/h^2 <= 1/(2d) */
#define PR_FINE_BACKWARD_EULER  1  /* (I - r h^2 L) u' = u, any r */
#define PR_FINE_TRAPEZOIDAL     2  /* (I - r/2 h^2 L) u' = (I + r/2 h^2 L) u, any r */
/* Implicit steps are solved like G: Thomas (1D) or CG to cg_tol (2D/3D).  The
 * adjoint (pr_grad) and batched handles take explicit F only. */

typedef struct pr_problem pr_problem;   /* opaque, library-owned */

typedef struct pr_config {
    int    dim;          /* 1, 2 or 3 */
    int    n;            /* interior points per dimension, >= 1 */
    double nu;           /* diffusivity, > 0 */
    double T;            /* end time, > 0 */
    int    nslices;      /* N >= 1 (the paper's p) */
    double dt_nominal;   /* requested fine step, > 0 */
    int    coarse;       /* PR_COARSE_* */
    double cg_tol;       /* CG relative residual ||r||_2 <= tol ||b||_2; <= 0 means 1e-12 */
    int    cg_maxit;     /* <= 0 means 10*n + 100 */
    double eps;          /* stop when ||lambda^k - lambda^{k-1}||_inf < eps; <= 0: run kmax */
    int    kmax;         /* iteration cap; <= 0 or > N means N (finite termination) */
    int    tb_depth;     /* fine steps per HBM pass (temporal block depth); 0 = default
                            (2D: 14; 3D: 4 when a slice has more than one step, else 1) */
    int    tile_rows;    /* 2D/3D fine kernel: rows a wave owns; 2D: below 96 a register
                            strip (rows held at once), from 96 on a sliding window (rows
                            marched per segment, two rows per time level held), 1000: a
                            sliding window whose segment length is chosen at each launch to
                            fill the chip's wave slots in whole rounds; 3D of depth > 1: the
                            rows of the lane's column in the z march; 0 = default */
    int    coarse_increment; /* 0: G(new) - G(old) as written in eq. (pr) / Algorithm 2;
                                1: G applied to the change new - old (G is linear, Section 3.1),
                                CG from 0 to an absolute residual tol*||new||; an unchanged input
                                gives exactly 0.  Fewer CG iterations, same fixed point. */
    int    fine_xpts;    /* x points per lane of the fine kernel (2D/3D); 0 = default.  The
                            first shape matching every nonzero (tb_depth, tile_rows,
                            fine_xpts) is used; none matching is PR_EINVAL. */
    int    fine;         /* PR_FINE_*: the fine propagator's time stepping */
    int    cg_precond;   /* 2D CG (coarse solves): degree of its Chebyshev polynomial
                            preconditioner; 0 = default (6), -1 = none (plain CG).  The
                            preconditioner changes iterates at the tolerance level only. */
} pr_config;

/* Derived discretisation of one problem (read-only view). */
typedef struct pr_info {
    int    m;            /* fine steps per slice */
    double dt, dT, h;
    double r;            /* nu*dt/h^2 */
    double s;            /* nu*dT/h^2 */
    long long npts;      /* n^dim */
    long long offset;    /* index of this problem's lambda_0[0] in a concatenated iterate */
    int    tb_depth, tile_rows;   /* fine-kernel shape in use */
    int    xpts, sliding;         /* its x points per lane; 1 for a sliding window */
    int    cg_precond;            /* degree of the CG preconditioner in use (2D), 0 = none */
} pr_info;

typedef struct pr_stats {
    /* inputs (optional, caller-owned host arrays) */
    int    *k_per_slice;     /* [N] local iteration counts k_i (async) or NULL */
    double *deltas;          /* [deltas_cap] ||lambda^k - lambda^{k-1}||_inf per iteration, or NULL */
    int     deltas_cap;
    /* outputs */
    int    iters;            /* sync: k at stop; async: kappa = max_i k_i; fine: 0 */
    int    kappa;
    int    converged;        /* 1 if the threshold (or exactness) was reached */
    double last_delta;
    double wall_ms;          /* whole call, device events */
    double fine_ms;          /* time in fine-propagator kernels (sync) */
    double coarse_ms;        /* time in coarse sweeps (sync) */
    double fine_lups;        /* lattice-site updates performed by F */
    long long cg_iters;      /* total CG iterations */
    long long g_solves;      /* coarse solves performed */
    long long g_skipped;     /* coarse solves skipped (unchanged input) */
    double kernel_ms;        /* async: duration of the persistent launch (device events) */
    long long kernel_cg_iters;  /* async: CG iterations inside the persistent launch */
    long long kernel_updates;   /* async: local iterations (sum of k_i) */
    int    teams;            /* async: concurrent slice teams used */
    long long copy_retries;  /* async: predecessor copies redone (slot overwritten meanwhile) */
    long long idle_rounds;   /* async: team rounds with nothing to update */
    /* async: mean per team of the time its leader saw in each phase of its
       updates (fine propagation, predecessor copy, coarse solve, correction
       and publication) and of the whole launch; the rest is idle waiting */
    double team_fine_ms, team_copy_ms, team_coarse_ms, team_corr_ms, team_total_ms;
    long long fine_cg_iters; /* CG iterations of implicit fine steps (2D/3D) */
} pr_stats;

/* Asynchronous-driver options (Algorithm 2 emulated by persistent teams). */
#define PR_ASYNC_FREE    0   /* read the newest predecessor; tolerance stop */
#define PR_ASYNC_EXACT   1   /* run until the finite-termination cascade reaches slice N */
#define PR_ASYNC_REPLAY  2   /* read the versions a host schedule names (deterministic) */
#define PR_ASYNC_PIPELINED 3 /* Algorithm 1: the synchronous iteration with per-slice waits
                                instead of a barrier (update k of slice i waits for version
                                k+1 of slice i-1); stops at the first k whose change is below
                                eps, detected on the device; output = that iterate, the same
                                as pr_solve_sync's.  Keeps every version ((N+2)(N+1)
                                states). */

typedef struct pr_async_opts {
    int mode;                /* PR_ASYNC_* */
    int teams;               /* concurrent slice teams, each holding the slices that
                                slice_blocks assigns it and updating them in turn;
                                0 = automatic: one per slice in 1D and in REPLAY (which
                                needs it), four of two XCDs each in 2D, two of four XCDs
                                each in 3D */
    int max_local_iters;     /* cap on k_i (<= 0: 4*N + 16) */
    const int *schedule;     /* REPLAY: host array [N][max_local_iters]: predecessor
                                version read by slice i's k-th coarse solve (slice 1: 0) */
    const int *delay_spins;  /* optional host array [N]: extra busy-wait per local iteration
                                (emulates slow processors / late messages); NULL = none */
    double time_limit_s;     /* device-side wall-clock cap of one solve (<= 0: 120 s); the
                                launch stops and the call returns PR_ETIMEOUT past it */
    double latency_us;       /* emulated message latency: a published version becomes
                                readable by the successor this long after publication
                                (0 = none; at most 1e7) */
    int slice_blocks;        /* which slices a team holds: 1 = a contiguous block, 2 = every
                                teams-th slice; 0 = default (blocks) */
    /* Failure injection (FREE and EXACT modes; NULL = none).  Section 2.1's
       assumptions (every slice updates infinitely often, bounded delays)
       still hold under both, so the iteration reaches the same fixed point. */
    const int *drop_every;   /* optional host array [N]: slice i's update number j is
                                computed but not published (a lost message) when
                                drop_every[i] >= 2 divides j; 0 = never.  A slice whose
                                last value was lost does not idle: it updates again. */
    const int *reset_after;  /* optional host array [N], FREE mode only: slice i loses its
                                state once, before update reset_after[i] + 1, and starts
                                again from the initial guess (F from lambda_{i-1}^0,
                                w_old = lambda_i^0); < 0 = never */
} pr_async_opts;

/* Create a handle for one problem (nproblems == 1) or a batch of independent
 * problems solved in one persistent launch (nproblems > 1).  device: HIP
 * device ordinal; stream: hipStream_t or NULL.  Validates every config
 * (PR_EINVAL, PR_EUNSTABLE) and allocates the synchronous workspace. */
int  pr_create(const pr_config *cfgs, int nproblems, int device, void *stream,
               pr_problem **out);
void pr_destroy(pr_problem *h);
const char *pr_last_error(void);
int  pr_get_info(const pr_problem *h, int problem, pr_info *out);

/* Synchronous Parareal, equation (pr), with the slice guards of Algorithm 1
 * (slices already exact are not recomputed).  u0: [sum npts]; lambda_out:
 * [sum (N+1)*npts], the final iterate.  stats: NULL or an array of nproblems.
 * Returns PR_ENOTCONV if some problem hit kmax (< N) first. */
int  pr_solve_sync (pr_problem *h, const double *u0, double *lambda_out, pr_stats *stats);

/* Asynchronous Parareal, equation (apr) as Algorithm 2: one team of
 * workgroups per slice (or per group of slices), no grid-wide barrier; each
 * team publishes its iterate through versioned device slots and reads the
 * newest (or scheduled) predecessor version.  Single problem only. */
int  pr_set_async_options(pr_problem *h, const pr_async_opts *opts);
int  pr_solve_async(pr_problem *h, const double *u0, double *lambda_out, pr_stats *stats);

/* Serial fine integration lambda_i = F(lambda_{i-1}) (Section 3.1), the
 * fixed point both Parareal variants reach. */
int  pr_solve_fine (pr_problem *h, const double *u0, double *lambda_out, pr_stats *stats);

/* Adjoint of the fine integration for L = 1/2 ||u(T) - u_target||^2 given
 * the upstream gradient gT = dL/du(T) [npts] and slice-boundary checkpoints
 * lambda [(N+1)*npts] (the converged iterate).  Writes dL/du0 [npts] (device)
 * and dL/dnu (host scalar).  Forward states inside a slice are recomputed
 * from lambda_{i-1} with sub-checkpoints.  Single problem only. */
int  pr_grad(pr_problem *h, const double *lambda, const double *gT,
             double *dLdu0, double *dLdnu);

/* Kernel-level entry points (tests, microbenchmarks); single problem only.
 * pr_apply_fine: out[c] = steps explicit-Euler steps of in[c], c < count
 *   (steps <= 0 means m); in and out may not overlap.
 * pr_apply_coarse: out[c] = G(in[c]) for c < count; cg_iters (host, may be
 *   NULL) receives the total CG iterations. */
int  pr_apply_fine  (pr_problem *h, const double *in, double *out, int count, int steps);
int  pr_apply_coarse(pr_problem *h, const double *in, double *out, int count, long long *cg_iters);

/* Allocation-free variant of pr_apply_coarse, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  out[c] = G(in[c]), c < count, for the
 * problem *cfg (2D or 3D, CG; the same solver and launch as pr_apply_coarse,
 * hence the same bits), with no handle: every scratch buffer (CG vectors,
 * reduction slots, team counters) lives in a fixed device array of the
 * library, 48 MiB per device, held from the first call on a device until the
 * process ends.  A state may hold at most 2^20 points (n <= 1024 in 2D,
 * n <= 101 in 3D); larger states, 1D problems, aliasing or NULL buffers are
 * PR_EINVAL.  device: HIP ordinal; stream: hipStream_t or NULL; in, out:
 * count * n^dim doubles on that device, caller-owned; cg_iters (host, may be
 * NULL): total CG iterations.  Calls no allocating routine; returns after the
 * work has completed.  All calls on one device share the array: calls that
 * overlap on one device (two threads, two streams) race and must not be made. */
int  pr_apply_coarse_static(const pr_config *cfg, int device, void *stream, const double *in, double *out,
                            int count, long long *cg_iters);

/* Fine-kernel shape control (autotuner and tests): the supported shapes are
 * enumerated by index; pr_set_fine_shape selects one for a problem. */
int  pr_fine_shape_count(int dim);
/* Project autotuner: times every fine-kernel shape for this problem's state
 * size (problem >= 0: its N states and, separately, the single state of the
 * serial fine run; problem == -1: every grid side of a batch) over m steps,
 * `reps` timed runs each, and selects the fastest.  Results are cached per
 * process and, if the environment variable PR_TUNE_CACHE names a file, in
 * that file.  Outputs (may be NULL): the chosen depth / rows and its time. */
int  pr_autotune(pr_problem *h, int problem, int reps, int *tb_depth, int *tile_rows, int *xpts,
                 double *best_ms);
/* Batched handles: capture one iteration of the whole batch as a hipGraph
 * and replay it (enable = 1, the default) or launch it directly (0). */
int  pr_set_graph(pr_problem *h, int enable);
int  pr_fine_shape_get(int dim, int index, int *tb_depth, int *tile_rows, int *xpts, int *sliding);
/* first shape matching every given (> 0) parameter; PR_EINVAL if none */
int  pr_set_fine_shape(pr_problem *h, int problem, int tb_depth, int tile_rows, int xpts);

#ifdef __cplusplus
}
#endif
#endif /* PARAREAL_H */
