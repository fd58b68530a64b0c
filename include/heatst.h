/*
 * heatst.h -- C ABI of libheatst, an MI355X (gfx950) implementation of the
 * data-parallel hot path of the space-time heat solver of Speck, Ruprecht,
 * Emmett, Bolten and Krause, "A space-time parallel solver for the
 * three-dimensional heat equation" (arXiv 1307.7867).
 *
 * Problem (section 1, eqs. (1)-(4)): u_t = nu Lap(u) + f on [0,1]^3 with
 * u = 0 on the boundary and the manufactured forcing
 *     f(x,t) = -s(x) (sin t - c nu pi^2 cos t),  s(x) = prod_d sin(pi x_d).
 * The paper prints c = 1; its analytic solution u = s(x) cos t (eq. (4))
 * holds for c = 3 in three dimensions.  c is a parameter (forcing_c).
 *
 * Space (section 1, method of lines): n interior points per axis,
 * h = 1/(n+1), n = 2^k - 1, 1 <= n <= 511.  L_h is the 7-point
 * second-order stencil (order 2) or the wide 13-point fourth-order stencil
 * (order 4) with the odd reflection u(-h) = -u(h) beyond each wall.
 *
 * Time (section 1.1): spectral deferred corrections on M Gauss-Lobatto
 * nodes (M = 2..5; the paper uses 5 on the fine and 3 on the coarse
 * level) with IMEX-Euler sweeps (eq. (7)); the node-to-node integrals use
 * the collocation matrix of eq. (6); each implicit substep solves
 * (I - nu dt_m L_h) U_{m+1} = rhs by geometric multigrid (section 1.2);
 * two-level MLSDC couples the levels by the FAS correction; PFASST runs
 * MLSDC iterations on consecutive time slices.
 *
 * Memory and data layout.
 *   - Every field is a contiguous float64 array in [z][y][x] order (x
 *     fastest) of n^3 interior values; point (i,j,k) sits at
 *     x = ((i+1)h, (j+1)h, (k+1)h).
 *   - A "lane" is one independent problem instance or one PFASST time
 *     slice.  Multi-lane user arrays are lane-major: lane b's field starts
 *     at the sum of n_{b'}^3 over b' < b.
 *   - All device memory is owned by the caller: hs_workspace_bytes gives
 *     the exact size, hs_plan_bind hands it over.  The library never
 *     allocates device memory; its one static device array (8 MiB per GPU)
 *     serves hs_mg_solve_static only.  The plan object itself is host
 *     memory owned by the library (hs_plan_create / hs_plan_destroy).
 *   - Pointers named d_* are device pointers, h_* host pointers.
 *   - stream is a hipStream_t (NULL = default stream).  Every call is
 *     asynchronous on it unless documented otherwise.
 *
 * Errors.  Every call returns an hs_status.  Arguments are validated on the
 * host before anything is launched; an invalid call changes nothing.
 * Numerical failures (a solve that hits its cycle limit, a non-finite
 * residual) are recorded per lane and reported by hs_stats_read and by
 * the calls that synchronise.
 */
#ifndef HEATST_H
#define HEATST_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HS_OK = 0,
    HS_EINVAL = -1,      /* invalid argument or problem description */
    HS_ENOMEM = -2,      /* workspace too small / admission budget exhausted */
    HS_ENOCONV = -3,     /* a solve or the SDC iteration hit its iteration cap */
    HS_ENONFINITE = -4,  /* a residual became NaN or Inf */
    HS_EDEVICE = -5,     /* a HIP call failed */
    HS_ESTATE = -6,      /* call out of order (e.g. plan not bound) */
    HS_PENDING = 1       /* serving: request not finished yet */
} hs_status;

typedef enum { HS_FP64 = 0, HS_MIXED = 1 } hs_precision;

/*
 * Level order code of the compact fourth-order pair (hs_compact_apply):
 * the semi-discrete equation B_h u' = nu A_h u + B_h f and eqs. (6)-(7)
 * multiplied by B_h, each substep (B_h - a A_h) U = rhs solved by the
 * multigrid below with the compact operator on every grid (Jacobi diagonal
 * 1/2 + 4 a / h^2, exact sine-basis solve on the coarsest grid).  The SDC
 * residual is the B-weighted one, max over m of
 * |B U_0 + dt sum_j q_mj (nu A U_j + B f_j) - B U_m|.  With a second level
 * (order 2 or 4) the plan runs two-level MLSDC: the FAS restriction takes the
 * fine integral with f^I = B_h^{-1}(nu A_h U) (section 1.2 has B_h inverted
 * for the FAS correction; the inverse is exact, through the sine basis).
 * FP64 plans with nlevels 1 or 2, nslices 1, no node-parallel sweeps, no
 * lane memory; such a plan supports hs_set_state / hs_get_state, hs_step,
 * hs_solve, hs_begin_step, hs_sdc_sweep, hs_mlsdc_iter, hs_end_step,
 * hs_set_nodes with node values only, and the statistics, and rejects
 * hs_lap_apply, hs_heat_rhs, hs_mg_vcycle, hs_solve_graph, hs_fas_restrict,
 * hs_fas_interp and hs_set_nodes with d_FI on level 0 (HS_EINVAL).  Its lanes
 * run one after another.
 */
#define HS_ORDER_COMPACT (-4)

/* One SDC level: grid, Laplacian order, collocation nodes. */
typedef struct {
    int32_t n;        /* interior points per axis, 2^k - 1, 1..511 */
    int32_t order;    /* 2 or 4; level 0 also HS_ORDER_COMPACT */
    int32_t nnodes;   /* Gauss-Lobatto nodes incl. both ends, 2..5 */
} hs_level_desc;

/*
 * Multigrid for (I - a L_h) u = b (section 1.2 states only that a parallel
 * geometric multigrid method is used).  Components: same-order
 * rediscretisation on grids n -> (n-1)/2 down to n_coarsest, weighted
 * Jacobi, full weighting, trilinear prolongation, exact solve on the
 * coarsest grid, V(nu1,nu2) cycles.
 * Stopping (FP64): before every cycle rho = |b - A u|_inf / |b|_inf; stop
 * when rho <= tol, fail (HS_ENOCONV) after max_cycles cycles.  With
 * fixed_cycles > 0 exactly that many cycles run and no norm is taken.
 * HS_MIXED: FP64 iterative refinement around one FP32 V(inner_nu1,
 * inner_nu2) cycle per iteration; tol / max_cycles then apply to the
 * refinement iterations.
 */
typedef struct {
    int32_t nu1, nu2;        /* pre / post smoothing sweeps (nu1 >= 1) */
    double omega;            /* Jacobi weight (6/7) */
    int32_t n_coarsest;      /* 3 or 1 */
    double tol;              /* relative max-norm residual target */
    int32_t max_cycles;
    int32_t fixed_cycles;    /* > 0: exactly this many cycles */
    int32_t precision;       /* hs_precision */
    int32_t inner_nu1, inner_nu2;
    int32_t fused_sweeps;    /* 0 or 1: one smoothing sweep per pass over the grid; 2: the finest
                                grids' first two pre-smoothing sweeps in one pass (temporal
                                blocking; FP64, grids of 127^3 and up, nu1 >= 2; same results,
                                measured slower than two passes on MI355X at 127^3 and 255^3) */
    int32_t cycle_graphs;    /* 1: a tolerance-driven FP64 solve launches its first cycle from the
                                host and replays cycles 1..pred-1 and the stopping test at pred
                                (pred = the previous solve's cycle count at this node) as one HIP
                                graph, captured on first use per (lane set, level, node, pred);
                                later cycles are launched one by one.  0: every kernel is launched
                                from the host.  Same results; with ROCm 7 on MI355X the graph
                                replay measured slower (29.0 vs 27.8 ms per 127^3 MLSDC step). */
} hs_mg_desc;

typedef struct {
    double nu;               /* diffusion coefficient (0.1 in the paper) */
    double t0, dt;           /* start time, step size */
    double forcing_c;        /* c of the forcing: 3 consistent, 1 as printed, 0 for s(x) sin t */
    int32_t nsteps;
    int32_t nlevels;         /* 1 = SDC; 2 or 3 = MLSDC / PFASST (section 1.1: a hierarchy of
                                levels with fewer nodes and points, tied by the FAS correction) */
    hs_level_desc lev[3];    /* lev[0] finest .. lev[nlevels-1] coarsest: n_l = (n_{l-1} - 1)/2,
                                nnodes_{l-1} - 1 a multiple of nnodes_l - 1 */
    hs_mg_desc mg;
    int32_t sweeps;          /* fixed sweeps (SDC) / iterations (MLSDC, PFASST); 0 = until sdc_tol */
    double sdc_tol;          /* absolute max-norm collocation residual target */
    int32_t max_sweeps;
    int32_t batch;           /* lanes */
    int32_t nslices;         /* 1, or = batch for PFASST time slices */
    const int32_t* h_lane_n; /* NULL, or per-lane fine n (uneven batches, nlevels = 1) */
    int32_t pfasst_pred_sweeps; /* PFASST: coarse sweeps per slice of the serial coarse predictor
                                   run before the first iteration (0 = none); see hs_pfasst_run */
    int32_t lane_memory;     /* 0: every lane's fields live in the plan workspace; 1: each lane's
                                fields live in device memory of its own, bound to the lane with
                                hs_plan_bind_lane while it holds a problem (the serving core's
                                plans); nslices must be 1 */
    int32_t sdc_node_parallel; /* 1: node-parallel SDC sweeps (single level, not in the paper): the
                                implicit part of the sweep is the diagonal tau_m instead of the
                                implicit-Euler substeps, so every node's right-hand side comes from
                                the previous iterate, (I - nu dt tau_m L_h) U_m = U_0 + dt (QF)_m
                                - nu dt tau_m L_h U_m^old, and the M-1 solves of all lanes run as one
                                batched multigrid solve; same collocation fixed point (eq. (6)) */
    int32_t pfasst_groups;   /* PFASST with sweeps > 0: 0 or 1 runs every iteration's fine sweeps as
                                one batch, then the coarse pipeline; G >= 2 (dividing nslices)
                                splits the slices into G groups of consecutive slices whose fine
                                sweeps and coarse pipeline overlap (see hs_pfasst_run); same
                                results; two levels only */
    int32_t fas_interp;      /* MLSDC / PFASST: spatial transfer of the coarse correction to the
                                fine level (section 1.1 leaves it to the references): 0 or 1
                                trilinear, 3 tricubic (4-point Lagrange per axis, odd reflection
                                beyond the walls; a scratch of M_c n_c n_f (n_c + n_f) values per
                                lane) */
} hs_problem;

/* Per-lane statistics (hs_stats_read). */
typedef struct {
    int32_t status;          /* sticky hs_status of the lane */
    int32_t steps_done;
    int32_t total_sweeps;
    int32_t total_solves;
    int64_t total_cycles;    /* V-cycles (FP64) or refinement iterations (mixed) */
    int32_t max_cycles;      /* most cycles of one solve */
    int32_t failed_solves;
    double last_rho;         /* relative residual of the last solve */
    double last_sdc_res;     /* last collocation residual taken */
    int64_t level_cycles[3]; /* total_cycles split by SDC level (finest first) */
} hs_lane_stats;

typedef struct hs_plan hs_plan;

const char* hs_status_string(hs_status s);

/* Library version and the collocation data it uses: nodes tau[M] and the
 * matrix Q[M*M] of eq. (6) (row m = node, column j = source node). */
hs_status hs_collocation(int32_t M, double* h_tau, double* h_Q);

/* Exact number of workspace bytes a plan for *pb needs. */
hs_status hs_workspace_bytes(const hs_problem* pb, size_t* bytes);

/* Validate *pb and build the host-side plan (no device work). */
hs_status hs_plan_create(const hs_problem* pb, hs_plan** plan);

/* Lay the plan out in caller-owned device memory d_ws (>= the size from
 * hs_workspace_bytes, 256-byte aligned) and upload its tables.  Synchronous.
 * Every lane starts active with the problem's nu, dt, t0, nsteps. */
hs_status hs_plan_bind(hs_plan* plan, void* d_ws, size_t bytes, void* stream);

hs_status hs_plan_destroy(hs_plan* plan);

/* Plans with lane_memory = 1.  hs_lane_bytes: the device bytes lane `lane`
 * of a plan for *pb needs (fields, multigrid hierarchy).
 * hs_plan_bind_lane lays the (inactive) lane out in caller-owned d_mem
 * (256-byte aligned, at least hs_lane_bytes) -- synchronous;
 * hs_plan_unbind_lane releases an inactive lane's memory back to the caller.
 * A lane must be bound before hs_set_lane activates it.  Calls that work on
 * every lane at once (hs_lap_apply, hs_heat_rhs, hs_mg_vcycle, hs_smooth,
 * hs_set_state, hs_get_state, hs_get_nodes, hs_set_nodes, hs_solve_graph,
 * hs_pfasst_run) return HS_EINVAL on such plans; the step-level calls run
 * over the active lanes. */
hs_status hs_lane_bytes(const hs_problem* pb, int32_t lane, size_t* bytes);
hs_status hs_plan_bind_lane(hs_plan* plan, int32_t lane, void* d_mem, size_t bytes, void* stream);
hs_status hs_plan_unbind_lane(hs_plan* plan, int32_t lane);

/* Number of lanes and lane l's fine n (for sizing user arrays). */
hs_status hs_plan_lanes(const hs_plan* plan, int32_t* lanes, int32_t* h_lane_n);

/* Lane parameters (per-lane nu, dt, t0, steps; active = 0 frees the lane). */
hs_status hs_set_lane(hs_plan* plan, int32_t lane, double nu, double dt, double t0,
                      int32_t nsteps, int32_t active, void* stream);

/* Kernel-level calls (section 1, method of lines) on lane-major arrays of
 * SDC level `level`:
 *   hs_lap_apply: d_y = alpha d_u + beta L_h d_u
 *   hs_heat_rhs:  d_fi = nu_l L_h d_u and d_fe = f(x, h_t[l]) per lane l
 *                 (either output may be NULL). */
hs_status hs_lap_apply(hs_plan* plan, int32_t level, double alpha, double beta,
                       const double* d_u, double* d_y, void* stream);
hs_status hs_heat_rhs(hs_plan* plan, int32_t level, const double* d_u, const double* h_t,
                      double* d_fi, double* d_fe, void* stream);

/* The compact fourth-order pair of the fine level (section 1 names a
 * fourth-order compact stencil there, section 1.2 a weighting matrix that
 * the multigrid solver inverts for the FAS correction; neither is given, and
 * the reading is the 19-point Mehrstellen pair):
 *   d_y = alpha B_h d_u + beta A_h d_u,
 *   A_h u = (2 (sum of the 6 face neighbours) + (sum of the 12 edge
 *            neighbours) - 24 u) / (6 h^2),
 *   B_h u = u / 2 + (sum of the 6 face neighbours) / 12,
 * zero beyond the walls (eq. (2)), on `batch` grids of n^3 points packed
 * lane-major ([grid][z][y][x], caller-owned device memory; d_u and d_y must
 * not overlap).  alpha = 1, beta = -a gives the implicit operator B_h - a A_h.
 * Stateless (no plan).  HS_EINVAL unless n = 2^k - 1 <= 511, batch >= 1 and
 * both pointers are non-null.  Asynchronous on `stream`. */
hs_status hs_compact_apply(int32_t n, int32_t batch, double alpha, double beta, const double* d_u,
                           double* d_y, void* stream);

/* Multigrid solve (I - a_l L_h) u = b per lane l of SDC level `level` as
 * configured in the plan's hs_mg_desc, from the initial guess in d_u
 * (overwritten with the solution).  h_a: host array of per-lane a.
 * Synchronises; returns the worst lane status. */
hs_status hs_mg_vcycle(hs_plan* plan, int32_t level, const double* h_a, double* d_u,
                       const double* d_b, void* stream);

/* nsweeps weighted-Jacobi sweeps (the multigrid smoother, section 1.2)
 * u <- u + omega D^{-1} (b - (I - a_l L_h) u) on the finest grid of SDC
 * level `level`, in place on the lane-major d_u, with right-hand side d_b,
 * per-lane a from the host array h_a and d_tmp (same size as d_u) as the
 * ping-pong partner, which is left holding garbage.  Every sweep is one
 * launch of the same kernel the solver uses on its finest grids. */
hs_status hs_smooth(hs_plan* plan, int32_t level, const double* h_a, double* d_u,
                    const double* d_b, double* d_tmp, int32_t nsweeps, void* stream);

/* Allocation-free variant of hs_mg_vcycle for one grid, for callers that
 * cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation).  It solves
 * (I - a L_h) u = b on one n^3 grid of the given Laplacian order with the
 * multigrid of *mg, from the initial guess in d_u (overwritten with the
 * solution; d_b is only read), exactly as hs_mg_vcycle does on a one-lane
 * plan (same kernels, same stopping rule, same results).  No plan or
 * workspace: the coarse grids, the lane state, the segment tables and the
 * reduction partials live in a static device array of 8 MiB per GPU, which
 * the GPU holds from the first call until the process ends.  n must be at
 * most HS_STATIC_MAX_N (63), else HS_ENOMEM and nothing is launched;
 * mg->cycle_graphs must be 0 (HS_EINVAL).  The call allocates nothing on
 * the device or in pinned host memory and creates no stream or event; it
 * synchronises `stream` and returns the solve's status (HS_ENOCONV,
 * HS_ENONFINITE as hs_mg_vcycle).  Every call on one GPU uses that GPU's
 * array and re-initialises all of it that it reads: calls that overlap on
 * one GPU (other host threads, other streams) race and must be serialised
 * by the caller. */
#define HS_STATIC_MAX_N 63
hs_status hs_mg_solve_static(int32_t n, int32_t order, double a, const hs_mg_desc* mg, double* d_u,
                             const double* d_b, void* stream);

/* State (the value at the start of the next step) of every lane, lane-major
 * fine-level fields.  hs_set_state also resets the lanes' step counters.
 * For PFASST plans d_u0 holds one field that every slice starts from and
 * hs_get_state returns the end value of the last slice. */
hs_status hs_set_state(hs_plan* plan, const double* d_u0, void* stream);
hs_status hs_get_state(hs_plan* plan, double* d_u, void* stream);

/* One lane's state (fine-level field of n_lane^3 values): set before the
 * lane's first step (with hs_set_lane), read after its last. */
hs_status hs_set_lane_state(hs_plan* plan, int32_t lane, const double* d_u0, void* stream);
hs_status hs_get_lane_state(hs_plan* plan, int32_t lane, double* d_u, void* stream);

/* Node data of SDC level `level`: d_U and d_FI are lane-major [lane][M][N]
 * (FI = nu L_h U); d_Ut / d_tau (coarse level of an MLSDC plan) hold the
 * restricted fine values and the FAS correction.  Any pointer may be NULL. */
hs_status hs_get_nodes(hs_plan* plan, int32_t level, double* d_U, double* d_FI, double* d_Ut,
                       double* d_tau, void* stream);
hs_status hs_set_nodes(hs_plan* plan, int32_t level, const double* d_U, const double* d_FI,
                       void* stream);

/* Step-level calls, in the order a time step uses them:
 *   hs_begin_step : step coefficients, predictor (spread the state to all nodes)
 *   hs_sdc_sweep  : one IMEX SDC sweep of SDC level `level` (eq. (7)); on
 *                   the coarser levels of an MLSDC plan it includes tau
 *   hs_fas_restrict / hs_fas_interp : FAS transfer between levels 0 and 1
 *   hs_mlsdc_iter : one MLSDC iteration as a V-cycle over the levels (section
 *                   1.1): a sweep on level 0; per level, restriction + tau
 *                   (which carries the finer level's own tau below level 1)
 *                   and a sweep, down to the coarsest; on the way up,
 *                   interpolation to each level and, on a level between the
 *                   finest and the coarsest, another sweep; no closing sweep
 *                   on level 0.  Two levels: fine sweep, restriction + tau,
 *                   coarse sweep, interpolation.
 *   hs_end_step   : the last node becomes the state (eq. (9)). */
hs_status hs_begin_step(hs_plan* plan, void* stream);
hs_status hs_sdc_sweep(hs_plan* plan, int32_t level, void* stream);
hs_status hs_fas_restrict(hs_plan* plan, void* stream);
hs_status hs_fas_interp(hs_plan* plan, void* stream);
hs_status hs_mlsdc_iter(hs_plan* plan, void* stream);
hs_status hs_end_step(hs_plan* plan, void* stream);

/* One full step (fixed sweeps, or sweeps until sdc_tol) / all nsteps. */
hs_status hs_step(hs_plan* plan, void* stream);
hs_status hs_solve(hs_plan* plan, void* stream);

/* PFASST (section 1.1; nslices = batch = P, nlevels = 2 or 3): nsteps / P
 * blocks of P time slices.  Every slice starts from the block's initial
 * value spread over its nodes.  With pfasst_pred_sweeps > 0 a coarse
 * predictor runs first: the coarsest level goes serially through the slices
 * without the FAS correction (slice p starts from slice p-1's coarse end
 * value, spread, and does pfasst_pred_sweeps coarse sweeps), then every
 * slice interpolates its coarse correction level by level to the finest.
 * Each iteration: fine hand-off (slice p takes slice p-1's fine end value
 * of the previous iteration), fine sweeps of all slices as one batch, FAS
 * restriction level by level (three levels: with a batched sweep of the
 * middle level in between), the coarsest sweeps as a blocking pipeline
 * p = 0..P-1, interpolation level by level (three levels: with a batched
 * middle-level sweep in between); the middle level of a slice has no
 * hand-off of its own, its node 0 comes from the restriction.
 * sweeps > 0: that many iterations.  sweeps = 0: iterate until every
 * slice's collocation residual, taken after the hand-off, is <= sdc_tol
 * (the paper's PFASST threshold, section 2), at most max_sweeps
 * iterations (then the lanes report HS_ENOCONV).  The lanes' total_sweeps
 * count the iterations.  Synchronises once per iteration in the
 * tolerance mode.
 *
 * pfasst_groups = G >= 2 (fixed iterations, two levels): the same operations in a
 * pipelined order.  The slices form G groups of P/G consecutive slices;
 * the fine sweep of one group runs as one batch on `stream` while the
 * coarse pipeline of the group before it runs on a second stream of the
 * plan, issued by a second host thread, so the coarse sweeps of PFASST's
 * pipeline overlap the fine work as the paper's processors do (section
 * 1.1).  Every operation sees the data it sees in the order above: a
 * group's first slice takes its fine and coarse hand-offs from copies of
 * the previous group's end values made at the point the serial order reads
 * them.  The call returns once all work is issued on `stream` (the second
 * stream's work is ordered before the end of it); it is not reentrant for
 * one plan. */
hs_status hs_pfasst_run(hs_plan* plan, void* stream);

/* Launch timer, a measurement aid: with kind > 0 every launch of one kernel
 * of the multigrid cycles on the finest grids of SDC level 0 is bracketed by
 * HIP events that record the kernel's own start and end on the call's
 * stream (hipExtLaunchKernelGGL), up to max_launches launches; kind 0 turns
 * it off.  The events are created here (not inside timed work).
 * hs_plan_timer_read synchronises on the last event and returns the number
 * of timed launches and their summed duration in milliseconds, then starts
 * a new count.  Kinds (add HS_TIMER_FP32 for the FP32 inner cycles of mixed
 * precision solves): */
#define HS_TIMER_PJAC 1       /* prolongation + first post-smoothing sweep */
#define HS_TIMER_RESID_FW 2   /* residual + full-weighting restriction */
#define HS_TIMER_SWEEP1 3     /* first pre-smoothing sweep (with the residual norm in FP64 solves) */
#define HS_TIMER_SWEEP2 4     /* second pre-smoothing sweep (with the stopping test when folded in) */
#define HS_TIMER_FP32 16
hs_status hs_plan_timer(hs_plan* plan, int32_t kind, int32_t max_launches);
hs_status hs_plan_timer_read(hs_plan* plan, int32_t* launches, double* total_ms);

/* Launch-shape tuning.  The plane-marching kernels (sweeps, residual +
 * restriction, prolongation + sweep) give each block `zb` consecutive z
 * planes of a 64 x 8 tile; a grid's launch shape is chosen per grid size n,
 * Laplacian order, precision (0 FP64, 1 FP32) and batch (how many grids of
 * that size one launch covers).  Without an entry the built-in rule applies
 * (the largest zb of 8, 4, 2, 1 that still gives 256 blocks per grid).  An
 * entry matches the largest batch <= the launch's count, else the smallest
 * batch.  Entries apply to plans created afterwards; a process-wide table
 * guarded by a lock.
 *   hs_tune_set:    add or replace one entry (zb 1..64, zb_rfw even 2..64);
 *   hs_tune_clear:  remove every entry;
 *   hs_tune_load:   read entries from a JSON file written by the autotuner
 *                   (paper_1307_7867_amd/tune.py): an object whose "entries"
 *                   array holds objects with integer fields n, order,
 *                   precision, batch, zb, zb_rfw (other fields ignored);
 *                   returns the number of entries read;
 *   hs_tune_lookup: the zb / zb_rfw a plan created now would use. */
hs_status hs_tune_set(int32_t n, int32_t order, int32_t precision, int32_t batch, int32_t zb, int32_t zb_rfw);
hs_status hs_tune_clear(void);
hs_status hs_tune_load(const char* json_path, int32_t* entries);
hs_status hs_tune_lookup(int32_t n, int32_t order, int32_t precision, int32_t batch, int32_t* zb,
                         int32_t* zb_rfw);

/* Capture hs_step into a HIP graph and replay it for the remaining steps
 * (fixed sweep and cycle counts only). */
hs_status hs_solve_graph(hs_plan* plan, void* stream);

/* Per-lane statistics; synchronises the stream.  h_out has `batch` entries. */
hs_status hs_stats_read(hs_plan* plan, hs_lane_stats* h_out, void* stream);

/* ------------------------------------------------------------------------
 * Serving: a request loop for many independent heat solves.
 *
 * Requests (grid n, nu, dt, t0, steps, initial field) are grouped by grid
 * size into classes.  Every class is one batched plan with `slots` lanes
 * whose shared workspace (lane states, tables, partials) sits at the front
 * of the caller's device pool.  The rest of the pool is a heap: a request
 * is admitted -- given a free lane of its class and its own fields and
 * multigrid hierarchy carved from the heap -- while the bytes of all
 * admitted requests stay within hbm_budget minus the shared workspace.
 * Admission follows arrival order; the oldest request that a lane is free
 * for but whose bytes do not fit reserves them, so the requests behind it
 * may only use what is left (a large request is not starved by small ones,
 * which still fill the room it cannot use).
 * Each class is driven by its own host thread on its own HIP stream
 * (default priority): at every time-step boundary it binds the memory of
 * newly admitted requests to their lanes, advances all of its active lanes
 * by one step in one batched launch sequence, then retires the lanes that
 * are done (copying their final field to the request's output) and
 * returns their memory, which admits waiting requests.  New requests
 * therefore join at the next step boundary and different classes overlap
 * on the device.  Every lane takes its own stopping decisions, so a
 * request's result does not depend on what else is in the batch.
 * ---------------------------------------------------------------------- */
#define HS_MAX_CLASSES 8

typedef struct {
    int32_t order, nnodes;        /* Laplacian order and Lobatto nodes for every request */
    hs_mg_desc mg;
    int32_t sweeps;               /* 0 = sweep until sdc_tol */
    double sdc_tol;
    int32_t max_sweeps;
    double forcing_c;
    int32_t nclasses;
    int32_t class_n[HS_MAX_CLASSES];
    int32_t class_slots[HS_MAX_CLASSES];   /* lanes of the class's plan (most of its requests at once) */
} hs_server_desc;

typedef struct {
    int32_t state;                /* 0 queued, 1 admitted / running, 2 done */
    int32_t status;               /* hs_status of the finished request */
    int32_t cls, lane;
    double t_submit, t_admit, t_done;   /* seconds since the server was created */
    hs_lane_stats stats;
} hs_request_info;

typedef struct hs_server hs_server;

/* Device bytes of the classes' shared workspaces, and that plus every lane
 * of every class holding a request (the most the pool can usefully hold). */
hs_status hs_server_pool_bytes(const hs_server_desc* d, size_t* shared_bytes, size_t* full_bytes);
/* Heap bytes one request of grid n holds while admitted. */
hs_status hs_server_request_bytes(const hs_server_desc* d, int32_t n, size_t* bytes);
/* d_pool: caller-owned device memory (256-byte aligned).  HS_ENOMEM unless
 * both pool_bytes and hbm_budget hold the shared workspaces plus one
 * request of the largest class. */
hs_status hs_server_create(const hs_server_desc* d, void* d_pool, size_t pool_bytes,
                           size_t hbm_budget, hs_server** server);
/* Queue a request.  d_u0 (n^3 values) must stay valid until the request is
 * admitted; d_out (n^3 values) receives the final field.  HS_EINVAL if no
 * class has grid n. */
hs_status hs_server_submit(hs_server* s, int32_t n, double nu, double dt, double t0, int32_t nsteps,
                           const double* d_u0, double* d_out, uint64_t* ticket);
/* HS_OK when the request is done (info filled), HS_PENDING otherwise. */
hs_status hs_server_poll(hs_server* s, uint64_t ticket, hs_request_info* info);
/* Heap bytes the admitted requests hold now, and the most they may hold. */
hs_status hs_server_resident(hs_server* s, size_t* resident_bytes, size_t* budget_bytes);
/* Block until every submitted request is done. */
hs_status hs_server_drain(hs_server* s);
/* Stop: running requests finish, queued ones are dropped. */
hs_status hs_server_destroy(hs_server* s);

#ifdef __cplusplus
}
#endif

#endif /* HEATST_H */
