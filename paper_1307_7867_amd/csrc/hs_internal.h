// Internal definitions shared by the device kernels and the host driver of
// libheatst.  Not part of the public C ABI (include/heatst.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define HS_MAXM 5          // collocation nodes per SDC level (3 and 5 are used)
#define HS_MAXLEV 3        // SDC levels of an MLSDC hierarchy
#define HS_MAXTAIL 5       // grids inside the single-workgroup coarse tail (15, 7, 3, 1)
#define HS_TAIL_N 15       // grids with n <= HS_TAIL_N are handled by the tail kernel
#define HS_BLOCK 512       // threads per block of the grid kernels (HS_TX x HS_TY)
#define HS_TX 64           // block tile along x (one wavefront per row)
#define HS_TY 8            // block tile along y
#define HS_TAIL_THREADS 1024
#define HS_ZB 8            // z planes per block of the z-marching stencil kernels

// Per-lane state in device memory.  A lane is one independent problem
// instance or one PFASST time slice.
struct LaneCtl {
    // parameters
    double nu, dt, t0, forcing_c;
    int32_t nsteps, step;        // requested / completed steps
    int32_t active, pad0;        // 1 = lane holds a live problem
    // coefficients of the current step, per SDC level
    double tn;
    double a[HS_MAXLEV][HS_MAXM];  // nu * dt_m (substep m)
    double g[HS_MAXLEV][HS_MAXM];  // forcing time factor -(sin t_j - c nu pi^2 cos t_j)
    double a_user;               // coefficient for stand-alone solves
    // control
    int32_t sdc_state;           // 0 iterate, 1 converged, 2 failed, 3 idle
    int32_t mg_state;            // 0 iterate, 1 converged, 2 failed, 3 idle
    int32_t mg_cycle;            // cycles of the current solve
    int32_t status;              // sticky hs_status of the lane
    uint32_t red_cnt[4];         // last-block counters of the reductions
    unsigned long long res_bits; // max-norm accumulators (bit patterns of
    unsigned long long bn_bits;  //  non-negative doubles order like integers)
    unsigned long long sdc_bits;
    double bnorm;                // |b|_inf of the current solve
    double mg_rho;               // last relative residual of a solve
    double sdc_res;              // last collocation residual
    // statistics
    long long total_cycles;
    int32_t total_solves, max_cycles, total_sweeps, sweeps_step;
    int32_t failed_solves;
    int32_t parent;              // node-parallel solver lane: its SDC lane, else -1
    long long level_cycles[HS_MAXLEV];  // cycles of the solves per SDC level
    // Every lane's state fills whole 256-byte blocks: lanes that kernels on
    // different streams update at the same time (PFASST slice groups) never
    // share a cache line.
    char pad_[72];
};
static_assert(sizeof(LaneCtl) % 256 == 0, "lane states must not share cache lines");

// One grid of one lane at one multigrid level.  The finest grid of an SDC
// solve lives inside the node array: its iterate is u + node * node_stride.
struct GridSeg {
    int32_t blk_begin;      // first block of this segment in its launch
    int32_t lane;
    int32_t n;              // interior points per axis
    int32_t nc;             // next coarser grid (0 if none)
    int32_t coarse;         // 1: correction grid whose first sweep starts from zero
    int32_t zb;             // z planes per block of the launch using this table
    int32_t moves;          // finest-grid tables: 1 if the grid lies above the coarse tail (its
                            // iterate changes buffer during a solve), else 0
    int32_t pad;
    long long node_stride;  // elements per node for the finest grid, else 0
    void* u;                // iterate
    void* t;                // ping-pong partner of u
    void* b;                // right-hand side
    void* cu;               // coarser grid's iterate (prolongation source)
    void* cb;               // coarser grid's right-hand side (restriction target)
};

// The coarse tail of one lane's hierarchy: every grid with n <= HS_TAIL_N,
// handled by one workgroup.  Level 0 of the tail may be the lane's finest
// grid (then it may carry a node stride and a non-zero initial guess).
struct TailSeg {
    int32_t lane;
    int32_t nlev;           // grids in the tail
    int32_t n[HS_MAXTAIL];
    int32_t coarse_table;   // LibConst::ct index of the exact solve on the last grid
    int32_t zero_guess;     // level 0 starts from zero (it is a correction grid)
    int32_t pad;
    long long node_stride;  // for level 0 only
    void* u[HS_MAXTAIL];
    void* t[HS_MAXTAIL];
    void* b[HS_MAXTAIL];
};

// Fields of one lane at one SDC level.
struct SdcSeg {
    int32_t blk_begin;
    int32_t lane;
    int32_t n;
    int32_t M;
    double* U;              // [M][N] node values
    double* FI;             // [M][N] nu L U at the nodes
    double* P;              // [M-1][N] sweep-constant part of the substep right-hand sides
    double* rhs;            // [N] right-hand side of the current solve
    double* Ut;             // [M][N] restricted fine values (coarse MLSDC level only)
    double* tau;            // [M][N] FAS correction (coarse MLSDC level only)
    const double* sig;      // [n] sin(pi (i+1) h)
    int32_t level;          // SDC level (0 fine, 1 coarse)
    int32_t pad;
};

// Fine/coarse pair of one lane for the FAS transfers.
struct FasSeg {
    int32_t blk_begin;
    int32_t lane;
    int32_t nf, nc;
    int32_t Mf, Mc;
    double *Uf, *FIf;             // fine [Mf][Nf]
    double *Uc, *FIc, *Ut, *tau;  // coarse [Mc][Nc]
    const double* sigf;
    const double* sigc;
    double* Ex;                   // tricubic transfer: [Mc][nc][nc][nf] x-interpolated corrections
    double* Exy;                  //   and [Mc][nc][nf][nf] xy-interpolated ones
    const double* tauf;           // the fine level's own FAS correction [Mf][Nf] (null on level 0)
    int32_t lf, pad;              // SDC level of the fine side (the coarse side is lf + 1)
};

// Exact solve on the coarsest grid (n = 3 or 1) by the discrete sine
// transform: x = S diag(1 / (1 - a (l_p + l_q + l_r))) S b with the
// orthonormal DST-I matrix S and the 1-D eigenvalues l of L_h.
struct CoarseTable {
    int32_t n;
    int32_t pad;
    double S[3][3];
    double lam[3];
};

// Collocation constants for M nodes, filled on the host.
struct SdcConst {
    int32_t M;
    int32_t pad;
    double tau[HS_MAXM];            // nodes on [0,1]
    double Q[HS_MAXM][HS_MAXM];     // Q[m][j] = int_0^tau_m l_j
    double S[HS_MAXM][HS_MAXM];     // S[m][j] = Q[m+1][j] - Q[m][j]
    double dtau[HS_MAXM];           // tau_{m+1} - tau_m
};

// Coarse-to-fine time interpolation for the FAS transfer (Mf, Mc nodes).
struct InterpConst {
    int32_t stride, pad;            // fine node of coarse node m is m * stride
    double w[HS_MAXM][HS_MAXM];     // w[mf][j] = l^c_j(tau^f_mf)
};

// Library-wide constants, identical for every plan: indexed by node count,
// by (fine, coarse) node counts and by (order, coarsest grid).
struct LibConst {
    SdcConst sdc[HS_MAXM + 1];
    InterpConst ip[HS_MAXM + 1][HS_MAXM + 1];
    CoarseTable ct[4];              // [(order == 4) * 2 + (n == 3)]
};

// ---------------------------------------------------------------------------
// Launch helpers implemented in hs_kernels.hip.  All return the hipError_t
// of the launch.  "nblk" is the total number of blocks of a segment table.
// ---------------------------------------------------------------------------
namespace hsk {

// Start / stop events of one timed launch (hipExtLaunchKernelGGL records the
// kernel's own start and end); both null = untimed.
struct EvPair {
    hipEvent_t start = nullptr, stop = nullptr;
};

struct MgArgs {
    int32_t L;         // SDC level whose coefficients apply
    int32_t m;         // substep (index into a[L][]); -1 = a_user
    double omega;
    int32_t node;      // node of the finest grid
    int32_t gate;      // 1 = skip lanes whose mg_state != 0; 2 (copy-back only) = skip lanes still solving
};

int grid_blocks(int n, int zb = 1);   // blocks covering an n^3 grid, zb planes per block
int choose_zb(int n);
int choose_zb_even(int n);   // even chunk length for resid_fw
int choose_zb_two(int n);    // chunk length for jac2                 // z planes per block of the plane-marching kernels
size_t tail_lds_bytes(int n0, int elem, int order);  // LDS of the tail kernel whose top grid is n0

hipError_t set_constants(const LibConst& lc);

// Source-buffer codes of the grid kernels: bit 0 picks t (else u) on the
// finest grids, bit 1 on the correction grids (GridSeg::coarse); bit 2
// (sweep only) leaves the correction grids untouched.  A table holds both
// kinds when its lanes have hierarchies of different depth.
inline int src_code(int finest_t, int coarse_t, int skip_coarse = 0)
{
    return (finest_t & 1) | ((coarse_t & 1) << 1) | (skip_coarse ? 4 : 0);
}

// Weighted-Jacobi sweep (mode 0) or residual r = b - A x written to the free
// buffer (mode 1) over a z-marching table.  norm 1 (finest grids, FP64): also
// write per-block maxima of |b - A x| (and |b| when cycle == 0) to partials;
// norm 2: first take the stopping test before cycle `cycle` (tol, max_cycles
// as mg_decide) from the maxima a norm-1 launch over the same table left, and
// sweep only the lanes that go on.
// src_is_t is a source-buffer code (src_code).  src (mode 0 only): 0 = x is
// the buffer the code picks; 1 = on correction grids x is the zero-guess
// first sweep omega D^{-1} b formed on the fly (finest grids as with 0).
template <typename T>
hipError_t sweep(LaneCtl* ctl, const GridSeg* segs, int nseg, int nblk, int order, MgArgs a,
                 int mode, int first_sweep, int src_is_t, int finest_only, int norm, int cycle,
                 double* partials, hipStream_t s, int src = 0, double tol = 0.0, int max_cycles = 0,
                 EvPair ev = {});

// Two weighted-Jacobi sweeps in one pass: dst = J(J(x)), x picked by
// src_is_t, dst the other buffer.  norm: per-block maxima of the first
// sweep's residual (and |b| when cycle == 0) to partials, as sweep does.
template <typename T>
hipError_t jac2(LaneCtl* ctl, const GridSeg* segs, int nseg, int nblk, int order, MgArgs a, int src_is_t,
                int norm, int cycle, double* partials, hipStream_t s);

// First post-smoothing sweep on x = u + P e: u picked by src_is_t, e the
// coarser grid's iterate (GridSeg::cu); the result goes to the other buffer.
template <typename T>
hipError_t pjac(LaneCtl* ctl, const GridSeg* segs, int nseg, int nblk, int order, MgArgs a, int src_is_t,
                hipStream_t s, EvPair ev = {});

// Copy the finest iterate from t back to u for the lanes whose grid moves
// (GridSeg::moves) and whose solve ran an odd number of V-cycles (when every
// cycle moves the iterate an odd number of times).  a.gate == 2: only lanes
// whose solve has stopped (issued before the host knows which have).
hipError_t mg_fixup(LaneCtl* ctl, const GridSeg* segs, int nseg, int nblk, MgArgs a, hipStream_t s);

// Residual b - A x (x picked by src_is_t) restricted by full weighting into
// GridSeg::cb in one pass; the table's chunks (zb) are even.
template <typename T>
hipError_t resid_fw(LaneCtl* ctl, const GridSeg* segs, int nseg, int nblk, int order, MgArgs a,
                    int src_is_t, hipStream_t s, EvPair ev = {});
template <typename T>
hipError_t prolong(LaneCtl* ctl, const GridSeg* segs, int nseg, int nblk, MgArgs a, int src_is_t,
                   int dst_is_t, hipStream_t s);
template <typename T>
hipError_t tail(LaneCtl* ctl, const TailSeg* segs, int nseg, int order, MgArgs a, int nu1, int nu2,
                size_t lds_bytes, hipStream_t s);

// stopping test of a solve from per-block maxima (one block per lane):
// rho = max|r| / max|b| (|b| taken at cycle 0); stop when rho <= tol, fail
// when cycle == max_cycles or rho is not finite
hipError_t mg_decide(LaneCtl* ctl, const GridSeg* segs, int nseg, int nblk, const double* partials,
                     int cycle, double tol, int max_cycles, int level, hipStream_t s);
// max-norm residual of an FP64 solve into partials (tables without a fused
// sweep); bit 0 of src_is_t: the iterate of grids with GridSeg::moves is in t
hipError_t mg_norm(LaneCtl* ctl, const GridSeg* segs, int nseg, int nblk, int order, MgArgs a,
                   int cycle, double* partials, int src_is_t, hipStream_t s);
// iterative refinement: r = b - A u in FP64, r32 = (float) r into the FP32
// hierarchy, per-block maxima into partials
hipError_t ir_resid(LaneCtl* ctl, const GridSeg* segs64, const GridSeg* segs32, int nseg, int nblk,
                    int order, MgArgs a, int iter, double* partials, hipStream_t s);
hipError_t ir_update(LaneCtl* ctl, const GridSeg* segs64, const GridSeg* segs32, int nseg,
                     int nblk, MgArgs a, hipStream_t s);

// SDC level kernels
hipError_t spread(LaneCtl* ctl, const SdcSeg* segs, int nseg, int nblk, int order, int src_node,
                  hipStream_t s);
hipError_t sweep_prep(LaneCtl* ctl, const SdcSeg* segs, int nseg, int nblk, int with_resid,
                      int gate, double* partials, hipStream_t s);
// SDC stopping test from the per-block maxima of sweep_prep / sdc_resid
hipError_t sdc_decide(LaneCtl* ctl, const SdcSeg* segs, int nseg, int nblk, const double* partials,
                      double sdc_tol, int max_sweeps, hipStream_t s);
hipError_t make_rhs(LaneCtl* ctl, const SdcSeg* segs, int nseg, int nblk, int m, int gate,
                    hipStream_t s);
// FI_m = nu L U_m at nodes m0..m1-1 (and rhs = U + P at node rhs_node, -1 for
// none) over the blocks of the lanes' finest-grid z-marching table gsegs; the
// SDC table ssegs holds the same lanes in the same order.  gate 1: lanes whose
// SDC iteration has stopped skip; gate 2: also lanes whose current solve is
// still running.
hipError_t fi_march(LaneCtl* ctl, const GridSeg* gsegs, const SdcSeg* ssegs, int nseg, int nblk, int order,
                    int m0, int m1, int rhs_node, int gate, hipStream_t s);
hipError_t sdc_resid(LaneCtl* ctl, const SdcSeg* segs, int nseg, int nblk, double* partials,
                     hipStream_t s);
hipError_t handoff(LaneCtl* ctl, const SdcSeg* dst, const SdcSeg* src, int nseg, int nblk,
                   int order, hipStream_t s);
hipError_t fas_restrict(LaneCtl* ctl, const FasSeg* segs, int nseg, int nblk, int corder, int gate,
                        hipStream_t s);
hipError_t fas_interp3(LaneCtl* ctl, const FasSeg* segs, int nseg, int nblk, int gate, hipStream_t s);
hipError_t fas_interp(LaneCtl* ctl, const FasSeg* segs, int nseg, int nblk, int gate,
                      hipStream_t s);

// lane bookkeeping
hipError_t begin_step(LaneCtl* ctl, int nlanes, int nlevels, const int* M, hipStream_t s);
hipError_t end_step(LaneCtl* ctl, int nlanes, hipStream_t s);
// lane states first .. first + nlanes - 1
hipError_t begin_solve(LaneCtl* ctl, int first, int nlanes, hipStream_t s);
hipError_t end_solve_fixed(LaneCtl* ctl, int first, int nlanes, int cycles, int level, hipStream_t s);
hipError_t begin_sweep(LaneCtl* ctl, int first, int nlanes, hipStream_t s);
hipError_t set_lane(LaneCtl* ctl, int lane, double nu, double dt, double t0, double forcing_c,
                    int nsteps, int active, hipStream_t s);
hipError_t set_a_user(LaneCtl* ctl, int lane, double a, hipStream_t s);
hipError_t copy(const double* src, double* dst, long long count, hipStream_t s);
hipError_t fill(double* dst, long long count, double v, hipStream_t s);
// lanes whose SDC state is "converged" go back to "iterate" (PFASST keeps
// every slice iterating until all of them meet the tolerance)
hipError_t sdc_reopen(LaneCtl* ctl, int nlanes, hipStream_t s);
// node-parallel SDC: solver lane (b, m) = nlanes + b (M - 1) + m - 1 solves
// node m of SDC lane b.  np_lanes: mode 0 makes them idle children of their
// lanes, mode 1 sets their a = nu (dt tau_m) for the current step.
hipError_t np_lanes(LaneCtl* ctl, int nlanes, int M, int mode, hipStream_t s);
// right-hand sides of the node-parallel sweep into SdcSeg::P (node m at
// P + (m-1) N): U_0 + dt sum_j Q_mj (FI_j + g_j s) - dt tau_m FI_m
hipError_t np_rhs(LaneCtl* ctl, const SdcSeg* segs, int nseg, int nblk, hipStream_t s);

// kernel-level calls of the public ABI on lane-major packed user arrays
hipError_t lap_apply(const GridSeg* segs, int nseg, int nblk, int order, double alpha, double beta,
                     const double* u, double* y, const long long* offs, hipStream_t s);
hipError_t heat_rhs(LaneCtl* ctl, const GridSeg* gsegs, const SdcSeg* ssegs, int nseg, int nblk, int order,
                    const double* u, const double* t, double* fi, double* fe,
                    const long long* offs, hipStream_t s);
// y = alpha B_h u + beta A_h u (compact pair) on `batch` packed n^3 grids
hipError_t compact_apply(int n, int batch, double alpha, double beta, const double* u, double* y, hipStream_t s);
// single-level SDC with the compact pair, one lane per launch; gate: skip
// the launch once the lane's solve has stopped
int compact_blocks(int n);
// mode 0 Jacobi, 1 residual, 2 substep rhs, 3 nu A, 4 norm partials, 5 Jacobi with
// the norm partials (see k_cmp)
hipError_t compact_op(int mode, int n, const double* src, double* dst, const double* b, const double* g2,
                      const LaneCtl* ctl, int lane, double dtau, double omega, double* partials, int gate,
                      hipStream_t s);
hipError_t compact_fw(int nf, const double* rf, double* bc, const LaneCtl* ctl, int lane, int gate, hipStream_t s);
// dst = src + P ec (dst may be src)
hipError_t compact_prolong(int nc, const double* ec, const double* src, double* dst, const LaneCtl* ctl, int lane,
                           int gate, hipStream_t s);
// first Jacobi sweep from a zero iterate: dst = omega b / D
hipError_t compact_zsweep(int n, const double* b, double* dst, const LaneCtl* ctl, int lane, double dtau,
                          double omega, int gate, hipStream_t s);
// the V-cycle below a top grid n0 <= HS_TAIL_N in one workgroup (LDS bytes: compact_tail_lds)
size_t compact_tail_lds(int n0, int n_coarsest);
hipError_t compact_tail(int n0, double* u, const double* b, int zero_guess, const LaneCtl* ctl, int lane, double dtau,
                        double omega, int nu1, int nu2, int n_coarsest, int gate, hipStream_t s);
hipError_t compact_quad(int n, int M, int m, const double* G, const double* base, double* dst, const double* sig,
                        const LaneCtl* ctl, int lane, int L, hipStream_t s);
// mode 0 solve norm, 1 / 2 SDC residual (set / max), 3 solve norm and stopping test before `cycle`
hipError_t compact_reduce(const double* partials, int nblk, LaneCtl* ctl, int lane, int mode, int cycle, double tol,
                          int max_cycles, hipStream_t s);
hipError_t compact_ctl(LaneCtl* ctl, int lane, int op, int cycles, int state, int level, int status, hipStream_t s);
// x = B_h^{-1} y exactly, through the sine basis (tab: the transposed DST-I
// matrix, then cos(pi (i+1) h)); t0, t1 scratch grids; x may be y
hipError_t compact_binv(int n, const double* tab, const double* y, double* x, double* t0, double* t1, hipStream_t s);

}  // namespace hsk
