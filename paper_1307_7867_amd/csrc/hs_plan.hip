// Host driver of libheatst: plan layout in caller-owned device memory,
// segment tables, and the multigrid / SDC / MLSDC / PFASST drivers behind
// the C ABI of include/heatst.h.
#include "heatst.h"
#include "hs_internal.h"

#include <algorithm>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <type_traits>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <set>
#include <string>
#include <thread>
#include <vector>

namespace {

// ---------------------------------------------------------------------------
// Collocation data (section 1.1, eq. (6)), computed once on the host.
// ---------------------------------------------------------------------------

// Gauss-Lobatto nodes on [0,1] in closed form (M = 2..5).
void lobatto(int M, long double* t)
{
    const long double h = 0.5L;
    switch (M) {
    case 2: t[0] = 0; t[1] = 1; break;
    case 3: t[0] = 0; t[1] = h; t[2] = 1; break;
    case 4: {
        long double d = sqrtl(5.0L) / 10.0L;
        t[0] = 0; t[1] = h - d; t[2] = h + d; t[3] = 1;
        break;
    }
    default: {
        long double d = sqrtl(21.0L) / 14.0L;
        t[0] = 0; t[1] = h - d; t[2] = h; t[3] = h + d; t[4] = 1;
        break;
    }
    }
}

// Q[m][j] = int_0^{tau_m} l_j(s) ds by expanding l_j in monomials.
void collocation(int M, long double* t, long double Q[HS_MAXM][HS_MAXM])
{
    lobatto(M, t);
    for (int j = 0; j < M; j++) {
        long double c[HS_MAXM + 1] = {0};
        c[0] = 1.0L;
        int deg = 0;
        long double den = 1.0L;
        for (int i = 0; i < M; i++) {
            if (i == j) continue;
            // c(s) *= (s - t_i)
            for (int p = deg + 1; p >= 0; p--) {
                long double lo = p > 0 ? c[p - 1] : 0.0L;
                c[p] = lo - t[i] * c[p];
            }
            deg++;
            den *= (t[j] - t[i]);
        }
        for (int m = 0; m < M; m++) {
            long double s = 0.0L, pw = t[m];
            for (int p = 0; p <= deg; p++) {
                s += c[p] * pw / (long double)(p + 1);
                pw *= t[m];
            }
            Q[m][j] = s / den;
        }
    }
}

long double lagrange_at(int M, const long double* t, int j, long double s)
{
    long double v = 1.0L;
    for (int i = 0; i < M; i++)
        if (i != j) v *= (s - t[i]) / (t[j] - t[i]);
    return v;
}

LibConst make_libconst()
{
    LibConst lc;
    std::memset(&lc, 0, sizeof(lc));
    for (int M = 2; M <= HS_MAXM; M++) {
        long double t[HS_MAXM], Q[HS_MAXM][HS_MAXM];
        collocation(M, t, Q);
        SdcConst& K = lc.sdc[M];
        K.M = M;
        for (int m = 0; m < M; m++) {
            K.tau[m] = (double)t[m];
            for (int j = 0; j < M; j++) K.Q[m][j] = (double)Q[m][j];
        }
        for (int m = 0; m + 1 < M; m++) {
            K.dtau[m] = (double)(t[m + 1] - t[m]);
            for (int j = 0; j < M; j++) K.S[m][j] = (double)(Q[m + 1][j] - Q[m][j]);
        }
    }
    for (int Mf = 2; Mf <= HS_MAXM; Mf++)
        for (int Mc = 2; Mc <= Mf; Mc++) {
            if ((Mf - 1) % (Mc - 1) != 0) continue;
            long double tf[HS_MAXM], tc[HS_MAXM];
            lobatto(Mf, tf);
            lobatto(Mc, tc);
            InterpConst& ip = lc.ip[Mf][Mc];
            ip.stride = (Mf - 1) / (Mc - 1);
            for (int mf = 0; mf < Mf; mf++)
                for (int j = 0; j < Mc; j++) ip.w[mf][j] = (double)lagrange_at(Mc, tc, j, tf[mf]);
        }
    // exact coarsest solves by the sine transform, n = 1 and 3, orders 2 and 4
    const long double PI = 3.14159265358979323846264338327950288L;
    for (int o = 0; o < 2; o++)
        for (int three = 0; three < 2; three++) {
            CoarseTable& ct = lc.ct[o * 2 + three];
            int n = three ? 3 : 1;
            ct.n = n;
            long double h = 1.0L / (n + 1);
            for (int p = 0; p < n; p++) {
                for (int i = 0; i < n; i++)
                    ct.S[p][i] = (double)(sqrtl(2.0L / (n + 1)) * sinl(PI * (i + 1) * (p + 1) / (n + 1)));
                long double th = PI * (p + 1) * h;
                if (o == 0) ct.lam[p] = (double)(-4.0L / (h * h) * sinl(th / 2) * sinl(th / 2));
                else ct.lam[p] = (double)(-(30.0L - 32.0L * cosl(th) + 2.0L * cosl(2 * th)) / (12.0L * h * h));
            }
        }
    return lc;
}

std::mutex g_const_mu;
std::set<int> g_const_devices;

const LibConst& host_consts()
{
    static const LibConst lc = make_libconst();
    return lc;
}

hipError_t ensure_constants()
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(g_const_mu);
    if (g_const_devices.count(dev)) return hipSuccess;
    e = hsk::set_constants(host_consts());
    if (e == hipSuccess) g_const_devices.insert(dev);
    return e;
}

// ---------------------------------------------------------------------------
// Plan layout
// ---------------------------------------------------------------------------

bool valid_n(int n) { return n >= 1 && n <= 511 && ((n + 1) & n) == 0; }
long long cube(int n) { return (long long)n * n * n; }

struct Bump {
    char* base;   // nullptr while sizing
    size_t off = 0;
    explicit Bump(char* b) : base(b) {}
    size_t take(size_t bytes)
    {
        off = (off + 255) & ~(size_t)255;
        size_t r = off;
        off += bytes;
        return r;
    }
    void* ptr(size_t o) const { return base ? (void*)(base + o) : (void*)(uintptr_t)(o + 1); }
    template <class T> T* arr(size_t count) { return (T*)ptr(take(count * sizeof(T))); }
};

template <class S>
struct Table {
    std::vector<S> h;
    S* d = nullptr;
    int nblk = 0;
    int finest = 0;     // grid tables: every segment is a finest grid
    int coarse_all = 0; // grid tables: every segment is a correction grid (zero first guess)
    int max_seg_blocks = 0;  // grid tables: most blocks of one segment
    int nseg() const { return (int)h.size(); }
};

// multigrid tables of one SDC level, one precision, one set of lanes
struct MgSet {
    int D = 0;                            // down steps above the tail
    std::vector<Table<GridSeg>> jac, pro;      // z-marching sweeps, prolongation (and the
                                               // two-sweep kernel on the finest grids)
    std::vector<Table<GridSeg>> rfw;           // fused residual + restriction (even z chunks)
    Table<TailSeg> tail;
    size_t tail_lds = 0;                  // LDS bytes of the tail kernel
    Table<GridSeg> fine;                  // finest grids (norms, refinement), z-marching
    int fused_norm = 0;                   // jac[0] holds every lane's finest grid
    int uniform = 0;                      // every stage holds only finest or only correction grids
    int moves = 0;                        // some finest grid lies above the tail
    int two = 0;                          // the finest grids' first two sweeps run as one pass
};

struct LaneSet {
    std::vector<int> lanes;
    int first = 0, span = 0;                   // lanes[] lie in first .. first + span - 1
    MgSet mg64[HS_MAXLEV], mg32[HS_MAXLEV];
    Table<SdcSeg> sdc[HS_MAXLEV];
    Table<FasSeg> fasc[HS_MAXLEV - 1], fasf[HS_MAXLEV - 1];   // level l -> l + 1, by coarse / fine points
};

struct LaneBufs {
    int n[HS_MAXLEV] = {};
    long long N[HS_MAXLEV] = {};
    double *U[HS_MAXLEV] = {}, *FI[HS_MAXLEV] = {}, *P[HS_MAXLEV] = {}, *rhs[HS_MAXLEV] = {}, *tmp[HS_MAXLEV] = {};
    double *Ut[HS_MAXLEV] = {}, *tau[HS_MAXLEV] = {};   // levels >= 1: restricted values, FAS correction
    double *fx[HS_MAXLEV - 1] = {}, *fxy[HS_MAXLEV - 1] = {};   // tricubic FAS transfer l+1 -> l: x- and
                                                                // xy-interpolated coarse corrections
    const double* sig[HS_MAXLEV] = {};
    std::vector<int> grids[HS_MAXLEV];                 // n of every multigrid grid, finest first
    std::vector<double*> gu[HS_MAXLEV], gt[HS_MAXLEV], gb[HS_MAXLEV];  // FP64 grids (index 0 unused)
    std::vector<float*> fu[HS_MAXLEV], ft[HS_MAXLEV], fb[HS_MAXLEV];   // FP32 grids (mixed precision)
};

}  // namespace

struct hs_plan {
    hs_problem pb;
    std::vector<int> lane_n;
    int B = 0, nlev = 1;
    int nctl = 0;                              // lane states: B SDC lanes, then node-parallel solver lanes
    bool np = false;                           // node-parallel SDC sweeps (pb.sdc_node_parallel)
    int order[HS_MAXLEV] = {2, 2, 2}, M[HS_MAXLEV] = {3, 3, 3};
    bool compact = false;                      // the compact pair (single level); the multigrid
                                               // tables are then built for order 2 and not used
    std::vector<int> cmp_pred;                 // compact solves: last cycle count per lane and substep
    bool mixed = false;
    size_t bytes = 0;
    char* ws = nullptr;
    bool bound = false;
    int device = 0;
    LaneCtl* ctl = nullptr;
    LaneCtl* h_ctl = nullptr;                  // pinned copy for read-backs
    std::vector<LaneBufs> lanes;
    LaneSet all;
    LaneSet run;                               // the active lanes (what a step launches over)
    LaneSet np_set;                            // node-parallel solver lanes (multigrid tables only)
    std::vector<int> active;                   // host view of every lane's active flag
    bool run_dirty = true;
    // device storage for the run set's tables, room for every lane in each
    struct RunStore {
        std::vector<GridSeg*> grid[HS_MAXLEV][2];   // [level][fp32]: jac/pro/rfw per stage, then fine
        TailSeg* tail[HS_MAXLEV][2];
        SdcSeg* sdc[HS_MAXLEV];
        FasSeg *fasc[HS_MAXLEV - 1], *fasf[HS_MAXLEV - 1];
    } store;
    std::vector<LaneSet> single;               // PFASST coarse pipeline, one lane each
    Table<SdcSeg> hf_dst, hf_src;              // PFASST fine hand-off p-1 -> p
    std::vector<Table<SdcSeg>> hc_dst, hc_src; // PFASST coarse hand-off, per slice
    Table<long long> offs[HS_MAXLEV];          // lane-major packing offsets per SDC level
    Table<GridSeg> user;                       // hs_smooth on caller arrays
    double* partials = nullptr;                // per-block maxima of the reductions
    const void* user_key[3] = {nullptr, nullptr, nullptr};
    int user_level = -1;
    double* d_times = nullptr;                 // per-lane times for hs_heat_rhs
    // predicted cycles per (level, substep, iteration within the step): the
    // warm start improves from one iteration to the next, so the first
    // iteration of a step needs more cycles than the last one of the step before
    static constexpr int PRED_K = 4;
    int cpred[HS_MAXLEV][HS_MAXM][PRED_K];
    int sweep_k = 0;                           // iterations (fine sweeps) done in this step
    int cpred_user = 0;
    int state_ready = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    // Graphs of the predicted part of tolerance-driven solves: cycles 1..K-1
    // and the stopping test at K of one (lane set, level, substep, node).
    struct CycleGraph {
        const LaneSet* set;
        unsigned epoch;
        int L, m, node, K;
        int par;                               // finest grids' buffer after the K cycles
        hipGraphExec_t exec;
    };
    std::vector<CycleGraph> cgraphs;
    unsigned set_epoch = 0;                    // bumped when a lane set's tables change
    hipStream_t cap = nullptr;                 // capture stream (nothing runs on it)
    hipEvent_t ev_ctl = nullptr;               // marks the lane states' copy to h_ctl
    // stand-alone solve in caller arrays (hs_mg_solve_static): the finest grid's
    // iterate is ext_u (node 0) and its right-hand side ext_b; no node data
    bool solve_only = false;
    double* ext_u = nullptr;
    const double* ext_b = nullptr;
    // sine tables per grid size; lanes' own memory (pb.lane_memory)
    std::map<int, double*> sig;
    std::map<int, double*> dst_tab;            // compact MLSDC: transposed DST-I matrix + cosines per fine n
    std::vector<void*> lane_base;
    // launch timer (hs_plan_timer): start / stop event pairs of the timed kind
    int timer_kind = 0;
    std::vector<hipEvent_t> timer_ev;
    int timer_used = 0;
    // PFASST slice-group pipeline (pb.pfasst_groups = G >= 2): the lane sets of
    // the G groups of consecutive slices, the fine hand-off into each group's
    // slices, the coarse hand-off into a group's first slice, and the end
    // values of each group's last slice that those two read (fine after the
    // group's interpolation, coarse after its coarse sweeps)
    int G = 0;
    std::vector<LaneSet> grp;
    std::vector<Table<SdcSeg>> gh_dst, gh_src, gc_src;
    std::vector<double*> snap_f, snap_c;
    // the coarse sweeps run on a stream of their own, issued by a second host
    // thread with host-side state of its own (see issuer())
    hipStream_t pipe = nullptr;
    double* partials2 = nullptr;
    LaneCtl* h_ctl2 = nullptr;
    hipEvent_t ev_ctl2 = nullptr;
    int sweep_k2 = 0;
    std::vector<hipEvent_t> ev_r, ev_c;        // group's restriction / coarse sweeps recorded
    hipEvent_t ev_go = nullptr;                // block started
};

namespace {

hs_status dev_err(hipError_t e) { return e == hipSuccess ? HS_OK : HS_EDEVICE; }

#define HS_TRY(x)                                   \
    do {                                            \
        hipError_t e_ = (x);                        \
        if (e_ != hipSuccess) return HS_EDEVICE;    \
    } while (0)

#define HS_CHECK(x)                                 \
    do {                                            \
        hs_status s_ = (x);                         \
        if (s_ < 0) return s_;                      \
    } while (0)

std::vector<int> mg_grids(int n, int n_coarsest)
{
    std::vector<int> g{n};
    while (g.back() > n_coarsest && g.back() > 1) g.push_back((g.back() - 1) / 2);
    return g;
}

int tail_start(const std::vector<int>& g)
{
    int d = 0;
    while (d < (int)g.size() && g[d] > HS_TAIL_N) d++;
    return d;
}

int ct_index(int order, int n) { return (order == 4 ? 2 : 0) + (n == 3 ? 1 : 0); }

template <class S>
void finish_table(Table<S>& t, Bump& bump)
{
    t.d = t.h.empty() ? nullptr : bump.arr<S>(t.h.size());
}

// ---------------------------------------------------------------------------
// Launch-shape table (hs_tune_*): z planes per block of the plane-marching
// kernels for the grids of size n, Laplacian order and precision when one
// launch covers `batch` grids of that size.  Filled by the autotuner;
// without an entry the built-in rule (hsk::choose_zb) applies.
// ---------------------------------------------------------------------------
struct TuneEntry {
    int n, order, prec, batch, zb, zb_rfw;
};
std::mutex g_tune_mu;
std::vector<TuneEntry> g_tune;

// The entry of the largest batch <= count, else the one of the smallest batch.
void tuned_zb(int n, int order, int prec, int count, int* zb, int* zb_rfw)
{
    *zb = hsk::choose_zb(n);
    *zb_rfw = hsk::choose_zb_even(n);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    const TuneEntry* best = nullptr;
    for (const TuneEntry& e : g_tune) {
        if (e.n != n || e.order != order || e.prec != prec) continue;
        if (!best) best = &e;
        else if (e.batch <= count && (best->batch > count || e.batch > best->batch)) best = &e;
        else if (e.batch > count && best->batch > count && e.batch < best->batch) best = &e;
    }
    if (best) {
        *zb = best->zb;
        *zb_rfw = best->zb_rfw;
    }
}

bool valid_tune(int n, int order, int prec, int batch, int zb, int zb_rfw)
{
    return n >= 1 && n <= 511 && ((n + 1) & n) == 0 && (order == 2 || order == 4) && (prec == 0 || prec == 1) &&
           batch >= 1 && zb >= 1 && zb <= 64 && zb_rfw >= 2 && zb_rfw <= 64 && (zb_rfw & 1) == 0;
}

// Build the multigrid tables of SDC level L for the lanes of `ls`.
template <typename T>
void build_mg(hs_plan* P, LaneSet& ls, int L, bool fp32, MgSet& S)
{
    int Dmax = 0;
    for (int b : ls.lanes) Dmax = std::max(Dmax, tail_start(P->lanes[b].grids[L]));
    S.D = Dmax;
    S.jac.assign(Dmax, {});
    S.pro.assign(Dmax, {});
    S.rfw.assign(Dmax, {});
    auto grid_ptrs = [&](const LaneBufs& lb, int l, void** u, void** t, void** b) {
        if (fp32) {
            *u = lb.fu[L][l]; *t = lb.ft[L][l]; *b = lb.fb[L][l];
        } else if (l == 0) {
            *u = lb.U[L]; *t = lb.tmp[L]; *b = lb.rhs[L];
        } else {
            *u = lb.gu[L][l]; *t = lb.gt[L][l]; *b = lb.gb[L][l];
        }
    };
    const int prec = fp32 ? 1 : 0;
    for (int s = 0; s < Dmax; s++) {
        int bj = 0, bp = 0, bf2 = 0;
        std::map<int, int> count;   // grids of each size in this stage
        for (int b : ls.lanes) {
            const LaneBufs& lb = P->lanes[b];
            int l = s - (Dmax - tail_start(lb.grids[L]));
            if (l >= 0) count[lb.grids[L][l]]++;
        }
        for (int b : ls.lanes) {
            const LaneBufs& lb = P->lanes[b];
            int Db = tail_start(lb.grids[L]);
            int l = s - (Dmax - Db);
            if (l < 0) continue;
            GridSeg g;
            std::memset(&g, 0, sizeof(g));
            g.lane = b;
            g.n = lb.grids[L][l];
            g.nc = lb.grids[L][l + 1];
            g.coarse = (l > 0 || fp32) ? 1 : 0;
            g.node_stride = (l == 0 && !fp32) ? lb.N[L] : 0;
            grid_ptrs(lb, l, &g.u, &g.t, &g.b);
            void *cu, *ct, *cb;
            grid_ptrs(lb, l + 1, &cu, &ct, &cb);
            g.cu = cu;
            g.cb = cb;
            int zb, zb_rfw;
            tuned_zb(g.n, P->order[L], prec, count[g.n], &zb, &zb_rfw);
            g.zb = zb;
            g.blk_begin = bj; bj += hsk::grid_blocks(g.n, g.zb); S.jac[s].h.push_back(g);
            g.zb = hsk::choose_zb_two(g.n);   // also the two-sweep kernel's table
            g.blk_begin = bp; bp += hsk::grid_blocks(g.n, g.zb); S.pro[s].h.push_back(g);
            g.zb = zb_rfw;
            g.blk_begin = bf2; bf2 += hsk::grid_blocks(g.n, g.zb); S.rfw[s].h.push_back(g);
        }
        S.jac[s].nblk = bj;
        S.jac[s].finest = 1;
        S.jac[s].coarse_all = 1;
        for (const GridSeg& g : S.jac[s].h)
            S.jac[s].max_seg_blocks = std::max(S.jac[s].max_seg_blocks, hsk::grid_blocks(g.n, g.zb));
        for (const GridSeg& g : S.jac[s].h) {
            if (g.coarse) S.jac[s].finest = 0;
            else S.jac[s].coarse_all = 0;
        }
        S.pro[s].nblk = bp;
        S.rfw[s].nblk = bf2;
    }
    int bf = 0;
    std::map<int, int> fcount;   // finest grids of each size
    for (int b : ls.lanes) fcount[P->lanes[b].grids[L][0]]++;
    for (int b : ls.lanes) {
        const LaneBufs& lb = P->lanes[b];
        const std::vector<int>& g = lb.grids[L];
        int Db = tail_start(g);
        TailSeg ts;
        std::memset(&ts, 0, sizeof(ts));
        ts.lane = b;
        ts.nlev = (int)g.size() - Db;
        for (int q = 0; q < ts.nlev; q++) {
            void *u, *t, *bb;
            grid_ptrs(lb, Db + q, &u, &t, &bb);
            ts.n[q] = g[Db + q];
            ts.u[q] = u; ts.t[q] = t; ts.b[q] = bb;
        }
        ts.coarse_table = ct_index(P->order[L], g.back());
        S.tail_lds = std::max(S.tail_lds, hsk::tail_lds_bytes(g[Db], fp32 ? 4 : 8, P->order[L]));
        ts.zero_guess = (Db > 0 || fp32) ? 1 : 0;
        ts.node_stride = (Db == 0 && !fp32) ? lb.N[L] : 0;
        S.tail.h.push_back(ts);
        GridSeg f;
        std::memset(&f, 0, sizeof(f));
        f.lane = b;
        f.n = g[0];
        f.nc = g.size() > 1 ? g[1] : 0;
        f.coarse = fp32 ? 1 : 0;
        f.node_stride = fp32 ? 0 : lb.N[L];
        int zb_rfw_unused;
        tuned_zb(f.n, P->order[L], prec, fcount[f.n], &f.zb, &zb_rfw_unused);
        f.moves = (Db > 0 && !fp32) ? 1 : 0;
        S.moves |= f.moves;
        grid_ptrs(lb, 0, &f.u, &f.t, &f.b);
        f.blk_begin = bf;
        bf += hsk::grid_blocks(f.n, f.zb);
        S.fine.h.push_back(f);
    }
    S.fine.nblk = bf;
    S.fused_norm = (Dmax > 0 && S.jac[0].finest && S.jac[0].nseg() == (int)ls.lanes.size()) ? 1 : 0;
    S.uniform = 1;
    for (int s = 0; s < Dmax; s++)
        if (!S.jac[s].finest && !S.jac[s].coarse_all) S.uniform = 0;
    if (Dmax > 0 && !S.jac[0].coarse_all && !S.fused_norm) S.uniform = 0;
    // the finest grids' first two sweeps in one pass, when asked for (chunks
    // of 127^3 and larger grids are long enough for the extra planes it forms)
    S.two = (P->pb.mg.fused_sweeps == 2 && S.uniform && Dmax > 0 && !S.jac[0].coarse_all &&
             S.jac[0].h[0].n >= 127) ? 1 : 0;
}

SdcSeg sdc_seg(hs_plan* P, int b, int L)
{
    const LaneBufs& lb = P->lanes[b];
    SdcSeg s;
    std::memset(&s, 0, sizeof(s));
    s.lane = b;
    s.n = lb.n[L];
    s.M = P->M[L];
    s.U = lb.U[L]; s.FI = lb.FI[L]; s.P = lb.P[L]; s.rhs = lb.rhs[L];
    s.Ut = lb.Ut[L];
    s.tau = lb.tau[L];
    s.sig = lb.sig[L];
    s.level = L;
    return s;
}

// Host contents of every table of the lanes in ls.lanes.
void build_set_host(hs_plan* P, LaneSet& ls)
{
    ls.first = ls.lanes.empty() ? 0 : *std::min_element(ls.lanes.begin(), ls.lanes.end());
    ls.span = ls.lanes.empty() ? 0 : *std::max_element(ls.lanes.begin(), ls.lanes.end()) - ls.first + 1;
    for (int L = 0; L < P->nlev; L++) {
        int bk = 0;
        ls.sdc[L].h.clear();
        for (int b : ls.lanes) {
            SdcSeg s = sdc_seg(P, b, L);
            s.blk_begin = bk;
            bk += hsk::grid_blocks(s.n);
            ls.sdc[L].h.push_back(s);
        }
        ls.sdc[L].nblk = bk;
        ls.mg64[L] = MgSet();
        ls.mg32[L] = MgSet();
        build_mg<double>(P, ls, L, false, ls.mg64[L]);
        if (P->mixed) build_mg<float>(P, ls, L, true, ls.mg32[L]);
    }
    for (int l = 0; l + 1 < P->nlev; l++) {
        int bc = 0, bf = 0;
        ls.fasc[l].h.clear();
        ls.fasf[l].h.clear();
        for (int b : ls.lanes) {
            const LaneBufs& lb = P->lanes[b];
            FasSeg f;
            std::memset(&f, 0, sizeof(f));
            f.lane = b;
            f.lf = l;
            f.nf = lb.n[l]; f.nc = lb.n[l + 1];
            f.Mf = P->M[l]; f.Mc = P->M[l + 1];
            f.Uf = lb.U[l]; f.FIf = lb.FI[l]; f.tauf = lb.tau[l];
            f.Uc = lb.U[l + 1]; f.FIc = lb.FI[l + 1]; f.Ut = lb.Ut[l + 1]; f.tau = lb.tau[l + 1];
            f.sigf = lb.sig[l]; f.sigc = lb.sig[l + 1];
            f.Ex = lb.fx[l];
            f.Exy = lb.fxy[l];
            f.blk_begin = bc; bc += hsk::grid_blocks(f.nc); ls.fasc[l].h.push_back(f);
            f.blk_begin = bf; bf += hsk::grid_blocks(f.nf); ls.fasf[l].h.push_back(f);
        }
        ls.fasc[l].nblk = bc;
        ls.fasf[l].nblk = bf;
    }
}

void build_set(hs_plan* P, LaneSet& ls, Bump& bump)
{
    build_set_host(P, ls);
    // device storage of every table
    for (int L = 0; L < P->nlev; L++) {
        finish_table(ls.sdc[L], bump);
        for (MgSet* S : {&ls.mg64[L], &ls.mg32[L]}) {
            for (auto& t : S->jac) finish_table(t, bump);
            for (auto& t : S->pro) finish_table(t, bump);
            for (auto& t : S->rfw) finish_table(t, bump);
            finish_table(S->tail, bump);
            finish_table(S->fine, bump);
        }
    }
    for (int l = 0; l + 1 < P->nlev; l++) {
        finish_table(ls.fasc[l], bump);
        finish_table(ls.fasf[l], bump);
    }
}

// Lay out the whole workspace.  With base == nullptr only sizes are taken.
// One lane's fields (node data, right-hand side, ping-pong buffer, the
// multigrid hierarchy in FP64 and, for mixed precision, FP32) from `bump`.
void lay_lane(hs_plan* P, int b, Bump& bump)
{
    LaneBufs& lb = P->lanes[b];
    lb = LaneBufs();
    const hs_mg_desc& mg = P->pb.mg;
    for (int L = 0; L < P->nlev; L++) {
        int n = L == 0 ? P->lane_n[b] : (lb.n[L - 1] - 1) / 2;
        long long N = cube(n);
        int M = P->M[L];
        lb.n[L] = n;
        lb.N[L] = N;
        lb.sig[L] = P->sig[n];
        if (P->solve_only) {
            lb.U[L] = P->ext_u;
            lb.FI[L] = lb.P[L] = nullptr;
            lb.rhs[L] = const_cast<double*>(P->ext_b);   // read only: no kernel writes a finest rhs
        } else {
            lb.U[L] = bump.arr<double>(M * N);
            lb.FI[L] = bump.arr<double>(M * N);
            lb.P[L] = bump.arr<double>((M - 1) * N);
            lb.rhs[L] = bump.arr<double>(N);
        }
        lb.tmp[L] = bump.arr<double>(N);
        if (L >= 1) {
            lb.Ut[L] = bump.arr<double>(M * N);
            lb.tau[L] = bump.arr<double>(M * N);
        }
        lb.grids[L] = mg_grids(n, mg.n_coarsest);
        size_t G = lb.grids[L].size();
        lb.gu[L].assign(G, nullptr); lb.gt[L].assign(G, nullptr); lb.gb[L].assign(G, nullptr);
        lb.fu[L].assign(G, nullptr); lb.ft[L].assign(G, nullptr); lb.fb[L].assign(G, nullptr);
        for (size_t l = 0; l < G; l++) {
            long long Ng = cube(lb.grids[L][l]);
            if (l > 0) {
                lb.gu[L][l] = bump.arr<double>(Ng);
                lb.gt[L][l] = bump.arr<double>(Ng);
                lb.gb[L][l] = bump.arr<double>(Ng);
            }
            if (P->mixed) {
                lb.fu[L][l] = bump.arr<float>(Ng);
                lb.ft[L][l] = bump.arr<float>(Ng);
                lb.fb[L][l] = bump.arr<float>(Ng);
            }
        }
    }
    if (P->pb.fas_interp == 3)
        for (int l = 0; l + 1 < P->nlev; l++) {
            lb.fx[l] = bump.arr<double>((size_t)P->M[l + 1] * lb.n[l + 1] * lb.n[l + 1] * lb.n[l]);
            lb.fxy[l] = bump.arr<double>((size_t)P->M[l + 1] * lb.n[l + 1] * lb.n[l] * lb.n[l]);
        }
}

// Node-parallel solver lane sl = B + b (M-1) + m - 1: its finest grid is node m
// of SDC lane b (iterate U_m, right-hand side in b's P array at m - 1), with
// a ping-pong buffer and a multigrid hierarchy of its own.
void lay_np_lane(hs_plan* P, int sl, Bump& bump)
{
    const int M = P->M[0];
    const int b = (sl - P->B) / (M - 1), m = (sl - P->B) % (M - 1) + 1;
    const LaneBufs& pb = P->lanes[b];
    LaneBufs& lb = P->lanes[sl];
    lb = LaneBufs();
    const int n = pb.n[0];
    const long long N = pb.N[0];
    lb.n[0] = n;
    lb.N[0] = N;
    lb.sig[0] = pb.sig[0];
    lb.U[0] = pb.U[0] + m * N;
    lb.FI[0] = lb.P[0] = nullptr;
    lb.rhs[0] = pb.P[0] + (m - 1) * N;
    lb.tmp[0] = bump.arr<double>(N);
    lb.grids[0] = mg_grids(n, P->pb.mg.n_coarsest);
    size_t G = lb.grids[0].size();
    lb.gu[0].assign(G, nullptr); lb.gt[0].assign(G, nullptr); lb.gb[0].assign(G, nullptr);
    lb.fu[0].assign(G, nullptr); lb.ft[0].assign(G, nullptr); lb.fb[0].assign(G, nullptr);
    for (size_t l = 0; l < G; l++) {
        long long Ng = cube(lb.grids[0][l]);
        if (l > 0) {
            lb.gu[0][l] = bump.arr<double>(Ng);
            lb.gt[0][l] = bump.arr<double>(Ng);
            lb.gb[0][l] = bump.arr<double>(Ng);
        }
        if (P->mixed) {
            lb.fu[0][l] = bump.arr<float>(Ng);
            lb.ft[0][l] = bump.arr<float>(Ng);
            lb.fb[0][l] = bump.arr<float>(Ng);
        }
    }
}

// Bytes of lane b's fields when each lane lives in memory of its own.
size_t lane_bytes_of(hs_plan* P, int b)
{
    LaneBufs keep = P->lanes[b];
    Bump sizing(nullptr);
    lay_lane(P, b, sizing);
    P->lanes[b] = keep;
    return (sizing.off + 255) & ~(size_t)255;
}

// Lay out the whole workspace.  With base == nullptr only sizes are taken.
// Plans with lane memory of their own (pb.lane_memory) keep every lane's
// fields out of the workspace: a bound lane's come from its memory
// (hs_plan_bind_lane), an unbound lane's pointers are placeholders that no
// launch reads (only active lanes, which must be bound, are launched over).
void layout(hs_plan* P, char* base)
{
    Bump bump(base);
    P->ctl = bump.arr<LaneCtl>(P->nctl);
    // sine tables, one per distinct n
    P->sig.clear();
    for (int b = 0; b < P->B; b++)
        for (int L = 0, n = P->lane_n[b]; L < P->nlev; L++, n = (n - 1) / 2)
            if (!P->sig.count(n)) P->sig[n] = bump.arr<double>(n);
    P->dst_tab.clear();
    if (P->compact && P->nlev == 2)
        for (int b = 0; b < P->B; b++)
            if (!P->dst_tab.count(P->lane_n[b]))
                P->dst_tab[P->lane_n[b]] = bump.arr<double>((size_t)P->lane_n[b] * (P->lane_n[b] + 1));
    P->lanes.assign(P->nctl, LaneBufs());
    if (P->lane_base.size() != (size_t)P->B) P->lane_base.assign(P->B, nullptr);
    for (int b = 0; b < P->B; b++) {
        if (!P->pb.lane_memory) {
            lay_lane(P, b, bump);
        } else {
            Bump own((char*)P->lane_base[b]);
            lay_lane(P, b, own);
        }
    }
    for (int sl = P->B; sl < P->nctl; sl++) lay_np_lane(P, sl, bump);
    for (int L = 0; L < P->nlev; L++) {
        P->offs[L].h.assign(P->B, 0);
        long long o = 0;
        for (int b = 0; b < P->B; b++) {
            P->offs[L].h[b] = o;
            o += P->lanes[b].N[L];
        }
        finish_table(P->offs[L], bump);
    }
    P->d_times = bump.arr<double>(P->B);
    P->user.h.assign(P->B, GridSeg());
    finish_table(P->user, bump);
    P->user.h.clear();
    // lane sets
    P->all = LaneSet();
    for (int b = 0; b < P->B; b++) P->all.lanes.push_back(b);
    build_set(P, P->all, bump);
    P->np_set = LaneSet();
    if (P->np) {
        for (int sl = P->B; sl < P->nctl; sl++) P->np_set.lanes.push_back(sl);
        for (MgSet* S : {&P->np_set.mg64[0], &P->np_set.mg32[0]}) *S = MgSet();
        build_mg<double>(P, P->np_set, 0, false, P->np_set.mg64[0]);
        if (P->mixed) build_mg<float>(P, P->np_set, 0, true, P->np_set.mg32[0]);
        for (MgSet* S : {&P->np_set.mg64[0], &P->np_set.mg32[0]}) {
            for (auto& t : S->jac) finish_table(t, bump);
            for (auto& t : S->pro) finish_table(t, bump);
            for (auto& t : S->rfw) finish_table(t, bump);
            finish_table(S->tail, bump);
            finish_table(S->fine, bump);
        }
    }
    // run set storage: every table can hold all lanes
    for (int L = 0; L < P->nlev; L++) {
        for (int f = 0; f < 2; f++) {
            const MgSet& S = f ? P->all.mg32[L] : P->all.mg64[L];
            P->store.grid[L][f].clear();
            for (int t = 0; t < 3 * S.D + 1; t++) P->store.grid[L][f].push_back(bump.arr<GridSeg>(P->B));
            P->store.tail[L][f] = bump.arr<TailSeg>(P->B);
        }
        P->store.sdc[L] = bump.arr<SdcSeg>(P->B);
    }
    for (int l = 0; l + 1 < HS_MAXLEV; l++) {
        P->store.fasc[l] = l + 1 < P->nlev ? bump.arr<FasSeg>(P->B) : nullptr;
        P->store.fasf[l] = l + 1 < P->nlev ? bump.arr<FasSeg>(P->B) : nullptr;
    }
    P->active.assign(P->B, 1);
    P->run_dirty = true;
    P->single.clear();
    P->hf_dst = Table<SdcSeg>();
    P->hf_src = Table<SdcSeg>();
    P->hc_dst.clear();
    P->hc_src.clear();
    if (P->pb.nslices > 1) {
        P->single.resize(P->B);
        for (int b = 0; b < P->B; b++) {
            P->single[b].lanes = {b};
            build_set(P, P->single[b], bump);
        }
        int bk = 0;
        for (int p = 1; p < P->B; p++) {
            SdcSeg d = sdc_seg(P, p, 0), s = sdc_seg(P, p - 1, 0);
            d.blk_begin = s.blk_begin = bk;
            bk += hsk::grid_blocks(d.n);
            P->hf_dst.h.push_back(d);
            P->hf_src.h.push_back(s);
        }
        P->hf_dst.nblk = P->hf_src.nblk = bk;
        finish_table(P->hf_dst, bump);
        finish_table(P->hf_src, bump);
        P->hc_dst.resize(P->B);
        P->hc_src.resize(P->B);
        const int C = P->nlev - 1;   // the coarsest level runs the serial pipeline
        for (int p = 1; p < P->B; p++) {
            SdcSeg d = sdc_seg(P, p, C), s = sdc_seg(P, p - 1, C);
            d.blk_begin = s.blk_begin = 0;
            P->hc_dst[p].h.push_back(d);
            P->hc_src[p].h.push_back(s);
            P->hc_dst[p].nblk = P->hc_src[p].nblk = hsk::grid_blocks(d.n);
            finish_table(P->hc_dst[p], bump);
            finish_table(P->hc_src[p], bump);
        }
    }
    // PFASST slice groups: lane sets, snapshots of the last slices' end values,
    // and the hand-off tables that read them at the group boundaries
    P->grp.clear();
    P->gh_dst.clear();
    P->gh_src.clear();
    P->gc_src.clear();
    P->snap_f.clear();
    P->snap_c.clear();
    P->G = P->pb.nslices > 1 && P->pb.pfasst_groups >= 2 ? P->pb.pfasst_groups : 0;
    if (P->G) {
        const int G = P->G, Q = P->B / G;
        P->grp.resize(G);
        P->gh_dst.resize(G);
        P->gh_src.resize(G);
        P->gc_src.resize(G);
        for (int g = 0; g < G; g++) {
            for (int b = g * Q; b < (g + 1) * Q; b++) P->grp[g].lanes.push_back(b);
            build_set(P, P->grp[g], bump);
            if (g + 1 < G) {
                P->snap_f.push_back(bump.arr<double>((size_t)P->lanes[0].N[0]));
                P->snap_c.push_back(bump.arr<double>((size_t)P->lanes[0].N[1]));
            }
        }
        for (int g = 0; g < G; g++) {
            int bk = 0;
            for (int p = std::max(1, g * Q); p < (g + 1) * Q; p++) {
                SdcSeg d = sdc_seg(P, p, 0), src = sdc_seg(P, p - 1, 0);
                if (p == g * Q) {   // across the boundary: the snapshot, a single node
                    src.U = P->snap_f[g - 1];
                    src.M = 1;
                }
                d.blk_begin = src.blk_begin = bk;
                bk += hsk::grid_blocks(d.n);
                P->gh_dst[g].h.push_back(d);
                P->gh_src[g].h.push_back(src);
            }
            P->gh_dst[g].nblk = P->gh_src[g].nblk = bk;
            finish_table(P->gh_dst[g], bump);
            finish_table(P->gh_src[g], bump);
            if (g > 0) {
                SdcSeg src = sdc_seg(P, g * Q - 1, 1);
                src.U = P->snap_c[g - 1];
                src.M = 1;
                src.blk_begin = 0;
                P->gc_src[g].h.push_back(src);
                P->gc_src[g].nblk = hsk::grid_blocks(src.n);
                finish_table(P->gc_src[g], bump);
            }
        }
    }
    // per-block maxima of the reductions: two doubles per block of the largest launch
    int maxblk = 1;
    auto upd = [&](int nb) { maxblk = std::max(maxblk, nb); };
    auto scan = [&](const LaneSet& ls) {
        for (int L = 0; L < P->nlev; L++) {
            upd(ls.sdc[L].nblk);
            for (const MgSet* S : {&ls.mg64[L], &ls.mg32[L]}) {
                upd(S->fine.nblk);
                for (auto& t : S->jac) upd(t.nblk);
                for (auto& t : S->pro) upd(t.nblk);
            }
        }
    };
    scan(P->all);
    for (auto& ls : P->single) scan(ls);
    for (const MgSet* S : {&P->np_set.mg64[0], &P->np_set.mg32[0]}) {
        upd(S->fine.nblk);
        for (auto& t : S->jac) upd(t.nblk);
        for (auto& t : S->pro) upd(t.nblk);
    }
    for (auto& ls : P->grp) scan(ls);
    if (P->compact)   // norm launches of the compact path, one lane at a time
        for (int b = 0; b < P->B; b++) upd(hsk::compact_blocks(P->lane_n[b]));
    P->partials = bump.arr<double>(2 * (size_t)maxblk);
    P->partials2 = P->G ? bump.arr<double>(2 * (size_t)maxblk) : nullptr;
    P->bytes = (bump.off + 255) & ~(size_t)255;
}

template <class S>
hipError_t upload(const Table<S>& t, hipStream_t s)
{
    if (t.h.empty()) return hipSuccess;
    return hipMemcpyAsync(t.d, t.h.data(), t.h.size() * sizeof(S), hipMemcpyHostToDevice, s);
}

hipError_t upload_set(hs_plan* P, const LaneSet& ls, hipStream_t s)
{
    hipError_t e = hipSuccess;
    for (int L = 0; L < P->nlev; L++) {
        if ((e = upload(ls.sdc[L], s)) != hipSuccess) return e;
        for (const MgSet* S : {&ls.mg64[L], &ls.mg32[L]}) {
            for (auto& t : S->jac) if ((e = upload(t, s)) != hipSuccess) return e;
            for (auto& t : S->pro) if ((e = upload(t, s)) != hipSuccess) return e;
            for (auto& t : S->rfw) if ((e = upload(t, s)) != hipSuccess) return e;
            if ((e = upload(S->tail, s)) != hipSuccess) return e;
            if ((e = upload(S->fine, s)) != hipSuccess) return e;
        }
    }
    for (int l = 0; l + 1 < P->nlev; l++) {
        if ((e = upload(ls.fasc[l], s)) != hipSuccess) return e;
        if ((e = upload(ls.fasf[l], s)) != hipSuccess) return e;
    }
    return e;
}

hs_status validate(const hs_problem* pb)
{
    if (!pb) return HS_EINVAL;
    if (pb->nlevels < 1 || pb->nlevels > HS_MAXLEV) return HS_EINVAL;
    if (pb->batch < 1 || pb->batch > 4096) return HS_EINVAL;
    if (!(pb->nu > 0.0) || !(pb->dt > 0.0) || pb->nsteps < 0) return HS_EINVAL;
    if (!std::isfinite(pb->t0) || !std::isfinite(pb->forcing_c)) return HS_EINVAL;
    for (int L = 0; L < pb->nlevels; L++) {
        const hs_level_desc& d = pb->lev[L];
        if (d.order != 2 && d.order != 4 && !(d.order == HS_ORDER_COMPACT && L == 0)) return HS_EINVAL;
        if (d.nnodes < 2 || d.nnodes > HS_MAXM) return HS_EINVAL;
        if (L == 0 && !pb->h_lane_n && !valid_n(d.n)) return HS_EINVAL;
    }
    if (pb->h_lane_n) {
        if (pb->nlevels != 1) return HS_EINVAL;
        for (int b = 0; b < pb->batch; b++)
            if (!valid_n(pb->h_lane_n[b])) return HS_EINVAL;
    }
    for (int L = 1; L < pb->nlevels; L++) {
        const hs_level_desc &f = pb->lev[L - 1], &c = pb->lev[L];
        if (f.n < 3 || c.n != (f.n - 1) / 2) return HS_EINVAL;
        if ((f.nnodes - 1) % (c.nnodes - 1) != 0) return HS_EINVAL;
    }
    const hs_mg_desc& mg = pb->mg;
    if (mg.nu1 < 1 || mg.nu2 < 0 || mg.nu1 > 16 || mg.nu2 > 16) return HS_EINVAL;
    if (!(mg.omega > 0.0 && mg.omega <= 1.0)) return HS_EINVAL;
    if (mg.n_coarsest != 1 && mg.n_coarsest != 3) return HS_EINVAL;
    if (mg.precision != HS_FP64 && mg.precision != HS_MIXED) return HS_EINVAL;
    if (mg.fixed_cycles < 0 || mg.max_cycles < 0 || mg.max_cycles > 100000) return HS_EINVAL;
    if (mg.fixed_cycles == 0 && !(mg.tol > 0.0)) return HS_EINVAL;
    if (mg.precision == HS_MIXED && (mg.inner_nu1 < 1 || mg.inner_nu2 < 0)) return HS_EINVAL;
    if (mg.fused_sweeps < 0 || mg.fused_sweeps > 2) return HS_EINVAL;
    if (mg.cycle_graphs < 0 || mg.cycle_graphs > 1) return HS_EINVAL;
    if (pb->sweeps < 0 || pb->max_sweeps < 0) return HS_EINVAL;
    if (pb->sweeps == 0 && !(pb->sdc_tol > 0.0)) return HS_EINVAL;
    if (pb->nslices < 1) return HS_EINVAL;
    if (pb->pfasst_pred_sweeps < 0 || pb->pfasst_pred_sweeps > 64) return HS_EINVAL;
    if (pb->lane_memory != 0 && pb->lane_memory != 1) return HS_EINVAL;
    if (pb->sdc_node_parallel != 0 &&
        (pb->sdc_node_parallel != 1 || pb->nlevels != 1 || pb->nslices != 1 || pb->lane_memory))
        return HS_EINVAL;
    if (pb->lane_memory && pb->nslices != 1) return HS_EINVAL;
    if (pb->pfasst_groups < 0 || pb->pfasst_groups > pb->nslices) return HS_EINVAL;
    if (pb->fas_interp != 0 && pb->fas_interp != 1 && pb->fas_interp != 3) return HS_EINVAL;
    if (pb->pfasst_groups >= 2 &&
        (pb->nslices % pb->pfasst_groups != 0 || pb->sweeps <= 0 || pb->mg.cycle_graphs || pb->nlevels != 2))
        return HS_EINVAL;
    // the compact pair: FP64 SDC or two-level MLSDC, one lane after another
    if (pb->lev[0].order == HS_ORDER_COMPACT &&
        (pb->nlevels > 2 || pb->nslices != 1 || mg.precision != HS_FP64 || pb->sdc_node_parallel ||
         pb->lane_memory))
        return HS_EINVAL;
    if (pb->nslices > 1) {
        if (pb->nslices != pb->batch || pb->nlevels < 2) return HS_EINVAL;
        if (pb->nsteps % pb->nslices != 0) return HS_EINVAL;
    } else if (pb->pfasst_pred_sweeps != 0) {
        return HS_EINVAL;
    }
    return HS_OK;
}

// ---------------------------------------------------------------------------
// Host-side control: lane states are read back to decide when to stop
// issuing cycles / sweeps (tolerance mode only).
// ---------------------------------------------------------------------------

// Host-side state of the thread that issues work on stream s: the per-block
// maxima of the reductions, the pinned copy of the lane states with the event
// that marks it, and the iteration count that indexes the cycle predictions.
// The coarse sweeps of the PFASST pipeline are issued on P->pipe by a thread
// of their own; everything else runs on the caller's stream.
struct Issuer {
    double* partials;
    LaneCtl* h_ctl;
    hipEvent_t ev_ctl;
    int* sweep_k;
};

Issuer issuer(hs_plan* P, hipStream_t s)
{
    if (P->pipe && s == P->pipe) return {P->partials2, P->h_ctl2, P->ev_ctl2, &P->sweep_k2};
    return {P->partials, P->h_ctl, P->ev_ctl, &P->sweep_k};
}

// The range of lane states that holds the lanes of ls (all of them for a
// null set).  A read-back copies only that range, so a stream never reads the
// lane states that kernels on another stream are writing.
void ctl_range(const hs_plan* P, const LaneSet* ls, int* first, int* count)
{
    if (!ls || ls->lanes.empty()) {
        *first = 0;
        *count = P->nctl;
        return;
    }
    const auto mm = std::minmax_element(ls->lanes.begin(), ls->lanes.end());
    *first = *mm.first;
    *count = *mm.second - *mm.first + 1;
}

hipError_t copy_ctl(hs_plan* P, const LaneSet* ls, hipStream_t s)
{
    int first, count;
    ctl_range(P, ls, &first, &count);
    return hipMemcpyAsync(issuer(P, s).h_ctl + first, P->ctl + first, sizeof(LaneCtl) * count,
                          hipMemcpyDeviceToHost, s);
}

hs_status read_ctl(hs_plan* P, hipStream_t s, const LaneSet* ls = nullptr)
{
    HS_TRY(copy_ctl(P, ls, s));
    HS_TRY(hipStreamSynchronize(s));
    return HS_OK;
}

bool all_mg_done(hs_plan* P, const LaneSet& ls, int* maxc, hipStream_t s)
{
    const LaneCtl* h = issuer(P, s).h_ctl;
    bool done = true;
    int mc = 0;
    for (int b : ls.lanes) {
        const LaneCtl& c = h[b];
        if (c.mg_state == 0) done = false;
        else if (c.mg_state != 3) mc = std::max(mc, c.mg_cycle);
    }
    *maxc = mc;
    return done;
}

bool all_sdc_done(hs_plan* P, const LaneSet& ls, hipStream_t s)
{
    const LaneCtl* h = issuer(P, s).h_ctl;
    for (int b : ls.lanes)
        if (h[b].sdc_state == 0) return false;
    return true;
}

// Events for a launch of timer kind `kind` (HS_TIMER_*) on the finest grids of
// SDC level L in precision T; empty unless the plan times that kind on level
// 0 and has events left.
template <typename T>
hsk::EvPair timer_events(hs_plan* P, int kind, int L)
{
    hsk::EvPair e;
    const int want = kind | (std::is_same<T, float>::value ? HS_TIMER_FP32 : 0);
    if (P->timer_kind != want || L != 0 || 2 * (P->timer_used + 1) > (int)P->timer_ev.size()) return e;
    e.start = P->timer_ev[2 * P->timer_used];
    e.stop = P->timer_ev[2 * P->timer_used + 1];
    P->timer_used++;
    return e;
}

// One V(nu1, nu2) cycle over the grids above the tail (section 1.2).  Each
// grid keeps its iterate in one of two buffers (0 = u, 1 = t) and every sweep
// moves it to the other one.  Correction grids start from zero: their first
// sweep, omega D^{-1} b, is formed where the second sweep reads it instead of
// being stored, and their first write goes to the buffer that makes the cycle
// end in u, where the next finer grid's prolongation reads the correction.
// The residual is restricted in the same pass that forms it, and the
// prolongated correction is applied as the first post-smoothing sweep reads
// its input (nu2 >= 1).  The finest grids start in buffer *par and end in
// *par ^ (number of passes that wrote it), written back to *par.  When the
// lanes' hierarchies differ in depth a stage holds finest grids of some lanes
// and correction grids of others: each launch then picks the buffer per grid
// role, and the finest grids' first sweep runs alone so that both kinds
// reach their second sweep in the same launch.
// sweeps_done / passes_done: the finest grids' first sweeps that already ran
// with the residual norm (and the stopping test), and the passes they took.
// On grids with S.two the first two sweeps run as one pass.
template <typename T>
hs_status vcycle(hs_plan* P, const MgSet& S, int order, hsk::MgArgs A, int nu1, int nu2,
                 int sweeps_done, int passes_done, int* par, hipStream_t s)
{
    const bool pj = nu2 >= 1;
    // correction grids: passes that write them, and the buffer of their first
    // (virtual) iterate that makes the last write land in u
    const int writes_c = (nu1 >= 2 ? nu1 - 1 : 1) + (pj ? nu2 : 0);
    const int cc0 = pj ? !((writes_c - 1) & 1) : 1;
    std::vector<int> locf(S.D), locc(S.D);
    for (int st = 0; st < S.D; st++) {
        const Table<GridSeg>& J = S.jac[st];
        const bool hasF = !J.coarse_all, hasC = !J.finest;
        int cf = *par, cc = cc0;
        auto code = [&](int skip = 0) { return hsk::src_code(cf, cc, skip); };
        if (!hasC) {
            int k0 = 0;
            if (sweeps_done) {
                cf ^= passes_done & 1;
                k0 = sweeps_done;
            } else if (S.two && nu1 >= 2) {
                const Table<GridSeg>& J2 = S.pro[st];
                HS_TRY(hsk::jac2<T>(P->ctl, J2.d, J2.nseg(), J2.nblk, order, A, code(), 0, 0, issuer(P, s).partials, s));
                cf ^= 1;
                k0 = 2;
            }
            for (int k = k0; k < nu1; k++, cf ^= 1) {
                hsk::EvPair ev;
                if (st == 0 && k < 2) ev = timer_events<T>(P, k == 0 ? HS_TIMER_SWEEP1 : HS_TIMER_SWEEP2, A.L);
                HS_TRY(hsk::sweep<T>(P->ctl, J.d, J.nseg(), J.nblk, order, A, 0, 0, code(), 1, 0, 0,
                                     issuer(P, s).partials, s, 0, 0.0, 0, ev));
            }
        } else if (nu1 >= 2) {
            // finest grids' first sweep alone, then the correction grids' second
            // sweep from their zero-guess first one, next to the finest grids' second
            if (hasF) {
                HS_TRY(hsk::sweep<T>(P->ctl, J.d, J.nseg(), J.nblk, order, A, 0, 0, code(1), 0, 0, 0,
                                     issuer(P, s).partials, s));
                cf ^= 1;
            }
            hsk::EvPair ev;
            if (st == 0 && !hasF && S.uniform) ev = timer_events<T>(P, HS_TIMER_SWEEP2, A.L);
            HS_TRY(hsk::sweep<T>(P->ctl, J.d, J.nseg(), J.nblk, order, A, 0, 0, code(), 0, 0, 0,
                                 issuer(P, s).partials, s, 1, 0.0, 0, ev));
            cf ^= 1; cc ^= 1;
            for (int k = 2; k < nu1; k++, cf ^= 1, cc ^= 1)
                HS_TRY(hsk::sweep<T>(P->ctl, J.d, J.nseg(), J.nblk, order, A, 0, 0, code(), 0, 0, 0,
                                     issuer(P, s).partials, s));
        } else {
            HS_TRY(hsk::sweep<T>(P->ctl, J.d, J.nseg(), J.nblk, order, A, 0, 1, code(), 0, 0, 0,
                                 issuer(P, s).partials, s));
            cf ^= 1; cc ^= 1;
        }
        locf[st] = cf;
        locc[st] = cc;
        // residual restricted by full weighting in one pass
        const Table<GridSeg>& RF = S.rfw[st];
        hsk::EvPair ev;
        if (st == 0 && S.uniform) ev = timer_events<T>(P, HS_TIMER_RESID_FW, A.L);
        HS_TRY(hsk::resid_fw<T>(P->ctl, RF.d, RF.nseg(), RF.nblk, order, A, code(), s, ev));
    }
    HS_TRY(hsk::tail<T>(P->ctl, S.tail.d, S.tail.nseg(), order, A, nu1, nu2, S.tail_lds, s));
    for (int st = S.D - 1; st >= 0; st--) {
        const Table<GridSeg>& J = S.jac[st];
        int cf = locf[st], cc = locc[st];
        auto code = [&]() { return hsk::src_code(cf, cc); };
        if (pj) {
            hsk::EvPair ev;
            if (st == 0 && S.uniform) ev = timer_events<T>(P, HS_TIMER_PJAC, A.L);
            HS_TRY(hsk::pjac<T>(P->ctl, J.d, J.nseg(), J.nblk, order, A, code(), s, ev));
            cf ^= 1; cc ^= 1;
            for (int k = 1; k < nu2; k++, cf ^= 1, cc ^= 1)
                HS_TRY(hsk::sweep<T>(P->ctl, J.d, J.nseg(), J.nblk, order, A, 0, 0, code(), J.finest, 0, 0,
                                     issuer(P, s).partials, s));
        } else {
            // no post-smoothing: the corrected iterate goes to u
            const Table<GridSeg>& Pr = S.pro[st];
            HS_TRY(hsk::prolong<T>(P->ctl, Pr.d, Pr.nseg(), Pr.nblk, A, code(), 0, s));
            cf = cc = 0;
        }
        if (!J.coarse_all) *par = cf;
    }
    return HS_OK;
}

// Finest iterates left in t by an odd number of buffer-moving cycles go back
// to the node fields.
hs_status mg_finish(hs_plan* P, const MgSet& S, hsk::MgArgs A, int nu1, int nu2, hipStream_t s)
{
    if (!S.moves || nu2 < 1) return HS_OK;
    const int writes = nu1 - (S.two && nu1 >= 2 ? 1 : 0) + nu2;   // passes that move the finest iterate
    if (!(writes & 1)) return HS_OK;
    HS_TRY(hsk::mg_fixup(P->ctl, S.fine.d, S.fine.nseg(), S.fine.nblk, A, s));
    return HS_OK;
}

// Destroy the cycle graphs (all, or only those recorded over tables that
// have since changed).  A graph may still be in flight: wait for the device.
void drop_cycle_graphs(hs_plan* P, bool stale_only = false)
{
    bool any = false;
    for (const auto& g : P->cgraphs) any |= !stale_only || g.epoch != P->set_epoch;
    if (!any) return;
    (void)hipDeviceSynchronize();
    std::vector<hs_plan::CycleGraph> keep;
    for (auto& g : P->cgraphs) {
        if (!stale_only || g.epoch != P->set_epoch) (void)hipGraphExecDestroy(g.exec);
        else keep.push_back(g);
    }
    P->cgraphs.swap(keep);
}

// The graph of cycles 1..K-1 and the stopping test at K of a solve over ls
// (level L, substep m, node), captured by `record` on the plan's capture
// stream on first use.  *par enters as the finest grids' buffer at cycle 1
// and leaves as the buffer after the K cycles.
template <class F>
hs_status cycle_graph(hs_plan* P, const LaneSet& ls, int L, int m, int node, int K, hipGraphExec_t* exec,
                      int* par, F record)
{
    for (const auto& g : P->cgraphs)
        if (g.set == &ls && g.epoch == P->set_epoch && g.L == L && g.m == m && g.node == node && g.K == K) {
            *exec = g.exec;
            *par = g.par;
            return HS_OK;
        }
    if (P->cgraphs.size() >= 64) drop_cycle_graphs(P);
    if (!P->cap) HS_TRY(hipStreamCreateWithFlags(&P->cap, hipStreamNonBlocking));
    HS_TRY(hipStreamBeginCapture(P->cap, hipStreamCaptureModeThreadLocal));
    int pg = *par;
    hs_status st = record(P->cap, &pg);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(P->cap, &g);
    if (st != HS_OK || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        return st != HS_OK ? st : HS_EDEVICE;
    }
    hipGraphExec_t ge = nullptr;
    e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    HS_TRY(e);
    P->cgraphs.push_back({&ls, P->set_epoch, L, m, node, K, pg, ge});
    *exec = ge;
    *par = pg;
    return HS_OK;
}

// The work that follows a substep's solve in an SDC sweep: F_I at the solved
// node (and the next substep's right-hand side), over the lanes' finest grids.
struct PostSolve {
    const Table<GridSeg>* F;
    const Table<SdcSeg>* T;
    int order, m0, m1, rhs_node;
    bool done = false;   // the launches issued at the final check were the real ones
};

// Read the lane states back at a check.  With post, the solve's closing
// launches (the iterate's copy-back and the post-solve work) are issued
// behind the states' copy, gated to the lanes whose solve has stopped: they
// run while the host waits for the copy and decides.  If every lane has
// stopped they were the real launches; otherwise they did the stopped lanes'
// share, and the launches after the solve repeat it with the same result.
hs_status read_ctl_ahead(hs_plan* P, const LaneSet& ls, const MgSet& S, hsk::MgArgs A, int nu1, int nu2,
                         const PostSolve* post, hipStream_t s)
{
    if (!post) return read_ctl(P, s, &ls);
    const Issuer I = issuer(P, s);
    HS_TRY(copy_ctl(P, &ls, s));
    HS_TRY(hipEventRecord(I.ev_ctl, s));
    hsk::MgArgs G = A;
    G.gate = 2;
    HS_CHECK(mg_finish(P, S, G, nu1, nu2, s));
    HS_TRY(hsk::fi_march(P->ctl, post->F->d, post->T->d, post->T->nseg(), post->F->nblk, post->order, post->m0,
                         post->m1, post->rhs_node, 2, s));
    HS_TRY(hipEventSynchronize(I.ev_ctl));
    return HS_OK;
}

// Solve (I - a L) U_node = rhs for the lanes of ls at SDC level L; a from
// the lane's a[L][m] (m >= 0) or a_user (m = -1).  post: see read_ctl_ahead;
// when post->done is set on return the post-solve work has been issued.
hs_status mg_solve(hs_plan* P, LaneSet& ls, int L, int m, int node, hipStream_t s, bool* synced,
                   PostSolve* post = nullptr)
{
    const hs_mg_desc& mg = P->pb.mg;
    int order = P->order[L];
    hsk::MgArgs A{L, m, mg.omega, node, 1};
    // the lane states this solve decides: the set's SDC lanes, or the node-parallel solver lanes
    const int c0 = &ls == &P->np_set ? P->B : ls.first;
    const int cn = &ls == &P->np_set ? P->nctl - P->B : ls.span;
    HS_TRY(hsk::begin_solve(P->ctl, c0, cn, s));
    int& pred = m >= 0 ? P->cpred[L][m][std::min(*issuer(P, s).sweep_k, hs_plan::PRED_K - 1)] : P->cpred_user;
    if (!P->mixed) {
        const MgSet& S = ls.mg64[L];
        int par = 0;
        if (mg.fixed_cycles > 0) {
            for (int c = 0; c < mg.fixed_cycles; c++)
                HS_CHECK(vcycle<double>(P, S, order, A, mg.nu1, mg.nu2, 0, 0, &par, s));
            HS_TRY(hsk::end_solve_fixed(P->ctl, c0, cn, mg.fixed_cycles, L, s));
            return mg_finish(P, S, A, mg.nu1, mg.nu2, s);
        }
        const bool two = S.two && mg.nu1 >= 2;
        // the second sweep takes the stopping test from the norm sweep's
        // maxima (no decision launch) while a lane's maxima are few enough
        // for every block to reduce them
        // (and while the launch is one wave of blocks: in a larger one every
        // block's extra reduction adds to each wave, measured 213 against
        // 162 us for the plain sweep on 16 lanes of 127^3, more than a
        // separate decision launch costs)
        const bool fold = S.fused_norm && !two && mg.nu1 >= 2 && S.jac[0].max_seg_blocks <= 1024 &&
                          S.jac[0].nblk <= 1024;
        // residual norm and stopping test before cycle c; the norm is fused
        // with cycle c's first sweep when possible
        auto head = [&](int c, int pc, hipStream_t st) -> hs_status {
            double* const part = issuer(P, st).partials;
            if (fold) {
                const Table<GridSeg>& J = S.jac[0];
                HS_TRY(hsk::sweep<double>(P->ctl, J.d, J.nseg(), J.nblk, order, A, 0, 1, hsk::src_code(pc, 0), 1,
                                          1, c, part, st, 0, 0.0, 0,
                                          timer_events<double>(P, HS_TIMER_SWEEP1, L)));
                HS_TRY(hsk::sweep<double>(P->ctl, J.d, J.nseg(), J.nblk, order, A, 0, 0, hsk::src_code(pc ^ 1, 0),
                                          1, 2, c, part, st, 0, mg.tol, mg.max_cycles,
                                          timer_events<double>(P, HS_TIMER_SWEEP2, L)));
            } else if (S.fused_norm && two) {
                const Table<GridSeg>& J2 = S.pro[0];
                HS_TRY(hsk::jac2<double>(P->ctl, J2.d, J2.nseg(), J2.nblk, order, A, hsk::src_code(pc, 0), 1, c,
                                         part, st));
                HS_TRY(hsk::mg_decide(P->ctl, J2.d, J2.nseg(), J2.nblk, part, c, mg.tol,
                                      mg.max_cycles, L, st));
            } else if (S.fused_norm) {
                const Table<GridSeg>& J = S.jac[0];
                HS_TRY(hsk::sweep<double>(P->ctl, J.d, J.nseg(), J.nblk, order, A, 0, 1, hsk::src_code(pc, 0), 1,
                                          1, c, part, st, 0, 0.0, 0,
                                          timer_events<double>(P, HS_TIMER_SWEEP1, L)));
                HS_TRY(hsk::mg_decide(P->ctl, J.d, J.nseg(), J.nblk, part, c, mg.tol,
                                      mg.max_cycles, L, st));
            } else {
                HS_TRY(hsk::mg_norm(P->ctl, S.fine.d, S.fine.nseg(), S.fine.nblk, order, A, c,
                                    part, pc, st));
                HS_TRY(hsk::mg_decide(P->ctl, S.fine.d, S.fine.nseg(), S.fine.nblk, part, c,
                                      mg.tol, mg.max_cycles, L, st));
            }
            return HS_OK;
        };
        const int sd = fold ? 2 : (S.fused_norm ? (two ? 2 : 1) : 0);   // sweeps and passes of head()
        const int pd = fold ? 2 : (S.fused_norm ? 1 : 0);
        // the host checks the lanes at the predicted cycle count, then after
        // every cycle: a miss is nearly always a count one above the last
        // solve's, and a round trip (a 4 us copy and about 20 us of host turn-
        // around) costs less than the gated surplus cycle (11 launches of
        // about 3 us) that a check every second cycle would let through
        int next_check = pred;
        int c = 0;
        bool head_done = false;
        if (mg.cycle_graphs && pred >= 2 && pred < mg.max_cycles) {
            // cycle 0 from the host, then cycles 1..pred-1 and the test at
            // pred from one graph, whose launch overlaps cycle 0
            HS_CHECK(head(0, par, s));
            HS_CHECK(vcycle<double>(P, S, order, A, mg.nu1, mg.nu2, sd, pd, &par, s));
            hipGraphExec_t ge = nullptr;
            HS_CHECK(cycle_graph(P, ls, L, m, node, pred, &ge, &par, [&](hipStream_t st, int* pp) -> hs_status {
                for (int k = 1; k < pred; k++) {
                    HS_CHECK(head(k, *pp, st));
                    HS_CHECK(vcycle<double>(P, S, order, A, mg.nu1, mg.nu2, sd, pd, pp, st));
                }
                return head(pred, *pp, st);
            }));
            HS_TRY(hipGraphLaunch(ge, s));
            c = pred;
            head_done = true;
        }
        for (;; c++) {
            if (!head_done) HS_CHECK(head(c, par, s));
            head_done = false;
            if (c >= next_check || c >= mg.max_cycles) {
                HS_CHECK(read_ctl_ahead(P, ls, S, A, mg.nu1, mg.nu2, post, s));
                if (synced) *synced = true;
                int mc = 0;
                if (all_mg_done(P, ls, &mc, s)) {
                    pred = mc;
                    if (post) {
                        post->done = true;
                        return HS_OK;
                    }
                    break;
                }
                next_check = c + 1;
            }
            if (c >= mg.max_cycles) break;
            HS_CHECK(vcycle<double>(P, S, order, A, mg.nu1, mg.nu2, sd, pd, &par, s));
        }
        return mg_finish(P, S, A, mg.nu1, mg.nu2, s);
    }
    // mixed precision: FP64 refinement around one FP32 cycle per iteration
    const MgSet& S64 = ls.mg64[L];
    const MgSet& S32 = ls.mg32[L];
    bool fixed = mg.fixed_cycles > 0;
    int limit = fixed ? mg.fixed_cycles : mg.max_cycles;
    int next_check = pred;
    for (int it = 0;; it++) {
        if (fixed && it >= limit) break;
        HS_TRY(hsk::ir_resid(P->ctl, S64.fine.d, S32.fine.d, S64.fine.nseg(), S64.fine.nblk, order, A,
                             it, issuer(P, s).partials, s));
        if (!fixed) {
            HS_TRY(hsk::mg_decide(P->ctl, S64.fine.d, S64.fine.nseg(), S64.fine.nblk, issuer(P, s).partials, it,
                                  mg.tol, limit, L, s));
            if (it >= next_check || it >= limit) {
                HS_CHECK(read_ctl(P, s, &ls));
                if (synced) *synced = true;
                int mc = 0;
                if (all_mg_done(P, ls, &mc, s)) {
                    pred = mc;
                    break;
                }
                next_check = it + 1;
            }
            if (it >= limit) break;
        }
        int par32 = 0;
        HS_CHECK(vcycle<float>(P, S32, order, A, mg.inner_nu1, mg.inner_nu2, 0, 0, &par32, s));
        HS_TRY(hsk::ir_update(P->ctl, S64.fine.d, S32.fine.d, S64.fine.nseg(), S64.fine.nblk, A, s));
    }
    if (fixed) HS_TRY(hsk::end_solve_fixed(P->ctl, c0, cn, limit, L, s));
    return HS_OK;
}

enum { SWEEP_RAN = 0, SWEEP_DONE = 1 };

// One SDC sweep of level L over ls (eq. (7)).  With_resid: take the
// collocation residual first and stop the lanes that meet sdc_tol.
// prep_done: the sweep-constant parts were formed by the caller's residual
// pass (and with_resid is false).
hs_status sweep(hs_plan* P, LaneSet& ls, int L, bool with_resid, bool count, hipStream_t s,
                int* outcome, bool prep_done = false)
{
    const Table<SdcSeg>& T = ls.sdc[L];
    const Table<GridSeg>& F = ls.mg64[L].fine;   // z-marching blocks over the same lanes
    int M = P->M[L];
    *outcome = SWEEP_RAN;
    if (!prep_done)
        HS_TRY(hsk::sweep_prep(P->ctl, T.d, T.nseg(), T.nblk, with_resid ? 1 : 0, 1, issuer(P, s).partials, s));
    if (with_resid) {
        HS_TRY(hsk::sdc_decide(P->ctl, T.d, T.nseg(), T.nblk, issuer(P, s).partials, P->pb.sdc_tol,
                               P->pb.max_sweeps, s));
        HS_CHECK(read_ctl(P, s, &ls));
        if (all_sdc_done(P, ls, s)) {
            *outcome = SWEEP_DONE;
            return HS_OK;
        }
    }
    if (count) HS_TRY(hsk::begin_sweep(P->ctl, ls.first, ls.span, s));
    if (P->np && L == 0) {
        // node-parallel sweep: every node's right-hand side from iterate k, the
        // M-1 solves of every lane as one batched multigrid solve, then F_I
        HS_TRY(hsk::np_rhs(P->ctl, T.d, T.nseg(), T.nblk, s));
        HS_CHECK(mg_solve(P, P->np_set, L, -1, 0, s, nullptr));
        HS_TRY(hsk::fi_march(P->ctl, F.d, T.d, T.nseg(), F.nblk, P->order[L], 1, M, -1, 1, s));
        (*issuer(P, s).sweep_k)++;
        return HS_OK;
    }
    HS_TRY(hsk::make_rhs(P->ctl, T.d, T.nseg(), T.nblk, 0, 1, s));
    for (int m = 0; m + 1 < M; m++) {
        PostSolve post{&F, &T, P->order[L], m + 1, m + 2, m + 2 < M ? m + 1 : -1};
        HS_CHECK(mg_solve(P, ls, L, m, m + 1, s, nullptr, &post));
        if (!post.done)
            HS_TRY(hsk::fi_march(P->ctl, F.d, T.d, T.nseg(), F.nblk, P->order[L], post.m0, post.m1, post.rhs_node,
                                 1, s));
    }
    if (P->nlev == 1) (*issuer(P, s).sweep_k)++;
    return HS_OK;
}

// Restriction + FAS correction of ls's lanes from SDC level l to l + 1.
hipError_t fas_restrict(hs_plan* P, const LaneSet& ls, int l, hipStream_t s)
{
    const Table<FasSeg>& T = ls.fasc[l];
    return hsk::fas_restrict(P->ctl, T.d, T.nseg(), T.nblk, P->order[l + 1], 1, s);
}

// Interpolation of the coarse corrections of ls's lanes from level l + 1 to
// the nodes of level l: trilinear, or tricubic with pb.fas_interp = 3
// (section 1.1 leaves the transfer to the references).
hipError_t fas_interp(hs_plan* P, const LaneSet& ls, int l, hipStream_t s)
{
    const Table<FasSeg>& T = ls.fasf[l];
    if (P->pb.fas_interp == 3) return hsk::fas_interp3(P->ctl, T.d, T.nseg(), T.nblk, 1, s);
    return hsk::fas_interp(P->ctl, T.d, T.nseg(), T.nblk, 1, s);
}

// fas_interp to level l, then F_I recomputed at every node of level l.
hipError_t interp_level(hs_plan* P, const LaneSet& ls, int l, hipStream_t s)
{
    hipError_t e = fas_interp(P, ls, l, s);
    if (e != hipSuccess) return e;
    return hsk::fi_march(P->ctl, ls.mg64[l].fine.d, ls.sdc[l].d, ls.sdc[l].nseg(), ls.mg64[l].fine.nblk,
                         P->order[l], 0, P->M[l], -1, 1, s);
}

// One MLSDC iteration as a V-cycle over the nlev levels: a sweep on level 0,
// then per level restriction + FAS correction and a sweep (with tau) down to
// the coarsest; on the way up interpolation to each level and, on the levels
// between the finest and the coarsest, another sweep; no closing sweep on
// level 0 (section 1.1; with two levels: fine sweep, restriction, coarse
// sweep, interpolation).
hs_status mlsdc_iter(hs_plan* P, LaneSet& ls, bool with_resid, hipStream_t s, int* outcome)
{
    HS_CHECK(sweep(P, ls, 0, with_resid, true, s, outcome));
    if (*outcome == SWEEP_DONE) return HS_OK;
    int o2;
    for (int l = 0; l + 1 < P->nlev; l++) {
        HS_TRY(fas_restrict(P, ls, l, s));
        HS_CHECK(sweep(P, ls, l + 1, false, false, s, &o2));
    }
    for (int l = P->nlev - 2; l >= 0; l--) {
        HS_TRY(interp_level(P, ls, l, s));
        if (l > 0) HS_CHECK(sweep(P, ls, l, false, false, s, &o2));
    }
    P->sweep_k++;
    return HS_OK;
}

// Rebuild the run set's tables for the lanes currently active and upload
// them (synchronous with respect to the host; ordered on stream s).
hs_status refresh_run(hs_plan* P, hipStream_t s)
{
    if (!P->run_dirty) return HS_OK;
    LaneSet& ls = P->run;
    ls = LaneSet();
    for (int b = 0; b < P->B; b++)
        if (P->active[b]) ls.lanes.push_back(b);
    build_set_host(P, ls);
    P->set_epoch++;   // graphs recorded over the old tables are stale
    for (int L = 0; L < P->nlev; L++) {
        for (int f = 0; f < 2; f++) {
            MgSet& S = f ? ls.mg32[L] : ls.mg64[L];
            const MgSet& A = f ? P->all.mg32[L] : P->all.mg64[L];
            // the run set never holds deeper lanes than the full set
            if (S.D > A.D) return HS_ESTATE;
            for (int st = 0; st < S.D; st++) {
                S.jac[st].d = P->store.grid[L][f][3 * st];
                S.pro[st].d = P->store.grid[L][f][3 * st + 1];
                S.rfw[st].d = P->store.grid[L][f][3 * st + 2];
            }
            S.fine.d = P->store.grid[L][f][3 * A.D];
            S.tail.d = P->store.tail[L][f];
            if (S.fine.h.empty()) S.fine.d = nullptr;
            if (S.tail.h.empty()) S.tail.d = nullptr;
        }
        ls.sdc[L].d = ls.sdc[L].h.empty() ? nullptr : P->store.sdc[L];
    }
    for (int l = 0; l + 1 < P->nlev; l++) {
        ls.fasc[l].d = ls.fasc[l].h.empty() ? nullptr : P->store.fasc[l];
        ls.fasf[l].d = ls.fasf[l].h.empty() ? nullptr : P->store.fasf[l];
    }
    HS_TRY(upload_set(P, ls, s));
    HS_TRY(hipStreamSynchronize(s));
    drop_cycle_graphs(P, true);
    P->run_dirty = false;
    return HS_OK;
}

// ---------------------------------------------------------------------------
// SDC with the compact pair (B-weighted form of eqs. (6)-(7)), and two-level
// MLSDC with it on the fine level: every substep solves (B - a A) U_{m+1} =
// rhs by V-cycles on the compact operator, rediscretised on each coarser grid.
// The lanes are taken one at a time with launches over one grid; the stopping
// test of each solve (the same rule as the second-order/fourth-order solves)
// runs on the device, and the host reads the lane state at the predicted
// cycle count.
// ---------------------------------------------------------------------------

// One V(nu1, nu2) cycle on grid l of lane `lane`'s hierarchy: the iterate in
// cur (taken as zero with `zero`), oth a scratch grid of the same size, b the
// right-hand side; *res receives the buffer (cur or oth) that holds the
// iterate after the cycle.  The sweeps ping-pong between the two buffers and
// the coarse correction is added in place.
// With `cycle` >= 0 the first pre-sweep also takes the residual norms of the
// incoming iterate and the stopping test before that cycle runs on the
// device (the rest of the cycle is gated off when the solve stops there).
// Grids with n <= HS_TAIL_N run as one LDS-resident workgroup, in place.
hs_status cmp_vcycle(hs_plan* P, int lane, int l, double* cur, double* oth, const double* b, double dtau, bool zero,
                     int gate, int cycle, hipStream_t s, double** res)
{
    const hs_mg_desc& mg = P->pb.mg;
    const LaneBufs& lb = P->lanes[lane];
    const int n = lb.grids[0][l];
    if (n <= HS_TAIL_N) {
        HS_TRY(hsk::compact_tail(n, cur, b, zero ? 1 : 0, P->ctl, lane, dtau, mg.omega, mg.nu1, mg.nu2,
                                 mg.n_coarsest, gate, s));
        *res = cur;
        return HS_OK;
    }
    double* const part = issuer(P, s).partials;
    for (int q = 0; q < mg.nu1; q++) {
        if (q == 0 && zero) {
            HS_TRY(hsk::compact_zsweep(n, b, oth, P->ctl, lane, dtau, mg.omega, gate, s));
        } else if (q == 0 && cycle >= 0) {
            HS_TRY(hsk::compact_op(5, n, cur, oth, b, nullptr, P->ctl, lane, dtau, mg.omega, part, gate, s));
            HS_TRY(hsk::compact_reduce(part, hsk::compact_blocks(n), P->ctl, lane, 3, cycle, mg.tol, mg.max_cycles, s));
        } else {
            HS_TRY(hsk::compact_op(0, n, cur, oth, b, nullptr, P->ctl, lane, dtau, mg.omega, nullptr, gate, s));
        }
        std::swap(cur, oth);
    }
    HS_TRY(hsk::compact_op(1, n, cur, oth, b, nullptr, P->ctl, lane, dtau, 0.0, nullptr, gate, s));
    const int nc = lb.grids[0][l + 1];
    double* cb = lb.gb[0][l + 1];
    HS_TRY(hsk::compact_fw(n, oth, cb, P->ctl, lane, gate, s));
    double* ec = nullptr;
    HS_CHECK(cmp_vcycle(P, lane, l + 1, lb.gu[0][l + 1], lb.gt[0][l + 1], cb, dtau, true, gate, -1, s, &ec));
    HS_TRY(hsk::compact_prolong(nc, ec, cur, cur, P->ctl, lane, gate, s));
    for (int q = 0; q < mg.nu2; q++) {
        HS_TRY(hsk::compact_op(0, n, cur, oth, b, nullptr, P->ctl, lane, dtau, mg.omega, nullptr, gate, s));
        std::swap(cur, oth);
    }
    *res = cur;
    return HS_OK;
}

// Solve (B - a A) u = b on the lane's finest grid from the guess in u,
// a = nu dt dtau (substep m).  Fixed cycles: the cycles, then the residual
// norm.  Tolerance mode: the norm and the stopping test before each cycle run
// on the device (fused with the cycle's first sweep) and the cycles after a
// stop are skipped there; the host reads the lane state at the cycle count of
// the lane's last solve of this substep, then after every cycle.  The
// iterate moves between u and the lane's scratch grid; the final one is
// copied back to u if it ends in the scratch grid.
hs_status cmp_solve(hs_plan* P, int lane, int m, double dtau, double* u, const double* b, hipStream_t s)
{
    const hs_mg_desc& mg = P->pb.mg;
    const LaneBufs& lb = P->lanes[lane];
    const int n = lb.n[0], nb = hsk::compact_blocks(n);
    const long long N = lb.N[0];
    const Issuer I = issuer(P, s);
    const bool tail = n <= HS_TAIL_N;   // the whole hierarchy in one workgroup, in place in u
    HS_TRY(hsk::begin_solve(P->ctl, lane, 1, s));
    double *cur = u, *oth = lb.tmp[0];
    if (mg.fixed_cycles > 0) {
        for (int c = 0; c < mg.fixed_cycles; c++) {
            double* r = nullptr;
            HS_CHECK(cmp_vcycle(P, lane, 0, cur, oth, b, dtau, false, 0, -1, s, &r));
            oth = r == cur ? oth : cur;
            cur = r;
        }
        if (cur != u) HS_TRY(hipMemcpyAsync(u, cur, N * sizeof(double), hipMemcpyDeviceToDevice, s));
        HS_TRY(hsk::compact_op(4, n, u, nullptr, b, nullptr, P->ctl, lane, dtau, 0.0, I.partials, 0, s));
        HS_TRY(hsk::compact_reduce(I.partials, nb, P->ctl, lane, 0, 0, 0.0, 0, s));
        HS_CHECK(read_ctl(P, s, &P->run));
        const double rho = I.h_ctl[lane].mg_rho;
        const bool bad = rho != rho;
        HS_TRY(hsk::compact_ctl(P->ctl, lane, 0, mg.fixed_cycles, bad ? 2 : 1, 0, bad ? HS_ENONFINITE : HS_OK, s));
        return HS_OK;
    }
    if (P->cmp_pred.size() != (size_t)P->B * HS_MAXM) P->cmp_pred.assign((size_t)P->B * HS_MAXM, 1);
    int& pred = P->cmp_pred[(size_t)lane * HS_MAXM + m];
    int next = pred;
    std::vector<double*> at{cur};   // at[c]: the buffer holding the iterate before cycle c
    for (int c = 0;; c++) {
        if (tail) {
            HS_TRY(hsk::compact_op(4, n, cur, nullptr, b, nullptr, P->ctl, lane, dtau, 0.0, I.partials, 1, s));
            HS_TRY(hsk::compact_reduce(I.partials, nb, P->ctl, lane, 3, c, mg.tol, mg.max_cycles, s));
        }
        // cycle c (its first sweep decides first when the hierarchy is not all tail)
        double* r = nullptr;
        HS_CHECK(cmp_vcycle(P, lane, 0, cur, oth, b, dtau, false, 1, tail ? -1 : c, s, &r));
        oth = r == cur ? oth : cur;
        cur = r;
        at.push_back(cur);
        if (c >= next || c >= mg.max_cycles) {
            HS_CHECK(read_ctl(P, s, &P->run));
            const LaneCtl& h = I.h_ctl[lane];
            if (h.mg_state != 0) {
                const int k = h.mg_cycle;
                if (k < 0 || k > c) return HS_EDEVICE;
                if (at[k] != u) HS_TRY(hipMemcpyAsync(u, at[k], N * sizeof(double), hipMemcpyDeviceToDevice, s));
                pred = std::max(1, k);
                return HS_OK;
            }
            if (c >= mg.max_cycles) return HS_EDEVICE;   // the test at max_cycles always stops the solve
            next = c + 1;
        }
    }
}

// Collocation residual of the B-weighted form,
//   R = max over m = 1..M-1 of |B U_0 + dt sum_j Q_mj F_j - B U_m|,
// into the lane's sdc_res (read back into *R).
hs_status cmp_residual(hs_plan* P, int lane, hipStream_t s, double* R)
{
    const LaneBufs& lb = P->lanes[lane];
    const int n = lb.n[0], M = P->M[0];
    const long long N = lb.N[0];
    const Issuer I = issuer(P, s);
    HS_TRY(hsk::compact_apply(n, 1, 1.0, 0.0, lb.U[0], lb.tmp[0], s));
    for (int m = 1; m < M; m++) {
        HS_TRY(hsk::compact_quad(n, M, m, lb.FI[0], lb.tmp[0], lb.rhs[0], lb.sig[0], P->ctl, lane, 0, s));
        HS_TRY(hsk::compact_op(4, n, lb.U[0] + m * N, nullptr, lb.rhs[0], nullptr, P->ctl, lane, 0.0, 0.0,
                               I.partials, 0, s));
        HS_TRY(hsk::compact_reduce(I.partials, hsk::compact_blocks(n), P->ctl, lane, m == 1 ? 1 : 2, 0, 0.0, 0, s));
    }
    HS_CHECK(read_ctl(P, s, &P->run));
    *R = I.h_ctl[lane].sdc_res;
    return HS_OK;
}

// One compact IMEX sweep of a lane: dt S^k F from iterate k, then per substep
// rhs = B U_m - dt_m G_{m+1} + dt S^k_m F, the solve for U_{m+1} from its
// old value, and G_{m+1} = nu A U_{m+1}.
hs_status cmp_sweep(hs_plan* P, int lane, hipStream_t s)
{
    const LaneBufs& lb = P->lanes[lane];
    const int n = lb.n[0], M = P->M[0];
    const long long N = lb.N[0];
    const SdcConst& K = host_consts().sdc[M];
    double *U = lb.U[0], *G = lb.FI[0];
    HS_TRY(hsk::begin_sweep(P->ctl, lane, 1, s));
    HS_TRY(hsk::compact_quad(n, M, -1, G, nullptr, lb.P[0], lb.sig[0], P->ctl, lane, 0, s));
    for (int m = 0; m + 1 < M; m++) {
        HS_TRY(hsk::compact_op(2, n, U + m * N, lb.rhs[0], lb.P[0] + m * N, G + (m + 1) * N, P->ctl, lane,
                               K.dtau[m], 0.0, nullptr, 0, s));
        HS_CHECK(cmp_solve(P, lane, m, K.dtau[m], U + (m + 1) * N, lb.rhs[0], s));
        HS_TRY(hsk::compact_op(3, n, U + (m + 1) * N, G + (m + 1) * N, nullptr, nullptr, P->ctl, lane, 0.0, 0.0,
                               nullptr, 0, s));
    }
    return HS_OK;
}

// The run set's lanes that iterate in the current step (host view).
std::vector<int> cmp_live(hs_plan* P, hipStream_t s)
{
    std::vector<int> live;
    const LaneCtl* h = issuer(P, s).h_ctl;
    for (int b : P->run.lanes)
        if (h[b].sdc_state == 0) live.push_back(b);
    return live;
}

// Start a step: coefficients, then every node's U = U_{M-1} (the state) and G = nu A U.
hs_status cmp_begin_step(hs_plan* P, hipStream_t s)
{
    HS_CHECK(refresh_run(P, s));
    P->sweep_k = 0;
    HS_TRY(hsk::begin_step(P->ctl, P->B, P->nlev, P->M, s));
    HS_CHECK(read_ctl(P, s));
    const int M = P->M[0];
    for (int b : cmp_live(P, s)) {
        const LaneBufs& lb = P->lanes[b];
        const long long N = lb.N[0];
        double *U = lb.U[0], *G = lb.FI[0];
        HS_TRY(hsk::compact_op(3, lb.n[0], U + (M - 1) * N, G + (M - 1) * N, nullptr, nullptr, P->ctl, b, 0.0, 0.0,
                               nullptr, 0, s));
        for (int m = 0; m + 1 < M; m++) {
            HS_TRY(hipMemcpyAsync(U + m * N, U + (M - 1) * N, N * sizeof(double), hipMemcpyDeviceToDevice, s));
            HS_TRY(hipMemcpyAsync(G + m * N, G + (M - 1) * N, N * sizeof(double), hipMemcpyDeviceToDevice, s));
        }
    }
    return HS_OK;
}

// One sweep of every live lane (read back first: a lane whose SDC
// iteration has ended is left alone).
hs_status cmp_sweep_all(hs_plan* P, hipStream_t s)
{
    HS_CHECK(read_ctl(P, s));
    for (int b : cmp_live(P, s)) HS_CHECK(cmp_sweep(P, b, s));
    return HS_OK;
}

hs_status cmp_step(hs_plan* P, hipStream_t s)
{
    HS_CHECK(cmp_begin_step(P, s));
    const hs_problem& pb = P->pb;
    for (int b : cmp_live(P, s)) {
        int state = 1, status = HS_OK;
        double R = 0.0;
        for (int k = 0;; k++) {
            if (pb.sweeps > 0) {
                if (k >= pb.sweeps) break;
            } else {
                HS_CHECK(cmp_residual(P, b, s, &R));
                if (R != R) { state = 2; status = HS_ENONFINITE; break; }
                if (R <= pb.sdc_tol) break;
                if (k >= pb.max_sweeps) { state = 2; status = HS_ENOCONV; break; }
            }
            HS_CHECK(cmp_sweep(P, b, s));
        }
        if (pb.sweeps > 0) HS_CHECK(cmp_residual(P, b, s, &R));
        HS_TRY(hsk::compact_ctl(P->ctl, b, 1, 0, state, 0, status, s));
    }
    HS_TRY(hsk::end_step(P->ctl, P->B, s));
    return HS_OK;
}

// One two-level MLSDC iteration with the compact fine level over the live
// lanes: the fine B-weighted sweeps (lane by lane); f^I = B_h^{-1} G at every
// fine node, in place of G, for the FAS restriction (which then reads it as
// the fine level's F_I); restriction, coarse sweep and interpolation of the
// coarse correction over the lane set; G = nu A_h U again at every fine node.
hs_status cmp_mlsdc_iter(hs_plan* P, hipStream_t s)
{
    HS_CHECK(read_ctl(P, s));
    const std::vector<int> live = cmp_live(P, s);
    if (live.empty()) return HS_OK;
    const int M = P->M[0];
    for (int b : live) HS_CHECK(cmp_sweep(P, b, s));
    for (int b : live) {
        const LaneBufs& lb = P->lanes[b];
        const long long N = lb.N[0];
        const double* tab = P->dst_tab.at(lb.n[0]);
        for (int j = 0; j < M; j++)
            HS_TRY(hsk::compact_binv(lb.n[0], tab, lb.FI[0] + j * N, lb.FI[0] + j * N, lb.tmp[0], lb.rhs[0], s));
    }
    LaneSet& ls = P->run;
    HS_TRY(fas_restrict(P, ls, 0, s));
    int outcome;
    HS_CHECK(sweep(P, ls, 1, false, false, s, &outcome));
    HS_TRY(fas_interp(P, ls, 0, s));
    for (int b : live) {
        const LaneBufs& lb = P->lanes[b];
        const long long N = lb.N[0];
        for (int j = 0; j < M; j++)
            HS_TRY(hsk::compact_op(3, lb.n[0], lb.U[0] + j * N, lb.FI[0] + j * N, nullptr, nullptr, P->ctl, b, 0.0,
                                   0.0, nullptr, 0, s));
    }
    return HS_OK;
}

// A step of two-level MLSDC with the compact fine level: `sweeps`
// iterations, or iterations until each lane's B-weighted fine residual meets
// sdc_tol (a lane that has stopped is left out of the later iterations).
hs_status cmp_mlsdc_step(hs_plan* P, hipStream_t s)
{
    HS_CHECK(cmp_begin_step(P, s));
    const hs_problem& pb = P->pb;
    if (pb.sweeps > 0) {
        for (int k = 0; k < pb.sweeps; k++) HS_CHECK(cmp_mlsdc_iter(P, s));
        for (int b : cmp_live(P, s)) {
            double R = 0.0;
            HS_CHECK(cmp_residual(P, b, s, &R));
            HS_TRY(hsk::compact_ctl(P->ctl, b, 1, 0, 1, 0, HS_OK, s));
        }
    } else {
        for (int k = 0;; k++) {
            HS_CHECK(read_ctl(P, s));
            const std::vector<int> live = cmp_live(P, s);
            if (live.empty()) break;
            for (int b : live) {
                double R = 0.0;
                HS_CHECK(cmp_residual(P, b, s, &R));
                int state = 0, status = HS_OK;
                if (R != R) { state = 2; status = HS_ENONFINITE; }
                else if (R <= pb.sdc_tol) state = 1;
                else if (k >= pb.max_sweeps) { state = 2; status = HS_ENOCONV; }
                if (state != 0) HS_TRY(hsk::compact_ctl(P->ctl, b, 1, 0, state, 0, status, s));
            }
            HS_CHECK(cmp_mlsdc_iter(P, s));
        }
    }
    HS_TRY(hsk::end_step(P->ctl, P->B, s));
    return HS_OK;
}

hs_status begin_step(hs_plan* P, hipStream_t s)
{
    if (P->compact) return cmp_begin_step(P, s);
    HS_CHECK(refresh_run(P, s));
    P->sweep_k = 0;
    HS_TRY(hsk::begin_step(P->ctl, P->B, P->nlev, P->M, s));
    if (P->np) HS_TRY(hsk::np_lanes(P->ctl, P->B, P->M[0], 1, s));
    const Table<SdcSeg>& T = P->run.sdc[0];
    HS_TRY(hsk::spread(P->ctl, T.d, T.nseg(), T.nblk, P->order[0], P->M[0] - 1, s));
    return HS_OK;
}

hs_status step(hs_plan* P, hipStream_t s)
{
    if (P->compact) return P->nlev == 2 ? cmp_mlsdc_step(P, s) : cmp_step(P, s);
    HS_CHECK(begin_step(P, s));
    const hs_problem& pb = P->pb;
    int outcome;
    LaneSet& ls = P->run;
    if (ls.lanes.empty()) {
        HS_TRY(hsk::end_step(P->ctl, P->B, s));
        return HS_OK;
    }
    if (pb.sweeps > 0) {
        for (int k = 0; k < pb.sweeps; k++) {
            if (P->nlev == 1) HS_CHECK(sweep(P, ls, 0, false, true, s, &outcome));
            else HS_CHECK(mlsdc_iter(P, ls, false, s, &outcome));
        }
    } else {
        for (int k = 0; k <= pb.max_sweeps + 1; k++) {
            if (P->nlev == 1) HS_CHECK(sweep(P, ls, 0, true, true, s, &outcome));
            else HS_CHECK(mlsdc_iter(P, ls, true, s, &outcome));
            if (outcome == SWEEP_DONE) break;
        }
    }
    HS_TRY(hsk::end_step(P->ctl, P->B, s));
    return HS_OK;
}

hs_status check_bound(const hs_plan* P)
{
    if (!P) return HS_EINVAL;
    if (!P->bound) return HS_ESTATE;
    return HS_OK;
}

hs_status lanes_status(hs_plan* P)
{
    int worst = HS_OK;
    for (int b = 0; b < P->B; b++) {
        int st = P->h_ctl[b].status;
        if (st < worst) worst = st;
    }
    return (hs_status)worst;
}

}  // namespace

// ---------------------------------------------------------------------------
// Device scratch of the allocation-free stand-alone solve (hs_mg_solve_static):
// one array per GPU, held until the process ends.  Host code never passes the
// array's name to a kernel or a copy: its device address is taken once per
// device with hipGetSymbolAddress and kept in g_scratch_ptr.
// ---------------------------------------------------------------------------
#define HS_STATIC_SCRATCH_BYTES (8u << 20)

static __device__ __align__(256) unsigned char scratch[HS_STATIC_SCRATCH_BYTES];

namespace {

std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_ptr;

// Device address of this device's scratch (taken on the first call per device).
hs_status scratch_address(void** out)
{
    int dev = 0;
    HS_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it == g_scratch_ptr.end()) {
        void* ptr = nullptr;
        hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) return HS_EDEVICE;
        it = g_scratch_ptr.emplace(dev, ptr).first;
    }
    *out = it->second;
    return HS_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char* hs_status_string(hs_status s)
{
    switch (s) {
    case HS_OK: return "ok";
    case HS_EINVAL: return "invalid argument";
    case HS_ENOMEM: return "workspace or budget too small";
    case HS_ENOCONV: return "iteration limit reached without convergence";
    case HS_ENONFINITE: return "non-finite residual";
    case HS_EDEVICE: return "HIP error";
    case HS_ESTATE: return "call out of order";
    case HS_PENDING: return "pending";
    }
    return "unknown status";
}

hs_status hs_collocation(int32_t M, double* h_tau, double* h_Q)
{
    if (M < 2 || M > HS_MAXM) return HS_EINVAL;
    long double t[HS_MAXM], Q[HS_MAXM][HS_MAXM];
    collocation(M, t, Q);
    for (int m = 0; m < M; m++) {
        if (h_tau) h_tau[m] = (double)t[m];
        if (h_Q)
            for (int j = 0; j < M; j++) h_Q[m * M + j] = (double)Q[m][j];
    }
    return HS_OK;
}

static void init_plan(hs_plan* P, const hs_problem* pb)
{
    P->pb = *pb;
    P->B = pb->batch;
    P->nlev = pb->nlevels;
    for (int L = 0; L < HS_MAXLEV; L++) {
        P->order[L] = L < pb->nlevels && pb->lev[L].order != HS_ORDER_COMPACT ? pb->lev[L].order : 2;
        P->M[L] = L < pb->nlevels ? pb->lev[L].nnodes : 2;
    }
    P->compact = pb->lev[0].order == HS_ORDER_COMPACT;
    P->mixed = pb->mg.precision == HS_MIXED;
    P->lane_n.assign(P->B, pb->lev[0].n);
    if (pb->h_lane_n)
        for (int b = 0; b < P->B; b++) P->lane_n[b] = pb->h_lane_n[b];
    P->np = pb->sdc_node_parallel != 0;
    P->nctl = P->B + (P->np ? P->B * (P->M[0] - 1) : 0);
    P->pb.h_lane_n = nullptr;
    for (int L = 0; L < HS_MAXLEV; L++)
        for (int m = 0; m < HS_MAXM; m++)
            for (int k = 0; k < hs_plan::PRED_K; k++) P->cpred[L][m][k] = 1;
    P->cpred_user = 1;
}

hs_status hs_workspace_bytes(const hs_problem* pb, size_t* bytes)
{
    HS_CHECK(validate(pb));
    if (!bytes) return HS_EINVAL;
    hs_plan P;
    init_plan(&P, pb);
    layout(&P, nullptr);
    *bytes = P.bytes;
    return HS_OK;
}

hs_status hs_plan_create(const hs_problem* pb, hs_plan** plan)
{
    if (!plan) return HS_EINVAL;
    HS_CHECK(validate(pb));
    hs_plan* P = new (std::nothrow) hs_plan();
    if (!P) return HS_ENOMEM;
    init_plan(P, pb);
    layout(P, nullptr);
    *plan = P;
    return HS_OK;
}

hs_status hs_plan_bind(hs_plan* P, void* d_ws, size_t bytes, void* stream)
{
    if (!P || !d_ws) return HS_EINVAL;
    if (((uintptr_t)d_ws & 255) != 0) return HS_EINVAL;
    if (bytes < P->bytes) return HS_ENOMEM;
    hipStream_t s = (hipStream_t)stream;
    HS_TRY(ensure_constants());
    HS_TRY(hipGetDevice(&P->device));
    P->ws = (char*)d_ws;
    drop_cycle_graphs(P);
    layout(P, P->ws);
    if (!P->h_ctl) HS_TRY(hipHostMalloc((void**)&P->h_ctl, sizeof(LaneCtl) * P->nctl, hipHostMallocDefault));
    if (!P->ev_ctl) HS_TRY(hipEventCreateWithFlags(&P->ev_ctl, hipEventDisableTiming));
    // sine tables sin(pi (i+1) h)
    std::map<const double*, int> sig;
    for (auto& lb : P->lanes)
        for (int L = 0; L < P->nlev; L++) sig[lb.sig[L]] = lb.n[L];
    std::vector<std::vector<double>> keep;
    for (auto& kv : sig) {
        int n = kv.second;
        keep.emplace_back(n);
        for (int i = 0; i < n; i++)
            keep.back()[i] = std::sin(3.14159265358979323846 * (double)(i + 1) / (double)(n + 1));
        HS_TRY(hipMemcpyAsync((void*)kv.first, keep.back().data(), n * sizeof(double),
                              hipMemcpyHostToDevice, s));
    }
    // B_h^{-1} tables of the compact MLSDC: tab[q n + i] = S_iq, S_iq = sqrt(2/(n+1)) sin(pi (i+1)(q+1)/(n+1)),
    // then cos(pi (i+1)/(n+1))
    for (auto& kv : P->dst_tab) {
        const int n = kv.first;
        keep.emplace_back((size_t)n * (n + 1));
        std::vector<double>& t = keep.back();
        for (int q = 0; q < n; q++)
            for (int i = 0; i < n; i++)
                t[(size_t)q * n + i] = std::sqrt(2.0 / (n + 1)) * std::sin(M_PI * (i + 1) * (q + 1) / (n + 1));
        for (int i = 0; i < n; i++) t[(size_t)n * n + i] = std::cos(M_PI * (i + 1) / (n + 1));
        HS_TRY(hipMemcpyAsync((void*)kv.second, t.data(), t.size() * sizeof(double), hipMemcpyHostToDevice, s));
    }
    if (!P->pb.lane_memory) HS_TRY(upload_set(P, P->all, s));   // else the lanes' pointers come later
    for (const MgSet* S : {&P->np_set.mg64[0], &P->np_set.mg32[0]}) {
        for (auto& t : S->jac) HS_TRY(upload(t, s));
        for (auto& t : S->pro) HS_TRY(upload(t, s));
        for (auto& t : S->rfw) HS_TRY(upload(t, s));
        HS_TRY(upload(S->tail, s));
        HS_TRY(upload(S->fine, s));
    }
    for (auto& ls : P->single) HS_TRY(upload_set(P, ls, s));
    HS_TRY(upload(P->hf_dst, s));
    HS_TRY(upload(P->hf_src, s));
    for (auto& t : P->hc_dst) HS_TRY(upload(t, s));
    for (auto& t : P->hc_src) HS_TRY(upload(t, s));
    for (auto& ls : P->grp) HS_TRY(upload_set(P, ls, s));
    for (auto* v : {&P->gh_dst, &P->gh_src, &P->gc_src})
        for (auto& t : *v) HS_TRY(upload(t, s));
    if (P->G) {
        // the coarse pipeline's stream (default priority) and its thread's read-back state
        if (!P->pipe) HS_TRY(hipStreamCreateWithFlags(&P->pipe, hipStreamNonBlocking));
        if (!P->h_ctl2) HS_TRY(hipHostMalloc((void**)&P->h_ctl2, sizeof(LaneCtl) * P->nctl, hipHostMallocDefault));
        if (!P->ev_ctl2) HS_TRY(hipEventCreateWithFlags(&P->ev_ctl2, hipEventDisableTiming));
        if (!P->ev_go) HS_TRY(hipEventCreateWithFlags(&P->ev_go, hipEventDisableTiming));
        for (auto* v : {&P->ev_r, &P->ev_c})
            while ((int)v->size() < P->G) {
                hipEvent_t e = nullptr;
                HS_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
                v->push_back(e);
            }
    }
    for (int L = 0; L < P->nlev; L++) HS_TRY(upload(P->offs[L], s));
    for (int b = 0; b < P->B; b++) {
        double t0 = P->pb.t0, nsteps = P->pb.nsteps;
        if (P->pb.nslices > 1) {
            t0 = P->pb.t0 + b * P->pb.dt;
            nsteps = 1;
        }
        const int active = P->pb.lane_memory ? 0 : 1;   // lanes of their own memory wait for it
        HS_TRY(hsk::set_lane(P->ctl, b, P->pb.nu, P->pb.dt, t0, P->pb.forcing_c, (int)nsteps, active, s));
        P->active[b] = active;
    }
    if (P->np) HS_TRY(hsk::np_lanes(P->ctl, P->B, P->M[0], 0, s));
    P->run_dirty = true;
    HS_TRY(hipStreamSynchronize(s));
    P->bound = true;
    return HS_OK;
}

hs_status hs_lane_bytes(const hs_problem* pb, int32_t lane, size_t* bytes)
{
    HS_CHECK(validate(pb));
    if (!bytes || lane < 0 || lane >= pb->batch) return HS_EINVAL;
    hs_plan P;
    init_plan(&P, pb);
    P.sig.clear();
    for (int L = 0; L < P.nlev; L++) {
        int n = L == 0 ? P.lane_n[lane] : (P.lane_n[lane] - 1) / 2;
        P.sig[n] = nullptr;
    }
    P.lanes.assign(P.B, LaneBufs());
    *bytes = lane_bytes_of(&P, lane);
    return HS_OK;
}

hs_status hs_plan_bind_lane(hs_plan* P, int32_t lane, void* d_mem, size_t bytes, void* stream)
{
    HS_CHECK(check_bound(P));
    if (!P->pb.lane_memory || lane < 0 || lane >= P->B || !d_mem || ((uintptr_t)d_mem & 255)) return HS_EINVAL;
    if (P->active[lane]) return HS_ESTATE;
    if (bytes < lane_bytes_of(P, lane)) return HS_ENOMEM;
    // the lane's sine tables stay where the workspace put them
    P->lane_base[lane] = d_mem;
    Bump own((char*)d_mem);
    lay_lane(P, lane, own);
    P->run_dirty = true;
    (void)stream;
    return HS_OK;
}

hs_status hs_plan_unbind_lane(hs_plan* P, int32_t lane)
{
    HS_CHECK(check_bound(P));
    if (!P->pb.lane_memory || lane < 0 || lane >= P->B) return HS_EINVAL;
    if (P->active[lane]) return HS_ESTATE;
    P->lane_base[lane] = nullptr;
    Bump none(nullptr);
    lay_lane(P, lane, none);
    P->run_dirty = true;
    return HS_OK;
}

hs_status hs_plan_destroy(hs_plan* P)
{
    if (!P) return HS_EINVAL;
    if (P->gexec) (void)hipGraphExecDestroy(P->gexec);
    if (P->graph) (void)hipGraphDestroy(P->graph);
    drop_cycle_graphs(P);
    if (P->cap) (void)hipStreamDestroy(P->cap);
    if (P->h_ctl) (void)hipHostFree(P->h_ctl);
    if (P->ev_ctl) (void)hipEventDestroy(P->ev_ctl);
    for (hipEvent_t e : P->timer_ev) (void)hipEventDestroy(e);
    if (P->pipe) (void)hipStreamDestroy(P->pipe);
    if (P->h_ctl2) (void)hipHostFree(P->h_ctl2);
    if (P->ev_ctl2) (void)hipEventDestroy(P->ev_ctl2);
    if (P->ev_go) (void)hipEventDestroy(P->ev_go);
    for (hipEvent_t e : P->ev_r) (void)hipEventDestroy(e);
    for (hipEvent_t e : P->ev_c) (void)hipEventDestroy(e);
    delete P;
    return HS_OK;
}

hs_status hs_plan_lanes(const hs_plan* P, int32_t* lanes, int32_t* h_lane_n)
{
    if (!P) return HS_EINVAL;
    if (lanes) *lanes = P->B;
    if (h_lane_n)
        for (int b = 0; b < P->B; b++) h_lane_n[b] = P->lane_n[b];
    return HS_OK;
}

hs_status hs_set_lane(hs_plan* P, int32_t lane, double nu, double dt, double t0, int32_t nsteps,
                      int32_t active, void* stream)
{
    HS_CHECK(check_bound(P));
    if (lane < 0 || lane >= P->B || !(nu > 0) || !(dt > 0) || nsteps < 0 || !std::isfinite(t0))
        return HS_EINVAL;
    if (active && P->pb.lane_memory && !P->lane_base[lane]) return HS_ESTATE;   // no memory bound yet
    HS_TRY(hsk::set_lane(P->ctl, lane, nu, dt, t0, P->pb.forcing_c, nsteps, active ? 1 : 0,
                         (hipStream_t)stream));
    if (P->active[lane] != (active ? 1 : 0)) {
        P->active[lane] = active ? 1 : 0;
        P->run_dirty = true;
    }
    return HS_OK;
}

hs_status hs_lap_apply(hs_plan* P, int32_t level, double alpha, double beta, const double* d_u,
                       double* d_y, void* stream)
{
    HS_CHECK(check_bound(P));
    if (P->compact) return HS_EINVAL;   // operators of orders 2 and 4 only
    if (P->pb.lane_memory) return HS_EINVAL;
    if (level < 0 || level >= P->nlev || !d_u || !d_y) return HS_EINVAL;
    const Table<GridSeg>& T = P->all.mg64[level].fine;   // the lanes' finest grids, z-chunked
    HS_TRY(hsk::lap_apply(T.d, T.nseg(), T.nblk, P->order[level], alpha, beta, d_u, d_y,
                          P->offs[level].d, (hipStream_t)stream));
    return HS_OK;
}

hs_status hs_compact_apply(int32_t n, int32_t batch, double alpha, double beta, const double* d_u, double* d_y,
                           void* stream)
{
    if (!valid_n(n) || batch < 1 || batch > 65536 || !d_u || !d_y) return HS_EINVAL;
    if ((long long)batch * cube(n) > (1LL << 34)) return HS_EINVAL;
    HS_TRY(hsk::compact_apply(n, batch, alpha, beta, d_u, d_y, (hipStream_t)stream));
    return HS_OK;
}

hs_status hs_heat_rhs(hs_plan* P, int32_t level, const double* d_u, const double* h_t, double* d_fi,
                      double* d_fe, void* stream)
{
    HS_CHECK(check_bound(P));
    if (P->compact) return HS_EINVAL;   // operators of orders 2 and 4 only
    if (P->pb.lane_memory) return HS_EINVAL;
    if (level < 0 || level >= P->nlev || (d_fi && !d_u) || (d_fe && !h_t)) return HS_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    std::vector<double> t(P->B, 0.0);
    if (h_t)
        for (int b = 0; b < P->B; b++) t[b] = h_t[b];
    HS_TRY(hipMemcpyAsync(P->d_times, t.data(), sizeof(double) * P->B, hipMemcpyHostToDevice, s));
    const Table<GridSeg>& T = P->all.mg64[level].fine;   // same lanes, same order as all.sdc[level]
    HS_TRY(hsk::heat_rhs(P->ctl, T.d, P->all.sdc[level].d, T.nseg(), T.nblk, P->order[level], d_u, P->d_times,
                         d_fi, d_fe, P->offs[level].d, s));
    HS_TRY(hipStreamSynchronize(s));
    return HS_OK;
}

hs_status hs_mg_vcycle(hs_plan* P, int32_t level, const double* h_a, double* d_u, const double* d_b,
                       void* stream)
{
    HS_CHECK(check_bound(P));
    if (P->compact) return HS_EINVAL;   // operators of orders 2 and 4 only
    if (P->pb.lane_memory) return HS_EINVAL;
    if (level < 0 || level >= P->nlev || !h_a || !d_u || !d_b) return HS_EINVAL;
    for (int b = 0; b < P->B; b++)
        if (!(h_a[b] >= 0.0) || !std::isfinite(h_a[b])) return HS_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    // the solve runs in place on node 1 of the lanes' node arrays
    for (int b = 0; b < P->B; b++) {
        const LaneBufs& lb = P->lanes[b];
        long long N = lb.N[level], o = P->offs[level].h[b];
        HS_TRY(hipMemcpyAsync(lb.U[level] + N, d_u + o, N * sizeof(double), hipMemcpyDeviceToDevice, s));
        HS_TRY(hipMemcpyAsync(lb.rhs[level], d_b + o, N * sizeof(double), hipMemcpyDeviceToDevice, s));
        HS_TRY(hsk::set_a_user(P->ctl, b, h_a[b], s));
    }
    HS_CHECK(mg_solve(P, P->all, level, -1, 1, s, nullptr));
    for (int b = 0; b < P->B; b++) {
        const LaneBufs& lb = P->lanes[b];
        long long N = lb.N[level], o = P->offs[level].h[b];
        HS_TRY(hipMemcpyAsync(d_u + o, lb.U[level] + N, N * sizeof(double), hipMemcpyDeviceToDevice, s));
    }
    HS_CHECK(read_ctl(P, s));
    int worst = HS_OK;
    for (int b = 0; b < P->B; b++) {
        const LaneCtl& c = P->h_ctl[b];
        if (c.mg_state == 2) worst = std::min(worst, c.status < 0 ? c.status : (int)HS_ENOCONV);
        // stand-alone solves leave the lanes idle for the SDC driver
    }
    for (int b = 0; b < P->B; b++) P->h_ctl[b].status = 0;
    return (hs_status)worst;
}

hs_status hs_mg_solve_static(int32_t n, int32_t order, double a, const hs_mg_desc* mg, double* d_u,
                             const double* d_b, void* stream)
{
    if (!mg || !d_u || !d_b || !(a >= 0.0) || !std::isfinite(a)) return HS_EINVAL;
    if (mg->cycle_graphs != 0) return HS_EINVAL;   // graph capture would allocate
    hs_problem pb;
    std::memset(&pb, 0, sizeof(pb));
    pb.nu = 1.0;
    pb.dt = 1.0;
    pb.nlevels = 1;
    pb.lev[0].n = n;
    if (order != 2 && order != 4) return HS_EINVAL;
    pb.lev[0].order = order;
    pb.lev[0].nnodes = 2;
    pb.mg = *mg;
    pb.sweeps = 1;
    pb.sdc_tol = 1.0;
    pb.max_sweeps = 1;
    pb.batch = 1;
    pb.nslices = 1;
    HS_CHECK(validate(&pb));
    if (n > HS_STATIC_MAX_N) return HS_ENOMEM;
    hipStream_t s = (hipStream_t)stream;
    hs_plan P;
    init_plan(&P, &pb);
    P.solve_only = true;
    P.ext_u = d_u;
    P.ext_b = d_b;
    layout(&P, nullptr);
    if (P.bytes > HS_STATIC_SCRATCH_BYTES) return HS_ENOMEM;
    void* base = nullptr;
    HS_CHECK(scratch_address(&base));
    HS_TRY(ensure_constants());
    P.ws = (char*)base;
    layout(&P, P.ws);
    LaneCtl h_ctl;                                 // pageable host copy for the stopping checks
    P.h_ctl = &h_ctl;
    P.bound = true;
    // every call re-initialises what it reads: tables, the lane state (all of
    // its fields that a solve reads), the per-lane coefficient
    HS_TRY(upload_set(&P, P.all, s));
    HS_TRY(hsk::set_lane(P.ctl, 0, 1.0, 1.0, 0.0, 0.0, 0, 1, s));
    HS_TRY(hsk::set_a_user(P.ctl, 0, a, s));
    hs_status st = mg_solve(&P, P.all, 0, -1, 0, s, nullptr);
    if (st == HS_OK) st = read_ctl(&P, s);
    P.h_ctl = nullptr;
    if (st != HS_OK) return st;
    if (h_ctl.mg_state == 2) return h_ctl.status < 0 ? (hs_status)h_ctl.status : HS_ENOCONV;
    return HS_OK;
}

hs_status hs_smooth(hs_plan* P, int32_t level, const double* h_a, double* d_u, const double* d_b,
                    double* d_tmp, int32_t nsweeps, void* stream)
{
    HS_CHECK(check_bound(P));
    if (P->pb.lane_memory) return HS_EINVAL;
    if (level < 0 || level >= P->nlev || !h_a || !d_u || !d_b || !d_tmp || nsweeps < 0)
        return HS_EINVAL;
    for (int b = 0; b < P->B; b++)
        if (!(h_a[b] >= 0.0) || !std::isfinite(h_a[b])) return HS_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    if (P->user_key[0] != d_u || P->user_key[1] != d_b || P->user_key[2] != d_tmp ||
        P->user_level != level) {
        P->user.h.clear();
        int bk = 0;
        for (int b = 0; b < P->B; b++) {
            const LaneBufs& lb = P->lanes[b];
            long long o = P->offs[level].h[b];
            GridSeg g;
            std::memset(&g, 0, sizeof(g));
            g.lane = b;
            g.n = lb.n[level];
            g.u = d_u + o;
            g.t = d_tmp + o;
            g.b = (void*)(d_b + o);
            g.zb = hsk::choose_zb(g.n);
            g.blk_begin = bk;
            bk += hsk::grid_blocks(g.n, g.zb);
            P->user.h.push_back(g);
        }
        P->user.nblk = bk;
        HS_TRY(upload(P->user, s));
        P->user_key[0] = d_u; P->user_key[1] = d_b; P->user_key[2] = d_tmp;
        P->user_level = level;
    }
    for (int b = 0; b < P->B; b++) HS_TRY(hsk::set_a_user(P->ctl, b, h_a[b], s));
    hsk::MgArgs A{level, -1, P->pb.mg.omega, 0, 0};
    const Table<GridSeg>& T = P->user;
    for (int k = 0; k < nsweeps; k++)
        HS_TRY(hsk::sweep<double>(P->ctl, T.d, T.nseg(), T.nblk, P->order[level], A, 0, 0, k & 1, 1, 0, 0,
                                  P->partials, s));
    if (nsweeps & 1)
        for (int b = 0; b < P->B; b++) {
            long long o = P->offs[level].h[b];
            HS_TRY(hipMemcpyAsync(d_u + o, d_tmp + o, P->lanes[b].N[level] * sizeof(double),
                                  hipMemcpyDeviceToDevice, s));
        }
    return HS_OK;
}

hs_status hs_set_state(hs_plan* P, const double* d_u0, void* stream)
{
    HS_CHECK(check_bound(P));
    if (P->pb.lane_memory) return HS_EINVAL;
    if (!d_u0) return HS_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    int M = P->M[0];
    for (int b = 0; b < P->B; b++) {
        const LaneBufs& lb = P->lanes[b];
        long long N = lb.N[0];
        long long o = P->pb.nslices > 1 ? 0 : P->offs[0].h[b];
        HS_TRY(hipMemcpyAsync(lb.U[0] + (M - 1) * N, d_u0 + o, N * sizeof(double), hipMemcpyDeviceToDevice, s));
        double t0 = P->pb.t0, nsteps = P->pb.nsteps;
        if (P->pb.nslices > 1) {
            t0 = P->pb.t0 + b * P->pb.dt;
            nsteps = 1;
        }
        HS_TRY(hsk::set_lane(P->ctl, b, P->pb.nu, P->pb.dt, t0, P->pb.forcing_c, (int)nsteps, 1, s));
    }
    P->state_ready = 1;
    return HS_OK;
}

hs_status hs_set_lane_state(hs_plan* P, int32_t lane, const double* d_u0, void* stream)
{
    HS_CHECK(check_bound(P));
    if (lane < 0 || lane >= P->B || !d_u0 || P->pb.nslices > 1) return HS_EINVAL;
    if (P->pb.lane_memory && !P->lane_base[lane]) return HS_ESTATE;
    const LaneBufs& lb = P->lanes[lane];
    int M = P->M[0];
    HS_TRY(hipMemcpyAsync(lb.U[0] + (M - 1) * lb.N[0], d_u0, lb.N[0] * sizeof(double),
                          hipMemcpyDeviceToDevice, (hipStream_t)stream));
    return HS_OK;
}

hs_status hs_get_lane_state(hs_plan* P, int32_t lane, double* d_u, void* stream)
{
    HS_CHECK(check_bound(P));
    if (lane < 0 || lane >= P->B || !d_u || P->pb.nslices > 1) return HS_EINVAL;
    if (P->pb.lane_memory && !P->lane_base[lane]) return HS_ESTATE;
    const LaneBufs& lb = P->lanes[lane];
    int M = P->M[0];
    HS_TRY(hipMemcpyAsync(d_u, lb.U[0] + (M - 1) * lb.N[0], lb.N[0] * sizeof(double),
                          hipMemcpyDeviceToDevice, (hipStream_t)stream));
    return HS_OK;
}

hs_status hs_get_state(hs_plan* P, double* d_u, void* stream)
{
    HS_CHECK(check_bound(P));
    if (P->pb.lane_memory) return HS_EINVAL;
    if (!d_u) return HS_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    int M = P->M[0];
    if (P->pb.nslices > 1) {
        const LaneBufs& lb = P->lanes[P->B - 1];
        HS_TRY(hipMemcpyAsync(d_u, lb.U[0] + (M - 1) * lb.N[0], lb.N[0] * sizeof(double),
                              hipMemcpyDeviceToDevice, s));
        return HS_OK;
    }
    for (int b = 0; b < P->B; b++) {
        const LaneBufs& lb = P->lanes[b];
        HS_TRY(hipMemcpyAsync(d_u + P->offs[0].h[b], lb.U[0] + (M - 1) * lb.N[0], lb.N[0] * sizeof(double),
                              hipMemcpyDeviceToDevice, s));
    }
    return HS_OK;
}

hs_status hs_get_nodes(hs_plan* P, int32_t level, double* d_U, double* d_FI, double* d_Ut,
                       double* d_tau, void* stream)
{
    HS_CHECK(check_bound(P));
    if (P->pb.lane_memory) return HS_EINVAL;
    if (level < 0 || level >= P->nlev) return HS_EINVAL;
    if ((d_Ut || d_tau) && level < 1) return HS_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    int M = P->M[level];
    for (int b = 0; b < P->B; b++) {
        const LaneBufs& lb = P->lanes[b];
        long long sz = M * lb.N[level], o = M * P->offs[level].h[b];
        if (d_U) HS_TRY(hipMemcpyAsync(d_U + o, lb.U[level], sz * 8, hipMemcpyDeviceToDevice, s));
        if (d_FI) HS_TRY(hipMemcpyAsync(d_FI + o, lb.FI[level], sz * 8, hipMemcpyDeviceToDevice, s));
        if (d_Ut) HS_TRY(hipMemcpyAsync(d_Ut + o, lb.Ut[level], sz * 8, hipMemcpyDeviceToDevice, s));
        if (d_tau) HS_TRY(hipMemcpyAsync(d_tau + o, lb.tau[level], sz * 8, hipMemcpyDeviceToDevice, s));
    }
    return HS_OK;
}

hs_status hs_set_nodes(hs_plan* P, int32_t level, const double* d_U, const double* d_FI, void* stream)
{
    HS_CHECK(check_bound(P));
    if (P->pb.lane_memory) return HS_EINVAL;
    if (level < 0 || level >= P->nlev) return HS_EINVAL;
    if (P->compact && level == 0 && d_FI) return HS_EINVAL;   // its node array holds nu A_h U, set by the step
    hipStream_t s = (hipStream_t)stream;
    int M = P->M[level];
    for (int b = 0; b < P->B; b++) {
        const LaneBufs& lb = P->lanes[b];
        long long sz = M * lb.N[level], o = M * P->offs[level].h[b];
        if (d_U) HS_TRY(hipMemcpyAsync(lb.U[level], d_U + o, sz * 8, hipMemcpyDeviceToDevice, s));
        if (d_FI) HS_TRY(hipMemcpyAsync(lb.FI[level], d_FI + o, sz * 8, hipMemcpyDeviceToDevice, s));
    }
    return HS_OK;
}

hs_status hs_begin_step(hs_plan* P, void* stream)
{
    HS_CHECK(check_bound(P));
    return begin_step(P, (hipStream_t)stream);
}

hs_status hs_sdc_sweep(hs_plan* P, int32_t level, void* stream)
{
    HS_CHECK(check_bound(P));
    if (level < 0 || level >= P->nlev) return HS_EINVAL;
    int outcome;
    HS_CHECK(refresh_run(P, (hipStream_t)stream));
    if (P->compact && level == 0) return cmp_sweep_all(P, (hipStream_t)stream);
    return sweep(P, P->run, level, false, level == 0, (hipStream_t)stream, &outcome);
}

hs_status hs_fas_restrict(hs_plan* P, void* stream)
{
    HS_CHECK(check_bound(P));
    if (P->nlev < 2 || P->compact) return HS_EINVAL;   // compact: inside hs_mlsdc_iter only
    HS_CHECK(refresh_run(P, (hipStream_t)stream));
    HS_TRY(fas_restrict(P, P->run, 0, (hipStream_t)stream));
    return HS_OK;
}

hs_status hs_fas_interp(hs_plan* P, void* stream)
{
    HS_CHECK(check_bound(P));
    if (P->nlev < 2 || P->compact) return HS_EINVAL;   // compact: inside hs_mlsdc_iter only
    hipStream_t s = (hipStream_t)stream;
    HS_CHECK(refresh_run(P, s));
    HS_TRY(interp_level(P, P->run, 0, s));
    return HS_OK;
}

hs_status hs_mlsdc_iter(hs_plan* P, void* stream)
{
    HS_CHECK(check_bound(P));
    if (P->nlev < 2) return HS_EINVAL;
    int outcome;
    HS_CHECK(refresh_run(P, (hipStream_t)stream));
    if (P->compact) return cmp_mlsdc_iter(P, (hipStream_t)stream);
    return mlsdc_iter(P, P->run, false, (hipStream_t)stream, &outcome);
}

hs_status hs_end_step(hs_plan* P, void* stream)
{
    HS_CHECK(check_bound(P));
    HS_TRY(hsk::end_step(P->ctl, P->B, (hipStream_t)stream));
    return HS_OK;
}

hs_status hs_step(hs_plan* P, void* stream)
{
    HS_CHECK(check_bound(P));
    if (P->pb.nslices > 1) return HS_EINVAL;
    return step(P, (hipStream_t)stream);
}

hs_status hs_solve(hs_plan* P, void* stream)
{
    HS_CHECK(check_bound(P));
    if (P->pb.nslices > 1) return hs_pfasst_run(P, stream);
    hipStream_t s = (hipStream_t)stream;
    for (int k = 0; k < P->pb.nsteps; k++) HS_CHECK(step(P, s));
    return HS_OK;
}

hs_status hs_solve_graph(hs_plan* P, void* stream)
{
    HS_CHECK(check_bound(P));
    if (P->pb.lane_memory) return HS_EINVAL;
    if (P->compact) return HS_EINVAL;
    if (P->pb.nslices > 1 || P->pb.sweeps <= 0 || P->pb.mg.fixed_cycles <= 0) return HS_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    // table uploads are not allowed inside a capture: bring them up to date first
    HS_CHECK(refresh_run(P, s));
    if (!P->gexec) {
        HS_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        hs_status st = step(P, s);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(s, &g);
        if (st != HS_OK || e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            (void)hipGetLastError();
            return st != HS_OK ? st : HS_EDEVICE;
        }
        HS_TRY(e);
        P->graph = g;
        HS_TRY(hipGraphInstantiate(&P->gexec, P->graph, nullptr, nullptr, 0));
    }
    if (P->run_dirty) return HS_ESTATE;   // lanes changed since the graph was captured
    for (int k = 0; k < P->pb.nsteps; k++) HS_TRY(hipGraphLaunch(P->gexec, s));
    return HS_OK;
}

}  // extern "C"

namespace {
__global__ void k_pfasst_block(LaneCtl* ctl, int P, double t0, double dt, int blk)
{
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    ctl[p].t0 = t0 + (double)(blk * P + p) * dt;
    ctl[p].step = 0;
    ctl[p].nsteps = 1;
}
}  // namespace

namespace {

// Coarse predictor of PFASST (see hs_pfasst_run): restriction of the spread
// fine values down to the coarsest level, that level run serially through the
// slices without the FAS correction, interpolation of the coarse correction
// level by level back to the finest.
hs_status pfasst_predictor(hs_plan* P, hipStream_t s)
{
    LaneSet& all = P->all;
    const int C = P->nlev - 1;
    for (int l = 0; l < C; l++) HS_TRY(fas_restrict(P, all, l, s));
    for (int b = 0; b < P->B; b++)
        HS_TRY(hsk::fill(P->lanes[b].tau[C], (long long)P->M[C] * P->lanes[b].N[C], 0.0, s));
    int outcome;
    for (int p = 0; p < P->B; p++) {
        if (p > 0) {
            // slice p's coarse step starts from slice p-1's coarse end value, spread over its nodes
            HS_TRY(hsk::handoff(P->ctl, P->hc_dst[p].d, P->hc_src[p].d, 1, P->hc_dst[p].nblk, P->order[C], s));
            const Table<SdcSeg>& T = P->single[p].sdc[C];
            HS_TRY(hsk::spread(P->ctl, T.d, T.nseg(), T.nblk, P->order[C], 0, s));
        }
        for (int j = 0; j < P->pb.pfasst_pred_sweeps; j++) HS_CHECK(sweep(P, P->single[p], C, false, false, s, &outcome));
    }
    for (int l = C - 1; l >= 0; l--) HS_TRY(interp_level(P, all, l, s));
    return HS_OK;
}

// Hand-shake of the two threads that issue a pipelined PFASST run: each
// side counts what it has recorded (a group's restriction, a group's coarse
// sweeps, a block's start); the other side waits on the host for the count it
// needs before it makes its stream wait on the event.  An event is recorded
// again only after the other side's stream wait on its previous record has
// been issued: each side's next record depends on what the other posts after
// that wait.
struct PipeSync {
    std::mutex mu;
    std::condition_variable cv;
    std::vector<int> r, c;
    int go = 0;
    bool abort = false;
    hs_status first = HS_OK;   // the failure that stopped the run
    void post(int& count)
    {
        {
            std::lock_guard<std::mutex> lk(mu);
            count++;
        }
        cv.notify_all();
    }
    // false when the other side has given up
    bool wait(const int& count, int need)
    {
        std::unique_lock<std::mutex> lk(mu);
        cv.wait(lk, [&] { return abort || count >= need; });
        return count >= need;
    }
    // a side that fails stops both; a wait that returns false reports HS_ESTATE
    void stop(hs_status st)
    {
        {
            std::lock_guard<std::mutex> lk(mu);
            if (!abort) first = st;
            abort = true;
        }
        cv.notify_all();
    }
};

// The end values of a group's last slice that the next group's hand-offs read.
hipError_t snapshot(hs_plan* P, int g, int L, hipStream_t s)
{
    const LaneBufs& lb = P->lanes[(g + 1) * (P->B / P->G) - 1];
    double* dst = L == 0 ? P->snap_f[g] : P->snap_c[g];
    return hipMemcpyAsync(dst, lb.U[L] + (long long)(P->M[L] - 1) * lb.N[L], lb.N[L] * sizeof(double),
                          hipMemcpyDeviceToDevice, s);
}

// Coarse side of a pipelined PFASST run (its own thread, stream P->pipe):
// per block the predictor's serial coarse sweeps, then per iteration and
// group, once the group's restriction is done, the coarse pipeline through
// the group's slices.
hs_status pipe_coarse(hs_plan* P, PipeSync& ps, int nblocks)
{
    hipStream_t c = P->pipe;
    HS_TRY(hipSetDevice(P->device));
    const int G = P->G, Q = P->B / G, K = P->pb.sweeps, pred = P->pb.pfasst_pred_sweeps;
    std::vector<int> got_r(G, 0);
    auto chain = [&](int g, bool predictor) -> hs_status {
        int outcome;
        for (int p = g * Q; p < (g + 1) * Q; p++) {
            if (p > 0) {
                // slice p's coarse start: slice p-1's end value (across a group boundary, its copy)
                const Table<SdcSeg>& src = p == g * Q ? P->gc_src[g] : P->hc_src[p];
                HS_TRY(hsk::handoff(P->ctl, P->hc_dst[p].d, src.d, 1, P->hc_dst[p].nblk, P->order[1], c));
                if (predictor) {
                    const Table<SdcSeg>& T = P->single[p].sdc[1];
                    HS_TRY(hsk::spread(P->ctl, T.d, T.nseg(), T.nblk, P->order[1], 0, c));
                }
            }
            for (int j = 0; j < (predictor ? pred : 1); j++)
                HS_CHECK(sweep(P, P->single[p], 1, false, false, c, &outcome));
        }
        if (g + 1 < G) HS_TRY(snapshot(P, g, 1, c));
        HS_TRY(hipEventRecord(P->ev_c[g], c));
        ps.post(ps.c[g]);
        return HS_OK;
    };
    for (int blk = 0; blk < nblocks; blk++) {
        if (!ps.wait(ps.go, blk + 1)) return HS_ESTATE;
        HS_TRY(hipStreamWaitEvent(c, P->ev_go, 0));
        P->sweep_k2 = 0;
        if (pred > 0)
            for (int g = 0; g < G; g++) HS_CHECK(chain(g, true));
        for (int k = 0; k < K; k++) {
            P->sweep_k2 = k;
            for (int g = 0; g < G; g++) {
                if (!ps.wait(ps.r[g], ++got_r[g])) return HS_ESTATE;
                HS_TRY(hipStreamWaitEvent(c, P->ev_r[g], 0));
                HS_CHECK(chain(g, false));
            }
        }
    }
    return HS_OK;
}

// Fine side of a pipelined PFASST run (the caller's thread and stream): per
// iteration and group, once the group's coarse sweeps of the previous
// iteration (or of the predictor) are done, their interpolation, the copy of
// the group's last end value for the next group, the group's fine hand-off,
// its fine sweeps as one batch and its restriction.
hs_status pipe_fine(hs_plan* P, PipeSync& ps, int nblocks, hipStream_t s)
{
    const int G = P->G, K = P->pb.sweeps, Mf = P->M[0];
    const bool pred = P->pb.pfasst_pred_sweeps > 0;
    std::vector<int> got_c(G, 0);
    auto interp = [&](int g) -> hs_status {
        if (!ps.wait(ps.c[g], ++got_c[g])) return HS_ESTATE;
        HS_TRY(hipStreamWaitEvent(s, P->ev_c[g], 0));
        HS_TRY(interp_level(P, P->grp[g], 0, s));
        return HS_OK;
    };
    for (int blk = 0; blk < nblocks; blk++) {
        if (blk > 0) {
            // the next block starts from the last slice's end value
            const LaneBufs& last = P->lanes[P->B - 1];
            for (int p = 0; p + 1 < P->B; p++) {
                const LaneBufs& lb = P->lanes[p];
                HS_TRY(hipMemcpyAsync(lb.U[0] + (Mf - 1) * lb.N[0], last.U[0] + (Mf - 1) * last.N[0],
                                      lb.N[0] * 8, hipMemcpyDeviceToDevice, s));
            }
        }
        hipLaunchKernelGGL(k_pfasst_block, dim3((P->B + 63) / 64), dim3(64), 0, s, P->ctl, P->B, P->pb.t0,
                           P->pb.dt, blk);
        HS_TRY(hipGetLastError());
        HS_CHECK(begin_step(P, s));
        if (pred) {
            // the predictor's restriction of the spread values, without the FAS correction
            HS_TRY(fas_restrict(P, P->all, 0, s));
            for (int b = 0; b < P->B; b++)
                HS_TRY(hsk::fill(P->lanes[b].tau[1], (long long)P->M[1] * P->lanes[b].N[1], 0.0, s));
        }
        HS_TRY(hipEventRecord(P->ev_go, s));
        ps.post(ps.go);
        for (int k = 0; k < K; k++) {
            for (int g = 0; g < G; g++) {
                LaneSet& gs = P->grp[g];
                if (pred || k > 0) HS_CHECK(interp(g));
                if (g + 1 < G) HS_TRY(snapshot(P, g, 0, s));
                if (P->gh_dst[g].nseg() > 0)
                    HS_TRY(hsk::handoff(P->ctl, P->gh_dst[g].d, P->gh_src[g].d, P->gh_dst[g].nseg(),
                                        P->gh_dst[g].nblk, P->order[0], s));
                int outcome;
                HS_CHECK(sweep(P, gs, 0, false, true, s, &outcome));
                HS_TRY(fas_restrict(P, gs, 0, s));
                HS_TRY(hipEventRecord(P->ev_r[g], s));
                ps.post(ps.r[g]);
            }
            P->sweep_k++;
        }
        for (int g = 0; g < G; g++) HS_CHECK(interp(g));
        HS_TRY(hsk::end_step(P->ctl, P->B, s));
    }
    return HS_OK;
}

hs_status pfasst_pipelined(hs_plan* P, int nblocks, hipStream_t s)
{
    PipeSync ps;
    ps.r.assign(P->G, 0);
    ps.c.assign(P->G, 0);
    std::thread worker;
    try {
        worker = std::thread([&] {
            hs_status st = pipe_coarse(P, ps, nblocks);
            if (st != HS_OK) ps.stop(st);
        });
    } catch (...) {
        return HS_EDEVICE;
    }
    hs_status st = pipe_fine(P, ps, nblocks, s);
    if (st != HS_OK) ps.stop(st);
    worker.join();
    return ps.abort ? ps.first : HS_OK;
}

}  // namespace

extern "C" hs_status hs_pfasst_run(hs_plan* P, void* stream)
{
    HS_CHECK(check_bound(P));
    if (P->pb.lane_memory) return HS_EINVAL;
    if (P->pb.nslices <= 1) return HS_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    if (P->G >= 2) return pfasst_pipelined(P, P->pb.nsteps / P->B, s);
    int Pn = P->B, Mf = P->M[0];
    const int C = P->nlev - 1;   // the coarsest level
    int nblocks = P->pb.nsteps / Pn;
    const bool fixed = P->pb.sweeps > 0;
    LaneSet& all = P->all;
    for (int blk = 0; blk < nblocks; blk++) {
        if (blk > 0) {
            // the next block starts from the last slice's end value
            const LaneBufs& last = P->lanes[Pn - 1];
            for (int p = 0; p + 1 < Pn; p++) {
                const LaneBufs& lb = P->lanes[p];
                HS_TRY(hipMemcpyAsync(lb.U[0] + (Mf - 1) * lb.N[0], last.U[0] + (Mf - 1) * last.N[0],
                                      lb.N[0] * 8, hipMemcpyDeviceToDevice, s));
            }
        }
        hipLaunchKernelGGL(k_pfasst_block, dim3((Pn + 63) / 64), dim3(64), 0, s, P->ctl, Pn,
                           P->pb.t0, P->pb.dt, blk);
        HS_TRY(hipGetLastError());
        HS_CHECK(begin_step(P, s));
        if (P->pb.pfasst_pred_sweeps > 0) HS_CHECK(pfasst_predictor(P, s));
        for (int k = 0;; k++) {
            if (fixed && k >= P->pb.sweeps) break;
            // (i) fine hand-off from the previous iteration
            HS_TRY(hsk::handoff(P->ctl, P->hf_dst.d, P->hf_src.d, P->hf_dst.nseg(), P->hf_dst.nblk,
                                P->order[0], s));
            bool prep_done = false;
            if (!fixed) {
                // every slice's collocation residual after the hand-off (formed with the
                // sweep's constant parts); stop when all meet sdc_tol
                const Table<SdcSeg>& T = all.sdc[0];
                HS_TRY(hsk::sweep_prep(P->ctl, T.d, T.nseg(), T.nblk, 1, 1, P->partials, s));
                HS_TRY(hsk::sdc_decide(P->ctl, T.d, T.nseg(), T.nblk, P->partials, P->pb.sdc_tol,
                                       P->pb.max_sweeps, s));
                HS_CHECK(read_ctl(P, s));
                bool done = true, failed = false;
                for (int b = 0; b < Pn; b++) {
                    int st = P->h_ctl[b].sdc_state;
                    if (st == 0) done = false;
                    if (st == 2) failed = true;
                }
                if (done || failed) break;   // a failure is recorded in the lanes' status
                HS_TRY(hsk::sdc_reopen(P->ctl, P->B, s));
                prep_done = true;
            }
            int outcome;
            HS_CHECK(sweep(P, all, 0, false, true, s, &outcome, prep_done));
            // (ii) restriction and FAS correction on every slice, level by level down to
            // the coarsest, with a sweep of every slice on each intermediate level
            for (int l = 0; l < C; l++) {
                HS_TRY(fas_restrict(P, all, l, s));
                if (l + 1 < C) HS_CHECK(sweep(P, all, l + 1, false, false, s, &outcome));
            }
            // (iii) coarse pipeline: slice p starts from slice p-1's new coarse end value
            for (int p = 0; p < Pn; p++) {
                if (p > 0)
                    HS_TRY(hsk::handoff(P->ctl, P->hc_dst[p].d, P->hc_src[p].d, 1, P->hc_dst[p].nblk,
                                        P->order[C], s));
                HS_CHECK(sweep(P, P->single[p], C, false, false, s, &outcome));
            }
            // (iv) interpolation on every slice, node 0 included, level by level up to
            // the finest, with a sweep of every slice on each intermediate level
            for (int l = C - 1; l >= 0; l--) {
                HS_TRY(interp_level(P, all, l, s));
                if (l > 0) HS_CHECK(sweep(P, all, l, false, false, s, &outcome));
            }
            P->sweep_k++;
        }
        HS_TRY(hsk::end_step(P->ctl, P->B, s));
    }
    return HS_OK;
}

extern "C" hs_status hs_plan_timer(hs_plan* P, int32_t kind, int32_t max_launches)
{
    HS_CHECK(check_bound(P));
    const int base = kind & ~HS_TIMER_FP32;
    if (kind < 0 || (kind != 0 && (base < HS_TIMER_PJAC || base > HS_TIMER_SWEEP2)) || max_launches < 0 ||
        max_launches > 65536)
        return HS_EINVAL;
    HS_TRY(hipDeviceSynchronize());   // no timed launch may still use the old events
    for (hipEvent_t e : P->timer_ev) (void)hipEventDestroy(e);
    P->timer_ev.clear();
    P->timer_used = 0;
    P->timer_kind = 0;
    if (kind == 0 || max_launches == 0) return HS_OK;
    for (int i = 0; i < 2 * max_launches; i++) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) {
            for (hipEvent_t x : P->timer_ev) (void)hipEventDestroy(x);
            P->timer_ev.clear();
            return HS_EDEVICE;
        }
        P->timer_ev.push_back(e);
    }
    P->timer_kind = kind;
    return HS_OK;
}

extern "C" hs_status hs_plan_timer_read(hs_plan* P, int32_t* launches, double* total_ms)
{
    HS_CHECK(check_bound(P));
    if (!launches || !total_ms) return HS_EINVAL;
    double ms = 0.0;
    for (int i = 0; i < P->timer_used; i++) {
        HS_TRY(hipEventSynchronize(P->timer_ev[2 * i + 1]));
        float t = 0.0f;
        HS_TRY(hipEventElapsedTime(&t, P->timer_ev[2 * i], P->timer_ev[2 * i + 1]));
        ms += t;
    }
    *launches = P->timer_used;
    *total_ms = ms;
    P->timer_used = 0;
    return HS_OK;
}

namespace {

// Integer fields of the flat objects of a tuning file: every {...} that has no
// nested object gives one map of "key": number pairs.
std::vector<std::map<std::string, long long>> parse_flat_objects(const std::string& t)
{
    std::vector<std::map<std::string, long long>> out;
    size_t i = 0;
    while ((i = t.find('{', i)) != std::string::npos) {
        size_t j = t.find_first_of("{}", i + 1);
        if (j == std::string::npos) break;
        if (t[j] == '{') {   // nested: the inner object is scanned next
            i = j;
            continue;
        }
        std::map<std::string, long long> obj;
        size_t k = i + 1;
        while (true) {
            size_t q0 = t.find('"', k);
            if (q0 == std::string::npos || q0 > j) break;
            size_t q1 = t.find('"', q0 + 1);
            if (q1 == std::string::npos || q1 > j) break;
            std::string key = t.substr(q0 + 1, q1 - q0 - 1);
            size_t c = t.find_first_not_of(" \t\r\n", q1 + 1);
            if (c == std::string::npos || c > j || t[c] != ':') { k = q1 + 1; continue; }
            size_t v = t.find_first_not_of(" \t\r\n", c + 1);
            if (v == std::string::npos || v > j) break;
            char* end = nullptr;
            long long val = std::strtoll(t.c_str() + v, &end, 10);
            size_t e = end ? (size_t)(end - t.c_str()) : v;
            if (e > v && e <= j && (t[e] == ',' || t[e] == '}' || t[e] == ' ' || t[e] == '\n' || t[e] == '\r' ||
                                   t[e] == '\t'))
                obj[key] = val;
            // skip the value (a string may hold commas)
            if (t[v] == '"') {
                size_t s1 = t.find('"', v + 1);
                k = s1 == std::string::npos ? j : s1 + 1;
            } else {
                k = e > v ? e : v + 1;
            }
        }
        out.push_back(obj);
        i = j + 1;
    }
    return out;
}

}  // namespace

extern "C" hs_status hs_tune_set(int32_t n, int32_t order, int32_t precision, int32_t batch, int32_t zb,
                                 int32_t zb_rfw)
{
    if (!valid_tune(n, order, precision, batch, zb, zb_rfw)) return HS_EINVAL;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (TuneEntry& e : g_tune)
        if (e.n == n && e.order == order && e.prec == precision && e.batch == batch) {
            e.zb = zb;
            e.zb_rfw = zb_rfw;
            return HS_OK;
        }
    g_tune.push_back({n, order, precision, batch, zb, zb_rfw});
    return HS_OK;
}

extern "C" hs_status hs_tune_clear(void)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.clear();
    return HS_OK;
}

extern "C" hs_status hs_tune_load(const char* json_path, int32_t* entries)
{
    if (!json_path) return HS_EINVAL;
    FILE* f = std::fopen(json_path, "rb");
    if (!f) return HS_EINVAL;
    std::string text;
    char buf[4096];
    size_t got;
    while ((got = std::fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, got);
    std::fclose(f);
    int count = 0;
    static const char* keys[] = {"n", "order", "precision", "batch", "zb", "zb_rfw"};
    for (const auto& obj : parse_flat_objects(text)) {
        bool all = true;
        for (const char* k : keys) all = all && obj.count(k);
        if (!all) continue;
        hs_status st = hs_tune_set((int)obj.at("n"), (int)obj.at("order"), (int)obj.at("precision"),
                                   (int)obj.at("batch"), (int)obj.at("zb"), (int)obj.at("zb_rfw"));
        if (st != HS_OK) return st;
        count++;
    }
    if (entries) *entries = count;
    return HS_OK;
}

extern "C" hs_status hs_tune_lookup(int32_t n, int32_t order, int32_t precision, int32_t batch, int32_t* zb,
                                    int32_t* zb_rfw)
{
    if (!zb || !zb_rfw || !valid_tune(n, order, precision, batch < 1 ? 1 : batch, 1, 2)) return HS_EINVAL;
    int a = 0, b = 0;
    tuned_zb(n, order, precision, batch, &a, &b);
    *zb = a;
    *zb_rfw = b;
    return HS_OK;
}

extern "C" hs_status hs_stats_read(hs_plan* P, hs_lane_stats* out, void* stream)
{
    HS_CHECK(check_bound(P));
    if (!out) return HS_EINVAL;
    HS_CHECK(read_ctl(P, (hipStream_t)stream));
    // a node-parallel lane's solves are done by its solver lanes
    for (int sl = P->B; sl < P->nctl; sl++) {
        const LaneCtl& c = P->h_ctl[sl];
        LaneCtl& p = P->h_ctl[c.parent];
        p.total_cycles += c.total_cycles;
        p.total_solves += c.total_solves;
        p.failed_solves += c.failed_solves;
        p.max_cycles = std::max(p.max_cycles, c.max_cycles);
        p.level_cycles[0] += c.level_cycles[0];
        p.mg_rho = std::max(p.mg_rho, c.mg_rho);
        if (c.status < p.status) p.status = c.status;
    }
    for (int b = 0; b < P->B; b++) {
        const LaneCtl& c = P->h_ctl[b];
        hs_lane_stats& o = out[b];
        o.status = c.status;
        o.steps_done = c.step;
        o.total_sweeps = c.total_sweeps;
        o.total_solves = c.total_solves;
        o.total_cycles = c.total_cycles;
        o.max_cycles = c.max_cycles;
        o.failed_solves = c.failed_solves;
        o.last_rho = c.mg_rho;
        o.last_sdc_res = c.sdc_res;
        for (int l = 0; l < HS_MAXLEV; l++) o.level_cycles[l] = c.level_cycles[l];
    }
    return lanes_status(P);
}
