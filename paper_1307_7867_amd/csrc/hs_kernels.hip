// HIP kernels of libheatst for gfx950 (MI355X).
//
// Every kernel of the multigrid and SDC hot path works on a table of
// segments: one segment is one grid of one lane (an independent problem or
// a PFASST time slice).  Blocks of 256 threads tile a grid as 64 x 4 points
// in x-y (one wavefront per x row, coalesced along x) and one z plane per
// block; a launch covers all segments of its table, so lanes of equal or of
// different sizes share one launch.  The hardware hands consecutive blocks
// to the 8 XCDs in turn; the block index is remapped so that every XCD works
// on one contiguous range of planes and reuses the z-neighbour planes from
// its own L2.
//
// The discrete operators follow the paper's section 1 (method of lines,
// 2nd- and 4th-order Laplacians, implicit-Euler substeps of the IMEX SDC
// sweep of eq. (7)) and section 1.2 (multigrid); the multigrid components
// (weighted Jacobi, full weighting, trilinear prolongation, exact solve on
// the coarsest grid) are this library's choice, the paper names none.
#include "hs_internal.h"

#include <math.h>

namespace {

__constant__ LibConst c_lc;

constexpr int XCDS = 8;

__device__ __forceinline__ int xcd_remap(int bid, int nblk)
{
    int q = nblk / XCDS, r = nblk % XCDS;
    int x = bid % XCDS, j = bid / XCDS;
    return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + j;
}

template <typename S>
__device__ __forceinline__ int find_seg(const S* segs, int nseg, int lb)
{
    int lo = 0, hi = nseg - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (segs[mid].blk_begin <= lb) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__host__ __device__ __forceinline__ int tiles_x(int n) { return (n + HS_TX - 1) / HS_TX; }
__host__ __device__ __forceinline__ int tiles_y(int n) { return (n + HS_TY - 1) / HS_TY; }

// position of this thread inside its segment's grid
struct Pos {
    int i, j, k;
    bool in;
};

__device__ __forceinline__ Pos grid_pos(int rel_blk, int n)
{
    int tx = tiles_x(n), ty = tiles_y(n);
    int bx = rel_blk % tx;
    int rest = rel_blk / tx;
    int by = rest % ty;
    int bz = rest / ty;
    Pos p;
    p.i = bx * HS_TX + (int)(threadIdx.x % HS_TX);
    p.j = by * HS_TY + (int)(threadIdx.x / HS_TX);
    p.k = bz;
    p.in = p.i < n && p.j < n && p.k < n;
    return p;
}

__device__ __forceinline__ long long lin(int i, int j, int k, int n)
{
    return ((long long)k * n + j) * n + i;
}

// Sum over the three axes of the un-scaled 1-D stencils at point p:
// order 2: u(-1) - 2 u(0) + u(+1); order 4: -u(-2) + 16 u(-1) - 30 u(0)
// + 16 u(+1) - u(+2), with u = 0 on the walls and the odd reflection
// u(-2) = -u(0), u(n+1) = -u(n-1) one point beyond them.  L_h u is this sum
// times 1/h^2 (order 2) or 1/(12 h^2) (order 4).
template <int ORDER, typename T, typename Ld>
__device__ __forceinline__ T lap_sum(const Ld& ld, int i, int j, int k, int n, T c)
{
    const T zero = T(0);
    if (ORDER == 2) {
        T xm = i > 0 ? ld(i - 1, j, k) : zero;
        T xp = i < n - 1 ? ld(i + 1, j, k) : zero;
        T ym = j > 0 ? ld(i, j - 1, k) : zero;
        T yp = j < n - 1 ? ld(i, j + 1, k) : zero;
        T zm = k > 0 ? ld(i, j, k - 1) : zero;
        T zp = k < n - 1 ? ld(i, j, k + 1) : zero;
        T c2 = T(2) * c;
        return ((xm - c2) + xp) + ((ym - c2) + yp) + ((zm - c2) + zp);
    } else {
        T ax, ay, az;
        {
            T m1 = i >= 1 ? ld(i - 1, j, k) : zero;
            T m2 = i >= 2 ? ld(i - 2, j, k) : (i == 1 ? zero : -c);
            T p1 = i <= n - 2 ? ld(i + 1, j, k) : zero;
            T p2 = i <= n - 3 ? ld(i + 2, j, k) : (i == n - 2 ? zero : -c);
            ax = (T(16) * (m1 + p1) - (m2 + p2)) - T(30) * c;
        }
        {
            T m1 = j >= 1 ? ld(i, j - 1, k) : zero;
            T m2 = j >= 2 ? ld(i, j - 2, k) : (j == 1 ? zero : -c);
            T p1 = j <= n - 2 ? ld(i, j + 1, k) : zero;
            T p2 = j <= n - 3 ? ld(i, j + 2, k) : (j == n - 2 ? zero : -c);
            ay = (T(16) * (m1 + p1) - (m2 + p2)) - T(30) * c;
        }
        {
            T m1 = k >= 1 ? ld(i, j, k - 1) : zero;
            T m2 = k >= 2 ? ld(i, j, k - 2) : (k == 1 ? zero : -c);
            T p1 = k <= n - 2 ? ld(i, j, k + 1) : zero;
            T p2 = k <= n - 3 ? ld(i, j, k + 2) : (k == n - 2 ? zero : -c);
            az = (T(16) * (m1 + p1) - (m2 + p2)) - T(30) * c;
        }
        return (ax + ay) + az;
    }
}

// scale that turns lap_sum into L_h u
template <int ORDER, typename T>
__device__ __forceinline__ T lap_scale(int n)
{
    T ih2 = T((double)(n + 1) * (double)(n + 1));
    return ORDER == 2 ? ih2 : ih2 / T(12);
}

// diagonal of A_a = I - a L_h at (i,j,k)
template <int ORDER, typename T>
__device__ __forceinline__ T diag_A(T a, int i, int j, int k, int n)
{
    T ih2 = T((double)(n + 1) * (double)(n + 1));
    if (ORDER == 2) return T(1) + a * ih2 * T(6);
    int walls = (i == 0) + (i == n - 1) + (j == 0) + (j == n - 1) + (k == 0) + (k == n - 1);
    return T(1) + a * ih2 * (T(90 - walls) / T(12));
}

template <typename T>
struct Ld3 {
    const T* __restrict__ u;
    int n;
    __device__ __forceinline__ T operator()(int i, int j, int k) const { return u[lin(i, j, k, n)]; }
};

// coarse-grid view of a fine field by injection: coarse (I,J,K) is fine (2I+1, 2J+1, 2K+1)
struct LdInj {
    const double* __restrict__ uf;
    int nf;
    __device__ __forceinline__ double operator()(int I, int J, int K) const
    {
        return uf[lin(2 * I + 1, 2 * J + 1, 2 * K + 1, nf)];
    }
};

__device__ __forceinline__ double lane_a(const LaneCtl* ctl, int lane, int L, int m)
{
    return m >= 0 ? ctl[lane].a[L][m] : ctl[lane].a_user;
}

// max that keeps NaN
template <typename T>
__device__ __forceinline__ T nmax(T a, T b) { return (b > a || b != b) ? b : a; }

__device__ __forceinline__ unsigned long long dbits(double x)
{
    return (unsigned long long)__double_as_longlong(x);
}

__device__ __forceinline__ double bitsd(unsigned long long x)
{
    return __longlong_as_double((long long)x);
}

// block-wide max; result valid in thread 0.  All threads must call it.
__device__ __forceinline__ double block_max(double v)
{
    __shared__ double sm[HS_BLOCK / 64 > 16 ? HS_BLOCK / 64 : 16];
    for (int off = 32; off > 0; off >>= 1) v = nmax(v, __shfl_xor(v, off, 64));
    int w = threadIdx.x / 64, l = threadIdx.x % 64;
    __syncthreads();
    if (l == 0) sm[w] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        int nw = (blockDim.x + 63) / 64;
        for (int q = 1; q < nw; q++) v = nmax(v, sm[q]);
    }
    return v;
}

// Accumulate a block's maximum into *acc and report whether this block is
// the last of `nblk_seg` blocks to do so (then *acc holds the final value).
__device__ __forceinline__ bool seg_reduce_last(double v, unsigned long long* acc, uint32_t* cnt,
                                                int nblk_seg, unsigned long long* acc2 = nullptr,
                                                double v2 = 0.0)
{
    __shared__ int last;
    double m = block_max(v);
    double m2 = acc2 ? block_max(v2) : 0.0;
    if (threadIdx.x == 0) {
        atomicMax(acc, dbits(m));
        if (acc2) atomicMax(acc2, dbits(m2));
        __threadfence();
        unsigned prev = atomicAdd(cnt, 1u);
        last = (prev == (unsigned)nblk_seg - 1u);
    }
    __syncthreads();
    return last != 0;
}

template <typename S>
__device__ __forceinline__ int seg_nblk(const S* segs, int nseg, int si, int nblk)
{
    return (si + 1 < nseg ? segs[si + 1].blk_begin : nblk) - segs[si].blk_begin;
}

// ---------------------------------------------------------------------------
// Multigrid kernels
// ---------------------------------------------------------------------------

// Weighted Jacobi: dst = src + omega D^{-1} (b - A_a src); from a zero guess
// dst = omega D^{-1} b.
template <typename T, int ORDER>
__global__ void __launch_bounds__(HS_BLOCK) k_jacobi(const GridSeg* __restrict__ segs, int nseg,
                                                     int nblk, const LaneCtl* __restrict__ ctl,
                                                     hsk::MgArgs A, int first_sweep, int src_is_t)
{
    int lb = xcd_remap(blockIdx.x, nblk);
    int si = find_seg(segs, nseg, lb);
    const GridSeg sg = segs[si];
    if (A.gate && ctl[sg.lane].mg_state != 0) return;
    int n = sg.n;
    Pos q = grid_pos(lb - sg.blk_begin, n);
    if (!q.in) return;
    T* U = (T*)sg.u + (long long)A.node * sg.node_stride;
    T* Tt = (T*)sg.t;
    const T* B = (const T*)sg.b;
    T* src = src_is_t ? Tt : U;
    T* dst = src_is_t ? U : Tt;
    T a = T(lane_a(ctl, sg.lane, A.L, A.m));
    T om = T(A.omega);
    long long p = lin(q.i, q.j, q.k, n);
    T D = diag_A<ORDER, T>(a, q.i, q.j, q.k, n);
    if (first_sweep && sg.coarse) {
        dst[p] = om * B[p] / D;
        return;
    }
    Ld3<T> ld{src, n};
    T c = src[p];
    T Au = c - a * (lap_scale<ORDER, T>(n) * lap_sum<ORDER, T>(ld, q.i, q.j, q.k, n, c));
    dst[p] = c + om * (B[p] - Au) / D;
}

// r = b - A_a u at fine point (i,j,k)
template <typename T, int ORDER>
__device__ __forceinline__ T resid_at(const T* __restrict__ u, const T* __restrict__ b, T a, T sc,
                                      int i, int j, int k, int n)
{
    long long p = lin(i, j, k, n);
    T c = u[p];
    Ld3<T> ld{u, n};
    return b[p] - (c - a * (sc * lap_sum<ORDER, T>(ld, i, j, k, n, c)));
}

// Residual and full-weighting restriction, one thread per coarse point:
// cb(I) = sum over the 27 fine neighbours of 2I+1 of (1/4,1/2,1/4)^3 r.
template <typename T, int ORDER>
__global__ void __launch_bounds__(HS_BLOCK) k_resid_restrict(const GridSeg* __restrict__ segs,
                                                             int nseg, int nblk,
                                                             const LaneCtl* __restrict__ ctl,
                                                             hsk::MgArgs A, int src_is_t)
{
    int lb = xcd_remap(blockIdx.x, nblk);
    int si = find_seg(segs, nseg, lb);
    const GridSeg sg = segs[si];
    if (A.gate && ctl[sg.lane].mg_state != 0) return;
    int n = sg.n, nc = sg.nc;
    Pos q = grid_pos(lb - sg.blk_begin, nc);
    if (!q.in) return;
    const T* u = src_is_t ? (const T*)sg.t : (const T*)sg.u + (long long)A.node * sg.node_stride;
    const T* b = (const T*)sg.b;
    T a = T(lane_a(ctl, sg.lane, A.L, A.m));
    T sc = lap_scale<ORDER, T>(n);
    const T w[3] = {T(0.25), T(0.5), T(0.25)};
    int fi = 2 * q.i + 1, fj = 2 * q.j + 1, fk = 2 * q.k + 1;
    T acc = T(0);
    for (int dz = -1; dz <= 1; dz++) {
        T az = T(0);
        for (int dy = -1; dy <= 1; dy++) {
            T ay = T(0);
            for (int dx = -1; dx <= 1; dx++)
                ay += w[dx + 1] * resid_at<T, ORDER>(u, b, a, sc, fi + dx, fj + dy, fk + dz, n);
            az += w[dy + 1] * ay;
        }
        acc += w[dz + 1] * az;
    }
    ((T*)sg.cb)[lin(q.i, q.j, q.k, nc)] = acc;
}

// trilinear interpolation of a coarse field at fine point (i,j,k); walls 0
template <typename T>
__device__ __forceinline__ T prolong_at(const T* __restrict__ c, int nc, int i, int j, int k)
{
    int ix[2], iy[2], iz[2], cx, cy, cz;
    T wx, wy, wz;
    if (i & 1) { ix[0] = (i - 1) >> 1; cx = 1; wx = T(1); }
    else { ix[0] = (i >> 1) - 1; ix[1] = i >> 1; cx = 2; wx = T(0.5); }
    if (j & 1) { iy[0] = (j - 1) >> 1; cy = 1; wy = T(1); }
    else { iy[0] = (j >> 1) - 1; iy[1] = j >> 1; cy = 2; wy = T(0.5); }
    if (k & 1) { iz[0] = (k - 1) >> 1; cz = 1; wz = T(1); }
    else { iz[0] = (k >> 1) - 1; iz[1] = k >> 1; cz = 2; wz = T(0.5); }
    T s = T(0);
    for (int c3 = 0; c3 < cz; c3++) {
        int K = iz[c3];
        if (K < 0 || K >= nc) continue;
        T sy = T(0);
        for (int c2 = 0; c2 < cy; c2++) {
            int J = iy[c2];
            if (J < 0 || J >= nc) continue;
            T sx = T(0);
            for (int c1 = 0; c1 < cx; c1++) {
                int I = ix[c1];
                if (I < 0 || I >= nc) continue;
                sx += c[lin(I, J, K, nc)];
            }
            sy += wx * sx;
        }
        s += wy * sy;
    }
    return wz * s;
}

// dst = src + P cu (in place when src and dst are the same buffer)
template <typename T>
__global__ void __launch_bounds__(HS_BLOCK) k_prolong(const GridSeg* __restrict__ segs, int nseg,
                                                      int nblk, const LaneCtl* __restrict__ ctl,
                                                      hsk::MgArgs A, int src_is_t, int dst_is_t)
{
    int lb = xcd_remap(blockIdx.x, nblk);
    int si = find_seg(segs, nseg, lb);
    const GridSeg sg = segs[si];
    if (A.gate && ctl[sg.lane].mg_state != 0) return;
    int n = sg.n;
    Pos q = grid_pos(lb - sg.blk_begin, n);
    if (!q.in) return;
    T* U = (T*)sg.u + (long long)A.node * sg.node_stride;
    T* Tt = (T*)sg.t;
    const T* src = src_is_t ? Tt : U;
    T* dst = dst_is_t ? Tt : U;
    long long p = lin(q.i, q.j, q.k, n);
    dst[p] = src[p] + prolong_at<T>((const T*)sg.cu, sg.nc, q.i, q.j, q.k);
}

// ---------------------------------------------------------------------------
// Coarse tail: every grid with n <= HS_TAIL_N of one lane, one workgroup
// ---------------------------------------------------------------------------

template <typename T, int ORDER>
__device__ void tail_jacobi(const T* __restrict__ src, T* __restrict__ dst, const T* __restrict__ b,
                            int n, T a, T om, bool zero)
{
    long long N = (long long)n * n * n;
    T sc = lap_scale<ORDER, T>(n);
    for (long long p = threadIdx.x; p < N; p += blockDim.x) {
        int i = (int)(p % n), j = (int)((p / n) % n), k = (int)(p / ((long long)n * n));
        T D = diag_A<ORDER, T>(a, i, j, k, n);
        if (zero) {
            dst[p] = om * b[p] / D;
        } else {
            Ld3<T> ld{src, n};
            T c = src[p];
            T Au = c - a * (sc * lap_sum<ORDER, T>(ld, i, j, k, n, c));
            dst[p] = c + om * (b[p] - Au) / D;
        }
    }
}

template <typename T, int ORDER>
__device__ void tail_restrict(const T* __restrict__ u, const T* __restrict__ b, T* __restrict__ cb,
                              int n, T a)
{
    int nc = (n - 1) / 2;
    long long Nc = (long long)nc * nc * nc;
    T sc = lap_scale<ORDER, T>(n);
    const T w[3] = {T(0.25), T(0.5), T(0.25)};
    for (long long p = threadIdx.x; p < Nc; p += blockDim.x) {
        int I = (int)(p % nc), J = (int)((p / nc) % nc), K = (int)(p / ((long long)nc * nc));
        int fi = 2 * I + 1, fj = 2 * J + 1, fk = 2 * K + 1;
        T acc = T(0);
        for (int dz = -1; dz <= 1; dz++) {
            T az = T(0);
            for (int dy = -1; dy <= 1; dy++) {
                T ay = T(0);
                for (int dx = -1; dx <= 1; dx++)
                    ay += w[dx + 1] * resid_at<T, ORDER>(u, b, a, sc, fi + dx, fj + dy, fk + dz, n);
                az += w[dy + 1] * ay;
            }
            acc += w[dz + 1] * az;
        }
        cb[p] = acc;
    }
}

template <typename T>
__device__ void tail_prolong(const T* __restrict__ src, T* __restrict__ dst, const T* __restrict__ c,
                             int n)
{
    int nc = (n - 1) / 2;
    long long N = (long long)n * n * n;
    for (long long p = threadIdx.x; p < N; p += blockDim.x) {
        int i = (int)(p % n), j = (int)((p / n) % n), k = (int)(p / ((long long)n * n));
        dst[p] = src[p] + prolong_at<T>(c, nc, i, j, k);
    }
}

// exact solve on a grid of n = 1 or 3 points per axis by the sine transform
template <typename T>
__device__ void tail_exact(const T* __restrict__ b, T* __restrict__ x, int n, T a, const CoarseTable& ct)
{
    __shared__ double bh[27];
    int N = n * n * n;
    int p = threadIdx.x;
    if (p < N) {
        int pi = p % n, pj = (p / n) % n, pk = p / (n * n);
        double s = 0.0;
        for (int k = 0; k < n; k++)
            for (int j = 0; j < n; j++)
                for (int i = 0; i < n; i++)
                    s += ct.S[pk][k] * ct.S[pj][j] * ct.S[pi][i] * (double)b[(k * n + j) * n + i];
        double mu = 1.0 - (double)a * (ct.lam[pi] + ct.lam[pj] + ct.lam[pk]);
        bh[p] = s / mu;
    }
    __syncthreads();
    if (p < N) {
        int i = p % n, j = (p / n) % n, k = p / (n * n);
        double s = 0.0;
        for (int pk = 0; pk < n; pk++)
            for (int pj = 0; pj < n; pj++)
                for (int pi = 0; pi < n; pi++)
                    s += ct.S[pk][k] * ct.S[pj][j] * ct.S[pi][i] * bh[(pk * n + pj) * n + pi];
        x[p] = T(s);
    }
    __syncthreads();
}

// One V(nu1,nu2) cycle over the tail grids of one lane.  Level 0 of the tail
// starts from the iterate in u[0] (or from zero when zero_guess), the lower
// levels from zero; the result is left in u[0].
template <typename T, int ORDER>
__global__ void __launch_bounds__(HS_TAIL_THREADS) k_tail(const TailSeg* __restrict__ segs,
                                                          const LaneCtl* __restrict__ ctl,
                                                          hsk::MgArgs A, int nu1, int nu2)
{
    const TailSeg& ts = segs[blockIdx.x];
    const int zero_guess = ts.zero_guess;
    if (A.gate && ctl[ts.lane].mg_state != 0) return;
    T a = T(lane_a(ctl, ts.lane, A.L, A.m));
    T om = T(A.omega);
    T* u[HS_MAXTAIL];
    T* t[HS_MAXTAIL];
    const T* b[HS_MAXTAIL];
    for (int l = 0; l < ts.nlev; l++) {
        u[l] = (T*)ts.u[l];
        t[l] = (T*)ts.t[l];
        b[l] = (const T*)ts.b[l];
    }
    u[0] += (long long)A.node * ts.node_stride;
    const CoarseTable& ct = c_lc.ct[ts.coarse_table];
    int last = ts.nlev - 1;
    bool in_t[HS_MAXTAIL];   // iterate of level l currently sits in t[l]
    // down
    for (int l = 0; l < last; l++) {
        int n = ts.n[l];
        bool zero = (l > 0) || zero_guess;
        in_t[l] = false;
        for (int s = 0; s < nu1; s++) {
            T* src = in_t[l] ? t[l] : u[l];
            T* dst = in_t[l] ? u[l] : t[l];
            tail_jacobi<T, ORDER>(src, dst, b[l], n, a, om, zero && s == 0);
            in_t[l] = !in_t[l];
            __syncthreads();
        }
        if (nu1 == 0 && zero) {
            long long N = (long long)n * n * n;
            for (long long p = threadIdx.x; p < N; p += blockDim.x) u[l][p] = T(0);
            __syncthreads();
        }
        tail_restrict<T, ORDER>(in_t[l] ? t[l] : u[l], b[l], (T*)b[l + 1], n, a);
        __syncthreads();
    }
    // coarsest grid: exact (an initial guess there is irrelevant)
    tail_exact<T>(b[last], u[last], ts.n[last], a, ct);
    // up
    for (int l = last - 1; l >= 0; l--) {
        int n = ts.n[l];
        T* cur = in_t[l] ? t[l] : u[l];
        tail_prolong<T>(cur, cur, u[l + 1], n);
        __syncthreads();
        for (int s = 0; s < nu2; s++) {
            T* src = in_t[l] ? t[l] : u[l];
            T* dst = in_t[l] ? u[l] : t[l];
            tail_jacobi<T, ORDER>(src, dst, b[l], n, a, om, false);
            in_t[l] = !in_t[l];
            __syncthreads();
        }
        if (in_t[l]) {
            long long N = (long long)n * n * n;
            for (long long p = threadIdx.x; p < N; p += blockDim.x) u[l][p] = t[l][p];
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
// Solve control
// ---------------------------------------------------------------------------

__device__ __forceinline__ void finish_solve(LaneCtl& c, int cycle, int state)
{
    c.mg_state = state;
    c.mg_cycle = cycle;
    c.total_cycles += cycle;
    c.total_solves += 1;
    if (cycle > c.max_cycles) c.max_cycles = cycle;
    if (state == 2) c.failed_solves += 1;
}

// Before cycle `cycle`: rho = |b - A u|_inf / |b|_inf (|b| = 0 -> 1); stop when
// rho <= tol, fail when cycle == max_cycles or rho is not finite.
__global__ void __launch_bounds__(HS_BLOCK) k_mg_norm(const GridSeg* __restrict__ segs, int nseg,
                                                      int nblk, LaneCtl* __restrict__ ctl,
                                                      hsk::MgArgs A, int order, int src_is_t,
                                                      int cycle, double tol, int max_cycles)
{
    int lb = xcd_remap(blockIdx.x, nblk);
    int si = find_seg(segs, nseg, lb);
    const GridSeg sg = segs[si];
    LaneCtl& c = ctl[sg.lane];
    if (c.mg_state != 0) return;
    int n = sg.n;
    Pos q = grid_pos(lb - sg.blk_begin, n);
    const double* u = src_is_t ? (const double*)sg.t
                               : (const double*)sg.u + (long long)A.node * sg.node_stride;
    const double* b = (const double*)sg.b;
    double a = lane_a(ctl, sg.lane, A.L, A.m);
    double r = 0.0, bb = 0.0;
    if (q.in) {
        double sc = order == 2 ? lap_scale<2, double>(n) : lap_scale<4, double>(n);
        r = order == 2 ? resid_at<double, 2>(u, b, a, sc, q.i, q.j, q.k, n)
                       : resid_at<double, 4>(u, b, a, sc, q.i, q.j, q.k, n);
        r = fabs(r);
        if (cycle == 0) bb = fabs(b[lin(q.i, q.j, q.k, n)]);
    }
    bool last = seg_reduce_last(r, &c.res_bits, &c.red_cnt[0], seg_nblk(segs, nseg, si, nblk),
                                cycle == 0 ? &c.bn_bits : nullptr, bb);
    if (last && threadIdx.x == 0) {
        double rmax = bitsd(atomicAdd(&c.res_bits, 0ull));
        if (cycle == 0) c.bnorm = bitsd(atomicAdd(&c.bn_bits, 0ull));
        double scale = c.bnorm > 0.0 ? c.bnorm : 1.0;
        double rho = rmax / scale;
        c.mg_rho = rho;
        if (rho != rho || rmax > 1.7e308) {
            finish_solve(c, cycle, 2);
            c.status = -4;
        } else if (rho <= tol) {
            finish_solve(c, cycle, 1);
        } else if (cycle >= max_cycles) {
            finish_solve(c, cycle, 2);
            if (c.status == 0) c.status = -3;
        }
        c.res_bits = 0ull;
        c.bn_bits = 0ull;
        c.red_cnt[0] = 0u;
    }
}

// Mixed-precision refinement step on the finest grid: optionally u += e
// (the FP32 correction), then r = b - A u in FP64, r32 = (float) r into the
// FP32 right-hand side, and the same stopping test as k_mg_norm.
template <int ORDER>
__global__ void __launch_bounds__(HS_BLOCK) k_ir_resid(const GridSeg* __restrict__ s64,
                                                       const GridSeg* __restrict__ s32, int nseg,
                                                       int nblk, LaneCtl* __restrict__ ctl,
                                                       hsk::MgArgs A, int iter, double tol,
                                                       int max_iter)
{
    int lb = xcd_remap(blockIdx.x, nblk);
    int si = find_seg(s64, nseg, lb);
    const GridSeg sg = s64[si];
    const GridSeg sf = s32[si];
    LaneCtl& c = ctl[sg.lane];
    if (c.mg_state != 0) return;
    int n = sg.n;
    Pos q = grid_pos(lb - sg.blk_begin, n);
    const double* u = (const double*)sg.u + (long long)A.node * sg.node_stride;
    const double* b = (const double*)sg.b;
    double a = lane_a(ctl, sg.lane, A.L, A.m);
    double r = 0.0, bb = 0.0;
    if (q.in) {
        r = resid_at<double, ORDER>(u, b, a, lap_scale<ORDER, double>(n), q.i, q.j, q.k, n);
        long long p = lin(q.i, q.j, q.k, n);
        ((float*)sf.b)[p] = (float)r;
        r = fabs(r);
        if (iter == 0) bb = fabs(b[p]);
    }
    bool last = seg_reduce_last(r, &c.res_bits, &c.red_cnt[2], seg_nblk(s64, nseg, si, nblk),
                                iter == 0 ? &c.bn_bits : nullptr, bb);
    if (last && threadIdx.x == 0) {
        double rmax = bitsd(atomicAdd(&c.res_bits, 0ull));
        if (iter == 0) c.bnorm = bitsd(atomicAdd(&c.bn_bits, 0ull));
        double scale = c.bnorm > 0.0 ? c.bnorm : 1.0;
        double rho = rmax / scale;
        c.mg_rho = rho;
        if (rho != rho || rmax > 1.7e308) {
            finish_solve(c, iter, 2);
            c.status = -4;
        } else if (rho <= tol) {
            finish_solve(c, iter, 1);
        } else if (iter >= max_iter) {
            finish_solve(c, iter, 2);
            if (c.status == 0) c.status = -3;
        }
        c.res_bits = 0ull;
        c.bn_bits = 0ull;
        c.red_cnt[2] = 0u;
    }
}

// u += (double) e on the finest grid
__global__ void __launch_bounds__(HS_BLOCK) k_ir_update(const GridSeg* __restrict__ s64,
                                                        const GridSeg* __restrict__ s32, int nseg,
                                                        int nblk, const LaneCtl* __restrict__ ctl,
                                                        hsk::MgArgs A)
{
    int lb = xcd_remap(blockIdx.x, nblk);
    int si = find_seg(s64, nseg, lb);
    const GridSeg sg = s64[si];
    if (ctl[sg.lane].mg_state != 0) return;
    int n = sg.n;
    Pos q = grid_pos(lb - sg.blk_begin, n);
    if (!q.in) return;
    double* u = (double*)sg.u + (long long)A.node * sg.node_stride;
    long long p = lin(q.i, q.j, q.k, n);
    u[p] += (double)((const float*)s32[si].u)[p];
}

// ---------------------------------------------------------------------------
// SDC level kernels (section 1.1)
// ---------------------------------------------------------------------------

__device__ __forceinline__ double sval(const double* __restrict__ sig, int i, int j, int k)
{
    return (sig[i] * sig[j]) * sig[k];
}

// Predictor: U_m = U_src and FI_m = nu L U_src at every node m.
template <int ORDER>
__global__ void __launch_bounds__(HS_BLOCK) k_spread(const SdcSeg* __restrict__ segs, int nseg,
                                                     int nblk, const LaneCtl* __restrict__ ctl,
                                                     int src_node)
{
    int lb = xcd_remap(blockIdx.x, nblk);
    int si = find_seg(segs, nseg, lb);
    const SdcSeg sg = segs[si];
    if (ctl[sg.lane].sdc_state == 3) return;
    int n = sg.n;
    Pos q = grid_pos(lb - sg.blk_begin, n);
    if (!q.in) return;
    long long N = (long long)n * n * n;
    long long p = lin(q.i, q.j, q.k, n);
    const double* src = sg.U + src_node * N;
    Ld3<double> ld{src, n};
    double c = src[p];
    double fi = ctl[sg.lane].nu * (lap_scale<ORDER, double>(n) * lap_sum<ORDER, double>(ld, q.i, q.j, q.k, n, c));
    for (int m = 0; m < sg.M; m++) {
        if (m != src_node) sg.U[m * N + p] = c;
        sg.FI[m * N + p] = fi;
    }
}

// Sweep-constant right-hand side parts, from iterate k before any update:
//   P_m = dt sum_j S_mj (FI_j + g_j s) - dt_m FI_{m+1} + (tau_{m+1} - tau_m)
// so that substep m solves A_{nu dt_m} U_{m+1} = U_m + P_m (eqs. (7)-(8)).
// With with_resid it also forms the collocation residual
//   R = max_m |U_0 + dt sum_j Q_mj (FI_j + g_j s) + tau_m - U_m|
// and applies the SDC stopping test.
__global__ void __launch_bounds__(HS_BLOCK) k_sweep_prep(const SdcSeg* __restrict__ segs, int nseg,
                                                         int nblk, LaneCtl* __restrict__ ctl,
                                                         int with_resid, double sdc_tol,
                                                         int max_sweeps, int gate)
{
    int lb = xcd_remap(blockIdx.x, nblk);
    int si = find_seg(segs, nseg, lb);
    const SdcSeg sg = segs[si];
    LaneCtl& c = ctl[sg.lane];
    if (gate && c.sdc_state != 0) return;
    int n = sg.n, M = sg.M;
    Pos q = grid_pos(lb - sg.blk_begin, n);
    const SdcConst& K = c_lc.sdc[M];
    double R = 0.0;
    if (q.in) {
        long long N = (long long)n * n * n;
        long long p = lin(q.i, q.j, q.k, n);
        double s = sval(sg.sig, q.i, q.j, q.k);
        double dt = c.dt;
        double F[HS_MAXM], tau[HS_MAXM];
        for (int j = 0; j < M; j++) {
            F[j] = sg.FI[j * N + p] + c.g[sg.level][j] * s;
            tau[j] = sg.tau ? sg.tau[j * N + p] : 0.0;
        }
        for (int m = 0; m < M - 1; m++) {
            double acc = 0.0;
            for (int j = 0; j < M; j++) acc += K.S[m][j] * F[j];
            double v = dt * acc - (dt * K.dtau[m]) * sg.FI[(m + 1) * N + p];
            if (sg.tau) v += tau[m + 1] - tau[m];
            sg.P[m * N + p] = v;
        }
        if (with_resid) {
            double u0 = sg.U[p];
            for (int m = 1; m < M; m++) {
                double acc = 0.0;
                for (int j = 0; j < M; j++) acc += K.Q[m][j] * F[j];
                double v = u0 + dt * acc + tau[m] - sg.U[m * N + p];
                R = nmax(R, fabs(v));
            }
        }
    }
    if (!with_resid) return;
    bool last = seg_reduce_last(R, &c.sdc_bits, &c.red_cnt[1], seg_nblk(segs, nseg, si, nblk));
    if (last && threadIdx.x == 0) {
        double r = bitsd(atomicAdd(&c.sdc_bits, 0ull));
        c.sdc_res = r;
        if (r != r || r > 1.7e308) {
            c.sdc_state = 2;
            c.status = -4;
        } else if (r <= sdc_tol) {
            c.sdc_state = 1;
        } else if (c.sweeps_step >= max_sweeps) {
            c.sdc_state = 2;
            if (c.status == 0) c.status = -3;
        }
        c.sdc_bits = 0ull;
        c.red_cnt[1] = 0u;
    }
}

// rhs = U_m + P_m
__global__ void __launch_bounds__(HS_BLOCK) k_make_rhs(const SdcSeg* __restrict__ segs, int nseg,
                                                       int nblk, const LaneCtl* __restrict__ ctl,
                                                       int m, int gate)
{
    int lb = xcd_remap(blockIdx.x, nblk);
    int si = find_seg(segs, nseg, lb);
    const SdcSeg sg = segs[si];
    if (gate && ctl[sg.lane].sdc_state != 0) return;
    int n = sg.n;
    Pos q = grid_pos(lb - sg.blk_begin, n);
    if (!q.in) return;
    long long N = (long long)n * n * n;
    long long p = lin(q.i, q.j, q.k, n);
    sg.rhs[p] = sg.U[m * N + p] + sg.P[m * N + p];
}

// FI_node = nu L U_node; with next_rhs also rhs = U_node + P_node (the
// right-hand side of the next substep, which starts from this node).
template <int ORDER>
__global__ void __launch_bounds__(HS_BLOCK) k_f_update(const SdcSeg* __restrict__ segs, int nseg,
                                                       int nblk, const LaneCtl* __restrict__ ctl,
                                                       int node, int next_rhs, int gate)
{
    int lb = xcd_remap(blockIdx.x, nblk);
    int si = find_seg(segs, nseg, lb);
    const SdcSeg sg = segs[si];
    if (gate && ctl[sg.lane].sdc_state != 0) return;
    int n = sg.n;
    Pos q = grid_pos(lb - sg.blk_begin, n);
    if (!q.in) return;
    long long N = (long long)n * n * n;
    long long p = lin(q.i, q.j, q.k, n);
    const double* un = sg.U + node * N;
    Ld3<double> ld{un, n};
    double c = un[p];
    sg.FI[node * N + p] = ctl[sg.lane].nu * (lap_scale<ORDER, double>(n) * lap_sum<ORDER, double>(ld, q.i, q.j, q.k, n, c));
    if (next_rhs) sg.rhs[p] = c + sg.P[node * N + p];
}

// FI_m = nu L U_m at every node
template <int ORDER>
__global__ void __launch_bounds__(HS_BLOCK) k_eval_fi_all(const SdcSeg* __restrict__ segs, int nseg,
                                                          int nblk, const LaneCtl* __restrict__ ctl,
                                                          int gate)
{
    int lb = xcd_remap(blockIdx.x, nblk);
    int si = find_seg(segs, nseg, lb);
    const SdcSeg sg = segs[si];
    if (gate && ctl[sg.lane].sdc_state != 0) return;
    int n = sg.n;
    Pos q = grid_pos(lb - sg.blk_begin, n);
    if (!q.in) return;
    long long N = (long long)n * n * n;
    long long p = lin(q.i, q.j, q.k, n);
    double nu = ctl[sg.lane].nu;
    double sc = lap_scale<ORDER, double>(n);
    for (int m = 0; m < sg.M; m++) {
        const double* um = sg.U + m * N;
        Ld3<double> ld{um, n};
        sg.FI[m * N + p] = nu * (sc * lap_sum<ORDER, double>(ld, q.i, q.j, q.k, n, um[p]));
    }
}

// PFASST hand-off: U_dst[0] = U_src[M_src - 1], FI_dst[0] = nu L U_dst[0]
template <int ORDER>
__global__ void __launch_bounds__(HS_BLOCK) k_handoff(const SdcSeg* __restrict__ dst,
                                                      const SdcSeg* __restrict__ src, int nseg,
                                                      int nblk, const LaneCtl* __restrict__ ctl)
{
    int lb = xcd_remap(blockIdx.x, nblk);
    int si = find_seg(dst, nseg, lb);
    const SdcSeg d = dst[si];
    const SdcSeg s = src[si];
    int n = d.n;
    Pos q = grid_pos(lb - d.blk_begin, n);
    if (!q.in) return;
    long long N = (long long)n * n * n;
    long long p = lin(q.i, q.j, q.k, n);
    const double* us = s.U + (long long)(s.M - 1) * N;
    Ld3<double> ld{us, n};
    double c = us[p];
    d.U[p] = c;
    d.FI[p] = ctl[d.lane].nu * (lap_scale<ORDER, double>(n) * lap_sum<ORDER, double>(ld, q.i, q.j, q.k, n, c));
}

// FAS restriction, one thread per coarse point:
//   Ut_m = Uc_m = inj(Uf_{m'}),  FIc_m = nu Lc Ut_m,
//   tau_m = inj(dt sum_j Qf_{m'j} Ff_j) - dt sum_j Qc_{mj} Fc_j
// where m' is the fine node of coarse node m and F = FI + g s.
template <int CORDER>
__global__ void __launch_bounds__(HS_BLOCK) k_fas_restrict(const FasSeg* __restrict__ segs, int nseg,
                                                           int nblk, const LaneCtl* __restrict__ ctl,
                                                           int gate)
{
    int lb = xcd_remap(blockIdx.x, nblk);
    int si = find_seg(segs, nseg, lb);
    const FasSeg sg = segs[si];
    const LaneCtl& c = ctl[sg.lane];
    if (gate && c.sdc_state != 0) return;
    int nc = sg.nc, nf = sg.nf;
    Pos q = grid_pos(lb - sg.blk_begin, nc);
    if (!q.in) return;
    long long Nc = (long long)nc * nc * nc, Nf = (long long)nf * nf * nf;
    long long pc = lin(q.i, q.j, q.k, nc);
    long long pf = lin(2 * q.i + 1, 2 * q.j + 1, 2 * q.k + 1, nf);
    const SdcConst& KF = c_lc.sdc[sg.Mf];
    const SdcConst& KC = c_lc.sdc[sg.Mc];
    int stride = c_lc.ip[sg.Mf][sg.Mc].stride;
    double nu = c.nu, dt = c.dt;
    double sc_ = sval(sg.sigc, q.i, q.j, q.k);
    double sf_ = sval(sg.sigf, 2 * q.i + 1, 2 * q.j + 1, 2 * q.k + 1);
    double Fc[HS_MAXM];
    double lsc = lap_scale<CORDER, double>(nc);
    for (int m = 0; m < sg.Mc; m++) {
        const double* uf = sg.Uf + (long long)(m * stride) * Nf;
        LdInj ld{uf, nf};
        double ut = uf[pf];
        double fi = nu * (lsc * lap_sum<CORDER, double>(ld, q.i, q.j, q.k, nc, ut));
        sg.Ut[m * Nc + pc] = ut;
        sg.Uc[m * Nc + pc] = ut;
        sg.FIc[m * Nc + pc] = fi;
        Fc[m] = fi + c.g[1][m] * sc_;
    }
    double Ff[HS_MAXM];
    for (int j = 0; j < sg.Mf; j++) Ff[j] = sg.FIf[j * Nf + pf] + c.g[0][j] * sf_;
    for (int m = 0; m < sg.Mc; m++) {
        int mf = m * stride;
        double fa = 0.0, ca = 0.0;
        for (int j = 0; j < sg.Mf; j++) fa += KF.Q[mf][j] * Ff[j];
        for (int j = 0; j < sg.Mc; j++) ca += KC.Q[m][j] * Fc[j];
        sg.tau[m * Nc + pc] = dt * fa - dt * ca;
    }
}

// FAS interpolation, one thread per fine point: dU_j = Uc_j - Ut_j,
// Uf_mf += sum_j w[mf][j] P(dU_j)  (trilinear in space, Lagrange in time).
__global__ void __launch_bounds__(HS_BLOCK) k_fas_interp(const FasSeg* __restrict__ segs, int nseg,
                                                         int nblk, const LaneCtl* __restrict__ ctl,
                                                         int gate)
{
    int lb = xcd_remap(blockIdx.x, nblk);
    int si = find_seg(segs, nseg, lb);
    const FasSeg sg = segs[si];
    if (gate && ctl[sg.lane].sdc_state != 0) return;
    int nf = sg.nf, nc = sg.nc;
    Pos q = grid_pos(lb - sg.blk_begin, nf);
    if (!q.in) return;
    long long Nc = (long long)nc * nc * nc, Nf = (long long)nf * nf * nf;
    long long pf = lin(q.i, q.j, q.k, nf);
    double e[HS_MAXM];
    int ix[2], iy[2], iz[2], cx, cy, cz;
    double wx, wy, wz;
    int i = q.i, j = q.j, k = q.k;
    if (i & 1) { ix[0] = (i - 1) >> 1; cx = 1; wx = 1.0; } else { ix[0] = (i >> 1) - 1; ix[1] = i >> 1; cx = 2; wx = 0.5; }
    if (j & 1) { iy[0] = (j - 1) >> 1; cy = 1; wy = 1.0; } else { iy[0] = (j >> 1) - 1; iy[1] = j >> 1; cy = 2; wy = 0.5; }
    if (k & 1) { iz[0] = (k - 1) >> 1; cz = 1; wz = 1.0; } else { iz[0] = (k >> 1) - 1; iz[1] = k >> 1; cz = 2; wz = 0.5; }
    for (int jn = 0; jn < sg.Mc; jn++) {
        const double* uc = sg.Uc + jn * Nc;
        const double* ut = sg.Ut + jn * Nc;
        double s = 0.0;
        for (int c3 = 0; c3 < cz; c3++) {
            int K = iz[c3];
            if (K < 0 || K >= nc) continue;
            double sy = 0.0;
            for (int c2 = 0; c2 < cy; c2++) {
                int J = iy[c2];
                if (J < 0 || J >= nc) continue;
                double sx = 0.0;
                for (int c1 = 0; c1 < cx; c1++) {
                    int I = ix[c1];
                    if (I < 0 || I >= nc) continue;
                    long long pc = lin(I, J, K, nc);
                    sx += uc[pc] - ut[pc];
                }
                sy += wx * sx;
            }
            s += wy * sy;
        }
        e[jn] = wz * s;
    }
    for (int mf = 0; mf < sg.Mf; mf++) {
        double corr = 0.0;
        const InterpConst& ip = c_lc.ip[sg.Mf][sg.Mc];
        if (mf % ip.stride == 0) {
            corr = e[mf / ip.stride];
        } else {
            for (int jn = 0; jn < sg.Mc; jn++) corr += ip.w[mf][jn] * e[jn];
        }
        sg.Uf[mf * Nf + pf] += corr;
    }
}

// SDC residual and stopping test (for the tolerance-driven sweep count)
__global__ void __launch_bounds__(HS_BLOCK) k_sdc_resid(const SdcSeg* __restrict__ segs, int nseg,
                                                        int nblk, LaneCtl* __restrict__ ctl,
                                                        double sdc_tol, int max_sweeps)
{
    int lb = xcd_remap(blockIdx.x, nblk);
    int si = find_seg(segs, nseg, lb);
    const SdcSeg sg = segs[si];
    LaneCtl& c = ctl[sg.lane];
    if (c.sdc_state != 0) return;
    int n = sg.n, M = sg.M;
    Pos q = grid_pos(lb - sg.blk_begin, n);
    const SdcConst& K = c_lc.sdc[M];
    double R = 0.0;
    if (q.in) {
        long long N = (long long)n * n * n;
        long long p = lin(q.i, q.j, q.k, n);
        double s = sval(sg.sig, q.i, q.j, q.k);
        double F[HS_MAXM];
        for (int j = 0; j < M; j++) F[j] = sg.FI[j * N + p] + c.g[sg.level][j] * s;
        double u0 = sg.U[p];
        for (int m = 1; m < M; m++) {
            double acc = 0.0;
            for (int j = 0; j < M; j++) acc += K.Q[m][j] * F[j];
            double v = u0 + c.dt * acc - sg.U[m * N + p];
            if (sg.tau) v += sg.tau[m * N + p];
            R = nmax(R, fabs(v));
        }
    }
    bool last = seg_reduce_last(R, &c.sdc_bits, &c.red_cnt[1], seg_nblk(segs, nseg, si, nblk));
    if (last && threadIdx.x == 0) {
        double r = bitsd(atomicAdd(&c.sdc_bits, 0ull));
        c.sdc_res = r;
        if (r != r || r > 1.7e308) {
            c.sdc_state = 2;
            c.status = -4;
        } else if (r <= sdc_tol) {
            c.sdc_state = 1;
        } else if (c.sweeps_step >= max_sweeps) {
            c.sdc_state = 2;
            if (c.status == 0) c.status = -3;
        }
        c.sdc_bits = 0ull;
        c.red_cnt[1] = 0u;
    }
}

// ---------------------------------------------------------------------------
// Lane bookkeeping
// ---------------------------------------------------------------------------

// Step coefficients: t_n = t0 + step dt; a[L][m] = nu dt (tau_{m+1} - tau_m);
// g[L][j] = -(sin t_j - c nu pi^2 cos t_j) at t_j = t_n + dt tau_j (eq. (3)).
__global__ void k_begin_step(LaneCtl* ctl, int nlanes, int nlevels, int M0, int M1)
{
    int lane = blockIdx.x * blockDim.x + threadIdx.x;
    if (lane >= nlanes) return;
    LaneCtl& c = ctl[lane];
    bool live = c.active && c.step < c.nsteps;
    c.sdc_state = live ? 0 : 3;
    c.sweeps_step = 0;
    c.tn = c.t0 + (double)c.step * c.dt;
    const double pi2 = 3.14159265358979323846 * 3.14159265358979323846;
    for (int L = 0; L < nlevels; L++) {
        const SdcConst& K = c_lc.sdc[L == 0 ? M0 : M1];
        for (int m = 0; m < K.M; m++) {
            double tj = c.tn + c.dt * K.tau[m];
            c.g[L][m] = -(sin(tj) - c.forcing_c * c.nu * pi2 * cos(tj));
            if (m < K.M - 1) c.a[L][m] = c.nu * (c.dt * K.dtau[m]);
        }
    }
}

__global__ void k_end_step(LaneCtl* ctl, int nlanes)
{
    int lane = blockIdx.x * blockDim.x + threadIdx.x;
    if (lane >= nlanes) return;
    LaneCtl& c = ctl[lane];
    if (c.sdc_state != 3) {
        c.step += 1;
        c.total_sweeps += c.sweeps_step;
    }
}

__global__ void k_begin_solve(LaneCtl* ctl, int nlanes)
{
    int lane = blockIdx.x * blockDim.x + threadIdx.x;
    if (lane >= nlanes) return;
    LaneCtl& c = ctl[lane];
    c.mg_state = c.sdc_state != 0 ? 3 : 0;
    c.mg_cycle = 0;
}

__global__ void k_end_solve_fixed(LaneCtl* ctl, int nlanes, int cycles)
{
    int lane = blockIdx.x * blockDim.x + threadIdx.x;
    if (lane >= nlanes) return;
    LaneCtl& c = ctl[lane];
    if (c.mg_state == 0) finish_solve(c, cycles, 1);
}

__global__ void k_begin_sweep(LaneCtl* ctl, int nlanes)
{
    int lane = blockIdx.x * blockDim.x + threadIdx.x;
    if (lane >= nlanes) return;
    LaneCtl& c = ctl[lane];
    if (c.sdc_state == 0) c.sweeps_step += 1;
}

__global__ void k_set_lane(LaneCtl* ctl, int lane, double nu, double dt, double t0, double fc,
                           int nsteps, int active)
{
    LaneCtl& c = ctl[lane];
    c.nu = nu; c.dt = dt; c.t0 = t0; c.forcing_c = fc;
    c.nsteps = nsteps; c.step = 0; c.active = active;
    c.sdc_state = active ? 0 : 3; c.mg_state = 3; c.status = 0;
    c.red_cnt[0] = c.red_cnt[1] = c.red_cnt[2] = c.red_cnt[3] = 0u;
    c.res_bits = c.bn_bits = c.sdc_bits = 0ull;
    c.bnorm = c.mg_rho = c.sdc_res = 0.0;
    c.total_cycles = 0; c.total_solves = 0; c.max_cycles = 0; c.total_sweeps = 0;
    c.sweeps_step = 0; c.failed_solves = 0; c.a_user = 0.0;
}

__global__ void k_set_a_user(LaneCtl* ctl, int lane, double a)
{
    ctl[lane].a_user = a;
    ctl[lane].mg_state = 0;
    ctl[lane].sdc_state = 0;
}

__global__ void k_copy(const double* __restrict__ src, double* __restrict__ dst, long long count)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long stride = (long long)gridDim.x * blockDim.x;
    for (; i < count; i += stride) dst[i] = src[i];
}

// y = alpha u + beta L u on user arrays (lane-major packing, offset pack_off)
template <int ORDER>
__global__ void __launch_bounds__(HS_BLOCK) k_lap_apply(const SdcSeg* __restrict__ segs, int nseg,
                                                        int nblk, double alpha, double beta,
                                                        const double* __restrict__ u,
                                                        double* __restrict__ y,
                                                        const long long* __restrict__ offs)
{
    int lb = xcd_remap(blockIdx.x, nblk);
    int si = find_seg(segs, nseg, lb);
    const SdcSeg sg = segs[si];
    int n = sg.n;
    Pos q = grid_pos(lb - sg.blk_begin, n);
    if (!q.in) return;
    const double* ul = u + offs[si];
    long long p = lin(q.i, q.j, q.k, n);
    Ld3<double> ld{ul, n};
    double c = ul[p];
    y[offs[si] + p] = alpha * c + beta * (lap_scale<ORDER, double>(n) * lap_sum<ORDER, double>(ld, q.i, q.j, q.k, n, c));
}

// f_impl = nu L u, f_expl = f(x, t) (eq. (3)) on user arrays
template <int ORDER>
__global__ void __launch_bounds__(HS_BLOCK) k_heat_rhs(const SdcSeg* __restrict__ segs, int nseg,
                                                       int nblk, const LaneCtl* __restrict__ ctl,
                                                       const double* __restrict__ u,
                                                       const double* __restrict__ t,
                                                       double* __restrict__ fi,
                                                       double* __restrict__ fe,
                                                       const long long* __restrict__ offs)
{
    int lb = xcd_remap(blockIdx.x, nblk);
    int si = find_seg(segs, nseg, lb);
    const SdcSeg sg = segs[si];
    int n = sg.n;
    Pos q = grid_pos(lb - sg.blk_begin, n);
    if (!q.in) return;
    const LaneCtl& c = ctl[sg.lane];
    long long p = lin(q.i, q.j, q.k, n);
    if (fi) {
        const double* ul = u + offs[si];
        Ld3<double> ld{ul, n};
        fi[offs[si] + p] = c.nu * (lap_scale<ORDER, double>(n) * lap_sum<ORDER, double>(ld, q.i, q.j, q.k, n, ul[p]));
    }
    if (fe) {
        const double pi2 = 3.14159265358979323846 * 3.14159265358979323846;
        double tt = t[si];
        double g = -(sin(tt) - c.forcing_c * c.nu * pi2 * cos(tt));
        fe[offs[si] + p] = sval(sg.sig, q.i, q.j, q.k) * g;
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// Launch helpers
// ---------------------------------------------------------------------------
namespace hsk {

static inline dim3 g1(int nblk) { return dim3((unsigned)nblk); }
static const dim3 BLK(HS_BLOCK);

int grid_blocks(int n) { return tiles_x(n) * tiles_y(n) * n; }

hipError_t set_constants(const LibConst& lc)
{
    return hipMemcpyToSymbol(HIP_SYMBOL(c_lc), &lc, sizeof(LibConst), 0, hipMemcpyHostToDevice);
}

#define HS_ORDER_DISPATCH(order, KERNEL2, KERNEL4, GRID, BLOCK, ...)                   \
    do {                                                                               \
        if ((order) == 2) hipLaunchKernelGGL(KERNEL2, GRID, BLOCK, 0, s, __VA_ARGS__); \
        else hipLaunchKernelGGL(KERNEL4, GRID, BLOCK, 0, s, __VA_ARGS__);              \
    } while (0)

template <typename T>
hipError_t jacobi(LaneCtl* ctl, const GridSeg* segs, int nseg, int nblk, int order, MgArgs a,
                  int first_sweep, int src_is_t, hipStream_t s)
{
    if (nblk <= 0) return hipSuccess;
    HS_ORDER_DISPATCH(order, (k_jacobi<T, 2>), (k_jacobi<T, 4>), g1(nblk), BLK, segs, nseg, nblk,
                      ctl, a, first_sweep, src_is_t);
    return hipGetLastError();
}

template <typename T>
hipError_t resid_restrict(LaneCtl* ctl, const GridSeg* segs, int nseg, int nblk, int order,
                          MgArgs a, int src_is_t, hipStream_t s)
{
    if (nblk <= 0) return hipSuccess;
    HS_ORDER_DISPATCH(order, (k_resid_restrict<T, 2>), (k_resid_restrict<T, 4>), g1(nblk), BLK,
                      segs, nseg, nblk, ctl, a, src_is_t);
    return hipGetLastError();
}

template <typename T>
hipError_t prolong(LaneCtl* ctl, const GridSeg* segs, int nseg, int nblk, MgArgs a, int src_is_t,
                   int dst_is_t, hipStream_t s)
{
    if (nblk <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_prolong<T>), g1(nblk), BLK, 0, s, segs, nseg, nblk, ctl, a, src_is_t,
                       dst_is_t);
    return hipGetLastError();
}

template <typename T>
hipError_t tail(LaneCtl* ctl, const TailSeg* segs, int nseg, int order, MgArgs a, int nu1, int nu2,
                hipStream_t s)
{
    if (nseg <= 0) return hipSuccess;
    HS_ORDER_DISPATCH(order, (k_tail<T, 2>), (k_tail<T, 4>), dim3((unsigned)nseg),
                      dim3(HS_TAIL_THREADS), segs, ctl, a, nu1, nu2);
    return hipGetLastError();
}

template hipError_t jacobi<double>(LaneCtl*, const GridSeg*, int, int, int, MgArgs, int, int, hipStream_t);
template hipError_t jacobi<float>(LaneCtl*, const GridSeg*, int, int, int, MgArgs, int, int, hipStream_t);
template hipError_t resid_restrict<double>(LaneCtl*, const GridSeg*, int, int, int, MgArgs, int, hipStream_t);
template hipError_t resid_restrict<float>(LaneCtl*, const GridSeg*, int, int, int, MgArgs, int, hipStream_t);
template hipError_t prolong<double>(LaneCtl*, const GridSeg*, int, int, MgArgs, int, int, hipStream_t);
template hipError_t prolong<float>(LaneCtl*, const GridSeg*, int, int, MgArgs, int, int, hipStream_t);
template hipError_t tail<double>(LaneCtl*, const TailSeg*, int, int, MgArgs, int, int, hipStream_t);
template hipError_t tail<float>(LaneCtl*, const TailSeg*, int, int, MgArgs, int, int, hipStream_t);

hipError_t mg_norm(LaneCtl* ctl, const GridSeg* segs, int nseg, int nblk, int order, MgArgs a,
                   int src_is_t, int cycle, double tol, int max_cycles, hipStream_t s)
{
    if (nblk <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mg_norm, g1(nblk), BLK, 0, s, segs, nseg, nblk, ctl, a, order, src_is_t,
                       cycle, tol, max_cycles);
    return hipGetLastError();
}

hipError_t ir_resid(LaneCtl* ctl, const GridSeg* segs64, const GridSeg* segs32, int nseg, int nblk,
                    int order, MgArgs a, int iter, double tol, int max_iter, hipStream_t s)
{
    if (nblk <= 0) return hipSuccess;
    HS_ORDER_DISPATCH(order, (k_ir_resid<2>), (k_ir_resid<4>), g1(nblk), BLK, segs64, segs32,
                      nseg, nblk, ctl, a, iter, tol, max_iter);
    return hipGetLastError();
}

hipError_t ir_update(LaneCtl* ctl, const GridSeg* segs64, const GridSeg* segs32, int nseg,
                     int nblk, MgArgs a, hipStream_t s)
{
    if (nblk <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_ir_update, g1(nblk), BLK, 0, s, segs64, segs32, nseg, nblk, ctl, a);
    return hipGetLastError();
}

hipError_t spread(LaneCtl* ctl, const SdcSeg* segs, int nseg, int nblk, int order, int src_node,
                  hipStream_t s)
{
    if (nblk <= 0) return hipSuccess;
    HS_ORDER_DISPATCH(order, (k_spread<2>), (k_spread<4>), g1(nblk), BLK, segs, nseg, nblk, ctl,
                      src_node);
    return hipGetLastError();
}

hipError_t sweep_prep(LaneCtl* ctl, const SdcSeg* segs, int nseg, int nblk, int with_resid,
                      double sdc_tol, int max_sweeps, int gate, hipStream_t s)
{
    if (nblk <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_sweep_prep, g1(nblk), BLK, 0, s, segs, nseg, nblk, ctl, with_resid,
                       sdc_tol, max_sweeps, gate);
    return hipGetLastError();
}

hipError_t make_rhs(LaneCtl* ctl, const SdcSeg* segs, int nseg, int nblk, int m, int gate,
                    hipStream_t s)
{
    if (nblk <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_make_rhs, g1(nblk), BLK, 0, s, segs, nseg, nblk, ctl, m, gate);
    return hipGetLastError();
}

hipError_t f_update(LaneCtl* ctl, const SdcSeg* segs, int nseg, int nblk, int order, int node,
                    int next_rhs, int gate, hipStream_t s)
{
    if (nblk <= 0) return hipSuccess;
    HS_ORDER_DISPATCH(order, (k_f_update<2>), (k_f_update<4>), g1(nblk), BLK, segs, nseg, nblk,
                      ctl, node, next_rhs, gate);
    return hipGetLastError();
}

hipError_t eval_fi_all(LaneCtl* ctl, const SdcSeg* segs, int nseg, int nblk, int order, int gate,
                       hipStream_t s)
{
    if (nblk <= 0) return hipSuccess;
    HS_ORDER_DISPATCH(order, (k_eval_fi_all<2>), (k_eval_fi_all<4>), g1(nblk), BLK, segs, nseg,
                      nblk, ctl, gate);
    return hipGetLastError();
}

hipError_t sdc_resid(LaneCtl* ctl, const SdcSeg* segs, int nseg, int nblk, double sdc_tol,
                     int max_sweeps, hipStream_t s)
{
    if (nblk <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_sdc_resid, g1(nblk), BLK, 0, s, segs, nseg, nblk, ctl, sdc_tol,
                       max_sweeps);
    return hipGetLastError();
}

hipError_t handoff(LaneCtl* ctl, const SdcSeg* dst, const SdcSeg* src, int nseg, int nblk,
                   int order, hipStream_t s)
{
    if (nblk <= 0) return hipSuccess;
    HS_ORDER_DISPATCH(order, (k_handoff<2>), (k_handoff<4>), g1(nblk), BLK, dst, src, nseg, nblk,
                      ctl);
    return hipGetLastError();
}

hipError_t fas_restrict(LaneCtl* ctl, const FasSeg* segs, int nseg, int nblk, int corder, int gate,
                        hipStream_t s)
{
    if (nblk <= 0) return hipSuccess;
    HS_ORDER_DISPATCH(corder, (k_fas_restrict<2>), (k_fas_restrict<4>), g1(nblk), BLK, segs, nseg,
                      nblk, ctl, gate);
    return hipGetLastError();
}

hipError_t fas_interp(LaneCtl* ctl, const FasSeg* segs, int nseg, int nblk, int gate,
                      hipStream_t s)
{
    if (nblk <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fas_interp, g1(nblk), BLK, 0, s, segs, nseg, nblk, ctl, gate);
    return hipGetLastError();
}

static inline dim3 lanes_grid(int n) { return dim3((unsigned)((n + 63) / 64)); }

hipError_t begin_step(LaneCtl* ctl, int nlanes, int nlevels, int M0, int M1, hipStream_t s)
{
    hipLaunchKernelGGL(k_begin_step, lanes_grid(nlanes), dim3(64), 0, s, ctl, nlanes, nlevels, M0, M1);
    return hipGetLastError();
}

hipError_t end_step(LaneCtl* ctl, int nlanes, hipStream_t s)
{
    hipLaunchKernelGGL(k_end_step, lanes_grid(nlanes), dim3(64), 0, s, ctl, nlanes);
    return hipGetLastError();
}

hipError_t begin_solve(LaneCtl* ctl, int nlanes, hipStream_t s)
{
    hipLaunchKernelGGL(k_begin_solve, lanes_grid(nlanes), dim3(64), 0, s, ctl, nlanes);
    return hipGetLastError();
}

hipError_t end_solve_fixed(LaneCtl* ctl, int nlanes, int cycles, hipStream_t s)
{
    hipLaunchKernelGGL(k_end_solve_fixed, lanes_grid(nlanes), dim3(64), 0, s, ctl, nlanes, cycles);
    return hipGetLastError();
}

hipError_t begin_sweep(LaneCtl* ctl, int nlanes, hipStream_t s)
{
    hipLaunchKernelGGL(k_begin_sweep, lanes_grid(nlanes), dim3(64), 0, s, ctl, nlanes);
    return hipGetLastError();
}

hipError_t set_lane(LaneCtl* ctl, int lane, double nu, double dt, double t0, double forcing_c,
                    int nsteps, int active, hipStream_t s)
{
    hipLaunchKernelGGL(k_set_lane, dim3(1), dim3(1), 0, s, ctl, lane, nu, dt, t0, forcing_c, nsteps,
                       active);
    return hipGetLastError();
}

hipError_t set_a_user(LaneCtl* ctl, int lane, double a, hipStream_t s)
{
    hipLaunchKernelGGL(k_set_a_user, dim3(1), dim3(1), 0, s, ctl, lane, a);
    return hipGetLastError();
}

hipError_t copy(const double* src, double* dst, long long count, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    long long blocks = (count + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(256), 0, s, src, dst, count);
    return hipGetLastError();
}

hipError_t lap_apply(const SdcSeg* segs, int nseg, int nblk, int order, double alpha, double beta,
                     const double* u, double* y, const long long* offs, hipStream_t s)
{
    if (nblk <= 0) return hipSuccess;
    HS_ORDER_DISPATCH(order, (k_lap_apply<2>), (k_lap_apply<4>), g1(nblk), BLK, segs, nseg, nblk,
                      alpha, beta, u, y, offs);
    return hipGetLastError();
}

hipError_t heat_rhs(LaneCtl* ctl, const SdcSeg* segs, int nseg, int nblk, int order,
                    const double* u, const double* t, double* fi, double* fe,
                    const long long* offs, hipStream_t s)
{
    if (nblk <= 0) return hipSuccess;
    HS_ORDER_DISPATCH(order, (k_heat_rhs<2>), (k_heat_rhs<4>), g1(nblk), BLK, segs, nseg, nblk,
                      ctl, u, t, fi, fe, offs);
    return hipGetLastError();
}

}  // namespace hsk
