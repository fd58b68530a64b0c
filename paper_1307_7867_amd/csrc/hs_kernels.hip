// HIP kernels of libheatst for gfx950 (MI355X).
//
// Every kernel of the multigrid and SDC hot path works on a table of
// segments: one segment is one grid of one lane (an independent problem or
// a PFASST time slice).  Blocks of 512 threads tile a grid as 64 x 8 points
// in x-y (one wavefront per x row, coalesced along x).  The stencil kernels
// march along z through a chunk of planes per block and keep the z
// neighbours of each column in registers; other kernels take one plane per
// block.  A launch covers all segments of its table, so lanes of equal or
// of different sizes share one launch.  The hardware hands consecutive
// blocks to the 8 XCDs in turn; the block index is remapped so that every
// XCD works on one contiguous range of planes and reuses neighbour planes
// from its own L2.
//
// Reductions (residual norms) write one maximum per block; a small kernel
// with one block per lane combines them and takes the stopping decision,
// so no two blocks ever contend for one address.
//
// The discrete operators follow the paper's section 1 (method of lines,
// 2nd- and 4th-order Laplacians, implicit-Euler substeps of the IMEX SDC
// sweep of eq. (7)) and section 1.2 (multigrid); the multigrid components
// (weighted Jacobi, full weighting, trilinear prolongation, exact solve on
// the coarsest grid) are this library's choice, the paper names none.
#include "hs_internal.h"

#include <hip/hip_ext.h>

#include <map>
#include <type_traits>
#include <mutex>

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

// buffer picked by a source-buffer code for this segment (1 = t)
__device__ __forceinline__ int seg_src(int code, const GridSeg& sg)
{
    return sg.coarse ? (code >> 1) & 1 : code & 1;
}

__host__ __device__ __forceinline__ int tiles_x(int n) { return (n + HS_TX - 1) / HS_TX; }
__host__ __device__ __forceinline__ int tiles_y(int n) { return (n + HS_TY - 1) / HS_TY; }

// position of this thread inside its segment's grid (one plane per block)
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

// position of this thread's column and z range (z-marching blocks)
struct PosZ {
    int i, j, z0, z1;
    bool in;
};

__device__ __forceinline__ PosZ grid_pos_z(int rel_blk, int n, int zb)
{
    int tx = tiles_x(n), ty = tiles_y(n);
    int bx = rel_blk % tx;
    int rest = rel_blk / tx;
    int by = rest % ty;
    int bz = rest / ty;
    PosZ p;
    p.i = bx * HS_TX + (int)(threadIdx.x % HS_TX);
    p.j = by * HS_TY + (int)(threadIdx.x / HS_TX);
    p.z0 = bz * zb;
    p.z1 = min(p.z0 + zb, n);
    p.in = p.i < n && p.j < n;
    return p;
}

// offset of point (i,j,k) inside one n^3 grid; n <= 511 keeps it below 2^31
__device__ __forceinline__ int lin(int i, int j, int k, int n)
{
    return (k * n + j) * n + i;
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

// Global-memory pointer.  The grid pointers come from the segment tables, so
// the compiler cannot tell they are global and would emit flat loads; those
// count against the LDS wait counter as well, and every wait for an LDS read
// would then also wait for the global loads in flight.  Kernels that mix LDS
// traffic with global loads cast their grid pointers to this type.
#define HS_G __attribute__((address_space(1)))

// (90 - w) / 12, the 4th-order centre weight (in units of 1/h^2) of a point
// next to w walls, as the division evaluates it
template <typename T>
__device__ __forceinline__ T centre4(int w)
{
    return w == 0 ? T(90) / T(12) : w == 1 ? T(89) / T(12) : w == 2 ? T(88) / T(12) :
           w == 3 ? T(87) / T(12) : w == 4 ? T(86) / T(12) : w == 5 ? T(85) / T(12) : T(84) / T(12);
}

// omega / D along the column (i, j) of an n^3 grid, D the diagonal of A_a.
// D depends on the number of walls next to a point, which along a column
// changes only on the planes z = 0 and z = n-1, so a column needs at most
// three values; sweeps multiply by them instead of dividing per point.
template <int ORDER, typename T>
struct ColRd {
    T r0 = T(0), r1 = T(0), r2 = T(0);   // 0, 1 and 2 walls along z
    ColRd() = default;
    __device__ __forceinline__ ColRd(T a, T om, int i, int j, int n)
    {
        const T ih2 = T((double)(n + 1) * (double)(n + 1));
        if (ORDER == 2) {
            r0 = r1 = r2 = om / (T(1) + a * ih2 * T(6));
        } else {
            const int w = (i == 0) + (i == n - 1) + (j == 0) + (j == n - 1);
            r0 = om / (T(1) + a * ih2 * centre4<T>(w));
            r1 = om / (T(1) + a * ih2 * centre4<T>(w + 1));
            r2 = n == 1 ? om / (T(1) + a * ih2 * centre4<T>(w + 2)) : r1;
        }
    }
    // Weighted sum with one weight 1 and the others 0 (exact: the values are
    // finite).  A select between the members would be turned into a load at
    // a computed member address, which keeps the enclosing object out of
    // registers.
    __device__ __forceinline__ T at(int z, int n) const
    {
        if (ORDER == 2) return r0;
        const int wz = (z == 0) + (z == n - 1);
        return (T(wz == 0) * r0 + T(wz == 1) * r1) + T(wz == 2) * r2;
    }
};

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

// record the end of a multigrid solve (state 1 converged, 2 failed)
__device__ __forceinline__ void finish_solve(LaneCtl& c, int cycle, int state, int level)
{
    c.mg_state = state;
    c.mg_cycle = cycle;
    c.total_cycles += cycle;
    if (level >= 0 && level < HS_MAXLEV) c.level_cycles[level] += cycle;
    c.total_solves += 1;
    if (cycle > c.max_cycles) c.max_cycles = cycle;
    if (state == 2) c.failed_solves += 1;
}

// A lane's multigrid state, read unconditionally (every lane of a table has
// an entry) so that the load is not tied to the gate flag's branch.
__device__ __forceinline__ int ld_state(const LaneCtl* ctl, int lane) { return ctl[lane].mg_state; }

__device__ __forceinline__ double lane_a(const LaneCtl* ctl, int lane, int L, int m)
{
    return m >= 0 ? ctl[lane].a[L][m] : ctl[lane].a_user;
}

// max that keeps NaN
template <typename T>
__device__ __forceinline__ T nmax(T a, T b) { return (b > a || b != b) ? b : a; }

template <typename T>
__device__ __forceinline__ T tabs(T x) { return x < T(0) ? -x : x; }

// block-wide max; result valid in thread 0.  All threads must call it.
__device__ __forceinline__ double block_max(double v)
{
    __shared__ double sm[16];
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

// block-wide maxima of two values at once (one pair of barriers); results
// valid in thread 0.  All threads must call it.
__device__ __forceinline__ void block_max2(double& v, double& u)
{
    __shared__ double sm[2][16];
    for (int off = 32; off > 0; off >>= 1) {
        v = nmax(v, __shfl_xor(v, off, 64));
        u = nmax(u, __shfl_xor(u, off, 64));
    }
    int w = threadIdx.x / 64, l = threadIdx.x % 64;
    __syncthreads();
    if (l == 0) {
        sm[0][w] = v;
        sm[1][w] = u;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int nw = (blockDim.x + 63) / 64;
        for (int q = 1; q < nw; q++) {
            v = nmax(v, sm[0][q]);
            u = nmax(u, sm[1][q]);
        }
    }
}

template <typename S>
__device__ __forceinline__ int seg_nblk(const S* segs, int nseg, int si, int nblk)
{
    return (si + 1 < nseg ? segs[si + 1].blk_begin : nblk) - segs[si].blk_begin;
}

// value of a column at plane z' with the wall rules of lap_sum along z
template <int ORDER, typename T>
__device__ __forceinline__ T zval(const T* __restrict__ col, int z, int n, long long nn)
{
    if (z >= 0 && z < n) return col[(long long)z * nn];
    if (ORDER == 4) {
        if (z == -2) return -col[0];
        if (z == n + 1) return -col[(long long)(n - 1) * nn];
    }
    return T(0);
}

// March one column (i, j) through planes z0..z1-1 of an n^3 field src,
// keeping the z neighbours in registers; for each plane call
// op(p, c, L) with p the linear index, c = src[p] and L = L_h src at p.
template <int ORDER, typename T, typename Op>
__device__ __forceinline__ void zmarch(const T* __restrict__ src, int n, int i, int j, int z0, int z1,
                                       Op& op)
{
    constexpr int R = ORDER == 2 ? 1 : 2;
    const long long nn = (long long)n * n;
    const T* col = src + (long long)j * n + i;
    const T sc = lap_scale<ORDER, T>(n);
    const T zero = T(0);
    T w[2 * R + 1];
#pragma unroll
    for (int d = -R; d < R; d++) w[d + R] = zval<ORDER, T>(col, z0 + d, n, nn);
    for (int z = z0; z < z1; z++) {
        w[2 * R] = zval<ORDER, T>(col, z + R, n, nn);
        const T c = w[R];
        const long long p = (long long)z * nn + (long long)j * n + i;
        const T* u = src + p;
        T L;
        if (ORDER == 2) {
            T xm = i > 0 ? u[-1] : zero;
            T xp = i < n - 1 ? u[1] : zero;
            T ym = j > 0 ? u[-n] : zero;
            T yp = j < n - 1 ? u[n] : zero;
            T c2 = T(2) * c;
            L = ((xm - c2) + xp) + ((ym - c2) + yp) + ((w[0] - c2) + w[2]);
        } else {
            T ax, ay, az;
            {
                T m1 = i >= 1 ? u[-1] : zero;
                T m2 = i >= 2 ? u[-2] : (i == 1 ? zero : -c);
                T p1 = i <= n - 2 ? u[1] : zero;
                T p2 = i <= n - 3 ? u[2] : (i == n - 2 ? zero : -c);
                ax = (T(16) * (m1 + p1) - (m2 + p2)) - T(30) * c;
            }
            {
                T m1 = j >= 1 ? u[-n] : zero;
                T m2 = j >= 2 ? u[-2 * n] : (j == 1 ? zero : -c);
                T p1 = j <= n - 2 ? u[n] : zero;
                T p2 = j <= n - 3 ? u[2 * n] : (j == n - 2 ? zero : -c);
                ay = (T(16) * (m1 + p1) - (m2 + p2)) - T(30) * c;
            }
            az = (T(16) * (w[1] + w[3]) - (w[0] + w[4])) - T(30) * c;
            L = (ax + ay) + az;
        }
        op(p, z, c, sc * L);
#pragma unroll
        for (int d = 0; d < 2 * R; d++) w[d] = w[d + 1];
    }
}

// Sources of the plane march: the value of the field the stencil is applied
// to at grid point p (linear index) on plane z of a column whose handle
// S.col(i, j) is taken once.
template <typename T>
struct SrcPlain {
    const HS_G T* __restrict__ u;
    static constexpr bool kSplit = false;
    struct Col {};
    __device__ __forceinline__ Col col(int, int) const { return Col{}; }
    __device__ __forceinline__ T raw(long long p) const { return u[p]; }
    __device__ __forceinline__ T fix(T v, const Col&, int) const { return v; }
    __device__ __forceinline__ T at(long long p, const Col& c, int z) const { return fix(raw(p), c, z); }
};

// The first weighted-Jacobi sweep from a zero guess, omega D^{-1} b,
// evaluated where it is read instead of being stored.
template <typename T, int ORDER>
struct SrcZeroJacobi {
    const HS_G T* __restrict__ b;
    T a, om;
    int n;
    static constexpr bool kSplit = true;   // the weights take divisions: form them while the loads fly
    using Col = ColRd<ORDER, T>;
    __device__ __forceinline__ Col col(int i, int j) const { return Col(a, om, i, j, n); }
    __device__ __forceinline__ T raw(long long p) const { return b[p]; }
    __device__ __forceinline__ T fix(T v, const Col& c, int z) const { return c.at(z, n) * v; }
    __device__ __forceinline__ T at(long long p, const Col& c, int z) const { return fix(raw(p), c, z); }
};

// Plane whose value the wall rules of the stencil along z read for plane z
// (itself inside the grid, the mirrored plane with a sign change for the
// 4th-order ghost planes -2 and n+1), or -1 where the value is 0.
template <int ORDER>
__device__ __forceinline__ int zmirror(int z, int n)
{
    if (z >= 0 && z < n) return z;
    if (ORDER == 4) {
        if (z == -2) return 0;
        if (z == n + 1) return n - 1;
    }
    return -1;
}

// Plane z of a column from the raw value loaded at plane zmirror(z): the
// source's own finishing step, then the wall sign.  Splitting the load from
// this step lets every load of a plane go out before any of them is used.
template <int ORDER, typename T, class Src>
__device__ __forceinline__ T zfix_src(const Src& S, const typename Src::Col& c, T raw, int z, int n)
{
    const int zm = zmirror<ORDER>(z, n);
    if (zm < 0) return T(0);
    const T v = S.fix(raw, c, zm);
    return zm == z ? v : -v;
}

// value of the source on the column with handle c (pij = j n + i) at plane
// z' with the wall rules of the stencil along z
template <int ORDER, typename T, class Src>
__device__ __forceinline__ T zval_src(const Src& S, const typename Src::Col& c, int z, int n, long long nn,
                                      long long pij)
{
    if (z >= 0 && z < n) return S.at(pij + (long long)z * nn, c, z);
    if (ORDER == 4) {
        if (z == -2) return -S.at(pij, c, 0);
        if (z == n + 1) return -S.at(pij + (long long)(n - 1) * nn, c, n - 1);
    }
    return T(0);
}

// L_h sum (before the 1/h^2 scale) at a point whose plane sits in LDS with
// row length LW (cell = its own cell) and whose z neighbours are the column
// window w (w[R] = centre).  Cells outside the grid hold 0; the reflected
// 4th-order taps one beyond a wall are -centre.
template <int ORDER, typename T, int LW>
__device__ __forceinline__ T plane_lap(const T* cell, const T* w, int i, int j, int n)
{
    if (ORDER == 2) {
        const T c = w[1];
        T c2 = T(2) * c;
        return ((cell[-1] - c2) + cell[1]) + ((cell[-LW] - c2) + cell[LW]) + ((w[0] - c2) + w[2]);
    } else {
        const T c = w[2];
        T m2 = i == 0 ? -c : cell[-2];
        T p2 = i == n - 1 ? -c : cell[2];
        T ax = (T(16) * (cell[-1] + cell[1]) - (m2 + p2)) - T(30) * c;
        m2 = j == 0 ? -c : cell[-2 * LW];
        p2 = j == n - 1 ? -c : cell[2 * LW];
        T ay = (T(16) * (cell[-LW] + cell[LW]) - (m2 + p2)) - T(30) * c;
        T az = (T(16) * (w[1] + w[3]) - (w[0] + w[4])) - T(30) * c;
        return (ax + ay) + az;
    }
}

// Plane march through LDS.  The block (64 x 8 threads) owns a 64 x 8 column
// tile and planes z0..z1-1.  The current plane, with a halo of R = ORDER/2
// points in x and y, sits in one of two LDS buffers; the z neighbours of each
// column sit in registers.  While plane z is computed, the halo of plane z+1
// and the column value of plane z+R+1 are already in flight, so one memory
// latency is hidden behind every plane.  Every thread of the block must call
// this (it synchronises); op(p, z, c, L) is called for the points inside the
// grid with p the linear index, c = src[p] and L = L_h src at p.  An op with a
// member pre(p) (a load of its own, such as the right-hand side) has it issued
// one plane ahead, with the plane loads, and gets the value as op(p, z, c, L, v).
// A block whose lane is gated (its solve has stopped) leaves after the
// prologue and the march returns false: the gate's load then goes out beside
// the prologue's loads instead of in front of them.  mid() is called by every
// thread once the prologue's loads are issued and before their values are
// used; when it returns false the march returns false (a decision that needs
// loads of its own overlaps them with the prologue's).
template <class Op, class = void>
struct OpPre {
    static constexpr bool value = false;
};
template <class Op>
struct OpPre<Op, std::void_t<decltype(&Op::pre)>> {
    static constexpr bool value = true;
};

template <class Op, class = void>
struct OpBegin {
    static constexpr bool value = false;
};
template <class Op>
struct OpBegin<Op, std::void_t<decltype(&Op::begin)>> {
    static constexpr bool value = true;
};

template <int ORDER>
struct Halo {
    static constexpr int R = ORDER == 2 ? 1 : 2;
    static constexpr int LW = HS_TX + 2 * R;
    static constexpr int LH = HS_TY + 2 * R;
    static constexpr int NH = 2 * R * HS_TY + 2 * R * LW;      // halo cells per plane
    static constexpr int HPT = (NH + HS_BLOCK - 1) / HS_BLOCK;  // halo cells per thread
};

struct MidNone {
    __device__ __forceinline__ bool operator()() const { return true; }
};

template <int ORDER, typename T, class Src, typename Op, class Mid = MidNone>
__device__ __forceinline__ bool lds_march_src(const Src& S, int n, int i0, int j0, int z0, int z1,
                                              T (*pl)[Halo<ORDER>::LH][Halo<ORDER>::LW], Op& op,
                                              bool gated = false, Mid mid = Mid())
{
    using H = Halo<ORDER>;
    constexpr int R = H::R;
    const long long nn = (long long)n * n;
    const int lx = threadIdx.x % HS_TX, ly = threadIdx.x / HS_TX;
    const int i = i0 + lx, j = j0 + ly;
    const bool in = i < n && j < n;
    const T sc = lap_scale<ORDER, T>(n);
    // this thread's halo cells
    int hrow[H::HPT], hcol[H::HPT], hgi[H::HPT], hgj[H::HPT];
    long long hoff[H::HPT];
    bool hin[H::HPT];
#pragma unroll
    for (int h = 0; h < H::HPT; h++) {
        int q = threadIdx.x + HS_BLOCK * h;
        int lrow = -1, lcol = 0;
        if (q < H::NH) {
            if (q < 2 * R * HS_TY) {
                lrow = q / (2 * R) + R;
                int c = q % (2 * R);
                lcol = c < R ? c : HS_TX + c;
            } else {
                int t = q - 2 * R * HS_TY;
                int rr = t / H::LW;
                lrow = rr < R ? rr : HS_TY + rr;
                lcol = t % H::LW;
            }
        }
        int gi = i0 + lcol - R, gj = j0 + lrow - R;
        hrow[h] = lrow;
        hcol[h] = lcol;
        hgi[h] = gi;
        hgj[h] = gj;
        hin[h] = lrow >= 0 && gi >= 0 && gi < n && gj >= 0 && gj < n;
        hoff[h] = hin[h] ? (long long)gj * n + gi : 0;
    }
    const long long pij = (long long)j * n + i;
    constexpr bool PRE = OpPre<Op>::value, SPLIT = Src::kSplit;
    T w[2 * R + 1], hr[H::HPT];
    T pv = T(0);
    typename Src::Col cc, hc[H::HPT];
    if constexpr (SPLIT) {
        // the prologue's loads first (column window, halo of plane z0, the
        // op's own value), then the column weights and the op's set-up while
        // they are in flight, then the finishing steps
#pragma unroll
        for (int d = -R; d <= R; d++) {
            const int zm = zmirror<ORDER>(z0 + d, n);
            w[d + R] = (in && zm >= 0) ? S.raw(pij + (long long)zm * nn) : T(0);
        }
#pragma unroll
        for (int h = 0; h < H::HPT; h++) hr[h] = hin[h] ? S.raw((long long)z0 * nn + hoff[h]) : T(0);
        if constexpr (PRE) pv = in ? op.pre(pij + (long long)z0 * nn) : T(0);
        if (!mid()) return false;
        if constexpr (OpBegin<Op>::value) op.begin();
        cc = S.col(i, j);
#pragma unroll
        for (int h = 0; h < H::HPT; h++) hc[h] = S.col(hgi[h], hgj[h]);
#pragma unroll
        for (int d = -R; d <= R; d++) w[d + R] = in ? zfix_src<ORDER, T>(S, cc, w[d + R], z0 + d, n) : T(0);
#pragma unroll
        for (int h = 0; h < H::HPT; h++) hr[h] = hin[h] ? S.fix(hr[h], hc[h], z0) : T(0);
    } else {
        // a plain source: the set-up first, then the loads with the wall rules
        // applied in place (measured faster for this form)
        if constexpr (OpBegin<Op>::value) op.begin();
        cc = S.col(i, j);
#pragma unroll
        for (int h = 0; h < H::HPT; h++) hc[h] = S.col(hgi[h], hgj[h]);
#pragma unroll
        for (int d = -R; d <= R; d++) w[d + R] = in ? zval_src<ORDER, T>(S, cc, z0 + d, n, nn, pij) : T(0);
        if constexpr (PRE) pv = in ? op.pre(pij + (long long)z0 * nn) : T(0);
#pragma unroll
        for (int h = 0; h < H::HPT; h++) hr[h] = hin[h] ? S.at((long long)z0 * nn + hoff[h], hc[h], z0) : T(0);
        if (!mid()) return false;
    }
#pragma unroll
    for (int h = 0; h < H::HPT; h++)
        if (hrow[h] >= 0) pl[0][hrow[h]][hcol[h]] = hr[h];
    pl[0][ly + R][lx + R] = w[R];
    __syncthreads();
    if (gated) return false;
    int buf = 0;
    for (int z = z0; z < z1; z++) {
        const bool more = z + 1 < z1;
        T hv[H::HPT];
        const long long pz1 = (long long)(z + 1) * nn;
#pragma unroll
        for (int h = 0; h < H::HPT; h++)
            hv[h] = (more && hin[h]) ? (SPLIT ? S.raw(pz1 + hoff[h]) : S.at(pz1 + hoff[h], hc[h], z + 1)) : T(0);
        T wn = T(0);
        if constexpr (SPLIT) {
            const int zmn = zmirror<ORDER>(z + R + 1, n);
            wn = (more && in && zmn >= 0) ? S.raw(pij + (long long)zmn * nn) : T(0);
        } else {
            wn = (more && in) ? zval_src<ORDER, T>(S, cc, z + R + 1, n, nn, pij) : T(0);
        }
        T pn = T(0);
        if constexpr (PRE) pn = (more && in) ? op.pre(pz1 + pij) : T(0);
        if (in) {
            const T L = plane_lap<ORDER, T, H::LW>(&pl[buf][ly + R][lx + R], w, i, j, n);
            if constexpr (PRE) op((long long)z * nn + pij, z, w[R], sc * L, pv);
            else op((long long)z * nn + pij, z, w[R], sc * L);
        }
        pv = pn;
        if (more) {
#pragma unroll
            for (int h = 0; h < H::HPT; h++)
                if (hrow[h] >= 0)
                    pl[buf ^ 1][hrow[h]][hcol[h]] = SPLIT ? (hin[h] ? S.fix(hv[h], hc[h], z + 1) : T(0)) : hv[h];
            pl[buf ^ 1][ly + R][lx + R] = w[R + 1];
        }
#pragma unroll
        for (int d = 0; d < 2 * R; d++) w[d] = w[d + 1];
        if constexpr (SPLIT) w[2 * R] = (more && in) ? zfix_src<ORDER, T>(S, cc, wn, z + R + 1, n) : T(0);
        else w[2 * R] = wn;
        __syncthreads();
        buf ^= 1;
    }
    return true;
}

template <int ORDER, typename T, typename Op, class Mid = MidNone>
__device__ __forceinline__ bool lds_march(const HS_G T* __restrict__ src, int n, int i0, int j0, int z0,
                                          int z1, T (*pl)[Halo<ORDER>::LH][Halo<ORDER>::LW], Op& op,
                                          bool gated = false, Mid mid = Mid())
{
    SrcPlain<T> S{src};
    return lds_march_src<ORDER, T>(S, n, i0, j0, z0, z1, pl, op, gated, mid);
}

// ---------------------------------------------------------------------------
// Multigrid kernels
// ---------------------------------------------------------------------------

template <typename T, int ORDER, int MODE, int NORM>
struct SweepOp {
    HS_G T* __restrict__ dst;
    const HS_G T* __restrict__ b;
    T a;
    ColRd<ORDER, T> rd;   // omega / D on this thread's column, formed by begin()
    T om;
    int i, j, n;
    int cycle;
    double rmax, bmax;
    __device__ __forceinline__ SweepOp(T a_, T om_, int i_, int j_, int n_) : a(a_), om(om_), i(i_), j(j_), n(n_) {}
    __device__ __forceinline__ void begin() { rd = ColRd<ORDER, T>(a, om, i, j, n); }
    __device__ __forceinline__ T pre(long long p) const { return b[p]; }
    __device__ __forceinline__ void operator()(long long p, int z, T c, T L, T bp)
    {
        T r = bp - (c - a * L);
        if (MODE == 0) dst[p] = c + rd.at(z, n) * r;
        else dst[p] = r;
        if (NORM) {
            rmax = nmax(rmax, (double)tabs(r));
            if (cycle == 0) bmax = nmax(bmax, (double)tabs(bp));
        }
    }
};

// MODE 0: weighted Jacobi  dst = x + omega D^{-1} (b - A_a x)  (from a zero
// guess on correction grids: dst = omega D^{-1} b); MODE 1: residual
// dst = b - A_a x.  x is the buffer picked by src_is_t, dst the other one.
// NORM 1: per-block maxima of |b - A_a x| (and |b| at cycle 0) to partials.
// NORM 2: first the stopping test before cycle `cycle` (as mg_decide takes
// it) from the maxima a NORM 1 launch over the same table left in partials;
// every block reduces its lane's maxima and decides alike, the lane's first
// block records the outcome, and lanes that stop return before sweeping.
// SRC 1: x is the zero-guess first sweep omega D^{-1} b, formed on the fly
// (this launch is the second sweep of a correction grid).
template <typename T, int ORDER, int MODE, int FINEST, int NORM_, int SRC>
__global__ void __launch_bounds__(HS_BLOCK) k_sweep(const GridSeg* __restrict__ segs, int nseg,
                                                    int nblk, LaneCtl* __restrict__ ctl,
                                                    hsk::MgArgs A, int first_sweep, int src_is_t,
                                                    double* __restrict__ partials, int cycle, double tol,
                                                    int max_cycles)
{
    constexpr int NORM = NORM_ == 1;
    int lb = xcd_remap(blockIdx.x, nblk);
    int si = find_seg(segs, nseg, lb);
    const GridSeg sg = segs[si];
    // the gate is read beside the first loads and tested after them
    const int lane_state = ld_state(ctl, sg.lane);
    const bool gated = A.gate && lane_state != 0;
    // NORM 2: the lane's partial maxima are loaded here (two per thread cover
    // a norm sweep of up to 2 HS_BLOCK blocks, a loop takes any more) and
    // reduced once the march's first loads are out
    const int b0 = sg.blk_begin, nb = NORM_ == 2 ? seg_nblk(segs, nseg, si, nblk) : 0;
    double pr[2] = {0.0, 0.0}, pb[2] = {0.0, 0.0};
    if (NORM_ == 2) {
#pragma unroll
        for (int k = 0; k < 2; k++) {
            const int q = (int)threadIdx.x + k * HS_BLOCK;
            if (q < nb) {
                pr[k] = partials[2 * (b0 + q)];
                if (cycle == 0) pb[k] = partials[2 * (b0 + q) + 1];
            }
        }
    }
    __shared__ int s_state;
    // the stopping test (NORM 2); false: the lane stops (or is gated) and the block returns
    auto decide = [&]() -> bool {
        double r = nmax(pr[0], pr[1]), bb = nmax(pb[0], pb[1]);
        for (int q = (int)threadIdx.x + 2 * HS_BLOCK; q < nb; q += HS_BLOCK) {
            r = nmax(r, partials[2 * (b0 + q)]);
            if (cycle == 0) bb = nmax(bb, partials[2 * (b0 + q) + 1]);
        }
        block_max2(r, bb);
        if (gated) return false;
        if (threadIdx.x == 0) {
            LaneCtl& c = ctl[sg.lane];
            const double bn = cycle == 0 ? bb : c.bnorm;
            const double rho = r / (bn > 0.0 ? bn : 1.0);
            const bool bad = rho != rho || r > 1.7e308;
            const int state = bad ? 2 : (rho <= tol ? 1 : (cycle >= max_cycles ? 2 : 0));
            if (lb == b0) {
                if (cycle == 0) c.bnorm = bn;
                c.mg_rho = rho;
                if (state != 0) {
                    finish_solve(c, cycle, state, A.L);
                    if (bad) c.status = -4;
                    else if (state == 2 && c.status == 0) c.status = -3;
                }
            }
            s_state = state;
        }
        __syncthreads();
        return s_state == 0;
    };
    if (NORM_ == 2 && (src_is_t & 4) && sg.coarse) {
        decide();
        return;
    }
    if ((src_is_t & 4) && sg.coarse) return;
    const int n = sg.n;
    PosZ q = grid_pos_z(lb - sg.blk_begin, n, sg.zb);
    HS_G T* U = (HS_G T*)sg.u + (long long)A.node * sg.node_stride;
    HS_G T* Tt = (HS_G T*)sg.t;
    const HS_G T* B = (const HS_G T*)sg.b;
    const int st = seg_src(src_is_t, sg);
    const HS_G T* src = st ? Tt : U;
    HS_G T* dst = st ? U : Tt;
    const T om = T(A.omega);
    SweepOp<T, ORDER, MODE, NORM> op(T(lane_a(ctl, sg.lane, A.L, A.m)), om, q.i, q.j, n);
    op.dst = dst;
    op.b = B;
    op.cycle = cycle;
    op.rmax = 0.0;
    op.bmax = 0.0;
    if (SRC == 0 && MODE == 0 && !FINEST && first_sweep && sg.coarse) {
        if (gated) return;
        op.begin();
        if (q.in)
            for (int z = q.z0; z < q.z1; z++) {
                long long p = lin(q.i, q.j, z, n);
                dst[p] = op.rd.at(z, n) * B[p];
            }
    } else {
        __shared__ T pl[2][Halo<ORDER>::LH][Halo<ORDER>::LW];
        const int i0 = q.i - (int)(threadIdx.x % HS_TX), j0 = q.j - (int)(threadIdx.x / HS_TX);
        // NORM 2 takes the gate with the stopping test, inside the march
        bool ran;
        if constexpr (NORM_ == 2) {
            ran = lds_march<ORDER, T>(src, n, i0, j0, q.z0, q.z1, pl, op, false, decide);
        } else if (SRC == 1 && sg.coarse) {
            SrcZeroJacobi<T, ORDER> S{B, op.a, om, n};
            ran = lds_march_src<ORDER, T>(S, n, i0, j0, q.z0, q.z1, pl, op, gated);
        } else {
            ran = lds_march<ORDER, T>(src, n, i0, j0, q.z0, q.z1, pl, op, gated);
        }
        if (!ran) return;
    }
    if (NORM) {
        // |b| is taken once per solve
        double m = op.rmax, mb = op.bmax;
        if (cycle == 0) {
            block_max2(m, mb);
        } else {
            m = block_max(m);
            mb = 0.0;
        }
        if (threadIdx.x == 0) {
            partials[2 * lb] = m;
            partials[2 * lb + 1] = mb;
        }
    }
}

// Two weighted-Jacobi sweeps in one pass (temporal blocking, the
// several-sweeps-per-pass remedy for the smoother's memory traffic):
// v = J(x), dst = J(v), x the buffer picked by src_is_t, dst the other one;
// v is never stored.  The block marches zj = z0-R .. z1-1+R.  On each plane
// zj it forms v over its tile plus a halo of R: the x/y neighbours come from
// plane zj of x over the tile plus 2R in LDS, the z neighbours from a
// register window per v point (each thread owns up to two v points).  v goes
// to an LDS ring of 2R+1 planes, from which dst is formed on plane zj-R over
// the tile.  v outside the grid is 0; its wall planes follow the stencil's z
// rules (v(-1) = v(n) = 0, v(-2) = -v(0), v(n+1) = -v(n-1)).  NORM: per-block
// maxima of the first sweep's residual over the tile's planes z0..z1-1 (and of
// |b| at cycle 0), as the sweep with the norm.  Same operations, in the same
// order, as two separate sweeps.
template <int ORDER>
struct J2Tile {
    static constexpr int R = ORDER == 2 ? 1 : 2;
    static constexpr int NZ = 2 * R + 1;                    // v ring planes
    static constexpr int UW = HS_TX + 4 * R, UH = HS_TY + 4 * R;
    static constexpr int VW = HS_TX + 2 * R, VH = HS_TY + 2 * R;
    static constexpr int NV = VW * VH;
    static constexpr int VPT = (NV + HS_BLOCK - 1) / HS_BLOCK;
    static constexpr int NO = UW * UH - NV;                  // x cells outside the v region
    static constexpr int OPT = (NO + HS_BLOCK - 1) / HS_BLOCK;
};

template <typename T, int ORDER, int NORM>
__global__ void __launch_bounds__(HS_BLOCK) k_jac2(const GridSeg* __restrict__ segs, int nseg, int nblk,
                                                  const LaneCtl* __restrict__ ctl, hsk::MgArgs A,
                                                  int src_is_t, double* __restrict__ partials, int cycle)
{
    using G = J2Tile<ORDER>;
    constexpr int R = G::R, NZ = G::NZ;
    static_assert(G::VPT <= 2 && G::OPT <= 1, "tile");
    __shared__ T ub[2][G::UH][G::UW];
    __shared__ T vr[NZ][G::VH][G::VW];
    const int lb = xcd_remap(blockIdx.x, nblk);
    const int si = find_seg(segs, nseg, lb);
    const GridSeg sg = segs[si];
    if (A.gate && ctl[sg.lane].mg_state != 0) return;
    const int n = sg.n;
    const PosZ q = grid_pos_z(lb - sg.blk_begin, n, sg.zb);
    const int t = (int)threadIdx.x;
    const int lx = t % HS_TX, ly = t / HS_TX;
    const int i = q.i, j = q.j, x0 = i - lx, y0 = j - ly;
    const int z0 = q.z0, z1 = q.z1;
    const bool in = i < n && j < n;
    const int nn = n * n;   // offsets stay below 2^31 for n <= 511
    HS_G T* U = (HS_G T*)sg.u + (long long)A.node * sg.node_stride;
    HS_G T* Tt = (HS_G T*)sg.t;
    const int st = seg_src(src_is_t, sg);
    const HS_G T* x = st ? Tt : U;
    HS_G T* dst = st ? U : Tt;
    const HS_G T* B = (const HS_G T*)sg.b;
    const T a = T(lane_a(ctl, sg.lane, A.L, A.m));
    const T om = T(A.omega);
    const T sc = lap_scale<ORDER, T>(n);
    SrcPlain<T> S{x};
    double rmax = 0.0, bmax = 0.0;
    // v points of this thread
    int vx[G::VPT], vy[G::VPT], vgi[G::VPT], vgj[G::VPT];
    bool vok[G::VPT], vin[G::VPT], vmain[G::VPT];
#pragma unroll
    for (int k = 0; k < G::VPT; k++) {
        const int c = t + HS_BLOCK * k;
        vok[k] = c < G::NV;
        vx[k] = vok[k] ? c % G::VW : 0;
        vy[k] = vok[k] ? c / G::VW : 0;
        vgi[k] = x0 - R + vx[k];
        vgj[k] = y0 - R + vy[k];
        vin[k] = vok[k] && vgi[k] >= 0 && vgi[k] < n && vgj[k] >= 0 && vgj[k] < n;
        vmain[k] = vin[k] && vx[k] >= R && vx[k] < R + HS_TX && vy[k] >= R && vy[k] < R + HS_TY;
    }
    ColRd<ORDER, T> vrd[G::VPT] = {};
#pragma unroll
    for (int k = 0; k < G::VPT; k++) vrd[k] = ColRd<ORDER, T>(a, om, vgi[k], vgj[k], n);
    const ColRd<ORDER, T> rd(a, om, i, j, n);
    // x cell outside the v region loaded by this thread
    int orow = -1, ocol = 0, ooff = 0, ogi = 0, ogj = 0;
    bool oin = false;
    if (t < G::NO) {
        const int top = R * G::UW, side = G::VH * 2 * R;
        if (t < top) {
            orow = t / G::UW;
            ocol = t % G::UW;
        } else if (t < top + side) {
            const int s = t - top;
            orow = R + s / (2 * R);
            const int kk = s % (2 * R);
            ocol = kk < R ? kk : G::VW + kk;
        } else {
            const int s = t - top - side;
            orow = R + G::VH + s / G::UW;
            ocol = s % G::UW;
        }
        ogi = x0 - 2 * R + ocol;
        ogj = y0 - 2 * R + orow;
        oin = ogi >= 0 && ogi < n && ogj >= 0 && ogj < n;
        ooff = oin ? ogj * n + ogi : 0;
    }
    auto xz = [&](int gi, int gj, int zz) -> T {   // x at (gi, gj, zz) with the z wall rules
        return zval_src<ORDER, T>(S, S.col(gi, gj), zz, n, nn, (long long)gj * n + gi);
    };
    const int zs = z0 - R, ze = z1 - 1 + R;   // v planes formed by the block
    // z windows of the v points: x planes zs-R .. zs+R
    T wv[G::VPT][2 * R + 1];
#pragma unroll
    for (int k = 0; k < G::VPT; k++)
#pragma unroll
        for (int d = 0; d <= 2 * R; d++) wv[k][d] = vin[k] ? xz(vgi[k], vgj[k], zs - R + d) : T(0);
    // x plane zs
    if (orow >= 0) ub[zs & 1][orow][ocol] = oin ? xz(ogi, ogj, zs) : T(0);
#pragma unroll
    for (int k = 0; k < G::VPT; k++)
        if (vok[k]) ub[zs & 1][vy[k] + R][vx[k] + R] = wv[k][R];
    __syncthreads();
    auto slot = [](int zz) { return ((zz % NZ) + NZ) % NZ; };
    for (int zj = zs; zj <= ze; zj++) {
        const bool more = zj + 1 <= ze;
        // loads for the next plane and this plane's right-hand sides
        T on = (more && oin) ? xz(ogi, ogj, zj + 1) : T(0);
        T wn[G::VPT], bv[G::VPT];
#pragma unroll
        for (int k = 0; k < G::VPT; k++) {
            wn[k] = (more && vin[k]) ? xz(vgi[k], vgj[k], zj + 1 + R) : T(0);
            bv[k] = (vin[k] && zj >= 0 && zj < n) ? B[zj * nn + vgj[k] * n + vgi[k]] : T(0);
        }
        const int zo = zj - R;   // plane of dst formed in this step
        const bool out = zo >= z0 && zo < z1 && in;
        const T bo = out ? B[zo * nn + j * n + i] : T(0);
        // first sweep on plane zj over the tile plus R
#pragma unroll
        for (int k = 0; k < G::VPT; k++) {
            if (!vok[k]) continue;
            T v = T(0);
            if (zj >= 0 && zj < n) {
                if (vin[k]) {
                    const T c = wv[k][R];
                    const T L = plane_lap<ORDER, T, G::UW>(&ub[zj & 1][vy[k] + R][vx[k] + R], wv[k], vgi[k],
                                                           vgj[k], n);
                    const T r = bv[k] - (c - a * (sc * L));
                    v = c + vrd[k].at(zj, n) * r;
                    if (NORM && vmain[k] && zj >= z0 && zj < z1) {
                        rmax = nmax(rmax, (double)tabs(r));
                        if (cycle == 0) bmax = nmax(bmax, (double)tabs(bv[k]));
                    }
                }
                if (ORDER == 4 && zj == 0) vr[slot(-2)][vy[k]][vx[k]] = -v;
            } else if (ORDER == 4 && zj == n + 1) {
                v = -vr[slot(n - 1)][vy[k]][vx[k]];
            }
            if (!(ORDER == 4 && zj == -2)) vr[slot(zj)][vy[k]][vx[k]] = v;
        }
        __syncthreads();
        // second sweep on plane zo over the tile
        if (out) {
            const int yy = ly + R, xx = lx + R;
            T w2[2 * R + 1];
#pragma unroll
            for (int d = 0; d <= 2 * R; d++) w2[d] = vr[slot(zo - R + d)][yy][xx];
            const T c = w2[R];
            const T L = plane_lap<ORDER, T, G::VW>(&vr[slot(zo)][yy][xx], w2, i, j, n);
            const T r = bo - (c - a * (sc * L));
            dst[zo * nn + j * n + i] = c + rd.at(zo, n) * r;
        }
        // x plane zj+1
        if (more) {
            if (orow >= 0) ub[(zj + 1) & 1][orow][ocol] = on;
#pragma unroll
            for (int k = 0; k < G::VPT; k++)
                if (vok[k]) ub[(zj + 1) & 1][vy[k] + R][vx[k] + R] = wv[k][R + 1];
        }
#pragma unroll
        for (int k = 0; k < G::VPT; k++) {
#pragma unroll
            for (int d = 0; d < 2 * R; d++) wv[k][d] = wv[k][d + 1];
            wv[k][2 * R] = wn[k];
        }
        __syncthreads();
    }
    if (NORM) {
        double m = rmax, mb = bmax;
        if (cycle == 0) {
            block_max2(m, mb);
        } else {
            m = block_max(m);
            mb = 0.0;
        }
        if (t == 0) {
            partials[2 * lb] = m;
            partials[2 * lb + 1] = mb;
        }
    }
}

// Residual and full weighting in one pass: cb(I) = sum over the 27 fine
// neighbours of 2I+1 of (1/4,1/2,1/4)^3 (b - A_a x), x the buffer picked by
// src_is_t; the fine residual is never stored.  The block owns the fine tile
// x0..x0+63, y0..y0+7, planes z0..z1-1 (x0, y0, z0 and the chunk length
// even) and the coarse points whose centre 2I+1 lies in it.  Their weights
// reach one fine column, row and plane beyond the tile on the high side, so
// the residual is formed on (64+1) x (8+1) points per plane and on planes
// z0..z1 (threads 0..72, waves 0-1, take the extra column and row with their
// own z window).  Per plane the residual goes to one of two LDS buffers; the
// 128 coarse-point owners (waves 2-3) add the xy-weighted sum of the previous
// plane's residual to their running z sum while the next one is formed, so a
// plane costs one barrier.  Per coarse point the weights are summed in the
// order: x within a row, rows within a plane, planes.
template <int ORDER>
struct RfwTile {
    static constexpr int R = ORDER == 2 ? 1 : 2;
    static constexpr int RX = HS_TX + 1, RY = HS_TY + 1;        // residual points per plane
    static constexpr int LW = RX + 2 * R, LH = RY + 2 * R;      // x plane in LDS
    static constexpr int NH = LW * LH - HS_TX * HS_TY;         // cells not owned by a main thread
    static constexpr int HPT = (NH + HS_BLOCK - 1) / HS_BLOCK;
    static constexpr int NX = HS_TY + RX;                       // extra residual points
    static constexpr int NC = (HS_TX / 2) * (HS_TY / 2);        // coarse points per tile
};

// At most 6 waves per SIMD (up to 80 VGPRs): with a 64-register cap the
// 4th-order kernel spilled.
template <typename T, int ORDER>
__global__ void __launch_bounds__(HS_BLOCK, 6) k_resid_fw(const GridSeg* __restrict__ segs, int nseg,
                                                       int nblk, const LaneCtl* __restrict__ ctl,
                                                       hsk::MgArgs A, int src_is_t)
{
    using G = RfwTile<ORDER>;
    constexpr int R = G::R;
    static_assert(G::HPT <= 2 && G::NX <= HS_BLOCK && G::NC <= HS_BLOCK, "tile");
    __shared__ T pl[2][G::LH][G::LW];
    __shared__ T rp[2][G::RY][G::RX];
    const int lb = xcd_remap(blockIdx.x, nblk);
    const int si = find_seg(segs, nseg, lb);
    const GridSeg sg = segs[si];
    // the gate is read beside the prologue loads and tested after them
    const int lane_state = ld_state(ctl, sg.lane);
    const bool gated = A.gate && lane_state != 0;
    const int n = sg.n, nc = sg.nc;
    const PosZ q = grid_pos_z(lb - sg.blk_begin, n, sg.zb);
    const int t = (int)threadIdx.x;
    const int lx = t % HS_TX, ly = t / HS_TX;
    const int x0 = q.i - lx, y0 = q.j - ly;
    const int z0 = q.z0, zl = min(q.z1, n - 1);   // residual planes z0..zl
    const int nn = n * n;   // offsets stay below 2^31 for n <= 511
    const HS_G T* U = (const HS_G T*)sg.u + (long long)A.node * sg.node_stride;
    const HS_G T* x = seg_src(src_is_t, sg) ? (const HS_G T*)sg.t : U;
    const HS_G T* B = (const HS_G T*)sg.b;
    HS_G T* cb = (HS_G T*)sg.cb;
    const T a = T(lane_a(ctl, sg.lane, A.L, A.m));
    const T sc = lap_scale<ORDER, T>(n);
    SrcPlain<T> S{x};
    // main point
    const int i = q.i, j = q.j;
    const bool in = i < n && j < n;
    const int pij = j * n + i;
    // extra point: column x0+64 (rows y0..y0+7), then row y0+8 (x0..x0+64)
    const bool has_x = t < G::NX;
    const int exl = t < HS_TY ? HS_TX : t - HS_TY, eyl = t < HS_TY ? t : HS_TY;
    const int ei = x0 + exl, ej = y0 + eyl;
    const bool ein = has_x && ei < n && ej < n;
    const int epij = ej * n + ei;
    // cells of the LDS plane loaded by this thread besides its main point
    int hrow[G::HPT], hcol[G::HPT], hgi[G::HPT], hgj[G::HPT];
    bool hin[G::HPT];
    int hoff[G::HPT];
#pragma unroll
    for (int h = 0; h < G::HPT; h++) {
        // enumerate the plane's cells, skipping the main 64 x 8 block
        int c = t + HS_BLOCK * h;
        int lrow = -1, lcol = 0;
        if (c < G::NH) {
            // rows above the main block, then rows beside it, then rows below
            const int top = R * G::LW;                        // rows 0..R-1
            const int side = HS_TY * (G::LW - HS_TX);         // rows R..R+7, cells outside the main columns
            if (c < top) {
                lrow = c / G::LW;
                lcol = c % G::LW;
            } else if (c < top + side) {
                const int s = c - top, per = G::LW - HS_TX;
                lrow = R + s / per;
                const int k = s % per;
                lcol = k < R ? k : HS_TX + k;
            } else {
                const int s = c - top - side;
                lrow = R + HS_TY + s / G::LW;
                lcol = s % G::LW;
            }
        }
        const int gi = x0 + lcol - R, gj = y0 + lrow - R;
        hrow[h] = lrow;
        hcol[h] = lcol;
        hgi[h] = gi;
        hgj[h] = gj;
        hin[h] = lrow >= 0 && gi >= 0 && gi < n && gj >= 0 && gj < n;
        hoff[h] = hin[h] ? gj * n + gi : 0;
    }
    // coarse point owned by this thread (waves 2-3)
    const int to = t - 2 * 64;
    const bool own = to >= 0 && to < G::NC;
    const int I = (x0 >> 1) + (to % (HS_TX / 2)), J = (y0 >> 1) + (to / (HS_TX / 2));
    const bool cin = own && I < nc && J < nc;
    const int cx = 2 * I + 1 - x0, cyy = 2 * J + 1 - y0;   // centre in rp
    T acc = T(0);
    int kopen = -1;   // coarse plane being summed
    const T wfw[3] = {T(0.25), T(0.5), T(0.25)};
    // column windows
    T w[2 * R + 1], we[2 * R + 1];
#pragma unroll
    for (int d = -R; d <= R; d++) {
        w[d + R] = in ? zval_src<ORDER, T>(S, S.col(i, j), z0 + d, n, nn, pij) : T(0);
        we[d + R] = ein ? zval_src<ORDER, T>(S, S.col(ei, ej), z0 + d, n, nn, epij) : T(0);
    }
    // right-hand side of the plane being formed, loaded one plane ahead
    T bv = in ? B[z0 * nn + pij] : T(0);
    T bev = ein ? B[z0 * nn + epij] : T(0);
    {
        const int pz = z0 * nn;
#pragma unroll
        for (int h = 0; h < G::HPT; h++)
            if (hrow[h] >= 0) pl[0][hrow[h]][hcol[h]] = hin[h] ? S.at(pz + hoff[h], S.col(0, 0), z0) : T(0);
        pl[0][ly + R][lx + R] = w[R];
    }
    __syncthreads();
    if (gated) return;
    // full weighting of residual plane zp (in rp[zp & 1]) into the running sums
    auto fw_plane = [&](int zp) {
        T az = T(0);
#pragma unroll
        for (int dy = -1; dy <= 1; dy++) {
            const T* row = &rp[zp & 1][cyy + dy][cx];
            T ay = (wfw[0] * row[-1] + wfw[1] * row[0]) + wfw[2] * row[1];
            az += wfw[dy + 1] * ay;
        }
        // coarse plane K takes fine planes 2K, 2K+1, 2K+2
        if (zp & 1) {
            if (kopen >= 0) acc += wfw[1] * az;
        } else {
            if (kopen >= 0) {
                acc += wfw[2] * az;
                cb[lin(I, J, kopen, nc)] = acc;
                kopen = -1;
            }
            const int K = zp >> 1;
            if (zp < q.z1 && K < nc) {
                acc = T(0);
                acc += wfw[0] * az;
                kopen = K;
            }
        }
    };
    int buf = 0;
    for (int z = z0; z <= zl; z++) {
        const bool more = z + 1 <= zl;
        T hv[G::HPT];
        const int pz1 = (z + 1) * nn;
#pragma unroll
        for (int h = 0; h < G::HPT; h++)
            hv[h] = (more && hin[h]) ? S.at(pz1 + hoff[h], S.col(0, 0), z + 1) : T(0);
        const T wn = (more && in) ? zval_src<ORDER, T>(S, S.col(i, j), z + R + 1, n, nn, pij) : T(0);
        const T wen = (more && ein) ? zval_src<ORDER, T>(S, S.col(ei, ej), z + R + 1, n, nn, epij) : T(0);
        const T bn = (more && in) ? B[pz1 + pij] : T(0);
        const T ben = (more && ein) ? B[pz1 + epij] : T(0);
        // residual on the main and the extra points of plane z
        T r = T(0);
        if (in) {
            const T L = plane_lap<ORDER, T, G::LW>(&pl[buf][ly + R][lx + R], w, i, j, n);
            r = bv - (w[R] - a * (sc * L));
        }
        rp[z & 1][ly][lx] = r;
        if (has_x) {
            T re = T(0);
            if (ein) {
                const T L = plane_lap<ORDER, T, G::LW>(&pl[buf][eyl + R][exl + R], we, ei, ej, n);
                re = bev - (we[R] - a * (sc * L));
            }
            rp[z & 1][eyl][exl] = re;
        }
        bv = bn;
        bev = ben;
        if (cin && z > z0) fw_plane(z - 1);
        if (more) {
#pragma unroll
            for (int h = 0; h < G::HPT; h++)
                if (hrow[h] >= 0) pl[buf ^ 1][hrow[h]][hcol[h]] = hv[h];
            pl[buf ^ 1][ly + R][lx + R] = w[R + 1];
        }
#pragma unroll
        for (int d = 0; d < 2 * R; d++) {
            w[d] = w[d + 1];
            we[d] = we[d + 1];
        }
        w[2 * R] = wn;
        we[2 * R] = wen;
        __syncthreads();
        buf ^= 1;
    }
    if (cin) fw_plane(zl);
}

// xy part of the trilinear interpolation of one coarse plane at fine column
// (i, j): wy * (sum over the coarse rows of wx * (sum over the coarse
// columns)).  Per axis a fine index either coincides with coarse (i-1)/2
// (weight 1) or lies between coarse i/2-1 and i/2 (weights 1/2); taps beyond
// a wall are 0.  The full interpolation is wz * (sum over the coarse planes
// of this term).
template <typename T>
struct ProlongXY {
    // coarse indices ix0 (ix1 = ix0 + 1 for even i, = ix0 for odd i), likewise
    // y; bit 0/1: odd i / odd j, bits 2-5: the four index pairs are inside the
    // grid (vx0, vx1, vy0, vy1)
    int ix0, iy0, f;
    ProlongXY() = default;
    __device__ __forceinline__ ProlongXY(int i, int j, int nc)
    {
        const int ox = i & 1, oy = j & 1;
        ix0 = ox ? (i - 1) >> 1 : (i >> 1) - 1;
        iy0 = oy ? (j - 1) >> 1 : (j >> 1) - 1;
        const int ix1 = ox ? ix0 : ix0 + 1, iy1 = oy ? iy0 : iy0 + 1;
        f = ox | (oy << 1) | ((ix0 >= 0) << 2) | ((!ox && ix1 < nc) << 3) | ((iy0 >= 0) << 4) |
            ((!oy && iy1 < nc) << 5);
    }
    __device__ __forceinline__ int ix1() const { return (f & 1) ? ix0 : ix0 + 1; }
    __device__ __forceinline__ int iy1() const { return (f & 2) ? iy0 : iy0 + 1; }
    __device__ __forceinline__ T wx() const { return (f & 1) ? T(1) : T(0.5); }
    __device__ __forceinline__ T wy() const { return (f & 2) ? T(1) : T(0.5); }
    // row base pointers: `plane` points at coarse (0, 0) of the plane (any
    // origin shift folded in), `pitch` is the row length
    template <class P>
    __device__ __forceinline__ T at(P plane, int pitch) const
    {
        const T wxv = wx();
        T sy = T(0);
#pragma unroll
        for (int cy = 0; cy < 2; cy++) {
            const bool vy = cy ? (f & 32) : (f & 16);
            if (!vy) continue;
            const auto row = plane + (cy ? iy1() : iy0) * pitch;
            T sx = T(0);
            if (f & 4) sx += row[ix0];
            if (f & 8) sx += row[ix1()];
            sy += wxv * sx;
        }
        return wy() * sy;
    }
};

// The xy term of ProlongXY read from a zero-padded LDS plane: every tap
// exists (outside the grid it reads 0), so the validity tests become 0/1
// weights and the four reads need no branches.  Adding the exact zeros
// leaves every sum as ProlongXY::at forms it.
template <typename T>
struct RingTap {
    int o;    // offset of coarse (ix0, iy0) in the padded plane
    int f;    // bit 0: odd i, bit 1: odd j
    RingTap() = default;
    __device__ __forceinline__ RingTap(int i, int j, int ox0, int oy0, int pitch)
    {
        const int odx = i & 1, ody = j & 1;
        const int ix0 = odx ? (i - 1) >> 1 : (i >> 1) - 1;
        const int iy0 = ody ? (j - 1) >> 1 : (j >> 1) - 1;
        o = (iy0 - oy0) * pitch + (ix0 - ox0);
        f = odx | (ody << 1);
    }
    template <class P>
    __device__ __forceinline__ T at(P plane, int pitch) const
    {
        const T ex = (f & 1) ? T(0) : T(1), ey = (f & 2) ? T(0) : T(1);
        const T wx = (f & 1) ? T(1) : T(0.5), wy = (f & 2) ? T(1) : T(0.5);
        const T* r0 = plane + o;
        const T* r1 = r0 + pitch;
        const T sx0 = r0[0] + ex * r0[1];
        const T sx1 = r1[0] + ex * r1[1];
        return wy * (wx * sx0 + ey * (wx * sx1));
    }
};

// dst = src + P cu (in place when src and dst are the same buffer).  Each
// thread marches its fine column through the block's planes; the xy
// interpolation of a coarse plane K serves the fine planes 2K, 2K+1, 2K+2
// and is computed once; the planes' terms are summed and scaled by wz as in
// ProlongXY's definition.
template <typename T>
__global__ void __launch_bounds__(HS_BLOCK) k_prolong(const GridSeg* __restrict__ segs, int nseg,
                                                      int nblk, const LaneCtl* __restrict__ ctl,
                                                      hsk::MgArgs A, int src_is_t, int dst_is_t)
{
    int lb = xcd_remap(blockIdx.x, nblk);
    int si = find_seg(segs, nseg, lb);
    const GridSeg sg = segs[si];
    if (A.gate && ctl[sg.lane].mg_state != 0) return;
    const int n = sg.n, nc = sg.nc;
    PosZ q = grid_pos_z(lb - sg.blk_begin, n, sg.zb);
    if (!q.in) return;
    HS_G T* U = (HS_G T*)sg.u + (long long)A.node * sg.node_stride;
    HS_G T* Tt = (HS_G T*)sg.t;
    const HS_G T* src = seg_src(src_is_t, sg) ? Tt : U;
    HS_G T* dst = dst_is_t ? Tt : U;
    const HS_G T* cu = (const HS_G T*)sg.cu;
    const int ncc = nc * nc;
    const ProlongXY<T> xy(q.i, q.j, nc);
    // xy terms of the two most recent coarse planes
    int ka = -2, kb = -2;
    T ea = T(0), eb = T(0);
    auto term = [&](int K) -> T {
        if (K == kb) return eb;
        if (K == ka) return ea;
        T e = xy.at(cu + K * ncc, nc);
        ka = kb;
        ea = eb;
        kb = K;
        eb = e;
        return e;
    };
    for (int z = q.z0; z < q.z1; z++) {
        T corr;
        if (z & 1) {
            corr = T(1) * (T(0) + term((z - 1) >> 1));
        } else {
            const int K0 = (z >> 1) - 1, K1 = z >> 1;
            T s = T(0);
            if (K0 >= 0) s += term(K0);
            if (K1 < nc) s += term(K1);
            corr = T(0.5) * s;
        }
        const int p = lin(q.i, q.j, z, n);
        dst[p] = src[p] + corr;
    }
}

// First post-smoothing sweep with the coarse-grid correction applied as the
// input is read: x = u + P e (u the buffer picked by src_is_t, e = GridSeg::cu
// on the nc^3 grid), dst = x + omega D^{-1} (b - A_a x) into the other buffer;
// the corrected x is never stored.  The coarse planes that the block's fine
// planes interpolate from are staged in an LDS ring of 4 planes, each over
// the 35 x 7 coarse points below the block's 68 x 12 (order 4) fine region
// plus one column and row, one iteration ahead of their first use (a ring
// slot is reused only once no fine plane still to be read interpolates from
// it); coarse points outside the grid are stored as zeros, so the taps read
// without branches.  Each correction adds the same nonzero terms, in the
// same order, as k_prolong, so the result equals k_prolong followed by a
// Jacobi sweep.
struct PjCoarse {
    // coarse cells per ring plane: the 35 x 7 that the fine region interpolates
    // from, plus one column and one row that the branch-free taps read with weight 0
    static constexpr int CW = HS_TX / 2 + 4, CH = HS_TY / 2 + 4;
    static constexpr int NCELL = CW * CH;
    static constexpr int NR = 4;                                   // ring planes
};

template <typename T, int ORDER>
__global__ void __launch_bounds__(HS_BLOCK, 6) k_pjac(const GridSeg* __restrict__ segs, int nseg, int nblk,
                                                  const LaneCtl* __restrict__ ctl, hsk::MgArgs A,
                                                  int src_is_t)
{
    using H = Halo<ORDER>;
    using C = PjCoarse;
    constexpr int R = H::R;
    static_assert(C::NCELL <= HS_BLOCK, "one coarse cell per thread");
    __shared__ T pl[2][H::LH][H::LW];
    __shared__ T cr[C::NR][C::CH][C::CW];
    const int lb = xcd_remap(blockIdx.x, nblk);
    const int si = find_seg(segs, nseg, lb);
    const GridSeg sg = segs[si];
    // the gate is read beside the prologue loads and tested after them
    const int lane_state = ld_state(ctl, sg.lane);
    const bool gated = A.gate && lane_state != 0;
    const int n = sg.n, nc = sg.nc;
    const PosZ q = grid_pos_z(lb - sg.blk_begin, n, sg.zb);
    const int t = (int)threadIdx.x;
    const int lx = t % HS_TX, ly = t / HS_TX;
    const int i = q.i, j = q.j, x0 = i - lx, y0 = j - ly;
    const int z0 = q.z0, z1 = q.z1;
    const bool in = i < n && j < n;
    const int nn = n * n, ncc = nc * nc;   // offsets stay below 2^31 for n <= 511
    HS_G T* U = (HS_G T*)sg.u + (long long)A.node * sg.node_stride;
    HS_G T* Tt = (HS_G T*)sg.t;
    const int st = seg_src(src_is_t, sg);
    const HS_G T* x = st ? Tt : U;
    HS_G T* dst = st ? U : Tt;
    const HS_G T* B = (const HS_G T*)sg.b;
    const HS_G T* cu = (const HS_G T*)sg.cu;
    const T a = T(lane_a(ctl, sg.lane, A.L, A.m));
    const T om = T(A.omega);
    const T sc = lap_scale<ORDER, T>(n);
    const int cx0 = (x0 >> 1) - 2, cy0 = (y0 >> 1) - 2;
    // coarse cell of this thread in a ring plane
    const bool has_c = t < C::NCELL;
    const int ccx = cx0 + t % C::CW, ccy = cy0 + t / C::CW;
    const bool cin = has_c && ccx >= 0 && ccx < nc && ccy >= 0 && ccy < nc;
    const int coff = cin ? ccy * nc + ccx : 0;
    int kl = -1;   // highest coarse plane staged
    // coarse planes fine plane zf interpolates from: klo(zf) .. kneed(zf)
    auto kneed = [&](int zf) { return min(nc - 1, max(0, zf >> 1)); };
    auto klo = [&](int zf) { return max(0, ((zf + 1) >> 1) - 1); };
    // xy term of coarse plane K at fine column (fi, fj), from the ring
    auto term = [&](const RingTap<T>& w, int K) -> T { return w.at(&cr[K & 3][0][0], C::CW); };
    // correction P e at fine plane zf (0 <= zf < n) of the column described by w
    auto corr = [&](const RingTap<T>& w, int zf) -> T {
        if (zf & 1) return T(1) * (T(0) + term(w, (zf - 1) >> 1));
        const int K0 = (zf >> 1) - 1, K1 = zf >> 1;
        T s = T(0);
        if (K0 >= 0) s += term(w, K0);
        if (K1 < nc) s += term(w, K1);
        return T(0.5) * s;
    };
    // value of x that the z wall rules of the stencil read for plane zf of a
    // column (0 beyond the reach of the rules), and the corrected value from it
    auto zraw = [&](int pij, int zf) -> T {
        if (zf >= 0 && zf < n) return x[zf * nn + pij];
        if (ORDER == 4) {
            if (zf == -2) return x[pij];
            if (zf == n + 1) return x[(n - 1) * nn + pij];
        }
        return T(0);
    };
    auto zfix = [&](const RingTap<T>& w, T raw, int zf) -> T {
        if (zf >= 0 && zf < n) return raw + corr(w, zf);
        if (ORDER == 4) {
            if (zf == -2) return -(raw + corr(w, 0));
            if (zf == n + 1) return -(raw + corr(w, n - 1));
        }
        return T(0);
    };
    // halo cells of this thread
    int hrow[H::HPT], hcol[H::HPT], hoff[H::HPT];
    bool hin[H::HPT];
    RingTap<T> hw[H::HPT] = {};
#pragma unroll
    for (int h = 0; h < H::HPT; h++) {
        int qq = t + HS_BLOCK * h;
        int lrow = -1, lcol = 0;
        if (qq < H::NH) {
            if (qq < 2 * R * HS_TY) {
                lrow = qq / (2 * R) + R;
                int c = qq % (2 * R);
                lcol = c < R ? c : HS_TX + c;
            } else {
                int tt = qq - 2 * R * HS_TY;
                int rr = tt / H::LW;
                lrow = rr < R ? rr : HS_TY + rr;
                lcol = tt % H::LW;
            }
        }
        const int gi = x0 + lcol - R, gj = y0 + lrow - R;
        hrow[h] = lrow;
        hcol[h] = lcol;
        hin[h] = lrow >= 0 && gi >= 0 && gi < n && gj >= 0 && gj < n;
        hoff[h] = hin[h] ? gj * n + gi : 0;
        hw[h] = RingTap<T>(hin[h] ? gi : x0 + 1, hin[h] ? gj : y0 + 1, cx0, cy0, C::CW);
    }
    const RingTap<T> mw(in ? i : x0 + 1, in ? j : y0 + 1, cx0, cy0, C::CW);
    const int pij = in ? j * n + i : 0;
    // The prologue's loads go out together: the raw column window and halo of
    // plane z0, the right-hand side of z0, and the coarse planes that the
    // prologue and the first iteration read (at most NR of them).
    T w[2 * R + 1];
#pragma unroll
    for (int d = -R; d <= R; d++) w[d + R] = in ? zraw(pij, z0 + d) : T(0);
    T hr[H::HPT];
#pragma unroll
    for (int h = 0; h < H::HPT; h++) hr[h] = hin[h] ? x[z0 * nn + hoff[h]] : T(0);
    T bv = in ? B[z0 * nn + pij] : T(0);
    {
        const int k0 = klo(z0 - R), kt = kneed(z0 + R + 1);
        T cs[C::NR];
#pragma unroll
        for (int s = 0; s < C::NR; s++) cs[s] = (cin && k0 + s <= kt) ? cu[(k0 + s) * ncc + coff] : T(0);
#pragma unroll
        for (int s = 0; s < C::NR; s++)
            if (has_c && k0 + s <= kt) cr[(k0 + s) & 3][t / C::CW][t % C::CW] = cs[s];
        kl = kt;
    }
    __syncthreads();
    if (gated) return;
    const ColRd<ORDER, T> rd(a, om, i, j, n);
#pragma unroll
    for (int d = -R; d <= R; d++) w[d + R] = in ? zfix(mw, w[d + R], z0 + d) : T(0);
#pragma unroll
    for (int h = 0; h < H::HPT; h++)
        if (hrow[h] >= 0) pl[0][hrow[h]][hcol[h]] = hin[h] ? hr[h] + corr(hw[h], z0) : T(0);
    pl[0][ly + R][lx + R] = w[R];
    __syncthreads();
    int buf = 0;
    for (int z = z0; z < z1; z++) {
        const bool more = z + 1 < z1;
        // raw values of the next plane's halo, the next column value, and the
        // coarse plane(s) the next iteration needs
        T hv[H::HPT];
#pragma unroll
        for (int h = 0; h < H::HPT; h++) hv[h] = (more && hin[h]) ? x[(z + 1) * nn + hoff[h]] : T(0);
        const int kt = more ? kneed(z + R + 2) : kl;
        T cv = (has_c && cin && kt > kl) ? cu[kt * ncc + coff] : T(0);
        const T wr = (more && in) ? zraw(pij, z + R + 1) : T(0);
        const T bn = (more && in) ? B[(z + 1) * nn + pij] : T(0);
        if (in) {
            const T L = plane_lap<ORDER, T, H::LW>(&pl[buf][ly + R][lx + R], w, i, j, n);
            const int p = z * nn + pij;
            const T c = w[R];
            const T r = bv - (c - a * (sc * L));
            dst[p] = c + rd.at(z, n) * r;
        }
        bv = bn;
        const T wn = (more && in) ? zfix(mw, wr, z + R + 1) : T(0);
        if (more) {
#pragma unroll
            for (int h = 0; h < H::HPT; h++)
                if (hrow[h] >= 0) pl[buf ^ 1][hrow[h]][hcol[h]] = hin[h] ? hv[h] + corr(hw[h], z + 1) : T(0);
            pl[buf ^ 1][ly + R][lx + R] = w[R + 1];
        }
        if (kt > kl) {
            if (has_c) cr[kt & 3][t / C::CW][t % C::CW] = cv;
            kl = kt;
        }
#pragma unroll
        for (int d = 0; d < 2 * R; d++) w[d] = w[d + 1];
        w[2 * R] = wn;
        __syncthreads();
        buf ^= 1;
    }
}

// After a solve whose V-cycles each leave the finest iterate in the other
// buffer, lanes that ran an odd number of cycles hold it in t: copy it back
// to the node field u.
__global__ void __launch_bounds__(HS_BLOCK) k_mg_fixup(const GridSeg* __restrict__ segs, int nseg,
                                                       int nblk, const LaneCtl* __restrict__ ctl,
                                                       hsk::MgArgs A)
{
    int lb = xcd_remap(blockIdx.x, nblk);
    int si = find_seg(segs, nseg, lb);
    const GridSeg sg = segs[si];
    const LaneCtl& c = ctl[sg.lane];
    if (!sg.moves || c.mg_state == 3 || (c.mg_cycle & 1) == 0) return;
    if (A.gate == 2 && c.mg_state == 0) return;   // issued ahead of the host's check: stopped solves only
    const int n = sg.n;
    PosZ q = grid_pos_z(lb - sg.blk_begin, n, sg.zb);
    if (!q.in) return;
    HS_G double* U = (HS_G double*)sg.u + (long long)A.node * sg.node_stride;
    const HS_G double* Tt = (const HS_G double*)sg.t;
    for (int z = q.z0; z < q.z1; z++) {
        int p = lin(q.i, q.j, z, n);
        U[p] = Tt[p];
    }
}

// ---------------------------------------------------------------------------
// Coarse tail: every grid with n <= HS_TAIL_N of one lane, one workgroup,
// all grids held in LDS (the right-hand side of the top grid is read from
// global memory).
// ---------------------------------------------------------------------------

// Sizes of the tail grids: level l of a tail whose top grid has n0 points
// per axis, and the LDS offset (in elements) of level l.  Level 0 holds the
// ping-pong pair X, Y (its right-hand side lives in registers); every lower
// level holds X, Y and its right-hand side B.  X and Y carry R = ORDER/2
// layers of zero cells on every face, so the stencil and the prolongation
// read their taps at fixed offsets without tests; B is unpadded.
constexpr int tail_n(int n0, int l) { return ((n0 + 1) >> l) - 1; }
constexpr int tail_cube(int n) { return n * n * n; }
constexpr int tail_r(int order) { return order == 4 ? 2 : 1; }
constexpr int tail_p(int n, int order) { return n + 2 * tail_r(order); }
constexpr int tail_pcube(int n, int order) { return tail_cube(tail_p(n, order)); }
constexpr int tail_words(int n, int order, bool top) { return 2 * tail_pcube(n, order) + (top ? 0 : tail_cube(n)); }
constexpr int tail_off(int n0, int order, int l)
{
    int o = 0;
    for (int q = 0; q < l; q++) o += tail_words(tail_n(n0, q), order, q == 0);
    return o;
}

// index of interior point (i, j, k) of an N^3 tail grid in its padded array
template <int N, int ORDER>
__device__ __forceinline__ int tpad(int i, int j, int k)
{
    constexpr int R = tail_r(ORDER), P = tail_p(N, ORDER);
    return ((k + R) * P + (j + R)) * P + (i + R);
}

// L_h sum at padded index q of a tail grid (row length P, zero cells beyond
// the walls).  The 4th-order tap two cells beyond a wall is the odd
// reflection -c: the zero cell leaves it out, and it is added back as +c per
// wall.
template <int ORDER, typename T, int P>
__device__ __forceinline__ T lap_pad(const T* u, int q, T c, int walls)
{
    constexpr int sy = P, sz = P * P;
    if (ORDER == 2) {
        const T c2 = T(2) * c;
        return ((u[q - 1] - c2) + u[q + 1]) + ((u[q - sy] - c2) + u[q + sy]) + ((u[q - sz] - c2) + u[q + sz]);
    } else {
        const T ax = (T(16) * (u[q - 1] + u[q + 1]) - (u[q - 2] + u[q + 2])) - T(30) * c;
        const T ay = (T(16) * (u[q - sy] + u[q + sy]) - (u[q - 2 * sy] + u[q + 2 * sy])) - T(30) * c;
        const T az = (T(16) * (u[q - sz] + u[q + sz]) - (u[q - 2 * sz] + u[q + 2 * sz])) - T(30) * c;
        return ((ax + ay) + az) + T(walls) * c;
    }
}

// trilinear interpolation at fine point (i, j, k) from a padded coarse tail
// grid of NC points per axis.  Per axis an odd fine index reads coarse
// (i-1)/2 with weight 1 (its second tap is the zero cell at -1), an even one
// coarse i/2-1 and i/2 with weight 1/2 (the zero cells stand for the walls).
template <typename T, int ORDER, int NC>
__device__ __forceinline__ T prolong_pad(const T* c, int i, int j, int k)
{
    constexpr int R = tail_r(ORDER), P = tail_p(NC, ORDER);
    int x0, x1, y0, y1, z0, z1;
    T wx, wy, wz;
    if (i & 1) { x0 = (i - 1) >> 1; x1 = -1; wx = T(1); } else { x0 = (i >> 1) - 1; x1 = i >> 1; wx = T(0.5); }
    if (j & 1) { y0 = (j - 1) >> 1; y1 = -1; wy = T(1); } else { y0 = (j >> 1) - 1; y1 = j >> 1; wy = T(0.5); }
    if (k & 1) { z0 = (k - 1) >> 1; z1 = -1; wz = T(1); } else { z0 = (k >> 1) - 1; z1 = k >> 1; wz = T(0.5); }
    T s = T(0);
#pragma unroll
    for (int cz = 0; cz < 2; cz++) {
        const int oz = ((cz ? z1 : z0) + R) * P * P;
        T sy_ = T(0);
#pragma unroll
        for (int cy = 0; cy < 2; cy++) {
            const int o = oz + ((cy ? y1 : y0) + R) * P + R;
            const T sx = c[o + x0] + c[o + x1];
            sy_ += wx * sx;
        }
        s += wy * sy_;
    }
    return wz * s;
}

// The 1024 threads cover an N^3 tail grid in passes of 64 x rows, 16 threads
// per row (N <= 15); tail_pt gives the point of this thread in pass q.
template <int N>
constexpr int tail_q() { return (N * N + 63) / 64; }

template <int N>
__device__ __forceinline__ bool tail_pt(int q, int& i, int& j, int& k, int& p)
{
    const int r = 64 * q + (int)(threadIdx.x >> 4);
    i = (int)(threadIdx.x & 15);
    if (i >= N || r >= N * N) return false;
    k = r / N;
    j = r - k * N;
    p = r * N + i;
    return true;
}

// one weighted-Jacobi sweep (zero: from a zero guess) on an N^3 tail grid in
// LDS; the right-hand side comes from registers (bv, top grid) or LDS (b);
// rd[w] = omega / D for a point next to w walls (D = diagonal of A_a)
template <typename T, int ORDER, int N, bool REG>
__device__ __forceinline__ void lds_jacobi(const T* src, T* dst, const T* b, const T* bv, T a,
                                           const T* rd, bool zero)
{
    constexpr int P = tail_p(N, ORDER);
    const T sc = lap_scale<ORDER, T>(N);
#pragma unroll
    for (int q = 0; q < tail_q<N>(); q++) {
        int i, j, k, p;
        if (!tail_pt<N>(q, i, j, k, p)) continue;
        const int pp = tpad<N, ORDER>(i, j, k);
        const T bp = REG ? bv[q] : b[p];
        const int walls =
            ORDER == 2 ? 0 : (i == 0) + (i == N - 1) + (j == 0) + (j == N - 1) + (k == 0) + (k == N - 1);
        const T r = rd[walls];
        if (zero) {
            dst[pp] = r * bp;
        } else {
            const T c = src[pp];
            const T Au = c - a * (sc * lap_pad<ORDER, T, P>(src, pp, c, walls));
            dst[pp] = c + r * (bp - Au);
        }
    }
}

template <typename T, int ORDER, int N, bool REG>
__device__ __forceinline__ void lds_resid(const T* u, const T* b, const T* bv, T* r, T a)
{
    constexpr int P = tail_p(N, ORDER);
    const T sc = lap_scale<ORDER, T>(N);
#pragma unroll
    for (int q = 0; q < tail_q<N>(); q++) {
        int i, j, k, p;
        if (!tail_pt<N>(q, i, j, k, p)) continue;
        const int pp = tpad<N, ORDER>(i, j, k);
        const int walls =
            ORDER == 2 ? 0 : (i == 0) + (i == N - 1) + (j == 0) + (j == N - 1) + (k == 0) + (k == N - 1);
        const T c = u[pp];
        r[pp] = (REG ? bv[q] : b[p]) - (c - a * (sc * lap_pad<ORDER, T, P>(u, pp, c, walls)));
    }
}

// full weighting of the N^3 residual r (padded) onto the coarse right-hand
// side cb (unpadded).  With NEXT the coarse grid's starting iterate is
// written too (padded, to nx): its first pre-smoothing sweep from the zero
// guess, omega D^{-1} cb with rdc[w] = omega / D next to w walls, the same
// product that sweep forms, or zero when the grid is not pre-smoothed
// (rdc null).  That saves the sweep a pass of its own.
template <typename T, int ORDER, int N, bool NEXT = false>
__device__ __forceinline__ void lds_restrict(const T* r, T* cb, T* nx = nullptr, const T* rdc = nullptr)
{
    constexpr int nc = (N - 1) / 2;
    constexpr int Nc = nc * nc * nc;
    constexpr int P = tail_p(N, ORDER);
    const T w[3] = {T(0.25), T(0.5), T(0.25)};
    for (int p = threadIdx.x; p < Nc; p += HS_TAIL_THREADS) {
        const int I = p % nc, J = (p / nc) % nc, K = p / (nc * nc);
        const T* c = r + tpad<N, ORDER>(2 * I + 1, 2 * J + 1, 2 * K + 1);
        T acc = T(0);
#pragma unroll
        for (int dz = -1; dz <= 1; dz++) {
            T az = T(0);
#pragma unroll
            for (int dy = -1; dy <= 1; dy++) {
                const T* row = c + dz * P * P + dy * P;
                T ay = (w[0] * row[-1] + w[1] * row[0]) + w[2] * row[1];
                az += w[dy + 1] * ay;
            }
            acc += w[dz + 1] * az;
        }
        cb[p] = acc;
        if constexpr (NEXT) {
            const int walls = ORDER == 2 ? 0
                                         : (I == 0) + (I == nc - 1) + (J == 0) + (J == nc - 1) + (K == 0) + (K == nc - 1);
            nx[tpad<nc, ORDER>(I, J, K)] = rdc ? rdc[walls] * acc : T(0);
        }
    }
}

// u += P c on an N^3 tail grid (both padded)
template <typename T, int ORDER, int N>
__device__ __forceinline__ void lds_prolong_add(T* u, const T* c)
{
#pragma unroll
    for (int q = 0; q < tail_q<N>(); q++) {
        int i, j, k, p;
        if (!tail_pt<N>(q, i, j, k, p)) continue;
        u[tpad<N, ORDER>(i, j, k)] += prolong_pad<T, ORDER, (N - 1) / 2>(c, i, j, k);
    }
}

// Exact solve on the coarsest grid (N = 1 or 3 points per axis) by the sine
// transform: x = S diag(1 / (1 - a (lam_i + lam_j + lam_k))) S b with the
// orthonormal, symmetric 1-D transform S and the 1-D eigenvalues lam (both
// staged in LDS); bh is LDS scratch of N^3 values.  b is unpadded, x padded.
template <typename T, int ORDER, int N, class PB>
__device__ __forceinline__ void lds_exact(PB b, T* x, T a, const double* S, const double* lam,
                                          double* bh)
{
    constexpr int NN = N * N * N;
    const int p = threadIdx.x;
    if (p < NN) {
        const int pi = p % N, pj = (p / N) % N, pk = p / (N * N);
        double si[N], sj[N], sk[N];
#pragma unroll
        for (int q = 0; q < N; q++) {
            si[q] = S[pi * 3 + q];
            sj[q] = S[pj * 3 + q];
            sk[q] = S[pk * 3 + q];
        }
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < N; k++)
#pragma unroll
            for (int j = 0; j < N; j++)
#pragma unroll
                for (int i = 0; i < N; i++)
                    s += sk[k] * sj[j] * si[i] * (double)b[(k * N + j) * N + i];
        const double mu = 1.0 - (double)a * (lam[pi] + lam[pj] + lam[pk]);
        bh[p] = s / mu;
    }
    __syncthreads();
    if (p < NN) {
        const int i = p % N, j = (p / N) % N, k = p / (N * N);
        double ci[N], cj[N], ck[N];
#pragma unroll
        for (int q = 0; q < N; q++) {
            ci[q] = S[q * 3 + i];
            cj[q] = S[q * 3 + j];
            ck[q] = S[q * 3 + k];
        }
        double s = 0.0;
#pragma unroll
        for (int pk = 0; pk < N; pk++)
#pragma unroll
            for (int pj = 0; pj < N; pj++)
#pragma unroll
                for (int pi = 0; pi < N; pi++)
                    s += ck[pk] * cj[pj] * ci[pi] * bh[(pk * N + pj) * N + pi];
        x[tpad<N, ORDER>(i, j, k)] = T(s);
    }
    __syncthreads();
}

// Shared state of one tail V-cycle.
template <typename T>
struct TailCtx {
    T* base;               // LDS grids
    const T* b0;           // right-hand side of the top grid, in registers (pass q -> b0[q])
    T a;
    const T (*rd)[8];      // omega / D per level and wall count
    int nu1, nu2;
    bool zero_top;         // the top grid starts from zero
    const double* S;       // exact-solve transform and eigenvalues
    const double* lam;
    double* bh;
    unsigned in_y;         // bit l: level l's iterate sits in Y(l)
    unsigned pre_done;     // bit l: level l's first pre-smoothing sweep was formed by the previous pass
};

// V(nu1, nu2) from level L down to the coarsest level LAST of a tail whose top
// grid has N0 points per axis; every grid size is a compile-time constant.
template <typename T, int ORDER, int N0, int L, int LAST>
struct TailV {
    static constexpr int n = tail_n(N0, L);
    static constexpr int nc = tail_n(N0, L + 1);
    __device__ static __forceinline__ void run(TailCtx<T>& c)
    {
        T* X = c.base + tail_off(N0, ORDER, L);
        T* Y = X + tail_pcube(n, ORDER);
        const T* B = L == 0 ? nullptr : Y + tail_pcube(n, ORDER);
        T* Xc = c.base + tail_off(N0, ORDER, L + 1);
        T* Yc = Xc + tail_pcube(nc, ORDER);
        T* Bc = Yc + tail_pcube(nc, ORDER);
        const bool zero = L > 0 || c.zero_top;
        for (int s = (int)((c.pre_done >> L) & 1u); s < c.nu1; s++) {
            const bool iy = (c.in_y >> L) & 1u;
            lds_jacobi<T, ORDER, n, L == 0>(iy ? Y : X, iy ? X : Y, B, c.b0, c.a, c.rd[L], zero && s == 0);
            c.in_y ^= 1u << L;
            __syncthreads();
        }
        {
            const bool iy = (c.in_y >> L) & 1u;
            T* r = iy ? X : Y;
            lds_resid<T, ORDER, n, L == 0>(iy ? Y : X, B, c.b0, r, c.a);
            __syncthreads();
            if constexpr (L + 1 < LAST) {
                // the coarse grid starts from zero: its first sweep (into Yc)
                // or its zero iterate (Xc) comes with its right-hand side
                const bool pre = c.nu1 > 0;
                lds_restrict<T, ORDER, n, true>(r, Bc, pre ? Yc : Xc, pre ? c.rd[L + 1] : nullptr);
                if (pre) {
                    c.in_y |= 1u << (L + 1);
                    c.pre_done |= 1u << (L + 1);
                }
            } else {
                lds_restrict<T, ORDER, n>(r, Bc);
            }
            __syncthreads();
        }
        TailV<T, ORDER, N0, L + 1, LAST>::run(c);
        {
            const bool iy = (c.in_y >> L) & 1u;
            lds_prolong_add<T, ORDER, n>(iy ? Y : X, ((c.in_y >> (L + 1)) & 1u) ? Yc : Xc);
            __syncthreads();
        }
        for (int s = 0; s < c.nu2; s++) {
            const bool iy = (c.in_y >> L) & 1u;
            lds_jacobi<T, ORDER, n, L == 0>(iy ? Y : X, iy ? X : Y, B, c.b0, c.a, c.rd[L], false);
            c.in_y ^= 1u << L;
            __syncthreads();
        }
    }
};

template <typename T, int ORDER, int N0, int LAST>
struct TailV<T, ORDER, N0, LAST, LAST> {
    static constexpr int n = tail_n(N0, LAST);
    __device__ static __forceinline__ void run(TailCtx<T>& c)
    {
        T* X = c.base + tail_off(N0, ORDER, LAST);
        lds_exact<T, ORDER, n>(X + 2 * tail_pcube(n, ORDER), X, c.a, c.S, c.lam, c.bh);
        c.in_y &= ~(1u << LAST);
    }
};

// One V-cycle over the NLEV tail grids of one lane, top grid N0^3: level 0
// starts from the iterate in global memory (or from zero when the top is a
// correction grid), the lower levels from zero; the result is written back
// to level 0's iterate.  A single-grid tail is just the exact solve.  The
// top grid's loads are issued first, so their latency overlaps the lane's
// state check and the set-up of the smoother weights.
template <typename T>
struct TailShared {
    T rd[HS_MAXTAIL][8];
    double S[9], lam[3], bh[27];
};

template <typename T, int ORDER, int N0, int NLEV>
__device__ __forceinline__ void tail_run(const TailSeg& ts, const LaneCtl* __restrict__ ctl,
                                         const hsk::MgArgs& A, int nu1, int nu2, T* base,
                                         TailShared<T>& sh)
{
    constexpr int N0c = tail_cube(N0);
    T (*s_rd)[8] = sh.rd;
    double* s_S = sh.S;
    double* s_lam = sh.lam;
    double* s_bh = sh.bh;
    const int t = (int)threadIdx.x;
    HS_G T* gu0 = (HS_G T*)ts.u[0] + (long long)A.node * ts.node_stride;
    const HS_G T* gb0 = (const HS_G T*)ts.b[0];
    const bool zero_top = ts.zero_guess != 0;
    T b0[tail_q<N0>()];
    T u0[tail_q<N0>()];
    if constexpr (NLEV > 1) {
#pragma unroll
        for (int q = 0; q < tail_q<N0>(); q++) {
            int i, j, k, p;
            const bool ok = tail_pt<N0>(q, i, j, k, p);
            b0[q] = ok ? gb0[p] : T(0);
            u0[q] = (ok && !zero_top) ? gu0[p] : T(0);
        }
    }
    if (A.gate && ctl[ts.lane].mg_state != 0) return;
    const T a = T(lane_a(ctl, ts.lane, A.L, A.m));
    if (t < NLEV * 7) {
        const int l = t / 7, w = t % 7;
        const int nl = tail_n(N0, l);
        const T ih2 = T((double)(nl + 1) * (double)(nl + 1));
        const T D = ORDER == 2 ? T(1) + a * ih2 * T(6) : T(1) + a * ih2 * (T(90 - w) / T(12));
        s_rd[l][w] = T(A.omega) / D;
    } else if (t >= 64 && t < 64 + 12) {
        const CoarseTable& ct = c_lc.ct[ts.coarse_table];
        if (t < 64 + 9) s_S[t - 64] = ct.S[(t - 64) / 3][(t - 64) % 3];
        else s_lam[t - 73] = ct.lam[t - 73];
    }
    TailCtx<T> c;
    c.base = base;
    c.b0 = b0;
    c.a = a;
    c.rd = s_rd;
    c.nu1 = nu1;
    c.nu2 = nu2;
    c.zero_top = zero_top;
    c.S = s_S;
    c.lam = s_lam;
    c.bh = s_bh;
    c.in_y = 0;
    c.pre_done = 0;
    // zero every grid, so the cells beyond the walls read 0 (16-byte stores)
    {
        constexpr int bytes = tail_off(N0, ORDER, NLEV) * (int)sizeof(T);
        uint4* b16 = reinterpret_cast<uint4*>(base);
        for (int w = t; w < bytes / 16; w += HS_TAIL_THREADS) b16[w] = make_uint4(0u, 0u, 0u, 0u);
        if constexpr (bytes % 16 != 0) {
            if (t < (bytes % 16) / (int)sizeof(T)) base[(bytes / 16) * (16 / (int)sizeof(T)) + t] = T(0);
        }
    }
    __syncthreads();
    // the top grid's result (padded) back to its global iterate
    auto store_top = [&](const T* res) {
        for (int p = t; p < N0c; p += HS_TAIL_THREADS) {
            const int i = p % N0, j = (p / N0) % N0, k = p / (N0 * N0);
            gu0[p] = res[tpad<N0, ORDER>(i, j, k)];
        }
    };
    if constexpr (NLEV == 1) {
        lds_exact<T, ORDER, N0>(gb0, c.base, c.a, c.S, c.lam, c.bh);
        store_top(c.base);
    } else {
        // the top grid's starting iterate: u0, or from a zero start its first
        // pre-smoothing sweep omega D^{-1} b (into Y, the product that sweep
        // forms) or zero when it is not pre-smoothed
        T* X0 = base;
        T* Y0 = base + tail_pcube(N0, ORDER);
        const bool pre = zero_top && nu1 > 0;
#pragma unroll
        for (int q = 0; q < tail_q<N0>(); q++) {
            int i, j, k, p;
            if (!tail_pt<N0>(q, i, j, k, p)) continue;
            const int pp = tpad<N0, ORDER>(i, j, k);
            if (!zero_top) {
                X0[pp] = u0[q];
            } else if (pre) {
                const int walls =
                    ORDER == 2 ? 0 : (i == 0) + (i == N0 - 1) + (j == 0) + (j == N0 - 1) + (k == 0) + (k == N0 - 1);
                Y0[pp] = s_rd[0][walls] * b0[q];
            } else {
                X0[pp] = T(0);
            }
        }
        if (pre) {
            c.in_y |= 1u;
            c.pre_done |= 1u;
        }
        __syncthreads();
        TailV<T, ORDER, N0, 0, NLEV - 1>::run(c);
        store_top((c.in_y & 1u) ? c.base + tail_pcube(N0, ORDER) : c.base);
    }
}

template <typename T, int ORDER>
__global__ void __launch_bounds__(HS_TAIL_THREADS) k_tail(const TailSeg* __restrict__ segs,
                                                          const LaneCtl* __restrict__ ctl,
                                                          hsk::MgArgs A, int nu1, int nu2)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ TailShared<T> sh;
    T* base = (T*)smem;
    const TailSeg& ts = segs[blockIdx.x];
    // the plan only builds tails of these shapes (top 2^k - 1 <= 15 down to 3 or 1)
    switch (ts.n[0] * 8 + ts.nlev) {
    case 15 * 8 + 3: tail_run<T, ORDER, 15, 3>(ts, ctl, A, nu1, nu2, base, sh); break;
    case 15 * 8 + 4: tail_run<T, ORDER, 15, 4>(ts, ctl, A, nu1, nu2, base, sh); break;
    case 7 * 8 + 2: tail_run<T, ORDER, 7, 2>(ts, ctl, A, nu1, nu2, base, sh); break;
    case 7 * 8 + 3: tail_run<T, ORDER, 7, 3>(ts, ctl, A, nu1, nu2, base, sh); break;
    case 3 * 8 + 1: tail_run<T, ORDER, 3, 1>(ts, ctl, A, nu1, nu2, base, sh); break;
    case 3 * 8 + 2: tail_run<T, ORDER, 3, 2>(ts, ctl, A, nu1, nu2, base, sh); break;
    case 1 * 8 + 1: tail_run<T, ORDER, 1, 1>(ts, ctl, A, nu1, nu2, base, sh); break;
    default: break;
    }
}

// ---------------------------------------------------------------------------
// Solve control
// ---------------------------------------------------------------------------


// Stopping test before cycle `cycle`, one block per lane:
// rho = |b - A u|_inf / |b|_inf (|b| = 0 -> 1); stop when rho <= tol, fail
// when cycle == max_cycles or rho is not finite.
__global__ void __launch_bounds__(HS_BLOCK) k_mg_decide(const GridSeg* __restrict__ segs, int nseg,
                                                        int nblk, const double* __restrict__ partials,
                                                        LaneCtl* __restrict__ ctl, int cycle,
                                                        double tol, int max_cycles, int level)
{
    int si = blockIdx.x;
    const GridSeg sg = segs[si];
    LaneCtl& c = ctl[sg.lane];
    if (c.mg_state != 0) return;
    int b0 = sg.blk_begin, nb = seg_nblk(segs, nseg, si, nblk);
    double r = 0.0, bb = 0.0;
    for (int q = threadIdx.x; q < nb; q += blockDim.x) {
        r = nmax(r, partials[2 * (b0 + q)]);
        if (cycle == 0) bb = nmax(bb, partials[2 * (b0 + q) + 1]);
    }
    r = block_max(r);
    if (cycle == 0) bb = block_max(bb);
    if (threadIdx.x == 0) {
        if (cycle == 0) c.bnorm = bb;
        double scale = c.bnorm > 0.0 ? c.bnorm : 1.0;
        double rho = r / scale;
        c.mg_rho = rho;
        if (rho != rho || r > 1.7e308) {
            finish_solve(c, cycle, 2, level);
            c.status = -4;
        } else if (rho <= tol) {
            finish_solve(c, cycle, 1, level);
        } else if (cycle >= max_cycles) {
            finish_solve(c, cycle, 2, level);
            if (c.status == 0) c.status = -3;
        }
    }
}

// max-norm residual of the FP64 iterate of the finest grid, per block
template <int ORDER>
__global__ void __launch_bounds__(HS_BLOCK) k_mg_norm(const GridSeg* __restrict__ segs, int nseg,
                                                      int nblk, const LaneCtl* __restrict__ ctl,
                                                      hsk::MgArgs A, int cycle,
                                                      double* __restrict__ partials, int src_is_t)
{
    int lb = xcd_remap(blockIdx.x, nblk);
    int si = find_seg(segs, nseg, lb);
    const GridSeg sg = segs[si];
    if (ctl[sg.lane].mg_state != 0) return;
    const int n = sg.n;
    PosZ q = grid_pos_z(lb - sg.blk_begin, n, sg.zb);
    const HS_G double* u = (sg.moves && (src_is_t & 1))
                               ? (const HS_G double*)sg.t
                               : (const HS_G double*)sg.u + (long long)A.node * sg.node_stride;
    struct Op {
        const HS_G double* b;
        double a;
        int cycle;
        double rmax, bmax;
        __device__ __forceinline__ void operator()(long long p, int, double c, double L)
        {
            double bp = b[p];
            rmax = nmax(rmax, fabs(bp - (c - a * L)));
            if (cycle == 0) bmax = nmax(bmax, fabs(bp));
        }
    } op{(const HS_G double*)sg.b, lane_a(ctl, sg.lane, A.L, A.m), cycle, 0.0, 0.0};
    __shared__ double pl[2][Halo<ORDER>::LH][Halo<ORDER>::LW];
    lds_march<ORDER, double>(u, n, q.i - (int)(threadIdx.x % HS_TX), q.j - (int)(threadIdx.x / HS_TX), q.z0,
                             q.z1, pl, op);
    double m = op.rmax, mb = op.bmax;
    block_max2(m, mb);
    if (threadIdx.x == 0) {
        partials[2 * lb] = m;
        partials[2 * lb + 1] = mb;
    }
}

// Mixed-precision refinement on the finest grid: r = b - A u in FP64,
// r32 = (float) r into the FP32 right-hand side, per-block maxima of |r|
// (and |b| at iteration 0).
template <int ORDER>
__global__ void __launch_bounds__(HS_BLOCK) k_ir_resid(const GridSeg* __restrict__ s64,
                                                       const GridSeg* __restrict__ s32, int nseg,
                                                       int nblk, const LaneCtl* __restrict__ ctl,
                                                       hsk::MgArgs A, int iter,
                                                       double* __restrict__ partials)
{
    int lb = xcd_remap(blockIdx.x, nblk);
    int si = find_seg(s64, nseg, lb);
    const GridSeg sg = s64[si];
    if (ctl[sg.lane].mg_state != 0) return;
    const int n = sg.n;
    PosZ q = grid_pos_z(lb - sg.blk_begin, n, sg.zb);
    const HS_G double* u = (const HS_G double*)sg.u + (long long)A.node * sg.node_stride;
    struct Op {
        const HS_G double* b;
        HS_G float* r32;
        double a;
        int iter;
        double rmax, bmax;
        __device__ __forceinline__ void operator()(long long p, int, double c, double L)
        {
            double bp = b[p];
            double r = bp - (c - a * L);
            r32[p] = (float)r;
            rmax = nmax(rmax, fabs(r));
            if (iter == 0) bmax = nmax(bmax, fabs(bp));
        }
    } op{(const HS_G double*)sg.b, (HS_G float*)s32[si].b, lane_a(ctl, sg.lane, A.L, A.m), iter, 0.0, 0.0};
    __shared__ double pl[2][Halo<ORDER>::LH][Halo<ORDER>::LW];
    lds_march<ORDER, double>(u, n, q.i - (int)(threadIdx.x % HS_TX), q.j - (int)(threadIdx.x / HS_TX), q.z0,
                             q.z1, pl, op);
    double m = op.rmax, mb = op.bmax;
    block_max2(m, mb);
    if (threadIdx.x == 0) {
        partials[2 * lb] = m;
        partials[2 * lb + 1] = mb;
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
    PosZ q = grid_pos_z(lb - sg.blk_begin, n, sg.zb);
    if (!q.in) return;
    HS_G double* u = (HS_G double*)sg.u + (long long)A.node * sg.node_stride;
    const HS_G float* e = (const HS_G float*)s32[si].u;
    for (int z = q.z0; z < q.z1; z++) {
        long long p = lin(q.i, q.j, z, n);
        u[p] += (double)e[p];
    }
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
// With with_resid it also writes per-block maxima of the collocation residual
//   R = max_m |U_0 + dt sum_j Q_mj (FI_j + g_j s) + tau_m - U_m|
// for the SDC stopping test (k_sdc_decide).
__global__ void __launch_bounds__(HS_BLOCK) k_sweep_prep(const SdcSeg* __restrict__ segs, int nseg,
                                                         int nblk, const LaneCtl* __restrict__ ctl,
                                                         int with_resid, int gate,
                                                         double* __restrict__ partials)
{
    int lb = xcd_remap(blockIdx.x, nblk);
    int si = find_seg(segs, nseg, lb);
    const SdcSeg sg = segs[si];
    const LaneCtl& c = ctl[sg.lane];
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
    double m = block_max(R);
    if (threadIdx.x == 0) partials[2 * lb] = m;
}

// Collocation residual alone (per-block maxima), for a check after a sweep
__global__ void __launch_bounds__(HS_BLOCK) k_sdc_resid(const SdcSeg* __restrict__ segs, int nseg,
                                                        int nblk, const LaneCtl* __restrict__ ctl,
                                                        double* __restrict__ partials)
{
    int lb = xcd_remap(blockIdx.x, nblk);
    int si = find_seg(segs, nseg, lb);
    const SdcSeg sg = segs[si];
    const LaneCtl& c = ctl[sg.lane];
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
    double m = block_max(R);
    if (threadIdx.x == 0) partials[2 * lb] = m;
}

// SDC stopping test, one block per lane: R from the lane's block maxima.
__global__ void __launch_bounds__(HS_BLOCK) k_sdc_decide(const SdcSeg* __restrict__ segs, int nseg,
                                                         int nblk, const double* __restrict__ partials,
                                                         LaneCtl* __restrict__ ctl, double sdc_tol,
                                                         int max_sweeps)
{
    int si = blockIdx.x;
    const SdcSeg sg = segs[si];
    LaneCtl& c = ctl[sg.lane];
    if (c.sdc_state != 0) return;
    int b0 = sg.blk_begin, nb = seg_nblk(segs, nseg, si, nblk);
    double r = 0.0;
    for (int q = threadIdx.x; q < nb; q += blockDim.x) r = nmax(r, partials[2 * (b0 + q)]);
    r = block_max(r);
    if (threadIdx.x == 0) {
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

// FI_m = nu L U_m at nodes m0..m1-1, and at node rhs_node also rhs = U + P
// (the right-hand side of the next substep, which starts from that node).
// The blocks follow a z-marching table of the same lanes' finest grids
// (gsegs); the node arrays come from the SDC table (ssegs, same order).
template <int ORDER>
__global__ void __launch_bounds__(HS_BLOCK) k_fi_march(const GridSeg* __restrict__ gsegs,
                                                       const SdcSeg* __restrict__ ssegs, int nseg, int nblk,
                                                       const LaneCtl* __restrict__ ctl, int m0, int m1,
                                                       int rhs_node, int gate)
{
    int lb = xcd_remap(blockIdx.x, nblk);
    int si = find_seg(gsegs, nseg, lb);
    const GridSeg sg = gsegs[si];
    const SdcSeg ss = ssegs[si];
    if (gate && ctl[sg.lane].sdc_state != 0) return;
    if (gate == 2 && ctl[sg.lane].mg_state == 0) return;   // issued ahead of the host's check: stopped solves only
    const int n = sg.n;
    PosZ q = grid_pos_z(lb - sg.blk_begin, n, sg.zb);
    const long long N = (long long)n * n * n;
    struct Op {
        HS_G double* fi;
        HS_G double* rhs;
        const HS_G double* P;
        double nu;
        __device__ __forceinline__ void operator()(long long p, int, double c, double L)
        {
            fi[p] = nu * L;
            if (rhs) rhs[p] = c + P[p];
        }
    };
    __shared__ double pl[2][Halo<ORDER>::LH][Halo<ORDER>::LW];
    const int i0 = q.i - (int)(threadIdx.x % HS_TX), j0 = q.j - (int)(threadIdx.x / HS_TX);
    for (int m = m0; m < m1; m++) {
        Op op{(HS_G double*)ss.FI + m * N, m == rhs_node ? (HS_G double*)ss.rhs : nullptr,
              (const HS_G double*)ss.P + m * N, ctl[sg.lane].nu};
        lds_march<ORDER, double>((const HS_G double*)ss.U + m * N, n, i0, j0, q.z0, q.z1, pl, op);
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

// FAS restriction from SDC level lf to lf + 1, one thread per coarse point:
//   Ut_m = Uc_m = inj(Uf_{m'}),  FIc_m = nu Lc Ut_m,
//   tau_m = inj(dt sum_j Qf_{m'j} Ff_j + tauf_{m'}) - dt sum_j Qc_{mj} Fc_j
// where m' is the fine node of coarse node m, F = FI + g s, and tauf is the
// fine level's own FAS correction when it is not the finest level (the
// coarse problem is the fine level's FAS-corrected collocation problem).
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
        Fc[m] = fi + c.g[sg.lf + 1][m] * sc_;
    }
    double Ff[HS_MAXM];
    for (int j = 0; j < sg.Mf; j++) Ff[j] = sg.FIf[j * Nf + pf] + c.g[sg.lf][j] * sf_;
    for (int m = 0; m < sg.Mc; m++) {
        int mf = m * stride;
        double fa = 0.0, ca = 0.0;
        for (int j = 0; j < sg.Mf; j++) fa += KF.Q[mf][j] * Ff[j];
        for (int j = 0; j < sg.Mc; j++) ca += KC.Q[m][j] * Fc[j];
        double fint = dt * fa;
        if (sg.tauf) fint += sg.tauf[mf * Nf + pf];
        sg.tau[m * Nc + pc] = fint - dt * ca;
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

// Tricubic transfer of the coarse correction (fas_interp = 3), as k_fas_interp
// but with 4-point Lagrange interpolation per axis: a fine index that
// coincides with a coarse one takes its value, a midpoint the weights
// (-1, 9, 9, -1)/16 on the two coarse points on either side; a tap on a wall
// is 0 and a tap one cell beyond a wall the odd reflection of the point one
// cell inside.  Separable, in three passes: along x into Ex, along y into
// Exy, then per fine point along z and the Lagrange combination in time of
// k_fas_interp.
struct Cubic1 {
    int idx[4];
    double w[4];
    int cnt;
};

__device__ __forceinline__ Cubic1 cubic1(int i)
{
    Cubic1 c;
    if (i & 1) {
        c.idx[0] = (i - 1) >> 1;
        c.w[0] = 1.0;
        c.cnt = 1;
    } else {
        const int m = i >> 1;
        c.idx[0] = m - 2; c.w[0] = -1.0 / 16.0;
        c.idx[1] = m - 1; c.w[1] = 9.0 / 16.0;
        c.idx[2] = m;     c.w[2] = 9.0 / 16.0;
        c.idx[3] = m + 1; c.w[3] = -1.0 / 16.0;
        c.cnt = 4;
    }
    return c;
}

// coarse index of a tap and its sign (0: the tap is on a wall)
__device__ __forceinline__ int cubic_fold(int I, int nc, double& sign)
{
    if (I == -1 || I == nc) {
        sign = 0.0;
        return 0;
    }
    if (I == -2) {
        sign = -sign;
        return 0;
    }
    if (I == nc + 1) {
        sign = -sign;
        return nc - 1;
    }
    return I;
}

// Ex[j][K][J][fi] = x interpolation of dU_j = Uc_j - Ut_j on coarse row (J, K)
// (blocks of the fine table whose row and plane indices are below nc; the
// rest return)
__global__ void __launch_bounds__(HS_BLOCK) k_fas_interp3_x(const FasSeg* __restrict__ segs, int nseg,
                                                            int nblk, const LaneCtl* __restrict__ ctl,
                                                            int gate)
{
    int lb = xcd_remap(blockIdx.x, nblk);
    int si = find_seg(segs, nseg, lb);
    const FasSeg sg = segs[si];
    if (gate && ctl[sg.lane].sdc_state != 0) return;
    const int nf = sg.nf, nc = sg.nc;
    Pos q = grid_pos(lb - sg.blk_begin, nf);
    if (!q.in || q.j >= nc || q.k >= nc) return;
    const long long Nc = (long long)nc * nc * nc, Nx = (long long)nc * nc * nf;
    const Cubic1 cx = cubic1(q.i);
    for (int jn = 0; jn < sg.Mc; jn++) {
        const double* uc = sg.Uc + jn * Nc;
        const double* ut = sg.Ut + jn * Nc;
        double sx = 0.0;
        for (int a = 0; a < cx.cnt; a++) {
            double sgn = 1.0;
            const int I = cubic_fold(cx.idx[a], nc, sgn);
            if (sgn == 0.0) continue;
            const long long pc = lin(I, q.j, q.k, nc);
            sx += cx.w[a] * (sgn * (uc[pc] - ut[pc]));
        }
        sg.Ex[jn * Nx + ((long long)q.k * nc + q.j) * nf + q.i] = sx;
    }
}

// Exy[j][K][fj][fi] = y interpolation of Ex on coarse plane K (blocks of the
// fine table whose plane index is below nc; the rest return)
__global__ void __launch_bounds__(HS_BLOCK) k_fas_interp3_y(const FasSeg* __restrict__ segs, int nseg,
                                                            int nblk, const LaneCtl* __restrict__ ctl,
                                                            int gate)
{
    int lb = xcd_remap(blockIdx.x, nblk);
    int si = find_seg(segs, nseg, lb);
    const FasSeg sg = segs[si];
    if (gate && ctl[sg.lane].sdc_state != 0) return;
    const int nf = sg.nf, nc = sg.nc;
    Pos q = grid_pos(lb - sg.blk_begin, nf);
    if (!q.in || q.k >= nc) return;
    const long long Nx = (long long)nc * nc * nf, Nxy = (long long)nc * nf * nf;
    const Cubic1 cy = cubic1(q.j);
    for (int jn = 0; jn < sg.Mc; jn++) {
        const double* X = sg.Ex + jn * Nx + (long long)q.k * nc * nf;
        double sy = 0.0;
        for (int b = 0; b < cy.cnt; b++) {
            double sgn = 1.0;
            const int J = cubic_fold(cy.idx[b], nc, sgn);
            if (sgn == 0.0) continue;
            sy += cy.w[b] * (sgn * X[(long long)J * nf + q.i]);
        }
        sg.Exy[jn * Nxy + ((long long)q.k * nf + q.j) * nf + q.i] = sy;
    }
}

// z interpolation of Exy at every fine point, then U_f += the Lagrange
// combination in time (as k_fas_interp)
__global__ void __launch_bounds__(HS_BLOCK) k_fas_interp3_z(const FasSeg* __restrict__ segs, int nseg,
                                                            int nblk, const LaneCtl* __restrict__ ctl,
                                                            int gate)
{
    int lb = xcd_remap(blockIdx.x, nblk);
    int si = find_seg(segs, nseg, lb);
    const FasSeg sg = segs[si];
    if (gate && ctl[sg.lane].sdc_state != 0) return;
    const int nf = sg.nf, nc = sg.nc;
    Pos q = grid_pos(lb - sg.blk_begin, nf);
    if (!q.in) return;
    const long long Nf = (long long)nf * nf * nf, Nxy = (long long)nc * nf * nf;
    const long long pf = lin(q.i, q.j, q.k, nf);
    const long long pxy = (long long)q.j * nf + q.i;
    const Cubic1 cz = cubic1(q.k);
    double e[HS_MAXM];
    for (int jn = 0; jn < sg.Mc; jn++) {
        const double* E = sg.Exy + jn * Nxy;
        double s = 0.0;
        for (int c = 0; c < cz.cnt; c++) {
            double sgn = 1.0;
            const int K = cubic_fold(cz.idx[c], nc, sgn);
            if (sgn == 0.0) continue;
            s += cz.w[c] * (sgn * E[(long long)K * nf * nf + pxy]);
        }
        e[jn] = s;
    }
    const InterpConst& ip = c_lc.ip[sg.Mf][sg.Mc];
    for (int mf = 0; mf < sg.Mf; mf++) {
        double corr = 0.0;
        if (mf % ip.stride == 0) {
            corr = e[mf / ip.stride];
        } else {
            for (int jn = 0; jn < sg.Mc; jn++) corr += ip.w[mf][jn] * e[jn];
        }
        sg.Uf[mf * Nf + pf] += corr;
    }
}

// ---------------------------------------------------------------------------
// Lane bookkeeping
// ---------------------------------------------------------------------------

// Step coefficients: t_n = t0 + step dt; a[L][m] = nu dt (tau_{m+1} - tau_m);
// g[L][j] = -(sin t_j - c nu pi^2 cos t_j) at t_j = t_n + dt tau_j (eq. (3)).
__global__ void k_begin_step(LaneCtl* ctl, int nlanes, int nlevels, int M0, int M1, int M2)
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
        const SdcConst& K = c_lc.sdc[L == 0 ? M0 : L == 1 ? M1 : M2];
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

__global__ void k_begin_solve(LaneCtl* ctl, int first, int nlanes)
{
    int lane = first + blockIdx.x * blockDim.x + threadIdx.x;
    if (lane >= first + nlanes) return;
    LaneCtl& c = ctl[lane];
    // a node-parallel solver lane solves while its SDC lane iterates
    const int sdc = c.parent >= 0 ? ctl[c.parent].sdc_state : c.sdc_state;
    c.mg_state = sdc != 0 ? 3 : 0;
    c.mg_cycle = 0;
}

__global__ void k_np_lanes(LaneCtl* ctl, int nlanes, int M, int mode)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nlanes * (M - 1)) return;
    const int b = s / (M - 1), m = s % (M - 1) + 1;
    LaneCtl& c = ctl[nlanes + s];
    if (mode == 0) {
        c.parent = b;
        c.active = 1;
        c.sdc_state = 0;
        c.mg_state = 3;
        c.status = 0;
        c.bnorm = c.mg_rho = c.sdc_res = 0.0;
        c.total_cycles = 0; c.total_solves = 0; c.max_cycles = 0; c.total_sweeps = 0;
        c.sweeps_step = 0; c.failed_solves = 0;
        for (int l = 0; l < HS_MAXLEV; l++) c.level_cycles[l] = 0;
        c.a_user = 0.0;
    } else {
        const LaneCtl& p = ctl[b];
        c.a_user = p.nu * (p.dt * c_lc.sdc[M].tau[m]);
    }
}

// Right-hand sides of the node-parallel sweep (all from iterate k):
//   rhs_m = U_0 + dt sum_j Q_mj (FI_j + g_j s) - dt tau_m FI_m,  m = 1..M-1,
// written to P + (m-1) N, where solver lane (b, m) takes its right-hand side.
__global__ void __launch_bounds__(HS_BLOCK) k_np_rhs(const SdcSeg* __restrict__ segs, int nseg, int nblk,
                                                     const LaneCtl* __restrict__ ctl)
{
    int lb = xcd_remap(blockIdx.x, nblk);
    int si = find_seg(segs, nseg, lb);
    const SdcSeg sg = segs[si];
    const LaneCtl& c = ctl[sg.lane];
    if (c.sdc_state != 0) return;
    int n = sg.n, M = sg.M;
    Pos q = grid_pos(lb - sg.blk_begin, n);
    if (!q.in) return;
    const SdcConst& K = c_lc.sdc[M];
    long long N = (long long)n * n * n;
    long long p = lin(q.i, q.j, q.k, n);
    double s = sval(sg.sig, q.i, q.j, q.k);
    double dt = c.dt;
    double F[HS_MAXM];
    for (int j = 0; j < M; j++) F[j] = sg.FI[j * N + p] + c.g[sg.level][j] * s;
    const double u0 = sg.U[p];
    for (int m = 1; m < M; m++) {
        double acc = 0.0;
        for (int j = 0; j < M; j++) acc += K.Q[m][j] * F[j];
        sg.P[(m - 1) * N + p] = (u0 + dt * acc) - (dt * K.tau[m]) * sg.FI[m * N + p];
    }
}

__global__ void k_end_solve_fixed(LaneCtl* ctl, int first, int nlanes, int cycles, int level)
{
    int lane = first + blockIdx.x * blockDim.x + threadIdx.x;
    if (lane >= first + nlanes) return;
    LaneCtl& c = ctl[lane];
    if (c.mg_state == 0) finish_solve(c, cycles, 1, level);
}

__global__ void k_begin_sweep(LaneCtl* ctl, int first, int nlanes)
{
    int lane = first + blockIdx.x * blockDim.x + threadIdx.x;
    if (lane >= first + nlanes) return;
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
    for (int l = 0; l < HS_MAXLEV; l++) c.level_cycles[l] = 0;
    c.parent = -1;
}

__global__ void k_set_a_user(LaneCtl* ctl, int lane, double a)
{
    ctl[lane].a_user = a;
    ctl[lane].mg_state = 0;
    ctl[lane].sdc_state = 0;
}

__global__ void k_fill(double* __restrict__ dst, long long count, double v)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long stride = (long long)gridDim.x * blockDim.x;
    for (; i < count; i += stride) dst[i] = v;
}

// PFASST residual test: lanes that met the tolerance keep iterating while
// another slice has not (state 1 -> 0); failed lanes stay failed.
__global__ void k_sdc_reopen(LaneCtl* ctl, int nlanes)
{
    int lane = blockIdx.x * blockDim.x + threadIdx.x;
    if (lane >= nlanes) return;
    if (ctl[lane].sdc_state == 1) ctl[lane].sdc_state = 0;
}

__global__ void k_copy(const double* __restrict__ src, double* __restrict__ dst, long long count)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long stride = (long long)gridDim.x * blockDim.x;
    for (; i < count; i += stride) dst[i] = src[i];
}

// y = alpha u + beta L u on user arrays (lane-major packing, offset pack_off)
template <int ORDER>
__global__ void __launch_bounds__(HS_BLOCK) k_lap_apply(const GridSeg* __restrict__ segs, int nseg,
                                                        int nblk, double alpha, double beta,
                                                        const double* __restrict__ u,
                                                        double* __restrict__ y,
                                                        const long long* __restrict__ offs)
{
    // y = alpha u + beta L_h u on the caller's lane-major arrays, as a plane
    // march over the z-chunks of the lanes' grid table (the same march as the
    // sweeps)
    const int lb = xcd_remap(blockIdx.x, nblk);
    const int si = find_seg(segs, nseg, lb);
    const GridSeg sg = segs[si];
    const int n = sg.n;
    const PosZ q = grid_pos_z(lb - sg.blk_begin, n, sg.zb);
    struct Op {
        HS_G double* y;
        double al, be;
        __device__ __forceinline__ void operator()(long long p, int, double c, double L) { y[p] = al * c + be * L; }
    } op{(HS_G double*)y + offs[si], alpha, beta};
    __shared__ double pl[2][Halo<ORDER>::LH][Halo<ORDER>::LW];
    lds_march<ORDER, double>((const HS_G double*)u + offs[si], n, q.i - (int)(threadIdx.x % HS_TX),
                             q.j - (int)(threadIdx.x / HS_TX), q.z0, q.z1, pl, op);
}

// f_impl = nu L u, f_expl = f(x, t) (eq. (3)) on user arrays; gsegs gives the
// march's blocks, ssegs (same lanes, same order) the sine tables
template <int ORDER>
__global__ void __launch_bounds__(HS_BLOCK) k_heat_rhs(const GridSeg* __restrict__ gsegs,
                                                       const SdcSeg* __restrict__ ssegs, int nseg,
                                                       int nblk, const LaneCtl* __restrict__ ctl,
                                                       const double* __restrict__ u,
                                                       const double* __restrict__ t,
                                                       double* __restrict__ fi,
                                                       double* __restrict__ fe,
                                                       const long long* __restrict__ offs)
{
    const int lb = xcd_remap(blockIdx.x, nblk);
    const int si = find_seg(gsegs, nseg, lb);
    const GridSeg sg = gsegs[si];
    const double* sig = ssegs[si].sig;
    const int n = sg.n;
    const PosZ q = grid_pos_z(lb - sg.blk_begin, n, sg.zb);
    const LaneCtl& c = ctl[sg.lane];
    const double pi2 = 3.14159265358979323846 * 3.14159265358979323846;
    const double g = -(sin(t[si]) - c.forcing_c * c.nu * pi2 * cos(t[si]));
    if (fi) {
        struct Op {
            HS_G double* fi;
            double nu;
            __device__ __forceinline__ void operator()(long long p, int, double, double L) { fi[p] = nu * L; }
        } op{(HS_G double*)fi + offs[si], c.nu};
        __shared__ double pl[2][Halo<ORDER>::LH][Halo<ORDER>::LW];
        lds_march<ORDER, double>((const HS_G double*)u + offs[si], n, q.i - (int)(threadIdx.x % HS_TX),
                                 q.j - (int)(threadIdx.x / HS_TX), q.z0, q.z1, pl, op);
    }
    if (fe && q.in)
        for (int z = q.z0; z < q.z1; z++) fe[offs[si] + lin(q.i, q.j, z, n)] = sval(sig, q.i, q.j, z) * g;
}

// ---------------------------------------------------------------------------
// Compact fourth-order pair (the fine level's compact stencil of section 1
// and its weighting matrix, section 1.2; the Mehrstellen reading):
//   A_h u = (2 (6 face neighbours) + (12 edge neighbours) - 24 u) / (6 h^2),
//   B_h u = u / 2 + (6 face neighbours) / 12,
// zero beyond the walls.  The 19-point stencil reaches the in-plane
// neighbours of planes z - 1 and z + 1, so the march keeps three planes of
// the 64 x 8 tile with a one-point halo (corners included) in a ring of four
// LDS planes and loads plane z + 2 into the fourth while plane z is formed:
// one barrier per plane.
// ---------------------------------------------------------------------------
// trilinear prolongation of ec (zero walls) at fine point (i, j, k)
__device__ __forceinline__ double cmp_prolong_at(const double* ec, int nc, int i, int j, int k)
{
    int ix[2], iy[2], iz[2];
    double wx[2], wy[2], wz[2];
    int cx, cy, cz;
    auto wts = [](int f, int* idx, double* wt, int* cnt) {
        if (f & 1) { idx[0] = (f - 1) >> 1; wt[0] = 1.0; *cnt = 1; }
        else { idx[0] = (f >> 1) - 1; wt[0] = 0.5; idx[1] = f >> 1; wt[1] = 0.5; *cnt = 2; }
    };
    wts(i, ix, wx, &cx);
    wts(j, iy, wy, &cy);
    wts(k, iz, wz, &cz);
    double s = 0.0;
    for (int c = 0; c < cz; c++)
        for (int b = 0; b < cy; b++)
            for (int a = 0; a < cx; a++) {
                const int I = ix[a], J = iy[b], K = iz[c];
                if (I < 0 || I >= nc || J < 0 || J >= nc || K < 0 || K >= nc) continue;
                s += wx[a] * wy[b] * wz[c] * ec[((long long)K * nc + J) * nc + I];
            }
    return s;
}

struct CmpTile {
    static constexpr int LW = HS_TX + 2, LH = HS_TY + 2;
    static constexpr int NH = LW * LH - HS_TX * HS_TY;   // halo cells per plane (148)
};

// op(p, c, A, B) at every grid point of planes z0..z1-1 of the column tile
// at (i0, j0); all threads of the block must call it
template <class Op>
__device__ __forceinline__ void cmp_march(const HS_G double* __restrict__ u, int n, int i0, int j0, int z0,
                                          int z1, double (*ring)[CmpTile::LH][CmpTile::LW], Op& op)
{
    using C = CmpTile;
    const int t = (int)threadIdx.x;
    const int lx = t % HS_TX, ly = t / HS_TX;
    const int i = i0 + lx, j = j0 + ly;
    const bool in = i < n && j < n;
    // this thread's halo cell, if any: row 0, row LH-1, then the side columns
    int hr = -1, hc = 0;
    if (t < C::NH) {
        if (t < C::LW) { hr = 0; hc = t; }
        else if (t < 2 * C::LW) { hr = C::LH - 1; hc = t - C::LW; }
        else { const int q = t - 2 * C::LW; hr = 1 + q / 2; hc = (q & 1) ? C::LW - 1 : 0; }
    }
    const int hi = i0 + hc - 1, hj = j0 + hr - 1;
    const bool hin = hr >= 0 && hi >= 0 && hi < n && hj >= 0 && hj < n;
    const long long nn = (long long)n * n;
    const long long pij = in ? (long long)j * n + i : 0, hoff = hin ? (long long)hj * n + hi : 0;
    auto ld = [&](bool ok, long long off, int z) -> double {
        return (ok && z >= 0 && z < n) ? u[(long long)z * nn + off] : 0.0;
    };
    auto slot = [](int z) { return (z + 4) & 3; };
    // planes z0-1, z0, z0+1
    for (int d = -1; d <= 1; d++) {
        const int z = z0 + d;
        const double cv = ld(in, pij, z), hv = ld(hin, hoff, z);
        ring[slot(z)][ly + 1][lx + 1] = cv;
        if (hr >= 0) ring[slot(z)][hr][hc] = hv;
    }
    __syncthreads();
    const double ih2 = (double)(n + 1) * (double)(n + 1);
    for (int z = z0; z < z1; z++) {
        const bool more = z + 1 < z1;
        const double cn = more ? ld(in, pij, z + 2) : 0.0, hn = more ? ld(hin, hoff, z + 2) : 0.0;
        if (in) {
            const double (*m)[C::LW] = ring[slot(z - 1)];
            const double (*o)[C::LW] = ring[slot(z)];
            const double (*q)[C::LW] = ring[slot(z + 1)];
            const int x = lx + 1, y = ly + 1;
            const double c = o[y][x];
            const double faces = ((o[y][x - 1] + o[y][x + 1]) + (o[y - 1][x] + o[y + 1][x])) + (m[y][x] + q[y][x]);
            const double exy = (o[y - 1][x - 1] + o[y - 1][x + 1]) + (o[y + 1][x - 1] + o[y + 1][x + 1]);
            const double exz = (m[y][x - 1] + m[y][x + 1]) + (q[y][x - 1] + q[y][x + 1]);
            const double eyz = (m[y - 1][x] + m[y + 1][x]) + (q[y - 1][x] + q[y + 1][x]);
            const double A = ((2.0 * faces + ((exy + exz) + eyz)) - 24.0 * c) * ih2 / 6.0;
            const double B = 0.5 * c + faces / 12.0;
            op((long long)z * nn + pij, c, A, B);
        }
        if (more) {
            ring[slot(z + 2)][ly + 1][lx + 1] = cn;
            if (hr >= 0) ring[slot(z + 2)][hr][hc] = hn;
        }
        __syncthreads();
    }
}

// y = alpha B_h u + beta A_h u on `batch` packed n^3 grids; block b covers
// column tile b % tiles of z chunk (b / tiles) % nz of grid b / (tiles nz)
__global__ void __launch_bounds__(HS_BLOCK) k_compact_apply(int n, int zb, int nz, double alpha, double beta,
                                                            const double* __restrict__ u, double* __restrict__ y)
{
    const int tx = tiles_x(n), tiles = tx * tiles_y(n);
    const int b = (int)blockIdx.x;
    const int tile = b % tiles, zc = (b / tiles) % nz, g = b / (tiles * nz);
    const long long N = (long long)n * n * n;
    const int i0 = (tile % tx) * HS_TX, j0 = (tile / tx) * HS_TY;
    const int z0 = zc * zb, z1 = min(z0 + zb, n);
    struct Op {
        HS_G double* y;
        double al, be;
        __device__ __forceinline__ void operator()(long long p, double, double A, double B) { y[p] = al * B + be * A; }
    } op{(HS_G double*)y + g * N, alpha, beta};
    __shared__ double ring[4][CmpTile::LH][CmpTile::LW];
    cmp_march((const HS_G double*)u + g * N, n, i0, j0, z0, z1, ring, op);
}

// Multigrid and SDC with the compact pair, one lane per launch.  MODE:
//   0  weighted Jacobi  dst = c + omega / D (b - (B - a A) c),  D = 1/2 + 4 a / h^2
//   1  residual         dst = b - (B - a A) c
//   2  substep rhs      dst = (B c - dt_m g2) + b   (b: dt S_m F, g2: nu A U_{m+1})
//   3  implicit part    dst = nu A c
//   4  norms            per-block maxima of |b - (B - a A) c| and |b| into partials
//   5  Jacobi as 0 with the norms of 4 (of the iterate before the sweep)
// with dt_m = dt dtau (dtau = tau_{m+1} - tau_m of the substep, 0 for B alone)
// and a = nu dt_m, dt and nu of the lane.  With gate set the launch does
// nothing once the lane's solve has stopped (mg_state != 0).
template <int MODE>
__global__ void __launch_bounds__(HS_BLOCK) k_cmp(int n, int zb, const double* __restrict__ src,
                                                  double* __restrict__ dst, const double* __restrict__ b,
                                                  const double* __restrict__ g2, const LaneCtl* __restrict__ ctl,
                                                  int lane, double dtau, double omega, double* __restrict__ partials,
                                                  int gate)
{
    const LaneCtl& c = ctl[lane];
    if (gate && c.mg_state != 0) return;
    const int tx = tiles_x(n), tiles = tx * tiles_y(n);
    const int tile = (int)blockIdx.x % tiles, zc = (int)blockIdx.x / tiles;
    const int i0 = (tile % tx) * HS_TX, j0 = (tile / tx) * HS_TY;
    const int z0 = zc * zb, z1 = min(z0 + zb, n);
    const double dtm = c.dt * dtau, a = c.nu * dtm;
    const double ih2 = (double)(n + 1) * (double)(n + 1);
    const double D = 0.5 + a * 24.0 * ih2 / 6.0;
    struct Op {
        HS_G double* dst;
        const HS_G double* b;
        const HS_G double* g2;
        double a, D, omega, nu, dtm;
        double rmax, bmax;
        __device__ __forceinline__ void operator()(long long p, double cv, double A, double B)
        {
            if (MODE == 0) dst[p] = cv + omega * (b[p] - (B - a * A)) / D;
            else if (MODE == 5) {
                const double bp = b[p], r = bp - (B - a * A);
                dst[p] = cv + omega * r / D;
                rmax = nmax(rmax, fabs(r));
                bmax = nmax(bmax, fabs(bp));
            }
            else if (MODE == 1) dst[p] = b[p] - (B - a * A);
            else if (MODE == 2) dst[p] = (B - dtm * g2[p]) + b[p];
            else if (MODE == 3) dst[p] = nu * A;
            else {
                const double bp = b[p];
                rmax = nmax(rmax, fabs(bp - (B - a * A)));
                bmax = nmax(bmax, fabs(bp));
            }
        }
    } op{(HS_G double*)dst, (const HS_G double*)b, (const HS_G double*)g2, a, D, omega, c.nu, dtm, 0.0, 0.0};
    __shared__ double ring[4][CmpTile::LH][CmpTile::LW];
    cmp_march((const HS_G double*)src, n, i0, j0, z0, z1, ring, op);
    if (MODE == 4 || MODE == 5) {
        double r = op.rmax, bb = op.bmax;
        block_max2(r, bb);
        if (threadIdx.x == 0) {
            partials[2 * blockIdx.x] = r;
            partials[2 * blockIdx.x + 1] = bb;
        }
    }
}

// full weighting of the fine residual at coarse point (I, J, K) (weights
// (1/4, 1/2, 1/4) per axis; every tap is inside the fine grid)
__device__ __forceinline__ double cmp_fw_at(const double* rf, int nf, int I, int J, int K)
{
    const double w[3] = {0.25, 0.5, 0.25};
    double s = 0.0;
    for (int dz = -1; dz <= 1; dz++)
        for (int dy = -1; dy <= 1; dy++)
            for (int dx = -1; dx <= 1; dx++) {
                const int i = 2 * I + 1 + dx, j = 2 * J + 1 + dy, k = 2 * K + 1 + dz;
                s += w[dx + 1] * w[dy + 1] * w[dz + 1] * rf[((long long)k * nf + j) * nf + i];
            }
    return s;
}

// exact solve of (B - a A) x = b for n <= 3 in the sine basis,
// x = S diag(1 / (lam_B - a lam_A)) S b with S the orthonormal DST-I; called
// by every thread of the block (t = threadIdx.x), bh a 27-entry scratch;
// x has a zero frame of one cell ((n+2)^3 layout), b none.
__device__ void cmp_exact_dev(int n, const double* b, double* x, double a, double* bh, double (*S)[3], double* cs)
{
    const int t = (int)threadIdx.x, N3 = n * n * n;
    const double pi = 3.14159265358979323846;
    if (t < n * n) S[t / n][t % n] = sqrt(2.0 / (n + 1)) * sin(pi * (t % n + 1) * (t / n + 1) / (n + 1));
    if (t < n) cs[t] = cos(pi * (t + 1) / (n + 1));
    __syncthreads();
    const double ih2 = (double)(n + 1) * (double)(n + 1);
    if (t < N3) {
        const int p = t % n, q = (t / n) % n, r = t / (n * n);
        double s = 0.0;
        for (int k = 0; k < n; k++)
            for (int j = 0; j < n; j++)
                for (int i = 0; i < n; i++) s += S[r][k] * S[q][j] * S[p][i] * b[(k * n + j) * n + i];
        const double sc = cs[p] + cs[q] + cs[r], pc = cs[p] * cs[q] + cs[p] * cs[r] + cs[q] * cs[r];
        const double la = (4.0 * sc + 4.0 * pc - 24.0) * ih2 / 6.0, lb = 0.5 + sc / 6.0;
        bh[t] = s / (lb - a * la);
    }
    __syncthreads();
    if (t < N3) {
        const int i = t % n, j = (t / n) % n, k = t / (n * n);
        double s = 0.0;
        for (int r = 0; r < n; r++)
            for (int q = 0; q < n; q++)
                for (int p = 0; p < n; p++) s += S[r][k] * S[q][j] * S[p][i] * bh[(r * n + q) * n + p];
        x[((k + 1) * (n + 2) + (j + 1)) * (n + 2) + (i + 1)] = s;
    }
    __syncthreads();
}

// grid: x over the points of one coarse plane, y the plane (32-bit index math)
__global__ void __launch_bounds__(HS_BLOCK) k_cmp_fw(int nf, const double* __restrict__ rf, double* __restrict__ bc,
                                                     const LaneCtl* __restrict__ ctl, int lane, int gate)
{
    if (gate && ctl[lane].mg_state != 0) return;
    const int nc = (nf - 1) / 2;
    const int q = (int)(blockIdx.x * HS_BLOCK + threadIdx.x), K = (int)blockIdx.y;
    if (q >= nc * nc) return;
    const int J = q / nc, I = q - J * nc;
    bc[((long long)K * nc + J) * nc + I] = cmp_fw_at(rf, nf, I, J, K);
}

// dst = src + trilinear prolongation of ec, one thread per fine point (dst
// may be src: the correction added in place); grid: x over the points of
// one fine plane, y the plane
__global__ void __launch_bounds__(HS_BLOCK) k_cmp_prolong(int nc, const double* __restrict__ ec, const double* src,
                                                          double* dst, const LaneCtl* __restrict__ ctl, int lane,
                                                          int gate)
{
    if (gate && ctl[lane].mg_state != 0) return;
    const int nf = 2 * nc + 1;
    const int q = (int)(blockIdx.x * HS_BLOCK + threadIdx.x), k = (int)blockIdx.y;
    if (q >= nf * nf) return;
    const int j = q / nf, i = q - j * nf;
    const long long p = ((long long)k * nf + j) * nf + i;
    dst[p] = src[p] + cmp_prolong_at(ec, nc, i, j, k);
}

// the first Jacobi sweep from a zero iterate: dst = omega b / D (the residual
// of a zero iterate is b), one thread per point
__global__ void __launch_bounds__(HS_BLOCK) k_cmp_zsweep(int n, const double* __restrict__ b, double* __restrict__ dst,
                                                         const LaneCtl* __restrict__ ctl, int lane, double dtau,
                                                         double omega, int gate)
{
    const LaneCtl& c = ctl[lane];
    if (gate && c.mg_state != 0) return;
    const long long q = (long long)blockIdx.x * HS_BLOCK + threadIdx.x;
    if (q >= (long long)n * n * n) return;
    const double a = c.nu * (c.dt * dtau), ih2 = (double)(n + 1) * (double)(n + 1);
    dst[q] = omega * b[q] / (0.5 + a * 24.0 * ih2 / 6.0);
}

// The grids of one compact V-cycle from n <= HS_TAIL_N down, in one
// workgroup with every field in LDS, the same operations in the same order
// as the per-grid launches.  Iterates carry a zero frame of one cell
// ((n+2)^3 values, the walls), so the 19-point stencil and the prolongation
// read their neighbours without bounds tests; right-hand sides are n^3.
// Threads: x = tid % 16, y = tid / 16 % 16, z = tid / 256 + 4 r.  The top
// grid's iterate comes from u (or starts at zero) and goes back to u; b is
// its right-hand side.  Dynamic LDS: compact_tail_lds bytes.
__global__ void __launch_bounds__(HS_TAIL_THREADS) k_cmp_tail(int n0, double* __restrict__ ug,
                                                              const double* __restrict__ bg, int zero_guess,
                                                              const LaneCtl* __restrict__ ctl, int lane, double dtau,
                                                              double omega, int nu1, int nu2, int n_coarsest, int gate)
{
    if (gate && ctl[lane].mg_state != 0) return;
    extern __shared__ double lds[];
    __shared__ double bh[27];
    __shared__ double Sm[3][3], cs[3];
    const int tid = (int)threadIdx.x;
    const int tx = tid & 15, ty = (tid >> 4) & 15, tz = tid >> 8;
    const double a = ctl[lane].nu * (ctl[lane].dt * dtau);
    // grids n_l = n0 >> l (n0 = 2^k - 1) down to the first with n <= n_coarsest
    // or n = 1; no arrays indexed at run time (they would live in scratch)
    int L = 0;
    while ((n0 >> L) > n_coarsest && (n0 >> L) > 1 && L + 1 < HS_MAXTAIL) L++;
    // level l's fields: X (padded iterate), Y (its ping-pong partner), R (rhs)
    auto base = [&](int l) -> double* {
        int o = 0;
        for (int j = 0; j < l; j++) {
            const int n = n0 >> j, P = n + 2;
            o += 2 * P * P * P + n * n * n;
        }
        return lds + o;
    };
    auto fieldX = [&](int l) -> double* { return base(l); };
    auto fieldY = [&](int l) -> double* { const int P = (n0 >> l) + 2; return base(l) + P * P * P; };
    auto fieldR = [&](int l) -> double* { const int P = (n0 >> l) + 2; return base(l) + 2 * P * P * P; };
    {
        double* end = fieldR(L) + (n0 >> L) * (n0 >> L) * (n0 >> L);
        const int total = (int)(end - lds);
        for (int p = tid; p < total; p += HS_TAIL_THREADS) lds[p] = 0.0;
    }
    __syncthreads();
    {
        const int n = n0, P = n + 2;
        double *X0 = fieldX(0), *R0 = fieldR(0);
        if (tx < n && ty < n)
            for (int z = tz; z < n; z += 4) {
                const int g = (z * n + ty) * n + tx;
                if (!zero_guess) X0[((z + 1) * P + ty + 1) * P + tx + 1] = ug[g];
                R0[g] = bg[g];
            }
    }
    __syncthreads();
    // the 19-point pair at padded cell c of x (the same sums as cmp_march)
    auto pairAB = [](const double* x, int c, int P, double ih2, double* A, double* B) {
        const int PP = P * P;
        const double cv = x[c];
        const double faces = ((x[c - 1] + x[c + 1]) + (x[c - P] + x[c + P])) + (x[c - PP] + x[c + PP]);
        const double exy = (x[c - P - 1] + x[c - P + 1]) + (x[c + P - 1] + x[c + P + 1]);
        const double exz = (x[c - PP - 1] + x[c - PP + 1]) + (x[c + PP - 1] + x[c + PP + 1]);
        const double eyz = (x[c - PP - P] + x[c - PP + P]) + (x[c + PP - P] + x[c + PP + P]);
        *A = ((2.0 * faces + ((exy + exz) + eyz)) - 24.0 * cv) * ih2 / 6.0;
        *B = 0.5 * cv + faces / 12.0;
    };
    // one Jacobi sweep x -> y on level l (x null: from zero)
    auto sweep = [&](int l, const double* x, double* y) {
        const int n = n0 >> l, P = n + 2;
        const double ih2 = (double)(n + 1) * (double)(n + 1);
        const double D = 0.5 + a * 24.0 * ih2 / 6.0;
        const double* R = fieldR(l);
        if (tx < n && ty < n)
            for (int z = tz; z < n; z += 4) {
                const int c = ((z + 1) * P + ty + 1) * P + tx + 1;
                const double bv = R[(z * n + ty) * n + tx];
                if (!x) {
                    y[c] = omega * bv / D;
                } else {
                    double A, B;
                    pairAB(x, c, P, ih2, &A, &B);
                    y[c] = x[c] + omega * (bv - (B - a * A)) / D;
                }
            }
        __syncthreads();
    };
    unsigned inY = 0;   // bit l: level l's iterate is in Y (else X)
    for (int l = 0; l < L; l++) {
        const int n = n0 >> l, P = n + 2, nc = n0 >> (l + 1);
        const double ih2 = (double)(n + 1) * (double)(n + 1);
        double *x = fieldX(l), *y = fieldY(l);
        const double* R = fieldR(l);
        const bool zg = l > 0 || zero_guess;
        for (int q = 0; q < nu1; q++) {
            sweep(l, (q == 0 && zg) ? nullptr : x, y);
            double* w = x; x = y; y = w;
        }
        if (nu1 & 1) inY |= 1u << l;
        // residual into y (interior), then full weighting into the next level's rhs
        if (tx < n && ty < n)
            for (int z = tz; z < n; z += 4) {
                const int c = ((z + 1) * P + ty + 1) * P + tx + 1;
                double A, B;
                pairAB(x, c, P, ih2, &A, &B);
                y[c] = R[(z * n + ty) * n + tx] - (B - a * A);
            }
        __syncthreads();
        double* Rc = fieldR(l + 1);
        if (tx < nc && ty < nc)
            for (int z = tz; z < nc; z += 4) {
                const double w[3] = {0.25, 0.5, 0.25};
                double sacc = 0.0;
                for (int dz = -1; dz <= 1; dz++)
                    for (int dy = -1; dy <= 1; dy++)
                        for (int dx = -1; dx <= 1; dx++)
                            sacc += w[dx + 1] * w[dy + 1] * w[dz + 1] *
                                    y[((2 * z + 2 + dz) * P + (2 * ty + 2 + dy)) * P + (2 * tx + 2 + dx)];
                Rc[(z * nc + ty) * nc + tx] = sacc;
            }
        __syncthreads();
    }
    cmp_exact_dev(n0 >> L, fieldR(L), fieldX(L), a, bh, Sm, cs);
    for (int l = L - 1; l >= 0; l--) {
        const int n = n0 >> l, P = n + 2, Pc = (n0 >> (l + 1)) + 2;
        const double* ec = ((inY >> (l + 1)) & 1u) ? fieldY(l + 1) : fieldX(l + 1);
        double* src = ((inY >> l) & 1u) ? fieldY(l) : fieldX(l);
        // the corrected iterate goes where the post-sweeps end in X
        double* dst = (nu2 & 1) ? fieldY(l) : fieldX(l);
        if (tx < n && ty < n)
            for (int z = tz; z < n; z += 4) {
                const int i = tx, j = ty, k = z;
                // per axis: odd i on coarse (i-1)/2; even i between i/2-1 and i/2
                // (padded coarse index +1; the frame supplies the zero walls)
                const int cx = (i & 1) ? 1 : 2, cy = (j & 1) ? 1 : 2, cz = (k & 1) ? 1 : 2;
                const int ix0 = (i & 1) ? (i - 1) / 2 + 1 : i / 2, iy0 = (j & 1) ? (j - 1) / 2 + 1 : j / 2;
                const int iz0 = (k & 1) ? (k - 1) / 2 + 1 : k / 2;
                const double wx = (i & 1) ? 1.0 : 0.5, wy = (j & 1) ? 1.0 : 0.5, wz = (k & 1) ? 1.0 : 0.5;
                double sacc = 0.0;
                for (int c3 = 0; c3 < cz; c3++)
                    for (int b3 = 0; b3 < cy; b3++)
                        for (int a3 = 0; a3 < cx; a3++)
                            sacc += wx * wy * wz * ec[((iz0 + c3) * Pc + iy0 + b3) * Pc + ix0 + a3];
                const int c = ((k + 1) * P + j + 1) * P + i + 1;
                dst[c] = src[c] + sacc;
            }
        __syncthreads();
        double *x = dst, *y = (nu2 & 1) ? fieldX(l) : fieldY(l);
        for (int q = 0; q < nu2; q++) {
            sweep(l, x, y);
            double* w = x; x = y; y = w;
        }
        inY &= ~(1u << l);   // X again
    }
    {
        const int n = n0, P = n + 2;
        const double* x = fieldX(0);
        if (tx < n && ty < n)
            for (int z = tz; z < n; z += 4) ug[(z * n + ty) * n + tx] = x[((z + 1) * P + ty + 1) * P + tx + 1];
    }
}

// Quadratures of the compact sweep over F_j = G_j + lam_B g_j s(x), the
// B-weighted right-hand side at node j (G_j = nu A U_j; for the forcing's
// sine mode B f = lam_B f, lam_B = 1/2 + cos(pi h) / 2).  One thread per point.
//   m < 0:  dst[mm N + p] = dt sum_j S_mm,j F_j for mm = 0..M-2 (iterate k)
//   m >= 0: dst[p] = base[p] + dt sum_j Q_m,j F_j (B U_0 plus the integral to tau_m)
__global__ void __launch_bounds__(HS_BLOCK) k_cmp_quad(int n, int M, int m, const double* __restrict__ G,
                                                       const double* __restrict__ base, double* __restrict__ dst,
                                                       const double* __restrict__ sig,
                                                       const LaneCtl* __restrict__ ctl, int lane, int L)
{
    const long long N = (long long)n * n * n;
    const long long p = (long long)blockIdx.x * HS_BLOCK + threadIdx.x;
    if (p >= N) return;
    const int i = (int)(p % n), j = (int)((p / n) % n), k = (int)(p / ((long long)n * n));
    const LaneCtl& c = ctl[lane];
    const SdcConst& K = c_lc.sdc[M];
    const double lamb = 0.5 + 0.5 * cos(3.14159265358979323846 / (n + 1));
    const double s = sval(sig, i, j, k);
    double F[HS_MAXM];
    for (int q = 0; q < M; q++) F[q] = G[q * N + p] + lamb * (c.g[L][q] * s);
    if (m < 0) {
        for (int mm = 0; mm + 1 < M; mm++) {
            double acc = 0.0;
            for (int q = 0; q < M; q++) acc += K.S[mm][q] * F[q];
            dst[mm * N + p] = c.dt * acc;
        }
    } else {
        double acc = 0.0;
        for (int q = 0; q < M; q++) acc += K.Q[m][q] * F[q];
        dst[p] = base[p] + c.dt * acc;
    }
}

// Maxima of the norm partials of one launch (pairs |r|, |b| per block).
//   mode 0: mg_rho = max|r| / max|b| (max|b| = 0 counts as 1), bnorm = max|b|
//   mode 1: sdc_res = max|r|;  mode 2: sdc_res = max(sdc_res, max|r|)
//   mode 3: the stopping test of a solve before its cycle `cycle`, as mode 0
//           and then: stop (state 1) when rho <= tol, fail (state 2) when
//           rho is not finite (status st_nonfinite) or cycle >= max_cycles
//           (status st_noconv); skipped once the solve has stopped
__global__ void __launch_bounds__(HS_BLOCK) k_cmp_reduce(const double* __restrict__ partials, int nblk,
                                                         LaneCtl* __restrict__ ctl, int lane, int mode, int cycle,
                                                         double tol, int max_cycles, int st_noconv, int st_nonfinite)
{
    if (mode == 3 && ctl[lane].mg_state != 0) return;
    double r = 0.0, bb = 0.0;
    for (int q = (int)threadIdx.x; q < nblk; q += HS_BLOCK) {
        r = nmax(r, partials[2 * q]);
        bb = nmax(bb, partials[2 * q + 1]);
    }
    block_max2(r, bb);
    if (threadIdx.x != 0) return;
    LaneCtl& c = ctl[lane];
    if (mode == 1 || mode == 2) {
        c.sdc_res = mode == 1 ? r : nmax(c.sdc_res, r);
        return;
    }
    c.bnorm = bb;
    const double rho = r / (bb > 0.0 ? bb : 1.0);
    c.mg_rho = rho;
    if (mode != 3) return;
    c.mg_cycle = cycle;
    if (rho != rho) {
        finish_solve(c, cycle, 2, 0);
        if (c.status == 0) c.status = st_nonfinite;
    } else if (rho <= tol) {
        finish_solve(c, cycle, 1, 0);
    } else if (cycle >= max_cycles) {
        finish_solve(c, cycle, 2, 0);
        if (c.status == 0) c.status = st_noconv;
    }
}

// B_h^{-1} in the sine basis (the FAS correction of MLSDC with the compact
// fine level): B_h = S diag(lambda) S with S the orthonormal DST-I along each
// axis.  One axis of the transform, one thread per output value:
//   out[(a n + i) C + c] = sum_q S_iq in[(a n + q) C + c]
// with C the axis stride (1, n, n^2); tab holds S transposed (tab[q n + i] =
// S_iq, so that the threads of a row read consecutive entries) followed by
// cos(pi (i+1) h), i < n.
__global__ void __launch_bounds__(HS_BLOCK) k_dst_axis(int n, int C, const double* __restrict__ tab,
                                                       const double* __restrict__ in, double* __restrict__ out)
{
    const int idx = (int)(blockIdx.x * HS_BLOCK + threadIdx.x);
    if (idx >= n * n * n) return;
    const int c = idx % C, r = idx / C, i = r % n, a = r / n;
    const double* src = in + (long long)a * n * C + c;
    double sum = 0.0;
    for (int q = 0; q < n; q++) sum += tab[q * n + i] * src[(long long)q * C];
    out[idx] = sum;
}

// x /= 1/2 + (cos(pi (i+1) h) + cos(pi (j+1) h) + cos(pi (k+1) h)) / 6, B_h's
// eigenvalue on sine mode (i, j, k)
__global__ void __launch_bounds__(HS_BLOCK) k_binv_scale(int n, const double* __restrict__ tab, double* __restrict__ x)
{
    const int idx = (int)(blockIdx.x * HS_BLOCK + threadIdx.x);
    if (idx >= n * n * n) return;
    const double* cs = tab + n * n;
    const int i = idx % n, j = (idx / n) % n, k = idx / (n * n);
    x[idx] /= 0.5 + ((cs[i] + cs[j]) + cs[k]) / 6.0;
}

// Lane bookkeeping of the compact path: op 0 ends a solve (finish_solve with
// cycles / state), op 1 sets the SDC state; a negative status is kept if the
// lane has none yet.
__global__ void k_cmp_ctl(LaneCtl* ctl, int lane, int op, int cycles, int state, int level, int status)
{
    if (threadIdx.x != 0) return;
    LaneCtl& c = ctl[lane];
    if (op == 0) finish_solve(c, cycles, state, level);
    else c.sdc_state = state;
    if (status < 0 && c.status == 0) c.status = status;
}

}  // namespace

// ---------------------------------------------------------------------------
// Launch helpers
// ---------------------------------------------------------------------------
namespace hsk {

static inline dim3 g1(int nblk) { return dim3((unsigned)nblk); }
static const dim3 BLK(HS_BLOCK);

int grid_blocks(int n, int zb) { return tiles_x(n) * tiles_y(n) * ((n + zb - 1) / zb); }

// z planes per block of the plane-marching kernels: as many as possible (up
// to 8, fewer halo reloads and window warm-ups) while one grid still gives
// 256 blocks of 512 threads (one per CU).  Measured: at 127^3 eight planes
// per block (512 blocks) beat four (1024 blocks) and sixteen (256 blocks);
// at 63^3 two planes (256 blocks) beat one (504 blocks).
int choose_zb(int n)
{
    long long tiles = (long long)tiles_x(n) * tiles_y(n);
    int zb = 8;
    while (zb > 1 && tiles * ((n + zb - 1) / zb) < 256) zb /= 2;
    return zb;
}

// z planes per block of the two-sweep kernel: twice the sweeps' (the first
// sweep is formed on R extra planes at each end of the block's chunk)
int choose_zb_two(int n)
{
    const int zb = 2 * choose_zb(n);
    return zb < 16 ? zb : 16;
}

// z planes per block of the fused residual and restriction: even (a coarse
// plane's centre and both its fine neighbours below lie in one chunk)
int choose_zb_even(int n)
{
    int zb = choose_zb(n);
    return zb < 2 ? 2 : zb;
}

size_t tail_lds_bytes(int n0, int elem, int order)
{
    size_t words = 0;
    int n = n0;
    bool top = true;
    while (true) {
        words += (size_t)tail_words(n, order, top);
        top = false;
        if (n <= 1) break;
        n = (n - 1) / 2;
    }
    return words * (size_t)elem;
}

hipError_t set_constants(const LibConst& lc)
{
    return hipMemcpyToSymbol(HIP_SYMBOL(c_lc), &lc, sizeof(LibConst), 0, hipMemcpyHostToDevice);
}

#define HS_ORDER_DISPATCH(order, KERNEL2, KERNEL4, GRID, BLOCK, SHMEM, ...)                 \
    do {                                                                                    \
        if ((order) == 2) hipLaunchKernelGGL(KERNEL2, GRID, BLOCK, SHMEM, s, __VA_ARGS__);  \
        else hipLaunchKernelGGL(KERNEL4, GRID, BLOCK, SHMEM, s, __VA_ARGS__);               \
    } while (0)

// As HS_ORDER_DISPATCH; with events in ev the launch records the kernel's
// own start and end in them (for the launch timer).
#define HS_ORDER_DISPATCH_EV(ev, order, KERNEL2, KERNEL4, GRID, BLOCK, SHMEM, ...)                          \
    do {                                                                                                    \
        if (!(ev).start) HS_ORDER_DISPATCH(order, KERNEL2, KERNEL4, GRID, BLOCK, SHMEM, __VA_ARGS__);       \
        else if ((order) == 2)                                                                              \
            hipExtLaunchKernelGGL(KERNEL2, GRID, BLOCK, SHMEM, s, (ev).start, (ev).stop, 0, __VA_ARGS__);   \
        else hipExtLaunchKernelGGL(KERNEL4, GRID, BLOCK, SHMEM, s, (ev).start, (ev).stop, 0, __VA_ARGS__);  \
    } while (0)

template <typename T, int MODE, int FINEST, int NORM, int SRC = 0>
static hipError_t sweep_launch(LaneCtl* ctl, const GridSeg* segs, int nseg, int nblk, int order,
                               MgArgs a, int first_sweep, int src_is_t, int cycle, double* partials,
                               hipStream_t s, double tol = 0.0, int max_cycles = 0, EvPair ev = {})
{
    HS_ORDER_DISPATCH_EV(ev, order, (k_sweep<T, 2, MODE, FINEST, NORM, SRC>), (k_sweep<T, 4, MODE, FINEST, NORM, SRC>),
                         g1(nblk), BLK, 0, segs, nseg, nblk, ctl, a, first_sweep, src_is_t, partials,
                         cycle, tol, max_cycles);
    return hipGetLastError();
}

template <typename T>
hipError_t sweep(LaneCtl* ctl, const GridSeg* segs, int nseg, int nblk, int order, MgArgs a,
                 int mode, int first_sweep, int src_is_t, int finest_only, int norm, int cycle,
                 double* partials, hipStream_t s, int src, double tol, int max_cycles, EvPair ev)
{
    if (nblk <= 0) return hipSuccess;
    if (mode == 1)
        return sweep_launch<T, 1, 1, 0>(ctl, segs, nseg, nblk, order, a, 0, src_is_t, 0, partials, s, 0.0, 0, ev);
    if (src == 1)
        return sweep_launch<T, 0, 0, 0, 1>(ctl, segs, nseg, nblk, order, a, 0, src_is_t, 0, partials, s, 0.0, 0, ev);
    if (norm == 1)
        return sweep_launch<T, 0, 1, 1>(ctl, segs, nseg, nblk, order, a, 0, src_is_t, cycle, partials, s, 0.0, 0, ev);
    if (norm == 2)
        return sweep_launch<T, 0, 1, 2>(ctl, segs, nseg, nblk, order, a, 0, src_is_t, cycle, partials, s, tol,
                                        max_cycles, ev);
    if (finest_only)
        return sweep_launch<T, 0, 1, 0>(ctl, segs, nseg, nblk, order, a, 0, src_is_t, 0, partials, s, 0.0, 0, ev);
    return sweep_launch<T, 0, 0, 0>(ctl, segs, nseg, nblk, order, a, first_sweep, src_is_t, 0, partials, s, 0.0, 0,
                                    ev);
}

template <typename T>
hipError_t jac2(LaneCtl* ctl, const GridSeg* segs, int nseg, int nblk, int order, MgArgs a, int src_is_t,
                int norm, int cycle, double* partials, hipStream_t s)
{
    if (nblk <= 0) return hipSuccess;
    if (norm)
        HS_ORDER_DISPATCH(order, (k_jac2<T, 2, 1>), (k_jac2<T, 4, 1>), g1(nblk), BLK, 0, segs, nseg, nblk, ctl,
                          a, src_is_t, partials, cycle);
    else
        HS_ORDER_DISPATCH(order, (k_jac2<T, 2, 0>), (k_jac2<T, 4, 0>), g1(nblk), BLK, 0, segs, nseg, nblk, ctl,
                          a, src_is_t, partials, cycle);
    return hipGetLastError();
}

template <typename T>
hipError_t resid_fw(LaneCtl* ctl, const GridSeg* segs, int nseg, int nblk, int order, MgArgs a,
                    int src_is_t, hipStream_t s, EvPair ev)
{
    if (nblk <= 0) return hipSuccess;
    HS_ORDER_DISPATCH_EV(ev, order, (k_resid_fw<T, 2>), (k_resid_fw<T, 4>), g1(nblk), BLK, 0, segs, nseg, nblk, ctl,
                         a, src_is_t);
    return hipGetLastError();
}

template <typename T>
hipError_t pjac(LaneCtl* ctl, const GridSeg* segs, int nseg, int nblk, int order, MgArgs a, int src_is_t,
                hipStream_t s, EvPair ev)
{
    if (nblk <= 0) return hipSuccess;
    HS_ORDER_DISPATCH_EV(ev, order, (k_pjac<T, 2>), (k_pjac<T, 4>), g1(nblk), BLK, 0, segs, nseg, nblk, ctl, a,
                         src_is_t);
    return hipGetLastError();
}

hipError_t mg_fixup(LaneCtl* ctl, const GridSeg* segs, int nseg, int nblk, MgArgs a, hipStream_t s)
{
    if (nblk <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mg_fixup, g1(nblk), BLK, 0, s, segs, nseg, nblk, ctl, a);
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
                size_t lds_bytes, hipStream_t s)
{
    if (nseg <= 0) return hipSuccess;
    // padded 4th-order tails of a 15^3 top grid need more than 64 KB of LDS;
    // the limit is raised once per device and kernel instance
    if (lds_bytes > 65536) {
        static std::mutex mu;
        static std::map<std::pair<int, int>, size_t> allowed;
        int dev = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) return e;
        std::lock_guard<std::mutex> lock(mu);
        size_t& al = allowed[{dev, order}];
        if (lds_bytes > al) {
            e = order == 4 ? hipFuncSetAttribute((const void*)k_tail<T, 4>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 (int)lds_bytes)
                           : hipFuncSetAttribute((const void*)k_tail<T, 2>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 (int)lds_bytes);
            if (e != hipSuccess) return e;
            al = lds_bytes;
        }
    }
    HS_ORDER_DISPATCH(order, (k_tail<T, 2>), (k_tail<T, 4>), dim3((unsigned)nseg),
                      dim3(HS_TAIL_THREADS), (unsigned)lds_bytes, segs, ctl, a, nu1, nu2);
    return hipGetLastError();
}

template hipError_t sweep<double>(LaneCtl*, const GridSeg*, int, int, int, MgArgs, int, int, int, int, int, int, double*, hipStream_t, int, double, int, EvPair);
template hipError_t sweep<float>(LaneCtl*, const GridSeg*, int, int, int, MgArgs, int, int, int, int, int, int, double*, hipStream_t, int, double, int, EvPair);
template hipError_t jac2<double>(LaneCtl*, const GridSeg*, int, int, int, MgArgs, int, int, int, double*, hipStream_t);
template hipError_t jac2<float>(LaneCtl*, const GridSeg*, int, int, int, MgArgs, int, int, int, double*, hipStream_t);
template hipError_t pjac<double>(LaneCtl*, const GridSeg*, int, int, int, MgArgs, int, hipStream_t, EvPair);
template hipError_t pjac<float>(LaneCtl*, const GridSeg*, int, int, int, MgArgs, int, hipStream_t, EvPair);
template hipError_t resid_fw<double>(LaneCtl*, const GridSeg*, int, int, int, MgArgs, int, hipStream_t, EvPair);
template hipError_t resid_fw<float>(LaneCtl*, const GridSeg*, int, int, int, MgArgs, int, hipStream_t, EvPair);
template hipError_t prolong<double>(LaneCtl*, const GridSeg*, int, int, MgArgs, int, int, hipStream_t);
template hipError_t prolong<float>(LaneCtl*, const GridSeg*, int, int, MgArgs, int, int, hipStream_t);
template hipError_t tail<double>(LaneCtl*, const TailSeg*, int, int, MgArgs, int, int, size_t, hipStream_t);
template hipError_t tail<float>(LaneCtl*, const TailSeg*, int, int, MgArgs, int, int, size_t, hipStream_t);

hipError_t mg_decide(LaneCtl* ctl, const GridSeg* segs, int nseg, int nblk, const double* partials,
                     int cycle, double tol, int max_cycles, int level, hipStream_t s)
{
    if (nseg <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mg_decide, dim3((unsigned)nseg), BLK, 0, s, segs, nseg, nblk, partials, ctl,
                       cycle, tol, max_cycles, level);
    return hipGetLastError();
}

hipError_t mg_norm(LaneCtl* ctl, const GridSeg* segs, int nseg, int nblk, int order, MgArgs a,
                   int cycle, double* partials, int src_is_t, hipStream_t s)
{
    if (nblk <= 0) return hipSuccess;
    HS_ORDER_DISPATCH(order, (k_mg_norm<2>), (k_mg_norm<4>), g1(nblk), BLK, 0, segs, nseg, nblk, ctl,
                      a, cycle, partials, src_is_t);
    return hipGetLastError();
}

hipError_t ir_resid(LaneCtl* ctl, const GridSeg* segs64, const GridSeg* segs32, int nseg, int nblk,
                    int order, MgArgs a, int iter, double* partials, hipStream_t s)
{
    if (nblk <= 0) return hipSuccess;
    HS_ORDER_DISPATCH(order, (k_ir_resid<2>), (k_ir_resid<4>), g1(nblk), BLK, 0, segs64, segs32,
                      nseg, nblk, ctl, a, iter, partials);
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
    HS_ORDER_DISPATCH(order, (k_spread<2>), (k_spread<4>), g1(nblk), BLK, 0, segs, nseg, nblk, ctl,
                      src_node);
    return hipGetLastError();
}

hipError_t sweep_prep(LaneCtl* ctl, const SdcSeg* segs, int nseg, int nblk, int with_resid,
                      int gate, double* partials, hipStream_t s)
{
    if (nblk <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_sweep_prep, g1(nblk), BLK, 0, s, segs, nseg, nblk, ctl, with_resid, gate,
                       partials);
    return hipGetLastError();
}

hipError_t sdc_decide(LaneCtl* ctl, const SdcSeg* segs, int nseg, int nblk, const double* partials,
                      double sdc_tol, int max_sweeps, hipStream_t s)
{
    if (nseg <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_sdc_decide, dim3((unsigned)nseg), BLK, 0, s, segs, nseg, nblk, partials, ctl,
                       sdc_tol, max_sweeps);
    return hipGetLastError();
}

hipError_t make_rhs(LaneCtl* ctl, const SdcSeg* segs, int nseg, int nblk, int m, int gate,
                    hipStream_t s)
{
    if (nblk <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_make_rhs, g1(nblk), BLK, 0, s, segs, nseg, nblk, ctl, m, gate);
    return hipGetLastError();
}

hipError_t fi_march(LaneCtl* ctl, const GridSeg* gsegs, const SdcSeg* ssegs, int nseg, int nblk, int order,
                    int m0, int m1, int rhs_node, int gate, hipStream_t s)
{
    if (nblk <= 0 || m1 <= m0) return hipSuccess;
    HS_ORDER_DISPATCH(order, (k_fi_march<2>), (k_fi_march<4>), g1(nblk), BLK, 0, gsegs, ssegs, nseg, nblk, ctl,
                      m0, m1, rhs_node, gate);
    return hipGetLastError();
}

hipError_t sdc_resid(LaneCtl* ctl, const SdcSeg* segs, int nseg, int nblk, double* partials,
                     hipStream_t s)
{
    if (nblk <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_sdc_resid, g1(nblk), BLK, 0, s, segs, nseg, nblk, ctl, partials);
    return hipGetLastError();
}

hipError_t handoff(LaneCtl* ctl, const SdcSeg* dst, const SdcSeg* src, int nseg, int nblk,
                   int order, hipStream_t s)
{
    if (nblk <= 0) return hipSuccess;
    HS_ORDER_DISPATCH(order, (k_handoff<2>), (k_handoff<4>), g1(nblk), BLK, 0, dst, src, nseg, nblk,
                      ctl);
    return hipGetLastError();
}

hipError_t fas_restrict(LaneCtl* ctl, const FasSeg* segs, int nseg, int nblk, int corder, int gate,
                        hipStream_t s)
{
    if (nblk <= 0) return hipSuccess;
    HS_ORDER_DISPATCH(corder, (k_fas_restrict<2>), (k_fas_restrict<4>), g1(nblk), BLK, 0, segs, nseg,
                      nblk, ctl, gate);
    return hipGetLastError();
}

hipError_t fas_interp3(LaneCtl* ctl, const FasSeg* segs, int nseg, int nblk, int gate, hipStream_t s)
{
    if (nblk <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fas_interp3_x, g1(nblk), BLK, 0, s, segs, nseg, nblk, ctl, gate);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_fas_interp3_y, g1(nblk), BLK, 0, s, segs, nseg, nblk, ctl, gate);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_fas_interp3_z, g1(nblk), BLK, 0, s, segs, nseg, nblk, ctl, gate);
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

hipError_t begin_step(LaneCtl* ctl, int nlanes, int nlevels, const int* M, hipStream_t s)
{
    hipLaunchKernelGGL(k_begin_step, lanes_grid(nlanes), dim3(64), 0, s, ctl, nlanes, nlevels, M[0],
                       nlevels > 1 ? M[1] : M[0], nlevels > 2 ? M[2] : M[0]);
    return hipGetLastError();
}

hipError_t end_step(LaneCtl* ctl, int nlanes, hipStream_t s)
{
    hipLaunchKernelGGL(k_end_step, lanes_grid(nlanes), dim3(64), 0, s, ctl, nlanes);
    return hipGetLastError();
}

hipError_t begin_solve(LaneCtl* ctl, int first, int nlanes, hipStream_t s)
{
    if (nlanes <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_begin_solve, lanes_grid(nlanes), dim3(64), 0, s, ctl, first, nlanes);
    return hipGetLastError();
}

hipError_t end_solve_fixed(LaneCtl* ctl, int first, int nlanes, int cycles, int level, hipStream_t s)
{
    if (nlanes <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_end_solve_fixed, lanes_grid(nlanes), dim3(64), 0, s, ctl, first, nlanes, cycles, level);
    return hipGetLastError();
}

hipError_t begin_sweep(LaneCtl* ctl, int first, int nlanes, hipStream_t s)
{
    if (nlanes <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_begin_sweep, lanes_grid(nlanes), dim3(64), 0, s, ctl, first, nlanes);
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

hipError_t fill(double* dst, long long count, double v, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    long long blocks = (count + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)blocks), dim3(256), 0, s, dst, count, v);
    return hipGetLastError();
}

hipError_t np_lanes(LaneCtl* ctl, int nlanes, int M, int mode, hipStream_t s)
{
    const int total = nlanes * (M - 1);
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_np_lanes, lanes_grid(total), dim3(64), 0, s, ctl, nlanes, M, mode);
    return hipGetLastError();
}

hipError_t np_rhs(LaneCtl* ctl, const SdcSeg* segs, int nseg, int nblk, hipStream_t s)
{
    if (nblk <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_np_rhs, g1(nblk), BLK, 0, s, segs, nseg, nblk, ctl);
    return hipGetLastError();
}

hipError_t sdc_reopen(LaneCtl* ctl, int nlanes, hipStream_t s)
{
    hipLaunchKernelGGL(k_sdc_reopen, lanes_grid(nlanes), dim3(64), 0, s, ctl, nlanes);
    return hipGetLastError();
}

hipError_t lap_apply(const GridSeg* segs, int nseg, int nblk, int order, double alpha, double beta,
                     const double* u, double* y, const long long* offs, hipStream_t s)
{
    if (nblk <= 0) return hipSuccess;
    HS_ORDER_DISPATCH(order, (k_lap_apply<2>), (k_lap_apply<4>), g1(nblk), BLK, 0, segs, nseg, nblk,
                      alpha, beta, u, y, offs);
    return hipGetLastError();
}

hipError_t heat_rhs(LaneCtl* ctl, const GridSeg* gsegs, const SdcSeg* ssegs, int nseg, int nblk, int order,
                    const double* u, const double* t, double* fi, double* fe,
                    const long long* offs, hipStream_t s)
{
    if (nblk <= 0) return hipSuccess;
    HS_ORDER_DISPATCH(order, (k_heat_rhs<2>), (k_heat_rhs<4>), g1(nblk), BLK, 0, gsegs, ssegs, nseg, nblk,
                      ctl, u, t, fi, fe, offs);
    return hipGetLastError();
}

hipError_t compact_apply(int n, int batch, double alpha, double beta, const double* u, double* y, hipStream_t s)
{
    if (batch <= 0) return hipSuccess;
    const int tiles = tiles_x(n) * tiles_y(n);
    int zb = 32;   // z chunks: enough blocks for the chip, long enough marches
    while (zb > 2 && (long long)batch * tiles * ((n + zb - 1) / zb) < 1024) zb /= 2;
    const int nz = (n + zb - 1) / zb;
    hipLaunchKernelGGL(k_compact_apply, dim3((unsigned)(batch * tiles * nz)), BLK, 0, s, n, zb, nz, alpha, beta, u,
                       y);
    return hipGetLastError();
}

static void cmp_shape(int n, int* zb, int* nz)
{
    const int tiles = tiles_x(n) * tiles_y(n);
    int z = 32;
    while (z > 2 && (long long)tiles * ((n + z - 1) / z) < 512) z /= 2;
    *zb = z;
    *nz = (n + z - 1) / z;
}

int compact_blocks(int n)
{
    int zb, nz;
    cmp_shape(n, &zb, &nz);
    return tiles_x(n) * tiles_y(n) * nz;
}

hipError_t compact_op(int mode, int n, const double* src, double* dst, const double* b, const double* g2,
                      const LaneCtl* ctl, int lane, double dtau, double omega, double* partials, int gate,
                      hipStream_t s)
{
    int zb, nz;
    cmp_shape(n, &zb, &nz);
    const dim3 grid((unsigned)(tiles_x(n) * tiles_y(n) * nz));
#define HS_CMP_LAUNCH(MD) \
    hipLaunchKernelGGL(k_cmp<MD>, grid, BLK, 0, s, n, zb, src, dst, b, g2, ctl, lane, dtau, omega, partials, gate)
    switch (mode) {
    case 0: HS_CMP_LAUNCH(0); break;
    case 1: HS_CMP_LAUNCH(1); break;
    case 2: HS_CMP_LAUNCH(2); break;
    case 3: HS_CMP_LAUNCH(3); break;
    case 4: HS_CMP_LAUNCH(4); break;
    default: HS_CMP_LAUNCH(5); break;
    }
#undef HS_CMP_LAUNCH
    return hipGetLastError();
}

hipError_t compact_fw(int nf, const double* rf, double* bc, const LaneCtl* ctl, int lane, int gate, hipStream_t s)
{
    const int nc = (nf - 1) / 2;
    if (nc <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_cmp_fw, dim3((unsigned)((nc * nc + HS_BLOCK - 1) / HS_BLOCK), (unsigned)nc), BLK, 0, s, nf,
                       rf, bc, ctl, lane, gate);
    return hipGetLastError();
}

hipError_t compact_prolong(int nc, const double* ec, const double* src, double* dst, const LaneCtl* ctl, int lane,
                           int gate, hipStream_t s)
{
    const int nf = 2 * nc + 1;
    hipLaunchKernelGGL(k_cmp_prolong, dim3((unsigned)((nf * nf + HS_BLOCK - 1) / HS_BLOCK), (unsigned)nf), BLK, 0, s,
                       nc, ec, src, dst, ctl, lane, gate);
    return hipGetLastError();
}

hipError_t compact_zsweep(int n, const double* b, double* dst, const LaneCtl* ctl, int lane, double dtau,
                          double omega, int gate, hipStream_t s)
{
    const long long N = (long long)n * n * n;
    hipLaunchKernelGGL(k_cmp_zsweep, dim3((unsigned)((N + HS_BLOCK - 1) / HS_BLOCK)), BLK, 0, s, n, b, dst, ctl, lane,
                       dtau, omega, gate);
    return hipGetLastError();
}

size_t compact_tail_lds(int n0, int n_coarsest)
{
    size_t pts = 0;
    int n = n0, l = 0;
    for (;;) {
        pts += 2 * (size_t)(n + 2) * (n + 2) * (n + 2) + (size_t)n * n * n;
        if (!(n > n_coarsest && n > 1 && l + 1 < HS_MAXTAIL)) break;
        n = (n - 1) / 2;
        l++;
    }
    return 8 * pts;
}

hipError_t compact_tail(int n0, double* u, const double* b, int zero_guess, const LaneCtl* ctl, int lane, double dtau,
                        double omega, int nu1, int nu2, int n_coarsest, int gate, hipStream_t s)
{
    if (n0 < 1 || n0 > HS_TAIL_N) return hipErrorInvalidValue;
    const size_t lds = compact_tail_lds(n0, n_coarsest);
    if (lds > 65536) {   // a 15^3 top grid needs about 104 KB; raised once per device
        static std::mutex mu;
        static std::map<int, size_t> allowed;
        int dev = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) return e;
        std::lock_guard<std::mutex> lock(mu);
        size_t& al = allowed[dev];
        if (lds > al) {
            e = hipFuncSetAttribute((const void*)k_cmp_tail, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
            al = lds;
        }
    }
    hipLaunchKernelGGL(k_cmp_tail, dim3(1), dim3(HS_TAIL_THREADS), (unsigned)lds, s, n0, u, b, zero_guess, ctl, lane,
                       dtau, omega, nu1, nu2, n_coarsest, gate);
    return hipGetLastError();
}

hipError_t compact_quad(int n, int M, int m, const double* G, const double* base, double* dst, const double* sig,
                        const LaneCtl* ctl, int lane, int L, hipStream_t s)
{
    const long long N = (long long)n * n * n;
    hipLaunchKernelGGL(k_cmp_quad, dim3((unsigned)((N + HS_BLOCK - 1) / HS_BLOCK)), BLK, 0, s, n, M, m, G, base, dst,
                       sig, ctl, lane, L);
    return hipGetLastError();
}

hipError_t compact_reduce(const double* partials, int nblk, LaneCtl* ctl, int lane, int mode, int cycle, double tol,
                          int max_cycles, hipStream_t s)
{
    hipLaunchKernelGGL(k_cmp_reduce, dim3(1), BLK, 0, s, partials, nblk, ctl, lane, mode, cycle, tol, max_cycles,
                       -3, -4);   // HS_ENOCONV, HS_ENONFINITE
    return hipGetLastError();
}

hipError_t compact_binv(int n, const double* tab, const double* y, double* x, double* t0, double* t1, hipStream_t s)
{
    const unsigned g = (unsigned)(((long long)n * n * n + HS_BLOCK - 1) / HS_BLOCK);
    const int C[3] = {1, n, n * n};
    const double* src = y;
    double* bufs[2] = {t0, t1};
    // S3 y into t0 (x, y, z axes: y -> t0 -> t1 -> t0)
    for (int ax = 0; ax < 3; ax++) {
        double* dst = bufs[ax & 1];
        hipLaunchKernelGGL(k_dst_axis, dim3(g), BLK, 0, s, n, C[ax], tab, src, dst);
        src = dst;
    }
    hipLaunchKernelGGL(k_binv_scale, dim3(g), BLK, 0, s, n, tab, t0);
    // S3 of the scaled values: t0 -> t1 -> t0 -> x
    hipLaunchKernelGGL(k_dst_axis, dim3(g), BLK, 0, s, n, C[0], tab, (const double*)t0, t1);
    hipLaunchKernelGGL(k_dst_axis, dim3(g), BLK, 0, s, n, C[1], tab, (const double*)t1, t0);
    hipLaunchKernelGGL(k_dst_axis, dim3(g), BLK, 0, s, n, C[2], tab, (const double*)t0, x);
    return hipGetLastError();
}

hipError_t compact_ctl(LaneCtl* ctl, int lane, int op, int cycles, int state, int level, int status, hipStream_t s)
{
    hipLaunchKernelGGL(k_cmp_ctl, dim3(1), dim3(64), 0, s, ctl, lane, op, cycles, state, level, status);
    return hipGetLastError();
}

}  // namespace hsk
