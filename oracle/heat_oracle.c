/*
 * heat_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, serial, deliberately unoptimised FP64 implementation of the
 * space-time heat solver of Speck, Ruprecht, Emmett, Bolten and Krause,
 * "A space-time parallel solver for the three-dimensional heat equation"
 * (arXiv 1307.7867).  It exists so that the GPU library can be checked
 * against something written straight from the mathematics.  Only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark may load
 * it; the GPU library never links against it and shares no code with it.
 *
 * Every function names the passage of the paper (section / equation) it
 * follows.  Where the paper is silent (multigrid components, stopping rules,
 * wall closure of the wide 4th-order stencil, predictor) the reading used is
 * stated at the function.
 *
 * Grid convention (section 1, eqs. (1)-(2)): n interior points per axis,
 * h = 1/(n+1), interior point (i,j,k), 0-based, sits at x = ((i+1)h,
 * (j+1)h, (k+1)h); u = 0 on the walls.  Arrays are [k][j][i] with i fastest.
 *
 * Compile with -ffp-contract=off: no fused multiply-adds, so every
 * expression is rounded exactly as written.
 *
 * Parity unpinned: the timing of PFASST's fine hand-off in or_pfasst (the
 * previous iteration's end value) and, with three levels, the sweep on the
 * middle level on the way up of the MLSDC V-cycle (mlsdc_vcycle) are
 * readings that no test fixes; every other function is pinned by
 * tests/test_oracle_pins.py.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ENOCONV (-3)
#define OR_ENONFINITE (-4)

#define OR_MAXM 8
#define OR_MAXLEV 3
#define OR_ORDER_COMPACT (-4)   /* level order code of the compact 4th-order scheme */

typedef struct {
    int32_t nu1, nu2;     /* pre / post smoothing sweeps */
    double omega;         /* Jacobi weight */
    int32_t n_coarsest;   /* grid solved exactly (1 or 3) */
    double tol;           /* relative max-norm residual target */
    int32_t max_cycles;   /* cap on V-cycles when iterating to tol */
    int32_t fixed_cycles; /* > 0: exactly this many V-cycles, no test */
} or_mg;

typedef struct {
    int32_t n;      /* interior points per axis */
    int32_t order;  /* 2 or 4, or OR_ORDER_COMPACT (finest level of SDC or two-level MLSDC) */
    int32_t M;      /* collocation nodes including both ends */
} or_level;

typedef struct {
    double nu, t0, dt, forcing_c;
    int32_t nsteps;
    int32_t sweeps;      /* fixed sweeps / MLSDC iterations; 0 = iterate to sdc_tol */
    double sdc_tol;
    int32_t max_sweeps;
    int32_t nlevels;     /* 1 = SDC, 2 or 3 = MLSDC */
    or_level lev[OR_MAXLEV]; /* lev[0] finest, lev[nlevels-1] coarsest */
    or_mg mg;
    int32_t node_parallel; /* single-level SDC: 1 = node-parallel sweeps (or_sdc_sweep_nodes) */
    int32_t fas_interp;    /* MLSDC / PFASST: spatial interpolation of the coarse correction,
                              1 (or 0) trilinear, 3 tricubic (or_prolong_add_cubic) */
} or_problem;

typedef struct {
    int32_t status;
    int32_t sweeps;          /* sweeps (or MLSDC iterations) of the last step */
    int32_t total_sweeps;
    int32_t total_solves;
    int64_t total_cycles;    /* V-cycles over all solves */
    int32_t max_cycles_seen;
    double last_residual;    /* collocation residual after the last sweep */
} or_stats;

/* ------------------------------------------------------------------ */
/* Grid helpers                                                        */
/* ------------------------------------------------------------------ */

static size_t cube(int n) { return (size_t)n * (size_t)n * (size_t)n; }

static int valid_n(int n)
{
    /* n = 2^k - 1 with 1 <= n <= 1023 */
    if (n < 1 || n > 1023) return 0;
    return ((n + 1) & n) == 0;
}

double or_grid_h(int n) { return 1.0 / (double)(n + 1); }

static double *alloc0(size_t count)
{
    double *p = (double *)calloc(count ? count : 1, sizeof(double));
    if (!p) abort();
    return p;
}

/*
 * Value of u along one axis at 0-based index q of a line whose other two
 * indices are fixed.  Indices 0..n-1 are interior points; -1 and n are the
 * walls where u = 0 (eq. (2)).  The wide 4th-order stencil also reaches -2
 * and n+1: there the odd reflection u(-2) = -u(0), u(n+1) = -u(n-1) is used
 * (the paper gives no wall closure for its 4th-order operator; the odd
 * reflection keeps the discrete sine modes exact eigenvectors).
 */
static double line_val(const double *u, int n, int i, int j, int k, int axis, int q)
{
    int sign = 1;
    if (q == -1 || q == n) return 0.0;
    if (q == -2) { q = 0; sign = -1; }
    if (q == n + 1) { q = n - 1; sign = -1; }
    if (q < 0 || q >= n) return 0.0;
    if (axis == 0) i = q;
    else if (axis == 1) j = q;
    else k = q;
    return sign * u[((size_t)k * n + j) * n + i];
}

/*
 * Discrete Laplacian L_h (section 1: method of lines; the coarse level uses
 * the classical second-order 7-point stencil, the fine level a fourth-order
 * stencil).  order 2: (u_{-1} - 2 u_0 + u_{+1}) / h^2 per axis.
 * order 4: (-u_{-2} + 16 u_{-1} - 30 u_0 + 16 u_{+1} - u_{+2}) / (12 h^2)
 * per axis (the wide 13-point stencil).  Axis sums are taken x, then y,
 * then z.
 */
void or_laplacian(int n, int order, const double *u, double *Lu)
{
    double h = or_grid_h(n);
    double ih2 = 1.0 / (h * h);
    for (int k = 0; k < n; k++)
        for (int j = 0; j < n; j++)
            for (int i = 0; i < n; i++) {
                int c[3] = {i, j, k};
                double sum = 0.0;
                for (int ax = 0; ax < 3; ax++) {
                    int q = c[ax];
                    double d;
                    if (order == 2) {
                        d = line_val(u, n, i, j, k, ax, q - 1)
                          - 2.0 * line_val(u, n, i, j, k, ax, q)
                          + line_val(u, n, i, j, k, ax, q + 1);
                        d = d * ih2;
                    } else {
                        d = -line_val(u, n, i, j, k, ax, q - 2)
                          + 16.0 * line_val(u, n, i, j, k, ax, q - 1)
                          - 30.0 * line_val(u, n, i, j, k, ax, q)
                          + 16.0 * line_val(u, n, i, j, k, ax, q + 1)
                          - line_val(u, n, i, j, k, ax, q + 2);
                        d = d * ih2 / 12.0;
                    }
                    sum += d;
                }
                Lu[((size_t)k * n + j) * n + i] = sum;
            }
}

/* y = alpha u + beta L_h u (method of lines, section 1). */
void or_lap_apply(int n, int order, double alpha, double beta, const double *u, double *y)
{
    size_t N = cube(n);
    double *L = alloc0(N);
    or_laplacian(n, order, u, L);
    for (size_t p = 0; p < N; p++) y[p] = alpha * u[p] + beta * L[p];
    free(L);
}

/* u at (i, j, k), 0 outside the grid (the walls and beyond, eq. (2)) */
static double val3(const double *u, int n, int i, int j, int k)
{
    if (i < 0 || j < 0 || k < 0 || i >= n || j >= n || k >= n) return 0.0;
    return u[((size_t)k * n + j) * n + i];
}

/*
 * The compact fourth-order pair of the fine level (section 1 names a
 * fourth-order compact stencil there, and sec. 1.2 a weighting matrix that
 * the multigrid solver inverts for the FAS correction; the paper gives
 * neither, so this is the reading: the 19-point Mehrstellen pair)
 *   A_h u = (2 (sum of the 6 face neighbours) + (sum of the 12 edge
 *            neighbours) - 24 u) / (6 h^2),
 *   B_h u = u / 2 + (sum of the 6 face neighbours) / 12 = (I + h^2/12 D_h) u
 * with the 7-point D_h, for which A_h u = B_h f is fourth-order accurate for
 * Laplace(u) = f.  y = alpha B_h u + beta A_h u, zero Dirichlet walls.
 * Sums: faces x, y, z (minus before plus); edges of the xy, xz, yz planes.
 */
void or_compact_apply(int n, double alpha, double beta, const double *u, double *y)
{
    double h = or_grid_h(n);
    double ih2 = 1.0 / (h * h);
    for (int k = 0; k < n; k++)
        for (int j = 0; j < n; j++)
            for (int i = 0; i < n; i++) {
                double c = val3(u, n, i, j, k);
                double faces = ((val3(u, n, i - 1, j, k) + val3(u, n, i + 1, j, k)) +
                                (val3(u, n, i, j - 1, k) + val3(u, n, i, j + 1, k))) +
                               (val3(u, n, i, j, k - 1) + val3(u, n, i, j, k + 1));
                double exy = (val3(u, n, i - 1, j - 1, k) + val3(u, n, i + 1, j - 1, k)) +
                             (val3(u, n, i - 1, j + 1, k) + val3(u, n, i + 1, j + 1, k));
                double exz = (val3(u, n, i - 1, j, k - 1) + val3(u, n, i + 1, j, k - 1)) +
                             (val3(u, n, i - 1, j, k + 1) + val3(u, n, i + 1, j, k + 1));
                double eyz = (val3(u, n, i, j - 1, k - 1) + val3(u, n, i, j + 1, k - 1)) +
                             (val3(u, n, i, j - 1, k + 1) + val3(u, n, i, j + 1, k + 1));
                double A = ((2.0 * faces + ((exy + exz) + eyz)) - 24.0 * c) * ih2 / 6.0;
                double B = 0.5 * c + faces / 12.0;
                y[((size_t)k * n + j) * n + i] = alpha * B + beta * A;
            }
}

/*
 * x = B_h^{-1} y, exactly, in the sine basis: every discrete sine mode is an
 * eigenvector of B_h with eigenvalue 1/2 + (cos(pi p h) + cos(pi q h) +
 * cos(pi r h))/6, so B_h = S diag(lambda) S with S the orthonormal DST-I
 * (S_ab = sqrt(2/(n+1)) sin(pi (a+1)(b+1)/(n+1)), applied along each axis;
 * S S = I).  Section 1.2 has the multigrid solver invert B_h for the FAS
 * correction; B_h is too ill-conditioned for that in 3-D (its smallest
 * eigenvalue is about pi^2 h^2 / 4), so the inverse is taken exactly (a
 * reading).
 */
static void dst_axis(int n, const double *S, const double *in, double *out, int axis)
{
    size_t st = axis == 0 ? 1 : axis == 1 ? (size_t)n : (size_t)n * n;
    for (int k = 0; k < n; k++)
        for (int j = 0; j < n; j++)
            for (int i = 0; i < n; i++) {
                int c[3] = {i, j, k};
                size_t p = ((size_t)k * n + j) * n + i;
                size_t base = p - (size_t)c[axis] * st;
                double sum = 0.0;
                for (int q = 0; q < n; q++) sum += S[(size_t)c[axis] * n + q] * in[base + (size_t)q * st];
                out[p] = sum;
            }
}

void or_compact_binv(int n, const double *y, double *x)
{
    size_t N = cube(n);
    double *S = alloc0((size_t)n * n), *cs = alloc0(n), *t1 = alloc0(N), *t2 = alloc0(N);
    for (int a = 0; a < n; a++) {
        cs[a] = cos(M_PI * (a + 1) / (n + 1));
        for (int b = 0; b < n; b++) S[(size_t)a * n + b] = sqrt(2.0 / (n + 1)) * sin(M_PI * (a + 1) * (b + 1) / (n + 1));
    }
    dst_axis(n, S, y, t1, 0);
    dst_axis(n, S, t1, t2, 1);
    dst_axis(n, S, t2, t1, 2);
    for (int k = 0; k < n; k++)
        for (int j = 0; j < n; j++)
            for (int i = 0; i < n; i++)
                t1[((size_t)k * n + j) * n + i] /= 0.5 + ((cs[i] + cs[j]) + cs[k]) / 6.0;
    dst_axis(n, S, t1, t2, 0);
    dst_axis(n, S, t2, t1, 1);
    dst_axis(n, S, t1, x, 2);
    free(S); free(cs); free(t1); free(t2);
}

/*
 * The implicit-Euler substep operator A_a = I - a L_h with a = nu * dt_m
 * (eq. (7): the implicit part of the IMEX sweep moved to the left); for the
 * compact scheme B_h - a A_h (the weighting matrix multiplies eq. (7)).
 */
void or_heat_op(int n, int order, double a, const double *u, double *y)
{
    if (order == OR_ORDER_COMPACT) or_compact_apply(n, 1.0, -a, u, y);
    else or_lap_apply(n, order, 1.0, -a, u, y);
}

/*
 * Diagonal of A_a, from the stencil weights: the centre weight of L_h per
 * axis is -2/h^2 (order 2) and -30/(12 h^2) (order 4), except that with the
 * odd reflection a wall-adjacent point also picks up +1/(12 h^2) from its
 * reflected far neighbour.  Compact scheme: 1/2 - a (-24/(6 h^2)).
 */
static double diag_op(int n, int order, double a, int i, int j, int k)
{
    double h = or_grid_h(n);
    double ih2 = 1.0 / (h * h);
    if (order == OR_ORDER_COMPACT) return 0.5 + a * 24.0 * ih2 / 6.0;   /* B_h: 1/2, A_h: -24/(6 h^2) */
    int c[3] = {i, j, k};
    double centre = 0.0;
    for (int ax = 0; ax < 3; ax++) {
        if (order == 2) {
            centre += -2.0 * ih2;
        } else {
            double w = -30.0;
            if (c[ax] == 0) w += 1.0;
            if (c[ax] == n - 1) w += 1.0;
            centre += w * ih2 / 12.0;
        }
    }
    return 1.0 - a * centre;
}

/* r = b - A_a u */
void or_residual(int n, int order, double a, const double *u, const double *b, double *r)
{
    size_t N = cube(n);
    double *Au = alloc0(N);
    or_heat_op(n, order, a, u, Au);
    for (size_t p = 0; p < N; p++) r[p] = b[p] - Au[p];
    free(Au);
}

/* Weighted Jacobi: u_new = u + omega D^{-1} (b - A_a u).  The paper names
 * no smoother (section 1.2); weighted Jacobi is the reading used here. */
void or_jacobi(int n, int order, double a, double omega, const double *u, const double *b,
               double *u_new)
{
    size_t N = cube(n);
    double *r = alloc0(N);
    or_residual(n, order, a, u, b, r);
    for (int k = 0; k < n; k++)
        for (int j = 0; j < n; j++)
            for (int i = 0; i < n; i++) {
                size_t p = ((size_t)k * n + j) * n + i;
                u_new[p] = u[p] + omega * r[p] / diag_op(n, order, a, i, j, k);
            }
    free(r);
}

/*
 * Full-weighting restriction: coarse point I (0-based) coincides with fine
 * point 2I+1; weights are the tensor product of (1/4, 1/2, 1/4).
 */
void or_restrict_fw(int nf, const double *rf, double *rc)
{
    int nc = (nf - 1) / 2;
    const double w[3] = {0.25, 0.5, 0.25};
    for (int K = 0; K < nc; K++)
        for (int J = 0; J < nc; J++)
            for (int I = 0; I < nc; I++) {
                double s = 0.0;
                for (int dz = -1; dz <= 1; dz++)
                    for (int dy = -1; dy <= 1; dy++)
                        for (int dx = -1; dx <= 1; dx++) {
                            int i = 2 * I + 1 + dx, j = 2 * J + 1 + dy, k = 2 * K + 1 + dz;
                            s += w[dx + 1] * w[dy + 1] * w[dz + 1]
                               * rf[((size_t)k * nf + j) * nf + i];
                        }
                rc[((size_t)K * nc + J) * nc + I] = s;
            }
}

/* weight and coarse index pair for one fine index along one axis */
static void prolong_weights(int nc, int i, int idx[2], double wt[2], int *cnt)
{
    if (i % 2 == 1) {            /* coincides with coarse (i-1)/2 */
        idx[0] = (i - 1) / 2; wt[0] = 1.0; *cnt = 1;
    } else {                     /* halfway between coarse i/2-1 and i/2 */
        idx[0] = i / 2 - 1; wt[0] = 0.5;
        idx[1] = i / 2;     wt[1] = 0.5;
        *cnt = 2;
    }
    (void)nc;
}

/* Trilinear prolongation added to a fine field: uf += P ec (walls are 0). */
void or_prolong_add(int nc, const double *ec, double *uf)
{
    int nf = 2 * nc + 1;
    for (int k = 0; k < nf; k++)
        for (int j = 0; j < nf; j++)
            for (int i = 0; i < nf; i++) {
                int ix[2], iy[2], iz[2], cx, cy, cz;
                double wx[2], wy[2], wz[2];
                prolong_weights(nc, i, ix, wx, &cx);
                prolong_weights(nc, j, iy, wy, &cy);
                prolong_weights(nc, k, iz, wz, &cz);
                double s = 0.0;
                for (int c = 0; c < cz; c++)
                    for (int b = 0; b < cy; b++)
                        for (int a = 0; a < cx; a++) {
                            int I = ix[a], J = iy[b], K = iz[c];
                            if (I < 0 || I >= nc || J < 0 || J >= nc || K < 0 || K >= nc) continue;
                            s += wx[a] * wy[b] * wz[c] * ec[((size_t)K * nc + J) * nc + I];
                        }
                uf[((size_t)k * nf + j) * nf + i] += s;
            }
}

/*
 * Tricubic interpolation added to a fine field: uf += P3 ec.  Per axis a
 * fine point that coincides with a coarse point takes its value; a point
 * halfway between coarse points takes the cubic Lagrange interpolant
 * through the two coarse points on either side, weights (-1, 9, 9, -1)/16.
 * A tap on a wall is 0; a tap one coarse cell beyond a wall takes the odd
 * reflection of the value one cell inside it (u(-x) = -u(x) about the wall),
 * which continues the zero Dirichlet data the way sine modes do.  The fine
 * value is the sum over the taps of wx wy wz ec, taps in x, y, z order.
 */
static double cubic_tap(const double *ec, int nc, int I, int J, int K)
{
    int idx[3] = {I, J, K};
    double sign = 1.0;
    for (int d = 0; d < 3; d++) {
        if (idx[d] == -1 || idx[d] == nc) return 0.0;
        if (idx[d] == -2) { idx[d] = 0; sign = -sign; }
        else if (idx[d] == nc + 1) { idx[d] = nc - 1; sign = -sign; }
    }
    return sign * ec[((size_t)idx[2] * nc + idx[1]) * nc + idx[0]];
}

static void cubic_weights(int i, int idx[4], double wt[4], int *cnt)
{
    if (i % 2 == 1) {            /* coincides with coarse (i-1)/2 */
        idx[0] = (i - 1) / 2; wt[0] = 1.0; *cnt = 1;
    } else {                     /* between coarse i/2-1 and i/2 */
        int m = i / 2;
        idx[0] = m - 2; wt[0] = -1.0 / 16.0;
        idx[1] = m - 1; wt[1] = 9.0 / 16.0;
        idx[2] = m;     wt[2] = 9.0 / 16.0;
        idx[3] = m + 1; wt[3] = -1.0 / 16.0;
        *cnt = 4;
    }
}

void or_prolong_add_cubic(int nc, const double *ec, double *uf)
{
    int nf = 2 * nc + 1;
    for (int k = 0; k < nf; k++)
        for (int j = 0; j < nf; j++)
            for (int i = 0; i < nf; i++) {
                int ix[4], iy[4], iz[4], cx, cy, cz;
                double wx[4], wy[4], wz[4];
                cubic_weights(i, ix, wx, &cx);
                cubic_weights(j, iy, wy, &cy);
                cubic_weights(k, iz, wz, &cz);
                double s = 0.0;
                for (int c = 0; c < cz; c++)
                    for (int b = 0; b < cy; b++)
                        for (int a = 0; a < cx; a++)
                            s += wx[a] * wy[b] * wz[c] * cubic_tap(ec, nc, ix[a], iy[b], iz[c]);
                uf[((size_t)k * nf + j) * nf + i] += s;
            }
}

/*
 * Exact solve of A_a x = b by assembling the dense matrix column by column
 * (A applied to unit vectors) and Gaussian elimination with partial
 * pivoting.  Used on the coarsest multigrid grid and, in tests, as the
 * brute-force reference on tiny grids.
 */
int or_dense_solve(int n, int order, double a, const double *b, double *x)
{
    size_t N = cube(n);
    if (N > 4096) return OR_EINVAL;
    double *A = alloc0(N * N);
    double *e = alloc0(N);
    double *col = alloc0(N);
    for (size_t q = 0; q < N; q++) {
        memset(e, 0, N * sizeof(double));
        e[q] = 1.0;
        or_heat_op(n, order, a, e, col);
        for (size_t p = 0; p < N; p++) A[p * N + q] = col[p];
    }
    double *rhs = alloc0(N);
    memcpy(rhs, b, N * sizeof(double));
    for (size_t c = 0; c < N; c++) {
        size_t piv = c;
        for (size_t p = c + 1; p < N; p++)
            if (fabs(A[p * N + c]) > fabs(A[piv * N + c])) piv = p;
        if (piv != c) {
            for (size_t q = 0; q < N; q++) {
                double t = A[c * N + q]; A[c * N + q] = A[piv * N + q]; A[piv * N + q] = t;
            }
            double t = rhs[c]; rhs[c] = rhs[piv]; rhs[piv] = t;
        }
        for (size_t p = c + 1; p < N; p++) {
            double f = A[p * N + c] / A[c * N + c];
            if (f == 0.0) continue;
            for (size_t q = c; q < N; q++) A[p * N + q] -= f * A[c * N + q];
            rhs[p] -= f * rhs[c];
        }
    }
    for (size_t c = N; c-- > 0;) {
        double s = rhs[c];
        for (size_t q = c + 1; q < N; q++) s -= A[c * N + q] * x[q];
        x[c] = s / A[c * N + c];
    }
    free(A); free(e); free(col); free(rhs);
    return OR_OK;
}

/*
 * One multigrid V(nu1,nu2) cycle for A_a u = b (section 1.2 says only that
 * a parallel geometric multigrid method is used; the components here are
 * the reading: same-order rediscretisation on every grid, weighted Jacobi,
 * full weighting, trilinear prolongation, exact solve on the coarsest grid).
 */
static void vcycle(int n, int order, double a, const or_mg *p, double *u, const double *b)
{
    size_t N = cube(n);
    if (n <= p->n_coarsest) {
        or_dense_solve(n, order, a, b, u);
        return;
    }
    double *t = alloc0(N);
    for (int s = 0; s < p->nu1; s++) {
        or_jacobi(n, order, a, p->omega, u, b, t);
        memcpy(u, t, N * sizeof(double));
    }
    double *r = alloc0(N);
    or_residual(n, order, a, u, b, r);
    int nc = (n - 1) / 2;
    double *bc = alloc0(cube(nc));
    double *ec = alloc0(cube(nc));
    or_restrict_fw(n, r, bc);
    vcycle(nc, order, a, p, ec, bc);
    or_prolong_add(nc, ec, u);
    for (int s = 0; s < p->nu2; s++) {
        or_jacobi(n, order, a, p->omega, u, b, t);
        memcpy(u, t, N * sizeof(double));
    }
    free(t); free(r); free(bc); free(ec);
}

static double maxabs(const double *v, size_t N)
{
    double m = 0.0;
    for (size_t p = 0; p < N; p++) {
        double x = fabs(v[p]);
        if (x > m || x != x) m = x;
        if (m != m) return m;
    }
    return m;
}

/*
 * Solve A_a u = b by V-cycles from the initial guess in u.  Stopping rule
 * (not given in the paper): before each cycle rho = |b - A u|_inf / |b|_inf
 * (|b|_inf replaced by 1 when b = 0); stop when rho <= tol, fail after
 * max_cycles cycles.  With fixed_cycles > 0 exactly that many cycles run.
 */
int or_mg_solve(int n, int order, double a, const or_mg *p, double *u, const double *b,
                int *cycles_out, double *rho_out)
{
    if (!valid_n(n) || (order != 2 && order != 4 && order != OR_ORDER_COMPACT)) return OR_EINVAL;
    size_t N = cube(n);
    double *r = alloc0(N);
    double bn = maxabs(b, N);
    double scale = bn > 0.0 ? bn : 1.0;
    int status = OR_OK, c = 0;
    double rho = 0.0;
    if (p->fixed_cycles > 0) {
        for (c = 0; c < p->fixed_cycles; c++) vcycle(n, order, a, p, u, b);
        or_residual(n, order, a, u, b, r);
        rho = maxabs(r, N) / scale;
        if (rho != rho) status = OR_ENONFINITE;
    } else {
        for (c = 0;; c++) {
            or_residual(n, order, a, u, b, r);
            rho = maxabs(r, N) / scale;
            if (rho != rho) { status = OR_ENONFINITE; break; }
            if (rho <= p->tol) break;
            if (c >= p->max_cycles) { status = OR_ENOCONV; break; }
            vcycle(n, order, a, p, u, b);
        }
    }
    if (cycles_out) *cycles_out = c;
    if (rho_out) *rho_out = rho;
    free(r);
    return status;
}

/* ------------------------------------------------------------------ */
/* Collocation nodes and weights (section 1.1, eqs. (5)-(6))           */
/* ------------------------------------------------------------------ */

/* Legendre P_N(x) and P_N'(x) by the three-term recurrence. */
static void legendre(int N, long double x, long double *P, long double *dP)
{
    long double p0 = 1.0L, p1 = x;
    if (N == 0) { *P = 1.0L; *dP = 0.0L; return; }
    for (int k = 2; k <= N; k++) {
        long double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
        p0 = p1; p1 = p2;
    }
    *P = p1;
    *dP = N * (x * p1 - p0) / (x * x - 1.0L);
}

/* Gauss-Lobatto nodes on [0,1] in long double (see or_lobatto_nodes). */
static void lobatto_nodes_ld(int M, long double *t)
{
    int N = M - 1;
    t[0] = 0.0L; t[N] = 1.0L;
    for (int j = 1; j < N; j++) {
        long double z = -cosl(3.14159265358979323846264338327950288L * j / N);
        for (int it = 0; it < 100; it++) {
            long double P, dP;
            legendre(N, z, &P, &dP);
            /* P'' from the Legendre differential equation */
            long double d2P = (2.0L * z * dP - N * (N + 1) * P) / (1.0L - z * z);
            long double dz = dP / d2P;
            z -= dz;
            if (fabsl(dz) < 1e-30L) break;
        }
        t[j] = (z + 1.0L) / 2.0L;
    }
}

/*
 * Gauss-Lobatto nodes on [0,1]: the two end points plus the roots of
 * P'_{M-1} (so that T^n and T^{n+1} are nodes, section 1.1).  M counts all
 * nodes including both ends.
 */
int or_lobatto_nodes(int M, double *tau)
{
    if (M < 2 || M > OR_MAXM) return OR_EINVAL;
    long double t[OR_MAXM];
    lobatto_nodes_ld(M, t);
    for (int j = 0; j < M; j++) tau[j] = (double)t[j];
    return OR_OK;
}

/* Lagrange basis polynomial l_j of the nodes t at s. */
static long double lagrange(int M, const long double *t, int j, long double s)
{
    long double v = 1.0L;
    for (int i = 0; i < M; i++)
        if (i != j) v *= (s - t[i]) / (t[j] - t[i]);
    return v;
}

/*
 * Collocation matrix of eq. (6): Q[m*M + j] = integral from 0 to tau_m of
 * l_j(s) ds (row m = node, column j = source node), on the unit interval.
 * Integrated with 8-point Gauss-Legendre quadrature in long double, exact
 * for the degree M-1 <= 15 integrands.
 */
int or_collocation_matrix(int M, double *Q)
{
    if (M < 2 || M > OR_MAXM) return OR_EINVAL;
    long double t[OR_MAXM];
    lobatto_nodes_ld(M, t);
    const int G = 8;
    long double gx[8], gw[8];
    for (int g = 0; g < G; g++) {
        long double z = cosl(3.14159265358979323846264338327950288L * (g + 0.75L) / (G + 0.5L));
        for (int it = 0; it < 100; it++) {
            long double P, dP;
            legendre(G, z, &P, &dP);
            long double dz = P / dP;
            z -= dz;
            if (fabsl(dz) < 1e-30L) break;
        }
        long double P, dP;
        legendre(G, z, &P, &dP);
        gx[g] = z;
        gw[g] = 2.0L / ((1.0L - z * z) * dP * dP);
    }
    for (int m = 0; m < M; m++)
        for (int j = 0; j < M; j++) {
            long double s = 0.0L;
            for (int g = 0; g < G; g++)
                s += gw[g] * lagrange(M, t, j, t[m] * (1.0L + gx[g]) / 2.0L);
            Q[m * M + j] = (double)(s * t[m] / 2.0L);
        }
    return OR_OK;
}

/* Lagrange interpolation weights from the coarse nodes to one point s. */
static void interp_weights(int Mc, double s, double *w)
{
    long double t[OR_MAXM];
    lobatto_nodes_ld(Mc, t);
    for (int j = 0; j < Mc; j++) w[j] = (double)lagrange(Mc, t, j, (long double)s);
}

/* ------------------------------------------------------------------ */
/* Right-hand side (eqs. (1)-(4))                                      */
/* ------------------------------------------------------------------ */

/*
 * Forcing of eq. (3): f(x,t) = -s(x) (sin t - c nu pi^2 cos t) with
 * s(x) = sin(pi x1) sin(pi x2) sin(pi x3).  As printed, c = 1; the stated
 * analytic solution u = s(x) cos t (eq. (4)) needs c = 3 in three
 * dimensions, so c is a parameter.
 */
void or_forcing(int n, double nu, double c, double t, double *f)
{
    double h = or_grid_h(n);
    double g = -(sin(t) - c * nu * M_PI * M_PI * cos(t));
    for (int k = 0; k < n; k++)
        for (int j = 0; j < n; j++)
            for (int i = 0; i < n; i++) {
                double s = sin(M_PI * (i + 1) * h) * sin(M_PI * (j + 1) * h) * sin(M_PI * (k + 1) * h);
                f[((size_t)k * n + j) * n + i] = s * g;
            }
}

/* Implicit part f^I(U) = nu L_h U (diffusion, treated implicitly). */
void or_heat_rhs(int n, int order, double nu, double c, double t, const double *u,
                 double *f_impl, double *f_expl)
{
    if (f_impl) or_lap_apply(n, order, 0.0, nu, u, f_impl);
    if (f_expl) or_forcing(n, nu, c, t, f_expl);
}

/* ------------------------------------------------------------------ */
/* SDC (section 1.1, eqs. (5)-(9))                                     */
/* ------------------------------------------------------------------ */

/*
 * Predictor (the paper defers it to its references): copy U_0 to every
 * node and evaluate f^I there.
 */
void or_spread(const or_level *L, double nu, const double *u0, double *U, double *FI)
{
    size_t N = cube(L->n);
    for (int m = 0; m < L->M; m++) {
        memcpy(U + (size_t)m * N, u0, N * sizeof(double));
        or_lap_apply(L->n, L->order, 0.0, nu, u0, FI + (size_t)m * N);
    }
}

/*
 * Collocation residual (eq. (6) moved to one side), max over nodes
 * m = 1..M-1 and grid points of |U_0 + dt sum_j q_{m,j} f(U_j, t_j)
 * (+ tau_m) - U_m|.  Absolute, max norm (the paper does not define the
 * residual it thresholds at 1e-10).
 */
double or_sdc_residual(const or_level *L, double nu, double tn, double dt, double c,
                       const double *U, const double *FI, const double *tau)
{
    int M = L->M;
    size_t N = cube(L->n);
    double Q[OR_MAXM * OR_MAXM], nodes[OR_MAXM];
    or_collocation_matrix(M, Q);
    or_lobatto_nodes(M, nodes);
    double **FE = (double **)malloc(M * sizeof(double *));
    for (int j = 0; j < M; j++) {
        FE[j] = alloc0(N);
        or_forcing(L->n, nu, c, tn + dt * nodes[j], FE[j]);
    }
    double R = 0.0;
    for (int m = 1; m < M; m++)
        for (size_t p = 0; p < N; p++) {
            double integral = 0.0;
            for (int j = 0; j < M; j++)
                integral += Q[m * M + j] * (FI[(size_t)j * N + p] + FE[j][p]);
            double v = U[p] + dt * integral;
            if (tau) v += tau[(size_t)m * N + p];
            v -= U[(size_t)m * N + p];
            double x = fabs(v);
            if (x > R || x != x) R = x;
        }
    for (int j = 0; j < M; j++) free(FE[j]);
    free(FE);
    return R;
}

/*
 * One IMEX-Euler SDC sweep, eq. (7).  With f^I = nu L_h U and f^E = f(x,t)
 * (independent of U), the explicit difference term of eq. (7) vanishes and
 * each substep is
 *   (I - dt_m nu L_h) U^{k+1}_{m+1} = U^{k+1}_m - dt_m nu L_h U^k_{m+1}
 *                                     + dt S^k_m (+ tau_{m+1} - tau_m)
 * with dt S^k_m = dt sum_j (q_{m+1,j} - q_{m,j}) f(U^k_j, t_j) (eq. (8)),
 * built from iterate k before any node is updated.  Each substep is solved
 * by or_mg_solve from the initial guess U^k_{m+1}.  tau (may be NULL) is the
 * FAS correction of a coarse MLSDC level.
 */
int or_sdc_sweep(const or_level *L, const or_mg *mg, double nu, double tn, double dt, double c,
                 double *U, double *FI, const double *tau, or_stats *st)
{
    int M = L->M, n = L->n;
    size_t N = cube(n);
    double Q[OR_MAXM * OR_MAXM], nodes[OR_MAXM];
    or_collocation_matrix(M, Q);
    or_lobatto_nodes(M, nodes);
    double *FE = alloc0((size_t)M * N);
    for (int j = 0; j < M; j++) or_forcing(n, nu, c, tn + dt * nodes[j], FE + (size_t)j * N);
    /* node-to-node integrals from iterate k */
    double *SF = alloc0((size_t)(M - 1) * N);
    for (int m = 0; m < M - 1; m++)
        for (size_t p = 0; p < N; p++) {
            double s = 0.0;
            for (int j = 0; j < M; j++)
                s += (Q[(m + 1) * M + j] - Q[m * M + j]) * (FI[(size_t)j * N + p] + FE[(size_t)j * N + p]);
            SF[(size_t)m * N + p] = dt * s;
        }
    double *rhs = alloc0(N);
    int status = OR_OK;
    for (int m = 0; m < M - 1; m++) {
        double dtm = dt * (nodes[m + 1] - nodes[m]);
        for (size_t p = 0; p < N; p++) {
            double v = U[(size_t)m * N + p] - dtm * FI[(size_t)(m + 1) * N + p] + SF[(size_t)m * N + p];
            if (tau) v += tau[(size_t)(m + 1) * N + p] - tau[(size_t)m * N + p];
            rhs[p] = v;
        }
        int cyc = 0;
        double rho = 0.0;
        int s = or_mg_solve(n, L->order, nu * dtm, mg, U + (size_t)(m + 1) * N, rhs, &cyc, &rho);
        if (s != OR_OK && status == OR_OK) status = s;
        if (st) {
            st->total_solves++;
            st->total_cycles += cyc;
            if (cyc > st->max_cycles_seen) st->max_cycles_seen = cyc;
        }
        or_lap_apply(n, L->order, 0.0, nu, U + (size_t)(m + 1) * N, FI + (size_t)(m + 1) * N);
    }
    if (st) st->total_sweeps++;
    free(FE); free(SF); free(rhs);
    return status;
}

/*
 * One node-parallel SDC sweep -- an addition, not in the paper.  The IMEX
 * sweep of eq. (7) treats the implicit part with the lower-triangular
 * matrix of the implicit-Euler substeps, so its M-1 solves run one after the
 * other.  Replacing that matrix by the diagonal d_m = tau_m (each node an
 * implicit Euler step over [t_0, t_m]) makes the solves independent:
 *   (I - dt tau_m nu L_h) U^{k+1}_m
 *       = U_0 + dt sum_j q_{m,j} f(U^k_j, t_j) - dt tau_m nu L_h U^k_m,
 * m = 1..M-1, every right-hand side built from iterate k, each solved by
 * or_mg_solve from the guess U^k_m; then f^I is recomputed at those nodes.
 * The collocation solution of eq. (6) is still the fixed point: there
 * U_m = U_0 + dt sum_j q_{m,j} f_j, so the right-hand side is
 * (I - dt tau_m nu L_h) U_m.
 */
int or_sdc_sweep_nodes(const or_level *L, const or_mg *mg, double nu, double tn, double dt, double c,
                       double *U, double *FI, or_stats *st)
{
    int M = L->M, n = L->n;
    size_t N = cube(n);
    double Q[OR_MAXM * OR_MAXM], nodes[OR_MAXM];
    or_collocation_matrix(M, Q);
    or_lobatto_nodes(M, nodes);
    double *FE = alloc0((size_t)M * N);
    for (int j = 0; j < M; j++) or_forcing(n, nu, c, tn + dt * nodes[j], FE + (size_t)j * N);
    /* every right-hand side from iterate k, before any node changes */
    double *rhs = alloc0((size_t)(M - 1) * N);
    for (int m = 1; m < M; m++) {
        double dm = dt * nodes[m];
        for (size_t p = 0; p < N; p++) {
            double s = 0.0;
            for (int j = 0; j < M; j++) s += Q[m * M + j] * (FI[(size_t)j * N + p] + FE[(size_t)j * N + p]);
            rhs[(size_t)(m - 1) * N + p] = U[p] + dt * s - dm * FI[(size_t)m * N + p];
        }
    }
    int status = OR_OK;
    for (int m = 1; m < M; m++) {
        int cyc = 0;
        double rho = 0.0;
        int s = or_mg_solve(n, L->order, nu * (dt * nodes[m]), mg, U + (size_t)m * N, rhs + (size_t)(m - 1) * N,
                            &cyc, &rho);
        if (s != OR_OK && status == OR_OK) status = s;
        if (st) {
            st->total_solves++;
            st->total_cycles += cyc;
            if (cyc > st->max_cycles_seen) st->max_cycles_seen = cyc;
        }
    }
    for (int m = 1; m < M; m++) or_lap_apply(n, L->order, 0.0, nu, U + (size_t)m * N, FI + (size_t)m * N);
    if (st) st->total_sweeps++;
    free(FE); free(rhs);
    return status;
}

/*
 * One single-level SDC time step [t_n, t_n + dt] from u (overwritten with
 * the end value U_{M-1}, i.e. the last collocation node, eq. (9)).
 */
static int sdc_step(const or_problem *pb, double tn, double *u, or_stats *st)
{
    const or_level *L = &pb->lev[0];
    size_t N = cube(L->n);
    double *U = alloc0((size_t)L->M * N), *FI = alloc0((size_t)L->M * N);
    or_spread(L, pb->nu, u, U, FI);
    int status = OR_OK, k = 0;
    for (k = 0;; k++) {
        if (pb->sweeps > 0) {
            if (k >= pb->sweeps) break;
        } else {
            double R = or_sdc_residual(L, pb->nu, tn, pb->dt, pb->forcing_c, U, FI, NULL);
            if (st) st->last_residual = R;
            if (R != R) { status = OR_ENONFINITE; break; }
            if (R <= pb->sdc_tol) break;
            if (k >= pb->max_sweeps) { status = OR_ENOCONV; break; }
        }
        int s = pb->node_parallel
                    ? or_sdc_sweep_nodes(L, &pb->mg, pb->nu, tn, pb->dt, pb->forcing_c, U, FI, st)
                    : or_sdc_sweep(L, &pb->mg, pb->nu, tn, pb->dt, pb->forcing_c, U, FI, NULL, st);
        if (s != OR_OK && status == OR_OK) status = s;
    }
    if (pb->sweeps > 0 && st)
        st->last_residual = or_sdc_residual(L, pb->nu, tn, pb->dt, pb->forcing_c, U, FI, NULL);
    if (st) st->sweeps = k;
    memcpy(u, U + (size_t)(L->M - 1) * N, N * sizeof(double));
    free(U); free(FI);
    return status;
}

/* ------------------------------------------------------------------ */
/* SDC with the compact scheme (single level)                          */
/* ------------------------------------------------------------------ */

/*
 * With the compact pair the semi-discrete heat equation is
 *   B_h u' = nu A_h u + B_h f,
 * and the collocation problem (eq. (6)) multiplied by B_h reads
 *   B U_m = B U_0 + dt sum_j q_{m,j} Ft_j,   Ft_j = nu A U_j + B f(t_j).
 * The IMEX sweep (eq. (7)) in this form needs no inverse of B:
 *   (B - dt_m nu A) U^{k+1}_{m+1} = B U^{k+1}_m - dt_m nu A U^k_{m+1} + dt S^k_m,
 *   dt S^k_m = dt sum_j (q_{m+1,j} - q_{m,j}) Ft(U^k_j, t_j),
 * each substep solved by or_mg_solve with the compact operator (multigrid on
 * B - a A, rediscretised on the coarser grids) from the guess U^k_{m+1}.
 * G holds nu A U at every node (Ft without the forcing).  The residual that
 * stops the sweeps is the one of this form, max over m = 1..M-1 and the
 * grid of |B U_0 + dt sum_j q_{m,j} Ft_j - B U_m| (a reading: the paper does
 * not say which residual it thresholds; without B^{-1} it is the one the
 * sweeps can evaluate).
 */
void or_spread_compact(const or_level *L, double nu, const double *u0, double *U, double *G)
{
    size_t N = cube(L->n);
    for (int m = 0; m < L->M; m++) {
        memcpy(U + (size_t)m * N, u0, N * sizeof(double));
        or_compact_apply(L->n, 0.0, nu, u0, G + (size_t)m * N);
    }
}

/* B f(t_j) at every node, the forcing's part of Ft */
static double **compact_forcing(const or_level *L, double nu, double tn, double dt, double c)
{
    int M = L->M;
    size_t N = cube(L->n);
    double nodes[OR_MAXM];
    or_lobatto_nodes(M, nodes);
    double **BF = (double **)malloc(M * sizeof(double *));
    double *f = alloc0(N);
    for (int j = 0; j < M; j++) {
        BF[j] = alloc0(N);
        or_forcing(L->n, nu, c, tn + dt * nodes[j], f);
        or_compact_apply(L->n, 1.0, 0.0, f, BF[j]);
    }
    free(f);
    return BF;
}

static void free_rows(double **r, int M)
{
    for (int j = 0; j < M; j++) free(r[j]);
    free(r);
}

double or_sdc_residual_compact(const or_level *L, double nu, double tn, double dt, double c, const double *U,
                               const double *G)
{
    int M = L->M;
    size_t N = cube(L->n);
    double Q[OR_MAXM * OR_MAXM];
    or_collocation_matrix(M, Q);
    double **BF = compact_forcing(L, nu, tn, dt, c);
    double *BU0 = alloc0(N), *BUm = alloc0(N);
    or_compact_apply(L->n, 1.0, 0.0, U, BU0);
    double R = 0.0;
    for (int m = 1; m < M; m++) {
        or_compact_apply(L->n, 1.0, 0.0, U + (size_t)m * N, BUm);
        for (size_t p = 0; p < N; p++) {
            double integral = 0.0;
            for (int j = 0; j < M; j++) integral += Q[m * M + j] * (G[(size_t)j * N + p] + BF[j][p]);
            double x = fabs((BU0[p] + dt * integral) - BUm[p]);
            if (x > R || x != x) R = x;
        }
    }
    free(BU0); free(BUm);
    free_rows(BF, M);
    return R;
}

int or_sdc_sweep_compact(const or_level *L, const or_mg *mg, double nu, double tn, double dt, double c,
                         double *U, double *G, or_stats *st)
{
    int M = L->M, n = L->n;
    size_t N = cube(n);
    double Q[OR_MAXM * OR_MAXM], nodes[OR_MAXM];
    or_collocation_matrix(M, Q);
    or_lobatto_nodes(M, nodes);
    double **BF = compact_forcing(L, nu, tn, dt, c);
    /* dt S^k_m from iterate k, before any node is updated */
    double *SF = alloc0((size_t)(M - 1) * N);
    for (int m = 0; m + 1 < M; m++)
        for (size_t p = 0; p < N; p++) {
            double s = 0.0;
            for (int j = 0; j < M; j++)
                s += (Q[(m + 1) * M + j] - Q[m * M + j]) * (G[(size_t)j * N + p] + BF[j][p]);
            SF[(size_t)m * N + p] = dt * s;
        }
    double *rhs = alloc0(N), *BUm = alloc0(N);
    int status = OR_OK;
    for (int m = 0; m + 1 < M; m++) {
        double dtm = dt * (nodes[m + 1] - nodes[m]);
        or_compact_apply(n, 1.0, 0.0, U + (size_t)m * N, BUm);
        for (size_t p = 0; p < N; p++)
            rhs[p] = (BUm[p] - dtm * G[(size_t)(m + 1) * N + p]) + SF[(size_t)m * N + p];
        int cycles = 0;
        double rho = 0.0;
        int s = or_mg_solve(n, OR_ORDER_COMPACT, nu * dtm, mg, U + (size_t)(m + 1) * N, rhs, &cycles, &rho);
        if (st) {
            st->total_solves++;
            st->total_cycles += cycles;
            if (cycles > st->max_cycles_seen) st->max_cycles_seen = cycles;
        }
        if (s != OR_OK && status == OR_OK) status = s;
        or_compact_apply(n, 0.0, nu, U + (size_t)(m + 1) * N, G + (size_t)(m + 1) * N);
    }
    if (st) st->total_sweeps++;
    free(rhs); free(BUm); free(SF);
    free_rows(BF, M);
    return status;
}

static int sdc_step_compact(const or_problem *pb, double tn, double *u, or_stats *st)
{
    const or_level *L = &pb->lev[0];
    size_t N = cube(L->n);
    double *U = alloc0((size_t)L->M * N), *G = alloc0((size_t)L->M * N);
    or_spread_compact(L, pb->nu, u, U, G);
    int status = OR_OK, k = 0;
    for (k = 0;; k++) {
        if (pb->sweeps > 0) {
            if (k >= pb->sweeps) break;
        } else {
            double R = or_sdc_residual_compact(L, pb->nu, tn, pb->dt, pb->forcing_c, U, G);
            if (st) st->last_residual = R;
            if (R != R) { status = OR_ENONFINITE; break; }
            if (R <= pb->sdc_tol) break;
            if (k >= pb->max_sweeps) { status = OR_ENOCONV; break; }
        }
        int s = or_sdc_sweep_compact(L, &pb->mg, pb->nu, tn, pb->dt, pb->forcing_c, U, G, st);
        if (s != OR_OK && status == OR_OK) status = s;
    }
    if (pb->sweeps > 0 && st) st->last_residual = or_sdc_residual_compact(L, pb->nu, tn, pb->dt, pb->forcing_c, U, G);
    if (st) st->sweeps = k;
    memcpy(u, U + (size_t)(L->M - 1) * N, N * sizeof(double));
    free(U); free(G);
    return status;
}

/* ------------------------------------------------------------------ */
/* MLSDC with FAS (section 1.1; space-time coarsening in the intro)    */
/* ------------------------------------------------------------------ */

/* Injection: coarse point I takes the fine value at 2I+1. */
void or_inject(int nf, const double *uf, double *uc)
{
    int nc = (nf - 1) / 2;
    for (int K = 0; K < nc; K++)
        for (int J = 0; J < nc; J++)
            for (int I = 0; I < nc; I++)
                uc[((size_t)K * nc + J) * nc + I] =
                    uf[((size_t)(2 * K + 1) * nf + (2 * J + 1)) * nf + (2 * I + 1)];
}

/* index of the fine node that coincides with coarse node m (nested nodes) */
static int fine_node_of(int Mf, int Mc, int m) { return m * ((Mf - 1) / (Mc - 1)); }

/*
 * Restriction to the next coarser MLSDC level plus FAS correction.
 * Ut[m] = inj(Uf[fine node of m]) (space: injection; time: node subset),
 * Uc = Ut, FIc = nu L_c Ut, and
 *   tau_m = inj(dt sum_j qf_{m',j} f^f_j + tauf_{m'}) - dt sum_j qc_{m,j} f^c(Ut_j)
 * where m' is the fine node of coarse node m and tauf (NULL on the finest
 * level) is the fine level's own FAS correction: the coarse problem is the
 * fine level's FAS-corrected collocation problem seen on the coarse nodes and
 * grid, so a restricted fine solution solves it.
 */
void or_fas_restrict_tau(const or_level *Lf, const or_level *Lc, double nu, double tn, double dt,
                         double c, const double *Uf, const double *FIf, const double *tauf, double *Uc,
                         double *FIc, double *Ut, double *tau)
{
    int Mf = Lf->M, Mc = Lc->M, nf = Lf->n, nc = Lc->n;
    size_t Nf = cube(nf), Nc = cube(nc);
    double Qf[OR_MAXM * OR_MAXM], Qc[OR_MAXM * OR_MAXM], tf[OR_MAXM], tc[OR_MAXM];
    or_collocation_matrix(Mf, Qf);
    or_collocation_matrix(Mc, Qc);
    or_lobatto_nodes(Mf, tf);
    or_lobatto_nodes(Mc, tc);
    double *FEf = alloc0((size_t)Mf * Nf), *FEc = alloc0((size_t)Mc * Nc);
    for (int j = 0; j < Mf; j++) or_forcing(nf, nu, c, tn + dt * tf[j], FEf + (size_t)j * Nf);
    for (int j = 0; j < Mc; j++) or_forcing(nc, nu, c, tn + dt * tc[j], FEc + (size_t)j * Nc);
    for (int m = 0; m < Mc; m++) {
        or_inject(nf, Uf + (size_t)fine_node_of(Mf, Mc, m) * Nf, Ut + (size_t)m * Nc);
        memcpy(Uc + (size_t)m * Nc, Ut + (size_t)m * Nc, Nc * sizeof(double));
        or_lap_apply(nc, Lc->order, 0.0, nu, Ut + (size_t)m * Nc, FIc + (size_t)m * Nc);
    }
    double *fint = alloc0(Nf), *cint = alloc0(Nc);
    for (int m = 0; m < Mc; m++) {
        int mf = fine_node_of(Mf, Mc, m);
        for (size_t p = 0; p < Nf; p++) {
            double s = 0.0;
            for (int j = 0; j < Mf; j++)
                s += Qf[mf * Mf + j] * (FIf[(size_t)j * Nf + p] + FEf[(size_t)j * Nf + p]);
            fint[p] = dt * s;
            if (tauf) fint[p] += tauf[(size_t)mf * Nf + p];
        }
        or_inject(nf, fint, cint);
        for (size_t p = 0; p < Nc; p++) {
            double s = 0.0;
            for (int j = 0; j < Mc; j++)
                s += Qc[m * Mc + j] * (FIc[(size_t)j * Nc + p] + FEc[(size_t)j * Nc + p]);
            tau[(size_t)m * Nc + p] = cint[p] - dt * s;
        }
    }
    free(FEf); free(FEc); free(fint); free(cint);
}

/* Restriction from the finest level (no fine FAS correction). */
void or_fas_restrict(const or_level *Lf, const or_level *Lc, double nu, double tn, double dt,
                     double c, const double *Uf, const double *FIf, double *Uc, double *FIc,
                     double *Ut, double *tau)
{
    or_fas_restrict_tau(Lf, Lc, nu, tn, dt, c, Uf, FIf, NULL, Uc, FIc, Ut, tau);
}

/*
 * Interpolation of the coarse correction back to the fine MLSDC level
 * (section 1.1; the paper leaves the transfer operators to its references).
 * dU_m = Uc_m - Ut_m at every coarse node; a fine node coinciding with a
 * coarse node takes P dU, the others take P(sum_j l_j(tau_f) dU_j)
 * (Lagrange in time on the coarse nodes), with P trilinear (interp 1 or 0)
 * or tricubic (interp 3) in space.  Then f^I is recomputed on the fine
 * level at every node.
 */
static void fas_interp_correction(const or_level *Lf, const or_level *Lc, double *Uf, const double *Uc,
                                  const double *Ut, int interp)
{
    int Mf = Lf->M, Mc = Lc->M, nf = Lf->n, nc = Lc->n;
    size_t Nf = cube(nf), Nc = cube(nc);
    double tf[OR_MAXM];
    or_lobatto_nodes(Mf, tf);
    double *dU = alloc0((size_t)Mc * Nc), *ec = alloc0(Nc);
    for (size_t p = 0; p < (size_t)Mc * Nc; p++) dU[p] = Uc[p] - Ut[p];
    for (int mf = 0; mf < Mf; mf++) {
        double w[OR_MAXM];
        interp_weights(Mc, tf[mf], w);
        int stride = (Mf - 1) / (Mc - 1);
        if (mf % stride == 0) {
            memcpy(ec, dU + (size_t)(mf / stride) * Nc, Nc * sizeof(double));
        } else {
            for (size_t p = 0; p < Nc; p++) {
                double s = 0.0;
                for (int j = 0; j < Mc; j++) s += w[j] * dU[(size_t)j * Nc + p];
                ec[p] = s;
            }
        }
        if (interp == 3) or_prolong_add_cubic(nc, ec, Uf + (size_t)mf * Nf);
        else or_prolong_add(nc, ec, Uf + (size_t)mf * Nf);
    }
    free(dU); free(ec);
}

void or_fas_interp(const or_level *Lf, const or_level *Lc, double nu, double *Uf, double *FIf,
                   const double *Uc, const double *Ut, int interp)
{
    size_t Nf = cube(Lf->n);
    fas_interp_correction(Lf, Lc, Uf, Uc, Ut, interp);
    for (int mf = 0; mf < Lf->M; mf++)
        or_lap_apply(Lf->n, Lf->order, 0.0, nu, Uf + (size_t)mf * Nf, FIf + (size_t)mf * Nf);
}

/* Node arrays of every MLSDC level of one time step (Ut, tau: levels >= 1). */
typedef struct {
    double *U[OR_MAXLEV], *FI[OR_MAXLEV], *Ut[OR_MAXLEV], *tau[OR_MAXLEV];
} or_hier;

static int hier_alloc(const or_problem *pb, or_hier *H)
{
    memset(H, 0, sizeof(*H));
    for (int l = 0; l < pb->nlevels; l++) {
        size_t S = (size_t)pb->lev[l].M * cube(pb->lev[l].n);
        H->U[l] = alloc0(S);
        H->FI[l] = alloc0(S);
        if (l > 0) {
            H->Ut[l] = alloc0(S);
            H->tau[l] = alloc0(S);
        }
    }
    return OR_OK;
}

static void hier_free(const or_problem *pb, or_hier *H)
{
    for (int l = 0; l < pb->nlevels; l++) {
        free(H->U[l]); free(H->FI[l]); free(H->Ut[l]); free(H->tau[l]);
    }
}

/* Restriction + FAS correction from level l to level l + 1. */
static void restrict_level(const or_problem *pb, int l, double tn, or_hier *H)
{
    or_fas_restrict_tau(&pb->lev[l], &pb->lev[l + 1], pb->nu, tn, pb->dt, pb->forcing_c, H->U[l], H->FI[l],
                        l > 0 ? H->tau[l] : NULL, H->U[l + 1], H->FI[l + 1], H->Ut[l + 1], H->tau[l + 1]);
}

/* Interpolation of level l + 1's correction to level l. */
static void interp_level(const or_problem *pb, int l, or_hier *H)
{
    or_fas_interp(&pb->lev[l], &pb->lev[l + 1], pb->nu, H->U[l], H->FI[l], H->U[l + 1], H->Ut[l + 1],
                  pb->fas_interp);
}

/*
 * One MLSDC iteration over the nlevels levels (section 1.1: sweeps on a
 * hierarchy of levels with fewer nodes and points, tied together by the FAS
 * correction), as a V-cycle:
 *   down: sweep on level 0; for l = 0 .. L-2: restriction + FAS correction
 *         to level l+1, then a sweep there (with its tau);
 *   up:   for l = L-2 .. 0: interpolation of level l+1's correction to level
 *         l, then, on the levels between the finest and the coarsest, a
 *         further sweep (with their tau); no closing sweep on level 0.
 * With two levels this is fine sweep, restriction, coarse sweep,
 * interpolation.  The sweep on an intermediate level on the way up is a
 * reading (the paper defers the details of MLSDC to its references).
 */
static int mlsdc_vcycle(const or_problem *pb, double tn, or_hier *H, or_stats *st)
{
    const int L = pb->nlevels;
    int status = or_sdc_sweep(&pb->lev[0], &pb->mg, pb->nu, tn, pb->dt, pb->forcing_c, H->U[0], H->FI[0], NULL, st);
    for (int l = 0; l + 1 < L; l++) {
        restrict_level(pb, l, tn, H);
        int s = or_sdc_sweep(&pb->lev[l + 1], &pb->mg, pb->nu, tn, pb->dt, pb->forcing_c, H->U[l + 1],
                             H->FI[l + 1], H->tau[l + 1], NULL);
        if (s != OR_OK && status == OR_OK) status = s;
    }
    for (int l = L - 2; l >= 0; l--) {
        interp_level(pb, l, H);
        if (l > 0) {
            int s = or_sdc_sweep(&pb->lev[l], &pb->mg, pb->nu, tn, pb->dt, pb->forcing_c, H->U[l], H->FI[l],
                                 H->tau[l], NULL);
            if (s != OR_OK && status == OR_OK) status = s;
        }
    }
    return status;
}

/*
 * One two-level MLSDC iteration on caller arrays: fine sweep, restriction +
 * FAS correction, coarse sweep with tau, interpolation of the coarse
 * correction (mlsdc_vcycle with two levels).
 */
int or_mlsdc_iter(const or_problem *pb, double tn, double *Uf, double *FIf, double *Uc,
                  double *FIc, double *Ut, double *tau, or_stats *st)
{
    if (pb->nlevels != 2 || pb->lev[0].order == OR_ORDER_COMPACT) return OR_EINVAL;
    or_hier H;
    memset(&H, 0, sizeof(H));
    H.U[0] = Uf; H.FI[0] = FIf;
    H.U[1] = Uc; H.FI[1] = FIc; H.Ut[1] = Ut; H.tau[1] = tau;
    return mlsdc_vcycle(pb, tn, &H, st);
}

static int mlsdc_step(const or_problem *pb, double tn, double *u, or_stats *st)
{
    const or_level *Lf = &pb->lev[0];
    size_t Nf = cube(Lf->n);
    or_hier H;
    hier_alloc(pb, &H);
    or_spread(Lf, pb->nu, u, H.U[0], H.FI[0]);
    int status = OR_OK, k;
    for (k = 0;; k++) {
        if (pb->sweeps > 0) {
            if (k >= pb->sweeps) break;
        } else {
            double R = or_sdc_residual(Lf, pb->nu, tn, pb->dt, pb->forcing_c, H.U[0], H.FI[0], NULL);
            if (st) st->last_residual = R;
            if (R != R) { status = OR_ENONFINITE; break; }
            if (R <= pb->sdc_tol) break;
            if (k >= pb->max_sweeps) { status = OR_ENOCONV; break; }
        }
        int s = mlsdc_vcycle(pb, tn, &H, st);
        if (s != OR_OK && status == OR_OK) status = s;
    }
    if (pb->sweeps > 0 && st)
        st->last_residual = or_sdc_residual(Lf, pb->nu, tn, pb->dt, pb->forcing_c, H.U[0], H.FI[0], NULL);
    if (st) st->sweeps = k;
    memcpy(u, H.U[0] + (size_t)(Lf->M - 1) * Nf, Nf * sizeof(double));
    hier_free(pb, &H);
    return status;
}

/*
 * Two-level MLSDC with the compact scheme on the fine level (a reading:
 * sec. 1.2 has B_h inverted for the FAS correction).  The fine sweeps are
 * the B-weighted ones (G = nu A_h U at the nodes); the FAS restriction needs
 * the fine integral in the plain form, whose implicit part is
 * f^I = nu B_h^{-1} A_h U = B_h^{-1} G, so FIf is formed from G by the exact
 * inverse first.  Coarse sweep and interpolation as for the other schemes;
 * after the interpolation G is recomputed.  One iteration on caller arrays:
 * Uf, G [Mf][Nf]; FIf [Mf][Nf] scratch for B^{-1} G; coarse as or_mlsdc_iter.
 */
int or_mlsdc_iter_compact(const or_problem *pb, double tn, double *Uf, double *G, double *FIf, double *Uc,
                          double *FIc, double *Ut, double *tau, or_stats *st)
{
    if (pb->nlevels != 2 || pb->lev[0].order != OR_ORDER_COMPACT) return OR_EINVAL;
    const or_level *Lf = &pb->lev[0], *Lc = &pb->lev[1];
    size_t Nf = cube(Lf->n);
    int status = or_sdc_sweep_compact(Lf, &pb->mg, pb->nu, tn, pb->dt, pb->forcing_c, Uf, G, st);
    for (int j = 0; j < Lf->M; j++) or_compact_binv(Lf->n, G + (size_t)j * Nf, FIf + (size_t)j * Nf);
    or_fas_restrict(Lf, Lc, pb->nu, tn, pb->dt, pb->forcing_c, Uf, FIf, Uc, FIc, Ut, tau);
    int s = or_sdc_sweep(Lc, &pb->mg, pb->nu, tn, pb->dt, pb->forcing_c, Uc, FIc, tau, NULL);
    if (s != OR_OK && status == OR_OK) status = s;
    fas_interp_correction(Lf, Lc, Uf, Uc, Ut, pb->fas_interp);
    for (int j = 0; j < Lf->M; j++) or_compact_apply(Lf->n, 0.0, pb->nu, Uf + (size_t)j * Nf, G + (size_t)j * Nf);
    return status;
}

static int mlsdc_step_compact(const or_problem *pb, double tn, double *u, or_stats *st)
{
    const or_level *Lf = &pb->lev[0];
    size_t Nf = cube(Lf->n);
    or_hier H;
    hier_alloc(pb, &H);
    double *G = alloc0((size_t)Lf->M * Nf);
    or_spread_compact(Lf, pb->nu, u, H.U[0], G);
    int status = OR_OK, k;
    for (k = 0;; k++) {
        if (pb->sweeps > 0) {
            if (k >= pb->sweeps) break;
        } else {
            double R = or_sdc_residual_compact(Lf, pb->nu, tn, pb->dt, pb->forcing_c, H.U[0], G);
            if (st) st->last_residual = R;
            if (R != R) { status = OR_ENONFINITE; break; }
            if (R <= pb->sdc_tol) break;
            if (k >= pb->max_sweeps) { status = OR_ENOCONV; break; }
        }
        int s = or_mlsdc_iter_compact(pb, tn, H.U[0], G, H.FI[0], H.U[1], H.FI[1], H.Ut[1], H.tau[1], st);
        if (s != OR_OK && status == OR_OK) status = s;
    }
    if (pb->sweeps > 0 && st)
        st->last_residual = or_sdc_residual_compact(Lf, pb->nu, tn, pb->dt, pb->forcing_c, H.U[0], G);
    if (st) st->sweeps = k;
    memcpy(u, H.U[0] + (size_t)(Lf->M - 1) * Nf, Nf * sizeof(double));
    free(G);
    hier_free(pb, &H);
    return status;
}

static int check_problem(const or_problem *pb)
{
    if (pb->nlevels < 1 || pb->nlevels > OR_MAXLEV) return OR_EINVAL;
    for (int l = 0; l < pb->nlevels; l++) {
        const or_level *L = &pb->lev[l];
        if (!valid_n(L->n) || (L->order != 2 && L->order != 4 && L->order != OR_ORDER_COMPACT)) return OR_EINVAL;
        if (L->order == OR_ORDER_COMPACT && (l != 0 || pb->nlevels > 2 || pb->node_parallel)) return OR_EINVAL;
        if (L->M < 2 || L->M > OR_MAXM) return OR_EINVAL;
    }
    for (int l = 1; l < pb->nlevels; l++) {
        if (pb->lev[l - 1].n < 3 || pb->lev[l].n != (pb->lev[l - 1].n - 1) / 2) return OR_EINVAL;
        if ((pb->lev[l - 1].M - 1) % (pb->lev[l].M - 1) != 0) return OR_EINVAL;
    }
    if (!(pb->dt > 0.0) || !(pb->nu > 0.0) || pb->nsteps < 0) return OR_EINVAL;
    if (pb->node_parallel != 0 && (pb->node_parallel != 1 || pb->nlevels != 1)) return OR_EINVAL;
    if (pb->fas_interp != 0 && pb->fas_interp != 1 && pb->fas_interp != 3) return OR_EINVAL;
    return OR_OK;
}

/*
 * Run nsteps time steps from u (overwritten with the final value), single
 * level SDC or MLSDC over 2 or 3 levels depending on nlevels.  t_n = t0 + n dt.
 */
int or_run(const or_problem *pb, double *u, or_stats *st)
{
    int s = check_problem(pb);
    if (s != OR_OK) return s;
    if (st) memset(st, 0, sizeof(*st));
    int status = OR_OK;
    for (int step = 0; step < pb->nsteps; step++) {
        double tn = pb->t0 + step * pb->dt;
        const int cmp = pb->lev[0].order == OR_ORDER_COMPACT;
        s = pb->nlevels > 1 ? (cmp ? mlsdc_step_compact(pb, tn, u, st) : mlsdc_step(pb, tn, u, st))
            : cmp ? sdc_step_compact(pb, tn, u, st) : sdc_step(pb, tn, u, st);
        if (s != OR_OK && status == OR_OK) status = s;
    }
    if (st) st->status = status;
    return status;
}

/* ------------------------------------------------------------------ */
/* PFASST over P time slices (section 1.1), run serially               */
/* ------------------------------------------------------------------ */

/*
 * The paper gives PFASST only in outline (MLSDC iterations run
 * concurrently on P time slices; new values are passed forward after each
 * level's sweep; the coarse level hands over in a blocking pipeline).  This
 * is the reading used, one block of P consecutive steps starting at t0 from
 * u:
 *  - every slice starts with u spread over all of its fine nodes;
 *  - optional coarse predictor (pred_sweeps > 0; also a reading: the paper
 *    leaves PFASST's start to its references and notes that early
 *    iterations on later slices start from inaccurate values): the coarsest
 *    level is run serially through the slices without the FAS correction.
 *    Slice p restricts its fine values down to the coarsest level; for
 *    p >= 1 its coarsest nodes all take the coarsest end value of slice p-1
 *    (spread, as a time step starts); then pred_sweeps coarse sweeps.  Every
 *    slice then interpolates its coarse correction (node 0 included) level
 *    by level to the finest level, without sweeps in between.  The coarse
 *    values this leaves are those of a serial coarse SDC run over the P
 *    steps with pred_sweeps sweeps each;
 *  - iteration: (i) for p >= 1, fine node 0 of slice p takes the fine end
 *    value of slice p-1 as it stood at the end of the previous iteration
 *    (the predictor's result before the first) -- parity unpinned: no pin
 *    distinguishes this timing from taking the end value of the current
 *    iteration; fine sweep on every slice;
 *    (ii) restriction + tau on every slice, level by level down to the
 *    coarsest, with a sweep on every slice of each intermediate level;
 *    (iii) slices in order p = 0..P-1: for p >= 1 coarse node 0 takes the
 *    coarse end value slice p-1 has just computed, then the coarse sweep;
 *    (iv) interpolation on every slice, node 0 included, level by level up
 *    to the finest, with a sweep on every slice of each intermediate level
 *    (three levels: the same V-cycle as mlsdc_vcycle; an intermediate
 *    level's node 0 is the restriction of the fine one, it has no hand-off
 *    of its own);
 *  - pb->sweeps > 0: exactly that many iterations.  pb->sweeps == 0: after
 *    the fine hand-off of every iteration the collocation residual of every
 *    slice is taken (eq. (6) moved to one side, max norm, absolute, as in
 *    or_sdc_residual); the iteration stops when the largest is at most
 *    pb->sdc_tol (section 2 thresholds the residual of the PFASST
 *    iterations) and fails with OR_ENOCONV after pb->max_sweeps iterations;
 *  - the result is the fine end value of slice P-1.
 * nsteps must be a multiple of P; blocks run one after the other.
 * st->sweeps: iterations of the last block.
 */
int or_pfasst(const or_problem *pb, int P, int pred_sweeps, double *u, or_stats *st)
{
    int s = check_problem(pb);
    if (s != OR_OK) return s;
    if (pb->nlevels < 2 || P < 1 || pb->nsteps % P != 0 || pb->sweeps < 0 || pred_sweeps < 0 ||
        pb->lev[0].order == OR_ORDER_COMPACT)
        return OR_EINVAL;
    const int NL = pb->nlevels, C = NL - 1;   /* C: the coarsest level */
    const or_level *Lf = &pb->lev[0], *Lc = &pb->lev[C];
    int Mf = Lf->M, Mc = Lc->M, nf = Lf->n, nc = Lc->n;
    size_t Nf = cube(nf), Nc = cube(nc);
    or_hier *H = (or_hier *)calloc((size_t)P, sizeof(or_hier));
    for (int p = 0; p < P; p++) hier_alloc(pb, &H[p]);
    double *ends = alloc0((size_t)P * Nf);
    if (st) memset(st, 0, sizeof(*st));
    int status = OR_OK, k = 0;
    for (int blk = 0; blk < pb->nsteps / P; blk++) {
        double tb = pb->t0 + (double)(blk * P) * pb->dt;
        for (int p = 0; p < P; p++) or_spread(Lf, pb->nu, u, H[p].U[0], H[p].FI[0]);
        if (pred_sweeps > 0) {
            for (int p = 0; p < P; p++) {
                double tn = tb + p * pb->dt;
                for (int l = 0; l < C; l++) restrict_level(pb, l, tn, &H[p]);
                if (p >= 1) {
                    /* the coarse step starts from slice p-1's end value, spread */
                    memcpy(ends, H[p - 1].U[C] + (size_t)(Mc - 1) * Nc, Nc * sizeof(double));
                    or_spread(Lc, pb->nu, ends, H[p].U[C], H[p].FI[C]);
                }
                for (int j = 0; j < pred_sweeps; j++) {
                    s = or_sdc_sweep(Lc, &pb->mg, pb->nu, tn, pb->dt, pb->forcing_c, H[p].U[C], H[p].FI[C],
                                     NULL, NULL);
                    if (s != OR_OK && status == OR_OK) status = s;
                }
            }
            for (int p = 0; p < P; p++)
                for (int l = C - 1; l >= 0; l--) interp_level(pb, l, &H[p]);
        }
        for (k = 0;; k++) {
            if (pb->sweeps > 0 && k >= pb->sweeps) break;
            /* (i) fine hand-off from the previous iteration's end values */
            for (int p = 0; p < P; p++)
                memcpy(ends + (size_t)p * Nf, H[p].U[0] + (size_t)(Mf - 1) * Nf, Nf * sizeof(double));
            for (int p = 1; p < P; p++) {
                memcpy(H[p].U[0], ends + (size_t)(p - 1) * Nf, Nf * sizeof(double));
                or_lap_apply(nf, Lf->order, 0.0, pb->nu, H[p].U[0], H[p].FI[0]);
            }
            if (pb->sweeps == 0) {
                double R = 0.0;
                for (int p = 0; p < P; p++) {
                    double r = or_sdc_residual(Lf, pb->nu, tb + p * pb->dt, pb->dt, pb->forcing_c, H[p].U[0],
                                               H[p].FI[0], NULL);
                    if (r > R || r != r) R = r;
                }
                if (st) st->last_residual = R;
                if (R != R) { if (status == OR_OK) status = OR_ENONFINITE; break; }
                if (R <= pb->sdc_tol) break;
                if (k >= pb->max_sweeps) { if (status == OR_OK) status = OR_ENOCONV; break; }
            }
            for (int p = 0; p < P; p++) {
                double tn = tb + p * pb->dt;
                s = or_sdc_sweep(Lf, &pb->mg, pb->nu, tn, pb->dt, pb->forcing_c, H[p].U[0], H[p].FI[0], NULL, st);
                if (s != OR_OK && status == OR_OK) status = s;
            }
            /* (ii) restriction and tau down to the coarsest level, with a sweep
               on every intermediate level on the way */
            for (int l = 0; l < C; l++)
                for (int p = 0; p < P; p++) {
                    double tn = tb + p * pb->dt;
                    restrict_level(pb, l, tn, &H[p]);
                    if (l + 1 < C) {
                        s = or_sdc_sweep(&pb->lev[l + 1], &pb->mg, pb->nu, tn, pb->dt, pb->forcing_c,
                                         H[p].U[l + 1], H[p].FI[l + 1], H[p].tau[l + 1], NULL);
                        if (s != OR_OK && status == OR_OK) status = s;
                    }
                }
            /* (iii) coarse pipeline */
            for (int p = 0; p < P; p++) {
                double tn = tb + p * pb->dt;
                if (p >= 1) {
                    memcpy(H[p].U[C], H[p - 1].U[C] + (size_t)(Mc - 1) * Nc, Nc * sizeof(double));
                    or_lap_apply(nc, Lc->order, 0.0, pb->nu, H[p].U[C], H[p].FI[C]);
                }
                s = or_sdc_sweep(Lc, &pb->mg, pb->nu, tn, pb->dt, pb->forcing_c, H[p].U[C], H[p].FI[C],
                                 H[p].tau[C], NULL);
                if (s != OR_OK && status == OR_OK) status = s;
            }
            /* (iv) interpolation up to the finest level, node 0 included, with a
               sweep on every intermediate level on the way */
            for (int l = C - 1; l >= 0; l--)
                for (int p = 0; p < P; p++) {
                    interp_level(pb, l, &H[p]);
                    if (l > 0) {
                        s = or_sdc_sweep(&pb->lev[l], &pb->mg, pb->nu, tb + p * pb->dt, pb->dt, pb->forcing_c,
                                         H[p].U[l], H[p].FI[l], H[p].tau[l], NULL);
                        if (s != OR_OK && status == OR_OK) status = s;
                    }
                }
        }
        memcpy(u, H[P - 1].U[0] + (size_t)(Mf - 1) * Nf, Nf * sizeof(double));
    }
    if (st) { st->status = status; st->sweeps = k; }
    for (int p = 0; p < P; p++) hier_free(pb, &H[p]);
    free(H); free(ends);
    return status;
}

/* PFASST with fixed iterations and no predictor (see or_pfasst). */
int or_pfasst_run(const or_problem *pb, int P, double *u, or_stats *st)
{
    if (pb->sweeps <= 0) return OR_EINVAL;
    return or_pfasst(pb, P, 0, u, st);
}
