/*
 * picoracle.c -- plain, slow, FP64 CPU oracle for the per-box particle-in-cell
 * step and the load-balancing arithmetic studied in Rowan et al., "In-Situ
 * Assessment of Device-Side Compute Work for Dynamic Load Balancing in a
 * GPU-Accelerated PIC Code" (arXiv 2104.11385).
 *
 * THIS FILE IS TEST INFRASTRUCTURE.  Only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark load it.  It shares no code, header,
 * table or constant with the HIP library; the product path never calls it.
 *
 * The paper states the PIC method only in words (Sec. 2.1: explicit Maxwell
 * time steps, markers moved by the Lorentz force, charged currents deposited
 * back to the grid, following Birdsall & Langdon) and names an FDTD solver and
 * third-order shapes (Sec. 3.1 and the footnote on heuristic weights).  The
 * numerical pieces below therefore follow the published methods those words
 * point to; every function names its source:
 *   - B-spline particle shapes of order 1..3;
 *   - Yee (1966) staggered grid and leapfrog curl update;
 *   - relativistic Boris rotation (Boris 1970, as given by Birdsall & Langdon);
 *   - charge-conserving current deposition of Esirkepov (2001).
 * The load-balancing part (Sec. 2.2, Eq. 1) is the paper's own.
 *
 * Units: c = eps0 = mu0 = 1, cell size 1 in every dimension, time in cell/c.
 * Field arrays are [9][nz][ny][nx] (x fastest), component order
 * Ex Ey Ez Bx By Bz Jx Jy Jz.  Yee locations of element [k][j][i]:
 *   Ex (i+1/2, j, k)      Ey (i, j+1/2, k)      Ez (i, j, k+1/2)
 *   Bx (i, j+1/2, k+1/2)  By (i+1/2, j, k+1/2)  Bz (i+1/2, j+1/2, k)
 *   J is co-located with E; charge density rho sits on nodes (i, j, k).
 * Particles: x and u are [np][3]; u is gamma*v (units of c).  Positions are
 * global and periodic in [0, n_d).
 *
 * Compile with -ffp-contract=off: the load-balancing results are compared
 * bit for bit and must not depend on fused multiply-adds.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NCOMP 9

/* ------------------------------------------------------------------------ */
/* Shapes                                                                    */
/* ------------------------------------------------------------------------ */

/* Centred B-spline of order m evaluated at distance d from a node:
 *   m=1: 1-|d|                                   (|d| < 1)
 *   m=2: 3/4-d^2 (|d|<=1/2),  (3/2-|d|)^2/2       (1/2 < |d| < 3/2)
 *   m=3: 2/3-d^2+|d|^3/2 (|d|<1), (2-|d|)^3/6     (1 <= |d| < 2)        */
double orc_shape(int m, double d)
{
    double a = fabs(d);
    if (m == 1)
        return a < 1.0 ? 1.0 - a : 0.0;
    if (m == 2) {
        if (a <= 0.5) return 0.75 - a * a;
        if (a < 1.5) { double t = 1.5 - a; return 0.5 * t * t; }
        return 0.0;
    }
    if (m == 3) {
        if (a < 1.0) return 2.0 / 3.0 - a * a + 0.5 * a * a * a;
        if (a < 2.0) { double t = 2.0 - a; return t * t * t / 6.0; }
        return 0.0;
    }
    return 0.0;
}

/* First node of the (m+1)-node stencil that covers coordinate xi. */
int64_t orc_first_node(int m, double xi)
{
    if (m == 2) return (int64_t)floor(xi + 0.5) - 1;
    if (m == 3) return (int64_t)floor(xi) - 1;
    return (int64_t)floor(xi);
}

static int64_t wrapi(int64_t i, int64_t n)
{
    int64_t r = i % n;
    return r < 0 ? r + n : r;
}

static size_t at(const int64_t n[3], int64_t i, int64_t j, int64_t k)
{
    return (size_t)(wrapi(i, n[0]) + n[0] * (wrapi(j, n[1]) + n[1] * wrapi(k, n[2])));
}

/* ------------------------------------------------------------------------ */
/* Field gather at the Yee stagger of each component                          */
/* ------------------------------------------------------------------------ */

/* Stagger offsets (in cells) of Ex Ey Ez Bx By Bz. */
static const double STAGGER[6][3] = {
    {0.5, 0.0, 0.0}, {0.0, 0.5, 0.0}, {0.0, 0.0, 0.5},
    {0.0, 0.5, 0.5}, {0.5, 0.0, 0.5}, {0.5, 0.5, 0.0},
};

/* EB[c] = sum over the stencil of S(x-s_x-i) S(y-s_y-j) S(z-s_z-k) F_c[i,j,k],
 * where s is the component's stagger: the same order-m spline for every
 * component, no reduced-order (Galerkin) variant. */
void orc_gather(int m, const int64_t n[3], const double *F, const double x[3], double EB[6])
{
    size_t N = (size_t)(n[0] * n[1] * n[2]);
    for (int c = 0; c < 6; ++c) {
        int64_t g[3];
        double wt[3][4];
        for (int d = 0; d < 3; ++d) {
            double xi = x[d] - STAGGER[c][d];
            g[d] = orc_first_node(m, xi);
            for (int a = 0; a <= m; ++a)
                wt[d][a] = orc_shape(m, xi - (double)(g[d] + a));
        }
        const double *Fc = F + (size_t)c * N;
        double sum = 0.0;
        for (int kk = 0; kk <= m; ++kk)
            for (int jj = 0; jj <= m; ++jj)
                for (int ii = 0; ii <= m; ++ii)
                    sum += wt[0][ii] * wt[1][jj] * wt[2][kk] *
                           Fc[at(n, g[0] + ii, g[1] + jj, g[2] + kk)];
        EB[c] = sum;
    }
}

/* ------------------------------------------------------------------------ */
/* Relativistic Boris push (Boris 1970; Birdsall & Langdon 1985)              */
/* ------------------------------------------------------------------------ */

/* u holds u^{n-1/2} on entry and u^{n+1/2} on return.  h = q dt / (2 m):
 *   u-  = u + h E
 *   t   = h B / gamma(u-),   s = 2 t / (1 + |t|^2)
 *   u'  = u- + u- x t,       u+ = u- + u' x s
 *   u   = u+ + h E                                                         */
void orc_boris(double q, double mass, double dt, const double E[3], const double B[3], double u[3])
{
    double h = q * dt / (2.0 * mass);
    double um[3] = {u[0] + h * E[0], u[1] + h * E[1], u[2] + h * E[2]};
    double gm = sqrt(1.0 + um[0] * um[0] + um[1] * um[1] + um[2] * um[2]);
    double t[3] = {h * B[0] / gm, h * B[1] / gm, h * B[2] / gm};
    double t2 = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
    double s[3] = {2.0 * t[0] / (1.0 + t2), 2.0 * t[1] / (1.0 + t2), 2.0 * t[2] / (1.0 + t2)};
    double up[3] = {um[0] + (um[1] * t[2] - um[2] * t[1]),
                    um[1] + (um[2] * t[0] - um[0] * t[2]),
                    um[2] + (um[0] * t[1] - um[1] * t[0])};
    double upl[3] = {um[0] + (up[1] * s[2] - up[2] * s[1]),
                     um[1] + (up[2] * s[0] - up[0] * s[2]),
                     um[2] + (up[0] * s[1] - up[1] * s[0])};
    u[0] = upl[0] + h * E[0];
    u[1] = upl[1] + h * E[1];
    u[2] = upl[2] + h * E[2];
}

/* ------------------------------------------------------------------------ */
/* Esirkepov (2001) charge-conserving current deposition                      */
/* ------------------------------------------------------------------------ */

/* Adds the current of one macro-particle of charge q*w that moves from x0 to
 * x1 (unwrapped; |x1-x0| < 1 per dimension) during dt.  In each dimension a
 * window of m+3 nodes starts one node below the first node of the order-m
 * node-centred stencil at x0, and holds S0 = S(x0 - node), S1 = S(x1 - node),
 * D = S1 - S0.  The density-decomposition weights are
 *   Wx[a,b,c] = Dx[a] (S0y S0z + Dy S0z/2 + S0y Dz/2 + Dy Dz/3)[b,c]
 * (Wy, Wz by permutation), and the face currents are the running sums
 *   Jx[o+a, b, c] += -(q w / dt) sum_{a' <= a} Wx[a', b, c],  a = 0..m+1,
 * likewise along y for Jy and along z for Jz.  The window's last running sum
 * is zero in exact arithmetic and is not deposited. */
void orc_deposit(int m, const int64_t n[3], double qw, double dt,
                 const double x0[3], const double x1[3], double *J)
{
    int L = m + 3;
    int64_t o[3];
    double S0[3][6], D[3][6];
    for (int d = 0; d < 3; ++d) {
        o[d] = orc_first_node(m, x0[d]) - 1;
        for (int a = 0; a < L; ++a) {
            double node = (double)(o[d] + a);
            S0[d][a] = orc_shape(m, x0[d] - node);
            D[d][a] = orc_shape(m, x1[d] - node) - S0[d][a];
        }
    }
    size_t N = (size_t)(n[0] * n[1] * n[2]);
    double *Jx = J, *Jy = J + N, *Jz = J + 2 * N;
    double coef = -qw / dt;
    const double third = 1.0 / 3.0;

    /* Jx: running sum along x */
    for (int c = 0; c < L; ++c)
        for (int b = 0; b < L; ++b) {
            double acc = 0.0;
            for (int a = 0; a < L - 1; ++a) {
                acc += D[0][a] * (S0[1][b] * S0[2][c] + 0.5 * D[1][b] * S0[2][c] +
                                  0.5 * S0[1][b] * D[2][c] + third * D[1][b] * D[2][c]);
                Jx[at(n, o[0] + a, o[1] + b, o[2] + c)] += coef * acc;
            }
        }
    /* Jy: running sum along y */
    for (int c = 0; c < L; ++c)
        for (int a = 0; a < L; ++a) {
            double acc = 0.0;
            for (int b = 0; b < L - 1; ++b) {
                acc += D[1][b] * (S0[0][a] * S0[2][c] + 0.5 * D[0][a] * S0[2][c] +
                                  0.5 * S0[0][a] * D[2][c] + third * D[0][a] * D[2][c]);
                Jy[at(n, o[0] + a, o[1] + b, o[2] + c)] += coef * acc;
            }
        }
    /* Jz: running sum along z */
    for (int b = 0; b < L; ++b)
        for (int a = 0; a < L; ++a) {
            double acc = 0.0;
            for (int c = 0; c < L - 1; ++c) {
                acc += D[2][c] * (S0[0][a] * S0[1][b] + 0.5 * D[0][a] * S0[1][b] +
                                  0.5 * S0[0][a] * D[1][b] + third * D[0][a] * D[1][b]);
                Jz[at(n, o[0] + a, o[1] + b, o[2] + c)] += coef * acc;
            }
        }
}

/* Node charge density rho[i,j,k] = sum_p q w S(x-i) S(y-j) S(z-k). */
void orc_rho(int m, const int64_t n[3], int64_t np, const double *x, const double *w,
             const int32_t *sp, const double *q, double *rho)
{
    size_t N = (size_t)(n[0] * n[1] * n[2]);
    memset(rho, 0, N * sizeof(double));
    for (int64_t p = 0; p < np; ++p) {
        int64_t g[3];
        double wt[3][4];
        for (int d = 0; d < 3; ++d) {
            g[d] = orc_first_node(m, x[3 * p + d]);
            for (int a = 0; a <= m; ++a)
                wt[d][a] = orc_shape(m, x[3 * p + d] - (double)(g[d] + a));
        }
        double qw = q[sp[p]] * w[p];
        for (int kk = 0; kk <= m; ++kk)
            for (int jj = 0; jj <= m; ++jj)
                for (int ii = 0; ii <= m; ++ii)
                    rho[at(n, g[0] + ii, g[1] + jj, g[2] + kk)] += qw * wt[0][ii] * wt[1][jj] * wt[2][kk];
    }
}

/* ------------------------------------------------------------------------ */
/* Yee (1966) FDTD update                                                    */
/* ------------------------------------------------------------------------ */

static void half_b(const int64_t n[3], double hdt, double *F)
{
    size_t N = (size_t)(n[0] * n[1] * n[2]);
    const double *Ex = F, *Ey = F + N, *Ez = F + 2 * N;
    double *Bx = F + 3 * N, *By = F + 4 * N, *Bz = F + 5 * N;
    for (int64_t k = 0; k < n[2]; ++k)
        for (int64_t j = 0; j < n[1]; ++j)
            for (int64_t i = 0; i < n[0]; ++i) {
                size_t c = at(n, i, j, k);
                double cx = (Ez[at(n, i, j + 1, k)] - Ez[c]) - (Ey[at(n, i, j, k + 1)] - Ey[c]);
                double cy = (Ex[at(n, i, j, k + 1)] - Ex[c]) - (Ez[at(n, i + 1, j, k)] - Ez[c]);
                double cz = (Ey[at(n, i + 1, j, k)] - Ey[c]) - (Ex[at(n, i, j + 1, k)] - Ex[c]);
                Bx[c] -= hdt * cx;
                By[c] -= hdt * cy;
                Bz[c] -= hdt * cz;
            }
}

static void full_e(const int64_t n[3], double dt, double *F)
{
    size_t N = (size_t)(n[0] * n[1] * n[2]);
    double *Ex = F, *Ey = F + N, *Ez = F + 2 * N;
    const double *Bx = F + 3 * N, *By = F + 4 * N, *Bz = F + 5 * N;
    const double *Jx = F + 6 * N, *Jy = F + 7 * N, *Jz = F + 8 * N;
    for (int64_t k = 0; k < n[2]; ++k)
        for (int64_t j = 0; j < n[1]; ++j)
            for (int64_t i = 0; i < n[0]; ++i) {
                size_t c = at(n, i, j, k);
                double cx = (Bz[c] - Bz[at(n, i, j - 1, k)]) - (By[c] - By[at(n, i, j, k - 1)]);
                double cy = (Bx[c] - Bx[at(n, i, j, k - 1)]) - (Bz[c] - Bz[at(n, i - 1, j, k)]);
                double cz = (By[c] - By[at(n, i - 1, j, k)]) - (Bx[c] - Bx[at(n, i, j - 1, k)]);
                Ex[c] += dt * (cx - Jx[c]);
                Ey[c] += dt * (cy - Jy[c]);
                Ez[c] += dt * (cz - Jz[c]);
            }
}

/* B -= dt/2 curl E;  E += dt (curl B - J);  B -= dt/2 curl E. */
void orc_yee(const int64_t n[3], double dt, double *F)
{
    half_b(n, 0.5 * dt, F);
    full_e(n, dt, F);
    half_b(n, 0.5 * dt, F);
}

/* ------------------------------------------------------------------------ */
/* One explicit PIC step (repeated nsteps times)                             */
/* ------------------------------------------------------------------------ */

static double wrapx(double x, double N)
{
    if (x < 0.0) x += N;
    if (x >= N) x -= N;
    return x;
}

/* Per step: J = 0; for every particle in array order: gather E^n, B^n at
 * x^n, Boris to u^{n+1/2}, x* = x^n + dt u/gamma, deposit the current of
 * x^n -> x*, then wrap x* periodically; finally the Yee update.
 * Returns 0, or -1 for bad arguments. */
int orc_pic_step(int m, const int64_t n[3], double dt, int64_t np, double *x, double *u,
                 const double *w, const int32_t *sp, const double *q, const double *mass,
                 double *F, int32_t nsteps)
{
    if (m < 1 || m > 3 || dt <= 0.0) return -1;
    size_t N = (size_t)(n[0] * n[1] * n[2]);
    double *J = F + 6 * N;
    for (int32_t s = 0; s < nsteps; ++s) {
        memset(J, 0, 3 * N * sizeof(double));
        for (int64_t p = 0; p < np; ++p) {
            double *xp = x + 3 * p, *up = u + 3 * p;
            double EB[6];
            orc_gather(m, n, F, xp, EB);
            int32_t sidx = sp[p];
            orc_boris(q[sidx], mass[sidx], dt, EB, EB + 3, up);
            double gam = sqrt(1.0 + up[0] * up[0] + up[1] * up[1] + up[2] * up[2]);
            double x1[3];
            for (int d = 0; d < 3; ++d) x1[d] = xp[d] + dt * up[d] / gam;
            orc_deposit(m, n, q[sidx] * w[p], dt, xp, x1, J);
            for (int d = 0; d < 3; ++d) xp[d] = wrapx(x1[d], (double)n[d]);
        }
        orc_yee(n, dt, F);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Box membership and the heuristic cost (Sec. 2.2)                          */
/* ------------------------------------------------------------------------ */

/* boxes: [nb][6] = lo_x lo_y lo_z hi_x hi_y hi_z (half-open cell ranges).
 * A particle is in box b iff lo_b <= floor(x) < hi_b in every dimension.
 * counts: [nb][nsp].  Returns -1 if a particle lies in no box. */
int orc_box_counts(int32_t nb, const int32_t *boxes, int64_t np, const double *x,
                   const int32_t *sp, int32_t nsp, int64_t *counts)
{
    memset(counts, 0, (size_t)nb * (size_t)nsp * sizeof(int64_t));
    for (int64_t p = 0; p < np; ++p) {
        int64_t c[3];
        for (int d = 0; d < 3; ++d) c[d] = (int64_t)floor(x[3 * p + d]);
        int32_t found = -1;
        for (int32_t b = 0; b < nb && found < 0; ++b) {
            const int32_t *bx = boxes + 6 * b;
            if (c[0] >= bx[0] && c[0] < bx[3] && c[1] >= bx[1] && c[1] < bx[4] &&
                c[2] >= bx[2] && c[2] < bx[5])
                found = b;
        }
        if (found < 0) return -1;
        counts[(size_t)found * nsp + sp[p]] += 1;
    }
    return 0;
}

/* Weighted linear sum of particles and cells per box:
 * cost_b = w_p * (sum over species of N_b) + w_c * cells_b. */
void orc_heuristic(int32_t nb, const int32_t *boxes, const int64_t *counts, int32_t nsp,
                   double wp, double wc, double *costs)
{
    for (int32_t b = 0; b < nb; ++b) {
        int64_t np = 0;
        for (int32_t s = 0; s < nsp; ++s) np += counts[(size_t)b * nsp + s];
        const int32_t *bx = boxes + 6 * b;
        int64_t cells = (int64_t)(bx[3] - bx[0]) * (bx[4] - bx[1]) * (bx[5] - bx[2]);
        double a = wp * (double)np;
        double c = wc * (double)cells;
        costs[b] = a + c;
    }
}

/* ------------------------------------------------------------------------ */
/* Load-balance efficiency (Eq. 1) and the improvement threshold             */
/* ------------------------------------------------------------------------ */

/* E = c_avg / c_max over ranks, where a rank's cost is the sum of its boxes'
 * costs (boxes visited in ascending index; ranks without boxes count with
 * cost 0).  E = 1 when every rank's cost is 0. */
double orc_efficiency(int32_t nb, const double *costs, const int32_t *rank, int32_t R)
{
    double *C = calloc((size_t)R, sizeof(double));
    for (int32_t b = 0; b < nb; ++b) C[rank[b]] += costs[b];
    double total = 0.0, mx = 0.0;
    for (int32_t r = 0; r < R; ++r) {
        total += C[r];
        if (C[r] > mx) mx = C[r];
    }
    free(C);
    if (mx == 0.0) return 1.0;
    return (total / (double)R) / mx;
}

/* The proposed mapping is adopted when its efficiency meets or exceeds the
 * current one improved by the relative threshold. */
int orc_should_adopt(double e_cur, double e_new, double thr)
{
    return e_new >= (1.0 + thr) * e_cur ? 1 : 0;
}

/* ------------------------------------------------------------------------ */
/* Space-filling-curve policy: Morton Z-order + contiguous min-max partition  */
/* ------------------------------------------------------------------------ */

/* Interleave: bit k of X, Y, Z goes to key bits 3k, 3k+1, 3k+2. */
uint64_t orc_morton3(uint32_t X, uint32_t Y, uint32_t Z)
{
    uint64_t key = 0;
    for (int b = 0; b < 21; ++b) {
        key |= (uint64_t)((X >> b) & 1u) << (3 * b);
        key |= (uint64_t)((Y >> b) & 1u) << (3 * b + 1);
        key |= (uint64_t)((Z >> b) & 1u) << (3 * b + 2);
    }
    return key;
}

static int64_t gcd64(int64_t a, int64_t b)
{
    while (b) { int64_t t = a % b; a = b; b = t; }
    return a < 0 ? -a : a;
}

static const uint64_t *g_sort_keys;
static int cmp_by_key(const void *pa, const void *pb)
{
    int32_t a = *(const int32_t *)pa, b = *(const int32_t *)pb;
    if (g_sort_keys[a] < g_sort_keys[b]) return -1;
    if (g_sort_keys[a] > g_sort_keys[b]) return 1;
    return 0;
}

static int cmp_double(const void *pa, const void *pb)
{
    double a = *(const double *)pa, b = *(const double *)pb;
    return (a > b) - (a < b);
}

/* Can the ordered costs be cut into at most R contiguous chunks, each with a
 * left-to-right sum <= B? (Greedy longest chunks decide this exactly.) */
static int fits(const double *c, int32_t nb, int32_t R, double B)
{
    int32_t chunks = 1;
    double acc = 0.0;
    for (int32_t i = 0; i < nb; ++i) {
        double nxt = acc + c[i];
        if (nxt <= B) {
            acc = nxt;
        } else {
            if (c[i] > B) return 0;
            ++chunks;
            acc = c[i];
        }
    }
    return chunks <= R;
}

/* Boxes are enumerated along the Morton curve of lo/g (g = gcd of every box
 * edge length); the ordering is cut into R contiguous chunks whose largest
 * sum B* is the smallest possible.  Chunk r (r < R-1) is the longest run
 * whose sum is <= B* that still leaves at least R-r-1 boxes; the last chunk
 * takes the rest.  With nb <= R each box goes to its own rank in curve order.
 * B* is found among all contiguous-run sums (the maximal chunk is one).
 * Returns 0, or -1 on bad input. */
int orc_sfc(int32_t nb, const int32_t *boxes, const double *costs, int32_t R, int32_t *rank,
            double *bstar_out)
{
    if (nb < 1 || R < 1) return -1;
    int64_t g = 0;
    for (int32_t b = 0; b < nb; ++b)
        for (int d = 0; d < 3; ++d) g = gcd64(g, (int64_t)(boxes[6 * b + 3 + d] - boxes[6 * b + d]));
    uint64_t *key = malloc(sizeof(uint64_t) * (size_t)nb);
    int32_t *ord = malloc(sizeof(int32_t) * (size_t)nb);
    for (int32_t b = 0; b < nb; ++b) {
        key[b] = orc_morton3((uint32_t)(boxes[6 * b] / g), (uint32_t)(boxes[6 * b + 1] / g),
                             (uint32_t)(boxes[6 * b + 2] / g));
        ord[b] = b;
    }
    g_sort_keys = key;
    qsort(ord, (size_t)nb, sizeof(int32_t), cmp_by_key);
    double *c = malloc(sizeof(double) * (size_t)nb);
    for (int32_t i = 0; i < nb; ++i) c[i] = costs[ord[i]];

    if (nb <= R) {
        for (int32_t i = 0; i < nb; ++i) rank[ord[i]] = i;
        double mx = 0.0;
        for (int32_t i = 0; i < nb; ++i) if (c[i] > mx) mx = c[i];
        if (bstar_out) *bstar_out = mx;
        free(key); free(ord); free(c);
        return 0;
    }
    /* every contiguous-run sum, summed left to right from its start */
    size_t ncand = (size_t)nb * (size_t)(nb + 1) / 2, q = 0;
    double *cand = malloc(sizeof(double) * ncand);
    for (int32_t i = 0; i < nb; ++i) {
        double acc = 0.0;
        for (int32_t j = i; j < nb; ++j) { acc += c[j]; cand[q++] = acc; }
    }
    qsort(cand, ncand, sizeof(double), cmp_double);
    size_t lo = 0, hi = ncand - 1; /* the total always fits */
    while (lo < hi) {
        size_t mid = lo + (hi - lo) / 2;
        if (fits(c, nb, R, cand[mid])) hi = mid; else lo = mid + 1;
    }
    double B = cand[lo];
    free(cand);

    int32_t p = 0;
    for (int32_t r = 0; r < R; ++r) {
        if (r == R - 1) {
            double acc = 0.0;
            for (; p < nb; ++p) { acc += c[p]; rank[ord[p]] = r; }
            if (acc > B) { free(key); free(ord); free(c); return -1; }
            break;
        }
        int32_t limit = nb - (R - r - 1);
        double acc = 0.0;
        int32_t start = p;
        while (p < limit) {
            double nxt = acc + c[p];
            if (nxt <= B || p == start) { acc = nxt; rank[ord[p]] = r; ++p; }
            else break;
        }
    }
    if (bstar_out) *bstar_out = B;
    free(key); free(ord); free(c);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Knapsack policy: longest-processing-time greedy with a box-count cap       */
/* ------------------------------------------------------------------------ */

static const double *g_sort_costs;
static int cmp_cost_desc(const void *pa, const void *pb)
{
    int32_t a = *(const int32_t *)pa, b = *(const int32_t *)pb;
    if (g_sort_costs[a] > g_sort_costs[b]) return -1;
    if (g_sort_costs[a] < g_sort_costs[b]) return 1;
    return (a > b) - (a < b);
}

/* Boxes in order of (cost descending, index ascending) each go to the rank
 * with the smallest (load, rank index) among ranks holding fewer than
 * cap = ceil(1.5 nb / R) boxes (the cap is 1.5 times the average number of
 * boxes per rank).  Returns 0, or -1 on bad input. */
int orc_knapsack(int32_t nb, const double *costs, int32_t R, int32_t *rank)
{
    if (nb < 1 || R < 1) return -1;
    int64_t cap = (3 * (int64_t)nb + 2 * (int64_t)R - 1) / (2 * (int64_t)R);
    int32_t *ord = malloc(sizeof(int32_t) * (size_t)nb);
    for (int32_t b = 0; b < nb; ++b) ord[b] = b;
    g_sort_costs = costs;
    qsort(ord, (size_t)nb, sizeof(int32_t), cmp_cost_desc);
    double *load = calloc((size_t)R, sizeof(double));
    int64_t *cnt = calloc((size_t)R, sizeof(int64_t));
    for (int32_t i = 0; i < nb; ++i) {
        int32_t b = ord[i], best = -1;
        for (int32_t r = 0; r < R; ++r) {
            if (cnt[r] >= cap) continue;
            if (best < 0 || load[r] < load[best]) best = r;
        }
        rank[b] = best;
        load[best] += costs[b];
        cnt[best] += 1;
    }
    free(ord); free(load); free(cnt);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Halo traffic of a distribution mapping                                     */
/* ------------------------------------------------------------------------ */

/* For every cell and each of its +x, +y, +z neighbours (periodic): if the two
 * cells lie in boxes owned by different ranks, each of the two ranks sends
 * `bytes` for that face.  per_rank[R] out.  Returns -1 if a cell lies in no
 * box. */
int orc_comm_volume(const int64_t n[3], int32_t nb, const int32_t *boxes, const int32_t *rank, int32_t R,
                    double bytes, double *per_rank)
{
    size_t N = (size_t)(n[0] * n[1] * n[2]);
    int32_t *owner = malloc(sizeof(int32_t) * N);
    for (size_t i = 0; i < N; ++i) owner[i] = -1;
    for (int32_t b = 0; b < nb; ++b) {
        const int32_t *bx = boxes + 6 * b;
        for (int64_t k = bx[2]; k < bx[5]; ++k)
            for (int64_t j = bx[1]; j < bx[4]; ++j)
                for (int64_t i = bx[0]; i < bx[3]; ++i) owner[at(n, i, j, k)] = b;
    }
    for (int32_t r = 0; r < R; ++r) per_rank[r] = 0.0;
    for (int64_t k = 0; k < n[2]; ++k)
        for (int64_t j = 0; j < n[1]; ++j)
            for (int64_t i = 0; i < n[0]; ++i) {
                int32_t a = owner[at(n, i, j, k)];
                if (a < 0) { free(owner); return -1; }
                int32_t nbr[3] = {owner[at(n, i + 1, j, k)], owner[at(n, i, j + 1, k)], owner[at(n, i, j, k + 1)]};
                for (int d = 0; d < 3; ++d) {
                    if (rank[a] == rank[nbr[d]]) continue;
                    per_rank[rank[a]] += bytes;
                    per_rank[rank[nbr[d]]] += bytes;
                }
            }
    free(owner);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Per-box features for the learned cost model                                */
/* ------------------------------------------------------------------------ */

/* feat: [nb][16]
 *  0,1   ln(1 + particles of species 0, 1)
 *  2..9  ln(1 + number of cells whose particle count (all species) is in
 *        [0], [1], [2,3], [4,7], [8,15], [16,31], [32,63], [64, inf))
 *  10    ln(cells)             11  shape order
 *  12    1 if the box touches a face of the domain, else 0
 *  13    ln(1 + particles in the box's outer cell layer)
 *  14    ln(1 + largest per-cell count)
 *  15    mean |u| over the box's particles (0 if none)                     */
int orc_box_features(const int64_t n[3], int32_t nb, const int32_t *boxes, int64_t np,
                     const double *x, const double *u, const int32_t *sp, int32_t nsp,
                     int32_t order, double *feat)
{
    size_t N = (size_t)(n[0] * n[1] * n[2]);
    int64_t *cellcnt = calloc(N, sizeof(int64_t));
    int32_t *owner = malloc(sizeof(int32_t) * N);
    for (size_t i = 0; i < N; ++i) owner[i] = -1;
    for (int32_t b = 0; b < nb; ++b) {
        const int32_t *bx = boxes + 6 * b;
        for (int64_t k = bx[2]; k < bx[5]; ++k)
            for (int64_t j = bx[1]; j < bx[4]; ++j)
                for (int64_t i = bx[0]; i < bx[3]; ++i) owner[at(n, i, j, k)] = b;
    }
    double *spc = calloc((size_t)nb * 2, sizeof(double));
    double *edge = calloc((size_t)nb, sizeof(double));
    double *usum = calloc((size_t)nb, sizeof(double));
    double *tot = calloc((size_t)nb, sizeof(double));
    for (int64_t p = 0; p < np; ++p) {
        int64_t c[3];
        for (int d = 0; d < 3; ++d) c[d] = (int64_t)floor(x[3 * p + d]);
        size_t ci = at(n, c[0], c[1], c[2]);
        int32_t b = owner[ci];
        if (b < 0) { free(cellcnt); free(owner); free(spc); free(edge); free(usum); free(tot); return -1; }
        cellcnt[ci] += 1;
        if (sp[p] < 2) spc[2 * b + sp[p]] += 1.0;
        tot[b] += 1.0;
        const int32_t *bx = boxes + 6 * b;
        int on_edge = 0;
        for (int d = 0; d < 3; ++d)
            if (c[d] == bx[d] || c[d] == bx[3 + d] - 1) on_edge = 1;
        if (on_edge) edge[b] += 1.0;
        const double *up = u + 3 * p;
        usum[b] += sqrt(up[0] * up[0] + up[1] * up[1] + up[2] * up[2]);
    }
    (void)nsp;
    for (int32_t b = 0; b < nb; ++b) {
        const int32_t *bx = boxes + 6 * b;
        double hist[8] = {0};
        int64_t mx = 0;
        for (int64_t k = bx[2]; k < bx[5]; ++k)
            for (int64_t j = bx[1]; j < bx[4]; ++j)
                for (int64_t i = bx[0]; i < bx[3]; ++i) {
                    int64_t v = cellcnt[at(n, i, j, k)];
                    int bin;
                    if (v == 0) bin = 0;
                    else if (v == 1) bin = 1;
                    else if (v < 4) bin = 2;
                    else if (v < 8) bin = 3;
                    else if (v < 16) bin = 4;
                    else if (v < 32) bin = 5;
                    else if (v < 64) bin = 6;
                    else bin = 7;
                    hist[bin] += 1.0;
                    if (v > mx) mx = v;
                }
        double *f = feat + 16 * (size_t)b;
        f[0] = log(1.0 + spc[2 * b]);
        f[1] = log(1.0 + spc[2 * b + 1]);
        for (int h = 0; h < 8; ++h) f[2 + h] = log(1.0 + hist[h]);
        double cells = (double)(bx[3] - bx[0]) * (double)(bx[4] - bx[1]) * (double)(bx[5] - bx[2]);
        f[10] = log(cells);
        f[11] = (double)order;
        int touch = 0;
        for (int d = 0; d < 3; ++d)
            if (bx[d] == 0 || bx[3 + d] == n[d]) touch = 1;
        f[12] = touch ? 1.0 : 0.0;
        f[13] = log(1.0 + edge[b]);
        f[14] = log(1.0 + (double)mx);
        f[15] = tot[b] > 0.0 ? usum[b] / tot[b] : 0.0;
    }
    free(cellcnt); free(owner); free(spc); free(edge); free(usum); free(tot);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Learned cost model: 16 -> 64 -> 64 -> 1 perceptron, MSE loss, Adam         */
/* ------------------------------------------------------------------------ */

#define MLP_IN 16
#define MLP_H 64
/* parameter layout: W1[64][16] b1[64] W2[64][64] b2[64] W3[64] b3[1] */
#define OFF_W1 0
#define OFF_B1 (OFF_W1 + MLP_H * MLP_IN)
#define OFF_W2 (OFF_B1 + MLP_H)
#define OFF_B2 (OFF_W2 + MLP_H * MLP_H)
#define OFF_W3 (OFF_B2 + MLP_H)
#define OFF_B3 (OFF_W3 + MLP_H)
#define MLP_NPARAM (OFF_B3 + 1)

int32_t orc_mlp_nparam(void) { return MLP_NPARAM; }

/* Round to the nearest bfloat16 (ties to even), via the float value. */
double orc_bf16(double v)
{
    float f = (float)v;
    uint32_t bits;
    memcpy(&bits, &f, 4);
    if ((bits & 0x7f800000u) == 0x7f800000u) return v; /* inf / nan */
    uint32_t lsb = (bits >> 16) & 1u;
    bits += 0x7fffu + lsb;
    bits &= 0xffff0000u;
    memcpy(&f, &bits, 4);
    return (double)f;
}

static double rb(double v, int mirror) { return mirror ? orc_bf16(v) : v; }

/* Mean squared error of yhat = W3 relu(W2 relu(W1 x + b1) + b2) + b3 against
 * y over n samples; optionally the gradient (ReLU'(0) = 0) and predictions.
 * mirror != 0 rounds to bfloat16 exactly where a bfloat16 matrix unit would
 * take its operands: inputs, weights, both hidden activations, and the
 * back-propagated pre-activation gradients feeding the weight and input
 * gradients of layers 1 and 2.  Biases, accumulations and the loss stay in
 * double. */
double orc_mlp_loss_grad(const double *P, const double *X, const double *y, int64_t n,
                         int32_t mirror, double *grad, double *yhat)
{
    double W1[MLP_H * MLP_IN], W2[MLP_H * MLP_H], W3[MLP_H];
    for (int i = 0; i < MLP_H * MLP_IN; ++i) W1[i] = rb(P[OFF_W1 + i], mirror);
    for (int i = 0; i < MLP_H * MLP_H; ++i) W2[i] = rb(P[OFF_W2 + i], mirror);
    for (int i = 0; i < MLP_H; ++i) W3[i] = rb(P[OFF_W3 + i], mirror);
    const double *b1 = P + OFF_B1, *b2 = P + OFF_B2, b3 = P[OFF_B3];
    if (grad) memset(grad, 0, sizeof(double) * MLP_NPARAM);
    double loss = 0.0;
    for (int64_t s = 0; s < n; ++s) {
        double xin[MLP_IN], z1[MLP_H], h1[MLP_H], z2[MLP_H], h2[MLP_H];
        for (int i = 0; i < MLP_IN; ++i) xin[i] = rb(X[s * MLP_IN + i], mirror);
        for (int o = 0; o < MLP_H; ++o) {
            double acc = 0.0;
            for (int i = 0; i < MLP_IN; ++i) acc += W1[o * MLP_IN + i] * xin[i];
            z1[o] = acc + b1[o];
            h1[o] = rb(z1[o] > 0.0 ? z1[o] : 0.0, mirror);
        }
        for (int o = 0; o < MLP_H; ++o) {
            double acc = 0.0;
            for (int i = 0; i < MLP_H; ++i) acc += W2[o * MLP_H + i] * h1[i];
            z2[o] = acc + b2[o];
            h2[o] = rb(z2[o] > 0.0 ? z2[o] : 0.0, mirror);
        }
        double out = 0.0;
        for (int i = 0; i < MLP_H; ++i) out += W3[i] * h2[i];
        out += b3;
        if (yhat) yhat[s] = out;
        double r = out - y[s];
        loss += r * r;
        if (!grad) continue;
        double dy = 2.0 * r / (double)n;
        double dz2[MLP_H], dz2r[MLP_H], dz1[MLP_H], dz1r[MLP_H];
        for (int i = 0; i < MLP_H; ++i) {
            grad[OFF_W3 + i] += dy * h2[i];
            dz2[i] = z2[i] > 0.0 ? dy * W3[i] : 0.0;
            dz2r[i] = rb(dz2[i], mirror);
        }
        grad[OFF_B3] += dy;
        for (int o = 0; o < MLP_H; ++o) {
            grad[OFF_B2 + o] += dz2[o];
            for (int i = 0; i < MLP_H; ++i) grad[OFF_W2 + o * MLP_H + i] += dz2r[o] * h1[i];
        }
        for (int i = 0; i < MLP_H; ++i) {
            double acc = 0.0;
            for (int o = 0; o < MLP_H; ++o) acc += dz2r[o] * W2[o * MLP_H + i];
            dz1[i] = z1[i] > 0.0 ? acc : 0.0;
            dz1r[i] = rb(dz1[i], mirror);
        }
        for (int o = 0; o < MLP_H; ++o) {
            grad[OFF_B1 + o] += dz1[o];
            for (int i = 0; i < MLP_IN; ++i) grad[OFF_W1 + o * MLP_IN + i] += dz1r[o] * xin[i];
        }
    }
    return loss / (double)n;
}

/* Adam (Kingma & Ba 2015) with bias correction; t counts from 1. */
void orc_adam(double *P, const double *g, double *mom, double *vel, int64_t np, int64_t t,
              double lr, double beta1, double beta2, double eps)
{
    double c1 = 1.0 - pow(beta1, (double)t), c2 = 1.0 - pow(beta2, (double)t);
    for (int64_t i = 0; i < np; ++i) {
        mom[i] = beta1 * mom[i] + (1.0 - beta1) * g[i];
        vel[i] = beta2 * vel[i] + (1.0 - beta2) * g[i] * g[i];
        double mh = mom[i] / c1, vh = vel[i] / c2;
        P[i] -= lr * mh / (sqrt(vh) + eps);
    }
}
