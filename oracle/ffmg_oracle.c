/*
 * ffmg_oracle.c -- plain FP64 CPU oracle for the complex-contour multigrid
 * far-field method of Cools, Reps & Vanroose, "An efficient multigrid
 * calculation of the Far Field map for Helmholtz and Schroedinger equations"
 * (arXiv 1211.4461).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the reference the GPU library is
 * checked against.  It shares no source, header or generated table with the
 * HIP library; only tests, the smoke check and the CPU-baseline leg of the
 * benchmark may load it.  It is written to be read against the paper, not to
 * be fast: every loop is the plain definition, in double precision, in the
 * order the paper states the steps.
 *
 * Conventions (readings of the paper, each argued in the design notes):
 *   - grid: n_k intervals per axis on [lo_k, hi_k], h_k = (hi_k-lo_k)/n_k,
 *     interior nodes x_i = lo_k + i*h_k, i = 1..n_k-1, x fastest; homogeneous
 *     Dirichlet values outside the interior (Sec. 4, the n^d mesh).
 *   - contour: z = e^{i gamma} x, 0 < gamma < pi/2 (Sec. 3.1, eq. I2complex).
 *   - operator: finite differences with complex spacing e^{i gamma} h give
 *       (A u)_j = sum_k c_k (2 u_j - u_{j-e_k} - u_{j+e_k}) - kappa_j u_j,
 *     c_k = e^{-2 i gamma}/h_k^2 (Sec. 3.2, eq. csg; the rotated 1D stencil
 *     of Sec. 5.2), kappa_j = k^2(z_j).
 *   - right-hand side: b_j = q_j exp(i k0 eta.z_j) with the contrast
 *     q_j = k^2(z_j) - k0^2 = k0^2 chi(z_j), i.e. k0^2 chi(z) u_in(z) of
 *     eq. helmholtz_cc (Sec. 2.1, 3.1).
 *   - far field: F(alpha) = e^{i d gamma} prod_k h_k
 *       sum_j exp(-i k0 alpha.z_j) q_j (u_in,j + u_j)
 *     i.e. eq. FFmap with g = k0^2 chi (u_in + u) moved onto the contour
 *     (eq. I2complex, with the d-dimensional Jacobian e^{i d gamma}).
 *   - multigrid: V(nu1,nu2) with omega-Jacobi smoothing, full-weighting
 *     restriction, bilinear/trilinear prolongation, rediscretised coarse
 *     operators with injected kappa, exact (LU) solve on the coarsest grid
 *     (Sec. 4: V-cycles, bilinear interpolation and full weighting; F(5)
 *     cycle of Sec. 5.7: coarsest 7^3 grid solved exactly).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double _Complex cplx;

/* ------------------------------------------------------------------ */
/* Grid helpers                                                        */
/* ------------------------------------------------------------------ */

static long npts(int dim, const long *m)
{
    long N = 1;
    for (int k = 0; k < dim; ++k) N *= m[k];
    return N;
}

/* Extent of each axis, with unused axes set to 1. */
static void extents(int dim, const long *m, long e[3])
{
    for (int k = 0; k < 3; ++k) e[k] = (k < dim) ? m[k] : 1;
}

/* Value of u at interior multi-index (ix,iy,iz) (0-based interior index),
 * zero outside the interior: homogeneous Dirichlet boundary. */
static cplx at(const cplx *u, const long e[3], long ix, long iy, long iz)
{
    if (ix < 0 || iy < 0 || iz < 0 || ix >= e[0] || iy >= e[1] || iz >= e[2])
        return 0.0;
    return u[ix + e[0] * (iy + e[1] * iz)];
}

/* Stencil coefficients c_k = e^{-2 i gamma} / h_k^2 (Sec. 3.2, eq. csg). */
static void stencil_coefs(int dim, const double *h, double gamma, cplx c[3])
{
    cplx rot = cexp(-2.0 * I * gamma);
    for (int k = 0; k < 3; ++k) c[k] = (k < dim) ? rot / (h[k] * h[k]) : 0.0;
}

/* (A u)_j for the contour operator, matrix free (Sec. 3.2, eq. csg). */
static cplx apply_point(int dim, const long e[3], const cplx c[3],
                        const cplx *kappa, const cplx *u,
                        long ix, long iy, long iz)
{
    long j = ix + e[0] * (iy + e[1] * iz);
    cplx uj = u[j];
    cplx lap = c[0] * (2.0 * uj - at(u, e, ix - 1, iy, iz) - at(u, e, ix + 1, iy, iz));
    if (dim >= 2)
        lap += c[1] * (2.0 * uj - at(u, e, ix, iy - 1, iz) - at(u, e, ix, iy + 1, iz));
    if (dim >= 3)
        lap += c[2] * (2.0 * uj - at(u, e, ix, iy, iz - 1) - at(u, e, ix, iy, iz + 1));
    return lap - kappa[j] * uj;
}

/* Au = A u. */
void or_apply(int dim, const long *m, const double *h, double gamma,
              const cplx *kappa, const cplx *u, cplx *Au)
{
    long e[3];
    cplx c[3];
    extents(dim, m, e);
    stencil_coefs(dim, h, gamma, c);
    #pragma omp parallel for schedule(static)
    for (long iz = 0; iz < e[2]; ++iz)
        for (long iy = 0; iy < e[1]; ++iy)
            for (long ix = 0; ix < e[0]; ++ix)
                Au[ix + e[0] * (iy + e[1] * iz)] =
                    apply_point(dim, e, c, kappa, u, ix, iy, iz);
}

/* r = b - A u. */
void or_residual(int dim, const long *m, const double *h, double gamma,
                 const cplx *kappa, const cplx *b, const cplx *u, cplx *r)
{
    long e[3];
    cplx c[3];
    extents(dim, m, e);
    stencil_coefs(dim, h, gamma, c);
    #pragma omp parallel for schedule(static)
    for (long iz = 0; iz < e[2]; ++iz)
        for (long iy = 0; iy < e[1]; ++iy)
            for (long ix = 0; ix < e[0]; ++ix) {
                long j = ix + e[0] * (iy + e[1] * iz);
                r[j] = b[j] - apply_point(dim, e, c, kappa, u, ix, iy, iz);
            }
}

/* One weighted-Jacobi sweep, out of place:
 *   u'_j = u_j + omega (b_j - (A u)_j) / D_j,  D_j = 2 sum_k c_k - kappa_j
 * (Sec. 4: omega-Jacobi smoother of the V(1,1) cycle). */
void or_jacobi(int dim, const long *m, const double *h, double gamma,
               const cplx *kappa, const cplx *b, const cplx *u, double omega,
               cplx *u_out)
{
    long e[3];
    cplx c[3];
    extents(dim, m, e);
    stencil_coefs(dim, h, gamma, c);
    cplx csum = 0.0;
    for (int k = 0; k < dim; ++k) csum += 2.0 * c[k];
    #pragma omp parallel for schedule(static)
    for (long iz = 0; iz < e[2]; ++iz)
        for (long iy = 0; iy < e[1]; ++iy)
            for (long ix = 0; ix < e[0]; ++ix) {
                long j = ix + e[0] * (iy + e[1] * iz);
                cplx D = csum - kappa[j];
                cplx res = b[j] - apply_point(dim, e, c, kappa, u, ix, iy, iz);
                u_out[j] = u[j] + omega * res / D;
            }
}

/* One red-black Gauss-Seidel sweep, in place (Sec. 3.3 names Gauss-Seidel
 * beside weighted Jacobi as the standard relaxation of the V-cycle): the
 * points with ix + iy + iz even (0-based interior indices, "red") are
 * relaxed first, u_j <- u_j + (b_j - (A u)_j) / D_j, then the others with
 * the red values already updated.  A red point's stencil neighbours are all
 * black and the other way round, so each half sweep is a set of independent
 * point updates. */
void or_rbgs(int dim, const long *m, const double *h, double gamma,
             const cplx *kappa, const cplx *b, cplx *u)
{
    long e[3];
    cplx c[3];
    extents(dim, m, e);
    stencil_coefs(dim, h, gamma, c);
    cplx csum = 0.0;
    for (int k = 0; k < dim; ++k) csum += 2.0 * c[k];
    for (int color = 0; color < 2; ++color) {
        #pragma omp parallel for schedule(static)
        for (long iz = 0; iz < e[2]; ++iz)
            for (long iy = 0; iy < e[1]; ++iy)
                for (long ix = 0; ix < e[0]; ++ix) {
                    if (((ix + iy + iz) & 1) != color) continue;
                    long j = ix + e[0] * (iy + e[1] * iz);
                    cplx D = csum - kappa[j];
                    u[j] += (b[j] - apply_point(dim, e, c, kappa, u, ix, iy, iz)) / D;
                }
    }
}

/* One GMRES(m) smoothing step from the guess u, in place (Sec. 3.3: GMRES(m),
 * m = 2 or 3, as the smoother that replaces weighted Jacobi and keeps the
 * V-cycle stable at rotation angles near 10 degrees).  It is one restart
 * cycle of GMRES: with r0 = b - A u and the Krylov space
 * K_m = span{r0, A r0, ..., A^{m-1} r0}, u is replaced by the u + z, z in
 * K_m, of least residual norm.  The basis is built by Arnoldi's process with
 * modified Gram-Schmidt and the Hermitian inner product sum conj(x) y; the
 * (m+1) x m least-squares problem is reduced by complex Givens rotations.
 * A breakdown (the Krylov space is invariant) ends the process early; the
 * least-squares solution then solves A u = b. */
void or_gmres(int dim, const long *m, const double *h, double gamma,
              const cplx *kappa, const cplx *b, cplx *u, int mk)
{
    if (mk > 16) mk = 16;                                    /* the small arrays below */
    long N = npts(dim, m);
    cplx *V = malloc((size_t)(mk + 1) * (size_t)N * sizeof(cplx));
    cplx *w = malloc((size_t)N * sizeof(cplx));
    cplx H[17][16], g[17], cs[16], sn[16];
    memset(H, 0, sizeof H);
    or_residual(dim, m, h, gamma, kappa, b, u, V);          /* V_0 = r0 */
    double beta = 0.0;
    for (long j = 0; j < N; ++j) beta += creal(V[j]) * creal(V[j]) + cimag(V[j]) * cimag(V[j]);
    beta = sqrt(beta);
    if (beta == 0.0 || mk < 1) { free(V); free(w); return; }
    for (long j = 0; j < N; ++j) V[j] /= beta;
    int k = 0;
    for (int jj = 0; jj < mk; ++jj) {
        or_apply(dim, m, h, gamma, kappa, V + (size_t)jj * N, w);   /* w = A v_j */
        for (int i = 0; i <= jj; ++i) {                              /* MGS */
            const cplx *vi = V + (size_t)i * N;
            cplx d = 0.0;
            for (long j = 0; j < N; ++j) d += conj(vi[j]) * w[j];
            H[i][jj] = d;
            for (long j = 0; j < N; ++j) w[j] -= d * vi[j];
        }
        double nw = 0.0;
        for (long j = 0; j < N; ++j) nw += creal(w[j]) * creal(w[j]) + cimag(w[j]) * cimag(w[j]);
        nw = sqrt(nw);
        H[jj + 1][jj] = nw;
        k = jj + 1;
        if (nw == 0.0) break;                                        /* invariant subspace */
        cplx *vn = V + (size_t)(jj + 1) * N;
        for (long j = 0; j < N; ++j) vn[j] = w[j] / nw;
    }
    /* least squares min || beta e1 - H y || by Givens rotations */
    for (int i = 0; i <= k; ++i) g[i] = 0.0;
    g[0] = beta;
    for (int j = 0; j < k; ++j) {
        for (int i = 0; i < j; ++i) {                                /* earlier rotations */
            cplx t = cs[i] * H[i][j] + sn[i] * H[i + 1][j];
            H[i + 1][j] = -conj(sn[i]) * H[i][j] + cs[i] * H[i + 1][j];
            H[i][j] = t;
        }
        cplx a = H[j][j], c = H[j + 1][j];
        double r = sqrt(creal(a) * creal(a) + cimag(a) * cimag(a) + creal(c) * creal(c) + cimag(c) * cimag(c));
        if (r == 0.0) { cs[j] = 1.0; sn[j] = 0.0; continue; }
        double aa = cabs(a);
        if (aa == 0.0) { cs[j] = 0.0; sn[j] = conj(c) / r; }
        else { cs[j] = aa / r; sn[j] = (a / aa) * conj(c) / r; }
        H[j][j] = cs[j] * a + sn[j] * c;
        H[j + 1][j] = 0.0;
        cplx t = cs[j] * g[j] + sn[j] * g[j + 1];
        g[j + 1] = -conj(sn[j]) * g[j] + cs[j] * g[j + 1];
        g[j] = t;
    }
    cplx y[16];
    for (int i = k - 1; i >= 0; --i) {                               /* back substitution */
        cplx t = g[i];
        for (int j = i + 1; j < k; ++j) t -= H[i][j] * y[j];
        y[i] = (H[i][i] != 0.0) ? t / H[i][i] : 0.0;
    }
    for (int j = 0; j < k; ++j) {
        const cplx *vj = V + (size_t)j * N;
        for (long p = 0; p < N; ++p) u[p] += y[j] * vj[p];
    }
    free(V);
    free(w);
}

/* Full-weighting restriction: 1D weights (1/4, 1/2, 1/4) at fine
 * 2I-1, 2I, 2I+1, tensorised over the axes (Sec. 4: full weighting).
 * mf = fine interior counts (odd: n_f - 1); coarse counts (mf-1)/2. */
void or_restrict(int dim, const long *mf, const cplx *rf, cplx *rc)
{
    long ef[3], ec[3];
    extents(dim, mf, ef);
    for (int k = 0; k < 3; ++k) ec[k] = (k < dim) ? (mf[k] - 1) / 2 : 1;
    static const double w[3] = {0.25, 0.5, 0.25};
    #pragma omp parallel for schedule(static)
    for (long Iz = 0; Iz < ec[2]; ++Iz)
        for (long Iy = 0; Iy < ec[1]; ++Iy)
            for (long Ix = 0; Ix < ec[0]; ++Ix) {
                /* coarse interior index I (0-based) is coarse node I+1,
                 * i.e. fine node 2(I+1), i.e. fine interior index 2I+1 */
                long fx = 2 * Ix + 1, fy = 2 * Iy + 1, fz = 2 * Iz + 1;
                cplx acc = 0.0;
                for (int dz = -1; dz <= 1; ++dz) {
                    if (dim < 3 && dz != 0) continue;
                    double wz = (dim < 3) ? 1.0 : w[dz + 1];
                    for (int dy = -1; dy <= 1; ++dy) {
                        if (dim < 2 && dy != 0) continue;
                        double wy = (dim < 2) ? 1.0 : w[dy + 1];
                        for (int dx = -1; dx <= 1; ++dx) {
                            double wx = w[dx + 1];
                            long x = fx + dx, y = (dim < 2) ? 0 : fy + dy,
                                 z = (dim < 3) ? 0 : fz + dz;
                            acc += wx * wy * wz * rf[x + ef[0] * (y + ef[1] * z)];
                        }
                    }
                }
                rc[Ix + ec[0] * (Iy + ec[1] * Iz)] = acc;
            }
}

/* 1D linear interpolation weight of coarse node I (1-based, coarse grid)
 * for fine node i (1-based): fine 2I gets 1, fine 2I+-1 get 1/2. */
static double interp_w(long i, long Ic)
{
    long d = i - 2 * Ic;
    if (d == 0) return 1.0;
    if (d == 1 || d == -1) return 0.5;
    return 0.0;
}

/* u_f += P e_c, bilinear (2D) / trilinear (3D) interpolation
 * (Sec. 4: bilinear interpolation), zero coarse values on the boundary.
 * mc = coarse interior counts; fine counts 2 mc + 1. */
void or_prolong_add(int dim, const long *mc, const cplx *ec_, cplx *uf)
{
    long ec[3], ef[3];
    extents(dim, mc, ec);
    for (int k = 0; k < 3; ++k) ef[k] = (k < dim) ? 2 * mc[k] + 1 : 1;
    #pragma omp parallel for schedule(static)
    for (long iz = 0; iz < ef[2]; ++iz)
        for (long iy = 0; iy < ef[1]; ++iy)
            for (long ix = 0; ix < ef[0]; ++ix) {
                /* fine 1-based node indices */
                long fx = ix + 1, fy = iy + 1, fz = iz + 1;
                cplx acc = 0.0;
                /* the coarse nodes that can touch fine node f are
                 * floor(f/2) and ceil(f/2) (1-based) */
                for (long Iz = (dim < 3 ? 1 : fz / 2); Iz <= (dim < 3 ? 1 : (fz + 1) / 2); ++Iz)
                    for (long Iy = (dim < 2 ? 1 : fy / 2); Iy <= (dim < 2 ? 1 : (fy + 1) / 2); ++Iy)
                        for (long Ix = fx / 2; Ix <= (fx + 1) / 2; ++Ix) {
                            double wx = interp_w(fx, Ix);
                            double wy = (dim < 2) ? 1.0 : interp_w(fy, Iy);
                            double wz = (dim < 3) ? 1.0 : interp_w(fz, Iz);
                            double wgt = wx * wy * wz;
                            if (wgt == 0.0) continue;
                            acc += wgt * at(ec_, ec, Ix - 1,
                                            (dim < 2) ? 0 : Iy - 1,
                                            (dim < 3) ? 0 : Iz - 1);
                        }
                uf[ix + ef[0] * (iy + ef[1] * iz)] += acc;
            }
}

/* kappa on the coarse grid by injection: coarse node I takes the value of
 * fine node 2I (reading: coarse operators rediscretised at 2h). */
void or_inject(int dim, const long *mf, const cplx *kf, cplx *kc)
{
    long ef[3], ec[3];
    extents(dim, mf, ef);
    for (int k = 0; k < 3; ++k) ec[k] = (k < dim) ? (mf[k] - 1) / 2 : 1;
    for (long Iz = 0; Iz < ec[2]; ++Iz)
        for (long Iy = 0; Iy < ec[1]; ++Iy)
            for (long Ix = 0; Ix < ec[0]; ++Ix) {
                long x = 2 * Ix + 1, y = (dim < 2) ? 0 : 2 * Iy + 1,
                     z = (dim < 3) ? 0 : 2 * Iz + 1;
                kc[Ix + ec[0] * (Iy + ec[1] * Iz)] = kf[x + ef[0] * (y + ef[1] * z)];
            }
}

/* ------------------------------------------------------------------ */
/* Dense LU with partial pivoting (coarsest grid, solved exactly).     */
/* ------------------------------------------------------------------ */

/* Assemble the dense matrix of A on a (small) grid, row-major NxN. */
void or_assemble_dense(int dim, const long *m, const double *h, double gamma,
                       const cplx *kappa, cplx *A)
{
    long N = npts(dim, m);
    cplx *ej = calloc((size_t)N, sizeof(cplx));
    cplx *col = malloc((size_t)N * sizeof(cplx));
    for (long j = 0; j < N; ++j) {
        ej[j] = 1.0;
        or_apply(dim, m, h, gamma, kappa, ej, col);
        for (long i = 0; i < N; ++i) A[i * N + j] = col[i];
        ej[j] = 0.0;
    }
    free(ej);
    free(col);
}

/* In-place LU with partial pivoting (Doolittle), row-major.  Returns 0, or
 * -1 if a zero pivot is met. */
int or_lu_factor(long N, cplx *A, long *piv)
{
    for (long k = 0; k < N; ++k) {
        long p = k;
        double best = cabs(A[k * N + k]);
        for (long i = k + 1; i < N; ++i) {
            double v = cabs(A[i * N + k]);
            if (v > best) { best = v; p = i; }
        }
        if (best == 0.0) return -1;
        piv[k] = p;
        if (p != k)
            for (long j = 0; j < N; ++j) {
                cplx t = A[k * N + j];
                A[k * N + j] = A[p * N + j];
                A[p * N + j] = t;
            }
        for (long i = k + 1; i < N; ++i) {
            cplx l = A[i * N + k] / A[k * N + k];
            A[i * N + k] = l;
            for (long j = k + 1; j < N; ++j) A[i * N + j] -= l * A[k * N + j];
        }
    }
    return 0;
}

/* Solve with the factors: x = A^{-1} b (b overwritten by x). */
void or_lu_solve(long N, const cplx *LU, const long *piv, cplx *x)
{
    for (long k = 0; k < N; ++k)
        if (piv[k] != k) {
            cplx t = x[k];
            x[k] = x[piv[k]];
            x[piv[k]] = t;
        }
    for (long i = 0; i < N; ++i)
        for (long j = 0; j < i; ++j) x[i] -= LU[i * N + j] * x[j];
    for (long i = N - 1; i >= 0; --i) {
        for (long j = i + 1; j < N; ++j) x[i] -= LU[i * N + j] * x[j];
        x[i] /= LU[i * N + i];
    }
}

/* ------------------------------------------------------------------ */
/* Multigrid hierarchy, V-cycle and solve                              */
/* ------------------------------------------------------------------ */

#define OR_MAXLEV 32

typedef struct {
    int dim, nlev, nu1, nu2;
    int smoother, krylov_m;   /* 0: omega-Jacobi; 1: GMRES(krylov_m); 2: red-black Gauss-Seidel */
    double gamma, omega;
    long m[OR_MAXLEV][3];
    double h[OR_MAXLEV][3];
    cplx *kappa[OR_MAXLEV];
    cplx *r[OR_MAXLEV];   /* residual / work */
    cplx *b[OR_MAXLEV];   /* coarse right-hand sides (level >= 1) */
    cplx *u[OR_MAXLEV];   /* coarse corrections (level >= 1) */
    cplx *t[OR_MAXLEV];   /* Jacobi ping-pong buffer */
    cplx *LU;
    long *piv;
    long Nc;
} or_mg;

/* Build the hierarchy n_l = n / 2^l down to min_k n_k = coarsest_n
 * (reading: coarsest 7^d interior unknowns, as in the F(5) cycle). */
void *or_mg_create(int dim, const long *n, const double *lo, const double *hi,
                   double gamma, const cplx *kappa, int nu1, int nu2,
                   double omega, long coarsest_n)
{
    or_mg *g = calloc(1, sizeof(or_mg));
    g->dim = dim; g->nu1 = nu1; g->nu2 = nu2; g->gamma = gamma; g->omega = omega;
    long nl[3];
    for (int k = 0; k < 3; ++k) nl[k] = (k < dim) ? n[k] : 2;
    int L = 0;
    for (;;) {
        for (int k = 0; k < 3; ++k) {
            g->m[L][k] = (k < dim) ? nl[k] - 1 : 1;
            g->h[L][k] = (k < dim) ? (hi[k] - lo[k]) / (double)nl[k] : 1.0;
        }
        long nmin = nl[0];
        for (int k = 1; k < dim; ++k) if (nl[k] < nmin) nmin = nl[k];
        if (nmin <= coarsest_n || L == OR_MAXLEV - 1) break;
        for (int k = 0; k < dim; ++k) nl[k] /= 2;
        ++L;
    }
    g->nlev = L + 1;
    for (int l = 0; l < g->nlev; ++l) {
        long N = npts(dim, g->m[l]);
        g->kappa[l] = malloc((size_t)N * sizeof(cplx));
        g->r[l] = calloc((size_t)N, sizeof(cplx));
        g->b[l] = calloc((size_t)N, sizeof(cplx));
        g->u[l] = calloc((size_t)N, sizeof(cplx));
        g->t[l] = calloc((size_t)N, sizeof(cplx));
        if (l == 0) memcpy(g->kappa[0], kappa, (size_t)N * sizeof(cplx));
        else or_inject(dim, g->m[l - 1], g->kappa[l - 1], g->kappa[l]);
    }
    int Lc = g->nlev - 1;
    g->Nc = npts(dim, g->m[Lc]);
    g->LU = malloc((size_t)(g->Nc * g->Nc) * sizeof(cplx));
    g->piv = malloc((size_t)g->Nc * sizeof(long));
    or_assemble_dense(dim, g->m[Lc], g->h[Lc], gamma, g->kappa[Lc], g->LU);
    or_lu_factor(g->Nc, g->LU, g->piv);
    return g;
}

void or_mg_destroy(void *p)
{
    or_mg *g = p;
    if (!g) return;
    for (int l = 0; l < g->nlev; ++l) {
        free(g->kappa[l]); free(g->r[l]); free(g->b[l]); free(g->u[l]); free(g->t[l]);
    }
    free(g->LU); free(g->piv); free(g);
}

int or_mg_nlev(void *p) { return ((or_mg *)p)->nlev; }
long or_mg_coarse_n(void *p) { return ((or_mg *)p)->Nc; }

/* Copy out kappa on level l (for tests). */
void or_mg_kappa(void *p, int l, cplx *out)
{
    or_mg *g = p;
    memcpy(out, g->kappa[l], (size_t)npts(g->dim, g->m[l]) * sizeof(cplx));
}

/* Choose the smoother of every level below the coarsest: omega-Jacobi
 * (smoother 0, the default), GMRES(m) steps (smoother 1) or red-black
 * Gauss-Seidel sweeps (smoother 2). */
void or_mg_set_smoother(void *p, int smoother, int m)
{
    or_mg *g = p;
    g->smoother = smoother;
    g->krylov_m = m;
}

static void smooth(or_mg *g, int l, const cplx *b, cplx *u, int nu)
{
    long N = npts(g->dim, g->m[l]);
    if (g->smoother == 1) {
        for (int s = 0; s < nu; ++s) or_gmres(g->dim, g->m[l], g->h[l], g->gamma, g->kappa[l], b, u, g->krylov_m);
        return;
    }
    if (g->smoother == 2) {
        for (int s = 0; s < nu; ++s) or_rbgs(g->dim, g->m[l], g->h[l], g->gamma, g->kappa[l], b, u);
        return;
    }
    for (int s = 0; s < nu; ++s) {
        or_jacobi(g->dim, g->m[l], g->h[l], g->gamma, g->kappa[l], b, u, g->omega, g->t[l]);
        memcpy(u, g->t[l], (size_t)N * sizeof(cplx));
    }
}

/* V(l, u, b): the recursive V(nu1, nu2) cycle. */
static void vcycle(or_mg *g, int l, const cplx *b, cplx *u)
{
    int dim = g->dim;
    long N = npts(dim, g->m[l]);
    if (l == g->nlev - 1) {
        memcpy(u, b, (size_t)N * sizeof(cplx));
        or_lu_solve(N, g->LU, g->piv, u);
        return;
    }
    smooth(g, l, b, u, g->nu1);                                     /* pre-smoothing   */
    or_residual(dim, g->m[l], g->h[l], g->gamma, g->kappa[l], b, u, g->r[l]);
    or_restrict(dim, g->m[l], g->r[l], g->b[l + 1]);                 /* b_c = FW r      */
    long Nc = npts(dim, g->m[l + 1]);
    memset(g->u[l + 1], 0, (size_t)Nc * sizeof(cplx));              /* e_c = 0         */
    vcycle(g, l + 1, g->b[l + 1], g->u[l + 1]);                      /* coarse solve    */
    or_prolong_add(dim, g->m[l + 1], g->u[l + 1], u);                /* u += P e_c      */
    smooth(g, l, b, u, g->nu2);                                      /* post-smoothing  */
}

/* One V-cycle on the finest level, in place. */
void or_mg_vcycle(void *p, const cplx *b, cplx *u)
{
    vcycle((or_mg *)p, 0, b, u);
}

/* Full multigrid start (Sec. 4 with Tables 3 and 4, the nested iteration of
 * V-cycles; Sec. 5.7, the F(5) cycle): the right-hand side of every coarser
 * level is the fine one sampled at the coarse nodes (injection: the same
 * problem discretized on the coarse grid, as the coefficients are), the
 * coarsest level is solved exactly, and on every level between it and the
 * finest the interpolated coarser solution is improved by k V-cycles.  u
 * receives the interpolated level-1 solution: the initial guess of the
 * finest-level solve. */
void or_mg_fmg(void *p, const cplx *b, cplx *u, int k)
{
    or_mg *g = p;
    int dim = g->dim, L = g->nlev - 1;
    long N0 = npts(dim, g->m[0]);
    if (L == 0) {                                  /* one level: exact solve */
        memcpy(u, b, (size_t)N0 * sizeof(cplx));
        or_lu_solve(N0, g->LU, g->piv, u);
        return;
    }
    cplx *fb[OR_MAXLEV], *fu[OR_MAXLEV];
    fb[0] = (cplx *)b;
    for (int l = 1; l <= L; ++l) {
        long N = npts(dim, g->m[l]);
        fb[l] = malloc((size_t)N * sizeof(cplx));
        fu[l] = calloc((size_t)N, sizeof(cplx));
        or_inject(dim, g->m[l - 1], fb[l - 1], fb[l]);            /* b_l = b_{l-1} at coarse nodes */
    }
    memcpy(fu[L], fb[L], (size_t)npts(dim, g->m[L]) * sizeof(cplx));
    or_lu_solve(npts(dim, g->m[L]), g->LU, g->piv, fu[L]);          /* exact on the coarsest */
    for (int l = L - 1; l >= 1; --l) {
        or_prolong_add(dim, g->m[l + 1], fu[l + 1], fu[l]);          /* u_l = P u_{l+1} (fu[l] = 0) */
        for (int c = 0; c < k; ++c) vcycle(g, l, fb[l], fu[l]);      /* k V-cycles on level l */
    }
    memset(u, 0, (size_t)N0 * sizeof(cplx));
    or_prolong_add(dim, g->m[1], fu[1], u);                          /* finest initial guess */
    for (int l = 1; l <= L; ++l) { free(fb[l]); free(fu[l]); }
}

static double norm2(long N, const cplx *v)
{
    double s = 0.0;
    for (long j = 0; j < N; ++j) s += creal(v[j]) * creal(v[j]) + cimag(v[j]) * cimag(v[j]);
    return sqrt(s);
}

/* Solve A u = b by repeated V-cycles from the guess in u.  Stops when
 * ||b - A u||_2 / ||b||_2 <= tol (residual-reduction tolerance, Sec. 4);
 * hist[k] = ||r_k||_2 for k = 0..cycles.  Returns 0 on convergence, 4 when
 * max_cycles is exceeded or the residual grows on 3 consecutive cycles.
 * A zero right-hand side returns u = 0 after 0 cycles. */
int or_mg_solve(void *p, const cplx *b, cplx *u, double tol, int max_cycles,
                double *hist, int *cycles)
{
    or_mg *g = p;
    long N = npts(g->dim, g->m[0]);
    double bn = norm2(N, b);
    *cycles = 0;
    if (bn == 0.0) {
        memset(u, 0, (size_t)N * sizeof(cplx));
        if (hist) hist[0] = 0.0;
        return 0;
    }
    or_residual(g->dim, g->m[0], g->h[0], g->gamma, g->kappa[0], b, u, g->r[0]);
    double rn = norm2(N, g->r[0]);
    if (hist) hist[0] = rn;
    if (rn / bn <= tol) return 0;
    int grow = 0;
    for (int k = 1; k <= max_cycles; ++k) {
        vcycle(g, 0, b, u);
        or_residual(g->dim, g->m[0], g->h[0], g->gamma, g->kappa[0], b, u, g->r[0]);
        double rk = norm2(N, g->r[0]);
        if (hist) hist[k] = rk;
        *cycles = k;
        if (rk / bn <= tol) return 0;
        grow = (rk >= rn) ? grow + 1 : 0;
        if (grow >= 3) return 4;
        rn = rk;
    }
    return 4;
}

/* ------------------------------------------------------------------ */
/* Right-hand side and far field                                       */
/* ------------------------------------------------------------------ */

static double coord(const double *lo, const double *h, int k, long i0)
{
    return lo[k] + (double)(i0 + 1) * h[k];   /* i0 = 0-based interior index */
}

/* b_j = q_j u_in(z_j), u_in(z) = exp(i k0 eta.z), z = e^{ig} x, with the
 * contrast q_j = k^2(z_j) - k0^2 = k0^2 chi(z_j) (Sec. 2.1 and
 * eq. helmholtz_cc).  The contrast is an input in its own right: forming it
 * as k^2 - k0^2 would cancel where chi is small, which is exactly where the
 * contour kernel is exponentially large (Sec. 3.3, last paragraph). */
void or_rhs_plane_wave(int dim, const long *m, const double *lo, const double *h,
                       double gamma, double k0, const cplx *q,
                       const double *eta, cplx *b)
{
    long e[3];
    extents(dim, m, e);
    cplx rot = cexp(I * gamma);
    #pragma omp parallel for schedule(static)
    for (long iz = 0; iz < e[2]; ++iz)
        for (long iy = 0; iy < e[1]; ++iy)
            for (long ix = 0; ix < e[0]; ++ix) {
                long j = ix + e[0] * (iy + e[1] * iz);
                double ex = eta[0] * coord(lo, h, 0, ix);
                if (dim >= 2) ex += eta[1] * coord(lo, h, 1, iy);
                if (dim >= 3) ex += eta[2] * coord(lo, h, 2, iz);
                cplx uin = cexp(I * k0 * rot * ex);
                b[j] = q[j] * uin;
            }
}

/* b_j = q_j exp(i k0 cos(gamma) eta.x_j): the phase of the incoming wave
 * along the real coordinates without the contour's growth factor
 * exp(-k0 sin(gamma) eta.x) -- a bounded right-hand side with the
 * oscillation of eq. helmholtz_cc, for solves at wavenumbers where the
 * contour plane wave exceeds the double range. */
void or_rhs_phase(int dim, const long *m, const double *lo, const double *h,
                  double gamma, double k0, const cplx *q,
                  const double *eta, cplx *b)
{
    long e[3];
    extents(dim, m, e);
    const double kc = k0 * cos(gamma);
    #pragma omp parallel for schedule(static)
    for (long iz = 0; iz < e[2]; ++iz)
        for (long iy = 0; iy < e[1]; ++iy)
            for (long ix = 0; ix < e[0]; ++ix) {
                long j = ix + e[0] * (iy + e[1] * iz);
                double ex = eta[0] * coord(lo, h, 0, ix);
                if (dim >= 2) ex += eta[1] * coord(lo, h, 1, iy);
                if (dim >= 3) ex += eta[2] * coord(lo, h, 2, iz);
                b[j] = q[j] * cexp(I * kc * ex);
            }
}

/* Far-field integrand s_j = q_j (u_in(z_j) + u_j): the source and the
 * scattered wave together, g = k0^2 chi (u_in + u) of eq. FFmap, i.e. the
 * integrands of eq. i1 and eq. i2 summed. */
void or_ff_integrand(int dim, const long *m, const double *lo, const double *h,
                     double gamma, double k0, const cplx *q,
                     const double *eta, const cplx *u, cplx *s)
{
    long N = npts(dim, m);
    or_rhs_plane_wave(dim, m, lo, h, gamma, k0, q, eta, s);
    if (u)
        for (long j = 0; j < N; ++j) s[j] += q[j] * u[j];
}

/* Dense far-field sum, one exponential per (direction, node):
 *   F_m = e^{i d gamma} prod h_k sum_j exp(-i k0 e^{ig} alpha_m.x_j) s_j
 * (eq. FFmap on the contour, eq. I2complex).  If absum is given it receives
 * sum_j |term_j| (times the same prefactor magnitude) per direction, from
 * which the conditioning sum|terms|/|F| follows. */
void or_ff_dense(int dim, const long *m, const double *lo, const double *h,
                 double gamma, double k0, const cplx *s, long ndirs,
                 const double *dirs, cplx *F, double *absum)
{
    long e[3];
    extents(dim, m, e);
    cplx rot = cexp(I * gamma);
    double vol = 1.0;
    for (int k = 0; k < dim; ++k) vol *= h[k];
    cplx pre = cexp(I * (double)dim * gamma) * vol;
    #pragma omp parallel for schedule(dynamic)
    for (long d = 0; d < ndirs; ++d) {
        const double *a = dirs + d * dim;
        cplx acc = 0.0;
        double aacc = 0.0;
        for (long iz = 0; iz < e[2]; ++iz)
            for (long iy = 0; iy < e[1]; ++iy)
                for (long ix = 0; ix < e[0]; ++ix) {
                    double ax = a[0] * coord(lo, h, 0, ix);
                    if (dim >= 2) ax += a[1] * coord(lo, h, 1, iy);
                    if (dim >= 3) ax += a[2] * coord(lo, h, 2, iz);
                    cplx term = cexp(-I * k0 * rot * ax) * s[ix + e[0] * (iy + e[1] * iz)];
                    acc += term;
                    aacc += cabs(term);
                }
        F[d] = pre * acc;
        if (absum) absum[d] = cabs(pre) * aacc;
    }
}

/* Same sum through the exact tensor factorisation of the kernel:
 *   exp(-i k0 e^{ig} alpha.x) = prod_k P_k(x_k),
 *   P_k(x_k) = exp(-i k0 e^{ig} alpha_k x_k),
 * summed axis by axis (x innermost), per direction. */
void or_ff_separable(int dim, const long *m, const double *lo, const double *h,
                     double gamma, double k0, const cplx *s, long ndirs,
                     const double *dirs, cplx *F)
{
    long e[3];
    extents(dim, m, e);
    cplx rot = cexp(I * gamma);
    double vol = 1.0;
    for (int k = 0; k < dim; ++k) vol *= h[k];
    cplx pre = cexp(I * (double)dim * gamma) * vol;
    #pragma omp parallel for schedule(dynamic)
    for (long d = 0; d < ndirs; ++d) {
        const double *a = dirs + d * dim;
        cplx *P[3];
        for (int k = 0; k < 3; ++k) {
            P[k] = malloc((size_t)e[k] * sizeof(cplx));
            for (long i = 0; i < e[k]; ++i)
                P[k][i] = (k < dim) ? cexp(-I * k0 * rot * a[k] * coord(lo, h, k, i)) : 1.0;
        }
        cplx accz = 0.0;
        for (long iz = 0; iz < e[2]; ++iz) {
            cplx accy = 0.0;
            for (long iy = 0; iy < e[1]; ++iy) {
                const cplx *row = s + e[0] * (iy + e[1] * iz);
                cplx accx = 0.0;
                for (long ix = 0; ix < e[0]; ++ix) accx += P[0][ix] * row[ix];
                accy += P[1][iy] * accx;
            }
            accz += P[2][iz] * accy;
        }
        F[d] = pre * accz;
        for (int k = 0; k < 3; ++k) free(P[k]);
    }
}

/* Threads the OpenMP loops of this build run on (1 without OpenMP). */
int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
