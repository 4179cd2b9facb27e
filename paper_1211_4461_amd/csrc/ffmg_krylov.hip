// ffmg_krylov.hip -- GMRES(m) smoothing steps for the multigrid V-cycle
// (Sec. 3.3: GMRES(m), m = 2 or 3, replaces weighted Jacobi and keeps the
// V-cycle stable at rotation angles near 10 degrees).
//
// One smoothing step is one restart cycle of GMRES from the current iterate:
// with r0 = b - A u, u is replaced by the u + z, z in span{r0, A r0, ...,
// A^{m-1} r0}, of least residual norm.  The basis is kept unnormalised,
// Z_0 = r0 and Z_{j+1} = A Z_j - sum_{i<=j} (d_ij / n_i) Z_i with
// d_ij = <Z_i, A Z_j> (Hermitian product, classical Gram-Schmidt: all d_ij
// of one step from one pass) and n_i = |Z_i|^2, so that v_i = Z_i / sqrt(n_i)
// is Arnoldi's orthonormal basis and H_ij = d_ij / sqrt(n_i n_j),
// H_{j+1,j} = sqrt(n_{j+1} / n_j).  The (m+1) x m least-squares problem
// min |sqrt(n_0) e_1 - H y| is solved on the device by one thread with
// complex Givens rotations (FP64), and u += sum_j (y_j / sqrt(n_j)) Z_j.
//
// Kernels (one point per thread, grid-stride, neighbours read from global
// memory): the residual with its partial norm; A Z_0 with the partial
// product <Z_0, A Z_0>; for j = 1 .. m - 1 one pass that forms Z_j from
// W = A Z_{j-1} and Z_0 .. Z_{j-1} (at the point and at its stencil
// neighbours, so that the orthogonalisation needs no pass of its own) and
// applies A to it, with the partial |Z_j|^2 and <Z_i, A Z_j>; the norm of
// Z_m (not stored); the small problem and the update.  Each pass adds the
// previous passes' partial sums itself, in block order (every block the same
// sums, so no pass waits on a one-block kernel): m + 3 launches per step.
// The reference kernel path (a pass per product and one for the
// orthogonalisation, each finished by a one-block kernel: 4 m + 3 launches)
// computes the same values in the same order, so both give the same bits.
// Partial sums are FP64 in both precisions.  A level of at most
// GM_BLOCK_MAX_POINTS points runs the whole step in one workgroup, of 256
// threads up to 1024 points and 1024 threads above (for small m with the
// vectors in registers and the stencil's input staged in LDS; the reference
// path reads and writes them in global memory).
#include "ffmg_internal.hpp"
#include "ffmg_point.hpp"

namespace ffmg {

namespace {

constexpr int GM_BLOCKS = 1024;   // grid-stride blocks (and partial sums per value)
// partial-sum slots: n_i at slot i (i <= m), d_ij (re, im) at NSLOT_D + 2 (j GMRES_MAX_M + i)
constexpr int NSLOT_D = GMRES_MAX_M + 1;

__device__ __forceinline__ void grid_coords(size_t j, int mx, int my, int &ix, int &iy, int &iz)
{
    split3(j, mx, my, ix, iy, iz);   // 32-bit divisions where j fits
}

// (A z)_j from the five (seven) stencil values, zero outside the grid: the
// point functions of every other kernel, so the bits agree with them.  zat(k)
// gives z at point k (a load, or a value formed on the fly); zc = zat(j).
template <typename T, int DIM, typename ZAt>
__device__ __forceinline__ cx<T> apply_at_f(const Stencil<T> &P, ZAt zat, cx<T> zc, cx<T> qj, size_t j)
{
    int ix, iy, iz;
    grid_coords(j, P.mx, P.my, ix, iy, iz);
    const cx<T> zero = {T(0), T(0)};
    const size_t sx = 1, sy = (size_t)P.mx, sz = (size_t)P.mx * P.my;
    cx<T> w = ix > 0 ? zat(j - sx) : zero, e = ix < P.mx - 1 ? zat(j + sx) : zero;
    cx<T> s = iy > 0 ? zat(j - sy) : zero, n = iy < P.my - 1 ? zat(j + sy) : zero;
    cx<T> L = lap_xy(P, zc, w, e, s, n);
    if (DIM == 3) {
        cx<T> d = iz > 0 ? zat(j - sz) : zero, up = iz < P.mz - 1 ? zat(j + sz) : zero;
        L = lap_add_z(P, L, zc, d, up);
    }
    return apply_point(P, L, zc, qj);
}

template <typename T, int DIM>
__device__ __forceinline__ cx<T> apply_at(const Stencil<T> &P, const cx<T> *__restrict__ z, cx<T> qj, size_t j)
{
    return apply_at_f<T, DIM>(P, [&](size_t k) { return z[k]; }, z[j], qj, j);
}

// Sums of NV doubles per thread of a 256-thread block into
// parts[slot[v] * GM_BLOCKS + blockIdx.x] (wave shuffles, then the four
// waves in order).
template <int NV>
__device__ __forceinline__ void block_partials(double (&acc)[NV], const int (&slot)[NV], double *__restrict__ parts)
{
    __shared__ double red[4][NV];
#pragma unroll
    for (int v = 0; v < NV; ++v)
        for (int off = 32; off > 0; off >>= 1) acc[v] += __shfl_down(acc[v], off, 64);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int v = 0; v < NV; ++v) red[wv][v] = acc[v];
    __syncthreads();
    if (threadIdx.x < NV) {
        const int v = threadIdx.x;
        parts[(size_t)slot[v] * GM_BLOCKS + blockIdx.x] = (red[0][v] + red[1][v]) + (red[2][v] + red[3][v]);
    }
}

// The sum over the nb blocks of the partials of slot slot0 + v into out[v],
// v < nv, in block order (lane-strided, then a wave tree; one wave per value):
// the order of k_gm_reduce.
__device__ __forceinline__ void reduce_slots(const double *parts, int nb, int slot0, int nv, double *out)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int v = wv; v < nv; v += 4) {
        double a = 0.0;
        for (int i = lane; i < nb; i += 64) a += parts[(size_t)(slot0 + v) * GM_BLOCKS + i];
        for (int off = 32; off > 0; off >>= 1) a += __shfl_down(a, off, 64);
        if (lane == 0) out[v] = a;
    }
}

// The small least-squares problem (one thread, FP64, working arrays in LDS):
// from the squared norms n[0..m] and the products d[2 (j GMRES_MAX_M + i)] =
// <Z_i, A Z_j> (re, im), the coefficients c[2 j] (re, im) of the
// unnormalised basis vectors, c_j = y_j / sqrt(n_j), zero past a breakdown.
struct GmWork {
    cd H[GMRES_MAX_M + 1][GMRES_MAX_M], g[GMRES_MAX_M + 1], cs[GMRES_MAX_M], sn[GMRES_MAX_M], y[GMRES_MAX_M];
};

__device__ void gm_solve_small(const double *n, const double *d, int m, double *c, GmWork &W)
{
    for (int j = 0; j < m; ++j) c[2 * j] = c[2 * j + 1] = 0.0;
    const double n0 = n[0];
    if (!(n0 > 0.0)) return;
    int k = m;
    for (int j = 0; j < m; ++j) {
        const double nj = n[j];
        for (int i = 0; i <= j; ++i) {
            const double sc = 1.0 / sqrt(n[i] * nj);
            W.H[i][j] = cd{d[2 * (j * GMRES_MAX_M + i)] * sc, d[2 * (j * GMRES_MAX_M + i) + 1] * sc};
        }
        for (int i = j + 1; i <= m; ++i) W.H[i][j] = cd{0.0, 0.0};
        const double nn = n[j + 1];
        W.H[j + 1][j] = cd{nn > 0.0 ? sqrt(nn / nj) : 0.0, 0.0};
        if (!(nn > 0.0)) {   // the Krylov space is invariant: solve with j + 1 columns
            k = j + 1;
            break;
        }
    }
    for (int i = 0; i <= k; ++i) W.g[i] = cd{0.0, 0.0};
    W.g[0] = cd{sqrt(n0), 0.0};
    for (int j = 0; j < k; ++j) {
        for (int i = 0; i < j; ++i) {
            cd t = W.cs[i] * W.H[i][j] + W.sn[i] * W.H[i + 1][j];
            W.H[i + 1][j] = cd{-W.sn[i].re, W.sn[i].im} * W.H[i][j] + W.cs[i] * W.H[i + 1][j];
            W.H[i][j] = t;
        }
        const cd a = W.H[j][j], cc = W.H[j + 1][j];
        const double r = sqrt(a.re * a.re + a.im * a.im + cc.re * cc.re + cc.im * cc.im);
        if (r == 0.0) {
            W.cs[j] = cd{1.0, 0.0};
            W.sn[j] = cd{0.0, 0.0};
            continue;
        }
        const double aa = sqrt(a.re * a.re + a.im * a.im);
        if (aa == 0.0) {
            W.cs[j] = cd{0.0, 0.0};
            W.sn[j] = cd{cc.re / r, -cc.im / r};
        } else {
            W.cs[j] = cd{aa / r, 0.0};
            const cd ph = {a.re / aa, a.im / aa};
            W.sn[j] = ph * cd{cc.re / r, -cc.im / r};
        }
        W.H[j][j] = W.cs[j] * a + W.sn[j] * cc;
        W.H[j + 1][j] = cd{0.0, 0.0};
        cd t = W.cs[j] * W.g[j] + W.sn[j] * W.g[j + 1];
        W.g[j + 1] = cd{-W.sn[j].re, W.sn[j].im} * W.g[j] + W.cs[j] * W.g[j + 1];
        W.g[j] = t;
    }
    for (int i = k - 1; i >= 0; --i) {
        cd t = W.g[i];
        for (int j = i + 1; j < k; ++j) t = t - W.H[i][j] * W.y[j];
        const cd dd_ = W.H[i][i];
        const double dd = dd_.re * dd_.re + dd_.im * dd_.im;
        W.y[i] = dd > 0.0 ? cd{(t.re * dd_.re + t.im * dd_.im) / dd, (t.im * dd_.re - t.re * dd_.im) / dd}
                          : cd{0.0, 0.0};
    }
    for (int j = 0; j < k; ++j) {
        const double sc = 1.0 / sqrt(n[j]);
        c[2 * j] = W.y[j].re * sc;
        c[2 * j + 1] = W.y[j].im * sc;
    }
}

// Z0 = b - A u (zero: u is 0 and is set to 0), partial n_0 = |Z0|^2.
template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_gm_resid(cx<T> *__restrict__ u, int zero, const cx<T> *__restrict__ b,
                                                  const cx<T> *__restrict__ q, cx<T> *__restrict__ z0, Stencil<T> P,
                                                  size_t N, double *__restrict__ parts, const int *__restrict__ stop)
{
    if (stop && *stop) return;
    double acc[1] = {0.0};
    for (size_t j = (size_t)blockIdx.x * 256 + threadIdx.x; j < N; j += (size_t)gridDim.x * 256) {
        cx<T> r = b[j];
        if (zero) {
            u[j] = cx<T>{T(0), T(0)};
        } else {
            cx<T> Au = apply_at<T, DIM>(P, u, q[j], j);
            r = cx<T>{r.re - Au.re, r.im - Au.im};
        }
        z0[j] = r;
        acc[0] += (double)r.re * (double)r.re + (double)r.im * (double)r.im;
    }
    const int slot[1] = {0};
    block_partials<1>(acc, slot, parts);
}

// W = A Z_j into w (the reference path: Z_{j+1}'s slot); partial d_ij =
// <Z_i, W> for i <= j (j = NJ - 1).
template <typename T, int DIM, int NJ>
__global__ __launch_bounds__(256) void k_gm_apply_dots(cx<T> *__restrict__ Z, cx<T> *__restrict__ w, size_t N,
                                                       const cx<T> *__restrict__ q, Stencil<T> P,
                                                       double *__restrict__ parts, const int *__restrict__ stop)
{
    if (stop && *stop) return;
    constexpr int j = NJ - 1;
    const cx<T> *zj = Z + (size_t)j * N;
    double acc[2 * NJ];
#pragma unroll
    for (int v = 0; v < 2 * NJ; ++v) acc[v] = 0.0;
    for (size_t p = (size_t)blockIdx.x * 256 + threadIdx.x; p < N; p += (size_t)gridDim.x * 256) {
        cx<T> Wp = apply_at<T, DIM>(P, zj, q[p], p);
        w[p] = Wp;
        const double wr = Wp.re, wi = Wp.im;
#pragma unroll
        for (int i = 0; i < NJ; ++i) {
            const cx<T> zi = Z[(size_t)i * N + p];
            acc[2 * i] += (double)zi.re * wr + (double)zi.im * wi;       // conj(z_i) w
            acc[2 * i + 1] += (double)zi.re * wi - (double)zi.im * wr;
        }
    }
    int slot[2 * NJ];
#pragma unroll
    for (int v = 0; v < 2 * NJ; ++v) slot[v] = NSLOT_D + 2 * (j * GMRES_MAX_M) + v;
    block_partials<2 * NJ>(acc, slot, parts);
}

// The coefficients of the orthogonalisation of A Z_{J-1} against Z_0 ..
// Z_{J-1}: g_i = d_{i,J-1} / n_i (zero where n_i is).
template <typename T, int J>
__device__ __forceinline__ void orth_coeffs(const double *__restrict__ S, cx<T> (&g)[J])
{
#pragma unroll
    for (int i = 0; i < J; ++i) {
        const double ni = S[i];
        const double dr = S[GM_D + 2 * ((J - 1) * GMRES_MAX_M + i)], di = S[GM_D + 2 * ((J - 1) * GMRES_MAX_M + i) + 1];
        g[i] = cx<T>{T(ni > 0.0 ? dr / ni : 0.0), T(ni > 0.0 ? di / ni : 0.0)};
    }
}

// Z_J = W - sum_{i<J} g_i Z_i at point p (W = A Z_{J-1}).
template <typename T, int J>
__device__ __forceinline__ cx<T> orth_at(const cx<T> *__restrict__ W, const cx<T> *__restrict__ Z, size_t N,
                                         const cx<T> (&g)[J], size_t p)
{
    cx<T> v = W[p];
#pragma unroll
    for (int i = 0; i < J; ++i) {
        const cx<T> zi = Z[(size_t)i * N + p];
        v = cx<T>{v.re - (g[i].re * zi.re - g[i].im * zi.im), v.im - (g[i].re * zi.im + g[i].im * zi.re)};
    }
    return v;
}

// The scalars a fused pass needs to orthogonalise A Z_{J-1} (the previous
// passes' results), into the block's copy Sl of the S layout: n_i (i < J - 1)
// from S, where the first block of an earlier pass left them; n_{J-1} and
// d_{i,J-1} (i < J) summed from the previous passes' partials in the order of
// k_gm_reduce (every block sums them; the first block also stores them in S
// for the later passes).
template <int J>
__device__ __forceinline__ void step_scalars(const double *__restrict__ parts, int nb, double *__restrict__ S,
                                             double *Sl)
{
    constexpr int dcol = GM_D + 2 * ((J - 1) * GMRES_MAX_M);
    if (threadIdx.x < J - 1) Sl[threadIdx.x] = S[threadIdx.x];
    reduce_slots(parts, nb, J - 1, 1, Sl + (J - 1));
    reduce_slots(parts, nb, NSLOT_D + 2 * ((J - 1) * GMRES_MAX_M), 2 * J, Sl + dcol);
    __syncthreads();
    if (blockIdx.x == 0) {
        if (threadIdx.x == 0) S[J - 1] = Sl[J - 1];
        if (threadIdx.x < 2 * J) S[dcol + threadIdx.x] = Sl[dcol + threadIdx.x];
    }
}

// One pass for 1 <= J < m: Z_J = A Z_{J-1} - sum_{i<J} g_i Z_i, formed from
// wprev = A Z_{J-1} at the point and its stencil neighbours and stored; wout
// = A Z_J; the partial |Z_J|^2 and <Z_i, A Z_J> (i <= J).  The values and
// partial sums of k_gm_orth<J> followed by k_gm_apply_dots<J + 1>.
template <typename T, int DIM, int J>
__global__ __launch_bounds__(256) void k_gm_orth_apply(cx<T> *__restrict__ Z, const cx<T> *__restrict__ wprev,
                                                       cx<T> *__restrict__ wout, size_t N,
                                                       const cx<T> *__restrict__ q, Stencil<T> P,
                                                       double *__restrict__ S, double *__restrict__ parts,
                                                       const int *__restrict__ stop)
{
    if (stop && *stop) return;
    __shared__ double Sl[GM_S];
    step_scalars<J>(parts, gridDim.x, S, Sl);
    cx<T> g[J];
    orth_coeffs<T, J>(Sl, g);
    cx<T> *zJ = Z + (size_t)J * N;
    constexpr int NV = 1 + 2 * (J + 1);   // |Z_J|^2, then <Z_i, A Z_J> (re, im) for i <= J
    double acc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = 0.0;
    for (size_t p = (size_t)blockIdx.x * 256 + threadIdx.x; p < N; p += (size_t)gridDim.x * 256) {
        const cx<T> zc = orth_at<T, J>(wprev, Z, N, g, p);
        const cx<T> Wp = apply_at_f<T, DIM>(P, [&](size_t k) { return orth_at<T, J>(wprev, Z, N, g, k); }, zc, q[p], p);
        zJ[p] = zc;
        wout[p] = Wp;
        acc[0] += (double)zc.re * (double)zc.re + (double)zc.im * (double)zc.im;
        const double wr = Wp.re, wi = Wp.im;
#pragma unroll
        for (int i = 0; i <= J; ++i) {
            const cx<T> zi = (i < J) ? Z[(size_t)i * N + p] : zc;
            acc[1 + 2 * i] += (double)zi.re * wr + (double)zi.im * wi;
            acc[2 + 2 * i] += (double)zi.re * wi - (double)zi.im * wr;
        }
    }
    int slot[NV];
    slot[0] = J;
#pragma unroll
    for (int v = 1; v < NV; ++v) slot[v] = NSLOT_D + 2 * (J * GMRES_MAX_M) + (v - 1);
    block_partials<NV>(acc, slot, parts);
}

// The last Arnoldi vector's partial norm: n_M = |A Z_{M-1} - sum_{i<M} g_i
// Z_i|^2 (the vector itself is not needed).
template <typename T, int M>
__global__ __launch_bounds__(256) void k_gm_orth_norm(const cx<T> *__restrict__ Z, const cx<T> *__restrict__ wprev,
                                                      size_t N, double *__restrict__ S, double *__restrict__ parts,
                                                      const int *__restrict__ stop)
{
    if (stop && *stop) return;
    __shared__ double Sl[GM_S];
    step_scalars<M>(parts, gridDim.x, S, Sl);
    cx<T> g[M];
    orth_coeffs<T, M>(Sl, g);
    double acc[1] = {0.0};
    for (size_t p = (size_t)blockIdx.x * 256 + threadIdx.x; p < N; p += (size_t)gridDim.x * 256) {
        const cx<T> v = orth_at<T, M>(wprev, Z, N, g, p);
        acc[0] += (double)v.re * (double)v.re + (double)v.im * (double)v.im;
    }
    const int slot[1] = {M};
    block_partials<1>(acc, slot, parts);
}

// The small problem and the update u += sum_j c_j Z_j in one pass: every
// block sums n_M from the partials, takes the other scalars from S and solves
// the small problem (the first block also stores n_M and the coefficients).
template <typename T, int M>
__global__ __launch_bounds__(256) void k_gm_solve_update(cx<T> *__restrict__ u, const cx<T> *__restrict__ Z,
                                                         size_t N, double *__restrict__ S,
                                                         const double *__restrict__ parts,
                                                         const int *__restrict__ stop)
{
    if (stop && *stop) return;
    __shared__ double Sl[GM_S];
    __shared__ GmWork W;
    if (threadIdx.x < M) Sl[threadIdx.x] = S[threadIdx.x];
    for (int t = threadIdx.x; t < 2 * M * GMRES_MAX_M; t += 256) Sl[GM_D + t] = S[GM_D + t];
    reduce_slots(parts, gridDim.x, M, 1, Sl + M);
    __syncthreads();
    if (threadIdx.x == 0) gm_solve_small(Sl, Sl + GM_D, M, Sl + GM_C, W);
    __syncthreads();
    if (blockIdx.x == 0) {
        if (threadIdx.x == 0) S[M] = Sl[M];
        if (threadIdx.x < 2 * M) S[GM_C + threadIdx.x] = Sl[GM_C + threadIdx.x];
    }
    cx<T> c[M];
#pragma unroll
    for (int j = 0; j < M; ++j) c[j] = cx<T>{T(Sl[GM_C + 2 * j]), T(Sl[GM_C + 2 * j + 1])};
    for (size_t p = (size_t)blockIdx.x * 256 + threadIdx.x; p < N; p += (size_t)gridDim.x * 256) {
        cx<T> v = u[p];
#pragma unroll
        for (int j = 0; j < M; ++j) {
            const cx<T> zj = Z[(size_t)j * N + p];
            v = cx<T>{v.re + (c[j].re * zj.re - c[j].im * zj.im), v.im + (c[j].re * zj.im + c[j].im * zj.re)};
        }
        u[p] = v;
    }
}

// Z_{j+1} = W - sum_{i<=j} (d_ij / n_i) Z_i in place, partial |Z_{j+1}|^2.
template <typename T, int NJ>
__global__ __launch_bounds__(256) void k_gm_orth(cx<T> *__restrict__ Z, size_t N, const double *__restrict__ S,
                                                 double *__restrict__ parts, const int *__restrict__ stop)
{
    if (stop && *stop) return;
    cx<T> g[NJ];
    orth_coeffs<T, NJ>(S, g);
    cx<T> *w = Z + (size_t)NJ * N;
    double acc[1] = {0.0};
    for (size_t p = (size_t)blockIdx.x * 256 + threadIdx.x; p < N; p += (size_t)gridDim.x * 256) {
        const cx<T> v = orth_at<T, NJ>(w, Z, N, g, p);
        w[p] = v;
        acc[0] += (double)v.re * (double)v.re + (double)v.im * (double)v.im;
    }
    const int slot[1] = {NJ};
    block_partials<1>(acc, slot, parts);
}

// out[v] = sum over the nb blocks of the partials of slot0 + v, in block order
// (one block, one wave per value), and likewise out1[v] from slot1 + v for
// v < nv1; solve_m > 0: then the small problem.
__global__ __launch_bounds__(256) void k_gm_reduce(const double *__restrict__ parts, int nb, int slot0, int nv,
                                                   double *__restrict__ out, int solve_m, double *__restrict__ S,
                                                   const int *__restrict__ stop, int slot1 = 0, int nv1 = 0,
                                                   double *__restrict__ out1 = nullptr)
{
    if (stop && *stop) return;
    reduce_slots(parts, nb, slot0, nv, out);
    if (nv1 > 0) reduce_slots(parts, nb, slot1, nv1, out1);
    if (solve_m > 0) {
        __shared__ GmWork W;
        __syncthreads();
        if (threadIdx.x == 0) gm_solve_small(S, S + GM_D, solve_m, S + GM_C, W);
    }
}

// u += sum_j c_j Z_j.
template <typename T, int M>
__global__ __launch_bounds__(256) void k_gm_update(cx<T> *__restrict__ u, const cx<T> *__restrict__ Z, size_t N,
                                                   const double *__restrict__ S, const int *__restrict__ stop)
{
    if (stop && *stop) return;
    cx<T> c[M];
#pragma unroll
    for (int j = 0; j < M; ++j) c[j] = cx<T>{T(S[GM_C + 2 * j]), T(S[GM_C + 2 * j + 1])};
    for (size_t p = (size_t)blockIdx.x * 256 + threadIdx.x; p < N; p += (size_t)gridDim.x * 256) {
        cx<T> v = u[p];
#pragma unroll
        for (int j = 0; j < M; ++j) {
            const cx<T> zj = Z[(size_t)j * N + p];
            v = cx<T>{v.re + (c[j].re * zj.re - c[j].im * zj.im), v.im + (c[j].re * zj.im + c[j].im * zj.re)};
        }
        u[p] = v;
    }
}

// A whole GMRES(M) step on a small level in one workgroup of BT threads: the
// same passes, separated by workgroup barriers (global memory written before
// a barrier is seen after it within the workgroup), the sums reduced in LDS
// and the small solve by thread 0.
constexpr int GM_BLOCK_THREADS = 1024;
constexpr int GM_SMALL_THREADS = 256;
constexpr size_t GM_SMALL_POINTS = 1024;   // = GM_REG_PTS * GM_SMALL_THREADS
constexpr size_t GM_BLOCK_MAX_POINTS = 4096;

template <int NV, int BT>
__device__ __forceinline__ void block_reduce_bt(double (&acc)[NV], double *out, double (*red)[2 * GMRES_MAX_M])
{
#pragma unroll
    for (int v = 0; v < NV; ++v)
        for (int off = 32; off > 0; off >>= 1) acc[v] += __shfl_down(acc[v], off, 64);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int v = 0; v < NV; ++v) red[wv][v] = acc[v];
    __syncthreads();
    if (threadIdx.x < NV) {
        double a = 0.0;
        for (int w_ = 0; w_ < BT / 64; ++w_) a += red[w_][threadIdx.x];
        out[threadIdx.x] = a;
    }
    __syncthreads();
}

template <typename T, int DIM, int NJ, int BT>
__device__ __forceinline__ void gm_block_arnoldi(cx<T> *__restrict__ Z, size_t N, const cx<T> *__restrict__ q,
                                                 const Stencil<T> &P, double *n, double *d,
                                                 double (*red)[2 * GMRES_MAX_M])
{
    constexpr int j = NJ - 1;
    const cx<T> *zj = Z + (size_t)j * N;
    cx<T> *w = Z + (size_t)NJ * N;
    double acc[2 * NJ];
#pragma unroll
    for (int v = 0; v < 2 * NJ; ++v) acc[v] = 0.0;
    for (size_t p = threadIdx.x; p < N; p += BT) {
        cx<T> Wp = apply_at<T, DIM>(P, zj, q[p], p);
        w[p] = Wp;
        const double wr = Wp.re, wi = Wp.im;
#pragma unroll
        for (int i = 0; i < NJ; ++i) {
            const cx<T> zi = Z[(size_t)i * N + p];
            acc[2 * i] += (double)zi.re * wr + (double)zi.im * wi;
            acc[2 * i + 1] += (double)zi.re * wi - (double)zi.im * wr;
        }
    }
    block_reduce_bt<2 * NJ, BT>(acc, d + 2 * (j * GMRES_MAX_M), red);
    cx<T> g[NJ];
#pragma unroll
    for (int i = 0; i < NJ; ++i) {
        const double ni = n[i];
        const double dr = d[2 * (j * GMRES_MAX_M + i)], di = d[2 * (j * GMRES_MAX_M + i) + 1];
        g[i] = cx<T>{T(ni > 0.0 ? dr / ni : 0.0), T(ni > 0.0 ? di / ni : 0.0)};
    }
    double nacc[1] = {0.0};
    for (size_t p = threadIdx.x; p < N; p += BT) {
        cx<T> v = w[p];
#pragma unroll
        for (int i = 0; i < NJ; ++i) {
            const cx<T> zi = Z[(size_t)i * N + p];
            v = cx<T>{v.re - (g[i].re * zi.re - g[i].im * zi.im), v.im - (g[i].re * zi.im + g[i].im * zi.re)};
        }
        w[p] = v;
        nacc[0] += (double)v.re * (double)v.re + (double)v.im * (double)v.im;
    }
    block_reduce_bt<1, BT>(nacc, n + NJ, red);
}

template <typename T, int DIM, int NJ, int M, int BT>
__device__ __forceinline__ void gm_block_arnoldi_all(cx<T> *Z, size_t N, const cx<T> *q, const Stencil<T> &P,
                                                     double *n, double *d, double (*red)[2 * GMRES_MAX_M])
{
    gm_block_arnoldi<T, DIM, NJ, BT>(Z, N, q, P, n, d, red);
    if constexpr (NJ < M) gm_block_arnoldi_all<T, DIM, NJ + 1, M, BT>(Z, N, q, P, n, d, red);
}

template <typename T, int DIM, int M, int BT>
__global__ __launch_bounds__(BT) void k_gm_step_block(const cx<T> *__restrict__ b, const cx<T> *__restrict__ q,
                                                        cx<T> *__restrict__ u, int zero, cx<T> *__restrict__ Z,
                                                        Stencil<T> P, size_t N, const int *__restrict__ stop)
{
    if (stop && *stop) return;
    __shared__ double red[BT / 64][2 * GMRES_MAX_M];
    __shared__ double n[GMRES_MAX_M + 1], d[2 * GMRES_MAX_M * GMRES_MAX_M], c[2 * GMRES_MAX_M];
    __shared__ GmWork W;
    double acc[1] = {0.0};
    for (size_t p = threadIdx.x; p < N; p += BT) {
        cx<T> r = b[p];
        if (zero) {
            u[p] = cx<T>{T(0), T(0)};
        } else {
            cx<T> Au = apply_at<T, DIM>(P, u, q[p], p);
            r = cx<T>{r.re - Au.re, r.im - Au.im};
        }
        Z[p] = r;
        acc[0] += (double)r.re * (double)r.re + (double)r.im * (double)r.im;
    }
    block_reduce_bt<1, BT>(acc, n, red);
    gm_block_arnoldi_all<T, DIM, 1, M, BT>(Z, N, q, P, n, d, red);
    if (threadIdx.x == 0) gm_solve_small(n, d, M, c, W);
    __syncthreads();
    cx<T> cc[M];
#pragma unroll
    for (int j = 0; j < M; ++j) cc[j] = cx<T>{T(c[2 * j]), T(c[2 * j + 1])};
    for (size_t p = threadIdx.x; p < N; p += BT) {
        cx<T> v = u[p];
#pragma unroll
        for (int j = 0; j < M; ++j) {
            const cx<T> zj = Z[(size_t)j * N + p];
            v = cx<T>{v.re + (cc[j].re * zj.re - cc[j].im * zj.im), v.im + (cc[j].re * zj.im + cc[j].im * zj.re)};
        }
        u[p] = v;
    }
}

// The same step with the level's vectors held in registers (thread t holds
// the points p = t + BT k, k < GM_REG_PTS) and only the vector that A is
// applied to staged in LDS (dynamic shared memory, N values): no global
// traffic inside the step but the loads of b, q, u and the store of u.  The
// values, the sums and their order are those of k_gm_step_block.
constexpr int GM_REG_PTS = (int)(GM_BLOCK_MAX_POINTS / GM_BLOCK_THREADS);   // also for the small blocks

template <typename T, int DIM, int NJ, int M, int BT>
__device__ __forceinline__ void gm_reg_arnoldi(cx<T> (&Z)[M + 1][GM_REG_PTS], const cx<T> (&qv)[GM_REG_PTS],
                                               cx<T> *stage, const Stencil<T> &P, int N, double *n, double *d,
                                               double (*red)[2 * GMRES_MAX_M])
{
    constexpr int j = NJ - 1;
    // the reduction before ended with a barrier: every thread is past its reads of the stage
#pragma unroll
    for (int k = 0; k < GM_REG_PTS; ++k) {
        const int p = (int)threadIdx.x + BT * k;
        if (p < N) stage[p] = Z[j][k];
    }
    __syncthreads();
    double acc[2 * NJ];
#pragma unroll
    for (int v = 0; v < 2 * NJ; ++v) acc[v] = 0.0;
#pragma unroll
    for (int k = 0; k < GM_REG_PTS; ++k) {
        const int p = (int)threadIdx.x + BT * k;
        if (p < N) {
            const cx<T> Wp = apply_at_f<T, DIM>(P, [&](size_t i) { return stage[i]; }, Z[j][k], qv[k], (size_t)p);
            Z[NJ][k] = Wp;
            const double wr = Wp.re, wi = Wp.im;
#pragma unroll
            for (int i = 0; i < NJ; ++i) {
                const cx<T> zi = Z[i][k];
                acc[2 * i] += (double)zi.re * wr + (double)zi.im * wi;
                acc[2 * i + 1] += (double)zi.re * wi - (double)zi.im * wr;
            }
        }
    }
    block_reduce_bt<2 * NJ, BT>(acc, d + 2 * (j * GMRES_MAX_M), red);
    cx<T> g[NJ];
#pragma unroll
    for (int i = 0; i < NJ; ++i) {
        const double ni = n[i];
        const double dr = d[2 * (j * GMRES_MAX_M + i)], di = d[2 * (j * GMRES_MAX_M + i) + 1];
        g[i] = cx<T>{T(ni > 0.0 ? dr / ni : 0.0), T(ni > 0.0 ? di / ni : 0.0)};
    }
    double nacc[1] = {0.0};
#pragma unroll
    for (int k = 0; k < GM_REG_PTS; ++k) {
        const int p = (int)threadIdx.x + BT * k;
        if (p < N) {
            cx<T> v = Z[NJ][k];
#pragma unroll
            for (int i = 0; i < NJ; ++i) {
                const cx<T> zi = Z[i][k];
                v = cx<T>{v.re - (g[i].re * zi.re - g[i].im * zi.im), v.im - (g[i].re * zi.im + g[i].im * zi.re)};
            }
            Z[NJ][k] = v;
            nacc[0] += (double)v.re * (double)v.re + (double)v.im * (double)v.im;
        }
    }
    block_reduce_bt<1, BT>(nacc, n + NJ, red);
    if constexpr (NJ < M) gm_reg_arnoldi<T, DIM, NJ + 1, M, BT>(Z, qv, stage, P, N, n, d, red);
}

template <typename T, int DIM, int M, int BT>
__global__ __launch_bounds__(BT) void k_gm_step_reg(const cx<T> *__restrict__ b, const cx<T> *__restrict__ q,
                                                      cx<T> *__restrict__ u, int zero, Stencil<T> P, int N,
                                                      const int *__restrict__ stop)
{
    if (stop && *stop) return;
    extern __shared__ __attribute__((aligned(16))) unsigned char gm_stage_raw[];
    cx<T> *stage = reinterpret_cast<cx<T> *>(gm_stage_raw);
    __shared__ double red[BT / 64][2 * GMRES_MAX_M];
    __shared__ double n[GMRES_MAX_M + 1], d[2 * GMRES_MAX_M * GMRES_MAX_M], c[2 * GMRES_MAX_M];
    __shared__ GmWork W;
    const cx<T> zc = {T(0), T(0)};
    cx<T> qv[GM_REG_PTS], uv[GM_REG_PTS], Z[M + 1][GM_REG_PTS];
#pragma unroll
    for (int k = 0; k < GM_REG_PTS; ++k) {
        const int p = (int)threadIdx.x + BT * k;
        qv[k] = uv[k] = zc;
#pragma unroll
        for (int j = 0; j <= M; ++j) Z[j][k] = zc;
        if (p < N) {
            qv[k] = q[p];
            if (!zero) {
                uv[k] = u[p];
                stage[p] = uv[k];
            }
        }
    }
    __syncthreads();
    double acc[1] = {0.0};
#pragma unroll
    for (int k = 0; k < GM_REG_PTS; ++k) {
        const int p = (int)threadIdx.x + BT * k;
        if (p < N) {
            cx<T> r = b[p];
            if (!zero) {
                const cx<T> Au = apply_at_f<T, DIM>(P, [&](size_t i) { return stage[i]; }, uv[k], qv[k], (size_t)p);
                r = cx<T>{r.re - Au.re, r.im - Au.im};
            }
            Z[0][k] = r;
            acc[0] += (double)r.re * (double)r.re + (double)r.im * (double)r.im;
        }
    }
    block_reduce_bt<1, BT>(acc, n, red);
    gm_reg_arnoldi<T, DIM, 1, M, BT>(Z, qv, stage, P, N, n, d, red);
    if (threadIdx.x == 0) gm_solve_small(n, d, M, c, W);
    __syncthreads();
    cx<T> cc[M];
#pragma unroll
    for (int j = 0; j < M; ++j) cc[j] = cx<T>{T(c[2 * j]), T(c[2 * j + 1])};
#pragma unroll
    for (int k = 0; k < GM_REG_PTS; ++k) {
        const int p = (int)threadIdx.x + BT * k;
        if (p < N) {
            cx<T> v = uv[k];
#pragma unroll
            for (int j = 0; j < M; ++j) {
                const cx<T> zj = Z[j][k];
                v = cx<T>{v.re + (cc[j].re * zj.re - cc[j].im * zj.im), v.im + (cc[j].re * zj.im + cc[j].im * zj.re)};
            }
            u[p] = v;
        }
    }
}

// Whether a step on a level of at most GM_BLOCK_MAX_POINTS points keeps its
// vectors in registers: small m (the m + 1 vectors, four points each, within
// the 128 registers a thread of a 1024-thread workgroup has).
template <typename T, int M>
constexpr bool gm_reg_step() { return sizeof(T) == 4 ? M <= 4 : M <= 3; }

template <typename T, int DIM, int M, int BT>
static void launch_step_reg(const cx<T> *b, const cx<T> *q, cx<T> *u, bool zero, const Stencil<T> &P, size_t N,
                            hipStream_t s, const int *stop)
{
    static const bool attr_set = [] {
        (void)hipFuncSetAttribute((const void *)k_gm_step_reg<T, DIM, M, BT>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)(GM_REG_PTS * BT * sizeof(cx<T>)));
        return true;
    }();
    (void)attr_set;
    hipLaunchKernelGGL((k_gm_step_reg<T, DIM, M, BT>), dim3(1), dim3(BT), N * sizeof(cx<T>), s, b, q, u, zero ? 1 : 0,
                       P, (int)N, stop);
}

template <typename T, int DIM, int NJ, int M>
void launch_arnoldi_all(cx<T> *Z, size_t N, const cx<T> *q, const Stencil<T> &P, double *S, double *parts, int nb,
                        hipStream_t s, const int *stop)
{
    constexpr int j = NJ - 1;
    hipLaunchKernelGGL((k_gm_apply_dots<T, DIM, NJ>), dim3(nb), dim3(256), 0, s, Z, Z + (size_t)NJ * N, N, q, P,
                       parts, stop);
    hipLaunchKernelGGL(k_gm_reduce, dim3(1), dim3(256), 0, s, parts, nb, NSLOT_D + 2 * (j * GMRES_MAX_M), 2 * NJ,
                       S + GM_D + 2 * (j * GMRES_MAX_M), 0, S, stop, 0, 0, nullptr);
    hipLaunchKernelGGL((k_gm_orth<T, NJ>), dim3(nb), dim3(256), 0, s, Z, N, S, parts, stop);
    hipLaunchKernelGGL(k_gm_reduce, dim3(1), dim3(256), 0, s, parts, nb, NJ, 1, S + NJ, NJ == M ? M : 0, S, stop, 0, 0,
                       nullptr);
    if constexpr (NJ < M) launch_arnoldi_all<T, DIM, NJ + 1, M>(Z, N, q, P, S, parts, nb, s, stop);
}

// The fused passes for J = 1 .. M - 1 (A Z_{J-1} in slot M + ((J - 1) & 1),
// A Z_J into the other of the two).
template <typename T, int DIM, int J, int M>
void launch_orth_apply_all(cx<T> *Z, size_t N, const cx<T> *q, const Stencil<T> &P, double *S, double *parts, int nb,
                           hipStream_t s, const int *stop)
{
    if constexpr (J < M) {
        hipLaunchKernelGGL((k_gm_orth_apply<T, DIM, J>), dim3(nb), dim3(256), 0, s, Z,
                           Z + (size_t)(M + ((J - 1) & 1)) * N, Z + (size_t)(M + (J & 1)) * N, N, q, P, S, parts,
                           stop);
        launch_orth_apply_all<T, DIM, J + 1, M>(Z, N, q, P, S, parts, nb, s, stop);
    }
}

template <typename T, int DIM, int M>
void launch_step_m(const LevelGeom &g, const Stencil<T> &P, const cx<T> *b, const cx<T> *q, cx<T> *u, bool zero,
                   cx<T> *Z, double *S, double *parts, hipStream_t s, const int *stop, bool fused)
{
    const size_t N = g.N();
    if (N <= GM_BLOCK_MAX_POINTS) {   // small level: the whole step in one workgroup
        // levels of at most GM_SMALL_POINTS points in a 256-thread workgroup (its
        // block-wide sums take 4 waves instead of 16)
        const bool small = N <= GM_SMALL_POINTS;
        if constexpr (gm_reg_step<T, M>()) {
            if (fused) {
                if (small) launch_step_reg<T, DIM, M, GM_SMALL_THREADS>(b, q, u, zero, P, N, s, stop);
                else launch_step_reg<T, DIM, M, GM_BLOCK_THREADS>(b, q, u, zero, P, N, s, stop);
                return;
            }
        }
        if (small)
            hipLaunchKernelGGL((k_gm_step_block<T, DIM, M, GM_SMALL_THREADS>), dim3(1), dim3(GM_SMALL_THREADS), 0, s,
                               b, q, u, zero ? 1 : 0, Z, P, N, stop);
        else
            hipLaunchKernelGGL((k_gm_step_block<T, DIM, M, GM_BLOCK_THREADS>), dim3(1), dim3(GM_BLOCK_THREADS), 0, s,
                               b, q, u, zero ? 1 : 0, Z, P, N, stop);
        return;
    }
    const int nb = (int)std::min<size_t>((N + 255) / 256, GM_BLOCKS);
    hipLaunchKernelGGL((k_gm_resid<T, DIM>), dim3(nb), dim3(256), 0, s, u, zero ? 1 : 0, b, q, Z, P, N, parts, stop);
    if (fused) {
        hipLaunchKernelGGL((k_gm_apply_dots<T, DIM, 1>), dim3(nb), dim3(256), 0, s, Z, Z + (size_t)M * N, N, q, P,
                           parts, stop);
        launch_orth_apply_all<T, DIM, 1, M>(Z, N, q, P, S, parts, nb, s, stop);
        hipLaunchKernelGGL((k_gm_orth_norm<T, M>), dim3(nb), dim3(256), 0, s, Z, Z + (size_t)(M + ((M - 1) & 1)) * N,
                           N, S, parts, stop);
        hipLaunchKernelGGL((k_gm_solve_update<T, M>), dim3(nb), dim3(256), 0, s, u, Z, N, S, parts, stop);
        return;
    }
    hipLaunchKernelGGL(k_gm_reduce, dim3(1), dim3(256), 0, s, parts, nb, 0, 1, S, 0, S, stop, 0, 0, nullptr);
    launch_arnoldi_all<T, DIM, 1, M>(Z, N, q, P, S, parts, nb, s, stop);
    hipLaunchKernelGGL((k_gm_update<T, M>), dim3(nb), dim3(256), 0, s, u, Z, N, S, stop);
}

template <typename T, int DIM>
void launch_step_dim(int m, const LevelGeom &g, const Stencil<T> &P, const cx<T> *b, const cx<T> *q, cx<T> *u,
                     bool zero, cx<T> *Z, double *S, double *parts, hipStream_t s, const int *stop, bool fused)
{
    switch (m) {
    case 1: launch_step_m<T, DIM, 1>(g, P, b, q, u, zero, Z, S, parts, s, stop, fused); break;
    case 2: launch_step_m<T, DIM, 2>(g, P, b, q, u, zero, Z, S, parts, s, stop, fused); break;
    case 3: launch_step_m<T, DIM, 3>(g, P, b, q, u, zero, Z, S, parts, s, stop, fused); break;
    case 4: launch_step_m<T, DIM, 4>(g, P, b, q, u, zero, Z, S, parts, s, stop, fused); break;
    case 5: launch_step_m<T, DIM, 5>(g, P, b, q, u, zero, Z, S, parts, s, stop, fused); break;
    case 6: launch_step_m<T, DIM, 6>(g, P, b, q, u, zero, Z, S, parts, s, stop, fused); break;
    case 7: launch_step_m<T, DIM, 7>(g, P, b, q, u, zero, Z, S, parts, s, stop, fused); break;
    default: launch_step_m<T, DIM, 8>(g, P, b, q, u, zero, Z, S, parts, s, stop, fused); break;
    }
}

}  // namespace

// One GMRES(m) smoothing step in place on a level: Z holds m + 2 vectors of
// N points, S the step's scalars (GM_S doubles), parts the partial sums
// (GM_PARTS doubles).  zero: u is 0 on entry (not read).  fused: the
// m + 3-launch passes, else the reference passes.
template <typename T>
void launch_gmres_step(const LevelGeom &g, const Stencil<T> &P, const cx<T> *b, const cx<T> *q, cx<T> *u, bool zero,
                       int m, cx<T> *Z, double *S, double *parts, hipStream_t s, const int *stop, bool fused)
{
    if (g.dim == 3) launch_step_dim<T, 3>(m, g, P, b, q, u, zero, Z, S, parts, s, stop, fused);
    else launch_step_dim<T, 2>(m, g, P, b, q, u, zero, Z, S, parts, s, stop, fused);
}
template void launch_gmres_step<double>(const LevelGeom &, const Stencil<double> &, const cd *, const cd *, cd *, bool,
                                        int, cd *, double *, double *, hipStream_t, const int *, bool);
template void launch_gmres_step<float>(const LevelGeom &, const Stencil<float> &, const cf *, const cf *, cf *, bool,
                                       int, cf *, double *, double *, hipStream_t, const int *, bool);

}  // namespace ffmg
