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
// memory): the residual with its partial norm; A Z_j fused with the partial
// products <Z_i, A Z_j>; the orthogonalisation with its partial norm; a
// deterministic single-block reduction after each of them; the small solve;
// the update.  Partial sums are FP64 in both precisions.  A V-cycle level is
// latency-bound here (16 launches per step for m = 3), which is the price of
// the smoother's robustness.
#include "ffmg_internal.hpp"
#include "ffmg_point.hpp"

namespace ffmg {

namespace {

constexpr int GM_BLOCKS = 1024;   // grid-stride blocks (and partial sums per value)

__device__ __forceinline__ void grid_coords(size_t j, int mx, int my, int &ix, int &iy, int &iz)
{
    ix = (int)(j % mx);
    size_t r = j / mx;
    iy = (int)(r % my);
    iz = (int)(r / my);
}

// (A z)_j from the five (seven) stencil values, zero outside the grid: the
// point functions of every other kernel, so the bits agree with them.
template <typename T, int DIM>
__device__ __forceinline__ cx<T> apply_at(const Stencil<T> &P, const cx<T> *__restrict__ z, cx<T> qj, size_t j)
{
    int ix, iy, iz;
    grid_coords(j, P.mx, P.my, ix, iy, iz);
    const cx<T> zero = {T(0), T(0)};
    const size_t sx = 1, sy = (size_t)P.mx, sz = (size_t)P.mx * P.my;
    cx<T> uc = z[j];
    cx<T> w = ix > 0 ? z[j - sx] : zero, e = ix < P.mx - 1 ? z[j + sx] : zero;
    cx<T> s = iy > 0 ? z[j - sy] : zero, n = iy < P.my - 1 ? z[j + sy] : zero;
    cx<T> L = lap_xy(P, uc, w, e, s, n);
    if (DIM == 3) {
        cx<T> d = iz > 0 ? z[j - sz] : zero, up = iz < P.mz - 1 ? z[j + sz] : zero;
        L = lap_add_z(P, L, uc, d, up);
    }
    return apply_point(P, L, uc, qj);
}

// Block sum of NV doubles per thread into parts[v * gridDim.x + blockIdx.x]
// (256 threads; wave shuffles, then the four waves in order).
template <int NV>
__device__ __forceinline__ void block_sums(double (&acc)[NV], double *__restrict__ parts)
{
    __shared__ double red[4][NV > 0 ? NV : 1];
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
        parts[(size_t)v * gridDim.x + blockIdx.x] = (red[0][v] + red[1][v]) + (red[2][v] + red[3][v]);
    }
}

// Z0 = b - A u (u null: Z0 = b), partial |Z0|^2.
template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_gm_resid(const cx<T> *__restrict__ u, const cx<T> *__restrict__ b,
                                                  const cx<T> *__restrict__ q, cx<T> *__restrict__ z0, Stencil<T> P,
                                                  size_t N, double *__restrict__ parts, const int *__restrict__ stop)
{
    if (stop && *stop) return;
    double acc[1] = {0.0};
    for (size_t j = (size_t)blockIdx.x * 256 + threadIdx.x; j < N; j += (size_t)gridDim.x * 256) {
        cx<T> r = b[j];
        if (u) {
            cx<T> Au = apply_at<T, DIM>(P, u, q[j], j);
            r = cx<T>{r.re - Au.re, r.im - Au.im};
        }
        z0[j] = r;
        acc[0] += (double)r.re * (double)r.re + (double)r.im * (double)r.im;
    }
    block_sums<1>(acc, parts);
}

// W = A Z_j into Z_{j+1}'s slot; partial <Z_i, W> for i <= j (re, im).
template <typename T, int DIM, int NJ>
__global__ __launch_bounds__(256) void k_gm_apply_dots(cx<T> *__restrict__ Z, size_t N, const cx<T> *__restrict__ q,
                                                       Stencil<T> P, double *__restrict__ parts,
                                                       const int *__restrict__ stop)
{
    if (stop && *stop) return;
    const cx<T> *zj = Z + (size_t)(NJ - 1) * N;
    cx<T> *w = Z + (size_t)NJ * N;
    double acc[2 * NJ];
#pragma unroll
    for (int v = 0; v < 2 * NJ; ++v) acc[v] = 0.0;
    for (size_t j = (size_t)blockIdx.x * 256 + threadIdx.x; j < N; j += (size_t)gridDim.x * 256) {
        cx<T> Wj = apply_at<T, DIM>(P, zj, q[j], j);
        w[j] = Wj;
        const double wr = Wj.re, wi = Wj.im;
#pragma unroll
        for (int i = 0; i < NJ; ++i) {
            const cx<T> zi = Z[(size_t)i * N + j];
            // conj(z_i) w
            acc[2 * i] += (double)zi.re * wr + (double)zi.im * wi;
            acc[2 * i + 1] += (double)zi.re * wi - (double)zi.im * wr;
        }
    }
    block_sums<2 * NJ>(acc, parts);
}

// Z_{j+1} = W - sum_{i<=j} (d_ij / n_i) Z_i in place; partial |Z_{j+1}|^2.
// S: n_i at S[i], d_ij at S[GM_D + 2 (j MAXM + i)] (re, im).
template <typename T, int NJ>
__global__ __launch_bounds__(256) void k_gm_orth(cx<T> *__restrict__ Z, size_t N, const double *__restrict__ S,
                                                 double *__restrict__ parts, const int *__restrict__ stop)
{
    if (stop && *stop) return;
    constexpr int j = NJ - 1;
    cx<T> g[NJ];
#pragma unroll
    for (int i = 0; i < NJ; ++i) {
        const double ni = S[i];
        const double dr = S[GM_D + 2 * (j * GMRES_MAX_M + i)], di = S[GM_D + 2 * (j * GMRES_MAX_M + i) + 1];
        g[i] = cx<T>{T(ni > 0.0 ? dr / ni : 0.0), T(ni > 0.0 ? di / ni : 0.0)};
    }
    cx<T> *w = Z + (size_t)NJ * N;
    double acc[1] = {0.0};
    for (size_t p = (size_t)blockIdx.x * 256 + threadIdx.x; p < N; p += (size_t)gridDim.x * 256) {
        cx<T> v = w[p];
#pragma unroll
        for (int i = 0; i < NJ; ++i) {
            const cx<T> zi = Z[(size_t)i * N + p];
            v = cx<T>{v.re - (g[i].re * zi.re - g[i].im * zi.im), v.im - (g[i].re * zi.im + g[i].im * zi.re)};
        }
        w[p] = v;
        acc[0] += (double)v.re * (double)v.re + (double)v.im * (double)v.im;
    }
    block_sums<1>(acc, parts);
}

// out[v] = sum of the nb partials of value v (one block per value, fixed order).
__global__ __launch_bounds__(256) void k_gm_reduce(const double *__restrict__ parts, int nb, double *__restrict__ out,
                                                   const int *__restrict__ stop)
{
    if (stop && *stop) return;
    const int v = blockIdx.x;
    double a = 0.0;
    for (int i = threadIdx.x; i < nb; i += 256) a += parts[(size_t)v * nb + i];
    __shared__ double red[4];
    for (int off = 32; off > 0; off >>= 1) a += __shfl_down(a, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) out[v] = (red[0] + red[1]) + (red[2] + red[3]);
}

// The small least-squares problem (one thread, FP64): coefficients of the
// unnormalised basis vectors, c_j = y_j / sqrt(n_j), zero past a breakdown.
__global__ void k_gm_small(double *__restrict__ S, int m, const int *__restrict__ stop)
{
    if (stop && *stop) return;
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    cd H[GMRES_MAX_M + 1][GMRES_MAX_M], g[GMRES_MAX_M + 1], cs[GMRES_MAX_M], sn[GMRES_MAX_M], y[GMRES_MAX_M];
    for (int j = 0; j < m; ++j) S[GM_C + 2 * j] = S[GM_C + 2 * j + 1] = 0.0;
    const double n0 = S[0];
    if (!(n0 > 0.0)) return;
    int k = m;
    for (int j = 0; j < m; ++j) {
        const double nj = S[j];
        for (int i = 0; i <= j; ++i) {
            const double ni = S[i], sc = 1.0 / sqrt(ni * nj);
            H[i][j] = cd{S[GM_D + 2 * (j * GMRES_MAX_M + i)] * sc, S[GM_D + 2 * (j * GMRES_MAX_M + i) + 1] * sc};
        }
        for (int i = j + 1; i <= m; ++i) H[i][j] = cd{0.0, 0.0};
        const double nn = S[j + 1];
        H[j + 1][j] = cd{nn > 0.0 ? sqrt(nn / nj) : 0.0, 0.0};
        if (!(nn > 0.0)) {   // the Krylov space is invariant: solve with j + 1 columns
            k = j + 1;
            break;
        }
    }
    for (int i = 0; i <= k; ++i) g[i] = cd{0.0, 0.0};
    g[0] = cd{sqrt(n0), 0.0};
    for (int j = 0; j < k; ++j) {
        for (int i = 0; i < j; ++i) {
            cd t = cs[i] * H[i][j] + sn[i] * H[i + 1][j];
            H[i + 1][j] = cd{-sn[i].re, sn[i].im} * H[i][j] + cs[i] * H[i + 1][j];
            H[i][j] = t;
        }
        const cd a = H[j][j], c = H[j + 1][j];
        const double r = sqrt(a.re * a.re + a.im * a.im + c.re * c.re + c.im * c.im);
        if (r == 0.0) {
            cs[j] = cd{1.0, 0.0};
            sn[j] = cd{0.0, 0.0};
            continue;
        }
        const double aa = sqrt(a.re * a.re + a.im * a.im);
        if (aa == 0.0) {
            cs[j] = cd{0.0, 0.0};
            sn[j] = cd{c.re / r, -c.im / r};
        } else {
            cs[j] = cd{aa / r, 0.0};
            const cd ph = {a.re / aa, a.im / aa};
            sn[j] = ph * cd{c.re / r, -c.im / r};
        }
        H[j][j] = cs[j] * a + sn[j] * c;
        H[j + 1][j] = cd{0.0, 0.0};
        cd t = cs[j] * g[j] + sn[j] * g[j + 1];
        g[j + 1] = cd{-sn[j].re, sn[j].im} * g[j] + cs[j] * g[j + 1];
        g[j] = t;
    }
    for (int i = k - 1; i >= 0; --i) {
        cd t = g[i];
        for (int j = i + 1; j < k; ++j) t = t - H[i][j] * y[j];
        const cd d = H[i][i];
        const double dd = d.re * d.re + d.im * d.im;
        y[i] = dd > 0.0 ? cd{(t.re * d.re + t.im * d.im) / dd, (t.im * d.re - t.re * d.im) / dd} : cd{0.0, 0.0};
    }
    for (int j = 0; j < k; ++j) {
        const double sc = 1.0 / sqrt(S[j]);
        S[GM_C + 2 * j] = y[j].re * sc;
        S[GM_C + 2 * j + 1] = y[j].im * sc;
    }
}

// u += sum_j c_j Z_j.
template <typename T>
__global__ __launch_bounds__(256) void k_gm_update(cx<T> *__restrict__ u, const cx<T> *__restrict__ Z, size_t N,
                                                   int m, const double *__restrict__ S, const int *__restrict__ stop)
{
    if (stop && *stop) return;
    cx<T> c[GMRES_MAX_M];
    for (int j = 0; j < m; ++j) c[j] = cx<T>{T(S[GM_C + 2 * j]), T(S[GM_C + 2 * j + 1])};
    for (size_t p = (size_t)blockIdx.x * 256 + threadIdx.x; p < N; p += (size_t)gridDim.x * 256) {
        cx<T> v = u[p];
        for (int j = 0; j < m; ++j) {
            const cx<T> zj = Z[(size_t)j * N + p];
            v = cx<T>{v.re + (c[j].re * zj.re - c[j].im * zj.im), v.im + (c[j].re * zj.im + c[j].im * zj.re)};
        }
        u[p] = v;
    }
}

template <typename T, int DIM, int NJ>
void launch_apply_dots(cx<T> *Z, size_t N, const cx<T> *q, const Stencil<T> &P, double *parts, int nb, hipStream_t s,
                       const int *stop)
{
    hipLaunchKernelGGL((k_gm_apply_dots<T, DIM, NJ>), dim3(nb), dim3(256), 0, s, Z, N, q, P, parts, stop);
}

template <typename T, int DIM>
void apply_dots_dispatch(int nj, cx<T> *Z, size_t N, const cx<T> *q, const Stencil<T> &P, double *parts, int nb,
                         hipStream_t s, const int *stop)
{
    switch (nj) {
    case 1: launch_apply_dots<T, DIM, 1>(Z, N, q, P, parts, nb, s, stop); break;
    case 2: launch_apply_dots<T, DIM, 2>(Z, N, q, P, parts, nb, s, stop); break;
    case 3: launch_apply_dots<T, DIM, 3>(Z, N, q, P, parts, nb, s, stop); break;
    case 4: launch_apply_dots<T, DIM, 4>(Z, N, q, P, parts, nb, s, stop); break;
    case 5: launch_apply_dots<T, DIM, 5>(Z, N, q, P, parts, nb, s, stop); break;
    case 6: launch_apply_dots<T, DIM, 6>(Z, N, q, P, parts, nb, s, stop); break;
    case 7: launch_apply_dots<T, DIM, 7>(Z, N, q, P, parts, nb, s, stop); break;
    default: launch_apply_dots<T, DIM, 8>(Z, N, q, P, parts, nb, s, stop); break;
    }
}

template <typename T>
void orth_dispatch(int nj, cx<T> *Z, size_t N, const double *S, double *parts, int nb, hipStream_t s,
                   const int *stop)
{
#define GM_ORTH(J) hipLaunchKernelGGL((k_gm_orth<T, J>), dim3(nb), dim3(256), 0, s, Z, N, S, parts, stop)
    switch (nj) {
    case 1: GM_ORTH(1); break;
    case 2: GM_ORTH(2); break;
    case 3: GM_ORTH(3); break;
    case 4: GM_ORTH(4); break;
    case 5: GM_ORTH(5); break;
    case 6: GM_ORTH(6); break;
    case 7: GM_ORTH(7); break;
    default: GM_ORTH(8); break;
    }
#undef GM_ORTH
}

}  // namespace

// One GMRES(m) smoothing step in place on a level: Z holds m + 1 vectors of
// N points, S the step's scalars (GM_S doubles), parts GM_BLOCKS x (2m + 1)
// partial sums.  zero: u is 0 on entry (not read).
template <typename T>
void launch_gmres_step(const LevelGeom &g, const Stencil<T> &P, const cx<T> *b, const cx<T> *q, cx<T> *u, bool zero,
                       int m, cx<T> *Z, double *S, double *parts, hipStream_t s, const int *stop)
{
    const size_t N = g.N();
    const int nb = (int)std::min<size_t>((N + 255) / 256, GM_BLOCKS);
    const bool d3 = (g.dim == 3);
    if (zero) launch_zero<T>(u, N, s, stop);
    if (d3)
        hipLaunchKernelGGL((k_gm_resid<T, 3>), dim3(nb), dim3(256), 0, s, zero ? nullptr : u, b, q, Z, P, N, parts,
                           stop);
    else
        hipLaunchKernelGGL((k_gm_resid<T, 2>), dim3(nb), dim3(256), 0, s, zero ? nullptr : u, b, q, Z, P, N, parts,
                           stop);
    hipLaunchKernelGGL(k_gm_reduce, dim3(1), dim3(256), 0, s, parts, nb, S, stop);
    for (int j = 0; j < m; ++j) {
        const int nj = j + 1;
        if (d3) apply_dots_dispatch<T, 3>(nj, Z, N, q, P, parts, nb, s, stop);
        else apply_dots_dispatch<T, 2>(nj, Z, N, q, P, parts, nb, s, stop);
        hipLaunchKernelGGL(k_gm_reduce, dim3(2 * nj), dim3(256), 0, s, parts, nb,
                           S + GM_D + 2 * (j * GMRES_MAX_M), stop);
        orth_dispatch<T>(nj, Z, N, S, parts, nb, s, stop);
        hipLaunchKernelGGL(k_gm_reduce, dim3(1), dim3(256), 0, s, parts, nb, S + j + 1, stop);
    }
    hipLaunchKernelGGL(k_gm_small, dim3(1), dim3(64), 0, s, S, m, stop);
    hipLaunchKernelGGL((k_gm_update<T>), dim3(nb), dim3(256), 0, s, u, Z, N, m, S, stop);
}
template void launch_gmres_step<double>(const LevelGeom &, const Stencil<double> &, const cd *, const cd *, cd *, bool,
                                        int, cd *, double *, double *, hipStream_t, const int *);
template void launch_gmres_step<float>(const LevelGeom &, const Stencil<float> &, const cf *, const cf *, cf *, bool,
                                       int, cf *, double *, double *, hipStream_t, const int *);

}  // namespace ffmg
