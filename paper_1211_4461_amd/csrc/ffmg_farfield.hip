// ffmg_farfield.hip -- the far-field quadrature on the contour grid
// (Sec. 2.2 eq. FFmap moved onto the contour, Sec. 3.1 eq. I2complex):
//
//   F_m = e^{i d gamma} prod h_k  sum_j exp(-i k0 alpha_m.z_j) s_j,
//   s_j = q_j (u_in(z_j) + u_j).
//
// The kernel exp(-i k0 e^{i gamma} alpha.x) is a product of one factor per
// axis, so the sum is a chain of contractions over one axis at a time, each a
// complex GEMM "C[m][n] = sum_k A[m][k] S[k][n]" whose S is the current field
// with the contracted axis slowest (row k) and the kept axes fastest (n).
// That is the only dense work on the path and it runs on the MFMA units:
//   2D:  T[m][x]   = sum_y Py[m][y] s[y][x];        F_m = sum_x Px[m][x] T[m][x]
//   3D:  T1[p][yx] = sum_z Pz[p][z] s[z][yx]       (p: distinct alpha_z)
//        T2[m][x]  = sum_y Py[m][y] T1[p(m)][y][x]  (one GEMM per p)
//        F_m       = sum_x Px[m][x] T2[m][x]
// A complex GEMM is run as one real GEMM: A' has rows (Re A[m], Im A[m]),
// S' is S viewed as reals (re/im interleaved along n), and the epilogue
// combines neighbouring rows/columns of C' = A' S' into Re/Im of C.
//
// Two number formats run the GEMMs:
//  * FP64 MFMA (v_mfma_f64_16x16x4f64), the plain method;
//  * split BF16 MFMA (v_mfma_f32_16x16x32_bf16) with FP32 accumulation: every
//    FP64 operand x is written as x0 + x1 (+ x2), each part a BF16 that holds
//    the next 8 significant bits, and a product is the sum of the part
//    products of order <= 1 (two parts, 3 products, about 16 bits) or <= 2
//    (three parts, 6 products, about 24 bits).  The FP32 accumulator of one
//    32-deep k-step is added into FP64 after every step, so the accumulation
//    error does not grow with the contraction length.
#include <math.h>

#include <algorithm>
#include <memory>
#include <mutex>
#include <vector>

#include "../../include/ffmg.h"
#include "ffmg_internal.hpp"

namespace ffmg {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned short us8 __attribute__((ext_vector_type(8)));

// ---------------------------------------------------------------------------
// BF16 splitting.  bf16_rne: round-to-nearest-even of a finite FP32 to the
// upper 16 bits.  split_bf16: NS parts whose sum approximates x; each
// residual r - part is exact in FP64.
__device__ __forceinline__ unsigned short bf16_rne(float f)
{
    unsigned u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}

template <int NS>
__device__ __forceinline__ void split_bf16(double x, unsigned short (&o)[NS])
{
    double r = x;
#pragma unroll
    for (int t = 0; t < NS; ++t) {
        unsigned short b = bf16_rne((float)r);
        o[t] = b;
        r -= (double)__uint_as_float((unsigned)b << 16);
    }
}

// Split 8 consecutive-k complex values of one column n and store them in the
// B-operand layout of v_mfma_f32_16x16x32_bf16: plane t holds, for k-block kb
// (k = 8 kb + e) and real column c (2n: Re, 2n + 1: Im), the 8 values of e
// contiguously (16 bytes), rows of ldP columns.
template <int NS>
__device__ __forceinline__ void store_split8(const cd (&v)[8], us8 *__restrict__ planes, long pstride, long row_off)
{
    us8 re[NS], im[NS];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        unsigned short a[NS], b[NS];
        split_bf16<NS>(v[e].re, a);
        split_bf16<NS>(v[e].im, b);
#pragma unroll
        for (int t = 0; t < NS; ++t) {
            re[t][e] = a[t];
            im[t][e] = b[t];
        }
    }
#pragma unroll
    for (int t = 0; t < NS; ++t) {
        planes[t * pstride + row_off] = re[t];
        planes[t * pstride + row_off + 1] = im[t];
    }
}

// ---------------------------------------------------------------------------
// Integrand: s_j = q_j (Ex[ix] Ey[iy] Ez[iz] + u_j), with the per-axis factors
// E_k[i] = exp(i k0 e^{i gamma} eta_k x_i) of the incoming plane wave.
__global__ __launch_bounds__(256) void k_ff_integrand(const cd *__restrict__ q, const cd *__restrict__ u,
                                                      const cd *__restrict__ E, cd *__restrict__ s, int mx, int my,
                                                      int mz)
{
    const cd *Ex = E, *Ey = E + mx, *Ez = E + mx + my;
    size_t N = (size_t)mx * my * mz;
    for (size_t j = (size_t)blockIdx.x * 256 + threadIdx.x; j < N; j += (size_t)gridDim.x * 256) {
        int ix = (int)(j % mx);
        size_t rest = j / mx;
        int iy = (int)(rest % my), iz = (int)(rest / my);
        cd uin = Ex[ix] * Ey[iy];
        if (mz > 1) uin = uin * Ez[iz];
        cd t = u ? uin + u[j] : uin;
        s[j] = q[j] * t;
    }
}

// The same integrand written as NS BF16 planes for the split GEMM: the
// slowest axis (y in 2D, z in 3D) is the contraction index k, the other axes
// form the column n.  One thread produces the 8 values k = 8 kb .. 8 kb + 7 of
// one column; rows k >= K and columns n >= Nc (padding) are zero.
template <int NS>
__global__ __launch_bounds__(256) void k_ff_integrand_split(const cd *__restrict__ q, const cd *__restrict__ u,
                                                            const cd *__restrict__ E, us8 *__restrict__ planes,
                                                            int mx, int my, int mz, int dim, int kb_tot,
                                                            long ldP, long pstride)
{
    const cd *Ex = E, *Ey = E + mx, *Ez = E + mx + my;
    const int K = (dim == 3) ? mz : my;
    const long Nc = (dim == 3) ? (long)mx * my : mx;
    const long ncols = ldP / 2;
    const long tot = (long)kb_tot * ncols;
    for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < tot; e += (long)gridDim.x * 256) {
        const long n = e % ncols;
        const int kb = (int)(e / ncols);
        const bool colin = n < Nc;
        const int ix = (int)(colin ? n % mx : 0);
        const int iy0 = (int)(colin ? n / mx : 0);   // 3D: y index of the column
        cd v[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int k = 8 * kb + i;
            const bool in = colin && k < K;
            const size_t j = in ? (size_t)k * Nc + n : 0;
            cd uin;
            if (dim == 3) uin = (Ex[ix] * Ey[iy0]) * Ez[in ? k : 0];
            else uin = Ex[ix] * Ey[in ? k : 0];
            cd t = u ? uin + u[j] : uin;
            cd sv = q[j] * t;
            v[i] = in ? sv : cd{0.0, 0.0};
        }
        store_split8<NS>(v, planes, pstride, (long)kb * ldP + 2 * n);
    }
}

// Split an FP64 complex field src[g][k][n] (K rows of Nc, group stride
// gstride) into BF16 planes (group stride plane_gstride), as above.
template <int NS>
__global__ __launch_bounds__(256) void k_split_field(const cd *__restrict__ src, long gstride, int K, long Nc,
                                                     us8 *__restrict__ planes, long plane_gstride, int kb_tot,
                                                     long ldP, long pstride)
{
    const cd *S = src + (size_t)blockIdx.y * gstride;
    us8 *P = planes + (size_t)blockIdx.y * plane_gstride;
    const long ncols = ldP / 2;
    const long tot = (long)kb_tot * ncols;
    for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < tot; e += (long)gridDim.x * 256) {
        const long n = e % ncols;
        const int kb = (int)(e / ncols);
        cd v[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int k = 8 * kb + i;
            const bool in = n < Nc && k < K;
            cd x = S[in ? (size_t)k * Nc + n : 0];
            v[i] = in ? x : cd{0.0, 0.0};
        }
        store_split8<NS>(v, P, pstride, (long)kb * ldP + 2 * n);
    }
}

// Axis factors exp(c * x_i), c complex, x_i = lo + (i+1) h, i < m.
__global__ __launch_bounds__(256) void k_axis_exp(cd *__restrict__ out, int m, double lo, double h, double cr,
                                                  double ci)
{
    int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= m) return;
    double x = lo + (double)(i + 1) * h;
    double mag = exp(cr * x), ph = ci * x;
    out[i] = cd{mag * cos(ph), mag * sin(ph)};
}

// Packed real-expanded factor matrix for the MFMA A operand of
// v_mfma_f64_16x16x4f64.  That instruction reads A[i][k] from lane i + 16 k
// and returns D[i][j] in lane j + 16 (i % 4), register i / 4.  Tile-local row
// i of a 16-row tile is mapped to direction m = 8 rt + (i % 4) + 4 (i / 8) and
// part c = (i / 4) % 2 (0: Re, 1: Im of P[m][k]), so that each lane's output
// registers (0, 1) and (2, 3) are the Re/Im rows of one direction.  Layout:
// [row tile rt][k step ks (4)][lane l (64)], element for tile row l % 16 and
// k = 4 ks + l / 16; zero outside M x K.
//   P[m][k] = exp(-i k0 e^{i gamma} alpha_m x_k),  x_k = lo + (k+1) h.
__device__ __forceinline__ void tile_row_map(int i, int &mloc, int &c)
{
    mloc = (i & 3) + 4 * (i >> 3);
    c = (i >> 2) & 1;
}

__global__ __launch_bounds__(256) void k_pack_factor(double *__restrict__ out, const double *__restrict__ alpha,
                                                     int M, int K, int rtiles, int ksteps, double lo, double h,
                                                     double k0, double gamma)
{
    size_t tot = (size_t)rtiles * ksteps * 64;
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < tot; e += (size_t)gridDim.x * 256) {
        int l = (int)(e % 64);
        size_t t = e / 64;
        int ks = (int)(t % ksteps), rt = (int)(t / ksteps);
        int mloc, c;
        tile_row_map(l % 16, mloc, c);
        int m = 8 * rt + mloc, k = 4 * ks + l / 16;
        double v = 0.0;
        if (m < M && k < K) {
            double x = lo + (double)(k + 1) * h;
            // -i k0 e^{i g} a x = (k0 sin g a x) + i (-k0 cos g a x)
            double a = alpha[m];
            double mag = exp(k0 * sin(gamma) * a * x);
            double ph = -(k0 * cos(gamma)) * a * x;
            v = c ? mag * sin(ph) : mag * cos(ph);
        }
        out[e] = v;
    }
}

// Packed factor matrix for the A operand of v_mfma_f32_16x16x32_bf16, split
// into NS BF16 planes.  That instruction reads A[i][k] from lane i + 16 (k / 8),
// element k % 8, and returns D[i][j] in lane j + 16 (i / 4), register i % 4.
// Tile row i holds direction m = 8 rt + 2 (i / 4) + (i / 2) % 2, part i % 2
// (0: Re, 1: Im), so that registers (0, 1) and (2, 3) of a lane are the Re/Im
// rows of two consecutive directions.  Layout per plane:
// [row tile rt][k step ks (32)][lane (64)] of 8 BF16; zero outside M x K.
__device__ __forceinline__ void tile_row_map_bf16(int i, int &mloc, int &c)
{
    mloc = 2 * (i >> 2) + ((i >> 1) & 1);
    c = i & 1;
}

template <int NS>
__global__ __launch_bounds__(256) void k_pack_factor_bf16(us8 *__restrict__ out, long sstride,
                                                          const double *__restrict__ alpha, int M, int K,
                                                          int rtiles, int ksteps, double lo, double h, double k0,
                                                          double gamma)
{
    const long tot = (long)rtiles * ksteps * 64;
    const double sg = k0 * sin(gamma), cg = k0 * cos(gamma);
    for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < tot; e += (long)gridDim.x * 256) {
        const int l = (int)(e % 64);
        const long t = e / 64;
        const int ks = (int)(t % ksteps), rt = (int)(t / ksteps);
        int mloc, c;
        tile_row_map_bf16(l % 16, mloc, c);
        const int m = 8 * rt + mloc;
        us8 v[NS];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int k = 32 * ks + 8 * (l / 16) + i;
            double val = 0.0;
            if (m < M && k < K) {
                double x = lo + (double)(k + 1) * h;
                double a = alpha[m];
                double mag = exp(sg * a * x), ph = -cg * a * x;
                val = c ? mag * sin(ph) : mag * cos(ph);
            }
            unsigned short p[NS];
            split_bf16<NS>(val, p);
#pragma unroll
            for (int s = 0; s < NS; ++s) v[s][i] = p[s];
        }
#pragma unroll
        for (int s = 0; s < NS; ++s) out[s * sstride + e] = v[s];
    }
}

// Plain complex factor table P[m][k] (row-major, M x K), for the last axis.
__global__ __launch_bounds__(256) void k_plain_factor(cd *__restrict__ out, const double *__restrict__ alpha, int M,
                                                      int K, double lo, double h, double k0, double gamma)
{
    size_t tot = (size_t)M * K;
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < tot; e += (size_t)gridDim.x * 256) {
        int m = (int)(e / K), k = (int)(e % K);
        double x = lo + (double)(k + 1) * h;
        double a = alpha[m];
        double mag = exp(k0 * sin(gamma) * a * x);
        double ph = -(k0 * cos(gamma)) * a * x;
        out[e] = cd{mag * cos(ph), mag * sin(ph)};
    }
}

// ---------------------------------------------------------------------------
// FP64 MFMA contraction.  Group g: C_g[m][n] = sum_k A_g[m][k] S_g[k][n],
// m < M_g, k < K, n < Nc (complex).  Each wave owns RT x CT tiles of 16 x 16
// of C' (real), i.e. 8 RT complex rows x 8 CT complex columns; the block has
// 4 waves side by side in n.
struct GemmGroup {
    const double *A;     // packed A' (see k_pack_factor)
    const double *S;     // S' : K rows of 2 Nc doubles (row stride ldS doubles)
    cd *C;               // C : M_g rows of Nc complex (row stride ldC complex)
    int M;
    int rtiles;          // row tiles of 16 in A' (8 directions each)
};

template <int RT, int CT>
__global__ __launch_bounds__(256) void k_ff_gemm_f64(const GemmGroup *__restrict__ groups, int K, int ksteps,
                                                     int Nc, long ldS, long ldC)
{
    const GemmGroup G = groups[blockIdx.z];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int rt0 = blockIdx.y * RT;
    if (rt0 * 8 >= G.M) return;
    const long col0 = ((long)blockIdx.x * 4 + wave) * (CT * 16);   // real column of C'
    const int lr = lane & 15, lk = lane >> 4;

    d4 acc[RT][CT];
#pragma unroll
    for (int i = 0; i < RT; ++i)
#pragma unroll
        for (int j = 0; j < CT; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

    const double *Ab = G.A + (size_t)rt0 * ksteps * 64 + lane;
    const long ncols = 2L * Nc;
    for (int ks = 0; ks < ksteps; ++ks) {
        const int k = 4 * ks + lk;
        double a[RT], bv[CT];
#pragma unroll
        for (int i = 0; i < RT; ++i) {
            int rt = rt0 + i;
            a[i] = (rt < G.rtiles) ? Ab[((size_t)i * ksteps + ks) * 64] : 0.0;
        }
#pragma unroll
        for (int j = 0; j < CT; ++j) {
            long c = col0 + j * 16 + lr;
            bv[j] = (k < K && c < ncols) ? G.S[(size_t)k * ldS + c] : 0.0;
        }
#pragma unroll
        for (int i = 0; i < RT; ++i)
#pragma unroll
            for (int j = 0; j < CT; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], bv[j], acc[i][j], 0, 0, 0);
    }
    // Epilogue: lane (j, lk) holds, for tile rt, C'[(m, Re)][c0 + j] in
    // register 0, C'[(m, Im)][..] in 1, and the same for m + 4 in 2, 3, with
    // m = 8 rt + lk (see tile_row_map).  Columns 2n / 2n+1 are Re / Im of
    // S[k][n]: the even lane writes C[m][n], the odd lane C[m + 4][n].
    const bool odd = (lane & 1) != 0;
#pragma unroll
    for (int i = 0; i < RT; ++i)
#pragma unroll
        for (int j = 0; j < CT; ++j) {
            d4 mine = acc[i][j];
            double p0 = __shfl_xor(mine[0], 1, 64), p1 = __shfl_xor(mine[1], 1, 64);
            double p2 = __shfl_xor(mine[2], 1, 64), p3 = __shfl_xor(mine[3], 1, 64);
            int m = 8 * (rt0 + i) + lk + (odd ? 4 : 0);
            long c = col0 + j * 16 + lr;
            long n = c >> 1;
            cd v;
            if (!odd) v = cd{mine[0] - p1, p0 + mine[1]};
            else v = cd{p2 - mine[3], mine[2] + p3};
            if (m < G.M && n < Nc) G.C[(size_t)m * ldC + n] = v;
        }
}

// Split-BF16 MFMA contraction.  Group g: C_g = A_g S_g as above, with A_g
// and S_g given as NS BF16 planes (padded: rtiles rows of tiles, K to a
// multiple of 32, ldP real columns, all zero-filled, so the inner loop has no
// bounds checks).  Each wave owns RT x CT tiles of 16 x 16 of C' (8 RT
// directions x 8 CT complex columns); the block has 4 waves side by side in n.
// The flat block index is mapped XCD-contiguously onto (column slab, row
// block) with row blocks fastest, so the blocks that share one slab of the
// integrand planes run on one XCD and share its L2.
struct GemmGroupB {
    const bf8 *A;     // factor planes [NS][rtiles][ksteps][64]
    long a_split;     // plane stride of A (bf8 units)
    const bf8 *S;     // integrand planes [NS][4 ksteps][ldP]
    long s_split;     // plane stride of S (bf8 units)
    cd *C;            // C : M rows of Nc complex (row stride ldC)
    long ldC;
    int M, Nc, rtiles;
};

template <int NS, int RT, int CT>
__global__ __launch_bounds__(256) void k_ff_gemm_bf16(const GemmGroupB *__restrict__ groups, int ksteps, long ldP,
                                                      int gx, int gy)
{
    const GemmGroupB G = groups[blockIdx.y];
    const int t = xcd_tile(blockIdx.x, gx * gy);
    const int bx = t / gy, by = t % gy;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int rt0 = by * RT;
    if (rt0 >= G.rtiles) return;
    const long col0 = ((long)bx * 4 + wave) * (CT * 16);
    const int lr = lane & 15, g = lane >> 4;

    double acc[RT][CT][4];
#pragma unroll
    for (int i = 0; i < RT; ++i)
#pragma unroll
        for (int j = 0; j < CT; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[i][j][v] = 0.0;

    const bf8 *Ab = G.A + (long)rt0 * ksteps * 64 + lane;
    const bf8 *Sb = G.S + (long)g * ldP + col0 + lr;
    for (int ks = 0; ks < ksteps; ++ks) {
        bf8 a[RT][NS], b[CT][NS];
#pragma unroll
        for (int i = 0; i < RT; ++i)
#pragma unroll
            for (int s = 0; s < NS; ++s) a[i][s] = Ab[s * G.a_split + ((long)i * ksteps + ks) * 64];
#pragma unroll
        for (int j = 0; j < CT; ++j)
#pragma unroll
            for (int s = 0; s < NS; ++s) b[j][s] = Sb[s * G.s_split + (long)ks * 4 * ldP + j * 16];
        f4 c[RT][CT];
#pragma unroll
        for (int i = 0; i < RT; ++i)
#pragma unroll
            for (int j = 0; j < CT; ++j) c[i][j] = f4{0.f, 0.f, 0.f, 0.f};
        // part products, smallest first: orders 2 (NS = 3), 1, then 0
        if constexpr (NS == 3) {
#pragma unroll
            for (int i = 0; i < RT; ++i)
#pragma unroll
                for (int j = 0; j < CT; ++j) {
                    c[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][2], b[j][0], c[i][j], 0, 0, 0);
                    c[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][1], b[j][1], c[i][j], 0, 0, 0);
                    c[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][0], b[j][2], c[i][j], 0, 0, 0);
                }
        }
#pragma unroll
        for (int i = 0; i < RT; ++i)
#pragma unroll
            for (int j = 0; j < CT; ++j) {
                c[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][1], b[j][0], c[i][j], 0, 0, 0);
                c[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][0], b[j][1], c[i][j], 0, 0, 0);
                c[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][0], b[j][0], c[i][j], 0, 0, 0);
            }
#pragma unroll
        for (int i = 0; i < RT; ++i)
#pragma unroll
            for (int j = 0; j < CT; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[i][j][v] += (double)c[i][j][v];
    }
    // Epilogue: lane (j, g) holds, for tile rt, C'[(m, Re)][c0 + j] and
    // C'[(m, Im)][..] in registers 0, 1 and the same for m + 1 in 2, 3, with
    // m = 8 rt + 2 g (see tile_row_map_bf16).  Columns 2n / 2n+1 are Re / Im
    // of S[k][n]: the even lane writes C[m][n], the odd lane C[m + 1][n].
    const bool odd = (lane & 1) != 0;
#pragma unroll
    for (int i = 0; i < RT; ++i)
#pragma unroll
        for (int j = 0; j < CT; ++j) {
            const double m0 = acc[i][j][0], m1 = acc[i][j][1], m2 = acc[i][j][2], m3 = acc[i][j][3];
            double p0 = __shfl_xor(m0, 1, 64), p1 = __shfl_xor(m1, 1, 64);
            double p2 = __shfl_xor(m2, 1, 64), p3 = __shfl_xor(m3, 1, 64);
            int m = 8 * (rt0 + i) + 2 * g + (odd ? 1 : 0);
            long n = (col0 + j * 16 + lr) >> 1;
            cd v;
            if (!odd) v = cd{m0 - p1, p0 + m1};
            else v = cd{p2 - m3, m2 + p3};
            if (m < G.M && n < G.Nc) G.C[(size_t)m * G.ldC + n] = v;
        }
}

// The same contraction with a block tile staged in LDS: BR row tiles x BC
// column tiles per 256-thread block, the four waves arranged WR x WC, each
// computing (BR / WR) x (BC / WC) tiles.  Per k-step the block copies its
// A fragments ([plane][row tile][lane], 1 KB each) and the BC * 16 columns of
// its four k-blocks of every S plane into one of two LDS buffers (the next
// k-step's loads are in flight while the MFMAs run on the current one), so
// each operand byte leaves L2 once per block instead of once per wave.  The
// MFMA sequence of every (tile, k-step) and the FP64 accumulation order are
// those of k_ff_gemm_bf16: the results are the same bits.  Rows are padded to
// a multiple of BR (BF_RT_PAD) and columns to a multiple of BC * 16.
template <int NS, int BR, int BC, int WR, int WC>
__global__ __launch_bounds__(256) void k_ff_gemm_bf16_lds(const GemmGroupB *__restrict__ groups, int ksteps,
                                                          long ldP, int gx, int gy)
{
    static_assert(WR * WC == 4 && BR % WR == 0 && BC % WC == 0, "four waves");
    constexpr int RW = BR / WR, CW = BC / WC;
    constexpr int A_EL = NS * BR * 64;        // 16-byte elements of A per k-step
    constexpr int B_EL = NS * 4 * BC * 16;    // and of S
    constexpr int NLD = (A_EL + B_EL + 255) / 256;
    // two buffers of A_EL + B_EL elements (dynamic: above the 64 KB of static LDS)
    extern __shared__ __attribute__((aligned(16))) unsigned char gemm_lds[];
    bf8(*lds)[A_EL + B_EL] = reinterpret_cast<bf8(*)[A_EL + B_EL]>(gemm_lds);
    const GemmGroupB G = groups[blockIdx.y];
    const int t = xcd_tile(blockIdx.x, gx * gy);
    const int bx = t / gy, by = t % gy;
    const int rt0 = by * BR;
    if (rt0 >= G.rtiles) return;
    const long col0 = (long)bx * (BC * 16);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wr = wave / WC, wc = wave % WC;
    const int lr = lane & 15, g = lane >> 4;

    bf8 pre[NLD];
    auto gload = [&](int ks) {
#pragma unroll
        for (int r = 0; r < NLD; ++r) {
            const int e = threadIdx.x + 256 * r;
            if (e < A_EL) {
                const int sp = e / (BR * 64), rem = e - sp * (BR * 64), i = rem >> 6, l = rem & 63;
                pre[r] = G.A[sp * G.a_split + ((long)(rt0 + i) * ksteps + ks) * 64 + l];
            } else if (e < A_EL + B_EL) {
                const int e2 = e - A_EL;
                const int sp = e2 / (4 * BC * 16), rem = e2 - sp * (4 * BC * 16);
                const int kb = rem / (BC * 16), c = rem - kb * (BC * 16);
                pre[r] = G.S[sp * G.s_split + (long)(4 * ks + kb) * ldP + col0 + c];
            }
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int r = 0; r < NLD; ++r) {
            const int e = threadIdx.x + 256 * r;
            if (e < A_EL + B_EL) lds[buf][e] = pre[r];
        }
    };

    double acc[RW][CW][4];
#pragma unroll
    for (int i = 0; i < RW; ++i)
#pragma unroll
        for (int j = 0; j < CW; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[i][j][v] = 0.0;

    gload(0);
    sstore(0);
    __syncthreads();
    for (int ks = 0; ks < ksteps; ++ks) {
        const int cur = ks & 1;
        if (ks + 1 < ksteps) gload(ks + 1);
        const bf8 *LA = lds[cur];
        const bf8 *LB = lds[cur] + A_EL;
        bf8 a[RW][NS], b[CW][NS];
#pragma unroll
        for (int i = 0; i < RW; ++i)
#pragma unroll
            for (int sp = 0; sp < NS; ++sp) a[i][sp] = LA[(sp * BR + wr * RW + i) * 64 + lane];
#pragma unroll
        for (int j = 0; j < CW; ++j)
#pragma unroll
            for (int sp = 0; sp < NS; ++sp) b[j][sp] = LB[(sp * 4 + g) * (BC * 16) + (wc * CW + j) * 16 + lr];
        f4 c[RW][CW];
#pragma unroll
        for (int i = 0; i < RW; ++i)
#pragma unroll
            for (int j = 0; j < CW; ++j) c[i][j] = f4{0.f, 0.f, 0.f, 0.f};
        // part products, smallest first: orders 2 (NS = 3), 1, then 0
        if constexpr (NS == 3) {
#pragma unroll
            for (int i = 0; i < RW; ++i)
#pragma unroll
                for (int j = 0; j < CW; ++j) {
                    c[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][2], b[j][0], c[i][j], 0, 0, 0);
                    c[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][1], b[j][1], c[i][j], 0, 0, 0);
                    c[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][0], b[j][2], c[i][j], 0, 0, 0);
                }
        }
#pragma unroll
        for (int i = 0; i < RW; ++i)
#pragma unroll
            for (int j = 0; j < CW; ++j) {
                c[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][1], b[j][0], c[i][j], 0, 0, 0);
                c[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][0], b[j][1], c[i][j], 0, 0, 0);
                c[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][0], b[j][0], c[i][j], 0, 0, 0);
            }
#pragma unroll
        for (int i = 0; i < RW; ++i)
#pragma unroll
            for (int j = 0; j < CW; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[i][j][v] += (double)c[i][j][v];
        if (ks + 1 < ksteps) sstore(cur ^ 1);
        __syncthreads();
    }
    // epilogue as k_ff_gemm_bf16
    const bool odd = (lane & 1) != 0;
#pragma unroll
    for (int i = 0; i < RW; ++i)
#pragma unroll
        for (int j = 0; j < CW; ++j) {
            const double m0 = acc[i][j][0], m1 = acc[i][j][1], m2 = acc[i][j][2], m3 = acc[i][j][3];
            double p0 = __shfl_xor(m0, 1, 64), p1 = __shfl_xor(m1, 1, 64);
            double p2 = __shfl_xor(m2, 1, 64), p3 = __shfl_xor(m3, 1, 64);
            int m = 8 * (rt0 + wr * RW + i) + 2 * g + (odd ? 1 : 0);
            long n = (col0 + (wc * CW + j) * 16 + lr) >> 1;
            cd v;
            if (!odd) v = cd{m0 - p1, p0 + m1};
            else v = cd{p2 - m3, m2 + p3};
            if (m < G.M && n < G.Nc) G.C[(size_t)m * G.ldC + n] = v;
        }
}

// F_m = pre * sum_x P[m][x] T[m][x]; one block per direction, the sums of
// its four waves combined in a fixed order.
__global__ __launch_bounds__(256) void k_ff_final(const cd *__restrict__ P, const cd *__restrict__ T, int M, int K,
                                                  cd pre, cd *__restrict__ F)
{
    __shared__ double red[2][4];
    const int m = blockIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (m >= M) return;
    double re = 0.0, im = 0.0;
    const cd *pr = P + (size_t)m * K, *tr = T + (size_t)m * K;
    for (int k = threadIdx.x; k < K; k += 256) {
        cd v = pr[k] * tr[k];
        re += v.re;
        im += v.im;
    }
    for (int off = 32; off > 0; off >>= 1) {
        re += __shfl_down(re, off, 64);
        im += __shfl_down(im, off, 64);
    }
    if (lane == 0) {
        red[0][wave] = re;
        red[1][wave] = im;
    }
    __syncthreads();
    if (threadIdx.x == 0)
        F[m] = pre * cd{(red[0][0] + red[0][1]) + (red[0][2] + red[0][3]),
                        (red[1][0] + red[1][1]) + (red[1][2] + red[1][3])};
}

// Scatter the sorted result into the caller's direction order.
__global__ __launch_bounds__(256) void k_unpermute(const cd *__restrict__ Fs, const int *__restrict__ perm, int M,
                                                   cd *__restrict__ F)
{
    int i = blockIdx.x * 256 + threadIdx.x;
    if (i < M) F[perm[i]] = Fs[i];
}

// ---------------------------------------------------------------------------
// Host-side plan.
static int ceil_div(long a, long b) { return (int)((a + b - 1) / b); }
static long round_up(long a, long b) { return (a + b - 1) / b * b; }

constexpr int GEMM_RT = 2, GEMM_CT = 2;

struct GemmLaunch {
    GemmGroup *d_groups = nullptr;
    int ngroups = 0, K = 0, Nc = 0, maxM = 0;
    long ldS = 0, ldC = 0;
};

static void launch_gemm(const GemmLaunch &L, hipStream_t s)
{
    int ksteps = ceil_div(L.K, 4);
    dim3 grid(ceil_div(2L * L.Nc, 4L * GEMM_CT * 16), ceil_div(2L * L.maxM, 16L * GEMM_RT), (unsigned)L.ngroups);
    hipLaunchKernelGGL((k_ff_gemm_f64<GEMM_RT, GEMM_CT>), grid, dim3(256), 0, s, L.d_groups, L.K, ksteps, L.Nc,
                       L.ldS, L.ldC);
}

// Split-GEMM tile variants: RT row tiles x CT column tiles per wave (four
// waves side by side in n), or (lds) an LDS-staged block of RT x CT tiles.
// Row tiles are padded to a multiple of BF_RT_PAD and columns to a multiple
// of BF_COL_PAD, which every variant divides.
struct BfVariant {
    int rt, ct;
    bool lds;
};
static const BfVariant BF_VARIANTS[] = {{2, 1, false}, {2, 2, false}, {4, 1, false}, {4, 2, false}, {2, 4, false},
                                        {4, 4, false}, {8, 4, true},  {4, 8, true},  {8, 8, true}};
constexpr int BF_NVARIANTS = (int)(sizeof(BF_VARIANTS) / sizeof(BF_VARIANTS[0]));
constexpr int BF_DEFAULT_VARIANT = 3;
constexpr int BF_RT_PAD = 8;
constexpr long BF_COL_PAD = 4 * 4 * 16;   // 4 waves x CT <= 4 tiles x 16 columns (LDS blocks: <= 8 x 16)

struct GemmLaunchB {
    GemmGroupB *d_groups = nullptr;
    int ngroups = 0, ksteps = 0, rtiles = 0;   // rtiles: the largest group's (padded)
    long ldP = 0;
};

// An LDS-staged variant: its two operand buffers (the attribute is raised
// once per instantiation, by a thread-safe static initialisation).
template <int NS, int BR, int BC>
static void launch_gemm_lds(dim3 grid, const GemmLaunchB &L, hipStream_t s)
{
    constexpr size_t bytes = 2 * (size_t)(NS * BR * 64 + NS * 4 * BC * 16) * 16;
    static const bool attr_set = [] {
        (void)hipFuncSetAttribute((const void *)k_ff_gemm_bf16_lds<NS, BR, BC, 2, 2>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        return true;
    }();
    (void)attr_set;
    hipLaunchKernelGGL((k_ff_gemm_bf16_lds<NS, BR, BC, 2, 2>), grid, dim3(256), bytes, s, L.d_groups, L.ksteps, L.ldP,
                       (int)(grid.x / ceil_div(L.rtiles, BR)), ceil_div(L.rtiles, BR));
}

template <int NS>
static void launch_gemm_bf16_ns(const GemmLaunchB &L, int variant, hipStream_t s)
{
    const BfVariant V = BF_VARIANTS[variant];
    if (V.lds) {
        const int gx = (int)(L.ldP / (V.ct * 16L)), gy = ceil_div(L.rtiles, V.rt);
        dim3 grid((unsigned)(gx * gy), (unsigned)L.ngroups);
        if (V.rt == 8 && V.ct == 4)
            launch_gemm_lds<NS, 8, 4>(grid, L, s);
        else if (V.rt == 4 && V.ct == 8)
            launch_gemm_lds<NS, 4, 8>(grid, L, s);
        else
            launch_gemm_lds<NS, 8, 8>(grid, L, s);
        return;
    }
    const int gx = (int)(L.ldP / (4L * V.ct * 16)), gy = ceil_div(L.rtiles, V.rt);
    dim3 grid((unsigned)(gx * gy), (unsigned)L.ngroups);
#define FF_BF_CASE(R, C)                                                                                             \
    if (V.rt == R && V.ct == C) {                                                                                    \
        hipLaunchKernelGGL((k_ff_gemm_bf16<NS, R, C>), grid, dim3(256), 0, s, L.d_groups, L.ksteps, L.ldP, gx, gy); \
        return;                                                                                                      \
    }
    FF_BF_CASE(2, 1)
    FF_BF_CASE(2, 2)
    FF_BF_CASE(4, 1)
    FF_BF_CASE(4, 2)
    FF_BF_CASE(2, 4)
    FF_BF_CASE(4, 4)
#undef FF_BF_CASE
}

static void launch_gemm_bf16(const GemmLaunchB &L, int ns, int variant, hipStream_t s)
{
    if (ns == 3) launch_gemm_bf16_ns<3>(L, variant, s);
    else launch_gemm_bf16_ns<2>(L, variant, s);
}

static unsigned grid_for(long work) { return (unsigned)std::max<long>(1, std::min<long>(65536, (work + 255) / 256)); }

struct FarFieldPlan {
    int dim = 0;
    int M = 0;
    int prec = -1;                 // ffmg_ff_precision of the built factors
    int ns = 0;                    // BF16 parts (split precisions)
    int variant = BF_DEFAULT_VARIANT;
    uint64_t gen = 0;              // rebuilds so far (every rebuild frees and reallocates the buffers below)
    std::vector<double> dirs;      // cache key
    std::vector<int> perm;         // sorted position -> direction index
    std::vector<int> gstart;       // group start in sorted order
    std::vector<double> gval;      // alpha_z per group
    std::vector<void *> bufs;      // everything allocated for this plan
    double *d_alpha = nullptr;     // sorted alphas per axis [3][M], then group alphas
    cd *d_s = nullptr;             // FP64 integrand
    cd *d_Plast = nullptr;         // plain Px [M][mx], sorted order
    cd *d_T1 = nullptr, *d_T2 = nullptr, *d_F = nullptr;
    int *d_perm = nullptr;
    GemmLaunch L1, L2;             // FP64 GEMM stages
    // split BF16
    us8 *d_S1b = nullptr;          // integrand planes
    us8 *d_S2b = nullptr;          // 3D: stage-1 result planes, per group
    int kb1 = 0, kb2 = 0;
    long ldP1 = 0, ldP2 = 0, ps1 = 0, ps2 = 0, gs2 = 0;
    GemmLaunchB B1, B2;
    GemmGroupB h_B2g{};            // 2D: the host copy of the one GEMM group (batched maps)
    template <typename P>
    hipError_t alloc(P **p, size_t bytes)
    {
        void *v = nullptr;
        hipError_t e = hipMalloc(&v, bytes ? bytes : 16);
        if (e != hipSuccess) return e;
        bufs.push_back(v);
        *p = (P *)v;
        return hipSuccess;
    }
    void release()
    {
        for (void *b : bufs) (void)hipFree(b);
        bufs.clear();
        d_alpha = nullptr;
        d_s = d_Plast = d_T1 = d_T2 = d_F = nullptr;
        d_perm = nullptr;
        d_S1b = d_S2b = nullptr;
        L1 = L2 = GemmLaunch{};
        B1 = B2 = GemmLaunchB{};
        M = dim = 0;
        prec = -1;
        dirs.clear();
    }
    ~FarFieldPlan() { release(); }
};

FarFieldPlan *ff_plan_create() { return new FarFieldPlan(); }
void ff_plan_destroy(FarFieldPlan *p) { delete p; }
int ff_plan_variants() { return BF_NVARIANTS; }
int ff_plan_default_variant() { return BF_DEFAULT_VARIANT; }
void ff_plan_set_variant(FarFieldPlan *p, int v) { p->variant = (v >= 0 && v < BF_NVARIANTS) ? v : BF_DEFAULT_VARIANT; }
int ff_plan_variant(const FarFieldPlan *p) { return p->variant; }
uint64_t ff_plan_generation(const FarFieldPlan *p) { return p->gen; }

#define FF_CHECK(x)                                                                                                  \
    do {                                                                                                             \
        hipError_t e_ = (x);                                                                                         \
        if (e_ != hipSuccess) return e_;                                                                             \
    } while (0)

template <typename T>
static hipError_t upload(FarFieldPlan *p, T **d, const std::vector<T> &h)
{
    FF_CHECK(p->alloc(d, h.size() * sizeof(T)));
    return hipMemcpy(*d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice);
}

// (Re)build the direction-dependent factors, the work buffers and the GEMM
// descriptors when the directions or the precision change.  Synchronises.
hipError_t ff_plan_prepare(FarFieldPlan *p, const LevelGeom &g, double k0, double gamma, int M, const double *dirs,
                           int prec, hipStream_t s)
{
    const int d = g.dim;
    std::vector<double> key(dirs, dirs + (size_t)M * d);
    if (p->M == M && p->dim == d && p->dirs == key && p->prec == prec) return hipSuccess;
    FF_CHECK(hipStreamSynchronize(s));
    p->release();
    ++p->gen;
    p->dim = d;
    p->M = M;
    p->prec = prec;   // the directions (the cache key) are recorded once the build has succeeded
    p->ns = (prec == 2) ? 3 : (prec == 1) ? 2 : 0;
    // group directions by their last component (exact equality) in 3D
    p->perm.resize(M);
    for (int i = 0; i < M; ++i) p->perm[i] = i;
    if (d == 3)
        std::stable_sort(p->perm.begin(), p->perm.end(),
                         [&](int a, int b) { return dirs[a * 3 + 2] < dirs[b * 3 + 2]; });
    p->gstart.clear();
    p->gval.clear();
    for (int i = 0; i < M; ++i) {
        double v = (d == 3) ? dirs[p->perm[i] * 3 + 2] : 0.0;
        if (i == 0 || (d == 3 && v != p->gval.back())) {
            p->gstart.push_back(i);
            p->gval.push_back(v);
        }
    }
    p->gstart.push_back(M);
    const int NG = (int)p->gval.size();
    std::vector<double> al((size_t)3 * M + NG, 0.0);
    for (int i = 0; i < M; ++i)
        for (int k = 0; k < d; ++k) al[(size_t)k * M + i] = dirs[(size_t)p->perm[i] * d + k];
    for (int gi = 0; gi < NG; ++gi) al[(size_t)3 * M + gi] = p->gval[gi];
    FF_CHECK(upload(p, &p->d_alpha, al));
    FF_CHECK(upload(p, &p->d_perm, p->perm));

    const int mx = g.m[0], my = g.m[1], mz = g.m[2];
    const long N = (long)g.N();
    FF_CHECK(p->alloc(&p->d_Plast, (size_t)M * mx * sizeof(cd)));
    hipLaunchKernelGGL(k_plain_factor, dim3(grid_for((long)M * mx)), dim3(256), 0, s, p->d_Plast, p->d_alpha, M, mx,
                       g.lo[0], g.h[0], k0, gamma);
    FF_CHECK(p->alloc(&p->d_T2, (size_t)M * mx * sizeof(cd)));
    FF_CHECK(p->alloc(&p->d_F, (size_t)M * sizeof(cd)));
    if (d == 3) FF_CHECK(p->alloc(&p->d_T1, (size_t)NG * mx * my * sizeof(cd)));
    int maxM = 0;
    for (int gi = 0; gi < NG; ++gi) maxM = std::max(maxM, p->gstart[gi + 1] - p->gstart[gi]);

    if (p->ns == 0) {
        // ---- FP64 MFMA
        FF_CHECK(p->alloc(&p->d_s, (size_t)N * sizeof(cd)));
        const int ks_y = ceil_div(my, 4);
        std::vector<size_t> off(NG);
        size_t tot = 0;
        for (int gi = 0; gi < NG; ++gi) {
            off[gi] = tot;
            tot += (size_t)ceil_div(2L * (p->gstart[gi + 1] - p->gstart[gi]), 16) * ks_y * 64;
        }
        double *A2 = nullptr;
        FF_CHECK(p->alloc(&A2, tot * sizeof(double)));
        for (int gi = 0; gi < NG; ++gi) {
            int Mg = p->gstart[gi + 1] - p->gstart[gi];
            int rt = ceil_div(2L * Mg, 16);
            hipLaunchKernelGGL(k_pack_factor, dim3(grid_for((long)rt * ks_y * 64)), dim3(256), 0, s, A2 + off[gi],
                               p->d_alpha + (size_t)1 * M + p->gstart[gi], Mg, my, rt, ks_y, g.lo[1], g.h[1], k0,
                               gamma);
        }
        std::vector<GemmGroup> gr;
        if (d == 3) {
            const int ks_z = ceil_div(mz, 4);
            int rt = ceil_div(2L * NG, 16);
            double *A1 = nullptr;
            FF_CHECK(p->alloc(&A1, (size_t)rt * ks_z * 64 * sizeof(double)));
            hipLaunchKernelGGL(k_pack_factor, dim3(grid_for((long)rt * ks_z * 64)), dim3(256), 0, s, A1,
                               p->d_alpha + (size_t)3 * M, NG, mz, rt, ks_z, g.lo[2], g.h[2], k0, gamma);
            // stage 1: T1[p][yx] = sum_z Pz[p][z] s[z][yx]
            gr.push_back(GemmGroup{A1, (const double *)p->d_s, p->d_T1, NG, rt});
        }
        for (int gi = 0; gi < NG; ++gi) {
            int Mg = p->gstart[gi + 1] - p->gstart[gi];
            const double *S = (d == 3) ? (const double *)(p->d_T1 + (size_t)gi * mx * my) : (const double *)p->d_s;
            gr.push_back(GemmGroup{A2 + off[gi], S, p->d_T2 + (size_t)p->gstart[gi] * mx, Mg, ceil_div(2L * Mg, 16)});
        }
        GemmGroup *dg = nullptr;
        FF_CHECK(upload(p, &dg, gr));
        if (d == 3) {
            p->L1 = GemmLaunch{dg, 1, mz, mx * my, NG, 2L * mx * my, (long)mx * my};
            p->L2 = GemmLaunch{dg + 1, NG, my, mx, maxM, 2L * mx, (long)mx};
        } else {
            p->L2 = GemmLaunch{dg, 1, my, mx, maxM, 2L * mx, (long)mx};
        }
    } else {
        // ---- split BF16 MFMA
        const int ns = p->ns;
        // integrand planes: contraction over the slowest axis
        const int K1 = (d == 3) ? mz : my;
        const long Nc1 = (d == 3) ? (long)mx * my : mx;
        const int ks1 = ceil_div(K1, 32);
        p->kb1 = 4 * ks1;
        p->ldP1 = round_up(2 * Nc1, BF_COL_PAD);
        p->ps1 = (long)p->kb1 * p->ldP1;
        FF_CHECK(p->alloc(&p->d_S1b, (size_t)ns * p->ps1 * sizeof(us8)));
        // last GEMM stage: contraction over y, per group
        const int ks_y = ceil_div(my, 32);
        std::vector<size_t> off(NG);
        std::vector<int> rts(NG);
        size_t tot = 0;
        int maxrt = 0;
        for (int gi = 0; gi < NG; ++gi) {
            int Mg = p->gstart[gi + 1] - p->gstart[gi];
            rts[gi] = (int)round_up(ceil_div(2L * Mg, 16), BF_RT_PAD);
            maxrt = std::max(maxrt, rts[gi]);
            off[gi] = tot;
            tot += (size_t)rts[gi] * ks_y * 64;
        }
        us8 *A2 = nullptr;
        FF_CHECK(p->alloc(&A2, (size_t)ns * tot * sizeof(us8)));
        for (int gi = 0; gi < NG; ++gi) {
            int Mg = p->gstart[gi + 1] - p->gstart[gi];
            long n = (long)rts[gi] * ks_y * 64;
            if (ns == 3)
                hipLaunchKernelGGL(k_pack_factor_bf16<3>, dim3(grid_for(n)), dim3(256), 0, s, A2 + off[gi],
                                   (long)tot, p->d_alpha + (size_t)1 * M + p->gstart[gi], Mg, my, rts[gi], ks_y,
                                   g.lo[1], g.h[1], k0, gamma);
            else
                hipLaunchKernelGGL(k_pack_factor_bf16<2>, dim3(grid_for(n)), dim3(256), 0, s, A2 + off[gi],
                                   (long)tot, p->d_alpha + (size_t)1 * M + p->gstart[gi], Mg, my, rts[gi], ks_y,
                                   g.lo[1], g.h[1], k0, gamma);
        }
        std::vector<GemmGroupB> gr;
        if (d == 3) {
            const int rt1 = (int)round_up(ceil_div(2L * NG, 16), BF_RT_PAD);
            us8 *A1 = nullptr;
            long n1 = (long)rt1 * ks1 * 64;
            FF_CHECK(p->alloc(&A1, (size_t)ns * n1 * sizeof(us8)));
            if (ns == 3)
                hipLaunchKernelGGL(k_pack_factor_bf16<3>, dim3(grid_for(n1)), dim3(256), 0, s, A1, n1,
                                   p->d_alpha + (size_t)3 * M, NG, mz, rt1, ks1, g.lo[2], g.h[2], k0, gamma);
            else
                hipLaunchKernelGGL(k_pack_factor_bf16<2>, dim3(grid_for(n1)), dim3(256), 0, s, A1, n1,
                                   p->d_alpha + (size_t)3 * M, NG, mz, rt1, ks1, g.lo[2], g.h[2], k0, gamma);
            gr.push_back(GemmGroupB{(const bf8 *)A1, n1, (const bf8 *)p->d_S1b, p->ps1, p->d_T1, (long)mx * my, NG,
                                    (int)Nc1, rt1});
            // stage-1 result planes for stage 2 (one set per group)
            p->kb2 = 4 * ks_y;
            p->ldP2 = round_up(2L * mx, BF_COL_PAD);
            p->ps2 = (long)p->kb2 * p->ldP2;
            p->gs2 = (long)ns * p->ps2;
            FF_CHECK(p->alloc(&p->d_S2b, (size_t)NG * p->gs2 * sizeof(us8)));
        }
        for (int gi = 0; gi < NG; ++gi) {
            int Mg = p->gstart[gi + 1] - p->gstart[gi];
            const us8 *S = (d == 3) ? p->d_S2b + (size_t)gi * p->gs2 : p->d_S1b;
            long ps = (d == 3) ? p->ps2 : p->ps1;
            gr.push_back(GemmGroupB{(const bf8 *)(A2 + off[gi]), (long)tot, (const bf8 *)S, ps,
                                    p->d_T2 + (size_t)p->gstart[gi] * mx, (long)mx, Mg, mx, rts[gi]});
        }
        GemmGroupB *dg = nullptr;
        FF_CHECK(upload(p, &dg, gr));
        if (d == 2) p->h_B2g = gr[0];
        if (d == 3) {
            p->B1 = GemmLaunchB{dg, 1, ks1, (int)round_up(ceil_div(2L * NG, 16), BF_RT_PAD), p->ldP1};
            p->B2 = GemmLaunchB{dg + 1, NG, ks_y, maxrt, p->ldP2};
        } else {
            p->B2 = GemmLaunchB{dg, 1, ks_y, maxrt, p->ldP1};
        }
    }
    FF_CHECK(hipGetLastError());
    FF_CHECK(hipStreamSynchronize(s));
    p->dirs = key;
    return hipSuccess;
}

// Integrand s = q (u_in + u) (u may be null: Born term), in FP64 or as BF16
// planes.
hipError_t ff_plan_integrand(FarFieldPlan *p, const LevelGeom &g, const cd *q, const cd *u, const cd *E,
                             hipStream_t s)
{
    const int d = g.dim, mx = g.m[0], my = g.m[1], mz = (d == 3) ? g.m[2] : 1;
    if (p->ns == 0) {
        hipLaunchKernelGGL(k_ff_integrand, dim3(grid_for((long)g.N())), dim3(256), 0, s, q, u, E, p->d_s, mx, my,
                           mz);
    } else {
        const long w1 = (long)p->kb1 * (p->ldP1 / 2);
        if (p->ns == 3)
            hipLaunchKernelGGL(k_ff_integrand_split<3>, dim3(grid_for(w1)), dim3(256), 0, s, q, u, E, p->d_S1b, mx,
                               my, mz, d, p->kb1, p->ldP1, p->ps1);
        else
            hipLaunchKernelGGL(k_ff_integrand_split<2>, dim3(grid_for(w1)), dim3(256), 0, s, q, u, E, p->d_S1b, mx,
                               my, mz, d, p->kb1, p->ldP1, p->ps1);
    }
    return hipGetLastError();
}

// The GEMM stages: T[m][x] (2D), or T1 then T2 (3D).
hipError_t ff_plan_contract(FarFieldPlan *p, const LevelGeom &g, hipStream_t s)
{
    const int d = g.dim, mx = g.m[0], my = g.m[1];
    if (p->ns == 0) {
        if (d == 3) launch_gemm(p->L1, s);
        launch_gemm(p->L2, s);
    } else {
        if (d == 3) {
            launch_gemm_bf16(p->B1, p->ns, p->variant, s);
            const int NG = (int)p->gval.size();
            const long w2 = (long)p->kb2 * (p->ldP2 / 2);
            dim3 grid(std::min<unsigned>(grid_for(w2), 4096u), (unsigned)NG);
            if (p->ns == 3)
                hipLaunchKernelGGL(k_split_field<3>, grid, dim3(256), 0, s, p->d_T1, (long)mx * my, my, (long)mx,
                                   p->d_S2b, p->gs2, p->kb2, p->ldP2, p->ps2);
            else
                hipLaunchKernelGGL(k_split_field<2>, grid, dim3(256), 0, s, p->d_T1, (long)mx * my, my, (long)mx,
                                   p->d_S2b, p->gs2, p->kb2, p->ldP2, p->ps2);
        }
        launch_gemm_bf16(p->B2, p->ns, p->variant, s);
    }
    return hipGetLastError();
}

// F_m = e^{i d gamma} prod h sum_x Px[m][x] T[m][x], into F_out (device, M
// complex, the caller's direction order).
hipError_t ff_plan_finish(FarFieldPlan *p, const LevelGeom &g, double gamma, cd *F_out, hipStream_t s)
{
    const int d = g.dim, M = p->M, mx = g.m[0];
    double vol = 1.0;
    for (int k = 0; k < d; ++k) vol *= g.h[k];
    cd pre = {vol * cos(d * gamma), vol * sin(d * gamma)};
    hipLaunchKernelGGL(k_ff_final, dim3(M), dim3(256), 0, s, p->d_Plast, p->d_T2, M, mx, pre, p->d_F);
    hipLaunchKernelGGL(k_unpermute, dim3(ceil_div(M, 256)), dim3(256), 0, s, p->d_F, p->d_perm, M, F_out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Far fields of many 2D instances with the split-BF16 contraction in one
// launch per stage (farfield_map_batched): the instances' axis factors, their
// integrand planes, the GEMMs of every instance of one grid size (one group
// per instance, each with its operator's factor planes), the final dot
// products and the reordering.  Each stage keeps the per-instance block
// structure of the single-map kernels, so every map equals farfield_map's.
struct FFBJob {
    const cd *q, *u;          // the operator's finest q, the instance's solution (null: the Born term)
    cd *E;                    // its plane-wave factors (mx + my)
    us8 *planes;              // its integrand planes
    cd *T, *Fs;               // its GEMM result (M x mx) and sorted map
    cd *F;                    // the output row (the caller's direction order)
    const cd *Plast;          // the operator's x factors (M x mx, sorted order)
    const int *perm;
    int mx, my, kb_tot;
    long ldP, pstride;
    double lo[2], h[2], cr[2], ci[2];
    cd pre;
};

__global__ __launch_bounds__(256) void k_ffb_axis(const FFBJob *__restrict__ jobs)
{
    const FFBJob &J = jobs[blockIdx.y];
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int ax = i < J.mx ? 0 : 1, k = i < J.mx ? i : i - J.mx;
    if (i >= J.mx + J.my) return;
    const double x = J.lo[ax] + (double)(k + 1) * J.h[ax];
    const double mag = exp(J.cr[ax] * x), ph = J.ci[ax] * x;
    J.E[i] = cd{mag * cos(ph), mag * sin(ph)};
}

template <int NS>
__global__ __launch_bounds__(256) void k_ffb_integrand(const FFBJob *__restrict__ jobs)
{
    const FFBJob &J = jobs[blockIdx.y];
    const int mx = J.mx, my = J.my;
    const cd *Ex = J.E, *Ey = J.E + mx;
    const long ncols = J.ldP / 2;
    const long tot = (long)J.kb_tot * ncols;
    for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < tot; e += (long)gridDim.x * 256) {
        const long n = e % ncols;
        const int kb = (int)(e / ncols);
        const bool colin = n < mx;
        const int ix = (int)(colin ? n : 0);
        cd v[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int k = 8 * kb + i;
            const bool in = colin && k < my;
            const size_t j = in ? (size_t)k * mx + n : 0;
            const cd uin = Ex[ix] * Ey[in ? k : 0];
            const cd t = J.u ? uin + J.u[j] : uin;
            const cd sv = J.q[j] * t;
            v[i] = in ? sv : cd{0.0, 0.0};
        }
        store_split8<NS>(v, J.planes, J.pstride, (long)kb * J.ldP + 2 * n);
    }
}

__global__ __launch_bounds__(256) void k_ffb_final(const FFBJob *__restrict__ jobs, int M)
{
    const FFBJob &J = jobs[blockIdx.y];
    __shared__ double red[2][4];
    const int m = blockIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (m >= M) return;
    const int K = J.mx;
    double re = 0.0, im = 0.0;
    const cd *pr = J.Plast + (size_t)m * K, *tr = J.T + (size_t)m * K;
    for (int k = threadIdx.x; k < K; k += 256) {
        cd v = pr[k] * tr[k];
        re += v.re;
        im += v.im;
    }
    for (int off = 32; off > 0; off >>= 1) {
        re += __shfl_down(re, off, 64);
        im += __shfl_down(im, off, 64);
    }
    if (lane == 0) {
        red[0][wave] = re;
        red[1][wave] = im;
    }
    __syncthreads();
    if (threadIdx.x == 0)
        J.Fs[m] = J.pre * cd{(red[0][0] + red[0][1]) + (red[0][2] + red[0][3]),
                             (red[1][0] + red[1][1]) + (red[1][2] + red[1][3])};
}

__global__ __launch_bounds__(256) void k_ffb_unpermute(const FFBJob *__restrict__ jobs, int M)
{
    const FFBJob &J = jobs[blockIdx.y];
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < M) J.F[J.perm[i]] = J.Fs[i];
}

struct FFBatch {
    std::vector<uint64_t> key;    // the operators' serials per instance, then M
    std::vector<void *> bufs;
    FFBJob *d_jobs = nullptr;
    std::vector<FFBJob> jobs;
    // one GEMM launch per grid size: its groups (uploaded) and shape
    std::vector<GemmLaunchB> gl;
    std::vector<int> gl_variant;
    int M = 0, ns = 0, max_cols = 0, max_ax = 0;
    ~FFBatch()
    {
        for (void *b : bufs) (void)hipFree(b);
    }
    template <typename P>
    hipError_t alloc(P **p, size_t bytes)
    {
        void *v = nullptr;
        hipError_t e = hipMalloc(&v, bytes ? bytes : 16);
        if (e != hipSuccess) return e;
        bufs.push_back(v);
        *p = (P *)v;
        return hipSuccess;
    }
};

void ff_batch_destroy(FFBatch *b) { delete b; }

hipError_t ff_batch_run(FFBatch **cache, const std::vector<uint64_t> &key, const std::vector<FFBInst> &in, int M,
                        hipStream_t s)
{
    const int n = (int)in.size();
    FFBatch *B = *cache;
    if (!B || B->key != key) {
        if (B) {
            FF_CHECK(hipStreamSynchronize(s));
            delete B;
            *cache = nullptr;
        }
        // built aside and published (with its key) only once complete, so a
        // failed build leaves no workspace behind
        std::unique_ptr<FFBatch> nb(new FFBatch());
        B = nb.get();
        B->M = M;
        B->ns = in[0].plan->ns;
        B->jobs.resize(n);
        // grid-size classes (the GEMM needs one ksteps and row stride per launch)
        std::vector<std::vector<int>> classes;
        std::vector<std::pair<int, int>> shapes;
        for (int i = 0; i < n; ++i) {
            const FarFieldPlan *p = in[i].plan;
            const LevelGeom &g = *in[i].g;
            FFBJob &J = B->jobs[i];
            J.mx = g.m[0];
            J.my = g.m[1];
            J.kb_tot = p->kb1;
            J.ldP = p->ldP1;
            J.pstride = p->ps1;
            J.Plast = p->d_Plast;
            J.perm = p->d_perm;
            FF_CHECK(B->alloc(&J.E, (size_t)(J.mx + J.my) * sizeof(cd)));
            FF_CHECK(B->alloc(&J.planes, (size_t)p->ns * p->ps1 * sizeof(us8)));
            FF_CHECK(B->alloc(&J.T, (size_t)M * J.mx * sizeof(cd)));
            FF_CHECK(B->alloc(&J.Fs, (size_t)M * sizeof(cd)));
            B->max_cols = std::max<int>(B->max_cols, (int)(p->kb1 * (p->ldP1 / 2)));
            B->max_ax = std::max(B->max_ax, J.mx + J.my);
            const std::pair<int, int> sh(J.mx, J.my);
            int c = (int)(std::find(shapes.begin(), shapes.end(), sh) - shapes.begin());
            if (c == (int)shapes.size()) {
                shapes.push_back(sh);
                classes.emplace_back();
            }
            classes[c].push_back(i);
        }
        for (const std::vector<int> &cl : classes) {
            std::vector<GemmGroupB> gr;
            int maxrt = 0;
            for (int i : cl) {
                const FarFieldPlan *p = in[i].plan;
                const GemmGroupB &G0 = p->h_B2g;   // the plan's own group (its factor planes)
                gr.push_back(GemmGroupB{G0.A, G0.a_split, (const bf8 *)B->jobs[i].planes, p->ps1, B->jobs[i].T,
                                        (long)B->jobs[i].mx, G0.M, G0.Nc, G0.rtiles});
                maxrt = std::max(maxrt, G0.rtiles);
            }
            GemmGroupB *dg = nullptr;
            FF_CHECK(B->alloc(&dg, gr.size() * sizeof(GemmGroupB)));
            FF_CHECK(hipMemcpy(dg, gr.data(), gr.size() * sizeof(GemmGroupB), hipMemcpyHostToDevice));
            const FarFieldPlan *p0 = in[cl[0]].plan;
            B->gl.push_back(GemmLaunchB{dg, (int)cl.size(), p0->B2.ksteps, maxrt, p0->ldP1});
            B->gl_variant.push_back(p0->variant);
        }
        FF_CHECK(B->alloc(&B->d_jobs, (size_t)n * sizeof(FFBJob)));
        B->key = key;
        *cache = nb.release();
    }
    // per call: the directions' plane waves, solutions and output rows
    for (int i = 0; i < n; ++i) {
        FFBJob &J = B->jobs[i];
        const LevelGeom &g = *in[i].g;
        J.q = in[i].q;
        J.u = in[i].u;
        J.F = in[i].F;
        const double ar = -(in[i].k0 * sin(in[i].gamma)), ai = in[i].k0 * cos(in[i].gamma);
        for (int k = 0; k < 2; ++k) {
            J.lo[k] = g.lo[k];
            J.h[k] = g.h[k];
            J.cr[k] = ar * in[i].eta[k];
            J.ci[k] = ai * in[i].eta[k];
        }
        const double vol = g.h[0] * g.h[1];
        J.pre = cd{vol * cos(2 * in[i].gamma), vol * sin(2 * in[i].gamma)};
    }
    FF_CHECK(hipMemcpyAsync(B->d_jobs, B->jobs.data(), (size_t)n * sizeof(FFBJob), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_ffb_axis, dim3(ceil_div(B->max_ax, 256), n), dim3(256), 0, s, B->d_jobs);
    const dim3 gi(std::min<unsigned>(grid_for(B->max_cols), 4096u), (unsigned)n);
    if (B->ns == 3) hipLaunchKernelGGL(k_ffb_integrand<3>, gi, dim3(256), 0, s, B->d_jobs);
    else hipLaunchKernelGGL(k_ffb_integrand<2>, gi, dim3(256), 0, s, B->d_jobs);
    for (size_t c = 0; c < B->gl.size(); ++c) launch_gemm_bf16(B->gl[c], B->ns, B->gl_variant[c], s);
    hipLaunchKernelGGL(k_ffb_final, dim3(M, n), dim3(256), 0, s, B->d_jobs, M);
    hipLaunchKernelGGL(k_ffb_unpermute, dim3(ceil_div(M, 256), n), dim3(256), 0, s, B->d_jobs, M);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Far-field map without device allocation (farfield_map_noalloc).  The FP64
// MFMA contraction of ff_plan_* with the same kernels and launch shapes, but
// every device buffer (axis factors, direction table, packed factors, GEMM
// descriptors, integrand, stage results, F) is carved from one file-scope
// device array.  Its device address is taken once per device at set-up
// (ff_scratch_init, called by mg_setup with the device current) and only that
// address is used on the host.  The direction grouping is staged in
// file-scope host arrays under a mutex, so no host heap is used either.
static __device__ __align__(256) unsigned char scratch[FFMG_NOALLOC_SCRATCH_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[NOALLOC_MAX_DEVICES];

struct NoAllocHost {
    int perm[FFMG_NOALLOC_MAX_DIRS];
    int gstart[FFMG_NOALLOC_MAX_DIRS + 1];
    double gval[FFMG_NOALLOC_MAX_DIRS];
    double al[4 * FFMG_NOALLOC_MAX_DIRS];
    GemmGroup gr[FFMG_NOALLOC_MAX_DIRS + 1];
};
static NoAllocHost g_na_host;
static std::mutex g_na_mu;

hipError_t ff_scratch_init(int device)
{
    if (device < 0 || device >= NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return hipSuccess;
    void *ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = ptr;
    return hipSuccess;
}

namespace {
// bump allocation inside the scratch array (256-byte aligned offsets)
struct Carve {
    size_t off = 0;
    template <typename T>
    size_t take(size_t count)
    {
        size_t o = off;
        off = (size_t)round_up((long)(o + count * sizeof(T)), 256);
        return o;
    }
};
}  // namespace

int ff_noalloc_map(const LevelGeom &g, double k0, double gamma, const double eta[3], const cd *q, const cd *u,
                   int M, const double *dirs, cd *F_out, bool out_on_device, int device, hipStream_t s,
                   size_t *need, hipError_t *herr)
{
    *herr = hipSuccess;
    unsigned char *base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (device >= 0 && device < NOALLOC_MAX_DEVICES) base = (unsigned char *)g_scratch_ptr[device];
    }
    if (!base) return 2;   // set-up did not run on this device
    if (M < 1 || M > FFMG_NOALLOC_MAX_DIRS) return 3;
    const int d = g.dim, mx = g.m[0], my = g.m[1], mz = g.m[2];
    const long N = (long)g.N();

    std::lock_guard<std::mutex> lk(g_na_mu);
    NoAllocHost &H = g_na_host;
    // group directions by their last component (exact equality) in 3D, in the
    // order a stable sort gives (ties keep the caller's order)
    for (int i = 0; i < M; ++i) H.perm[i] = i;
    if (d == 3)
        std::sort(H.perm, H.perm + M, [&](int a, int b) {
            const double za = dirs[a * 3 + 2], zb = dirs[b * 3 + 2];
            return za < zb || (za == zb && a < b);
        });
    int NG = 0;
    for (int i = 0; i < M; ++i) {
        double v = (d == 3) ? dirs[H.perm[i] * 3 + 2] : 0.0;
        if (i == 0 || (d == 3 && v != H.gval[NG - 1])) {
            H.gstart[NG] = i;
            H.gval[NG] = v;
            ++NG;
        }
    }
    H.gstart[NG] = M;
    int maxM = 0;
    for (int gi = 0; gi < NG; ++gi) maxM = std::max(maxM, H.gstart[gi + 1] - H.gstart[gi]);

    // layout
    const int ks_y = ceil_div(my, 4), ks_z = ceil_div(mz, 4);
    const int rt1 = ceil_div(2L * NG, 16);
    Carve c;
    const size_t oE = c.take<cd>((size_t)mx + my + mz);
    const size_t oAl = c.take<double>((size_t)3 * M + NG);
    const size_t oPerm = c.take<int>((size_t)M);
    const size_t oPl = c.take<cd>((size_t)M * mx);
    const size_t oT2 = c.take<cd>((size_t)M * mx);
    const size_t oF = c.take<cd>((size_t)M);
    const size_t oFo = out_on_device ? 0 : c.take<cd>((size_t)M);
    const size_t oS = c.take<cd>((size_t)N);
    size_t a2tot = 0;
    for (int gi = 0; gi < NG; ++gi) a2tot += (size_t)ceil_div(2L * (H.gstart[gi + 1] - H.gstart[gi]), 16) * ks_y * 64;
    const size_t oA2 = c.take<double>(a2tot);
    const size_t oA1 = (d == 3) ? c.take<double>((size_t)rt1 * ks_z * 64) : 0;
    const size_t oT1 = (d == 3) ? c.take<cd>((size_t)NG * mx * my) : 0;
    const size_t oGr = c.take<GemmGroup>((size_t)NG + 1);
    *need = c.off;
    if (c.off > (size_t)FFMG_NOALLOC_SCRATCH_BYTES) return 1;

    cd *dE = (cd *)(base + oE), *dPl = (cd *)(base + oPl), *dT2 = (cd *)(base + oT2), *dF = (cd *)(base + oF);
    cd *dS = (cd *)(base + oS), *dT1 = (cd *)(base + oT1);
    double *dAl = (double *)(base + oAl), *dA2 = (double *)(base + oA2), *dA1 = (double *)(base + oA1);
    int *dPerm = (int *)(base + oPerm);
    GemmGroup *dGr = (GemmGroup *)(base + oGr);
    cd *Fd = out_on_device ? F_out : (cd *)(base + oFo);

    // direction table: sorted alphas per axis [3][M], then one alpha_z per group
    for (size_t i = 0; i < (size_t)3 * M + NG; ++i) H.al[i] = 0.0;
    for (int i = 0; i < M; ++i)
        for (int k = 0; k < d; ++k) H.al[(size_t)k * M + i] = dirs[(size_t)H.perm[i] * d + k];
    for (int gi = 0; gi < NG; ++gi) H.al[(size_t)3 * M + gi] = H.gval[gi];
    // GEMM descriptors (device addresses inside the scratch array)
    int ng = 0;
    size_t off2 = 0;
    if (d == 3) H.gr[ng++] = GemmGroup{dA1, (const double *)dS, dT1, NG, rt1};
    for (int gi = 0; gi < NG; ++gi) {
        const int Mg = H.gstart[gi + 1] - H.gstart[gi], rt = ceil_div(2L * Mg, 16);
        const double *S = (d == 3) ? (const double *)(dT1 + (size_t)gi * mx * my) : (const double *)dS;
        H.gr[ng++] = GemmGroup{dA2 + off2, S, dT2 + (size_t)H.gstart[gi] * mx, Mg, rt};
        off2 += (size_t)rt * ks_y * 64;
    }
#define NA_CHECK(x)                                                                                                  \
    do {                                                                                                             \
        hipError_t e_ = (x);                                                                                         \
        if (e_ != hipSuccess) {                                                                                      \
            *herr = e_;                                                                                              \
            return 4;                                                                                                \
        }                                                                                                            \
    } while (0)
    // pageable host sources: each copy has consumed its source when it returns
    NA_CHECK(hipMemcpyAsync(dAl, H.al, ((size_t)3 * M + NG) * sizeof(double), hipMemcpyHostToDevice, s));
    NA_CHECK(hipMemcpyAsync(dPerm, H.perm, (size_t)M * sizeof(int), hipMemcpyHostToDevice, s));
    NA_CHECK(hipMemcpyAsync(dGr, H.gr, (size_t)ng * sizeof(GemmGroup), hipMemcpyHostToDevice, s));

    // plane-wave axis factors exp(i k0 e^{ig} eta_k x): c = -k0 sin g eta_k + i k0 cos g eta_k
    int eo = 0;
    for (int k = 0; k < 3; ++k) {
        const double ek = (k < d) ? eta[k] : 0.0;
        hipLaunchKernelGGL(k_axis_exp, dim3(ceil_div(g.m[k], 256)), dim3(256), 0, s, dE + eo, g.m[k], g.lo[k],
                           g.h[k], -(k0 * sin(gamma)) * ek, (k0 * cos(gamma)) * ek);
        eo += g.m[k];
    }
    hipLaunchKernelGGL(k_plain_factor, dim3(grid_for((long)M * mx)), dim3(256), 0, s, dPl, dAl, M, mx, g.lo[0],
                       g.h[0], k0, gamma);
    off2 = 0;
    for (int gi = 0; gi < NG; ++gi) {
        const int Mg = H.gstart[gi + 1] - H.gstart[gi], rt = ceil_div(2L * Mg, 16);
        hipLaunchKernelGGL(k_pack_factor, dim3(grid_for((long)rt * ks_y * 64)), dim3(256), 0, s, dA2 + off2,
                           dAl + (size_t)1 * M + H.gstart[gi], Mg, my, rt, ks_y, g.lo[1], g.h[1], k0, gamma);
        off2 += (size_t)rt * ks_y * 64;
    }
    if (d == 3)
        hipLaunchKernelGGL(k_pack_factor, dim3(grid_for((long)rt1 * ks_z * 64)), dim3(256), 0, s, dA1,
                           dAl + (size_t)3 * M, NG, mz, rt1, ks_z, g.lo[2], g.h[2], k0, gamma);
    hipLaunchKernelGGL(k_ff_integrand, dim3(grid_for(N)), dim3(256), 0, s, q, u, (const cd *)dE, dS, mx, my,
                       (d == 3) ? mz : 1);
    if (d == 3) {
        launch_gemm(GemmLaunch{dGr, 1, mz, mx * my, NG, 2L * mx * my, (long)mx * my}, s);
        launch_gemm(GemmLaunch{dGr + 1, NG, my, mx, maxM, 2L * mx, (long)mx}, s);
    } else {
        launch_gemm(GemmLaunch{dGr, 1, my, mx, maxM, 2L * mx, (long)mx}, s);
    }
    double vol = 1.0;
    for (int k = 0; k < d; ++k) vol *= g.h[k];
    const cd pre = {vol * cos(d * gamma), vol * sin(d * gamma)};
    hipLaunchKernelGGL(k_ff_final, dim3(M), dim3(256), 0, s, (const cd *)dPl, (const cd *)dT2, M, mx, pre, dF);
    hipLaunchKernelGGL(k_unpermute, dim3(ceil_div(M, 256)), dim3(256), 0, s, (const cd *)dF, (const int *)dPerm, M,
                       Fd);
    NA_CHECK(hipGetLastError());
    if (!out_on_device) {
        NA_CHECK(hipMemcpyAsync(F_out, Fd, (size_t)M * sizeof(cd), hipMemcpyDeviceToHost, s));
        NA_CHECK(hipStreamSynchronize(s));
    }
#undef NA_CHECK
    return 0;
}

void launch_axis_exp(cd *out, int m, double lo, double h, double cr, double ci, hipStream_t s)
{
    hipLaunchKernelGGL(k_axis_exp, dim3(ceil_div(m, 256)), dim3(256), 0, s, out, m, lo, h, cr, ci);
}

// ---------------------------------------------------------------------------
// The same FP64 MFMA contraction for a caller's factor table instead of the
// plane-wave exponentials (the test-function integrals of the ionisation
// amplitudes): C[m][n] = sum_k A[m][k] S[k][n].  A is packed into the A'
// layout of k_ff_gemm_f64 (Re / Im rows per tile_row_map), the group
// descriptor is written on the device, and one launch runs the GEMM.
__global__ __launch_bounds__(256) void k_pack_table(double *__restrict__ out, const cd *__restrict__ A, int M, int K,
                                                    int rtiles, int ksteps)
{
    size_t tot = (size_t)rtiles * ksteps * 64;
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < tot; e += (size_t)gridDim.x * 256) {
        int l = (int)(e % 64);
        size_t t = e / 64;
        int ks = (int)(t % ksteps), rt = (int)(t / ksteps);
        int mloc, c;
        tile_row_map(l % 16, mloc, c);
        int m = 8 * rt + mloc, k = 4 * ks + l / 16;
        double v = 0.0;
        if (m < M && k < K) {
            cd a = A[(size_t)m * K + k];
            v = c ? a.im : a.re;
        }
        out[e] = v;
    }
}

__global__ void k_set_group(GemmGroup *g, const double *A, const double *S, cd *C, int M, int rtiles)
{
    *g = GemmGroup{A, S, C, M, rtiles};
}

static size_t align256(size_t b) { return (b + 255) / 256 * 256; }

size_t table_gemm_ws_bytes(int M, int K)
{
    const int rt = ceil_div(2L * M, 16), ks = ceil_div(K, 4);
    return align256(sizeof(GemmGroup)) + align256((size_t)rt * ks * 64 * sizeof(double));
}

void table_gemm_f64(const cd *A, int M, int K, const cd *S, int Nc, cd *C, void *ws, hipStream_t s)
{
    const int rt = ceil_div(2L * M, 16), ks = ceil_div(K, 4);
    GemmGroup *dg = (GemmGroup *)ws;
    double *Ap = (double *)((char *)ws + align256(sizeof(GemmGroup)));
    hipLaunchKernelGGL(k_pack_table, dim3(grid_for((long)rt * ks * 64)), dim3(256), 0, s, Ap, A, M, K, rt, ks);
    hipLaunchKernelGGL(k_set_group, dim3(1), dim3(1), 0, s, dg, (const double *)Ap, (const double *)S, C, M, rt);
    GemmLaunch L{dg, 1, K, Nc, M, 2L * Nc, (long)Nc};
    launch_gemm(L, s);
}

void launch_rows_dot(const cd *P, const cd *T, int M, int K, cd pre, cd *F, hipStream_t s)
{
    hipLaunchKernelGGL(k_ff_final, dim3(M), dim3(256), 0, s, P, T, M, K, pre, F);
}

}  // namespace ffmg
