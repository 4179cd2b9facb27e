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
#include <math.h>

#include <algorithm>
#include <vector>

#include "ffmg_internal.hpp"

namespace ffmg {

typedef double d4 __attribute__((ext_vector_type(4)));

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

// F_m = pre * sum_x P[m][x] T[m][x]; one wave per direction.
__global__ __launch_bounds__(256) void k_ff_final(const cd *__restrict__ P, const cd *__restrict__ T, int M, int K,
                                                  cd pre, cd *__restrict__ F)
{
    int m = blockIdx.x * 4 + (threadIdx.x >> 6);
    int lane = threadIdx.x & 63;
    if (m >= M) return;
    double re = 0.0, im = 0.0;
    const cd *pr = P + (size_t)m * K, *tr = T + (size_t)m * K;
    for (int k = lane; k < K; k += 64) {
        cd v = pr[k] * tr[k];
        re += v.re;
        im += v.im;
    }
    for (int off = 32; off > 0; off >>= 1) {
        re += __shfl_down(re, off, 64);
        im += __shfl_down(im, off, 64);
    }
    if (lane == 0) F[m] = pre * cd{re, im};
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

struct FarFieldPlan {
    int dim = 0;
    int M = 0;
    const cd *s_field = nullptr;   // integrand buffer the groups point at
    std::vector<double> dirs;      // cache key
    std::vector<int> perm;         // sorted position -> direction index
    std::vector<int> gstart;       // group start in sorted order
    std::vector<double> gval;      // alpha_z per group
    double *d_alpha = nullptr;     // sorted alphas per axis [3][M], then group alphas
    double *d_A1 = nullptr;        // packed Pz (3D): rows = groups
    double *d_A2 = nullptr;        // packed Py, one block per group
    cd *d_Plast = nullptr;         // plain Px [M][mx], sorted order
    cd *d_T1 = nullptr, *d_T2 = nullptr, *d_F = nullptr;
    int *d_perm = nullptr;
    GemmGroup *d_groups = nullptr; // [0]: stage 1 (3D), [1..]: last GEMM stage
    GemmLaunch L1, L2;
    void release()
    {
        (void)hipFree(d_alpha);
        (void)hipFree(d_A1);
        (void)hipFree(d_A2);
        (void)hipFree(d_Plast);
        (void)hipFree(d_T1);
        (void)hipFree(d_T2);
        (void)hipFree(d_F);
        (void)hipFree(d_perm);
        (void)hipFree(d_groups);
        d_alpha = d_A1 = d_A2 = nullptr;
        d_Plast = d_T1 = d_T2 = d_F = nullptr;
        d_perm = nullptr;
        d_groups = nullptr;
        M = dim = 0;
        dirs.clear();
    }
    ~FarFieldPlan() { release(); }
};

FarFieldPlan *ff_plan_create() { return new FarFieldPlan(); }
void ff_plan_destroy(FarFieldPlan *p) { delete p; }

#define FF_CHECK(x)                                                                                                  \
    do {                                                                                                             \
        hipError_t e_ = (x);                                                                                         \
        if (e_ != hipSuccess) return e_;                                                                             \
    } while (0)

// (Re)build the direction-dependent factors and the GEMM descriptors when the
// directions (or the integrand buffer) change.  Synchronises the stream.
hipError_t ff_plan_prepare(FarFieldPlan *p, const LevelGeom &g, double k0, double gamma, int M, const double *dirs,
                           const cd *s_field, hipStream_t s)
{
    const int d = g.dim;
    std::vector<double> key(dirs, dirs + (size_t)M * d);
    if (p->M == M && p->dim == d && p->dirs == key && p->s_field == s_field) return hipSuccess;
    FF_CHECK(hipStreamSynchronize(s));
    p->release();
    p->dim = d;
    p->M = M;
    p->dirs = key;
    p->s_field = s_field;
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
    FF_CHECK(hipMalloc(&p->d_alpha, al.size() * sizeof(double)));
    FF_CHECK(hipMemcpy(p->d_alpha, al.data(), al.size() * sizeof(double), hipMemcpyHostToDevice));
    FF_CHECK(hipMalloc(&p->d_perm, (size_t)M * sizeof(int)));
    FF_CHECK(hipMemcpy(p->d_perm, p->perm.data(), (size_t)M * sizeof(int), hipMemcpyHostToDevice));

    const int mx = g.m[0], my = g.m[1], mz = g.m[2];
    FF_CHECK(hipMalloc(&p->d_Plast, (size_t)M * mx * sizeof(cd)));
    hipLaunchKernelGGL(k_plain_factor, dim3(std::min(65536, ceil_div((long)M * mx, 256))), dim3(256), 0, s,
                       p->d_Plast, p->d_alpha, M, mx, g.lo[0], g.h[0], k0, gamma);
    // packed Py per group (rows = the directions of the group)
    const int ks_y = ceil_div(my, 4);
    std::vector<size_t> off(NG);
    size_t tot = 0;
    for (int gi = 0; gi < NG; ++gi) {
        int Mg = p->gstart[gi + 1] - p->gstart[gi];
        off[gi] = tot;
        tot += (size_t)ceil_div(2L * Mg, 16) * ks_y * 64;
    }
    FF_CHECK(hipMalloc(&p->d_A2, tot * sizeof(double)));
    for (int gi = 0; gi < NG; ++gi) {
        int Mg = p->gstart[gi + 1] - p->gstart[gi];
        int rt = ceil_div(2L * Mg, 16);
        size_t n = (size_t)rt * ks_y * 64;
        hipLaunchKernelGGL(k_pack_factor, dim3((unsigned)std::min<size_t>(65536, (n + 255) / 256)), dim3(256), 0,
                           s, p->d_A2 + off[gi], p->d_alpha + (size_t)1 * M + p->gstart[gi], Mg, my, rt, ks_y,
                           g.lo[1], g.h[1], k0, gamma);
    }
    std::vector<GemmGroup> gr;
    if (d == 3) {
        const int ks_z = ceil_div(mz, 4);
        int rt = ceil_div(2L * NG, 16);
        size_t n = (size_t)rt * ks_z * 64;
        FF_CHECK(hipMalloc(&p->d_A1, n * sizeof(double)));
        hipLaunchKernelGGL(k_pack_factor, dim3((unsigned)std::min<size_t>(65536, (n + 255) / 256)), dim3(256), 0,
                           s, p->d_A1, p->d_alpha + (size_t)3 * M, NG, mz, rt, ks_z, g.lo[2], g.h[2], k0, gamma);
        FF_CHECK(hipMalloc(&p->d_T1, (size_t)NG * mx * my * sizeof(cd)));
        // stage 1: T1[p][yx] = sum_z Pz[p][z] s[z][yx]
        gr.push_back(GemmGroup{p->d_A1, (const double *)s_field, p->d_T1, NG, rt});
    }
    FF_CHECK(hipMalloc(&p->d_T2, (size_t)M * mx * sizeof(cd)));
    FF_CHECK(hipMalloc(&p->d_F, (size_t)M * sizeof(cd)));
    int maxM = 0;
    for (int gi = 0; gi < NG; ++gi) {
        int Mg = p->gstart[gi + 1] - p->gstart[gi];
        maxM = std::max(maxM, Mg);
        const double *S = (d == 3) ? (const double *)(p->d_T1 + (size_t)gi * mx * my) : (const double *)s_field;
        gr.push_back(GemmGroup{p->d_A2 + off[gi], S, p->d_T2 + (size_t)p->gstart[gi] * mx, Mg, ceil_div(2L * Mg, 16)});
    }
    FF_CHECK(hipMalloc(&p->d_groups, gr.size() * sizeof(GemmGroup)));
    FF_CHECK(hipMemcpy(p->d_groups, gr.data(), gr.size() * sizeof(GemmGroup), hipMemcpyHostToDevice));
    if (d == 3) {
        p->L1 = GemmLaunch{p->d_groups, 1, mz, mx * my, NG, 2L * mx * my, (long)mx * my};
        p->L2 = GemmLaunch{p->d_groups + 1, NG, my, mx, maxM, 2L * mx, (long)mx};
    } else {
        p->L2 = GemmLaunch{p->d_groups, 1, my, mx, maxM, 2L * mx, (long)mx};
    }
    FF_CHECK(hipGetLastError());
    return hipStreamSynchronize(s);
}

// Contract the integrand (the buffer given at prepare) into F (device, M
// complex, the caller's direction order).
hipError_t ff_plan_execute(FarFieldPlan *p, const LevelGeom &g, double gamma, cd *F_out, hipStream_t s)
{
    const int d = g.dim, M = p->M, mx = g.m[0];
    if (d == 3) launch_gemm(p->L1, s);
    launch_gemm(p->L2, s);
    double vol = 1.0;
    for (int k = 0; k < d; ++k) vol *= g.h[k];
    cd pre = {vol * cos(d * gamma), vol * sin(d * gamma)};
    hipLaunchKernelGGL(k_ff_final, dim3(ceil_div(M, 4)), dim3(256), 0, s, p->d_Plast, p->d_T2, M, mx, pre, p->d_F);
    hipLaunchKernelGGL(k_unpermute, dim3(ceil_div(M, 256)), dim3(256), 0, s, p->d_F, p->d_perm, M, F_out);
    return hipGetLastError();
}

void launch_ff_integrand(const LevelGeom &g, const cd *q, const cd *u, const cd *E, cd *s, hipStream_t st)
{
    size_t N = g.N();
    size_t nb = (N + 255) / 256;
    if (nb > 65536) nb = 65536;
    hipLaunchKernelGGL(k_ff_integrand, dim3((unsigned)nb), dim3(256), 0, st, q, u, E, s, g.m[0], g.m[1],
                       g.dim == 3 ? g.m[2] : 1);
}

void launch_axis_exp(cd *out, int m, double lo, double h, double cr, double ci, hipStream_t s)
{
    hipLaunchKernelGGL(k_axis_exp, dim3(ceil_div(m, 256)), dim3(256), 0, s, out, m, lo, h, cr, ci);
}

}  // namespace ffmg
