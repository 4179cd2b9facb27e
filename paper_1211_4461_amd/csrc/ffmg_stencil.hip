// ffmg_stencil.hip -- the multigrid kernels of the contour solver on gfx950:
// operator / residual / weighted-Jacobi sweeps (Sec. 3.2 eq. csg; Sec. 4
// omega-Jacobi), full-weighting restriction and bilinear / trilinear
// interpolation (Sec. 4), residual norms, and the setup kernels (contrast,
// injected coarse coefficients, exact inverse of the coarsest operator as in
// the F(5) cycle of Sec. 5.7, plane-wave right-hand side of Sec. 2.1).
//
// All of these are HBM-bandwidth bound (about one flop per byte).  The sweeps
// stage a u tile with its halo in LDS (2D: one 64 x TY tile; 3D: the centre
// z-plane of a 64 x 8 column that marches in z, with the z-neighbours held in
// registers), read b and q once, coalesced, and write the result once.
#include <math.h>

#include <algorithm>

#include "ffmg_internal.hpp"
#include "ffmg_point.hpp"

namespace ffmg {

constexpr int TY2 = 16;   // 2D tile: 64 x 16 points per 256-thread block
constexpr int TY3 = 8;    // 3D tile: 64 x 8 points per plane
constexpr int TZ3 = 32;   // 3D: planes per block on large grids (fewer on small ones, planes_per_block)
// A z-marching block is latency bound (one plane after the other), so small
// grids get fewer planes per block and more blocks: the planes per block
// halve from the maximum until the grid has at least min_blocks blocks.  A
// pass that runs ahead of its output recomputes its lead planes in every
// block, so the two-sweep and fused pre-smoothing passes keep more planes (a
// lower floor): on the coarse levels of a 511^3 solve 23.0 ms against 23.7
// with the common floor, the finest level unchanged.
constexpr int MIN_BLOCKS3 = 2048;
constexpr int MIN_BLOCKS_SWEEP3 = 1024;   // two-sweep pass, two planes ahead
constexpr int MIN_BLOCKS_SRR3 = 512;      // fused pre-smoothing pass, seven planes ahead

static int planes_per_block(long xy_tiles, int mz, int maxp, long min_blocks = MIN_BLOCKS3)
{
    int tz = maxp;
    while (tz > 1 && xy_tiles * ((mz + tz - 1) / tz) < min_blocks) tz >>= 1;
    return tz;
}

template <typename T>
Stencil<T> make_stencil(const LevelGeom &g, double gamma, double k02, double omega)
{
    Stencil<T> P;
    P.mx = g.m[0];
    P.my = g.m[1];
    P.mz = g.m[2];
    double cr = cos(-2.0 * gamma), ci = sin(-2.0 * gamma);
    double s2 = 0.0;
    P.rot = cx<T>{T(cr), T(ci)};
    for (int k = 0; k < 3; ++k) {
        if (k < g.dim) {
            double ih2 = 1.0 / (g.h[k] * g.h[k]);
            P.c[k] = cx<T>{T(cr * ih2), T(ci * ih2)};
            P.ih2[k] = T(ih2);
            s2 += 2.0 * ih2;
        } else {
            P.c[k] = cx<T>{T(0), T(0)};
            P.ih2[k] = T(0);
        }
    }
    P.csum2 = cx<T>{T(cr * s2), T(ci * s2)};
    P.k02 = T(k02);
    P.omega = T(omega);
    P.omc = T(1.0 - omega);
    return P;
}
template Stencil<double> make_stencil<double>(const LevelGeom &, double, double, double);
template Stencil<float> make_stencil<float>(const LevelGeom &, double, double, double);

// ---------------------------------------------------------------------------
// The point update shared by all stencil kernels.
// MODE_RESID writes rscale * r converted to TO (the FP64 residual of the
// refinement loop is written as a scaled FP32 right-hand side this way).
// L = sum_k (2u - u_- - u_+)/h_k^2, the weighted second differences, except
// for MODE_JACOBI, where it is the neighbour sum N = sum_k (u_- + u_+)/h_k^2.
template <typename T, typename TO, int MODE>
__device__ __forceinline__ void point_update(const Stencil<T> &P, T rscale, cx<T> uc, cx<T> L, size_t j,
                                             const cx<T> *__restrict__ b, const cx<T> *__restrict__ q,
                                             cx<TO> *__restrict__ out, double &acc)
{
    cx<T> qj = q[j];
    if (MODE == MODE_APPLY) {
        out[j] = cvt<TO>(apply_point(P, L, uc, qj));
    } else if (MODE == MODE_JACOBI0) {
        out[j] = cvt<TO>(jacobi0_w(b[j], jweight(P, qj)));
    } else if (MODE == MODE_JACOBI) {
        out[j] = cvt<TO>(jacobi_n(P, L, uc, b[j], jweight(P, qj)));
    } else {
        cx<T> r = resid_from(P, L, uc, b[j], qj);
        if (MODE == MODE_RESID) out[j] = cvt<TO>(rscale * r);
        acc += (double)abs2(r);
    }
}

// The point update of a 3D pass with b_j and q_j already in registers.
template <typename T, typename TO, int MODE>
__device__ __forceinline__ void point_update_v(const Stencil<T> &P, T rscale, cx<T> uc, cx<T> L, size_t j, cx<T> bj,
                                               cx<T> qj, cx<TO> *__restrict__ out, double &acc)
{
    if (MODE == MODE_APPLY) {
        out[j] = cvt<TO>(apply_point(P, L, uc, qj));
    } else if (MODE == MODE_JACOBI0) {
        out[j] = cvt<TO>(jacobi0_w(bj, jweight(P, qj)));
    } else if (MODE == MODE_JACOBI) {
        out[j] = cvt<TO>(jacobi_n(P, L, uc, bj, jweight(P, qj)));
    } else {
        cx<T> r = resid_from(P, L, uc, bj, qj);
        if (MODE == MODE_RESID) out[j] = cvt<TO>(rscale * r);
        acc += (double)abs2(r);
    }
}

__device__ __forceinline__ void block_sum_256(double acc, double *slot)
{
    __shared__ double red[4];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) red[w] = acc;
    __syncthreads();
    if (threadIdx.x == 0) *slot = (red[0] + red[1]) + (red[2] + red[3]);
}

// 2D: 256 threads as 64 (x) x 4 (y), tile 64 x TY2, u tile + halo in LDS.
// TAG only separates the finest-level launches into their own kernel symbol
// (so a profiler's per-kernel statistics cover exactly those launches).
// PW: the right-hand side is the plane wave's q u_in from the factors pwf
// (b not read; FP64 residuals only).
template <typename T, typename TO, int MODE, bool PW = false>
__device__ __forceinline__ void stencil2d_body(const cx<T> *__restrict__ u, const cx<T> *__restrict__ b,
                                               const cx<T> *__restrict__ q, cx<TO> *__restrict__ out,
                                               const Stencil<T> &P, T rscale, int tiles_x, int tile,
                                               double *__restrict__ slot, const cd *__restrict__ pwf = nullptr)
{
    static_assert(!PW || (sizeof(T) == 8 && MODE == MODE_RESID), "plane-wave b: FP64 residuals");
    __shared__ cx<T> s[TY2 + 2][66];
    const int mx = P.mx, my = P.my;
    int tx0 = (tile % tiles_x) * 64, ty0 = (tile / tiles_x) * TY2;
    const bool zero_u = (MODE == MODE_JACOBI0);
    if (!zero_u) {
        for (int i = threadIdx.x; i < (TY2 + 2) * 66; i += 256) {
            int ly = i / 66, lx = i - ly * 66;
            int gx = tx0 + lx - 1, gy = ty0 + ly - 1;
            s[ly][lx] = ld_masked(u, (size_t)gy * mx + gx, gx >= 0 && gx < mx && gy >= 0 && gy < my);
        }
        __syncthreads();
    }
    const int lx = threadIdx.x & 63;
    const int gx = tx0 + lx;
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < TY2 / 4; ++k) {
        int ly = (threadIdx.x >> 6) + 4 * k;
        int gy = ty0 + ly;
        if (gx < mx && gy < my) {
            size_t j = (size_t)gy * mx + gx;
            cx<T> uc = {T(0), T(0)}, lap = {T(0), T(0)};
            if (!zero_u) {
                uc = s[ly + 1][lx + 1];
                if (MODE == MODE_JACOBI)
                    lap = nsum_xy(P, s[ly + 1][lx], s[ly + 1][lx + 2], s[ly][lx + 1], s[ly + 2][lx + 1]);
                else
                    lap = lap_xy(P, uc, s[ly + 1][lx], s[ly + 1][lx + 2], s[ly][lx + 1], s[ly + 2][lx + 1]);
            }
            if constexpr (PW) {
                const cx<T> qj = q[j];
                point_update_v<T, TO, MODE>(P, rscale, uc, lap, j, qj * pw_uin(pwf, gx, gy, 0, mx, my, 2), qj, out,
                                            acc);
            } else {
                point_update<T, TO, MODE>(P, rscale, uc, lap, j, b, q, out, acc);
            }
        }
    }
    if (MODE == MODE_RESID || MODE == MODE_RNORM)
        if (slot) block_sum_256(acc, slot);
}

template <typename T, typename TO, int MODE, int TAG>
__global__ __launch_bounds__(256) void k_stencil2d(const cx<T> *__restrict__ u, const cx<T> *__restrict__ b,
                                                   const cx<T> *__restrict__ q, cx<TO> *__restrict__ out,
                                                   Stencil<T> P, T rscale, int tiles_x, double *__restrict__ partial,
                                                   const SolveCtl *__restrict__ ctl, const int *__restrict__ stop)
{
    if (stop && *stop) return;
    if (ctl) rscale = T(1.0 / ctl->scale_next);
    stencil2d_body<T, TO, MODE>(u, b, q, out, P, rscale, tiles_x, xcd_tile(blockIdx.x, gridDim.x),
                                partial ? partial + blockIdx.x : nullptr);
}

// Linear interpolation: fine node f (1-based) takes coarse nodes floor(f/2)
// and ceil(f/2) with weights 1 (f even) or 1/2 (f odd), tensorised; coarse
// boundary values are zero.  One thread per fine point, summed z-outer.
template <typename T>
__device__ __forceinline__ T iw(int f, int C)
{
    int d = f - 2 * C;
    return d == 0 ? T(1) : ((d == 1 || d == -1) ? T(0.5) : T(0));
}

// Trilinear weights of a fine node along one axis (1-based fine index f):
// the lower coarse node (f >> 1) - 1 (0-based) and the next one take 1 and 0
// (f even: the fine node lies on the coarse one) or 1/2 and 1/2 (f odd).
template <typename T>
__device__ __forceinline__ void lin_w(int f, T (&w)[2])
{
    w[0] = (f & 1) ? T(0.5) : T(1);
    w[1] = (f & 1) ? T(0.5) : T(0);
}

// The 3D interpolation in the order every 3D kernel uses (so that the fused
// and the one-operation paths agree bit for bit): at each of the four coarse
// (x, y) neighbours the two coarse planes are combined first,
//   ez = wz0 c(az) + wz1 c(az + 1),
// then acc = sum over (y, x) neighbours of (wx wy) ez, y outer, from zero;
// every term is formed, coarse values outside the grid being zero.
template <typename T>
__device__ __forceinline__ cx<T> zpair(T w0, cx<T> c0, T w1, cx<T> c1)
{
    return w0 * c0 + w1 * c1;
}

// (P e_c) at fine interior point (ix, iy, iz) (0-based).
template <typename T, int DIM>
__device__ __forceinline__ cx<T> prolong_at(const cx<T> *__restrict__ ec, int ix, int iy, int iz, int mxc, int myc,
                                            int mzc)
{
    int fx = ix + 1, fy = iy + 1, fz = iz + 1;
    if constexpr (DIM == 3) {
        T wx[2], wy[2], wz[2];
        lin_w(fx, wx);
        lin_w(fy, wy);
        lin_w(fz, wz);
        const int ax = (fx >> 1) - 1, ay = (fy >> 1) - 1, az = (fz >> 1) - 1;
        auto c = [&](int x, int y, int z) -> cx<T> {
            const bool in = x >= 0 && y >= 0 && z >= 0 && x < mxc && y < myc && z < mzc;
            return in ? ec[((size_t)z * myc + y) * mxc + x] : cx<T>{T(0), T(0)};
        };
        cx<T> acc = {T(0), T(0)};
        for (int jy = 0; jy < 2; ++jy)
            for (int jx = 0; jx < 2; ++jx)
                acc = acc + (wx[jx] * wy[jy]) * zpair(wz[0], c(ax + jx, ay + jy, az), wz[1], c(ax + jx, ay + jy, az + 1));
        return acc;
    }
    cx<T> acc = {T(0), T(0)};
    int zlo = (DIM == 3) ? fz / 2 : 1, zhi = (DIM == 3) ? (fz + 1) / 2 : 1;
    for (int Cz = zlo; Cz <= zhi; ++Cz)
        for (int Cy = fy / 2; Cy <= (fy + 1) / 2; ++Cy)
            for (int Cx = fx / 2; Cx <= (fx + 1) / 2; ++Cx) {
                T wgt = iw<T>(fx, Cx) * iw<T>(fy, Cy) * ((DIM == 3) ? iw<T>(fz, Cz) : T(1));
                if (wgt == T(0)) continue;
                int ax = Cx - 1, ay = Cy - 1, az = (DIM == 3) ? Cz - 1 : 0;
                if (ax < 0 || ay < 0 || az < 0 || ax >= mxc || ay >= myc || az >= mzc) continue;
                acc = acc + wgt * ec[((size_t)az * myc + ay) * mxc + ax];
            }
    return acc;
}

// 3D: 256 threads as 64 (x) x 4 (y); each block owns a 64 x TY3 column of
// TZ3 planes and marches up in z.  The centre plane (with its x/y halo) is
// staged in a double-buffered LDS plane; u at z-1 and z+1 stays in registers.
// SRC says where the u values of the stencil come from:
//   SRC_MEM   u in memory;
//   SRC_ZERO2 the first of two sweeps from a zero guess, omega b / D, formed
//             for every value the second sweep reads (two sweeps in one pass);
//   SRC_PROL  u + P e_c, the coarse-grid correction formed on the fly (the
//             interpolation fused into the first post-smoothing sweep); the
//             coarse planes the tile needs are staged in an LDS ring as the
//             block marches up, and the interpolation is branch free: the
//             terms are summed in the order of k_prolong_add, whose skipped
//             terms (zero weight, or coarse nodes outside the grid, zero in
//             LDS) add exact zeros here.
// The per-point arithmetic is that of the separate kernels, so the fused
// passes reproduce them bit for bit.
//   SRC_UPD   u + s d, the FP64 update of the mixed-precision refinement
//             with the FP32 correction d (the residual of the updated
//             iterate is formed in the same pass, and the updated iterate
//             written to unew at the block's own points).
enum { SRC_MEM = 0, SRC_ZERO2 = 1, SRC_PROL = 2, SRC_UPD = 3, SRC_PSET = 4, SRC_PSETUPD = 5 };

// SRC_PSET: u = s P e_c, the full multigrid start's interpolation of the FP32
// first-level solution e_c scaled by s (the arithmetic of k_prolong_set<float,
// double, 3>), formed in the pass and stored.  SRC_PSETUPD: the first
// refinement step's update of that start, s P e_c + scale d (SRC_UPD with the
// iterate formed instead of read).
// Full multigrid transfers.  The scale s = sqrt(bnorm2) / sqrt(N) (the RMS
// of the finest right-hand side; 1 without bnorm2) keeps an FP32 hierarchy
// at unit size: the start is computed for b / s and multiplied back by s.
__device__ __forceinline__ double fmg_scale(const double *bnorm2, double inv_sqN)
{
    if (!bnorm2) return 1.0;
    double s = sqrt(bnorm2[0]) * inv_sqN;
    return (s > 0.0 && isfinite(s)) ? s : 1.0;
}

struct PsetArgs {
    const cf *ec = nullptr;
    const double *bnorm2 = nullptr;   // the scale s = fmg_scale(bnorm2, inv_sqN)
    double inv_sqN = 1.0;
};
template <int SRC, typename T>
struct CoarseType {
    using type = T;
};
template <typename T>
struct CoarseType<SRC_PSET, T> {
    using type = float;
};
template <typename T>
struct CoarseType<SRC_PSETUPD, T> {
    using type = float;
};


// Raw loads of one stencil value (the source form is applied when it is used).
template <typename T>
struct Raw3 {
    cx<T> a;   // u (SRC_MEM, SRC_PROL, SRC_UPD) or b (SRC_ZERO2)
    cx<T> c;   // d widened exactly (SRC_UPD) or q (SRC_ZERO2)
};

// PW: the right-hand side is the plane-wave one, formed as q u_in from the
// per-axis factors pwf where a point needs it (b is not read; FP64 only).
template <typename T, typename TO, int MODE, int SRC, bool PW = false>
__device__ __forceinline__ void stencil3d_body(const cx<T> *__restrict__ u, const cx<T> *__restrict__ ec,
                                               const cx<T> *__restrict__ b, const cx<T> *__restrict__ q,
                                               cx<TO> *__restrict__ out, const Stencil<T> &P, T rscale, int tiles_x,
                                               int tiles_y, int tz, double *__restrict__ partial,
                                               const cf *__restrict__ dcorr = nullptr, double dscale = 0.0,
                                               cx<T> *__restrict__ unew = nullptr, const cd *__restrict__ pwf = nullptr,
                                               PsetArgs pset = PsetArgs())
{
    static_assert(!PW || (sizeof(T) == 8 && MODE != MODE_APPLY && SRC != SRC_ZERO2), "plane-wave b: FP64 residuals");
    static_assert((SRC != SRC_PSET && SRC != SRC_PSETUPD) || sizeof(T) == 8, "the start's interpolation: FP64");
    using TC = typename CoarseType<SRC, T>::type;   // number type of the staged coarse planes
    const double psc = (SRC == SRC_PSET || SRC == SRC_PSETUPD) ? fmg_scale(pset.bnorm2, pset.inv_sqN) : 1.0;
    constexpr bool STAGE = (SRC == SRC_PROL || SRC == SRC_PSET || SRC == SRC_PSETUPD);
    constexpr bool PSET = (SRC == SRC_PSET || SRC == SRC_PSETUPD);
    constexpr int PY = TY3 / 4;
    constexpr int NH = 2 * TY3 + 2 * 66;   // halo values of a plane: the x sides, then the y rows
    // coarse tile of the fine tile plus its one-point halo: 34 x (TY3/2 + 2)
    constexpr int CW = 34, CH = TY3 / 2 + 2, NCS = STAGE ? 4 : 1;
    constexpr bool ZU = (MODE == MODE_JACOBI0);   // the stencil's u is zero: no u is read
    constexpr bool NEED_B = (MODE != MODE_APPLY);
    __shared__ cx<T> s[2][TY3 + 2][66];
    __shared__ cx<TC> cs[NCS][STAGE ? CH : 1][STAGE ? CW : 1];
    const int mx = P.mx, my = P.my, mz = P.mz;
    const int mxc = (mx - 1) / 2, myc = (my - 1) / 2, mzc = (mz - 1) / 2;
    int tile = xcd_tile(blockIdx.x, gridDim.x);
    int txi = tile % tiles_x;
    int rest = tile / tiles_x;
    int tyi = rest % tiles_y, tzi = rest / tiles_y;
    const int x0 = txi * 64, y0 = tyi * TY3, z0 = tzi * tz;
    const int z1 = min(z0 + tz, mz);
    const int lx = threadIdx.x & 63, ly0 = threadIdx.x >> 6;
    const int gx = x0 + lx;
    const size_t plane = (size_t)mx * my;
    const unsigned pbytes = (unsigned)(plane * sizeof(cx<T>));
    const cx<T> zero = {T(0), T(0)};
    const int cx0 = (x0 >> 1) - 1, cy0 = (y0 >> 1) - 1;   // coarse origin of cs

    // coarse plane a (0-based) into ring slot a & 3, zero outside the grid
    auto load_coarse = [&](int a) {
        for (int t = threadIdx.x; t < CH * CW; t += 256) {
            const int yy = t / CW, xx = t - yy * CW;
            const int ax = cx0 + xx, ay = cy0 + yy;
            const bool in = a >= 0 && a < mzc && ax >= 0 && ax < mxc && ay >= 0 && ay < myc;
            const size_t ci = ((size_t)a * myc + ay) * mxc + ax;
            if constexpr (PSET) cs[a & (NCS - 1)][yy][xx] = ld_masked(pset.ec, ci, in);
            else cs[a & (NCS - 1)][yy][xx] = ld_masked(ec, ci, in);
        }
    };
    // (P e_c) at fine point (x, y, z) from the staged coarse planes (the
    // order of prolong_at<T, 3>)
    auto interp = [&](int x, int y, int z) -> cx<TC> {
        const int fx = x + 1, fy = y + 1, fz = z + 1;
        const int ex = (fx >> 1) - 1 - cx0, ey = (fy >> 1) - 1 - cy0, az = (fz >> 1) - 1;
        TC wx[2], wy[2], wz[2];
        lin_w(fx, wx);
        lin_w(fy, wy);
        lin_w(fz, wz);
        const int s0 = az & (NCS - 1), s1 = (az + 1) & (NCS - 1);
        cx<TC> acc = {TC(0), TC(0)};
#pragma unroll
        for (int jy = 0; jy < 2; ++jy)
#pragma unroll
            for (int jx = 0; jx < 2; ++jx)
                acc = acc + (wx[jx] * wy[jy]) * zpair(wz[0], cs[s0][ey + jy][ex + jx], wz[1], cs[s1][ey + jy][ex + jx]);
        return acc;
    };

    // own points (gx, y0 + ly0 + 4 i) and this thread's halo value of a plane
    unsigned offo[PY];
    bool ino[PY];
#pragma unroll
    for (int i = 0; i < PY; ++i) {
        const int gy = y0 + ly0 + 4 * i;
        ino[i] = gx < mx && gy < my;
        offo[i] = ino[i] ? (unsigned)(gy * mx + gx) * (unsigned)sizeof(cx<T>) : BUF_OOB;
    }
    const bool hact = threadIdx.x < NH;   // this thread loads a halo value
    int hly = 0, hlx = 0;                 // its LDS position
    {
        const int t = threadIdx.x;
        if (t < 2 * TY3) {
            const int side = t / TY3, yy = t - side * TY3;
            hlx = side ? 65 : 0;
            hly = yy + 1;
        } else {
            const int t2 = t - 2 * TY3;
            const int side = t2 / 66, xx = t2 - side * 66;
            hly = side ? TY3 + 1 : 0;
            hlx = xx;
        }
    }
    const int hx = x0 + hlx - 1, hy = y0 + hly - 1;
    const bool inh = hact && hx >= 0 && hx < mx && hy >= 0 && hy < my;
    const unsigned offh = inh ? (unsigned)(hy * mx + hx) * (unsigned)sizeof(cx<T>) : BUF_OOB;

    // raw loads of a plane at the byte offset off (zero outside the grid)
    auto fetch = [&](int z, unsigned off) -> Raw3<T> {
        const bool zin = z >= 0 && z < mz;
        const size_t o = zin ? (size_t)z * plane : 0;
        const unsigned nb = zin ? pbytes : 0u;
        Raw3<T> r;
        r.c = zero;
        if constexpr (SRC == SRC_ZERO2) {
            r.a = ld_buf<T>(buf_rsrc(b + o, nb), off);
            r.c = ld_buf<T>(buf_rsrc(q + o, nb), off);
        } else if constexpr (SRC == SRC_PSET) {
            r.a = zero;   // u is formed from the staged coarse planes
        } else if constexpr (SRC == SRC_PSETUPD) {
            r.a = zero;   // u is formed from the staged coarse planes, d is read
            const unsigned offd = (off == BUF_OOB) ? BUF_OOB : off / 2u;
            const cf dj = ld_buf<float>(buf_rsrc(dcorr + o, nb / 2u), offd);
            r.c = cx<T>{(T)dj.re, (T)dj.im};
        } else {
            r.a = ld_buf<T>(buf_rsrc(u + o, nb), off);
            if constexpr (SRC == SRC_UPD) {
                const unsigned offd = (off == BUF_OOB) ? BUF_OOB : off / 2u;   // FP32 complex: half the bytes
                const cf dj = ld_buf<float>(buf_rsrc(dcorr + o, nb / 2u), offd);
                r.c = cx<T>{(T)dj.re, (T)dj.im};
            }
        }
        return r;
    };
    // the stencil value from its raw loads (in: the point lies in the grid)
    auto finish = [&](const Raw3<T> &r, bool in, int x, int y, int z) -> cx<T> {
        if constexpr (SRC == SRC_ZERO2) {
            return in ? jacobi0_w(r.a, jweight(P, r.c)) : zero;
        } else if constexpr (SRC == SRC_PROL) {
            return in ? r.a + interp(x, y, z) : r.a;
        } else if constexpr (SRC == SRC_PSET) {
            if (!in) return zero;
            const cx<TC> v = interp(x, y, z);
            return cx<T>{(T)v.re * psc, (T)v.im * psc};
        } else if constexpr (SRC == SRC_PSETUPD) {
            if (!in) return zero;
            const cx<TC> v = interp(x, y, z);
            const cx<T> uo = {(T)v.re * psc, (T)v.im * psc};
            return cx<T>{uo.re + dscale * r.c.re, uo.im + dscale * r.c.im};
        } else if constexpr (SRC == SRC_UPD) {
            return in ? cx<T>{r.a.re + dscale * r.c.re, r.a.im + dscale * r.c.im} : r.a;
        } else {
            return r.a;
        }
    };
    auto zin_of = [&](int z) { return z >= 0 && z < mz; };

    // coarse planes a = ((iz + 1) >> 1) - 1 .. (iz + 1) >> 1 serve fine plane iz
    int a_hi = 0;
    if (STAGE) {
        for (int a = (z0 >> 1) - 1; a <= ((z0 + 1) >> 1); ++a) load_coarse(a);
        a_hi = (z0 + 1) >> 1;
        __syncthreads();
    }

    cx<T> prev[PY], cur[PY], nxt[PY];
    Raw3<T> rn[PY], rh;   // loads of the next plane (own points) and of this plane's halo, one plane ahead
    cx<T> bo[PY], qo[PY];  // b, q of the own points of the next plane
    if (!ZU) {
#pragma unroll
        for (int i = 0; i < PY; ++i) {
            const int gy = y0 + ly0 + 4 * i;
            prev[i] = finish(fetch(z0 - 1, offo[i]), ino[i] && zin_of(z0 - 1), gx, gy, z0 - 1);
            cur[i] = finish(fetch(z0, offo[i]), ino[i] && zin_of(z0), gx, gy, z0);
            rn[i] = fetch(z0 + 1, offo[i]);
        }
        rh = fetch(z0, offh);
    }
    // plane-wave b: E_x E_y of the own points (fixed through the march)
    cx<T> exy[PY];
#pragma unroll
    for (int i = 0; i < PY; ++i) {
        exy[i] = zero;
        if constexpr (PW)
            if (ino[i]) exy[i] = pwf[gx] * pwf[mx + y0 + ly0 + 4 * i];
    }
    auto fetch_bq = [&](int z) {
        const bool zin = zin_of(z);
        const size_t o = zin ? (size_t)z * plane : 0;
        const unsigned nb = zin ? pbytes : 0u;
        const auto rq = buf_rsrc(q + o, nb);
        if constexpr (PW) {
            const cx<T> ez = zin ? pwf[mx + my + z] : zero;
#pragma unroll
            for (int i = 0; i < PY; ++i) {
                qo[i] = ld_buf<T>(rq, offo[i]);
                bo[i] = qo[i] * (exy[i] * ez);
            }
        } else {
            const auto rb = buf_rsrc(b + o, nb);
#pragma unroll
            for (int i = 0; i < PY; ++i) {
                if (NEED_B) bo[i] = ld_buf<T>(rb, offo[i]);
                qo[i] = ld_buf<T>(rq, offo[i]);
            }
        }
    };
#pragma unroll
    for (int i = 0; i < PY; ++i) bo[i] = qo[i] = zero;
    fetch_bq(z0);

    double acc = 0.0;
    int it = 0;
    for (int z = z0; z < z1; ++z, ++it) {
        const int buf = it & 1;
        if (STAGE && ((z + 2) >> 1) > a_hi) {
            // the slot it takes held plane a_hi - 3, which no fine plane >= z
            // reads; every thread has passed the barrier after its last use
            load_coarse(++a_hi);
            __syncthreads();
        }
        cx<T> bc[PY], qc[PY];
#pragma unroll
        for (int i = 0; i < PY; ++i) {
            bc[i] = bo[i];
            qc[i] = qo[i];
        }
        if (!ZU) {
#pragma unroll
            for (int i = 0; i < PY; ++i) s[buf][ly0 + 4 * i + 1][lx + 1] = cur[i];
            if (hact) s[buf][hly][hlx] = finish(rh, inh && zin_of(z), hx, hy, z);
#pragma unroll
            for (int i = 0; i < PY; ++i)
                nxt[i] = finish(rn[i], ino[i] && zin_of(z + 1), gx, y0 + ly0 + 4 * i, z + 1);
            // the next plane's loads, in flight across the barrier
            if (z + 1 < z1) {
#pragma unroll
                for (int i = 0; i < PY; ++i) rn[i] = fetch(z + 2, offo[i]);
                rh = fetch(z + 1, offh);
            }
        }
        if (z + 1 < z1) fetch_bq(z + 1);
        if (!ZU) lds_barrier();
#pragma unroll
        for (int i = 0; i < PY; ++i) {
            int ly = ly0 + 4 * i;
            int gy = y0 + ly;
            if (ino[i]) {
                size_t j = (size_t)z * plane + (size_t)gy * mx + gx;
                cx<T> uc = {T(0), T(0)}, lap = {T(0), T(0)};
                if (!ZU) {
                    uc = cur[i];
                    if (MODE == MODE_JACOBI) {
                        lap = nsum_xy(P, s[buf][ly + 1][lx], s[buf][ly + 1][lx + 2], s[buf][ly][lx + 1],
                                      s[buf][ly + 2][lx + 1]);
                        lap = nsum_add_z(P, lap, prev[i], nxt[i]);
                    } else {
                        lap = lap_xy(P, uc, s[buf][ly + 1][lx], s[buf][ly + 1][lx + 2], s[buf][ly][lx + 1],
                                     s[buf][ly + 2][lx + 1]);
                        lap = lap_add_z(P, lap, uc, prev[i], nxt[i]);
                    }
                }
                point_update_v<T, TO, MODE>(P, rscale, uc, lap, j, bc[i], qc[i], out, acc);
                if constexpr (SRC == SRC_UPD || SRC == SRC_PSETUPD) unew[j] = uc;
                if constexpr (SRC == SRC_PSET)
                    if (unew) unew[j] = uc;
            }
        }
        if (!ZU) {
#pragma unroll
            for (int i = 0; i < PY; ++i) {
                prev[i] = cur[i];
                cur[i] = nxt[i];
            }
        }
    }
    if (MODE == MODE_RESID || MODE == MODE_RNORM)
        if (partial) block_sum_256(acc, partial + blockIdx.x);
}

template <typename T, typename TO, int MODE, int TAG>
__global__ __launch_bounds__(256) void k_stencil3d(const cx<T> *__restrict__ u, const cx<T> *__restrict__ b,
                                                   const cx<T> *__restrict__ q, cx<TO> *__restrict__ out,
                                                   Stencil<T> P, T rscale, int tiles_x, int tiles_y, int tz,
                                                   double *__restrict__ partial, const SolveCtl *__restrict__ ctl,
                                                   const int *__restrict__ stop)
{
    if (stop && *stop) return;
    if (ctl) rscale = T(1.0 / ctl->scale_next);
    stencil3d_body<T, TO, MODE, SRC_MEM>(u, nullptr, b, q, out, P, rscale, tiles_x, tiles_y, tz, partial);
}

// One Jacobi sweep whose input is formed on the fly (SRC_ZERO2, SRC_PROL).
template <typename T, int SRC, int TAG>
__global__ __launch_bounds__(256) void k_sweep3d(const cx<T> *__restrict__ u, const cx<T> *__restrict__ ec,
                                                 const cx<T> *__restrict__ b, const cx<T> *__restrict__ q,
                                                 cx<T> *__restrict__ out, Stencil<T> P, int tiles_x, int tiles_y,
                                                 int tz, const int *__restrict__ stop)
{
    if (stop && *stop) return;
    stencil3d_body<T, T, MODE_JACOBI, SRC>(u, ec, b, q, out, P, T(1), tiles_x, tiles_y, tz, nullptr);
}

// Two weighted-Jacobi sweeps in one z-marching pass (temporal blocking).  A
// block owns a TXW x TY output tile of tz planes.  Its NT threads cover the
// tile with a two-point halo, (TXW + 4) x (TY + 4) columns, thread t taking
// the columns t, t + NT, ...; every thread keeps a column's last three
// values of each stage in registers (the z-neighbours) and the stage's
// current plane goes through LDS for the x/y neighbours:
//   stage 0  the input at plane z: u (SRC_MEM) or u + P e_c (SRC_PROL, the
//            coarse planes staged in an LDS ring), or zero (SRC_ZERO2: the
//            first sweep from a zero guess is omega b / D, which needs no
//            neighbour, so stage 0 does nothing);
//   stage 1  the first sweep at plane z - 1 on the tile with a one-point
//            halo (zero outside the grid);
//   stage 2  the second sweep at plane z - 2 on the tile, written to out.
// The planes of each stage alternate between two LDS buffers, so one
// barrier per plane orders every write before the reads of the next plane;
// the barrier fences LDS only, and every global load (u of the next plane, b
// and q of the plane stage 1 takes next, the next coarse plane) is issued one
// plane ahead, so that it is in flight across the barrier.  b and omega/D of
// a column are read at stage 1 and kept for stage 2.  The per-point
// arithmetic and its order are those of the single sweeps, so the result is
// bit for bit that of two k_stencil3d / k_sweep3d passes.
template <typename T, int SRC, int TY, int TAG, int TXW, int NT = 256>
__global__ __launch_bounds__(NT) void k_sweep2_3d(const cx<T> *__restrict__ u, const cx<T> *__restrict__ ec,
                                                   const cx<T> *__restrict__ b, const cx<T> *__restrict__ q,
                                                   cx<T> *__restrict__ out, Stencil<T> P, int tiles_x, int tiles_y,
                                                   int tz, const int *__restrict__ stop)
{
    if (stop && *stop) return;
    constexpr int W = TXW + 4, H = TY + 4, NP = W * H, NS = (NP + NT - 1) / NT;
    constexpr bool PROL = (SRC == SRC_PROL), ZERO = (SRC == SRC_ZERO2);
    constexpr int CW = TXW / 2 + 4, CH = TY / 2 + 4, NCS = PROL ? 4 : 1;
    constexpr int NCL = PROL ? (CH * CW + NT - 1) / NT : 1;   // coarse values per thread and plane
    __shared__ cx<T> L0[ZERO ? 1 : 2][ZERO ? 1 : NP], L1[2][NP];
    __shared__ cx<T> cs[NCS][PROL ? CH : 1][PROL ? CW : 1];
    // the coarse correction combined in z for a fine plane (the first step of
    // the interpolation), double-buffered by the fine plane's parity
    __shared__ cx<T> ezs[PROL ? 2 : 1][PROL ? CH * CW : 1];
    const int mx = P.mx, my = P.my, mz = P.mz;
    const int mxc = (mx - 1) / 2, myc = (my - 1) / 2, mzc = (mz - 1) / 2;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int txi = tile % tiles_x, rest = tile / tiles_x;
    const int tyi = rest % tiles_y, tzi = rest / tiles_y;
    const int x0 = txi * TXW, y0 = tyi * TY, z0 = tzi * tz, z1 = min(z0 + tz, mz);
    const size_t plane = (size_t)mx * my;
    const cx<T> zero = {T(0), T(0)};
    const int cx0 = (x0 >> 1) - 2, cy0 = (y0 >> 1) - 2;   // coarse origin of cs

    // column of slot k: region row r, column c; grid point (gx, gy).  Byte
    // offsets inside a plane for the buffer loads (BUF_OOB outside the grid,
    // or, for b and q, outside the stage-1 region).
    int ofs[NS];            // gy * mx + gx (valid where `ing` holds)
    unsigned offu[NS], offbq[NS];
    unsigned ing = 0, st1 = 0, st2 = 0;   // per slot: in the grid (x, y), stage-1 region, output
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        const int t = threadIdx.x + NT * k;
        const int r = t / W, c = t - r * W;
        const int gx = x0 - 2 + c, gy = y0 - 2 + r;
        const bool v = t < NP;
        const bool in = v && gx >= 0 && gx < mx && gy >= 0 && gy < my;
        const bool s1 = v && r >= 1 && r < H - 1 && c >= 1 && c < W - 1;
        ofs[k] = in ? gy * mx + gx : 0;
        offu[k] = in ? (unsigned)ofs[k] * (unsigned)sizeof(cx<T>) : BUF_OOB;
        offbq[k] = (in && s1) ? offu[k] : BUF_OOB;
        ing |= (unsigned)in << k;
        st1 |= (unsigned)s1 << k;
        st2 |= (unsigned)(in && r >= 2 && r < H - 2 && c >= 2 && c < W - 2) << k;
    }
    auto slot_in = [&](unsigned m, int k) { return ((m >> k) & 1u) != 0u; };
    const unsigned pbytes = (unsigned)(plane * sizeof(cx<T>));

    // coarse planes: values of plane a into registers (one plane ahead), then LDS
    cx<T> creg[NCL];
    unsigned offc[NCL];
#pragma unroll
    for (int i = 0; i < NCL; ++i) {
        const int t = threadIdx.x + NT * i;
        const int yy = t / CW, xx = t - yy * CW;
        const int ax = cx0 + xx, ay = cy0 + yy;
        const bool in = t < CH * CW && ax >= 0 && ax < mxc && ay >= 0 && ay < myc;
        offc[i] = in ? (unsigned)(ay * mxc + ax) * (unsigned)sizeof(cx<T>) : BUF_OOB;
    }
    auto fetch_coarse = [&](int a) {
        const bool ain = a >= 0 && a < mzc;
        const size_t cpl = (size_t)mxc * myc;
        const auto rc = buf_rsrc(ec + (ain ? (size_t)a * cpl : 0), ain ? (unsigned)(cpl * sizeof(cx<T>)) : 0u);
#pragma unroll
        for (int i = 0; i < NCL; ++i) creg[i] = ld_buf<T>(rc, offc[i]);
    };
    auto store_coarse = [&](int a) {
        cx<T> *dst = &cs[a & (NCS - 1)][0][0];
#pragma unroll
        for (int i = 0; i < NCL; ++i) {
            const int t = threadIdx.x + NT * i;
            if (t < CH * CW) dst[t] = creg[i];
        }
    };
    // the z step of the interpolation for fine plane z: ezs = wz0 c(az) + wz1 c(az + 1)
    auto combine_z = [&](int z) {
        T wz[2];
        lin_w(z + 1, wz);
        const int az = ((z + 1) >> 1) - 1;
        const cx<T> *c0 = &cs[az & (NCS - 1)][0][0], *c1 = &cs[(az + 1) & (NCS - 1)][0][0];
        cx<T> *dst = ezs[z & 1];
        for (int t = threadIdx.x; t < CH * CW; t += NT) dst[t] = zpair(wz[0], c0[t], wz[1], c1[t]);
    };
    // the x/y step at slot k: sum over (y, x) neighbours of (wx wy) ez, y outer
    // The weights depend only on the parities of the fine coordinates (x0 and
    // y0 are even, so on those of the slot's column and row): kept as two bits
    // per slot, the products (exact: 1, 1/2, 1/4, 0) formed at use.
    int eoff[NS];        // LDS offset of the slot's lower coarse (x, y) neighbour in ezs
    unsigned par = 0;    // bits 2k, 2k + 1: parity of fx, fy of slot k
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        const int t = threadIdx.x + NT * k;
        const int r = t / W, c = t - r * W;
        const int fx = x0 - 2 + c + 1, fy = y0 - 2 + r + 1;
        eoff[k] = (t < NP) ? ((fy >> 1) - 1 - cy0) * CW + ((fx >> 1) - 1 - cx0) : 0;
        par |= (unsigned)((fx & 1) | ((fy & 1) << 1)) << (2 * k);
    }
    auto interp_xy = [&](int k, const cx<T> *ez) -> cx<T> {
        const cx<T> *e = ez + eoff[k];
        T wx[2], wy[2];
        lin_w((int)((par >> (2 * k)) & 1u), wx);
        lin_w((int)((par >> (2 * k + 1)) & 1u), wy);
        cx<T> acc = {T(0), T(0)};
        acc = acc + (wx[0] * wy[0]) * e[0];
        acc = acc + (wx[1] * wy[0]) * e[1];
        acc = acc + (wx[0] * wy[1]) * e[CW];
        acc = acc + (wx[1] * wy[1]) * e[CW + 1];
        return acc;
    };
    // global loads of one plane: u (stage 0) and b, q (stage 1)
    cx<T> pu[NS], pb[NS], pq[NS];
    auto fetch_u = [&](int z) {
        const bool zin = z >= 0 && z < mz;
        const auto ru = buf_rsrc(u + (zin ? (size_t)z * plane : 0), zin ? pbytes : 0u);
#pragma unroll
        for (int k = 0; k < NS; ++k) pu[k] = ld_buf<T>(ru, offu[k]);
    };
    auto fetch_bq = [&](int z) {
        const bool zin = z >= 0 && z < mz;
        const size_t o = zin ? (size_t)z * plane : 0;
        const auto rb = buf_rsrc(b + o, zin ? pbytes : 0u), rq = buf_rsrc(q + o, zin ? pbytes : 0u);
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            pb[k] = ld_buf<T>(rb, offbq[k]);
            pq[k] = ld_buf<T>(rq, offbq[k]);
        }
    };

    // prologue: the coarse planes of the first three stage-0 planes in LDS
    // and the z step of the first; u of plane z0 - 2.  In the loop, the coarse
    // plane the z step will need two planes later is fetched into registers,
    // stored into the ring the next iteration and combined (at the end of
    // an iteration, for the next stage-0 plane) after a barrier.
    int a_reg = 0;
    bool c_pending = false;
    if (PROL) {
        const int Alo = ((z0 - 1) >> 1) - 1;
        for (int a = Alo; a <= ((z0 + 1) >> 1); ++a) {
            fetch_coarse(a);
            store_coarse(a);
        }
        a_reg = (z0 + 1) >> 1;
        lds_barrier();
        combine_z(z0 - 2);
        lds_barrier();
    }
#pragma unroll
    for (int k = 0; k < NS; ++k) pu[k] = pb[k] = pq[k] = zero;
    if (!ZERO) fetch_u(z0 - 2);

    cx<T> a0[NS], a1[NS], a2[NS];   // stage 0 at planes z - 2, z - 1, z
    cx<T> c0[NS], c1[NS], c2[NS];   // stage 1 at planes z - 3, z - 2, z - 1
    cx<T> bB[NS], wB[NS];           // b, omega / D at plane z - 2 (kept from stage 1)
    cx<T> wn[NS];                   // omega / D at plane z - 1
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        a0[k] = a1[k] = a2[k] = zero;
        c0[k] = c1[k] = c2[k] = zero;
        bB[k] = wB[k] = wn[k] = zero;
    }
    for (int z = z0 - 2; z <= z1 + 1; ++z) {
        // this plane's loads (issued last iteration), then the next plane's
        cx<T> un[NS], bn[NS], qn[NS];
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            un[k] = pu[k];
            bn[k] = pb[k];
            qn[k] = pq[k];
        }
        if (PROL) {
            if (c_pending) {   // fetched last iteration; combined from the next iteration on
                store_coarse(a_reg);
                c_pending = false;
            }
            if (((z + 4) >> 1) > a_reg) {
                fetch_coarse(++a_reg);
                c_pending = true;
            }
        }
        if (!ZERO && z + 1 <= z1 + 1) fetch_u(z + 1);
        if (z >= z0 - 1 && z <= z1) fetch_bq(z);

        // stage 0: the input at plane z
        if (!ZERO) {
            cx<T> *l0w = L0[z & 1];
            const bool zin = z >= 0 && z < mz;
#pragma unroll
            for (int k = 0; k < NS; ++k) {
                const int t = threadIdx.x + NT * k;
                cx<T> v = un[k];
                if (PROL && zin && slot_in(ing, k)) v = v + interp_xy(k, ezs[z & 1]);
                a0[k] = a1[k];
                a1[k] = a2[k];
                a2[k] = v;
                if (t < NP) l0w[t] = v;
            }
        }
        // stage 1: the first sweep at plane p1 = z - 1
        const int p1 = z - 1;
        if (p1 >= z0 - 1) {
            const cx<T> *l0r = L0[ZERO ? 0 : (p1 & 1)];
            cx<T> *l1w = L1[p1 & 1];
            const bool pin = p1 >= 0 && p1 < mz;
#pragma unroll
            for (int k = 0; k < NS; ++k) {
                const int t = threadIdx.x + NT * k;
                c0[k] = c1[k];
                c1[k] = c2[k];
                cx<T> v = zero, wj = zero;
                if (pin && slot_in(ing & st1, k)) {
                    wj = jweight(P, qn[k]);
                    if (ZERO) {
                        v = jacobi0_w(bn[k], wj);
                    } else {
                        cx<T> N = nsum_xy(P, l0r[t - 1], l0r[t + 1], l0r[t - W], l0r[t + W]);
                        N = nsum_add_z(P, N, a0[k], a2[k]);
                        v = jacobi_n(P, N, a1[k], bn[k], wj);
                    }
                }
                wn[k] = wj;
                c2[k] = v;
                if (slot_in(st1, k)) l1w[t] = v;
            }
        }
        // stage 2: the second sweep at plane p2 = z - 2, the block's output
        const int p2 = z - 2;
        if (p2 >= z0) {
            const cx<T> *l1r = L1[p2 & 1];
#pragma unroll
            for (int k = 0; k < NS; ++k) {
                const int t = threadIdx.x + NT * k;
                if (slot_in(st2, k)) {
                    cx<T> N = nsum_xy(P, l1r[t - 1], l1r[t + 1], l1r[t - W], l1r[t + W]);
                    N = nsum_add_z(P, N, c0[k], c2[k]);
                    out[(size_t)p2 * plane + ofs[k]] = jacobi_n(P, N, c1[k], bB[k], wB[k]);
                }
            }
        }
        // b, omega / D of plane z - 1 serve stage 2 next iteration
        if (p1 >= z0 - 1) {
#pragma unroll
            for (int k = 0; k < NS; ++k) {
                bB[k] = bn[k];
                wB[k] = wn[k];
            }
        }
        // the z step of the next stage-0 plane (its coarse planes have passed a barrier)
        if (PROL && z + 1 <= z1 + 1) combine_z(z + 1);
        lds_barrier();
    }
}

// The FP64 step of the mixed-precision refinement in one pass: u' = u + s d
// (s = ctl->scale_cur) into unew, and the residual b - A u' written as FP32
// scaled by 1 / ctl->scale_next, with the per-block FP64 sums of |b - A u'|^2.
// The same arithmetic as k_refine_update followed by the FP64 residual.
// START: the iterate is the full multigrid start s P e_c (PsetArgs), formed
// from the staged FP32 coarse planes instead of read.
template <bool PW, bool START = false>
__global__ __launch_bounds__(256) void k_refine3d(const cd *__restrict__ u, const cf *__restrict__ d,
                                                  const cd *__restrict__ b, const cd *__restrict__ q,
                                                  cd *__restrict__ unew, cf *__restrict__ r32, Stencil<double> P,
                                                  int tiles_x, int tiles_y, int tz, double *__restrict__ partial,
                                                  const SolveCtl *__restrict__ ctl, const int *__restrict__ stop,
                                                  const cd *__restrict__ pwf, PsetArgs ps)
{
    if (stop && *stop) return;
    const double rscale = 1.0 / ctl->scale_next;
    stencil3d_body<double, float, MODE_RESID, START ? SRC_PSETUPD : SRC_UPD, PW>(
        u, nullptr, b, q, r32, P, rscale, tiles_x, tiles_y, tz, partial, d, ctl->scale_cur, unew, pwf, ps);
}

// The FP64 residual of the plane-wave right-hand side written as scaled FP32
// (the 3D form of launch_resid_to_f32_ctl with b formed from pwf).
__global__ __launch_bounds__(256) void k_resid3d_pw(const cd *__restrict__ u, const cd *__restrict__ q,
                                                    cf *__restrict__ r32, Stencil<double> P, int tiles_x,
                                                    int tiles_y, int tz, double *__restrict__ partial,
                                                    const SolveCtl *__restrict__ ctl, const cd *__restrict__ pwf)
{
    const double rscale = 1.0 / ctl->scale_next;
    stencil3d_body<double, float, MODE_RESID, SRC_MEM, true>(u, nullptr, nullptr, q, r32, P, rscale, tiles_x,
                                                             tiles_y, tz, partial, nullptr, 0.0, nullptr, pwf);
}

// Blocks of a stencil launch on grid g: tiles in x (tx) and y (ty) and, in
// 3D, the planes each block marches through (tz).
static void grid_of(const LevelGeom &g, int &nb, int &tx, int &ty, int &tz)
{
    tx = (g.m[0] + 63) / 64;
    if (g.dim == 2) {
        ty = (g.m[1] + TY2 - 1) / TY2;
        tz = 1;
        nb = tx * ty;
    } else {
        ty = (g.m[1] + TY3 - 1) / TY3;
        tz = planes_per_block((long)tx * ty, g.m[2], TZ3);
        nb = tx * ty * ((g.m[2] + tz - 1) / tz);
    }
}

int stencil_blocks(const LevelGeom &g)
{
    int nb, tx, ty, tz;
    grid_of(g, nb, tx, ty, tz);
    return nb;
}

void stencil_grid2d(const LevelGeom &g, int *nb, int *tiles_x)
{
    int ty, tz;
    grid_of(g, *nb, *tiles_x, ty, tz);
}

template <typename T, typename TO, int MODE, int TAG = 0>
static void launch_mode(const LevelGeom &g, const Stencil<T> &P, T rscale, const cx<T> *u, const cx<T> *b,
                        const cx<T> *q, cx<TO> *out, double *partial, hipStream_t s, const SolveCtl *ctl = nullptr,
                        const int *stop = nullptr)
{
    int nb, tx, ty, tz;
    grid_of(g, nb, tx, ty, tz);
    if (g.dim == 2)
        hipLaunchKernelGGL((k_stencil2d<T, TO, MODE, TAG>), dim3(nb), dim3(256), 0, s, u, b, q, out, P, rscale, tx,
                           partial, ctl, stop);
    else
        hipLaunchKernelGGL((k_stencil3d<T, TO, MODE, TAG>), dim3(nb), dim3(256), 0, s, u, b, q, out, P, rscale, tx,
                           ty, tz, partial, ctl, stop);
}

template <typename T>
void launch_stencil(int mode, const LevelGeom &g, const Stencil<T> &P, const cx<T> *u, const cx<T> *b,
                    const cx<T> *q, cx<T> *out, double *partial, hipStream_t s, bool finest, const int *stop)
{
    const T one = T(1);
    if (finest && mode == MODE_JACOBI) {
        launch_mode<T, T, MODE_JACOBI, 1>(g, P, one, u, b, q, out, partial, s, nullptr, stop);
        return;
    }
    switch (mode) {
    case MODE_APPLY: launch_mode<T, T, MODE_APPLY>(g, P, one, u, b, q, out, partial, s, nullptr, stop); break;
    case MODE_RESID: launch_mode<T, T, MODE_RESID>(g, P, one, u, b, q, out, partial, s, nullptr, stop); break;
    case MODE_RNORM: launch_mode<T, T, MODE_RNORM>(g, P, one, u, b, q, out, partial, s, nullptr, stop); break;
    case MODE_JACOBI0: launch_mode<T, T, MODE_JACOBI0>(g, P, one, u, b, q, out, partial, s, nullptr, stop); break;
    default: launch_mode<T, T, MODE_JACOBI>(g, P, one, u, b, q, out, partial, s, nullptr, stop); break;
    }
}
template void launch_stencil<double>(int, const LevelGeom &, const Stencil<double> &, const cd *, const cd *,
                                     const cd *, cd *, double *, hipStream_t, bool, const int *);
template void launch_stencil<float>(int, const LevelGeom &, const Stencil<float> &, const cf *, const cf *,
                                    const cf *, cf *, double *, hipStream_t, bool, const int *);

template <typename T>
void launch_sweep3d_fused(bool zero2, const LevelGeom &g, const Stencil<T> &P, const cx<T> *u, const cx<T> *ec,
                          const cx<T> *b, const cx<T> *q, cx<T> *out, hipStream_t s, bool finest, const int *stop)
{
    int nb, tx, ty, tz;
    grid_of(g, nb, tx, ty, tz);
    if (zero2) {
        if (finest)
            hipLaunchKernelGGL((k_sweep3d<T, SRC_ZERO2, 1>), dim3(nb), dim3(256), 0, s, u, ec, b, q, out, P, tx, ty,
                               tz, stop);
        else
            hipLaunchKernelGGL((k_sweep3d<T, SRC_ZERO2, 0>), dim3(nb), dim3(256), 0, s, u, ec, b, q, out, P, tx, ty,
                               tz, stop);
    } else {
        if (finest)
            hipLaunchKernelGGL((k_sweep3d<T, SRC_PROL, 1>), dim3(nb), dim3(256), 0, s, u, ec, b, q, out, P, tx, ty,
                               tz, stop);
        else
            hipLaunchKernelGGL((k_sweep3d<T, SRC_PROL, 0>), dim3(nb), dim3(256), 0, s, u, ec, b, q, out, P, tx, ty,
                               tz, stop);
    }
}
// Tile of the fused two-sweep 3D kernel (its LDS and registers grow with
// the tile), by FFMG_TUNE_SWEEP3D variant: 0 the default per type (64 x 8
// FP32, 64 x 4 FP64), 2 twice the rows, 3 half the width and twice the rows
// (fewer halo columns per output point) for the interpolating pass and the
// default for the others (measured: the narrow tile pays off where the pass
// also stages coarse planes).
template <typename T> constexpr int sweep2_rows(int shape)
{
    return sizeof(T) == 4 ? (shape == 0 ? 8 : 16) : (shape == 0 ? 4 : 8);
}
constexpr int sweep2_width(int shape) { return shape == 3 ? 32 : 64; }

template <typename T, int TY, int TXW, int NT = 256>
static void launch_sweep2_3d_tile(const LevelGeom &g, const Stencil<T> &P, const cx<T> *u, const cx<T> *ec,
                                  const cx<T> *b, const cx<T> *q, cx<T> *out, hipStream_t s, bool finest,
                                  const int *stop, bool zero)
{
    const int tx = (g.m[0] + TXW - 1) / TXW, ty = (g.m[1] + TY - 1) / TY;
    const int tz = planes_per_block((long)tx * ty, g.m[2], TZ3, MIN_BLOCKS_SWEEP3);
    const int nb = tx * ty * ((g.m[2] + tz - 1) / tz);
    if (zero) {
        // u is not read: any valid pointer serves the unused loads' base
        if (finest)
            hipLaunchKernelGGL((k_sweep2_3d<T, SRC_ZERO2, TY, 1, TXW, NT>), dim3(nb), dim3(NT), 0, s, b, ec, b, q, out,
                               P, tx, ty, tz, stop);
        else
            hipLaunchKernelGGL((k_sweep2_3d<T, SRC_ZERO2, TY, 0, TXW, NT>), dim3(nb), dim3(NT), 0, s, b, ec, b, q, out,
                               P, tx, ty, tz, stop);
    } else if (ec) {
        if (finest)
            hipLaunchKernelGGL((k_sweep2_3d<T, SRC_PROL, TY, 1, TXW, NT>), dim3(nb), dim3(NT), 0, s, u, ec, b, q, out,
                               P, tx, ty, tz, stop);
        else
            hipLaunchKernelGGL((k_sweep2_3d<T, SRC_PROL, TY, 0, TXW, NT>), dim3(nb), dim3(NT), 0, s, u, ec, b, q, out,
                               P, tx, ty, tz, stop);
    } else {
        if (finest)
            hipLaunchKernelGGL((k_sweep2_3d<T, SRC_MEM, TY, 1, TXW, NT>), dim3(nb), dim3(NT), 0, s, u, ec, b, q, out, P,
                               tx, ty, tz, stop);
        else
            hipLaunchKernelGGL((k_sweep2_3d<T, SRC_MEM, TY, 0, TXW, NT>), dim3(nb), dim3(NT), 0, s, u, ec, b, q, out, P,
                               tx, ty, tz, stop);
    }
}

template <typename T>
void launch_sweep2_3d(const LevelGeom &g, const Stencil<T> &P, const cx<T> *u, const cx<T> *ec, const cx<T> *b,
                      const cx<T> *q, cx<T> *out, hipStream_t s, bool finest, const int *stop, bool zero, int shape)
{
    if (shape == 2)
        launch_sweep2_3d_tile<T, sweep2_rows<T>(2), sweep2_width(2)>(g, P, u, ec, b, q, out, s, finest, stop, zero);
    else if ((shape == 3 || shape == 4) && ec && !zero)
        launch_sweep2_3d_tile<T, sweep2_rows<T>(3), sweep2_width(3)>(g, P, u, ec, b, q, out, s, finest, stop, zero);
    else
        launch_sweep2_3d_tile<T, sweep2_rows<T>(0), sweep2_width(0)>(g, P, u, ec, b, q, out, s, finest, stop, zero);
}
template void launch_sweep2_3d<double>(const LevelGeom &, const Stencil<double> &, const cd *, const cd *, const cd *,
                                       const cd *, cd *, hipStream_t, bool, const int *, bool, int);
template void launch_sweep2_3d<float>(const LevelGeom &, const Stencil<float> &, const cf *, const cf *, const cf *,
                                      const cf *, cf *, hipStream_t, bool, const int *, bool, int);

void launch_refine3d(const LevelGeom &g, const Stencil<double> &P, const cd *u, const cf *d, const cd *b,
                     const cd *q, cd *unew, cf *r32, const SolveCtl *ctl, double *partial, hipStream_t s,
                     const int *stop, const cd *pwf)
{
    int nb, tx, ty, tz;
    grid_of(g, nb, tx, ty, tz);
    if (b)
        hipLaunchKernelGGL((k_refine3d<false>), dim3(nb), dim3(256), 0, s, u, d, b, q, unew, r32, P, tx, ty, tz,
                           partial, ctl, stop, nullptr, PsetArgs());
    else
        hipLaunchKernelGGL((k_refine3d<true>), dim3(nb), dim3(256), 0, s, u, d, nullptr, q, unew, r32, P, tx, ty, tz,
                           partial, ctl, stop, pwf, PsetArgs());
}

__global__ __launch_bounds__(256) void k_resid2d_pw(const cd *__restrict__ u, const cd *__restrict__ q,
                                                    cf *__restrict__ r32, Stencil<double> P, int tiles_x,
                                                    double *__restrict__ partial, const SolveCtl *__restrict__ ctl,
                                                    const cd *__restrict__ pwf)
{
    const double rscale = 1.0 / ctl->scale_next;
    stencil2d_body<double, float, MODE_RESID, true>(u, nullptr, q, r32, P, rscale, tiles_x,
                                                    xcd_tile(blockIdx.x, gridDim.x), partial + blockIdx.x, pwf);
}

void launch_refine3d_start(const LevelGeom &g, const Stencil<double> &P, const cf *ec, const cf *d, const cd *b,
                           const cd *q, cd *unew, cf *r32, const SolveCtl *ctl, double *partial, hipStream_t s,
                           const int *stop, const cd *pwf, const double *bnorm2)
{
    int nb, tx, ty, tz;
    grid_of(g, nb, tx, ty, tz);
    PsetArgs ps;
    ps.ec = ec;
    ps.bnorm2 = bnorm2;
    ps.inv_sqN = 1.0 / sqrt((double)g.N());
    if (b)
        hipLaunchKernelGGL((k_refine3d<false, true>), dim3(nb), dim3(256), 0, s, nullptr, d, b, q, unew, r32, P, tx,
                           ty, tz, partial, ctl, stop, nullptr, ps);
    else
        hipLaunchKernelGGL((k_refine3d<true, true>), dim3(nb), dim3(256), 0, s, nullptr, d, nullptr, q, unew, r32, P,
                           tx, ty, tz, partial, ctl, stop, pwf, ps);
}

void launch_resid_pw(const LevelGeom &g, const Stencil<double> &P, const cd *u, const cd *q, cf *r32,
                     const SolveCtl *ctl, double *partial, const cd *pwf, hipStream_t s)
{
    int nb, tx, ty, tz;
    grid_of(g, nb, tx, ty, tz);
    if (g.dim == 2)
        hipLaunchKernelGGL(k_resid2d_pw, dim3(nb), dim3(256), 0, s, u, q, r32, P, tx, partial, ctl, pwf);
    else
        hipLaunchKernelGGL(k_resid3d_pw, dim3(nb), dim3(256), 0, s, u, q, r32, P, tx, ty, tz, partial, ctl, pwf);
}

template void launch_sweep3d_fused<double>(bool, const LevelGeom &, const Stencil<double> &, const cd *, const cd *,
                                           const cd *, const cd *, cd *, hipStream_t, bool, const int *);
template void launch_sweep3d_fused<float>(bool, const LevelGeom &, const Stencil<float> &, const cf *, const cf *,
                                          const cf *, const cf *, cf *, hipStream_t, bool, const int *);


// Copy / zero with the loop's stop flag.
template <typename T>
__global__ __launch_bounds__(256) void k_copy(const cx<T> *__restrict__ src, cx<T> *__restrict__ dst, size_t N,
                                              const int *__restrict__ stop)
{
    if (stop && *stop) return;
    for (size_t j = (size_t)blockIdx.x * 256 + threadIdx.x; j < N; j += (size_t)gridDim.x * 256)
        dst[j] = src ? src[j] : cx<T>{T(0), T(0)};
}

template <typename T>
void launch_copy(const cx<T> *src, cx<T> *dst, size_t N, hipStream_t s, const int *stop)
{
    size_t nb = std::min<size_t>((N + 255) / 256, 65536);
    hipLaunchKernelGGL((k_copy<T>), dim3((unsigned)nb), dim3(256), 0, s, src, dst, N, stop);
}
template <typename T>
void launch_zero(cx<T> *dst, size_t N, hipStream_t s, const int *stop)
{
    launch_copy<T>(nullptr, dst, N, s, stop);
}
template void launch_copy<double>(const cd *, cd *, size_t, hipStream_t, const int *);
template void launch_copy<float>(const cf *, cf *, size_t, hipStream_t, const int *);
template void launch_zero<double>(cd *, size_t, hipStream_t, const int *);
template void launch_zero<float>(cf *, size_t, hipStream_t, const int *);

// ---------------------------------------------------------------------------
// Full weighting: coarse node I <- fine 2I-1, 2I, 2I+1 with (1/4, 1/2, 1/4),
// tensorised; summed z-outer, x-inner.  One thread per coarse point.
template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_restrict(const cx<T> *__restrict__ rf, cx<T> *__restrict__ bc,
                                                  int mxf, int myf, int mxc, int myc, int mzc,
                                                  const int *__restrict__ stop)
{
    if (stop && *stop) return;
    size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
    size_t Nc = (size_t)mxc * myc * mzc;
    if (idx >= Nc) return;
    int I, J, K;
    split3(idx, mxc, myc, I, J, K);
    const T w[3] = {T(0.25), T(0.5), T(0.25)};
    int fx = 2 * I + 1, fy = 2 * J + 1, fz = 2 * K + 1;
    cx<T> acc = {T(0), T(0)};
    for (int dz = (DIM == 3 ? -1 : 0); dz <= (DIM == 3 ? 1 : 0); ++dz) {
        T wz = (DIM == 3) ? w[dz + 1] : T(1);
        for (int dy = -1; dy <= 1; ++dy) {
            T wy = w[dy + 1];
            for (int dx = -1; dx <= 1; ++dx) {
                T wx = w[dx + 1];
                int z = (DIM == 3) ? fz + dz : 0;
                size_t j = ((size_t)z * myf + (fy + dy)) * mxf + (fx + dx);
                acc = acc + ((wx * wy) * wz) * rf[j];
            }
        }
    }
    bc[idx] = acc;
}

template <typename T>
void launch_restrict(const LevelGeom &f, const cx<T> *rf, cx<T> *bc, hipStream_t s, const int *stop)
{
    int mxc = (f.m[0] - 1) / 2, myc = (f.m[1] - 1) / 2, mzc = (f.dim == 3) ? (f.m[2] - 1) / 2 : 1;
    size_t Nc = (size_t)mxc * myc * mzc;
    int nb = (int)((Nc + 255) / 256);
    if (f.dim == 2)
        hipLaunchKernelGGL((k_restrict<T, 2>), dim3(nb), dim3(256), 0, s, rf, bc, f.m[0], f.m[1], mxc, myc, mzc,
                           stop);
    else
        hipLaunchKernelGGL((k_restrict<T, 3>), dim3(nb), dim3(256), 0, s, rf, bc, f.m[0], f.m[1], mxc, myc, mzc,
                           stop);
}
template void launch_restrict<double>(const LevelGeom &, const cd *, cd *, hipStream_t, const int *);
template void launch_restrict<float>(const LevelGeom &, const cf *, cf *, hipStream_t, const int *);

// Residual + full weighting in 3D, one pass: a block owns a coarse tile of
// RX3 x RY3 points and RZ3 planes and marches up through the fine planes it
// needs (fine 2K .. 2K + 2 for coarse plane K).  u planes (with a one-point
// halo) rotate through a ring of three LDS planes, the fine residual planes
// through a second ring of three; a coarse plane is emitted once its third
// fine plane is done.  The residual and the weighted sum are those of
// k_stencil3d (MODE_RESID) and k_restrict, in the same order, so the result
// is bit for bit that of the two passes.
constexpr int RX3 = 32, RY3 = 4, RZ3 = 24;   // RZ3: coarse planes per block on large grids (measured: 24 beats 16, 20, 28 and 32 at 511^3)
constexpr int RFW = 2 * RX3 + 1, RFH = 2 * RY3 + 1;   // fine residual region of a plane
constexpr int RUW = RFW + 2, RUH = RFH + 2;           // u region (one halo)

template <typename T>
__global__ __launch_bounds__(256) void k_resid_restrict3d(const cx<T> *__restrict__ u, const cx<T> *__restrict__ b,
                                                          const cx<T> *__restrict__ q, cx<T> *__restrict__ bc,
                                                          Stencil<T> P, int tiles_x, int tiles_y, int rz,
                                                          const int *__restrict__ stop)
{
    if (stop && *stop) return;
    __shared__ cx<T> us[3][RUH][RUW];
    __shared__ cx<T> rs[3][RFH][RFW];
    const int mx = P.mx, my = P.my, mz = P.mz;
    const int mxc = (mx - 1) / 2, myc = (my - 1) / 2, mzc = (mz - 1) / 2;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int txi = tile % tiles_x, rest = tile / tiles_x;
    const int tyi = rest % tiles_y, tzi = rest / tiles_y;
    const int I0 = txi * RX3, J0 = tyi * RY3, K0 = tzi * rz;
    const int K1 = min(K0 + rz, mzc);
    const int fx0 = 2 * I0, fy0 = 2 * J0;                 // fine origin of the residual region
    const size_t plane = (size_t)mx * my;
    const T w[3] = {T(0.25), T(0.5), T(0.25)};

    // Loads run one plane ahead through registers: while residual plane fz is
    // formed, u of plane fz + 2 and b, q of plane fz + 1 are in flight (buffer
    // loads, zero outside the grid; the barriers fence LDS only, so the loads
    // stay in flight across them).
    constexpr int NUL = (RUH * RUW + 255) / 256, NRL = (RFH * RFW + 255) / 256;
    cx<T> un[NUL], bn[NRL], qn[NRL];
    unsigned offu[NUL], offr[NRL];
    const unsigned pbytes = (unsigned)(plane * sizeof(cx<T>));
#pragma unroll
    for (int k = 0; k < NUL; ++k) {
        const int t = threadIdx.x + 256 * k;
        const int yy = t / RUW, xx = t - yy * RUW;
        const int gx = fx0 - 1 + xx, gy = fy0 - 1 + yy;
        const bool in = t < RUH * RUW && gx >= 0 && gx < mx && gy >= 0 && gy < my;
        offu[k] = in ? (unsigned)(gy * mx + gx) * (unsigned)sizeof(cx<T>) : BUF_OOB;
    }
#pragma unroll
    for (int k = 0; k < NRL; ++k) {
        const int t = threadIdx.x + 256 * k;
        const int yy = t / RFW, xx = t - yy * RFW;
        const int gx = fx0 + xx, gy = fy0 + yy;
        const bool in = t < RFH * RFW && gx < mx && gy < my;
        offr[k] = in ? (unsigned)(gy * mx + gx) * (unsigned)sizeof(cx<T>) : BUF_OOB;
    }
    auto issue_u = [&](int fz) {
        const bool zin = fz >= 0 && fz < mz;
        const auto ru = buf_rsrc(u + (zin ? (size_t)fz * plane : 0), zin ? pbytes : 0u);
#pragma unroll
        for (int k = 0; k < NUL; ++k) un[k] = ld_buf<T>(ru, offu[k]);
    };
    auto store_u = [&](int fz) {
        cx<T> *dst = &us[(fz + 3) % 3][0][0];
#pragma unroll
        for (int k = 0; k < NUL; ++k) {
            const int t = threadIdx.x + 256 * k;
            if (t < RUH * RUW) dst[t] = un[k];
        }
    };
    auto issue_bq = [&](int fz) {
        const bool zin = fz >= 0 && fz < mz;
        const size_t o = zin ? (size_t)fz * plane : 0;
        const auto rb = buf_rsrc(b + o, zin ? pbytes : 0u), rq = buf_rsrc(q + o, zin ? pbytes : 0u);
#pragma unroll
        for (int k = 0; k < NRL; ++k) {
            bn[k] = ld_buf<T>(rb, offr[k]);
            qn[k] = ld_buf<T>(rq, offr[k]);
        }
    };
    const int fz_first = 2 * K0, fz_last = 2 * K1;        // fine residual planes of the block
    issue_u(fz_first - 1);
    store_u(fz_first - 1);
    issue_u(fz_first);
    store_u(fz_first);
    issue_u(fz_first + 1);
    issue_bq(fz_first);
    for (int fz = fz_first; fz <= fz_last; ++fz) {
        store_u(fz + 1);
        cx<T> bc_[NRL], qc_[NRL];
#pragma unroll
        for (int k = 0; k < NRL; ++k) {
            bc_[k] = bn[k];
            qc_[k] = qn[k];
        }
        lds_barrier();
        if (fz < fz_last) {
            issue_u(fz + 2);
            issue_bq(fz + 1);
        }
        // fine residual plane fz on the RFW x RFH region (0 outside the grid)
        const cx<T>(&um)[RUH][RUW] = us[(fz + 2) % 3];
        const cx<T>(&uc_)[RUH][RUW] = us[fz % 3];
        const cx<T>(&up)[RUH][RUW] = us[(fz + 1) % 3];
        cx<T> *rd = &rs[fz % 3][0][0];
#pragma unroll
        for (int k = 0; k < NRL; ++k) {
            const int t = threadIdx.x + 256 * k;
            if (t < RFH * RFW) {
                const int yy = t / RFW, xx = t - yy * RFW;
                const int gx = fx0 + xx, gy = fy0 + yy;
                cx<T> r = {T(0), T(0)};
                if (gx < mx && gy < my && fz < mz) {
                    const cx<T> uc = uc_[yy + 1][xx + 1];
                    cx<T> lap = lap_xy(P, uc, uc_[yy + 1][xx], uc_[yy + 1][xx + 2], uc_[yy][xx + 1],
                                       uc_[yy + 2][xx + 1]);
                    lap = lap_add_z(P, lap, uc, um[yy + 1][xx + 1], up[yy + 1][xx + 1]);
                    r = resid_from(P, lap, uc, bc_[k], qc_[k]);
                }
                rd[t] = r;
            }
        }
        lds_barrier();
        // coarse plane K = (fz - 2) / 2 once fine planes 2K .. 2K + 2 are done
        if (fz >= fz_first + 2 && ((fz - fz_first) & 1) == 0) {
            const int K = (fz - 2) / 2;
            for (int t = threadIdx.x; t < RX3 * RY3; t += 256) {
                const int cy = t / RX3, cxx = t - cy * RX3;
                const int I = I0 + cxx, J = J0 + cy;
                if (I < mxc && J < myc) {
                    cx<T> acc = {T(0), T(0)};
                    for (int dz = -1; dz <= 1; ++dz) {
                        const cx<T>(&rz)[RFH][RFW] = rs[(2 * K + 1 + dz) % 3];
                        for (int dy = -1; dy <= 1; ++dy)
                            for (int dx = -1; dx <= 1; ++dx)
                                acc = acc + ((w[dx + 1] * w[dy + 1]) * w[dz + 1]) *
                                                rz[2 * cy + 1 + dy][2 * cxx + 1 + dx];
                    }
                    bc[((size_t)K * myc + J) * mxc + I] = acc;
                }
            }
        }
    }
}

// Pre-smoothing + residual + full weighting in one z-marching pass (the 3D
// form of k_smooth_rr2d): two weighted-Jacobi sweeps from u (or from a zero
// guess), written to out on the block's tile, then the residual of the
// smoothed iterate and its full weighting into the coarse right-hand side.
// A block owns a fine tile of TXW x TY points (x0 and y0 even) and tz fine
// planes (tz even), and so the coarse tile of TXW/2 x TY/2 points and tz/2
// planes whose full weighting reads the fine residual on [x0, x0 + TXW] x
// [y0, y0 + TY] (one point beyond the tile on the high sides).  Five stages
// march up through the planes, each a plane behind the one before:
//   stage 0  the input at plane z (u; nothing from a zero guess),
//   stage 1  the first sweep at z - 1 (region: the residual's plus 2),
//   stage 2  the second sweep at z - 2 (plus 1), written out on the tile,
//   stage 3  the residual at z - 3 (the residual region) into an LDS plane,
//   stage 4  the residual plane z - 4 weighted into the coarse plane it
//            belongs to: one running sum per coarse point, the planes 2K,
//            2K + 1, 2K + 2 in turn, written when 2K + 2 is added.
// Every stage's current plane goes through LDS (two buffers by parity, one
// barrier per plane); each thread keeps its columns' last three planes of
// stages 0-2 and the b, q of the planes stages 1-3 take in registers.  The
// sweeps are those of k_sweep2_3d and the residual and the weighted sum
// (terms and order) those of k_resid_restrict3d, so out and bc are bit for
// bit those of the two passes.
// TAG: 1 for the finest level (a symbol of its own in profiles), else 0.
template <typename T, bool ZERO, int TY, int TXW, int TAG, int NT>
__global__ __launch_bounds__(NT) void k_sweep2rr_3d(const cx<T> *__restrict__ u, const cx<T> *__restrict__ b,
                                                     const cx<T> *__restrict__ q, cx<T> *__restrict__ out,
                                                     cx<T> *__restrict__ bc, Stencil<T> P, int tiles_x, int tiles_y,
                                                     int tz, const int *__restrict__ stop)
{
    if (stop && *stop) return;
    constexpr int W = TXW + 7, H = TY + 7, NP = W * H, NS = (NP + NT - 1) / NT;
    constexpr int RW = TXW + 1, RH = TY + 1;          // the fine residual region
    constexpr int CXN = TXW / 2, CYN = TY / 2;        // the coarse tile
    static_assert(CXN * CYN <= NT, "one coarse point per thread");
    __shared__ cx<T> L0[ZERO ? 1 : 2][ZERO ? 1 : NP], L1[2][NP], L2[2][NP];
    __shared__ cx<T> R[2][RH * RW];
    const int mx = P.mx, my = P.my, mz = P.mz;
    const int mxc = (mx - 1) / 2, myc = (my - 1) / 2, mzc = (mz - 1) / 2;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int txi = tile % tiles_x, rest = tile / tiles_x;
    const int tyi = rest % tiles_y, tzi = rest / tiles_y;
    const int x0 = txi * TXW, y0 = tyi * TY, z0 = tzi * tz, z1 = min(z0 + tz, mz);
    const size_t plane = (size_t)mx * my;
    const cx<T> zero = {T(0), T(0)};
    const T w3[3] = {T(0.25), T(0.5), T(0.25)};

    // slot k: region row r, column c, grid point (x0 - 3 + c, y0 - 3 + r)
    int ofs[NS];
    unsigned offu[NS], offbq[NS];
    unsigned ing = 0, st1 = 0, st2 = 0, st3 = 0, own = 0;
    int rofs[NS];   // index of the slot in the residual plane (stage 3)
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        const int t = threadIdx.x + NT * k;
        const int r = t / W, c = t - r * W;
        const int gx = x0 - 3 + c, gy = y0 - 3 + r;
        const bool v = t < NP;
        const bool in = v && gx >= 0 && gx < mx && gy >= 0 && gy < my;
        const bool s1 = v && r >= 1 && r < H - 1 && c >= 1 && c < W - 1;
        ofs[k] = in ? gy * mx + gx : 0;
        offu[k] = in ? (unsigned)ofs[k] * (unsigned)sizeof(cx<T>) : BUF_OOB;
        offbq[k] = (in && s1) ? offu[k] : BUF_OOB;
        ing |= (unsigned)in << k;
        st1 |= (unsigned)s1 << k;
        st2 |= (unsigned)(v && r >= 2 && r < H - 2 && c >= 2 && c < W - 2) << k;
        st3 |= (unsigned)(v && r >= 3 && r < H - 3 && c >= 3 && c < W - 3) << k;
        own |= (unsigned)(in && r >= 3 && r < 3 + TY && c >= 3 && c < 3 + TXW) << k;
        rofs[k] = (r - 3) * RW + (c - 3);
    }
    auto slot_in = [&](unsigned m, int k) { return ((m >> k) & 1u) != 0u; };
    const unsigned pbytes = (unsigned)(plane * sizeof(cx<T>));

    cx<T> pu[NS], pb[NS], pq[NS];
    auto fetch_u = [&](int z) {
        const bool zin = z >= 0 && z < mz;
        const auto ru = buf_rsrc(u + (zin ? (size_t)z * plane : 0), zin ? pbytes : 0u);
#pragma unroll
        for (int k = 0; k < NS; ++k) pu[k] = ld_buf<T>(ru, offu[k]);
    };
    auto fetch_bq = [&](int z) {
        const bool zin = z >= 0 && z < mz;
        const size_t o = zin ? (size_t)z * plane : 0;
        const auto rb = buf_rsrc(b + o, zin ? pbytes : 0u), rq = buf_rsrc(q + o, zin ? pbytes : 0u);
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            pb[k] = ld_buf<T>(rb, offbq[k]);
            pq[k] = ld_buf<T>(rq, offbq[k]);
        }
    };

    // the coarse point of this thread (stage 4) and its running sum
    const int cyy = (int)threadIdx.x / CXN, cxx = (int)threadIdx.x - cyy * CXN;
    const int ci = x0 / 2 + cxx, cj = y0 / 2 + cyy;
    const bool cown = (int)threadIdx.x < CXN * CYN && ci < mxc && cj < myc;
    cx<T> cacc = zero;

    const int zb = z0 - 3, ze = z0 + tz + 4;   // input planes of the march (stage 4 ends at z0 + tz)
#pragma unroll
    for (int k = 0; k < NS; ++k) pu[k] = pb[k] = pq[k] = zero;
    if (!ZERO) fetch_u(zb);

    cx<T> a0[NS], a1[NS], a2[NS];   // stage 0 at planes z - 2, z - 1, z
    cx<T> c0[NS], c1[NS], c2[NS];   // stage 1 at planes z - 3, z - 2, z - 1
    cx<T> e0[NS], e1[NS], e2[NS];   // stage 2 at planes z - 4, z - 3, z - 2
    cx<T> bB[NS], qB[NS];           // b, q at plane z - 2 (stage 2)
    cx<T> b3[NS], q3[NS];           // b, q at plane z - 3 (stage 3)
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        a0[k] = a1[k] = a2[k] = zero;
        c0[k] = c1[k] = c2[k] = zero;
        e0[k] = e1[k] = e2[k] = zero;
        bB[k] = qB[k] = b3[k] = q3[k] = zero;
    }
    for (int z = zb; z <= ze; ++z) {
        cx<T> un[NS], bn[NS], qn[NS];
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            un[k] = pu[k];
            bn[k] = pb[k];
            qn[k] = pq[k];
        }
        if (!ZERO && z + 1 <= z0 + tz + 3) fetch_u(z + 1);
        if (z >= z0 - 2 && z <= z0 + tz + 2) fetch_bq(z);   // b, q of plane z: stage 1 of the next iteration
        // stage 0: the input at plane z
        if (!ZERO) {
            cx<T> *l0w = L0[z & 1];
#pragma unroll
            for (int k = 0; k < NS; ++k) {
                const int t = threadIdx.x + NT * k;
                a0[k] = a1[k];
                a1[k] = a2[k];
                a2[k] = un[k];
                if (t < NP) l0w[t] = un[k];
            }
        }
        // stage 1: the first sweep at plane p1 = z - 1
        const int p1 = z - 1;
        if (p1 >= z0 - 2 && p1 <= z0 + tz + 2) {
            const cx<T> *l0r = L0[ZERO ? 0 : (p1 & 1)];
            cx<T> *l1w = L1[p1 & 1];
            const bool pin = p1 >= 0 && p1 < mz;
#pragma unroll
            for (int k = 0; k < NS; ++k) {
                const int t = threadIdx.x + NT * k;
                c0[k] = c1[k];
                c1[k] = c2[k];
                cx<T> v = zero;
                if (pin && slot_in(ing & st1, k)) {
                    const cx<T> wj = jweight(P, qn[k]);
                    if (ZERO) {
                        v = jacobi0_w(bn[k], wj);
                    } else {
                        cx<T> N = nsum_xy(P, l0r[t - 1], l0r[t + 1], l0r[t - W], l0r[t + W]);
                        N = nsum_add_z(P, N, a0[k], a2[k]);
                        v = jacobi_n(P, N, a1[k], bn[k], wj);
                    }
                }
                c2[k] = v;
                if (slot_in(st1, k)) l1w[t] = v;
            }
        }
        // stage 2: the second sweep at plane p2 = z - 2, written out on the tile
        const int p2 = z - 2;
        if (p2 >= z0 - 1 && p2 <= z0 + tz + 1) {
            const cx<T> *l1r = L1[p2 & 1];
            cx<T> *l2w = L2[p2 & 1];
            const bool pin = p2 >= 0 && p2 < mz;
            const bool wr = p2 >= z0 && p2 < z1;
#pragma unroll
            for (int k = 0; k < NS; ++k) {
                const int t = threadIdx.x + NT * k;
                e0[k] = e1[k];
                e1[k] = e2[k];
                cx<T> v = zero;
                if (pin && slot_in(ing & st2, k)) {
                    cx<T> N = nsum_xy(P, l1r[t - 1], l1r[t + 1], l1r[t - W], l1r[t + W]);
                    N = nsum_add_z(P, N, c0[k], c2[k]);
                    v = jacobi_n(P, N, c1[k], bB[k], jweight(P, qB[k]));
                    if (wr && slot_in(own, k)) out[(size_t)p2 * plane + ofs[k]] = v;
                }
                e2[k] = v;
                if (slot_in(st2, k)) l2w[t] = v;
            }
        }
        // stage 3: the residual at plane p3 = z - 3 (zero outside the grid)
        const int p3 = z - 3;
        if (p3 >= z0 && p3 <= z0 + tz) {
            const cx<T> *l2r = L2[p3 & 1];
            cx<T> *rw = R[p3 & 1];
            const bool pin = p3 < mz;
#pragma unroll
            for (int k = 0; k < NS; ++k) {
                const int t = threadIdx.x + NT * k;
                if (slot_in(st3, k)) {
                    cx<T> r = zero;
                    if (pin && slot_in(ing, k)) {
                        const cx<T> uc = e1[k];
                        cx<T> lap = lap_xy(P, uc, l2r[t - 1], l2r[t + 1], l2r[t - W], l2r[t + W]);
                        lap = lap_add_z(P, lap, uc, e0[k], e2[k]);
                        r = resid_from(P, lap, uc, b3[k], q3[k]);
                    }
                    rw[rofs[k]] = r;
                }
            }
        }
        // stage 4: residual plane p4 = z - 4 into the running coarse sums:
        // plane 2K + 2 ends coarse plane K, 2K starts it, 2K + 1 is its middle
        const int p4 = z - 4;
        if (p4 >= z0 && p4 <= z0 + tz && cown) {
            const cx<T> *rr = R[p4 & 1];
            const int odd = p4 & 1;
            if (!odd && p4 > z0) {   // dz = +1 of K = p4 / 2 - 1, then K is complete
#pragma unroll
                for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
                    for (int dx = -1; dx <= 1; ++dx)
                        cacc = cacc + ((w3[dx + 1] * w3[dy + 1]) * w3[2]) * rr[(2 * cyy + 1 + dy) * RW + 2 * cxx + 1 + dx];
                const int K = p4 / 2 - 1;
                if (K < mzc) bc[((size_t)K * myc + cj) * mxc + ci] = cacc;
            }
            if (!odd && p4 < z0 + tz) {   // dz = -1 of K = p4 / 2: a new sum
                cacc = zero;
#pragma unroll
                for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
                    for (int dx = -1; dx <= 1; ++dx)
                        cacc = cacc + ((w3[dx + 1] * w3[dy + 1]) * w3[0]) * rr[(2 * cyy + 1 + dy) * RW + 2 * cxx + 1 + dx];
            }
            if (odd) {   // dz = 0
#pragma unroll
                for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
                    for (int dx = -1; dx <= 1; ++dx)
                        cacc = cacc + ((w3[dx + 1] * w3[dy + 1]) * w3[1]) * rr[(2 * cyy + 1 + dy) * RW + 2 * cxx + 1 + dx];
            }
        }
        // b, q move one stage on: plane z - 1 serves stage 2, z - 2 stage 3 next iteration
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            b3[k] = bB[k];
            q3[k] = qB[k];
            bB[k] = bn[k];
            qB[k] = qn[k];
        }
        lds_barrier();
    }
}

// Tile and block size of the fused pre-smoothing + residual + restriction pass.
constexpr int SRR3_TXW = 32, SRR3_TY = 16, SRR3_NT = 512;   // measured at 511^3 (solve): 24.24 ms against 24.68 with 32 x 8 tiles of 256 threads, 24.64 with 1024 threads; 32 x 24 and 48 x 8 slower
constexpr int SRR3_TZ = 64;   // planes per block on large grids (the pass runs 7 planes ahead of its output): 23.6 ms against 24.2 with 32

bool sweep2rr_3d_fits(const LevelGeom &g) { return g.dim == 3 && g.m[0] >= 3 && g.m[1] >= 3 && g.m[2] >= 3; }

template <typename T>
void launch_sweep2rr_3d(const LevelGeom &g, const Stencil<T> &P, const cx<T> *u, const cx<T> *b, const cx<T> *q,
                        cx<T> *out, cx<T> *bc, hipStream_t s, bool finest, const int *stop)
{
    constexpr int TX = SRR3_TXW, TY = SRR3_TY, NT = SRR3_NT;
    const int tx = (g.m[0] + TX - 1) / TX, ty = (g.m[1] + TY - 1) / TY;
    int tz = planes_per_block((long)tx * ty, g.m[2], SRR3_TZ, MIN_BLOCKS_SRR3);
    tz = std::max(2, tz & ~1);   // even: the coarse planes of a block are whole
    const int nb = tx * ty * ((g.m[2] + tz - 1) / tz);
    if (!u && finest)
        hipLaunchKernelGGL((k_sweep2rr_3d<T, true, TY, TX, 1, NT>), dim3(nb), dim3(NT), 0, s, b, b, q, out, bc, P, tx,
                           ty, tz, stop);
    else if (!u)
        hipLaunchKernelGGL((k_sweep2rr_3d<T, true, TY, TX, 0, NT>), dim3(nb), dim3(NT), 0, s, b, b, q, out, bc, P, tx,
                           ty, tz, stop);
    else if (finest)
        hipLaunchKernelGGL((k_sweep2rr_3d<T, false, TY, TX, 1, NT>), dim3(nb), dim3(NT), 0, s, u, b, q, out, bc, P,
                           tx, ty, tz, stop);
    else
        hipLaunchKernelGGL((k_sweep2rr_3d<T, false, TY, TX, 0, NT>), dim3(nb), dim3(NT), 0, s, u, b, q, out, bc, P,
                           tx, ty, tz, stop);
}
template void launch_sweep2rr_3d<float>(const LevelGeom &, const Stencil<float> &, const cf *, const cf *, const cf *,
                                        cf *, cf *, hipStream_t, bool, const int *);

template <typename T>
void launch_resid_restrict3d(const LevelGeom &f, const Stencil<T> &P, const cx<T> *u, const cx<T> *b, const cx<T> *q,
                             cx<T> *bc, hipStream_t s, const int *stop)
{
    const int mxc = (f.m[0] - 1) / 2, myc = (f.m[1] - 1) / 2, mzc = (f.m[2] - 1) / 2;
    const int tx = (mxc + RX3 - 1) / RX3, ty = (myc + RY3 - 1) / RY3;
    const int rz = planes_per_block((long)tx * ty, mzc, RZ3), tz = (mzc + rz - 1) / rz;
    hipLaunchKernelGGL(k_resid_restrict3d<T>, dim3(tx * ty * tz), dim3(256), 0, s, u, b, q, bc, P, tx, ty, rz, stop);
}
template void launch_resid_restrict3d<double>(const LevelGeom &, const Stencil<double> &, const cd *, const cd *,
                                              const cd *, cd *, hipStream_t, const int *);
template void launch_resid_restrict3d<float>(const LevelGeom &, const Stencil<float> &, const cf *, const cf *,
                                             const cf *, cf *, hipStream_t, const int *);

template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_prolong_add(const cx<T> *__restrict__ ec, cx<T> *__restrict__ uf,
                                                     int mxf, int myf, int mzf, int mxc, int myc, int mzc,
                                                     const int *__restrict__ stop)
{
    if (stop && *stop) return;
    size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
    size_t Nf = (size_t)mxf * myf * mzf;
    if (idx >= Nf) return;
    int ix, iy, iz;
    split3(idx, mxf, myf, ix, iy, iz);
    uf[idx] = uf[idx] + prolong_at<T, DIM>(ec, ix, iy, iz, mxc, myc, mzc);
}

template <typename T>
void launch_prolong_add(const LevelGeom &f, const cx<T> *ec, cx<T> *uf, hipStream_t s, const int *stop)
{
    int mxc = (f.m[0] - 1) / 2, myc = (f.m[1] - 1) / 2, mzc = (f.dim == 3) ? (f.m[2] - 1) / 2 : 1;
    size_t Nf = f.N();
    int nb = (int)((Nf + 255) / 256);
    if (f.dim == 2)
        hipLaunchKernelGGL((k_prolong_add<T, 2>), dim3(nb), dim3(256), 0, s, ec, uf, f.m[0], f.m[1], 1, mxc, myc, 1,
                           stop);
    else
        hipLaunchKernelGGL((k_prolong_add<T, 3>), dim3(nb), dim3(256), 0, s, ec, uf, f.m[0], f.m[1], f.m[2], mxc,
                           myc, mzc, stop);
}
template void launch_prolong_add<double>(const LevelGeom &, const cd *, cd *, hipStream_t, const int *);
template void launch_prolong_add<float>(const LevelGeom &, const cf *, cf *, hipStream_t, const int *);

// ---------------------------------------------------------------------------
// Deterministic sum of per-block partials (one block, fixed order).
__device__ __forceinline__ double sum_parts_256(const double *__restrict__ parts, int n)
{
    __shared__ double red[4];
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) acc += parts[i];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) red[w] = acc;
    __syncthreads();
    return (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ __launch_bounds__(256) void k_sum(const double *__restrict__ parts, int n, double *__restrict__ out)
{
    double s = sum_parts_256(parts, n);
    if (threadIdx.x == 0) out[0] = s;
}

// Solve control.  Init: from ||b||^2.  Update (after each cycle's residual
// norm, and once for the initial residual with k = 0): the stopping test
// ||r_k|| <= tol ||b|| (Sec. 4), the growth test (3 consecutive increases),
// the cycle limit, and the scales of the next FP32 right-hand side.
__device__ __forceinline__ void ctl_init_store(SolveCtl *ctl, double b2, double tol, double inv_sqN, int max_cycles)
{
    SolveCtl c;
    c.tol2b2 = tol * tol * b2;
    c.inv_sqN = inv_sqN;
    c.r0_2 = c.rk2 = c.prev2 = 0.0;
    c.scale_cur = sqrt(b2) * inv_sqN;
    c.scale_next = c.scale_cur;
    c.done = 0;
    c.k = -1;          // the first update is the initial residual
    c.grow = 0;
    c.max_cycles = max_cycles;
    c.b2 = b2;
    *ctl = c;
}

__global__ void k_ctl_init(SolveCtl *ctl, const double *__restrict__ bnorm2, double tol, double inv_sqN,
                           int max_cycles)
{
    if (threadIdx.x != 0) return;
    const double b2 = bnorm2[0];
    ctl_init_store(ctl, b2, tol, inv_sqN, max_cycles);
    // b = 0 (solution 0) or a non-finite b: every later kernel of the solve
    // sees the stop flag and does nothing; the host decides from b2
    if (!(b2 > 0.0) || !isfinite(b2)) ctl->done = 5;
}

// One update from the n per-block partial sums of |r_k|^2 (256 threads).
__device__ __forceinline__ void ctl_update_body(SolveCtl *ctl, const double *__restrict__ parts, int n)
{
    if (ctl->done) return;
    double s2 = sum_parts_256(parts, n);
    if (threadIdx.x != 0) return;
    SolveCtl c = *ctl;
    c.k += 1;
    c.rk2 = s2;
    c.scale_cur = c.scale_next;
    c.scale_next = sqrt(s2) * c.inv_sqN;
    if (c.k == 0) {
        c.r0_2 = s2;
    } else {
        c.grow = (s2 >= c.prev2) ? c.grow + 1 : 0;
    }
    if (!isfinite(s2)) c.done = 4;
    else if (s2 <= c.tol2b2) c.done = 1;
    else if (c.grow >= 3) c.done = 2;
    else if (c.k >= c.max_cycles) c.done = 3;
    c.prev2 = s2;
    *ctl = c;
}

__global__ __launch_bounds__(256) void k_ctl_update(SolveCtl *ctl, const double *__restrict__ parts, int n)
{
    ctl_update_body(ctl, parts, n);
}

void launch_ctl_init(SolveCtl *ctl, const double *bnorm2, double tol, size_t N, int max_cycles, hipStream_t s)
{
    hipLaunchKernelGGL(k_ctl_init, dim3(1), dim3(64), 0, s, ctl, bnorm2, tol, 1.0 / sqrt((double)N), max_cycles);
}

void launch_ctl_update(SolveCtl *ctl, const double *parts, int nparts, hipStream_t s)
{
    hipLaunchKernelGGL(k_ctl_update, dim3(1), dim3(256), 0, s, ctl, parts, nparts);
}

void launch_sum(const double *parts, int nparts, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, s, parts, nparts, out);
}

// ---------------------------------------------------------------------------
// Setup: contrast q = scale * coef (Helmholtz scale 1; Schroedinger -2, i.e.
// q = -2V) and a count of non-finite inputs per block.
__global__ __launch_bounds__(256) void k_make_q(const cd *__restrict__ coef, cd *__restrict__ q, size_t N,
                                                double scale, double *__restrict__ bad)
{
    double nbad = 0.0;
    for (size_t j = (size_t)blockIdx.x * 256 + threadIdx.x; j < N; j += (size_t)gridDim.x * 256) {
        cd c = coef[j];
        if (!isfinite(c.re) || !isfinite(c.im)) nbad += 1.0;
        q[j] = cd{scale * c.re, scale * c.im};
    }
    block_sum_256(nbad, bad + blockIdx.x);
}

void launch_make_q(const cd *coef, cd *q, size_t N, double scale, double *bad_parts, int nparts, hipStream_t s)
{
    hipLaunchKernelGGL(k_make_q, dim3(nparts), dim3(256), 0, s, coef, q, N, scale, bad_parts);
}

// Coarse coefficients by injection: coarse node I <- fine node 2I.
template <typename T>
__global__ __launch_bounds__(256) void k_inject(const cx<T> *__restrict__ qf, cx<T> *__restrict__ qc, int mxf,
                                                int myf, int mxc, int myc, int mzc, int dim)
{
    size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
    size_t Nc = (size_t)mxc * myc * mzc;
    if (idx >= Nc) return;
    int I, J, K;
    split3(idx, mxc, myc, I, J, K);
    int z = (dim == 3) ? 2 * K + 1 : 0;
    qc[idx] = qf[((size_t)z * myf + (2 * J + 1)) * mxf + (2 * I + 1)];
}

template <typename T>
void launch_inject(const LevelGeom &f, const cx<T> *qf, cx<T> *qc, hipStream_t s)
{
    int mxc = (f.m[0] - 1) / 2, myc = (f.m[1] - 1) / 2, mzc = (f.dim == 3) ? (f.m[2] - 1) / 2 : 1;
    size_t Nc = (size_t)mxc * myc * mzc;
    hipLaunchKernelGGL((k_inject<T>), dim3((Nc + 255) / 256), dim3(256), 0, s, qf, qc, f.m[0], f.m[1], mxc, myc,
                       mzc, f.dim);
}
template void launch_inject<double>(const LevelGeom &, const cd *, cd *, hipStream_t);
template void launch_inject<float>(const LevelGeom &, const cf *, cf *, hipStream_t);


// b_1 = b_0 / s at the coarse nodes (injection of the finest right-hand side).
// (bf = null: b is the plane-wave right-hand side q u_in, formed from q and
// the factors pwf at the injected points.)
template <typename TO>
__global__ __launch_bounds__(256) void k_inject_rhs(const cd *__restrict__ bf, cx<TO> *__restrict__ bc, int mxf,
                                                    int myf, int mxc, int myc, int mzc, int dim,
                                                    const double *__restrict__ bnorm2, double inv_sqN,
                                                    const cd *__restrict__ qf, const cd *__restrict__ pwf)
{
    size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
    size_t Nc = (size_t)mxc * myc * mzc;
    if (idx >= Nc) return;
    const double inv = 1.0 / fmg_scale(bnorm2, inv_sqN);
    int I, J, K;
    split3(idx, mxc, myc, I, J, K);
    int z = (dim == 3) ? 2 * K + 1 : 0;
    const size_t j = ((size_t)z * myf + (2 * J + 1)) * mxf + (2 * I + 1);
    cd v = bf ? bf[j] : qf[j] * pw_uin(pwf, 2 * I + 1, 2 * J + 1, z, mxf, myf, dim);
    bc[idx] = cvt<TO>(cd{v.re * inv, v.im * inv});
}

template <typename TO>
void launch_inject_rhs(const LevelGeom &f, const cd *bf, cx<TO> *bc, const double *bnorm2, hipStream_t s,
                       const cd *qf, const cd *pwf)
{
    int mxc = (f.m[0] - 1) / 2, myc = (f.m[1] - 1) / 2, mzc = (f.dim == 3) ? (f.m[2] - 1) / 2 : 1;
    size_t Nc = (size_t)mxc * myc * mzc;
    hipLaunchKernelGGL((k_inject_rhs<TO>), dim3((unsigned)((Nc + 255) / 256)), dim3(256), 0, s, bf, bc, f.m[0],
                       f.m[1], mxc, myc, mzc, f.dim, bnorm2, 1.0 / sqrt((double)f.N()), qf, pwf);
}
template void launch_inject_rhs<double>(const LevelGeom &, const cd *, cd *, const double *, hipStream_t, const cd *,
                                        const cd *);
template void launch_inject_rhs<float>(const LevelGeom &, const cd *, cf *, const double *, hipStream_t, const cd *,
                                       const cd *);

// uf = s P ec: the interpolated coarse solution overwrites uf (the initial
// guess of the next finer level).
template <typename TC, typename TF, int DIM>
__global__ __launch_bounds__(256) void k_prolong_set(const cx<TC> *__restrict__ ec, cx<TF> *__restrict__ uf, int mxf,
                                                     int myf, int mzf, int mxc, int myc, int mzc,
                                                     const double *__restrict__ bnorm2, double inv_sqN)
{
    size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
    size_t Nf = (size_t)mxf * myf * mzf;
    if (idx >= Nf) return;
    int ix, iy, iz;
    split3(idx, mxf, myf, ix, iy, iz);
    cx<TC> v = prolong_at<TC, DIM>(ec, ix, iy, iz, mxc, myc, mzc);
    if (bnorm2) {
        const double sc = fmg_scale(bnorm2, inv_sqN);
        uf[idx] = cvt<TF>(cd{(double)v.re * sc, (double)v.im * sc});
    } else {
        uf[idx] = cvt<TF>(v);
    }
}

template <typename TC, typename TF>
void launch_prolong_set(const LevelGeom &f, const cx<TC> *ec, cx<TF> *uf, const double *bnorm2, double inv_sqN,
                        hipStream_t s)
{
    int mxc = (f.m[0] - 1) / 2, myc = (f.m[1] - 1) / 2, mzc = (f.dim == 3) ? (f.m[2] - 1) / 2 : 1;
    size_t Nf = f.N();
    unsigned nb = (unsigned)((Nf + 255) / 256);
    if (f.dim == 2)
        hipLaunchKernelGGL((k_prolong_set<TC, TF, 2>), dim3(nb), dim3(256), 0, s, ec, uf, f.m[0], f.m[1], 1, mxc, myc,
                           1, bnorm2, inv_sqN);
    else
        hipLaunchKernelGGL((k_prolong_set<TC, TF, 3>), dim3(nb), dim3(256), 0, s, ec, uf, f.m[0], f.m[1], f.m[2],
                           mxc, myc, mzc, bnorm2, inv_sqN);
}
template void launch_prolong_set<double, double>(const LevelGeom &, const cd *, cd *, const double *, double,
                                                 hipStream_t);
template void launch_prolong_set<float, float>(const LevelGeom &, const cf *, cf *, const double *, double,
                                               hipStream_t);
template void launch_prolong_set<float, double>(const LevelGeom &, const cf *, cd *, const double *, double,
                                                hipStream_t);

// The last step of the FP32 full multigrid start fused with the initial
// residual of the refinement (3D): u = s P e_c written (u = null: not
// stored), and r32 = (b - A u) / ctl->scale_next with the block sums of
// |b - A u|^2, the bits of k_prolong_set<float, double, 3> followed by the
// FP64 residual pass.
template <bool PW>
__global__ __launch_bounds__(256) void k_fmg_resid3d(const cf *__restrict__ ec, const cd *__restrict__ b,
                                                     const cd *__restrict__ q, cd *__restrict__ u,
                                                     cf *__restrict__ r32, Stencil<double> P, int tiles_x,
                                                     int tiles_y, int tz, double *__restrict__ partial,
                                                     const SolveCtl *__restrict__ ctl,
                                                     const double *__restrict__ bnorm2, double inv_sqN,
                                                     const cd *__restrict__ pwf)
{
    const double rscale = 1.0 / ctl->scale_next;
    PsetArgs ps;
    ps.ec = ec;
    ps.bnorm2 = bnorm2;
    ps.inv_sqN = inv_sqN;
    stencil3d_body<double, float, MODE_RESID, SRC_PSET, PW>(nullptr, nullptr, b, q, r32, P, rscale, tiles_x, tiles_y,
                                                            tz, partial, nullptr, 0.0, u, pwf, ps);
}

void launch_fmg_resid3d(const LevelGeom &g, const Stencil<double> &P, const cf *ec, const cd *b, const cd *q, cd *u,
                        cf *r32, const SolveCtl *ctl, double *partial, const double *bnorm2, const cd *pwf,
                        hipStream_t s)
{
    int nb, tx, ty, tz;
    grid_of(g, nb, tx, ty, tz);
    const double inv_sqN = 1.0 / sqrt((double)g.N());
    if (b)
        hipLaunchKernelGGL(k_fmg_resid3d<false>, dim3(nb), dim3(256), 0, s, ec, b, q, u, r32, P, tx, ty, tz, partial,
                           ctl, bnorm2, inv_sqN, nullptr);
    else
        hipLaunchKernelGGL(k_fmg_resid3d<true>, dim3(nb), dim3(256), 0, s, ec, nullptr, q, u, r32, P, tx, ty, tz,
                           partial, ctl, bnorm2, inv_sqN, pwf);
}

template <typename To, typename Ti>
__global__ __launch_bounds__(256) void k_convert(const cx<Ti> *__restrict__ in, cx<To> *__restrict__ out, size_t N)
{
    for (size_t j = (size_t)blockIdx.x * 256 + threadIdx.x; j < N; j += (size_t)gridDim.x * 256)
        out[j] = cvt<To>(in[j]);
}

template <typename To, typename Ti>
void launch_convert(const cx<Ti> *in, cx<To> *out, size_t N, hipStream_t s)
{
    size_t nb = (N + 255) / 256;
    if (nb > 65536) nb = 65536;
    hipLaunchKernelGGL((k_convert<To, Ti>), dim3((unsigned)nb), dim3(256), 0, s, in, out, N);
}
template void launch_convert<float, double>(const cd *, cf *, size_t, hipStream_t);
template void launch_convert<double, float>(const cf *, cd *, size_t, hipStream_t);

// Dense [A | I] of the coarsest operator (n x 2n, row-major).
__global__ __launch_bounds__(256) void k_build_coarse(const cd *__restrict__ q, cd *__restrict__ aug,
                                                      Stencil<double> P, int dim)
{
    const int mx = P.mx, my = P.my, mz = P.mz;
    const int n = mx * my * mz;
    for (int e = blockIdx.x * 256 + threadIdx.x; e < n * 2 * n; e += gridDim.x * 256) {
        int i = e / (2 * n), j = e - i * 2 * n;
        cd v = {0.0, 0.0};
        if (j >= n) {
            if (j - n == i) v = cd{1.0, 0.0};
        } else {
            int ix = i % mx, iy = (i / mx) % my, iz = i / (mx * my);
            int jx = j % mx, jy = (j / mx) % my, jz = j / (mx * my);
            int dx = jx - ix, dy = jy - iy, dz = jz - iz;
            if (i == j) {
                cd qj = q[i];
                v = P.csum2 - cd{P.k02 + qj.re, qj.im};
            } else if (dy == 0 && dz == 0 && (dx == 1 || dx == -1)) {
                v = cd{-P.c[0].re, -P.c[0].im};
            } else if (dx == 0 && dz == 0 && (dy == 1 || dy == -1)) {
                v = cd{-P.c[1].re, -P.c[1].im};
            } else if (dim == 3 && dx == 0 && dy == 0 && (dz == 1 || dz == -1)) {
                v = cd{-P.c[2].re, -P.c[2].im};
            }
        }
        aug[e] = v;
    }
}

void launch_build_coarse(const LevelGeom &g, const Stencil<double> &P, const cd *q, cd *aug, hipStream_t s)
{
    size_t n = g.N();
    size_t tot = n * 2 * n;
    unsigned nb = (unsigned)((tot + 255) / 256);
    if (nb > 65536) nb = 65536;
    hipLaunchKernelGGL(k_build_coarse, dim3(nb), dim3(256), 0, s, q, aug, P, g.dim);
}

// Gauss-Jordan elimination with partial pivoting on [A | I] (n x 2n), one
// block of 1024 threads; leaves A^{-1} in the right half.  info[0] = 0 on
// success, k+1 if a zero pivot was met in column k.
__global__ __launch_bounds__(1024) void k_gauss_jordan(cd *__restrict__ a, int n, int *__restrict__ info)
{
    __shared__ double bestv[1024];
    __shared__ int besti[1024];
    __shared__ cd pivrow_scale;
    const int W = 2 * n;
    const int t = threadIdx.x;
    for (int k = 0; k < n; ++k) {
        double bv = -1.0;
        int bi = k;
        for (int i = k + t; i < n; i += 1024) {
            double v = abs2(a[(size_t)i * W + k]);
            if (v > bv) {
                bv = v;
                bi = i;
            }
        }
        bestv[t] = bv;
        besti[t] = bi;
        __syncthreads();
        for (int off = 512; off > 0; off >>= 1) {
            if (t < off) {
                double o = bestv[t + off];
                int oi = besti[t + off];
                if (o > bestv[t] || (o == bestv[t] && oi < besti[t])) {
                    bestv[t] = o;
                    besti[t] = oi;
                }
            }
            __syncthreads();
        }
        int p = besti[0];
        if (bestv[0] <= 0.0) {
            if (t == 0) info[0] = k + 1;
            return;
        }
        if (p != k)
            for (int j = t; j < W; j += 1024) {
                cd tmp = a[(size_t)k * W + j];
                a[(size_t)k * W + j] = a[(size_t)p * W + j];
                a[(size_t)p * W + j] = tmp;
            }
        __syncthreads();
        if (t == 0) pivrow_scale = recip(a[(size_t)k * W + k]);
        __syncthreads();
        cd sc = pivrow_scale;
        for (int j = t; j < W; j += 1024) a[(size_t)k * W + j] = a[(size_t)k * W + j] * sc;
        __syncthreads();
        // eliminate column k from every other row (columns < k of the left
        // half are already zero in the rows below and above)
        const int ncols = W - k;
        for (size_t e = t; e < (size_t)n * ncols; e += 1024) {
            int i = (int)(e / ncols), j = k + (int)(e - (size_t)i * ncols);
            if (i == k || j == k) continue;
            cd f = a[(size_t)i * W + k];
            a[(size_t)i * W + j] = a[(size_t)i * W + j] - f * a[(size_t)k * W + j];
        }
        __syncthreads();
        for (int i = t; i < n; i += 1024)
            if (i != k) a[(size_t)i * W + k] = cd{0.0, 0.0};
        __syncthreads();
    }
    if (t == 0) info[0] = 0;
}

// Blocked Gauss-Jordan for coarsest grids too large for one block to stream
// (up to 1024 unknowns): the columns are taken GJB at a time.  For a panel
// [k0, k0 + GJB), k_gjb_panel (one block, thread t holding row t's panel
// columns in registers) runs the panel's pivot steps with partial pivoting,
// recording in each row the transformation the steps apply to the rows:
// a row's new content is its old content (rows outside the pivot positions
// k0 .. k0 + GJB - 1) plus sum_t Tr[row][t] (old pivot row t), where the
// columns Tr start at zero and pivot step t sets Tr[pivot][t] = 1 before
// scaling the pivot row, so the same row operations that clear the panel
// build Tr.  It applies the recorded row swaps to the columns right of the
// panel and copies the old pivot rows there (P); k_gjb_update then forms
// every row's columns right of the panel as that combination, a rank-GJB
// update.  The panel columns themselves are not written back: columns left of
// the current panel are never read again, and the inverse is the right half.
// info[0] = k + 1 for a zero pivot in column k (then later launches return).
constexpr int GJB = 8;

__global__ void k_gj_init(int *__restrict__ info) { info[0] = 0; }

__global__ __launch_bounds__(1024) void k_gjb_panel(cd *__restrict__ a, int n, int k0, cd *__restrict__ P,
                                                    cd *__restrict__ Tr, int *__restrict__ info)
{
    __shared__ double wbest[16];
    __shared__ int wbi[16];
    __shared__ double bestv0;
    __shared__ int besti0;
    __shared__ cd prow[2 * GJB];          // the scaled pivot row: panel, then Tr
    __shared__ cd xch[2][2 * GJB];        // row exchange
    __shared__ int piv[GJB];
    if (info[0] != 0) return;
    const int W = 2 * n, t = threadIdx.x;
    const int bw = min(GJB, n - k0);
    const bool mine = t < n;
    cd pan[GJB], tr[GJB];
#pragma unroll
    for (int j = 0; j < GJB; ++j) {
        pan[j] = (mine && j < bw) ? a[(size_t)t * W + k0 + j] : cd{0.0, 0.0};
        tr[j] = cd{0.0, 0.0};
    }
    // unrolled, so that every register index below is a constant
#pragma unroll
    for (int kk = 0; kk < GJB; ++kk) {
        if (kk >= bw) break;
        const int k = k0 + kk;
        // pivot: the largest |a[i][k]|, i >= k (ties: the lowest row)
        double v = -1.0;
        int vi = t;
        if (mine && t >= k) v = abs2(pan[kk]);
        // arg-max within each wave (shuffles), then over the 16 waves
#pragma unroll 1
        for (int off = 32; off > 0; off >>= 1) {
            const double o = __shfl_xor(v, off, 64);
            const int oi = __shfl_xor(vi, off, 64);
            if (o > v || (o == v && oi < vi)) {
                v = o;
                vi = oi;
            }
        }
        if ((t & 63) == 0) {
            wbest[t >> 6] = v;
            wbi[t >> 6] = vi;
        }
        __syncthreads();
        if (t < 64) {
            v = (t < 16) ? wbest[t] : -2.0;
            vi = (t < 16) ? wbi[t] : 0x7fffffff;
#pragma unroll 1
            for (int off = 8; off > 0; off >>= 1) {
                const double o = __shfl_xor(v, off, 64);
                const int oi = __shfl_xor(vi, off, 64);
                if (o > v || (o == v && oi < vi)) {
                    v = o;
                    vi = oi;
                }
            }
            if (t == 0) {
                bestv0 = v;
                besti0 = vi;
            }
        }
        __syncthreads();
        const int p = besti0;
        if (bestv0 <= 0.0) {
            if (t == 0) info[0] = k + 1;
            return;
        }
        if (t == 0) piv[kk] = p;
        // exchange the register rows of positions k and p
        if (p != k) {
            if (t == k || t == p) {
                const int slot = (t == k) ? 0 : 1;
#pragma unroll
                for (int j = 0; j < GJB; ++j) {
                    xch[slot][j] = pan[j];
                    xch[slot][GJB + j] = tr[j];
                }
            }
            __syncthreads();
            if (t == k || t == p) {
                const int slot = (t == k) ? 1 : 0;
#pragma unroll
                for (int j = 0; j < GJB; ++j) {
                    pan[j] = xch[slot][j];
                    tr[j] = xch[slot][GJB + j];
                }
            }
        }
        // the pivot row: Tr[k][kk] = 1, then scaled
        if (t == k) {
            tr[kk] = cd{1.0, 0.0};
            const cd sc = recip(pan[kk]);
#pragma unroll
            for (int j = 0; j < GJB; ++j) {
                pan[j] = pan[j] * sc;
                tr[j] = tr[j] * sc;
                prow[j] = pan[j];
                prow[GJB + j] = tr[j];
            }
        }
        __syncthreads();
        // eliminate column k from every other row, in the panel and in Tr
        if (mine && t != k) {
            const cd f = pan[kk];
#pragma unroll
            for (int j = 0; j < GJB; ++j) {
                pan[j] = (j == kk) ? cd{0.0, 0.0} : pan[j] - f * prow[j];
                tr[j] = tr[j] - f * prow[GJB + j];
            }
        }
        // (the next step rewrites prow only after its two reduction
        // barriers, by which every thread has finished this elimination)
    }
    __syncthreads();   // piv[] complete
    if (mine)
#pragma unroll
        for (int j = 0; j < GJB; ++j) Tr[(size_t)t * GJB + j] = tr[j];
    // the recorded swaps on the columns right of the panel, in order
    const int c0 = k0 + bw, nc = W - c0;
    for (int kk = 0; kk < bw; ++kk) {
        const int k = k0 + kk, p = piv[kk];
        if (p != k)
            for (int j = t; j < nc; j += 1024) {
                const cd x = a[(size_t)k * W + c0 + j];
                a[(size_t)k * W + c0 + j] = a[(size_t)p * W + c0 + j];
                a[(size_t)p * W + c0 + j] = x;
            }
        __syncthreads();
    }
    // the old pivot rows (after the swaps), right of the panel
    for (int e = t; e < bw * nc; e += 1024) {
        const int r = e / nc, j = e - r * nc;
        P[(size_t)r * nc + j] = a[(size_t)(k0 + r) * W + c0 + j];
    }
}

// rows 4 blockIdx.y .. +3, columns c0 + 256 blockIdx.x + threadIdx.x
__global__ __launch_bounds__(256) void k_gjb_update(cd *__restrict__ a, int n, int k0, const cd *__restrict__ P,
                                                    const cd *__restrict__ Tr, const int *__restrict__ info)
{
    if (info[0] != 0) return;
    const int W = 2 * n, bw = min(GJB, n - k0), c0 = k0 + bw, nc = W - c0;
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= nc) return;
    cd pc[GJB];
#pragma unroll
    for (int q = 0; q < GJB; ++q) pc[q] = (q < bw) ? P[(size_t)q * nc + j] : cd{0.0, 0.0};
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = blockIdx.y * 4 + r;
        if (i >= n) continue;
        cd acc = (i >= k0 && i < c0) ? cd{0.0, 0.0} : a[(size_t)i * W + c0 + j];
#pragma unroll
        for (int q = 0; q < GJB; ++q) acc = acc + Tr[(size_t)i * GJB + q] * pc[q];
        a[(size_t)i * W + c0 + j] = acc;
    }
}

void launch_gauss_jordan(cd *aug, int n, int *info, hipStream_t s, cd *ws)
{
    if (n <= GJ_ONE_BLOCK_MAX || !ws) {
        hipLaunchKernelGGL(k_gauss_jordan, dim3(1), dim3(1024), 0, s, aug, n, info);
        return;
    }
    cd *P = ws, *Tr = ws + (size_t)GJB * 2 * n;
    hipLaunchKernelGGL(k_gj_init, dim3(1), dim3(1), 0, s, info);
    for (int k0 = 0; k0 < n; k0 += GJB) {
        hipLaunchKernelGGL(k_gjb_panel, dim3(1), dim3(1024), 0, s, aug, n, k0, P, Tr, info);
        const int nc = 2 * n - std::min(n, k0 + GJB);
        dim3 grid((unsigned)((nc + 255) / 256), (unsigned)((n + 3) / 4));
        hipLaunchKernelGGL(k_gjb_update, grid, dim3(256), 0, s, aug, n, k0, (const cd *)P, (const cd *)Tr,
                           (const int *)info);
    }
}

// Workspace of launch_gauss_jordan above the one-block size: the old pivot
// rows (GJB x 2n) and the transformation columns (n x GJB), complex.
size_t gauss_jordan_ws(int n) { return (size_t)GJB * 2 * n + (size_t)n * GJB; }

// Coarsest solve u = A^{-1} b with the stored inverse (right half of the
// augmented matrix, row stride 2n), in FP64 whatever T is.  One wave per row.
template <typename T>
__global__ __launch_bounds__(256) void k_coarse_apply(const cd *__restrict__ aug, int n, const cx<T> *__restrict__ b,
                                                      cx<T> *__restrict__ u, const int *__restrict__ stop)
{
    if (stop && *stop) return;
    int row = blockIdx.x * 4 + (threadIdx.x >> 6);
    int lane = threadIdx.x & 63;
    if (row >= n) return;
    const cd *ar = aug + (size_t)row * 2 * n + n;
    double re = 0.0, im = 0.0;
    for (int k = lane; k < n; k += 64) {
        cd a = ar[k];
        cx<T> bk = b[k];
        double br = (double)bk.re, bi = (double)bk.im;
        re += a.re * br - a.im * bi;
        im += a.re * bi + a.im * br;
    }
    for (int off = 32; off > 0; off >>= 1) {
        re += __shfl_down(re, off, 64);
        im += __shfl_down(im, off, 64);
    }
    if (lane == 0) u[row] = cx<T>{T(re), T(im)};
}

template <typename T>
void launch_coarse_apply(const cd *Ainv, int n, const cx<T> *b, cx<T> *u, hipStream_t s, const int *stop)
{
    hipLaunchKernelGGL((k_coarse_apply<T>), dim3((n + 3) / 4), dim3(256), 0, s, Ainv, n, b, u, stop);
}
template void launch_coarse_apply<double>(const cd *, int, const cd *, cd *, hipStream_t, const int *);
template void launch_coarse_apply<float>(const cd *, int, const cf *, cf *, hipStream_t, const int *);

// ---------------------------------------------------------------------------
// b_j = q_j exp(i k0 e^{i gamma} eta.x_j): the plane wave on the contour.
// b = q exp(i k0 cos(gamma) eta.x) at point j: the plane wave's phase along
// the real coordinates without the contour's growth factor (the stress
// right-hand side at k0 h = 1/2, where exp(i k0 eta.z) leaves the
// floating-point range).
__device__ __forceinline__ cd phase_rhs_point(const cd *__restrict__ q, size_t j, int mx, int my, int dim,
                                              double lx, double ly, double lz, double hx, double hy, double hz,
                                              double ex, double ey, double ez, double ai_s)
{
    int ix = (int)(j % mx);
    size_t rest = j / mx;
    int iy = (int)(rest % my), iz = (int)(rest / my);
    double t = ex * (lx + (double)(ix + 1) * hx);
    if (dim >= 2) t += ey * (ly + (double)(iy + 1) * hy);
    if (dim >= 3) t += ez * (lz + (double)(iz + 1) * hz);
    double ph = ai_s * t;
    return q[j] * cd{cos(ph), sin(ph)};
}

__global__ __launch_bounds__(256) void k_rhs_phase(const cd *__restrict__ q, cd *__restrict__ b, int mx, int my,
                                                   int mz, int dim, double lx, double ly, double lz, double hx,
                                                   double hy, double hz, double ex, double ey, double ez,
                                                   double ai_s)
{
    size_t N = (size_t)mx * my * mz;
    for (size_t j = (size_t)blockIdx.x * 256 + threadIdx.x; j < N; j += (size_t)gridDim.x * 256)
        b[j] = phase_rhs_point(q, j, mx, my, dim, lx, ly, lz, hx, hy, hz, ex, ey, ez, ai_s);
}

// The plane wave's per-axis factors on grid g (the layout of pw_uin), from
// c_k = cr_k + i ci_k.
__global__ __launch_bounds__(256) void k_pw_factors(cd *__restrict__ f, int mx, int my, int mz, double lx,
                                                    double ly, double lz, double hx, double hy, double hz,
                                                    double crx, double cix, double cry, double ciy, double crz,
                                                    double ciz)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < mx) f[i] = pw_factor(i, lx, hx, crx, cix);
    else if (i < mx + my) f[i] = pw_factor(i - mx, ly, hy, cry, ciy);
    else if (i < mx + my + mz) f[i] = pw_factor(i - mx - my, lz, hz, crz, ciz);
}

void launch_pw_factors(const LevelGeom &g, double gamma, double k0, const double eta[3], cd *f, hipStream_t s)
{
    // i k0 e^{i gamma} eta_k = (-k0 sin gamma) eta_k + i (k0 cos gamma) eta_k
    const double ar = -(k0 * sin(gamma)), ai = k0 * cos(gamma);
    const int n = g.m[0] + g.m[1] + g.m[2];
    hipLaunchKernelGGL(k_pw_factors, dim3((n + 255) / 256), dim3(256), 0, s, f, g.m[0], g.m[1], g.m[2], g.lo[0],
                       g.lo[1], g.lo[2], g.h[0], g.h[1], g.h[2], ar * eta[0], ai * eta[0], ar * eta[1], ai * eta[1],
                       ar * eta[2], ai * eta[2]);
}

// b = q u_in point by point from the factors f.
__global__ __launch_bounds__(256) void k_rhs(const cd *__restrict__ q, const cd *__restrict__ f, cd *__restrict__ b,
                                             int mx, int my, int mz, int dim)
{
    const size_t N = (size_t)mx * my * mz;
    const size_t j0 = (size_t)blockIdx.x * 256 + threadIdx.x, S = (size_t)gridDim.x * 256;
    GridWalk w(j0, S, mx, my);
    for (size_t j = j0; j < N; j += S, w.step()) b[j] = q[j] * pw_uin(f, w.x, w.y, w.z, mx, my, dim);
}

void launch_rhs_plane_wave(const LevelGeom &g, const cd *q, const cd *f, cd *b, hipStream_t s)
{
    size_t N = g.N();
    size_t nb = (N + 255) / 256;
    if (nb > 65536) nb = 65536;
    hipLaunchKernelGGL(k_rhs, dim3((unsigned)nb), dim3(256), 0, s, q, f, b, g.m[0], g.m[1], g.m[2], g.dim);
}

void launch_rhs_phase(const LevelGeom &g, double gamma, double k0, const double eta[3], const cd *q, cd *b,
                      hipStream_t s)
{
    size_t N = g.N();
    size_t nb = (N + 255) / 256;
    if (nb > 65536) nb = 65536;
    hipLaunchKernelGGL(k_rhs_phase, dim3((unsigned)nb), dim3(256), 0, s, q, b, g.m[0], g.m[1], g.m[2], g.dim,
                       g.lo[0], g.lo[1], g.lo[2], g.h[0], g.h[1], g.h[2], eta[0], eta[1], eta[2], k0 * cos(gamma));
}

// ---------------------------------------------------------------------------
// Mixed-precision refinement kernels (one-operation form).  The FP64 update
// u += s d uses s = ctl->scale_cur, the scale of the FP32 right-hand side the
// correction d was solved for.
__global__ __launch_bounds__(256) void k_refine_update(const cf *__restrict__ d, cd *__restrict__ u,
                                                       const SolveCtl *__restrict__ ctl, size_t N,
                                                       const int *__restrict__ stop)
{
    if (stop && *stop) return;
    const double scale = ctl->scale_cur;
    for (size_t j = (size_t)blockIdx.x * 256 + threadIdx.x; j < N; j += (size_t)gridDim.x * 256) {
        cf dj = d[j];
        cd uj = u[j];
        u[j] = cd{uj.re + scale * (double)dj.re, uj.im + scale * (double)dj.im};
    }
}

void launch_refine_update(const cf *d, cd *u, const SolveCtl *ctl, size_t N, hipStream_t s, const int *stop)
{
    size_t nb = (N + 255) / 256;
    if (nb > 65536) nb = 65536;
    hipLaunchKernelGGL(k_refine_update, dim3((unsigned)nb), dim3(256), 0, s, d, u, ctl, N, stop);
}

// FP64 residual written as FP32 after scaling: r32 = (b - A u) * inv_scale,
// with the FP64 sum |b - A u|^2 per block.
void launch_resid_to_f32(const LevelGeom &g, const Stencil<double> &P, const cd *u, const cd *b, const cd *q,
                         cf *r32, double inv_scale, double *partial, hipStream_t s)
{
    launch_mode<double, float, MODE_RESID>(g, P, inv_scale, u, b, q, r32, partial, s);
}

// The same with the scale 1 / ctl->scale_next read on the device.
void launch_resid_to_f32_ctl(const LevelGeom &g, const Stencil<double> &P, const cd *u, const cd *b, const cd *q,
                             cf *r32, const SolveCtl *ctl, double *partial, hipStream_t s, const int *stop)
{
    launch_mode<double, float, MODE_RESID>(g, P, 1.0, u, b, q, r32, partial, s, ctl, stop);
}

// ---------------------------------------------------------------------------
// Batched solve: per-instance setup and control, one launch for all
// instances (blockIdx.y = instance where a kernel needs several blocks), in
// the block structure of the single-instance kernels so that every sum is
// formed in the same order.
int norm2_blocks(size_t N) { return (int)std::min<size_t>((N + 255) / 256, 1024); }

// The plane wave's per-axis factors of every instance (the values of
// k_pw_factors for its grid and direction).
__global__ __launch_bounds__(256) void k_init_pw_batch(const InitJob *__restrict__ jobs)
{
    const InitJob &J = jobs[blockIdx.y];
    const LevelGeom &g = J.g;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < g.m[0]) J.f[i] = pw_factor(i, g.lo[0], g.h[0], J.ar_s * J.eta[0], J.ai_s * J.eta[0]);
    else if (i < g.m[0] + g.m[1])
        J.f[i] = pw_factor(i - g.m[0], g.lo[1], g.h[1], J.ar_s * J.eta[1], J.ai_s * J.eta[1]);
}

// u = 0 (the start when there is no full multigrid start).
__global__ __launch_bounds__(256) void k_init_zero_batch(const InitJob *__restrict__ jobs)
{
    const InitJob &J = jobs[blockIdx.y];
    const size_t N = (size_t)J.g.m[0] * J.g.m[1];
    for (size_t j = (size_t)blockIdx.x * 256 + threadIdx.x; j < N; j += (size_t)gridDim.x * 256)
        J.u[j] = cd{0.0, 0.0};
}

// per-block |b|^2, b = q u_in, with the partition of the single-instance norm
__global__ __launch_bounds__(256) void k_init_norm_batch(const InitJob *__restrict__ jobs)
{
    const InitJob &J = jobs[blockIdx.y];
    const int nb = J.nb_norm;
    if ((int)blockIdx.x >= nb) return;
    const int mx = J.g.m[0], my = J.g.m[1];
    const size_t N = (size_t)mx * my;
    double acc = 0.0;
    const size_t j0 = (size_t)blockIdx.x * 256 + threadIdx.x, S = (size_t)nb * 256;
    GridWalk w(j0, S, mx, my);
    for (size_t j = j0; j < N; j += S, w.step()) acc += abs2(J.q[j] * pw_uin(J.f, w.x, w.y, 0, mx, my, 2));
    block_sum_256(acc, J.partial + blockIdx.x);
}

// ||b||^2 and the control block (one block per instance)
__global__ __launch_bounds__(256) void k_init_ctl_batch(const InitJob *__restrict__ jobs)
{
    const InitJob &J = jobs[blockIdx.x];
    double b2 = sum_parts_256(J.partial, J.nb_norm);
    if (threadIdx.x != 0) return;
    ctl_init_store(J.ctl, b2, J.tol, J.inv_sqN, J.max_cycles);
}

// initial residual b - A u (u = 0) as the scaled FP32 right-hand side
__global__ __launch_bounds__(256) void k_init_resid_batch(const InitJob *__restrict__ jobs)
{
    const InitJob &J = jobs[blockIdx.y];
    const int nb = J.nb_res;
    if ((int)blockIdx.x >= nb) return;
    const double rscale = 1.0 / J.ctl->scale_next;
    stencil2d_body<double, float, MODE_RESID, true>(J.u, nullptr, J.q, J.r32, J.P, rscale, J.tiles_x,
                                                    xcd_tile(blockIdx.x, nb), J.partial + blockIdx.x, J.f);
}

__global__ __launch_bounds__(256) void k_ctl_update_batch(const CtlJob *__restrict__ jobs)
{
    const CtlJob &J = jobs[blockIdx.x];
    ctl_update_body(J.ctl, J.parts, J.n);
}

__global__ __launch_bounds__(256) void k_count_done(const CtlJob *__restrict__ jobs, int n, int *__restrict__ ndone)
{
    __shared__ int cnt;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += 256)
        if (jobs[i].ctl->done) atomicAdd(&cnt, 1);
    __syncthreads();
    if (threadIdx.x == 0) *ndone = cnt;
}

// after the loop: the iterate of an instance that took an odd number of
// refinement steps is in the other buffer
__global__ __launch_bounds__(256) void k_finish_batch(const FinishJob *__restrict__ jobs)
{
    const FinishJob &J = jobs[blockIdx.y];
    if (J.ctl->k <= 0 || (J.ctl->k & 1) == 0) return;
    for (size_t j = (size_t)blockIdx.x * 256 + threadIdx.x; j < J.N; j += (size_t)gridDim.x * 256) J.u[j] = J.t[j];
}

void launch_init_batch(const InitJob *jobs, int n, int max_nb_norm, int max_m, bool zero, hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_init_pw_batch, dim3((2 * max_m + 255) / 256, n), dim3(256), 0, s, jobs);
    if (zero) hipLaunchKernelGGL(k_init_zero_batch, dim3(1024, n), dim3(256), 0, s, jobs);
    hipLaunchKernelGGL(k_init_norm_batch, dim3(max_nb_norm, n), dim3(256), 0, s, jobs);
    hipLaunchKernelGGL(k_init_ctl_batch, dim3(n), dim3(256), 0, s, jobs);
}

void launch_init_resid_batch(const InitJob *jobs, int n, int max_nb_res, hipStream_t s)
{
    if (n > 0) hipLaunchKernelGGL(k_init_resid_batch, dim3(max_nb_res, n), dim3(256), 0, s, jobs);
}

// Batched full multigrid transfers (blockIdx.y = job), point for point the
// arithmetic of k_inject_rhs, k_inject and k_prolong_set on a 2D level.
template <int KIND>
__global__ __launch_bounds__(256) void k_xfer_batch(const XferJob *__restrict__ jobs)
{
    const XferJob &J = jobs[blockIdx.y];
    if (J.stop && *J.stop) return;
    const int mxf = J.mxf, mxc = J.mxc;
    if constexpr (KIND <= 1) {
        const size_t Nc = (size_t)mxc * J.myc;
        for (size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x; idx < Nc; idx += (size_t)gridDim.x * 256) {
            const int I = (int)(idx % mxc), K = (int)(idx / mxc);
            const size_t f = (size_t)(2 * K + 1) * mxf + (2 * I + 1);
            if constexpr (KIND == 0) {
                const double inv = 1.0 / fmg_scale(J.bnorm2, J.inv_sqN);
                const cd v = J.src ? static_cast<const cd *>(J.src)[f]
                                   : J.qf[f] * pw_uin(J.pwf, 2 * I + 1, 2 * K + 1, 0, mxf, J.myf, 2);
                static_cast<cf *>(J.dst)[idx] = cvt<float>(cd{v.re * inv, v.im * inv});
            } else {
                static_cast<cf *>(J.dst)[idx] = static_cast<const cf *>(J.src)[f];
            }
        }
    } else {
        const size_t Nf = (size_t)mxf * J.myf;
        const cf *ec = static_cast<const cf *>(J.src);
        for (size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x; idx < Nf; idx += (size_t)gridDim.x * 256) {
            const int ix = (int)(idx % mxf), iy = (int)(idx / mxf);
            const cf v = prolong_at<float, 2>(ec, ix, iy, 0, mxc, J.myc, 1);
            if constexpr (KIND == 3) {
                const double sc = fmg_scale(J.bnorm2, J.inv_sqN);
                static_cast<cd *>(J.dst)[idx] = cd{(double)v.re * sc, (double)v.im * sc};
            } else {
                static_cast<cf *>(J.dst)[idx] = v;
            }
        }
    }
}

void launch_xfer_batch(int kind, const XferJob *jobs, int njobs, size_t max_n, hipStream_t s)
{
    if (njobs <= 0 || max_n == 0) return;
    const dim3 grid((unsigned)std::min<size_t>((max_n + 255) / 256, 1024), (unsigned)njobs);
    switch (kind) {
    case 0: hipLaunchKernelGGL(k_xfer_batch<0>, grid, dim3(256), 0, s, jobs); break;
    case 1: hipLaunchKernelGGL(k_xfer_batch<1>, grid, dim3(256), 0, s, jobs); break;
    case 2: hipLaunchKernelGGL(k_xfer_batch<2>, grid, dim3(256), 0, s, jobs); break;
    default: hipLaunchKernelGGL(k_xfer_batch<3>, grid, dim3(256), 0, s, jobs); break;
    }
}

void launch_ctl_update_batch(const CtlJob *jobs, int n, hipStream_t s)
{
    if (n > 0) hipLaunchKernelGGL(k_ctl_update_batch, dim3(n), dim3(256), 0, s, jobs);
}

void launch_count_done(const CtlJob *jobs, int n, int *ndone, hipStream_t s)
{
    hipLaunchKernelGGL(k_count_done, dim3(1), dim3(256), 0, s, jobs, n, ndone);
}

void launch_finish_batch(const FinishJob *jobs, int n, hipStream_t s)
{
    if (n > 0) hipLaunchKernelGGL(k_finish_batch, dim3(1024, n), dim3(256), 0, s, jobs);
}

// Pseudo-random complex values in [-1, 1)^2 from a counter-based hash of
// (seed, index) (the splitmix64 finaliser), for calibration runs.
__device__ __forceinline__ unsigned long long mix64(unsigned long long z)
{
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ __launch_bounds__(256) void k_hash_fill(cd *__restrict__ out, size_t N, unsigned long long seed)
{
    for (size_t j = (size_t)blockIdx.x * 256 + threadIdx.x; j < N; j += (size_t)gridDim.x * 256) {
        unsigned long long a = mix64(seed ^ (2 * j)), c = mix64(seed ^ (2 * j + 1));
        out[j] = cd{(double)(a >> 11) * 0x1.0p-52 - 1.0, (double)(c >> 11) * 0x1.0p-52 - 1.0};
    }
}

void launch_hash_fill(cd *out, size_t N, unsigned long long seed, hipStream_t s)
{
    size_t nb = std::min<size_t>((N + 255) / 256, 65536);
    hipLaunchKernelGGL(k_hash_fill, dim3((unsigned)nb), dim3(256), 0, s, out, N, seed);
}

}  // namespace ffmg
