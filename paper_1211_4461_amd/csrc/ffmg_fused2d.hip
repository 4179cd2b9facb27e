// ffmg_fused2d.hip -- fused 2D multigrid kernels for gfx950.
//
// The V-cycle of Sec. 4 is, per level: nu1 omega-Jacobi sweeps, restriction
// of the residual, coarse correction, interpolation, nu2 sweeps.  Done one
// operation per launch it streams every field through HBM about 23 times per
// level and pays ~7 launches.  These kernels run one level in 3 launches:
//
//   k_smooth2d<NS, ZERO, PROL>  NS (1 or 2) sweeps in one pass: the u tile is
//       staged in LDS with an NS-deep halo, sweep 1 is computed on the tile
//       plus an (NS-1) halo, sweep 2 on the tile.  ZERO: the incoming u is 0
//       (coarse corrections), so sweep 1 is omega b / D and u is not read.
//       PROL: u + P e_c (bilinear interpolation of the coarse correction) is
//       formed while staging, i.e. the coarse-grid correction is fused into
//       the first post-smoothing sweep.
//   k_resid_restrict2d  r = b - A u on the fine points a coarse tile needs,
//       kept in LDS, then full weighting (1/4, 1/2, 1/4)^2 to b_c.
//   k_refine2d  the FP64 outer step of the mixed-precision solve: u' = u +
//       s d (FP64 update of the FP32 correction), r = b - A u' in FP64,
//       written as FP32 r / s' (the next scaled right-hand side) with the
//       FP64 sum |r|^2 per block.
//   k_tail2d  the coarse end of the cycle (all levels small enough for LDS and
//       the exact coarsest solve) in one 1024-thread workgroup: on those
//       levels a launch per operation would cost far more than the work.
//
// Per point the arithmetic is the same as the one-operation kernels in
// ffmg_stencil.hip (same operation order, same reduction order in the
// coarsest solve), so the fused path reproduces them bit for bit.
#include <algorithm>

#include "ffmg_internal.hpp"
#include "ffmg_point.hpp"

namespace ffmg {

constexpr int FTX = 64;     // tile width (one wavefront of x)
constexpr int FTY = 16;     // tile height
constexpr int RCX = 32;     // resid_restrict: coarse tile 32 x 8 (one point per thread)
constexpr int RCY = 8;

// Interpolated coarse correction at fine interior point (ix, iy) (0-based):
// coarse nodes floor(f/2), ceil(f/2) of fine node f = i + 1, weights 1 or 1/2,
// summed y-outer / x-inner as in the one-operation kernel.  The coarse field
// is read from ec[(ay - oy) * ld + (ax - ox)] (a tile of it, or all of it).
template <typename T>
__device__ __forceinline__ cx<T> interp2d(const cx<T> *ec, int ld, int ox, int oy, int mxc, int myc, int ix, int iy)
{
    int fx = ix + 1, fy = iy + 1;
    cx<T> acc = {T(0), T(0)};
    for (int Cy = fy / 2; Cy <= (fy + 1) / 2; ++Cy)
        for (int Cx = fx / 2; Cx <= (fx + 1) / 2; ++Cx) {
            int dx = fx - 2 * Cx, dy = fy - 2 * Cy;
            T wx = dx == 0 ? T(1) : T(0.5), wy = dy == 0 ? T(1) : T(0.5);
            T wgt = wx * wy * T(1);
            int ax = Cx - 1, ay = Cy - 1;
            if (ax < 0 || ay < 0 || ax >= mxc || ay >= myc) continue;
            acc = acc + wgt * ec[(ay - oy) * ld + (ax - ox)];
        }
    return acc;
}

// Tile heights of the smoothing kernel (rows of 64 points): a tunable of the
// handle (FFMG_TUNE_SMOOTH); the batched path its own (FFMG_TUNE_BATCH).  Every
// height computes the same bits.
// (smoothing, one-pass pre-smoothing) tile heights of the batched path, by
// FFMG_TUNE_BATCH variant
constexpr int BATCH_TILES[][2] = {{8, 16}, {4, 16}, {16, 16}, {8, 8}};
constexpr int BATCH_VARIANTS = (int)(sizeof(BATCH_TILES) / sizeof(BATCH_TILES[0]));
static_assert(BATCH_VARIANTS == BATCH_TUNE_VARIANTS, "batch tile table");

// k_smooth2d runs in four phases separated by barriers:
//   1. every global load of the block is issued together (fully unrolled
//      loops): the u tile with its NS-deep halo and the coarse-correction tile
//      (PROL) into LDS, b and q of the thread's own points into registers;
//   2. (PROL) u += P e_c in LDS;
//   3. (NS = 2) sweep 1 on the tile plus a one-point halo;
//   4. the last sweep on the tile, written to out.
// Each thread keeps the same points of the sweep-1 region (the tile plus an
// (NS-1) halo) in phases 3 and 4, so b and omega / D of its points stay in
// registers; only u values that neighbours read pass through LDS.
template <typename T, int NS, bool ZERO, bool PROL, int TH>
__device__ __forceinline__ void smooth2d_body(const cx<T> *__restrict__ u, const cx<T> *__restrict__ ec,
                                              const cx<T> *__restrict__ b, const cx<T> *__restrict__ q,
                                              cx<T> *__restrict__ out, const Stencil<T> &P, int tiles_x, int tile)
{
    static_assert(TH % 4 == 0 && TH >= 4, "tile height: a multiple of the 4 rows of a 256-thread block");
    constexpr int H = NS;                                  // halo depth of the staged u
    constexpr int UW = FTX + 2 * H, UH = TH + 2 * H;
    constexpr int BO = NS - 1;                             // sweep-1 region: tile + (NS-1) halo
    constexpr int BW = FTX + 2 * BO, BH = TH + 2 * BO;
    constexpr int ECW = FTX / 2 + 4, ECH = TH / 2 + 4;     // coarse tile covering the u region
    constexpr int U1H = NS == 2 ? BH : 1, U1W = NS == 2 ? BW : 1;
    constexpr int ECH_ = PROL ? ECH : 1, ECW_ = PROL ? ECW : 1;
    __shared__ cx<T> U0[ZERO ? 1 : UH][ZERO ? 1 : UW];
    // the coarse tile is dead once phase 2 has ended (barrier), before sweep 1
    // writes U1: the two share storage
    __shared__ cx<T> U1EC[U1H * U1W > ECH_ * ECW_ ? U1H * U1W : ECH_ * ECW_];
    cx<T>(&U1)[U1H][U1W] = *reinterpret_cast<cx<T>(*)[U1H][U1W]>(&U1EC[0]);
    cx<T>(&EC)[ECH_][ECW_] = *reinterpret_cast<cx<T>(*)[ECH_][ECW_]>(&U1EC[0]);
    const int mx = P.mx, my = P.my;
    const int mxc = (mx - 1) / 2, myc = (my - 1) / 2;
    const int x0 = (tile % tiles_x) * FTX, y0 = (tile / tiles_x) * TH;
    const int ecx0 = x0 / 2 - 2, ecy0 = y0 / 2 - 2;
    const cx<T> zero = {T(0), T(0)};

    // phase 1: loads, issued into registers first so that all of them are in
    // flight together, then the shared ones stored to LDS
    constexpr int NU = ZERO ? 1 : (UH * UW + 255) / 256;
    constexpr int NP = (BH * BW + 255) / 256;             // the thread's points: slot k is point tid + 256 k
    constexpr int NE = PROL ? (ECH * ECW + 255) / 256 : 1;
    cx<T> ru[NU], rb[NP], rw[NP], re[NE];
    int px[NP], py[NP];
    bool act[NP], ing[NP];
    if (!ZERO) {
#pragma unroll
        for (int k = 0; k < NU; ++k) {
            int i = threadIdx.x + 256 * k;
            int ly = i / UW, lx = i - ly * UW;
            int gx = x0 + lx - H, gy = y0 + ly - H;
            bool in = i < UH * UW && gx >= 0 && gx < mx && gy >= 0 && gy < my;
            ru[k] = ld_masked(u, (size_t)gy * mx + gx, in);
        }
    }
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        int i = threadIdx.x + 256 * k;
        py[k] = i / BW;
        px[k] = i - py[k] * BW;
        act[k] = i < BH * BW;
        int gx = x0 + px[k] - BO, gy = y0 + py[k] - BO;
        ing[k] = act[k] && gx >= 0 && gx < mx && gy >= 0 && gy < my;
        size_t j = (size_t)gy * mx + gx;
        rb[k] = ld_masked(b, j, ing[k]);
        rw[k] = ld_masked(q, j, ing[k]);
    }
    if (PROL) {
#pragma unroll
        for (int k = 0; k < NE; ++k) {
            int i = threadIdx.x + 256 * k;
            int ly = i / ECW, lx = i - ly * ECW;
            int cx_ = ecx0 + lx, cy_ = ecy0 + ly;
            bool in = i < ECH * ECW && cx_ >= 0 && cx_ < mxc && cy_ >= 0 && cy_ < myc;
            re[k] = ld_masked(ec, (size_t)cy_ * mxc + cx_, in);
        }
    }
    if (!ZERO) {
#pragma unroll
        for (int k = 0; k < NU; ++k) {
            int i = threadIdx.x + 256 * k;
            if (i < UH * UW) (&U0[0][0])[i] = ru[k];
        }
    }
    if (PROL) {
#pragma unroll
        for (int k = 0; k < NE; ++k) {
            int i = threadIdx.x + 256 * k;
            if (i < ECH * ECW) (&EC[0][0])[i] = re[k];
        }
    }
#pragma unroll
    for (int k = 0; k < NP; ++k) rw[k] = jweight(P, rw[k]);   // q -> omega / D
    __syncthreads();
    // phase 2: coarse-grid correction u += P e_c on the staged u.  Branch
    // free: fine node f = g + 1 takes coarse interior nodes f/2 - 1 (weight 1
    // if f is even, 1/2 if odd) and f/2 (weight 0 if even, 1/2 if odd); coarse
    // nodes outside the grid are zero in EC.  The terms are summed in the
    // order of the one-operation kernel; the extra zero-weight terms add 0.
    if (PROL) {
        for (int i = threadIdx.x; i < UH * UW; i += 256) {
            int ly = i / UW, lx = i - ly * UW;
            int gx = x0 + lx - H, gy = y0 + ly - H;
            if (gx >= 0 && gx < mx && gy >= 0 && gy < my) {
                int fx = gx + 1, fy = gy + 1;
                int ex = (fx >> 1) - 1 - ecx0, ey = (fy >> 1) - 1 - ecy0;
                T wx0 = (fx & 1) ? T(0.5) : T(1), wx1 = (fx & 1) ? T(0.5) : T(0);
                T wy0 = (fy & 1) ? T(0.5) : T(1), wy1 = (fy & 1) ? T(0.5) : T(0);
                cx<T> acc = {T(0), T(0)};
                acc = acc + (wx0 * wy0 * T(1)) * EC[ey][ex];
                acc = acc + (wx1 * wy0 * T(1)) * EC[ey][ex + 1];
                acc = acc + (wx0 * wy1 * T(1)) * EC[ey + 1][ex];
                acc = acc + (wx1 * wy1 * T(1)) * EC[ey + 1][ex + 1];
                U0[ly][lx] = U0[ly][lx] + acc;
            }
        }
        __syncthreads();
    }
    // phase 3: sweep 1 on the tile plus a one-point halo (zero outside the domain)
    if (NS == 2) {
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            if (!act[k]) continue;
            const int sx = px[k], sy = py[k];
            cx<T> v = zero;
            if (ing[k]) {
                if (ZERO) {
                    v = jacobi0_w(rb[k], rw[k]);
                } else {
                    int ux = sx + 1, uy = sy + 1;            // same point in U0 (halo 2)
                    v = jacobi_point<T>(P, U0[uy][ux], U0[uy][ux - 1], U0[uy][ux + 1], U0[uy - 1][ux],
                                        U0[uy + 1][ux], rb[k], rw[k]);
                }
            }
            U1[sy][sx] = v;
        }
        __syncthreads();
    }
    // phase 4: last sweep on the tile (the thread's points inside it)
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const int sx = px[k], sy = py[k];
        if (!ing[k] || sx < BO || sx >= BO + FTX || sy < BO || sy >= BO + TH) continue;
        const size_t j = (size_t)(y0 + sy - BO) * mx + (x0 + sx - BO);
        cx<T> v;
        if (NS == 2) {
            v = jacobi_point<T>(P, U1[sy][sx], U1[sy][sx - 1], U1[sy][sx + 1], U1[sy - 1][sx], U1[sy + 1][sx], rb[k],
                                rw[k]);
        } else if (ZERO) {
            v = jacobi0_w(rb[k], rw[k]);
        } else {
            int ax = sx + H, ay = sy + H;
            v = jacobi_point<T>(P, U0[ay][ax], U0[ay][ax - 1], U0[ay][ax + 1], U0[ay - 1][ax], U0[ay + 1][ax], rb[k],
                                rw[k]);
        }
        out[j] = v;
    }
}

template <typename T, int NS, bool ZERO, bool PROL, int TAG, int TH>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_smooth2d(const cx<T> *__restrict__ u, const cx<T> *__restrict__ ec,
                                                  const cx<T> *__restrict__ b, const cx<T> *__restrict__ q,
                                                  cx<T> *__restrict__ out, Stencil<T> P, int tiles_x,
                                                  const int *__restrict__ stop)
{
    if (stop && *stop) return;
    smooth2d_body<T, NS, ZERO, PROL, TH>(u, ec, b, q, out, P, tiles_x, xcd_tile(blockIdx.x, gridDim.x));
}

// Residual + full weighting.  Coarse tile RCX x RCY; the fine residual is
// needed at fine interior indices [2 I0, 2 (I0 + RCX)] x [2 J0, 2 (J0 + RCY)].
template <typename T>
__device__ __forceinline__ void resid_restrict2d_body(const cx<T> *__restrict__ u, const cx<T> *__restrict__ b,
                                                      const cx<T> *__restrict__ q, cx<T> *__restrict__ bc,
                                                      const Stencil<T> &P, int ctiles_x, int tile)
{
    constexpr int RW = 2 * RCX + 1, RH = 2 * RCY + 1;   // residual region
    constexpr int UW = RW + 2, UH = RH + 2;             // u region (one halo)
    __shared__ cx<T> U[UH][UW];
    __shared__ cx<T> R[RH][RW];
    const int mx = P.mx, my = P.my;
    const int mxc = (mx - 1) / 2, myc = (my - 1) / 2;
    const int I0 = (tile % ctiles_x) * RCX, J0 = (tile / ctiles_x) * RCY;
    const int fx0 = 2 * I0, fy0 = 2 * J0;               // first fine index of R
    const cx<T> zero = {T(0), T(0)};
    // all global loads of the block first: u with its halo, b and q on the
    // residual region (fully unrolled so they are in flight together)
    constexpr int NR = (RH * RW + 255) / 256;
    cx<T> breg[NR], qreg[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        int i = threadIdx.x + 256 * k;
        int ly = i / RW, lx = i - ly * RW;
        int gx = fx0 + lx, gy = fy0 + ly;
        bool in = i < RH * RW && gx < mx && gy < my;
        size_t j = (size_t)gy * mx + gx;
        breg[k] = ld_masked(b, j, in);
        qreg[k] = ld_masked(q, j, in);
    }
#pragma unroll
    for (int k = 0; k < (UH * UW + 255) / 256; ++k) {
        int i = threadIdx.x + 256 * k;
        if (i < UH * UW) {
            int ly = i / UW, lx = i - ly * UW;
            int gx = fx0 + lx - 1, gy = fy0 + ly - 1;
            bool in = gx >= 0 && gx < mx && gy >= 0 && gy < my;
            U[ly][lx] = ld_masked(u, (size_t)gy * mx + gx, in);
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        int i = threadIdx.x + 256 * k;
        if (i < RH * RW) {
            int ly = i / RW, lx = i - ly * RW;
            int gx = fx0 + lx, gy = fy0 + ly;
            cx<T> r = zero;
            if (gx < mx && gy < my)
                r = resid_point<T>(P, U[ly + 1][lx + 1], U[ly + 1][lx], U[ly + 1][lx + 2], U[ly][lx + 1],
                                   U[ly + 2][lx + 1], breg[k], qreg[k]);
            R[ly][lx] = r;
        }
    }
    __syncthreads();
    const int ci = threadIdx.x % RCX, cj = threadIdx.x / RCX;
    const int I = I0 + ci, J = J0 + cj;
    if (I < mxc && J < myc) {
        const T w[3] = {T(0.25), T(0.5), T(0.25)};
        cx<T> acc = {T(0), T(0)};
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                T wgt = (w[dx + 1] * w[dy + 1]) * T(1);
                acc = acc + wgt * R[2 * cj + 1 + dy][2 * ci + 1 + dx];
            }
        bc[(size_t)J * mxc + I] = acc;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_resid_restrict2d(const cx<T> *__restrict__ u, const cx<T> *__restrict__ b,
                                                          const cx<T> *__restrict__ q, cx<T> *__restrict__ bc,
                                                          Stencil<T> P, int ctiles_x, const int *__restrict__ stop)
{
    if (stop && *stop) return;
    resid_restrict2d_body<T>(u, b, q, bc, P, ctiles_x, xcd_tile(blockIdx.x, gridDim.x));
}

// Pre-smoothing (two sweeps), residual and full weighting in one pass.  The
// block owns the fine points [x0, x0 + 64) x [y0, y0 + FH) (written to out:
// the smoothed u) and the coarse points whose centre lies there, I in
// [x0/2, x0/2 + 32), J in [y0/2, y0/2 + FH/2) (written to bc).  Their full
// weighting needs the residual on [x0, x0 + 64] x [y0, y0 + FH] (one column
// and one row past the owned points); the residual needs the smoothed u one
// point further out, sweep 2 needs sweep 1 one point further, sweep 1 needs u
// one point further:
//   R   [x0, x0 + 64]      x [y0, y0 + FH]          residual
//   S2  [x0 - 1, x0 + 65]  x [y0 - 1, y0 + FH + 1]  sweep 2 (the smoothed u)
//   S1  [x0 - 2, x0 + 66]  x [y0 - 2, y0 + FH + 2]  sweep 1
//   U0  [x0 - 3, x0 + 67]  x [y0 - 3, y0 + FH + 3]  incoming u (not ZERO)
// Each thread keeps the same points of S1 through sweep 1, sweep 2 and the
// residual (S2 and R lie inside S1), so b, q and omega / D of its points stay
// in registers and only the u values that neighbours read pass through LDS.
// Values outside the grid are 0 (the Dirichlet border).  Every value is
// formed by the same point functions as in k_smooth2d and
// k_resid_restrict2d, so the pass equals the two launches bit for bit; it
// skips their re-read of the smoothed u, b and q and one launch.
template <typename T, bool ZERO, int FH>
__device__ __forceinline__ void smooth_rr2d_body(const cx<T> *__restrict__ u, const cx<T> *__restrict__ b,
                                                 const cx<T> *__restrict__ q, cx<T> *__restrict__ out,
                                                 cx<T> *__restrict__ bc, const Stencil<T> &P, int tiles_x, int tile)
{
    static_assert(FH % 8 == 0, "fine tile height: a multiple of 8 rows");
    constexpr int RW = FTX + 1, RH = FH + 1;
    constexpr int S2W = FTX + 3, S2H = FH + 3;
    constexpr int S1W = FTX + 5, S1H = FH + 5;
    constexpr int UW = FTX + 7, UH = FH + 7;
    constexpr int A0 = (ZERO ? S2H * S2W : (UH * UW > S2H * S2W ? UH * UW : S2H * S2W));
    constexpr int A1 = S1H * S1W > RH * RW ? S1H * S1W : RH * RW;
    // U0 is dead once sweep 1 is done, S1 once sweep 2 is done (barriers)
    __shared__ cx<T> L0[A0];
    __shared__ cx<T> L1[A1];
    cx<T>(&U0)[UH][UW] = *reinterpret_cast<cx<T>(*)[UH][UW]>(&L0[0]);
    cx<T>(&S2)[S2H][S2W] = *reinterpret_cast<cx<T>(*)[S2H][S2W]>(&L0[0]);
    cx<T>(&S1)[S1H][S1W] = *reinterpret_cast<cx<T>(*)[S1H][S1W]>(&L1[0]);
    cx<T>(&R)[RH][RW] = *reinterpret_cast<cx<T>(*)[RH][RW]>(&L1[0]);
    const int mx = P.mx, my = P.my;
    const int mxc = (mx - 1) / 2, myc = (my - 1) / 2;
    const int x0 = (tile % tiles_x) * FTX, y0 = (tile / tiles_x) * FH;
    const cx<T> zero = {T(0), T(0)};

    // the thread's points of S1: slot k is point threadIdx.x + 256 k
    constexpr int NP = (S1H * S1W + 255) / 256;
    int px[NP], py[NP];
    bool act[NP], ing[NP];
    cx<T> rb[NP], rq[NP], rw[NP];
    constexpr int NU = ZERO ? 1 : (UH * UW + 255) / 256;
    cx<T> ru[NU];
    if (!ZERO) {
#pragma unroll
        for (int k = 0; k < NU; ++k) {
            int i = threadIdx.x + 256 * k;
            int ly = i / UW, lx = i - ly * UW;
            int gx = x0 + lx - 3, gy = y0 + ly - 3;
            bool in = i < UH * UW && gx >= 0 && gx < mx && gy >= 0 && gy < my;
            ru[k] = ld_masked(u, (size_t)gy * mx + gx, in);
        }
    }
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        int i = threadIdx.x + 256 * k;
        py[k] = i / S1W;
        px[k] = i - py[k] * S1W;
        act[k] = i < S1H * S1W;
        int gx = x0 + px[k] - 2, gy = y0 + py[k] - 2;
        ing[k] = act[k] && gx >= 0 && gx < mx && gy >= 0 && gy < my;
        size_t j = (size_t)gy * mx + gx;
        rb[k] = ld_masked(b, j, ing[k]);
        rq[k] = ld_masked(q, j, ing[k]);
    }
    if (!ZERO) {
#pragma unroll
        for (int k = 0; k < NU; ++k) {
            int i = threadIdx.x + 256 * k;
            if (i < UH * UW) (&U0[0][0])[i] = ru[k];
        }
    }
#pragma unroll
    for (int k = 0; k < NP; ++k) rw[k] = jweight(P, rq[k]);
    __syncthreads();
    // sweep 1 on S1
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        if (!act[k]) continue;
        const int sx = px[k], sy = py[k];
        cx<T> v = zero;
        if (ing[k]) {
            if (ZERO) {
                v = jacobi0_w(rb[k], rw[k]);
            } else {
                int ux = sx + 1, uy = sy + 1;
                v = jacobi_point<T>(P, U0[uy][ux], U0[uy][ux - 1], U0[uy][ux + 1], U0[uy - 1][ux], U0[uy + 1][ux],
                                    rb[k], rw[k]);
            }
        }
        S1[sy][sx] = v;
    }
    __syncthreads();
    // sweep 2 on S2 (over U0's storage); the owned points go to out
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const int sx = px[k], sy = py[k];                     // S1 coordinates; S2 is S1 less its rim
        if (!act[k] || sx < 1 || sx > S2W || sy < 1 || sy > S2H) continue;
        cx<T> v = zero;
        if (ing[k]) {
            v = jacobi_point<T>(P, S1[sy][sx], S1[sy][sx - 1], S1[sy][sx + 1], S1[sy - 1][sx], S1[sy + 1][sx], rb[k],
                                rw[k]);
            if (sx >= 2 && sx <= FTX + 1 && sy >= 2 && sy <= FH + 1)
                out[(size_t)(y0 + sy - 2) * mx + (x0 + sx - 2)] = v;
        }
        S2[sy - 1][sx - 1] = v;
    }
    __syncthreads();
    // residual on R (over S1's storage)
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const int sx = px[k], sy = py[k];                     // R is S1 less two rims, low sides
        if (!act[k] || sx < 2 || sx > RW + 1 || sy < 2 || sy > RH + 1) continue;
        const int tx = sx - 1, ty = sy - 1;                   // same point in S2
        cx<T> r = zero;
        if (ing[k])
            r = resid_point<T>(P, S2[ty][tx], S2[ty][tx - 1], S2[ty][tx + 1], S2[ty - 1][tx], S2[ty + 1][tx], rb[k],
                               rq[k]);
        R[sy - 2][sx - 2] = r;
    }
    __syncthreads();
    // full weighting at the owned coarse points
    const int I0 = x0 / 2, J0 = y0 / 2;
    for (int i = threadIdx.x; i < (FTX / 2) * (FH / 2); i += 256) {
        const int cj = i / (FTX / 2), ci = i - cj * (FTX / 2);
        const int I = I0 + ci, J = J0 + cj;
        if (I < mxc && J < myc) {
            const T w[3] = {T(0.25), T(0.5), T(0.25)};
            cx<T> acc = {T(0), T(0)};
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    T wgt = (w[dx + 1] * w[dy + 1]) * T(1);
                    acc = acc + wgt * R[2 * cj + 1 + dy][2 * ci + 1 + dx];
                }
            bc[(size_t)J * mxc + I] = acc;
        }
    }
}

template <typename T, bool ZERO, int TAG, int FH>
__global__ __launch_bounds__(256) void k_smooth_rr2d(const cx<T> *__restrict__ u, const cx<T> *__restrict__ b,
                                                     const cx<T> *__restrict__ q, cx<T> *__restrict__ out,
                                                     cx<T> *__restrict__ bc, Stencil<T> P, int tiles_x,
                                                     const int *__restrict__ stop)
{
    if (stop && *stop) return;
    smooth_rr2d_body<T, ZERO, FH>(u, b, q, out, bc, P, tiles_x, xcd_tile(blockIdx.x, gridDim.x));
}

// Mixed-precision outer step: u' = u + s d with s = ctl->scale_cur;
// r = b - A u' (FP64); r32 = r / ctl->scale_next; per-block sum |r|^2.
// Out of place in u.
// b = null: the right-hand side is the plane wave's q u_in from the factors pwf.
__device__ __forceinline__ void refine2d_body(const cd *__restrict__ u, const cf *__restrict__ d,
                                              const cd *__restrict__ b, const cd *__restrict__ q,
                                              cd *__restrict__ u_out, cf *__restrict__ r32,
                                              const SolveCtl *__restrict__ ctl, const Stencil<double> &P,
                                              int tiles_x, int tile, double *__restrict__ partial_slot,
                                              const cd *__restrict__ pwf)
{
    const double s = ctl->scale_cur;
    const double inv_scale = 1.0 / ctl->scale_next;
    __shared__ cd U[FTY + 2][FTX + 2];
    const int mx = P.mx, my = P.my;
    const int x0 = (tile % tiles_x) * FTX, y0 = (tile / tiles_x) * FTY;
#pragma unroll
    for (int k = 0; k < ((FTY + 2) * (FTX + 2) + 255) / 256; ++k) {
        int i = threadIdx.x + 256 * k;
        if (i < (FTY + 2) * (FTX + 2)) {
            int ly = i / (FTX + 2), lx = i - ly * (FTX + 2);
            int gx = x0 + lx - 1, gy = y0 + ly - 1;
            bool in = gx >= 0 && gx < mx && gy >= 0 && gy < my;
            size_t j = (size_t)gy * mx + gx;
            cd uj = ld_masked(u, j, in);
            cf dj = ld_masked(d, j, in);
            U[ly][lx] = cd{uj.re + s * (double)dj.re, uj.im + s * (double)dj.im};
        }
    }
    __syncthreads();
    const int lx = threadIdx.x & 63;
    const int gx = x0 + lx;
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < FTY / 4; ++k) {
        int ly = (threadIdx.x >> 6) + 4 * k;
        int gy = y0 + ly;
        if (gx < mx && gy < my) {
            size_t j = (size_t)gy * mx + gx;
            cd uc = U[ly + 1][lx + 1];
            const cd qj = q[j];
            const cd bj = b ? b[j] : qj * pw_uin(pwf, gx, gy, 0, mx, my, 2);
            cd r = resid_point<double>(P, uc, U[ly + 1][lx], U[ly + 1][lx + 2], U[ly][lx + 1], U[ly + 2][lx + 1],
                                       bj, qj);
            u_out[j] = uc;
            r32[j] = cvt<float>(inv_scale * r);
            acc += abs2(r);
        }
    }
    __shared__ double red[4];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) *partial_slot = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ __launch_bounds__(256) void k_refine2d(const cd *__restrict__ u, const cf *__restrict__ d,
                                                  const cd *__restrict__ b, const cd *__restrict__ q,
                                                  cd *__restrict__ u_out, cf *__restrict__ r32,
                                                  const SolveCtl *__restrict__ ctl, Stencil<double> P, int tiles_x,
                                                  double *__restrict__ partial, const int *__restrict__ stop,
                                                  const cd *__restrict__ pwf)
{
    if (stop && *stop) return;
    refine2d_body(u, d, b, q, u_out, r32, ctl, P, tiles_x, xcd_tile(blockIdx.x, gridDim.x), partial + blockIdx.x,
                  pwf);
}

// ---------------------------------------------------------------------------
// The coarse end of the V-cycle in one workgroup.  Every tail level keeps
// b, u, t and a copy of q in LDS, each as a (mx + 2) x (my + 2) array whose
// one-point border stays zero (the Dirichlet values), so stencil reads need
// no bounds tests.  Level 0 of the tail starts from a zero guess with b read
// from b_top; its correction is written to u_top.  Steps are separated by
// workgroup barriers.
template <typename T>
struct TailView {
    cx<T> *b, *u, *t, *q;
    int mx, my, W, N;
    float inv_mx;
    // padded index of interior point (x, y)
    __device__ __forceinline__ int at(int x, int y) const { return (y + 1) * W + x + 1; }
    // (x, y) of the j-th interior point, j < 2^16 (the float quotient is
    // exact there: its distance to the next integer is >= 0.5 / mx)
    __device__ __forceinline__ void xy(int j, int &x, int &y) const
    {
        y = (int)(((float)j + 0.5f) * inv_mx);
        x = j - y * mx;
    }
};

template <typename T>
__device__ __forceinline__ TailView<T> tail_view(cx<T> *lds, const TailLevel<T> &L)
{
    TailView<T> v;
    v.mx = L.mx;
    v.my = L.my;
    v.W = L.mx + 2;
    v.N = L.mx * L.my;
    v.inv_mx = 1.f / (float)L.mx;
    const int np = (L.mx + 2) * (L.my + 2);
    v.b = lds + L.off;
    v.u = v.b + np;
    v.t = v.u + np;
    v.q = v.t + np;
    return v;
}

// nu sweeps on one tail level into v.u; zero: the incoming u is 0.
template <typename T>
__device__ void tail_smooth(const TailView<T> &v, const TailLevel<T> &L, int nu, bool zero)
{
    cx<T> *src = v.u, *dst = v.t;
    for (int s = 0; s < nu; ++s) {
        for (int j = threadIdx.x; j < v.N; j += blockDim.x) {
            int x, y;
            v.xy(j, x, y);
            const int k = v.at(x, y);
            cx<T> bj = v.b[k], qj = v.q[k];
            if (s == 0 && zero) {
                dst[k] = jacobi0_w(bj, jweight(L.P, qj));
            } else {
                dst[k] = jacobi_point<T>(L.P, src[k], src[k - 1], src[k + 1], src[k - v.W], src[k + v.W], bj,
                                         jweight(L.P, qj));
            }
        }
        __syncthreads();
        cx<T> *tmp = src;
        src = dst;
        dst = tmp;
    }
    if (src != v.u) {
        for (int j = threadIdx.x; j < v.N; j += blockDim.x) {
            int x, y;
            v.xy(j, x, y);
            v.u[v.at(x, y)] = src[v.at(x, y)];
        }
        __syncthreads();
    }
    if (nu == 0 && zero) {
        for (int j = threadIdx.x; j < v.N; j += blockDim.x) {
            int x, y;
            v.xy(j, x, y);
            v.u[v.at(x, y)] = cx<T>{T(0), T(0)};
        }
        __syncthreads();
    }
}

// Zero every array (borders included), then b of tail level s0 from b_top
// and q of all levels.
template <typename T>
__device__ __forceinline__ void tail_load(const TailParams<T> &tp, const cx<T> *__restrict__ b_top, cx<T> *lds,
                                          int s0)
{
    const int nt = tp.nt;
    const TailLevel<T> &last = tp.lv[nt - 1];
    const int total = last.off + 4 * (last.mx + 2) * (last.my + 2);
    for (int j = threadIdx.x; j < total; j += blockDim.x) lds[j] = cx<T>{T(0), T(0)};
    __syncthreads();
    TailView<T> v0 = tail_view(lds, tp.lv[s0]);
    for (int j = threadIdx.x; j < v0.N; j += blockDim.x) {
        int x, y;
        v0.xy(j, x, y);
        v0.b[v0.at(x, y)] = b_top[j];
    }
    for (int i = 0; i < nt; ++i) {
        TailView<T> v = tail_view(lds, tp.lv[i]);
        const cx<T> *qs = tp.lv[i].q;
        for (int j = threadIdx.x; j < v.N; j += blockDim.x) {
            int x, y;
            v.xy(j, x, y);
            v.q[v.at(x, y)] = qs[j];
        }
    }
    __syncthreads();
}

// Coarsest tail level: u = A^{-1} b in FP64, one wave per row, lane-strided
// sums then a shuffle tree (the order of the one-operation kernel).
template <typename T>
__device__ __forceinline__ void tail_coarsest(const TailParams<T> &tp, cx<T> *lds)
{
    TailView<T> c = tail_view(lds, tp.lv[tp.nt - 1]);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int n = tp.nc;
    for (int row = wave; row < n; row += nw) {
        const cd *ar = tp.aug + (size_t)row * 2 * n + n;
        double re = 0.0, im = 0.0;
        for (int k = lane; k < n; k += 64) {
            cd a = ar[k];
            int x, y;
            c.xy(k, x, y);
            cx<T> bk = c.b[c.at(x, y)];
            double br = (double)bk.re, bi = (double)bk.im;
            re += a.re * br - a.im * bi;
            im += a.re * bi + a.im * br;
        }
        for (int off = 32; off > 0; off >>= 1) {
            re += __shfl_down(re, off, 64);
            im += __shfl_down(im, off, 64);
        }
        if (lane == 0) {
            int x, y;
            c.xy(row, x, y);
            c.u[c.at(x, y)] = cx<T>{T(re), T(im)};
        }
    }
    __syncthreads();
}

// One V-cycle from tail level i0 (its b and u in LDS; zero_top: its u is
// taken as 0): pre-smoothing, residual and restriction down to the coarsest
// level (every coarser level from a zero guess), exact solve, then
// interpolation of the correction and post-smoothing back up to i0.
template <typename T>
__device__ __forceinline__ void tail_vcycle(const TailParams<T> &tp, cx<T> *lds, int i0, bool zero_top)
{
    const int nt = tp.nt;
    for (int i = i0; i + 1 < nt; ++i) {
        const TailLevel<T> &L = tp.lv[i];
        TailView<T> v = tail_view(lds, L);
        tail_smooth<T>(v, L, tp.nu1, zero_top || i > i0);
        for (int j = threadIdx.x; j < v.N; j += blockDim.x) {
            int x, y;
            v.xy(j, x, y);
            const int k = v.at(x, y);
            v.t[k] = resid_point<T>(L.P, v.u[k], v.u[k - 1], v.u[k + 1], v.u[k - v.W], v.u[k + v.W], v.b[k], v.q[k]);
        }
        __syncthreads();
        TailView<T> c = tail_view(lds, tp.lv[i + 1]);
        const T w[3] = {T(0.25), T(0.5), T(0.25)};
        for (int J = threadIdx.x; J < c.N; J += blockDim.x) {
            int I, K;
            c.xy(J, I, K);
            const int fk = v.at(2 * I + 1, 2 * K + 1);
            cx<T> acc = {T(0), T(0)};
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    T wgt = (w[dx + 1] * w[dy + 1]) * T(1);
                    acc = acc + wgt * v.t[fk + dy * v.W + dx];
                }
            c.b[c.at(I, K)] = acc;
        }
        __syncthreads();
    }
    tail_coarsest<T>(tp, lds);
    for (int i = nt - 2; i >= i0; --i) {
        const TailLevel<T> &L = tp.lv[i];
        TailView<T> v = tail_view(lds, L);
        TailView<T> c = tail_view(lds, tp.lv[i + 1]);
        const cx<T> *cu = c.u + c.W + 1;   // interior (0, 0) of the coarse correction, row stride c.W
        for (int j = threadIdx.x; j < v.N; j += blockDim.x) {
            int x, y;
            v.xy(j, x, y);
            const int k = v.at(x, y);
            v.u[k] = v.u[k] + interp2d<T>(cu, c.W, 0, 0, c.mx, c.my, x, y);
        }
        __syncthreads();
        tail_smooth<T>(v, L, tp.nu2, false);
    }
}

template <typename T>
__device__ __forceinline__ void tail_store(const TailParams<T> &tp, cx<T> *lds, int s0, cx<T> *__restrict__ u_top)
{
    TailView<T> v0 = tail_view(lds, tp.lv[s0]);
    for (int j = threadIdx.x; j < v0.N; j += blockDim.x) {
        int x, y;
        v0.xy(j, x, y);
        u_top[j] = v0.u[v0.at(x, y)];
    }
}

template <typename T>
__device__ __forceinline__ void tail2d_body(const TailParams<T> &tp, const cx<T> *__restrict__ b_top,
                                            cx<T> *__restrict__ u_top, cx<T> *lds)
{
    tail_load<T>(tp, b_top, lds, 0);
    tail_vcycle<T>(tp, lds, 0, true);
    tail_store<T>(tp, lds, 0, u_top);
}

// Full multigrid start on the tail levels s0 .. nt - 1 in one workgroup: b of
// level s0 from b_top, injected level by level down to the coarsest, exact
// solve there, then on each level up to s0 the interpolated coarser solution
// as the guess and k V-cycles; u_top receives level s0's solution.
template <typename T>
__device__ __forceinline__ void tail2d_fmg_body(const TailParams<T> &tp, const cx<T> *__restrict__ b_top,
                                                cx<T> *__restrict__ u_top, int s0, int k, cx<T> *lds)
{
    const int nt = tp.nt;
    tail_load<T>(tp, b_top, lds, s0);
    for (int i = s0; i + 1 < nt; ++i) {
        TailView<T> v = tail_view(lds, tp.lv[i]);
        TailView<T> c = tail_view(lds, tp.lv[i + 1]);
        for (int J = threadIdx.x; J < c.N; J += blockDim.x) {
            int I, K;
            c.xy(J, I, K);
            c.b[c.at(I, K)] = v.b[v.at(2 * I + 1, 2 * K + 1)];
        }
        __syncthreads();
    }
    tail_coarsest<T>(tp, lds);
    for (int i = nt - 2; i >= s0; --i) {
        TailView<T> v = tail_view(lds, tp.lv[i]);
        TailView<T> c = tail_view(lds, tp.lv[i + 1]);
        const cx<T> *cu = c.u + c.W + 1;
        for (int j = threadIdx.x; j < v.N; j += blockDim.x) {
            int x, y;
            v.xy(j, x, y);
            v.u[v.at(x, y)] = interp2d<T>(cu, c.W, 0, 0, c.mx, c.my, x, y);
        }
        __syncthreads();
        for (int c2 = 0; c2 < k; ++c2) tail_vcycle<T>(tp, lds, i, false);
    }
    tail_store<T>(tp, lds, s0, u_top);
}

template <typename T>
__global__ __launch_bounds__(1024) void k_tail2d_fmg(TailParams<T> tp, const cx<T> *__restrict__ b_top,
                                                     cx<T> *__restrict__ u_top, int s0, int k)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char tail_lds_f[];
    tail2d_fmg_body<T>(tp, b_top, u_top, s0, k, reinterpret_cast<cx<T> *>(tail_lds_f));
}

template <typename T>
__global__ __launch_bounds__(1024) void k_tail2d(TailParams<T> tp, const cx<T> *__restrict__ b_top,
                                                 cx<T> *__restrict__ u_top, const int *__restrict__ stop)
{
    if (stop && *stop) return;
    extern __shared__ __attribute__((aligned(16))) unsigned char tail_lds[];
    tail2d_body<T>(tp, b_top, u_top, reinterpret_cast<cx<T> *>(tail_lds));
}

// ---------------------------------------------------------------------------
static int tiles2d(const LevelGeom &g, int &tx)
{
    tx = (g.m[0] + FTX - 1) / FTX;
    return tx * ((g.m[1] + FTY - 1) / FTY);
}

int fused2d_blocks(const LevelGeom &g)
{
    int tx;
    return tiles2d(g, tx);
}

template <typename T, int TH>
static void launch_smooth2d_th(const LevelGeom &g, const Stencil<T> &P, int nsweeps, bool zero, const cx<T> *u,
                               const cx<T> *ec, const cx<T> *b, const cx<T> *q, cx<T> *out, hipStream_t s,
                               bool finest, const int *stop)
{
    const int tx = (g.m[0] + FTX - 1) / FTX;
    const int nb = tx * ((g.m[1] + TH - 1) / TH);
    dim3 G(nb), B(256);
#define SM(NS, Z, PR, TAG) \
    launch_maybe_timed((k_smooth2d<T, NS, Z, PR, TAG, TH>), G, B, 0, s, u, ec, b, q, out, P, tx, stop)
    const bool prol = (ec != nullptr);
    if (nsweeps == 2) {
        if (zero) {
            if (finest) SM(2, true, false, 1); else SM(2, true, false, 0);
        } else if (prol) {
            if (finest) SM(2, false, true, 1); else SM(2, false, true, 0);
        } else {
            if (finest) SM(2, false, false, 1); else SM(2, false, false, 0);
        }
    } else {
        if (zero) SM(1, true, false, 0);
        else if (prol) SM(1, false, true, 0);
        else SM(1, false, false, 0);
    }
#undef SM
}

template <typename T>
void launch_smooth2d(const LevelGeom &g, const Stencil<T> &P, int nsweeps, bool zero, const cx<T> *u,
                     const cx<T> *ec, const cx<T> *b, const cx<T> *q, cx<T> *out, hipStream_t s, bool finest,
                     const int *stop, int th)
{
    switch (th) {
    case 4: launch_smooth2d_th<T, 4>(g, P, nsweeps, zero, u, ec, b, q, out, s, finest, stop); break;
    case 16: launch_smooth2d_th<T, 16>(g, P, nsweeps, zero, u, ec, b, q, out, s, finest, stop); break;
    default: launch_smooth2d_th<T, 8>(g, P, nsweeps, zero, u, ec, b, q, out, s, finest, stop); break;
    }
}
template void launch_smooth2d<double>(const LevelGeom &, const Stencil<double> &, int, bool, const cd *, const cd *,
                                      const cd *, const cd *, cd *, hipStream_t, bool, const int *, int);
template void launch_smooth2d<float>(const LevelGeom &, const Stencil<float> &, int, bool, const cf *, const cf *,
                                     const cf *, const cf *, cf *, hipStream_t, bool, const int *, int);

template <typename T>
void launch_resid_restrict2d(const LevelGeom &g, const Stencil<T> &P, const cx<T> *u, const cx<T> *b,
                             const cx<T> *q, cx<T> *bc, hipStream_t s, const int *stop)
{
    int mxc = (g.m[0] - 1) / 2, myc = (g.m[1] - 1) / 2;
    int ctx = (mxc + RCX - 1) / RCX, cty = (myc + RCY - 1) / RCY;
    hipLaunchKernelGGL((k_resid_restrict2d<T>), dim3(ctx * cty), dim3(256), 0, s, u, b, q, bc, P, ctx, stop);
}
template void launch_resid_restrict2d<double>(const LevelGeom &, const Stencil<double> &, const cd *, const cd *,
                                              const cd *, cd *, hipStream_t, const int *);
template void launch_resid_restrict2d<float>(const LevelGeom &, const Stencil<float> &, const cf *, const cf *,
                                             const cf *, cf *, hipStream_t, const int *);

// Fine tile height of the fused pre-smoothing + residual + restriction pass:
// 8 or 16 rows (FP32 16 rows: 25 KB of LDS; FP64 8 rows: 31 KB).
template <typename T>
struct SmoothRR {
    static constexpr int FH = sizeof(T) == 4 ? 16 : 8;
};

template <typename T, int FH>
static void launch_smooth_rr2d_fh(const LevelGeom &g, const Stencil<T> &P, bool zero, const cx<T> *u, const cx<T> *b,
                                  const cx<T> *q, cx<T> *out, cx<T> *bc, hipStream_t s, bool finest, const int *stop)
{
    const int tx = (g.m[0] + FTX - 1) / FTX;
    const int nb = tx * ((g.m[1] + FH - 1) / FH);
#define FFMG_SRR(Z, TG) \
    launch_maybe_timed((k_smooth_rr2d<T, Z, TG, FH>), dim3(nb), dim3(256), 0, s, u, b, q, out, bc, P, tx, stop)
    if (zero) {
        if (finest) FFMG_SRR(true, 1);
        else FFMG_SRR(true, 0);
    } else {
        if (finest) FFMG_SRR(false, 1);
        else FFMG_SRR(false, 0);
    }
#undef FFMG_SRR
}

template <typename T>
void launch_smooth_rr2d(const LevelGeom &g, const Stencil<T> &P, bool zero, const cx<T> *u, const cx<T> *b,
                        const cx<T> *q, cx<T> *out, cx<T> *bc, hipStream_t s, bool finest, const int *stop, int fh)
{
    if (fh <= 0) fh = SmoothRR<T>::FH;
    if (fh == 16) launch_smooth_rr2d_fh<T, 16>(g, P, zero, u, b, q, out, bc, s, finest, stop);
    else launch_smooth_rr2d_fh<T, 8>(g, P, zero, u, b, q, out, bc, s, finest, stop);
}
template void launch_smooth_rr2d<double>(const LevelGeom &, const Stencil<double> &, bool, const cd *, const cd *,
                                         const cd *, cd *, cd *, hipStream_t, bool, const int *, int);
template void launch_smooth_rr2d<float>(const LevelGeom &, const Stencil<float> &, bool, const cf *, const cf *,
                                        const cf *, cf *, cf *, hipStream_t, bool, const int *, int);

void launch_refine2d(const LevelGeom &g, const Stencil<double> &P, const cd *u, const cf *d, const cd *b,
                     const cd *q, cd *u_out, cf *r32, const SolveCtl *ctl, double *partial, hipStream_t st,
                     const int *stop, const cd *pwf)
{
    int tx;
    int nb = tiles2d(g, tx);
    launch_maybe_timed(k_refine2d, dim3(nb), dim3(256), 0, st, u, d, b, q, u_out, r32, ctl, P, tx, partial, stop,
                       pwf);
}

template <typename T>
size_t tail2d_lds_bytes(const int *mx, const int *my, int nt)
{
    size_t n = 0;
    for (int i = 0; i < nt; ++i) n += 3 * (size_t)mx[i] * my[i];
    return n * sizeof(cx<T>);
}
template size_t tail2d_lds_bytes<double>(const int *, const int *, int);
template size_t tail2d_lds_bytes<float>(const int *, const int *, int);

template <typename T>
void launch_tail2d(const TailParams<T> &tp, size_t lds_bytes, const cx<T> *b_top, cx<T> *u_top, hipStream_t s,
                   const int *stop)
{
    // once per instantiation (a thread-safe static initialisation)
    static const bool attr_set = [] {
        (void)hipFuncSetAttribute((const void *)k_tail2d<T>, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        return true;
    }();
    (void)attr_set;
    hipLaunchKernelGGL((k_tail2d<T>), dim3(1), dim3(1024), lds_bytes, s, tp, b_top, u_top, stop);
}
template <typename T>
void launch_tail2d_fmg(const TailParams<T> &tp, size_t lds_bytes, const cx<T> *b_top, cx<T> *u_top, int s0, int k,
                       hipStream_t s)
{
    // once per instantiation (a thread-safe static initialisation)
    static const bool attr_set = [] {
        (void)hipFuncSetAttribute((const void *)k_tail2d_fmg<T>, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        return true;
    }();
    (void)attr_set;
    hipLaunchKernelGGL((k_tail2d_fmg<T>), dim3(1), dim3(1024), lds_bytes, s, tp, b_top, u_top, s0, k);
}
template void launch_tail2d_fmg<double>(const TailParams<double> &, size_t, const cd *, cd *, int, int, hipStream_t);
template void launch_tail2d_fmg<float>(const TailParams<float> &, size_t, const cf *, cf *, int, int, hipStream_t);
template void launch_tail2d<double>(const TailParams<double> &, size_t, const cd *, cd *, hipStream_t, const int *);
template void launch_tail2d<float>(const TailParams<float> &, size_t, const cf *, cf *, hipStream_t, const int *);

// ---------------------------------------------------------------------------
// Batched launches.  The flat block index is mapped XCD-contiguously onto the
// concatenated tiles of all jobs; within a job the tile and the slot of its
// partial sum are those of the single-instance launch (block b of that launch
// owns tile xcd_tile(b, n) and writes partial[b]), so the results, sums
// included, are bit for bit those of one launch per instance.
template <typename T, int NS, bool ZERO, bool PROL, int TH>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_smooth2d_batch(const SmoothJob<T> *__restrict__ jobs,
                                                        const int *__restrict__ tile_job)
{
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const SmoothJob<T> J = jobs[tile_job[t]];
    if (J.stop && *J.stop) return;
    smooth2d_body<T, NS, ZERO, PROL, TH>(J.u, J.ec, J.b, J.q, J.out, J.P, J.tiles_x, t - J.tile0);
}

template <typename T, bool ZERO, int TH>
__global__ __launch_bounds__(256) void k_smooth_rr2d_batch(const SRRJob<T> *__restrict__ jobs,
                                                           const int *__restrict__ tile_job)
{
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const SRRJob<T> J = jobs[tile_job[t]];
    if (J.stop && *J.stop) return;
    smooth_rr2d_body<T, ZERO, TH>(J.u, J.b, J.q, J.out, J.bc, J.P, J.tiles_x, t - J.tile0);
}

template <typename T>
__global__ __launch_bounds__(256) void k_resid_restrict2d_batch(const RRJob<T> *__restrict__ jobs,
                                                                const int *__restrict__ tile_job)
{
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const RRJob<T> J = jobs[tile_job[t]];
    if (J.stop && *J.stop) return;
    resid_restrict2d_body<T>(J.u, J.b, J.q, J.bc, J.P, J.ctiles_x, t - J.tile0);
}

__global__ __launch_bounds__(256) void k_refine2d_batch(const RefineJob *__restrict__ jobs,
                                                        const int *__restrict__ tile_job)
{
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const RefineJob J = jobs[tile_job[t]];
    if (J.stop && *J.stop) return;
    const int tile = t - J.tile0;
    refine2d_body(J.u, J.d, J.b, J.q, J.u_out, J.r32, J.ctl, J.P, J.tiles_x, tile,
                  J.partial + xcd_tile_inv(tile, J.ntiles), J.f);
}

template <typename T>
__global__ __launch_bounds__(1024) void k_tail2d_batch(const TailJob<T> *__restrict__ jobs)
{
    const TailJob<T> &J = jobs[blockIdx.x];
    if (J.stop && *J.stop) return;
    extern __shared__ __attribute__((aligned(16))) unsigned char tail_lds_b[];
    tail2d_body<T>(J.tp, J.b_top, J.u_top, reinterpret_cast<cx<T> *>(tail_lds_b));
}

// The full multigrid start of every tail in one launch (one workgroup per
// job, from the first tail level).
template <typename T>
__global__ __launch_bounds__(1024) void k_tail2d_fmg_batch(const TailJob<T> *__restrict__ jobs, int k)
{
    const TailJob<T> &J = jobs[blockIdx.x];
    if (J.stop && *J.stop) return;
    extern __shared__ __attribute__((aligned(16))) unsigned char tail_lds_fb[];
    tail2d_fmg_body<T>(J.tp, J.b_top, J.u_top, 0, k, reinterpret_cast<cx<T> *>(tail_lds_fb));
}

void batch_tiles(int variant, int *th_smooth, int *th_srr)
{
    const int v = (variant >= 0 && variant < BATCH_VARIANTS) ? variant : 0;
    *th_smooth = BATCH_TILES[v][0];
    *th_srr = BATCH_TILES[v][1];
}

template <typename T>
int smooth2d_tiles(const LevelGeom &g, int *tiles_x, int th)
{
    *tiles_x = (g.m[0] + FTX - 1) / FTX;
    return *tiles_x * ((g.m[1] + th - 1) / th);
}
template int smooth2d_tiles<double>(const LevelGeom &, int *, int);
template int smooth2d_tiles<float>(const LevelGeom &, int *, int);

template <typename T>
int smooth_rr2d_tiles(const LevelGeom &g, int *tiles_x, int th)
{
    *tiles_x = (g.m[0] + FTX - 1) / FTX;
    return *tiles_x * ((g.m[1] + th - 1) / th);
}
template int smooth_rr2d_tiles<double>(const LevelGeom &, int *, int);
template int smooth_rr2d_tiles<float>(const LevelGeom &, int *, int);

int resid_restrict2d_tiles(const LevelGeom &g, int *ctiles_x)
{
    int mxc = (g.m[0] - 1) / 2, myc = (g.m[1] - 1) / 2;
    *ctiles_x = (mxc + RCX - 1) / RCX;
    return *ctiles_x * ((myc + RCY - 1) / RCY);
}

int refine2d_tiles(const LevelGeom &g, int *tiles_x) { return tiles2d(g, *tiles_x); }

template <typename T, int TH>
static void launch_smooth2d_batch_th(int nsweeps, bool zero, bool prol, const SmoothJob<T> *jobs, const int *tile_job,
                                     int ntiles, hipStream_t s)
{
    dim3 G(ntiles), B(256);
#define SMB(NS, Z, PR) hipLaunchKernelGGL((k_smooth2d_batch<T, NS, Z, PR, TH>), G, B, 0, s, jobs, tile_job)
    if (nsweeps == 2) {
        if (zero) SMB(2, true, false);
        else if (prol) SMB(2, false, true);
        else SMB(2, false, false);
    } else {
        if (zero) SMB(1, true, false);
        else if (prol) SMB(1, false, true);
        else SMB(1, false, false);
    }
#undef SMB
}

template <typename T>
void launch_smooth2d_batch(int nsweeps, bool zero, bool prol, const SmoothJob<T> *jobs, const int *tile_job,
                           int ntiles, hipStream_t s, int th)
{
    if (ntiles <= 0) return;
    if (th == 4) launch_smooth2d_batch_th<T, 4>(nsweeps, zero, prol, jobs, tile_job, ntiles, s);
    else if (th == 16) launch_smooth2d_batch_th<T, 16>(nsweeps, zero, prol, jobs, tile_job, ntiles, s);
    else launch_smooth2d_batch_th<T, 8>(nsweeps, zero, prol, jobs, tile_job, ntiles, s);
}
template void launch_smooth2d_batch<float>(int, bool, bool, const SmoothJob<float> *, const int *, int, hipStream_t,
                                           int);
template void launch_smooth2d_batch<double>(int, bool, bool, const SmoothJob<double> *, const int *, int,
                                            hipStream_t, int);

template <typename T>
void launch_smooth_rr2d_batch(bool zero, const SRRJob<T> *jobs, const int *tile_job, int ntiles, hipStream_t s, int th)
{
    if (ntiles <= 0) return;
#define SRB(Z, TH) hipLaunchKernelGGL((k_smooth_rr2d_batch<T, Z, TH>), dim3(ntiles), dim3(256), 0, s, jobs, tile_job)
    if (th == 8) {
        if (zero) SRB(true, 8);
        else SRB(false, 8);
    } else {
        if (zero) SRB(true, 16);
        else SRB(false, 16);
    }
#undef SRB
}
template void launch_smooth_rr2d_batch<float>(bool, const SRRJob<float> *, const int *, int, hipStream_t, int);
template void launch_smooth_rr2d_batch<double>(bool, const SRRJob<double> *, const int *, int, hipStream_t, int);

template <typename T>
void launch_resid_restrict2d_batch(const RRJob<T> *jobs, const int *tile_job, int ntiles, hipStream_t s)
{
    if (ntiles <= 0) return;
    hipLaunchKernelGGL((k_resid_restrict2d_batch<T>), dim3(ntiles), dim3(256), 0, s, jobs, tile_job);
}
template void launch_resid_restrict2d_batch<float>(const RRJob<float> *, const int *, int, hipStream_t);
template void launch_resid_restrict2d_batch<double>(const RRJob<double> *, const int *, int, hipStream_t);

void launch_refine2d_batch(const RefineJob *jobs, const int *tile_job, int ntiles, hipStream_t s)
{
    if (ntiles <= 0) return;
    hipLaunchKernelGGL(k_refine2d_batch, dim3(ntiles), dim3(256), 0, s, jobs, tile_job);
}

template <typename T>
void launch_tail2d_batch(const TailJob<T> *jobs, int njobs, size_t lds_bytes, hipStream_t s)
{
    // once per instantiation (a thread-safe static initialisation)
    static const bool attr_set = [] {
        (void)hipFuncSetAttribute((const void *)k_tail2d_batch<T>, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        return true;
    }();
    (void)attr_set;
    if (njobs <= 0) return;
    hipLaunchKernelGGL((k_tail2d_batch<T>), dim3(njobs), dim3(1024), lds_bytes, s, jobs);
}
template <typename T>
void launch_tail2d_fmg_batch(const TailJob<T> *jobs, int njobs, int k, size_t lds_bytes, hipStream_t s)
{
    // once per instantiation (a thread-safe static initialisation)
    static const bool attr_set = [] {
        (void)hipFuncSetAttribute((const void *)k_tail2d_fmg_batch<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  160 * 1024);
        return true;
    }();
    (void)attr_set;
    if (njobs <= 0) return;
    hipLaunchKernelGGL((k_tail2d_fmg_batch<T>), dim3(njobs), dim3(1024), lds_bytes, s, jobs, k);
}
template void launch_tail2d_fmg_batch<float>(const TailJob<float> *, int, int, size_t, hipStream_t);
template void launch_tail2d_batch<float>(const TailJob<float> *, int, size_t, hipStream_t);
template void launch_tail2d_batch<double>(const TailJob<double> *, int, size_t, hipStream_t);

}  // namespace ffmg
