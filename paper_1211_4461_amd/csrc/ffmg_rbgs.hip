// ffmg_rbgs.hip -- red-black Gauss-Seidel smoothing sweeps (Sec. 3.3 names
// Gauss-Seidel beside weighted Jacobi as the standard relaxation of the
// V-cycle).  A sweep relaxes the "red" points (0-based interior indices
// ix + iy + iz even) and then the black ones, u_j <- u_j + (b_j - (A u)_j) /
// D_j, each with the values of the other colour it reads already final: in
// the 5/7-point stencil a point's neighbours all have the other colour, so a
// half sweep is one launch of independent point updates, in place.
#include "ffmg_internal.hpp"
#include "ffmg_point.hpp"

namespace ffmg {

namespace {

// One half sweep: thread t owns the t-th point of colour `color`
// (ix = 2 k + ((iy + iz + color) & 1) in row (iy, iz)).
template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_rbgs_half(cx<T> *__restrict__ u, const cx<T> *__restrict__ b,
                                                   const cx<T> *__restrict__ q, Stencil<T> P, int color, int half_x,
                                                   const int *__restrict__ stop)
{
    if (stop && *stop) return;
    const size_t t = (size_t)blockIdx.x * 256 + threadIdx.x;
    const int mx = P.mx, my = P.my, mz = P.mz;
    const size_t rows = (size_t)my * mz;
    if (t >= (size_t)half_x * rows) return;
    int k, iy, iz;
    split3(t, half_x, my, k, iy, iz);   // 32-bit divisions where t fits
    const int ix = 2 * k + ((iy + iz + color) & 1);
    if (ix >= mx) return;
    const size_t j = ((size_t)iz * my + iy) * mx + ix;
    const size_t sy = (size_t)mx, sz = (size_t)mx * my;
    const cx<T> zero = {T(0), T(0)};
    const cx<T> uc = u[j];
    cx<T> w = ix > 0 ? u[j - 1] : zero, e = ix < mx - 1 ? u[j + 1] : zero;
    cx<T> s = iy > 0 ? u[j - sy] : zero, n = iy < my - 1 ? u[j + sy] : zero;
    cx<T> L = lap_xy(P, uc, w, e, s, n);
    if (DIM == 3) {
        cx<T> d = iz > 0 ? u[j - sz] : zero, up = iz < mz - 1 ? u[j + sz] : zero;
        L = lap_add_z(P, L, uc, d, up);
    }
    const cx<T> qj = q[j];
    const cx<T> r = resid_from(P, L, uc, b[j], qj);
    const cx<T> D = {P.csum2.re - (P.k02 + qj.re), P.csum2.im - qj.im};
    const cx<T> c = cmul(r, crecip(D));
    u[j] = cx<T>{uc.re + c.re, uc.im + c.im};
}

}  // namespace

template <typename T>
void launch_rbgs_sweep(const LevelGeom &g, const Stencil<T> &P, const cx<T> *b, const cx<T> *q, cx<T> *u,
                       hipStream_t s, const int *stop)
{
    const int half_x = (g.m[0] + 1) / 2;
    const size_t n = (size_t)half_x * g.m[1] * (g.dim == 3 ? g.m[2] : 1);
    const unsigned nb = (unsigned)((n + 255) / 256);
    for (int color = 0; color < 2; ++color) {
        if (g.dim == 3)
            hipLaunchKernelGGL((k_rbgs_half<T, 3>), dim3(nb), dim3(256), 0, s, u, b, q, P, color, half_x, stop);
        else
            hipLaunchKernelGGL((k_rbgs_half<T, 2>), dim3(nb), dim3(256), 0, s, u, b, q, P, color, half_x, stop);
    }
}
template void launch_rbgs_sweep<double>(const LevelGeom &, const Stencil<double> &, const cd *, const cd *, cd *,
                                        hipStream_t, const int *);
template void launch_rbgs_sweep<float>(const LevelGeom &, const Stencil<float> &, const cf *, const cf *, cf *,
                                       hipStream_t, const int *);

}  // namespace ffmg
