// ffmg_ion.hip -- ionisation observables of the 2D radial partial-wave
// Schroedinger model (Sec. 5.1-5.4):
//
//   source right-hand side   b = 2 phi            (Sec. 5 introduction)
//   bound state              eq. boundstate, on one contour axis
//   test functions           eq. testfunction, regular solutions with free
//                            amplitude 1/sqrt(k)
//   amplitudes               eq. single-ionization / eq. double-ionization,
//                            a_m = h~x h~y sum tx[m][x] ty[m][y] (phi - V12 u),
//                            and the optical-theorem product <phi, u>
//   cross sections           half the outgoing flux per kind of channel
//
// The amplitudes are the far field's separable contraction with the
// test-function tables in place of the plane-wave factors: the integrand is
// one elementwise pass, the y contraction runs on the FP64 MFMA GEMM of the
// far field, and the x contraction is one block per amplitude.  The 1D parts
// (bound state, test functions) are three-term recurrences and tridiagonal
// solves along one axis, inherently sequential and tiny (one thread per
// function).
#include <math.h>

#include <algorithm>

#include "ffmg_handle.hpp"

using namespace ffmg;

namespace {

constexpr double V_NEGLIGIBLE = 1e-13;   // |V| below this counts as zero for the normalisation point
constexpr int BOUND_MAX_IT = 60;

__device__ __forceinline__ cd csqrt_pos(cd z)
{
    // principal square root, then the root with non-negative real part
    double r = sqrt(z.re * z.re + z.im * z.im);
    double re = sqrt(0.5 * (r + z.re));
    double im = copysign(sqrt(0.5 * (r - z.re)), z.im);
    return cd{re, im};
}

// b = s src
__global__ __launch_bounds__(256) void k_rhs_source(const cd *__restrict__ src, double s, size_t N, cd *__restrict__ b)
{
    for (size_t j = (size_t)blockIdx.x * 256 + threadIdx.x; j < N; j += (size_t)gridDim.x * 256) b[j] = s * src[j];
}

// eq. boundstate: inverse iteration (three steps at the given shift, then
// Rayleigh-quotient shifts) on the rotated 1D Hamiltonian
//   H = -1/2 e^{-2i gamma} D2 / h^2 + diag(V(z_i)),
// complex symmetric tridiagonal: diagonal c + V_i, off-diagonal -c/2 with
// c = 1/h~^2.  Each step is one tridiagonal solve (elimination without
// pivoting) and a 2-norm scaling; the eigenvalue estimate is the
// non-conjugated Rayleigh quotient x^T H x / x^T x of a complex symmetric
// matrix.  Converged one step after ||H x - lambda x|| <= tol ||x||.  One
// thread.
// out: [0, 1] lambda, [2] residual, [3] iterations, [4] status (0 ok,
// 1 not converged, 2 zero pivot).
__global__ void k_bound_state(const cd *__restrict__ v, int m, cd c, cd ht, double shift, double tol, cd *__restrict__ x,
                              cd *__restrict__ y, cd *__restrict__ dp, cd *__restrict__ phi, double *__restrict__ out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const cd off = cd{-0.5 * c.re, -0.5 * c.im};
    for (int i = 0; i < m; ++i) x[i] = cd{1.0, 0.0};
    cd sigma = cd{shift, 0.0}, lam = sigma;
    double res = INFINITY;
    int status = 1, it = 0;
    bool close = false;
    for (; it < BOUND_MAX_IT; ++it) {
        bool zero = false;
        cd d = c + v[0] - sigma;
        if (abs2(d) == 0.0) zero = true;
        dp[0] = d;
        y[0] = x[0];
        for (int i = 1; i < m && !zero; ++i) {
            cd l = off * recip(dp[i - 1]);
            cd di = (c + v[i] - sigma) - l * off;
            if (abs2(di) == 0.0) zero = true;
            dp[i] = di;
            y[i] = x[i] - l * y[i - 1];
        }
        if (zero) {
            status = 2;
            break;
        }
        y[m - 1] = y[m - 1] * recip(dp[m - 1]);
        for (int i = m - 2; i >= 0; --i) y[i] = (y[i] - off * y[i + 1]) * recip(dp[i]);
        double nn = 0.0;
        for (int i = 0; i < m; ++i) nn += abs2(y[i]);
        const double sc = 1.0 / sqrt(nn);
        for (int i = 0; i < m; ++i) x[i] = sc * y[i];
        cd num = cd{0.0, 0.0}, den = cd{0.0, 0.0};
        for (int i = 0; i < m; ++i) {
            cd hx = (c + v[i]) * x[i];
            if (i > 0) hx = hx + off * x[i - 1];
            if (i + 1 < m) hx = hx + off * x[i + 1];
            y[i] = hx;   // H x, kept for the residual
            num = num + x[i] * hx;
            den = den + x[i] * x[i];
        }
        lam = num * recip(den);
        double rr = 0.0;
        for (int i = 0; i < m; ++i) rr += abs2(y[i] - lam * x[i]);
        res = sqrt(rr);
        if (res <= tol) {
            // one more Rayleigh step takes the vector to the rounding level
            if (close) {
                status = 0;
                ++it;
                break;
            }
            close = true;
        }
        if (it >= 2) sigma = lam;
    }
    // normalise: sum phi^2 h~ = 1, Re phi_1 > 0
    cd s = cd{0.0, 0.0};
    for (int i = 0; i < m; ++i) s = s + x[i] * x[i];
    s = s * ht;
    cd inv = recip(csqrt_pos(s));
    if ((inv * x[0]).re < 0.0) inv = cd{-inv.re, -inv.im};
    for (int i = 0; i < m; ++i) phi[i] = inv * x[i];
    out[0] = lam.re;
    out[1] = lam.im;
    out[2] = res;
    out[3] = (double)it;
    out[4] = (double)status;
}

// Index of the first node past the last one with |V| > V_NEGLIGIBLE (0 if
// none); one block.
__global__ __launch_bounds__(256) void k_ref_index(const cd *__restrict__ v, int m, int *__restrict__ out)
{
    __shared__ int red[256];
    int best = -1;
    for (int i = threadIdx.x; i < m; i += 256)
        if (abs2(v[i]) > V_NEGLIGIBLE * V_NEGLIGIBLE) best = max(best, i);
    red[threadIdx.x] = best;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] = max(red[threadIdx.x], red[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0] + 1;
}

// eq. testfunction: one thread per wavenumber.  The regular solution from
// p_0 = 0 (the Dirichlet node), p_1 = 1 by the recurrence of the rotated
// stencil, p_{i+1} = 2 p_i - p_{i-1} + h~^2 (2 V_i - k^2) p_i, then scaled by
// 1/(A sqrt k), where A^2 = (p_r^2 + p_{r+1}^2 - 2 c p_r p_{r+1}) / (1 - c^2),
// c = 1 - h~^2 k^2 / 2, is the squared free-wave amplitude at the reference
// node r (the invariant of the free recurrence), A with Re A > 0.
__global__ __launch_bounds__(64) void k_test_functions(const cd *__restrict__ v, int m, cd ht2,
                                                       const double *__restrict__ kk, int M,
                                                       const int *__restrict__ ref, cd *__restrict__ out)
{
    const int t = blockIdx.x * 64 + threadIdx.x;
    if (t >= M) return;
    const double k = kk[t];
    cd *p = out + (size_t)t * m;
    const cd k2 = cd{k * k, 0.0};
    cd prev = cd{0.0, 0.0}, cur = cd{1.0, 0.0};
    p[0] = cur;
    for (int i = 0; i + 1 < m; ++i) {
        cd g = ht2 * (2.0 * v[i] - k2);
        cd nxt = (2.0 * cur - prev) + g * cur;
        p[i + 1] = nxt;
        prev = cur;
        cur = nxt;
    }
    const int r = ref[0];
    const cd c = cd{1.0, 0.0} - 0.5 * (ht2 * k2);
    const cd pr = p[r], pn = p[r + 1];
    const cd num = (pr * pr + pn * pn) - 2.0 * (c * (pr * pn));
    const cd a2 = num * recip(cd{1.0, 0.0} - c * c);
    const cd A = csqrt_pos(a2);
    const cd sc = recip(sqrt(k) * A);
    for (int i = 0; i < m; ++i) p[i] = sc * p[i];
}

// rho = phi - V12 u (the contraction operand, x fastest), and per-block
// partial sums of phi u (the optical-theorem product), re / im.
__global__ __launch_bounds__(256) void k_ion_integrand(const cd *__restrict__ src, const cd *__restrict__ v12,
                                                       const cd *__restrict__ u, size_t N, cd *__restrict__ rho,
                                                       double *__restrict__ parts)
{
    __shared__ double red[2][4];
    double sr = 0.0, si = 0.0;
    for (size_t j = (size_t)blockIdx.x * 256 + threadIdx.x; j < N; j += (size_t)gridDim.x * 256) {
        const cd s = src[j], uj = u[j];
        rho[j] = s - v12[j] * uj;
        const cd p = s * uj;
        sr += p.re;
        si += p.im;
    }
    for (int o = 32; o > 0; o >>= 1) {
        sr += __shfl_down(sr, o, 64);
        si += __shfl_down(si, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = sr;
        red[1][threadIdx.x >> 6] = si;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        parts[2 * blockIdx.x] = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
        parts[2 * blockIdx.x + 1] = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
    }
}

// out = pre sum_b parts[b] in a fixed order (one block).
__global__ __launch_bounds__(256) void k_sum_parts(const double *__restrict__ parts, int nb, cd pre, cd *__restrict__ out)
{
    __shared__ double red[2][256];
    double sr = 0.0, si = 0.0;
    for (int b = threadIdx.x; b < nb; b += 256) {
        sr += parts[2 * b];
        si += parts[2 * b + 1];
    }
    red[0][threadIdx.x] = sr;
    red[1][threadIdx.x] = si;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            red[0][threadIdx.x] += red[0][threadIdx.x + o];
            red[1][threadIdx.x] += red[1][threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = pre * cd{red[0][0], red[1][0]};
}

// A workspace slot of at least `bytes` (grown on demand, kept on the handle).
ffmg_status ion_ws(ffmg_handle *h, int slot, size_t bytes, void **p)
{
    bytes = std::max<size_t>(bytes, 256);
    if (h->ion_cap[slot] < bytes) {
        if (h->ion_buf[slot]) {
            HIPCHK(h, hipStreamSynchronize(h->stream));
            (void)hipFree(h->ion_buf[slot]);
            h->ion_buf[slot] = nullptr;
            h->ion_cap[slot] = 0;
        }
        void *v = nullptr;
        hipError_t e = hipMalloc(&v, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(h, FFMG_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
        }
        h->ion_buf[slot] = v;
        h->ion_cap[slot] = bytes;
    }
    *p = h->ion_buf[slot];
    return FFMG_OK;
}

ffmg_status axis_args(ffmg_handle *h, int axis, int *m, double *hk)
{
    if (axis < 0 || axis >= h->prob.dim) return fail(h, FFMG_EINVAL, "axis %d out of range", axis);
    const LevelGeom &g = h->L[0].g;
    *m = g.m[axis];
    *hk = g.h[axis];
    return FFMG_OK;
}

unsigned blocks_for(size_t N) { return (unsigned)std::max<size_t>(1, std::min<size_t>(1024, (N + 255) / 256)); }

}  // namespace

extern "C" {

ffmg_status mg_rhs_source(ffmg_handle *h, const void *src, void *b)
{
    NOT_PENDING(h);
    if (!h || !src || !b) return fail(h, FFMG_EINVAL, "null argument");
    const size_t N = h->L[0].g.N();
    const double s = (h->prob.kind == FFMG_SCHRODINGER) ? 2.0 : 1.0;
    hipLaunchKernelGGL(k_rhs_source, dim3(blocks_for(N)), dim3(256), 0, h->stream, (const cd *)src, s, N, (cd *)b);
    HIPCHK(h, hipGetLastError());
    return FFMG_OK;
}

ffmg_status ion_bound_state(ffmg_handle *h, int axis, const void *v, double shift, double lambda[2], void *phi)
{
    NOT_PENDING(h);
    if (!h || !v || !lambda || !phi || !isfinite(shift)) return fail(h, FFMG_EINVAL, "null argument or bad shift");
    int m;
    double hk;
    TRY(axis_args(h, axis, &m, &hk));
    if (m < 2) return fail(h, FFMG_EINVAL, "axis %d has fewer than 2 nodes", axis);
    void *ws;
    TRY(ion_ws(h, 4, (size_t)3 * m * sizeof(cd) + 256, &ws));
    cd *x = (cd *)ws, *y = x + m, *dp = y + m;
    double *dout = (double *)(dp + m);
    const double g = h->prob.gamma;
    const cd ht = cd{hk * cos(g), hk * sin(g)};
    const cd c = recip(ht * ht);
    // residual target relative to ||H|| ~ 2|c|; the step after it reaches the
    // rounding level
    const double tol = 1e-10 * (2.0 * sqrt(abs2(c)) + 1.0);
    hipLaunchKernelGGL(k_bound_state, dim3(1), dim3(64), 0, h->stream, (const cd *)v, m, c, ht, shift, tol, x, y, dp,
                       (cd *)phi, dout);
    HIPCHK(h, hipGetLastError());
    double o[5];
    HIPCHK(h, hipMemcpyAsync(o, dout, sizeof(o), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    lambda[0] = o[0];
    lambda[1] = o[1];
    if (o[4] == 2.0) return fail(h, FFMG_ENOCONV, "bound state: zero pivot at the shift");
    if (o[4] != 0.0 || !isfinite(o[0]) || !isfinite(o[1]))
        return fail(h, FFMG_ENOCONV, "bound state: residual %.3g after %d iterations", o[2], (int)o[3]);
    return FFMG_OK;
}

ffmg_status ion_wavenumbers(double energy, const double lambda[2], int M, double *kn, double *k1, double *k2,
                            double *w)
{
    if (!lambda || !kn || M < 0 || (M > 0 && (!k1 || !k2 || !w)) || !isfinite(energy)) return FFMG_EINVAL;
    *kn = (energy > lambda[0]) ? sqrt(2.0 * (energy - lambda[0])) : 0.0;
    for (int i = 0; i < M; ++i) {
        if (energy > 0.0) {
            const double eps = ((double)i + 0.5) * (energy / (double)M);
            k1[i] = sqrt(2.0 * eps);
            k2[i] = sqrt(2.0 * (energy - eps));
            w[i] = energy / (double)M;
        } else {
            k1[i] = k2[i] = w[i] = 0.0;
        }
    }
    return FFMG_OK;
}

ffmg_status ion_test_functions(ffmg_handle *h, int axis, const void *v, int M, const double *k, void *out)
{
    NOT_PENDING(h);
    if (!h || !v || !k || !out || M < 1) return fail(h, FFMG_EINVAL, "null argument or M < 1");
    for (int i = 0; i < M; ++i)
        if (!(k[i] > 0.0) || !isfinite(k[i])) return fail(h, FFMG_EINVAL, "wavenumber %d must be positive", i);
    int m;
    double hk;
    TRY(axis_args(h, axis, &m, &hk));
    void *ws;
    TRY(ion_ws(h, 5, (size_t)M * sizeof(double) + 256, &ws));
    int *dref = (int *)ws;
    double *dk = (double *)((char *)ws + 256);
    HIPCHK(h, hipMemcpyAsync(dk, k, (size_t)M * sizeof(double), hipMemcpyHostToDevice, h->stream));
    hipLaunchKernelGGL(k_ref_index, dim3(1), dim3(256), 0, h->stream, (const cd *)v, m, dref);
    int r = 0;
    HIPCHK(h, hipMemcpyAsync(&r, dref, sizeof(int), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    if (r + 1 >= m) return fail(h, FFMG_EINVAL, "the potential does not fall below %g inside the box", V_NEGLIGIBLE);
    const double g = h->prob.gamma;
    const cd ht = cd{hk * cos(g), hk * sin(g)};
    hipLaunchKernelGGL(k_test_functions, dim3((M + 63) / 64), dim3(64), 0, h->stream, (const cd *)v, m, ht * ht,
                       (const double *)dk, M, (const int *)dref, (cd *)out);
    HIPCHK(h, hipGetLastError());
    HIPCHK(h, hipStreamSynchronize(h->stream));   // k is the caller's host array
    return FFMG_OK;
}

ffmg_status ion_amplitudes(ffmg_handle *h, const void *src, const void *v12, const void *u, int M, const void *tx,
                           const void *ty, double *amp, double opt[2])
{
    NOT_PENDING(h);
    if (!h || !src || !v12 || !u || !tx || !ty || !amp || !opt || M < 1)
        return fail(h, FFMG_EINVAL, "null argument or M < 1");
    if (h->prob.dim != 2) return fail(h, FFMG_EINVAL, "the ionisation amplitudes are defined in 2D");
    const LevelGeom &g = h->L[0].g;
    const int mx = g.m[0], my = g.m[1];
    const size_t N = g.N();
    const unsigned nb = blocks_for(N);
    void *w_rho, *w_c, *w_g, *w_f;
    TRY(ion_ws(h, 0, N * sizeof(cd), &w_rho));
    TRY(ion_ws(h, 1, (size_t)M * mx * sizeof(cd), &w_c));
    TRY(ion_ws(h, 2, table_gemm_ws_bytes(M, my), &w_g));
    TRY(ion_ws(h, 3, (size_t)(M + 1) * sizeof(cd) + (size_t)2 * nb * sizeof(double), &w_f));
    cd *F = (cd *)w_f;
    double *parts = (double *)(F + M + 1);
    const double gm = h->prob.gamma;
    const double hh = g.h[0] * g.h[1];
    const cd pre = cd{hh * cos(2.0 * gm), hh * sin(2.0 * gm)};
    hipLaunchKernelGGL(k_ion_integrand, dim3(nb), dim3(256), 0, h->stream, (const cd *)src, (const cd *)v12,
                       (const cd *)u, N, (cd *)w_rho, parts);
    // C[m][x] = sum_y ty[m][y] rho[y][x]; a_m = pre sum_x tx[m][x] C[m][x]
    table_gemm_f64((const cd *)ty, M, my, (const cd *)w_rho, mx, (cd *)w_c, w_g, h->stream);
    launch_rows_dot((const cd *)tx, (const cd *)w_c, M, mx, pre, F, h->stream);
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, h->stream, (const double *)parts, (int)nb, pre, F + M);
    HIPCHK(h, hipGetLastError());
    HIPCHK(h, hipMemcpyAsync(amp, F, (size_t)M * sizeof(cd), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipMemcpyAsync(opt, F + M, sizeof(cd), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return FFMG_OK;
}

ffmg_status ion_cross_sections(int open_single, const double s0[2], int M, const double *f, const double *w,
                               const double opt[2], double sigma[3])
{
    if (!sigma || !opt || M < 0 || (open_single && !s0) || (M > 0 && (!f || !w))) return FFMG_EINVAL;
    sigma[0] = open_single ? 4.0 * (s0[0] * s0[0] + s0[1] * s0[1]) : 0.0;
    double d = 0.0;
    for (int i = 0; i < M; ++i) d += w[i] * (f[2 * i] * f[2 * i] + f[2 * i + 1] * f[2 * i + 1]);
    sigma[1] = (4.0 / M_PI) * d;
    sigma[2] = opt[1];
    return FFMG_OK;
}

}  // extern "C"
