// ffmg_capi.hip -- the multigrid driver and the C ABI declared in
// include/ffmg.h.  Every arithmetic step runs in the library's HIP kernels.
// The host sequences launches; the stopping test (Sec. 4: V-cycles to a
// residual-reduction tolerance) runs on the device in k_ctl_update, so the
// host enqueues several cycles at a time and reads the control block back
// once per batch instead of once per cycle.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <atomic>

#include "ffmg_handle.hpp"
#include "ffmg_learned.hpp"

using namespace ffmg;

namespace ffmg {

thread_local KernelTiming tl_kernel_timing;

// An event pair for kernel k, or -1 when k is not being timed.
static int prof_acquire(ffmg_handle *h, int k)
{
    if (!(h->profile_mask & (1 << k))) return -1;
    std::pair<hipEvent_t, hipEvent_t> e;
    if (!h->ev_free.empty()) {
        e = h->ev_free.back();
        h->ev_free.pop_back();
    } else {
        if (hipEventCreate(&e.first) != hipSuccess || hipEventCreate(&e.second) != hipSuccess) return -1;
    }
    h->ev[k].push_back(e);
    return (int)h->ev[k].size() - 1;
}

// A region of the stream (any number of launches): events recorded on the
// stream before and after it.
int prof_begin(ffmg_handle *h, int k)
{
    const int idx = prof_acquire(h, k);
    if (idx >= 0) (void)hipEventRecord(h->ev[k][idx].first, h->stream);
    return idx;
}

void prof_end(ffmg_handle *h, int k, int idx)
{
    if (idx < 0) return;
    (void)hipEventRecord(h->ev[k][idx].second, h->stream);
}

// Exactly one launch made through launch_maybe_timed: the runtime stamps the
// events at that kernel's own start and end.
int prof_kernel_begin(ffmg_handle *h, int k)
{
    const int idx = prof_acquire(h, k);
    if (idx >= 0) tl_kernel_timing = KernelTiming{h->ev[k][idx].first, h->ev[k][idx].second, false};
    return idx;
}

void prof_kernel_end(ffmg_handle *h, int k, int idx)
{
    if (idx < 0) return;
    if (!tl_kernel_timing.used) {   // nothing was launched: an empty interval
        (void)hipEventRecord(h->ev[k][idx].first, h->stream);
        (void)hipEventRecord(h->ev[k][idx].second, h->stream);
    }
    tl_kernel_timing = KernelTiming{};
}

ffmg_status fail(ffmg_handle *h, ffmg_status s, const char *fmt, ...)
{
    if (h) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        h->err = buf;
    }
    return s;
}

// log of the largest magnitude of exp(+-i k0 e^{i gamma} a.x) over the box
// for unit a: k0 sin(gamma) |x|_max.
double exponent_budget(const ffmg_handle *h)
{
    double r2 = 0.0;
    for (int k = 0; k < h->prob.dim; ++k) {
        double m = std::max(fabs(h->prob.lo[k]), fabs(h->prob.hi[k]));
        r2 += m * m;
    }
    return h->k0 * sin(h->prob.gamma) * sqrt(r2);
}

// Smoothing sweeps on level l: nu1 / nu2 on the finest level, nu_coarse
// (when set) on the coarser ones.
int nu_pre(const ffmg_handle *h, int l) { return (l > 0 && h->opt.nu_coarse > 0) ? h->opt.nu_coarse : h->opt.nu1; }
int nu_post(const ffmg_handle *h, int l) { return (l > 0 && h->opt.nu_coarse > 0) ? h->opt.nu_coarse : h->opt.nu2; }

}  // namespace ffmg

namespace {

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

// Sum of the first n partials -> host double (synchronises the stream).
ffmg_status reduce_to_host(ffmg_handle *h, int n, double *out)
{
    launch_sum(h->d_parts, n, h->d_scalar, h->stream);
    HIPCHK(h, hipMemcpyAsync(h->h_scalar, h->d_scalar, sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    *out = *h->h_scalar;
    return FFMG_OK;
}

constexpr int NORM_BATCH = 8;   // loads in flight per thread in the norm kernels (measured: 502 against 586 us at 511^3)

__global__ __launch_bounds__(256) void k_norm2(const cd *__restrict__ v, size_t N, double *__restrict__ parts)
{
    __shared__ double red[4];
    double acc = 0.0;
    const size_t S = (size_t)gridDim.x * 256;
    size_t j = (size_t)blockIdx.x * 256 + threadIdx.x;
    // NORM_BATCH loads issued together, then added in order
    for (; j + (NORM_BATCH - 1) * S < N; j += NORM_BATCH * S) {
        cd vv[NORM_BATCH];
#pragma unroll
        for (int i = 0; i < NORM_BATCH; ++i) vv[i] = v[j + i * S];
#pragma unroll
        for (int i = 0; i < NORM_BATCH; ++i) acc += abs2(vv[i]);
    }
    for (; j < N; j += S) acc += abs2(v[j]);
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) parts[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// The same sums for the plane-wave right-hand side q u_in (the values
// k_rhs would store, in the same order).
__global__ __launch_bounds__(256) void k_norm2_pw(const cd *__restrict__ q, const cd *__restrict__ f, int mx, int my,
                                                  int dim, size_t N, double *__restrict__ parts)
{
    __shared__ double red[4];
    double acc = 0.0;
    const size_t j0 = (size_t)blockIdx.x * 256 + threadIdx.x, S = (size_t)gridDim.x * 256;
    GridWalk w(j0, S, mx, my);
    // NORM_BATCH loads issued together (a plain unrolled loop keeps its
    // bound test between them), then added in order: the order of k_norm2
    size_t j = j0;
    for (; j + (NORM_BATCH - 1) * S < N; j += NORM_BATCH * S) {
        cd qv[NORM_BATCH], pv[NORM_BATCH];
#pragma unroll
        for (int i = 0; i < NORM_BATCH; ++i) qv[i] = q[j + i * S];
#pragma unroll
        for (int i = 0; i < NORM_BATCH; ++i) {
            pv[i] = pw_uin(f, w.x, w.y, w.z, mx, my, dim);
            w.step();
        }
#pragma unroll
        for (int i = 0; i < NORM_BATCH; ++i) acc += abs2(qv[i] * pv[i]);
    }
    for (; j < N; j += S, w.step()) acc += abs2(q[j] * pw_uin(f, w.x, w.y, w.z, mx, my, dim));
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) parts[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// ||v||_2^2 into h->d_scalar (device) and *out (host).
int norm2_blocks(size_t N) { return (int)std::min<size_t>((N + 255) / 256, 1024); }

// per-block partial sums of ||v||^2 (v = null: the plane-wave right-hand side)
void launch_norm2_parts(ffmg_handle *h, const cd *v, size_t N, int nb)
{
    if (v) {
        hipLaunchKernelGGL(k_norm2, dim3(nb), dim3(256), 0, h->stream, v, N, h->d_parts);
    } else {
        const LevelGeom &g = h->L[0].g;
        hipLaunchKernelGGL(k_norm2_pw, dim3(nb), dim3(256), 0, h->stream, h->L[0].q, h->pw_f, g.m[0], g.m[1], g.dim,
                           N, h->d_parts);
    }
}

ffmg_status norm2_of(ffmg_handle *h, const cd *v, size_t N, double *out)
{
    const int nb = norm2_blocks(N);
    launch_norm2_parts(h, v, N, nb);
    HIPCHK(h, hipGetLastError());
    TRY(reduce_to_host(h, nb, out));
    return FFMG_OK;
}

// ||v||^2 into h->d_scalar, queued on the stream; the host does not wait.
void enqueue_norm2(ffmg_handle *h, const cd *v, size_t N)
{
    const int nb = norm2_blocks(N);
    launch_norm2_parts(h, v, N, nb);
    launch_sum(h->d_parts, nb, h->d_scalar, h->stream);
}

// ||b - A u||_2 on the finest level, FP64.
ffmg_status resid_norm(ffmg_handle *h, const cd *b, const cd *u, double *out)
{
    Level &l0 = h->L[0];
    launch_stencil<double>(MODE_RNORM, l0.g, l0.P64, u, b, l0.q, (cd *)nullptr, h->d_parts, h->stream);
    HIPCHK(h, hipGetLastError());
    double s2;
    TRY(reduce_to_host(h, stencil_blocks(l0.g), &s2));
    *out = sqrt(s2);
    return FFMG_OK;
}

template <typename T>
struct LvlPtr;
template <>
struct LvlPtr<double> {
    static cd *q(Level &l) { return l.q; }
    static cd *u(Level &l) { return l.u; }
    static cd *b(Level &l) { return l.b; }
    static cd *r(Level &l) { return l.r; }
    static cd *t(Level &l) { return l.t; }
    static const Stencil<double> &P(Level &l) { return l.P64; }
    static cd *gz(Level &l) { return l.gz; }
    static const TailParams<double> &tail(ffmg_handle *h) { return h->tail64; }
    static size_t tail_lds(ffmg_handle *h) { return h->tail_lds[0]; }
};
template <>
struct LvlPtr<float> {
    static cf *q(Level &l) { return l.q32; }
    static cf *u(Level &l) { return l.u32; }
    static cf *b(Level &l) { return l.b32; }
    static cf *r(Level &l) { return l.r32; }
    static cf *t(Level &l) { return l.t32; }
    static const Stencil<float> &P(Level &l) { return l.P32; }
    static cf *gz(Level &l) { return l.gz32; }
    static const TailParams<float> &tail(ffmg_handle *h) { return h->tail32; }
    static size_t tail_lds(ffmg_handle *h) { return h->tail_lds[1]; }
};

// nu weighted-Jacobi sweeps in place on u (ping-pong through t), one sweep
// per launch.  With zero_guess the incoming u is taken as 0 without being read.
template <typename T>
void smooth(ffmg_handle *h, Level &lv, const cx<T> *b, cx<T> *u, int nu, bool zero_guess, const int *stop)
{
    using LP = LvlPtr<T>;
    cx<T> *t = LP::t(lv);
    const cx<T> *q = LP::q(lv);
    const Stencil<T> &P = LP::P(lv);
    cx<T> *src = u, *dst = t;
    const bool finest = (&lv == &h->L[0]);
    for (int s = 0; s < nu; ++s) {
        int mode = (s == 0 && zero_guess) ? MODE_JACOBI0 : MODE_JACOBI;
        int pi = (finest && mode == MODE_JACOBI) ? prof_begin(h, PROF_PRE) : -1;
        launch_stencil<T>(mode, lv.g, P, src, b, q, dst, nullptr, h->stream, finest, stop);
        prof_end(h, PROF_PRE, pi);
        std::swap(src, dst);
    }
    if (src != u) launch_copy<T>(src, u, lv.g.N(), h->stream, stop);
}

// Tile height (rows of 64 points) of the fused 2D smoothing kernel per
// FFMG_TUNE_SMOOTH variant.
constexpr int SMOOTH_TH[] = {8, 16, 4};
constexpr int SMOOTH_VARIANTS = (int)(sizeof(SMOOTH_TH) / sizeof(SMOOTH_TH[0]));

// Fused 3D smoothing chain: nu sweeps from src (0 when zero; src + P ec when
// ec is given) into dst.  From a zero guess the first two sweeps are one
// pass reading b and q only.  Otherwise, with the two-sweep form (tunable
// FFMG_TUNE_SWEEP3D, variants 0, 2, 3: three tile shapes) every pair of
// sweeps is one z-marching pass with the planes of the first sweep in LDS
// (the interpolation formed inside the first pass when ec is given); with
// variant 1 every sweep is its own pass (the interpolation inside the first
// one).  tmp is a third buffer, so
// that the last launch lands in dst without a copy.
template <typename T>
void smooth_chain3d(ffmg_handle *h, Level &lv, const cx<T> *b, const cx<T> *src, cx<T> *dst, cx<T> *tmp, int nu,
                    bool zero, const cx<T> *ec, int prof_id, const int *stop)
{
    using LP = LvlPtr<T>;
    const bool finest = (&lv == &h->L[0]);
    const Stencil<T> &P = LP::P(lv);
    const cx<T> *q = LP::q(lv);
    const bool pairs = (h->sweep3d_variant != 1);
    const int shape = h->sweep3d_variant;
    // sweeps done by launch kk of the chain
    auto sweeps_of = [&](int kk, int left) { return ((kk == 0 && zero) || pairs) ? std::min(2, left) : 1; };
    int nk = 0;
    for (int left = nu; left > 0; ++nk) left -= sweeps_of(nk, left);
    const bool alias = (src == dst);      // then launches alternate tmp, dst, ... (a copy ends an odd count)
    const cx<T> *cur = src;
    int left = nu;
    for (int kk = 0; kk < nk; ++kk) {
        const int ns = sweeps_of(kk, left);
        left -= ns;
        cx<T> *o = alias ? ((kk % 2 == 0) ? tmp : dst) : (((nk - 1 - kk) % 2 == 0) ? dst : tmp);
        const cx<T> *e = (kk == 0) ? ec : nullptr;
        const int pi = finest ? prof_begin(h, prof_id) : -1;
        if (kk == 0 && zero && ns == 2 && pairs)
            launch_sweep2_3d<T>(lv.g, P, nullptr, nullptr, b, q, o, h->stream, finest, stop, true, shape);
        else if (kk == 0 && zero && ns == 2)
            launch_sweep3d_fused<T>(true, lv.g, P, nullptr, nullptr, b, q, o, h->stream, finest, stop);
        else if (kk == 0 && zero)
            launch_stencil<T>(MODE_JACOBI0, lv.g, P, cur, b, q, o, nullptr, h->stream, finest, stop);
        else if (ns == 2)
            launch_sweep2_3d<T>(lv.g, P, cur, e, b, q, o, h->stream, finest, stop, false, shape);
        else if (e)
            launch_sweep3d_fused<T>(false, lv.g, P, cur, e, b, q, o, h->stream, finest, stop);
        else
            launch_stencil<T>(MODE_JACOBI, lv.g, P, cur, b, q, o, nullptr, h->stream, finest, stop);
        prof_end(h, prof_id, pi);
        cur = o;
    }
    if (cur != dst) launch_copy<T>(cur, dst, lv.g.N(), h->stream, stop);
}

// Fused 2D smoothing chain: nu sweeps from src (0 when zero; src + P ec when
// ec is given) into dst, two sweeps per launch; tmp is a third buffer for
// chains of more than one launch.
template <typename T>
void smooth_chain2d(ffmg_handle *h, Level &lv, const cx<T> *b, const cx<T> *src, cx<T> *dst, cx<T> *tmp, int nu,
                    bool zero, const cx<T> *ec, int prof_id, const int *stop)
{
    using LP = LvlPtr<T>;
    const bool finest = (&lv == &h->L[0]);
    const cx<T> *cur = src;
    int left = nu, kk = 0;
    int nk = (nu + 1) / 2;
    const bool alias = (src == dst);   // then launches alternate tmp, dst, ... (a copy ends an odd count)
    while (left > 0) {
        int ns = left >= 2 ? 2 : 1;
        left -= ns;
        cx<T> *o = alias ? ((kk % 2 == 0) ? tmp : dst) : (((nk - 1 - kk) % 2 == 0) ? dst : tmp);
        int pi = finest ? prof_kernel_begin(h, prof_id) : -1;
        launch_smooth2d<T>(lv.g, LP::P(lv), ns, zero, cur, ec, b, LP::q(lv), o, h->stream, finest && ns == 2, stop,
                           SMOOTH_TH[finest ? h->smooth_variant : h->smooth_coarse_variant]);
        prof_kernel_end(h, prof_id, pi);
        cur = o;
        zero = false;
        ec = nullptr;
        ++kk;
    }
    if (cur != dst) launch_copy<T>(cur, dst, lv.g.N(), h->stream, stop);
}

// One V(nu1, nu2) cycle with the fused 2D kernels: pre-smoothing u -> t,
// residual + restriction from t, coarse correction (the LDS tail kernel once
// the levels are small), then interpolation fused into post-smoothing t -> u.
template <typename T>
void vcycle_fused2d(ffmg_handle *h, int l, const cx<T> *b, cx<T> *u, bool zero_guess, const int *stop)
{
    using LP = LvlPtr<T>;
    Level &lv = h->L[l];
    Level &lc = h->L[l + 1];
    cx<T> *t = LP::t(lv), *scratch = LP::r(lv);
    cx<T> *cur = u;
    const int nu1 = nu_pre(h, l), nu2 = nu_post(h, l);
    if (nu1 == 2 && h->pre_variant != 1) {
        // two sweeps, residual and full weighting in one pass
        const bool finest = (l == 0);
        int pi = finest ? prof_kernel_begin(h, PROF_PRE) : -1;
        // finest level: the type's default tile height (16 rows FP32, 8 FP64;
        // variant 0) or the other one (variant 2); coarse levels: 16 rows
        // with the 16-row smoothing tile, else 8
        const int fdef = sizeof(T) == 4 ? 16 : 8;
        const int fh = finest ? (h->pre_variant == 2 ? 24 - fdef : fdef)
                              : (SMOOTH_TH[h->smooth_coarse_variant] >= 16 ? 16 : 8);
        launch_smooth_rr2d<T>(lv.g, LP::P(lv), zero_guess, u, b, LP::q(lv), t, LP::b(lc), h->stream, finest, stop,
                              fh);
        prof_kernel_end(h, PROF_PRE, pi);
        cur = t;
    } else {
        if (nu1 > 0) {
            smooth_chain2d<T>(h, lv, b, u, t, scratch, nu1, zero_guess, nullptr, PROF_PRE, stop);
            cur = t;
        } else if (zero_guess) {
            launch_zero<T>(u, lv.g.N(), h->stream, stop);
        }
        launch_resid_restrict2d<T>(lv.g, LP::P(lv), cur, b, LP::q(lv), LP::b(lc), h->stream, stop);
    }
    const TailParams<T> &tp = LP::tail(h);
    if (h->opt.tile_config == TILE_FUSED && tp.nt > 0 && l + 1 == (int)h->L.size() - tp.nt)
        launch_tail2d<T>(tp, LP::tail_lds(h), LP::b(lc), LP::u(lc), h->stream, stop);
    else
        vcycle<T>(h, l + 1, LP::b(lc), LP::u(lc), true, stop);
    if (nu2 > 0) {
        smooth_chain2d<T>(h, lv, b, cur, u, scratch, nu2, false, LP::u(lc), PROF_POST, stop);
    } else {
        if (cur != u) launch_copy<T>(cur, u, lv.g.N(), h->stream, stop);
        launch_prolong_add<T>(lv.g, LP::u(lc), u, h->stream, stop);
    }
}

ffmg_status validate_problem(const ffmg_problem *p, const ffmg_options *o, ffmg_handle *tmp)
{
    if (!p || !o) return fail(tmp, FFMG_EINVAL, "null problem or options");
    if (p->dim != 2 && p->dim != 3) return fail(tmp, FFMG_EINVAL, "dim must be 2 or 3 (got %d)", p->dim);
    if (o->coarsest_n < 4 || !is_pow2(o->coarsest_n))
        return fail(tmp, FFMG_EINVAL, "coarsest_n must be a power of two >= 4");
    for (int k = 0; k < p->dim; ++k) {
        if (!is_pow2(p->n[k]) || p->n[k] < o->coarsest_n || p->n[k] > (1 << 16))
            return fail(tmp, FFMG_EINVAL, "n[%d] = %lld must be a power of two in [coarsest_n, 65536]", k,
                        (long long)p->n[k]);
        if (!(p->hi[k] > p->lo[k]) || !isfinite(p->lo[k]) || !isfinite(p->hi[k]))
            return fail(tmp, FFMG_EINVAL, "box axis %d: need finite lo < hi", k);
    }
    if (!(p->gamma > 0.0 && p->gamma < M_PI / 2))
        return fail(tmp, FFMG_EINVAL, "gamma must lie in (0, pi/2) (got %g)", p->gamma);
    if (p->kind == FFMG_HELMHOLTZ) {
        if (!(p->k0 > 0.0) || !isfinite(p->k0)) return fail(tmp, FFMG_EINVAL, "k0 must be positive");
    } else if (p->kind == FFMG_SCHRODINGER) {
        if (!isfinite(p->energy)) return fail(tmp, FFMG_EINVAL, "energy must be finite");
    } else {
        return fail(tmp, FFMG_EINVAL, "unknown problem kind %d", p->kind);
    }
    if (!p->coef) return fail(tmp, FFMG_EINVAL, "coef is null");
    if (o->nu1 < 0 || o->nu2 < 0 || o->nu1 + o->nu2 < 1 || o->nu1 > 64 || o->nu2 > 64)
        return fail(tmp, FFMG_EINVAL, "need 0 <= nu1, nu2 <= 64 and nu1 + nu2 >= 1");
    if (o->nu_coarse < 0 || o->nu_coarse > 64) return fail(tmp, FFMG_EINVAL, "nu_coarse must lie in [0, 64]");
    if (o->learned_levels < 0) return fail(tmp, FFMG_EINVAL, "learned_levels must be a bit mask >= 0");
    if (!(o->omega > 0.0 && o->omega <= 1.0)) return fail(tmp, FFMG_EINVAL, "omega must lie in (0, 1]");
    if (o->max_cycles < 1) return fail(tmp, FFMG_EINVAL, "max_cycles must be >= 1");
    if (o->precision != FFMG_FP64 && o->precision != FFMG_FP32_IR)
        return fail(tmp, FFMG_EINVAL, "unknown precision %d", o->precision);
    if (o->smoother == FFMG_SMOOTH_LEARNED) {
        if (!o->smoother_weights) return fail(tmp, FFMG_EINVAL, "the learned smoother needs smoother_weights");
        if (p->dim != 2 || o->precision != FFMG_FP64)
            return fail(tmp, FFMG_EINVAL, "the learned smoother runs in 2D FP64 V-cycles");
        double hx = (p->hi[0] - p->lo[0]) / (double)p->n[0], hy = (p->hi[1] - p->lo[1]) / (double)p->n[1];
        if (fabs(hx - hy) > 1e-12 * hx) return fail(tmp, FFMG_EINVAL, "the learned smoother needs square cells");
        for (int k = 0; k < 2 * FFMG_NET_WEIGHTS; ++k)
            if (!isfinite(o->smoother_weights[k])) return fail(tmp, FFMG_ENAN, "smoother weight %d is not finite", k);
    } else if (o->smoother != FFMG_SMOOTH_JACOBI && o->smoother != FFMG_SMOOTH_GMRES &&
               o->smoother != FFMG_SMOOTH_RBGS) {
        return fail(tmp, FFMG_EINVAL, "unknown smoother %d", o->smoother);
    }
    if (o->krylov_m < 0 || o->krylov_m > GMRES_MAX_M)
        return fail(tmp, FFMG_EINVAL, "krylov_m must be in [0, %d]", GMRES_MAX_M);
    if (o->ff_precision != FFMG_FF_FP64 && o->ff_precision != FFMG_FF_BF16X3 && o->ff_precision != FFMG_FF_BF16X6)
        return fail(tmp, FFMG_EINVAL, "unknown far-field precision %d", o->ff_precision);
    if (o->tile_config < 0 || o->tile_config > 2) return fail(tmp, FFMG_EINVAL, "unknown tile_config");
    if (o->inner_cycles < 0 || o->inner_cycles > 16) return fail(tmp, FFMG_EINVAL, "inner_cycles must be in [0, 16]");
    if (o->fmg_cycles < 0 || o->fmg_cycles > 64) return fail(tmp, FFMG_EINVAL, "fmg_cycles must be in [0, 64]");
    return FFMG_OK;
}

// Unique per handle configuration of this process (keys batched workspaces).
uint64_t next_handle_serial()
{
    static std::atomic<uint64_t> next{1};
    return next++;
}

// Largest level of the LDS tail per FFMG_TUNE_TAIL variant (interior points).
constexpr int TAIL_POINTS[] = {4096, 1024, 256};
constexpr int TAIL_VARIANTS = (int)(sizeof(TAIL_POINTS) / sizeof(TAIL_POINTS[0]));

// Coarse levels handled by the one-workgroup LDS tail (2D): the longest
// run of levels l >= 1 ending at the coarsest level whose b, u, t, q fit in LDS
// and that hold at most TAIL_POINTS[tail_variant] points each.
template <typename T>
void plan_tail(ffmg_handle *h, TailParams<T> &tp, size_t &lds)
{
    const size_t max_points = (size_t)TAIL_POINTS[h->tail_variant];
    tp = TailParams<T>{};
    lds = 0;
    const int nl = (int)h->L.size();
    if (h->prob.dim != 2 || h->opt.tile_config != TILE_FUSED || nl < 3 || h->opt.smoother == FFMG_SMOOTH_GMRES ||
        h->opt.smoother == FFMG_SMOOTH_RBGS)
        return;
    const size_t budget = 144 * 1024;
    size_t bytes = 0;
    int top = nl;   // first tail level
    for (int l = nl - 1; l >= 1; --l) {
        const Level &lv = h->L[l];
        // b, u, t and a copy of q, each with a one-point zero border
        size_t add = 4 * (size_t)(lv.g.m[0] + 2) * (lv.g.m[1] + 2) * sizeof(cx<T>);
        if (lv.g.N() > max_points || bytes + add > budget || nl - l > TAIL_MAX_LEVELS) break;
        bytes += add;
        top = l;
    }
    int nt = nl - top;
    if (nt < 2) return;   // the coarsest level alone is one matrix-vector product
    tp.nt = nt;
    tp.nu1 = nu_pre(h, 1);     // tail levels are coarse levels
    tp.nu2 = nu_post(h, 1);
    tp.aug = h->aug;
    tp.nc = h->nc;
    int off = 0;
    for (int i = 0; i < nt; ++i) {
        Level &lv = h->L[top + i];
        TailLevel<T> &t = tp.lv[i];
        t.mx = lv.g.m[0];
        t.my = lv.g.m[1];
        t.off = off;
        t.P = LvlPtr<T>::P(lv);
        t.q = LvlPtr<T>::q(lv);
        off += 4 * (t.mx + 2) * (t.my + 2);
    }
    lds = bytes;
}

// The learned smoother: weight fragments, kappa h^2 on the finest level, and
// the convergence factor of the Jacobi V-cycle on this operator (measured on
// a pseudo-random right-hand side), which the learned cycle has to beat.
ffmg_status setup_learned(ffmg_handle *h)
{
    Level &l0 = h->L[0];
    const size_t N = l0.g.N();
    std::vector<unsigned short> frag(net_mfma_frag_count());
    pack_net_mfma(h->opt.smoother_weights, frag.data());
    TRY(dalloc(h, &h->d_wfrag, frag.size() * sizeof(unsigned short)));
    HIPCHK(h, hipMemcpy(h->d_wfrag, frag.data(), frag.size() * sizeof(unsigned short), hipMemcpyHostToDevice));
    h->d_kh2.assign(h->L.size(), nullptr);
    for (size_t l = 0; l < h->L.size(); ++l) {
        if (!learned_level(h, (int)l)) continue;
        Level &lv = h->L[l];
        TRY(dalloc(h, &h->d_kh2[l], lv.g.N() * sizeof(unsigned)));
        launch_kappa_h2(lv.q, h->k02, lv.g.h[0] * lv.g.h[1], lv.g.N(), h->d_kh2[l], h->stream);
    }
    HIPCHK(h, hipGetLastError());
    // reference: Jacobi V-cycles from u = 0 on a pseudo-random b
    cd *b = nullptr, *u = nullptr;
    HIPCHK(h, hipMalloc(&b, N * sizeof(cd)));
    if (hipMalloc(&u, N * sizeof(cd)) != hipSuccess) {
        (void)hipFree(b);
        return fail(h, FFMG_ENOMEM, "hipMalloc failed");
    }
    launch_hash_fill(b, N, 0x5eed5eedull, h->stream);
    launch_zero<double>(u, N, h->stream, nullptr);
    // asymptotic factor: the mean reduction of cycles 7 .. 12
    h->learned_on = false;
    double r6 = 0.0, r12 = 0.0;
    ffmg_status st = FFMG_OK;
    for (int c = 1; c <= 12 && st == FFMG_OK; ++c) {
        vcycle<double>(h, 0, b, u, c == 1, nullptr);
        if (c == 6) st = resid_norm(h, b, u, &r6);
        if (c == 12 && st == FFMG_OK) st = resid_norm(h, b, u, &r12);
    }
    (void)hipFree(b);
    (void)hipFree(u);
    TRY(st);
    h->rho_jacobi = (r6 > 0.0) ? pow(r12 / r6, 1.0 / 6.0) : 0.0;
    h->learned_on = true;
    return FFMG_OK;
}

ffmg_status setup_impl(ffmg_handle *h)
{
    const ffmg_problem &p = h->prob;
    HIPCHK(h, hipGetLastError());
    HIPCHK(h, hipGetDevice(&h->device));
    // the no-allocation far field's scratch array: its address on this device
    HIPCHK(h, ff_scratch_init(h->device));
    // hierarchy n/2^l down to min_k n_k == coarsest_n
    int64_t nl[3] = {p.n[0], p.dim >= 2 ? p.n[1] : 2, p.dim >= 3 ? p.n[2] : 2};
    for (;;) {
        Level lv;
        lv.g.dim = p.dim;
        for (int k = 0; k < 3; ++k) {
            lv.g.m[k] = (k < p.dim) ? (int)(nl[k] - 1) : 1;
            lv.g.h[k] = (k < p.dim) ? (p.hi[k] - p.lo[k]) / (double)nl[k] : 1.0;
            lv.g.lo[k] = (k < p.dim) ? p.lo[k] : 0.0;
        }
        lv.P64 = make_stencil<double>(lv.g, p.gamma, h->k02, h->opt.omega);
        lv.P32 = make_stencil<float>(lv.g, p.gamma, h->k02, h->opt.omega);
        h->L.push_back(lv);
        int64_t nmin = nl[0];
        for (int k = 1; k < p.dim; ++k) nmin = std::min(nmin, nl[k]);
        if (nmin <= h->opt.coarsest_n) break;
        for (int k = 0; k < p.dim; ++k) nl[k] /= 2;
    }
    h->nc = (int)h->L.back().g.N();
    if (h->nc > 1024)
        return fail(h, FFMG_EINVAL, "coarsest grid has %d unknowns (> 1024): use more equal n per axis", h->nc);
    const bool ir = (h->opt.precision == FFMG_FP32_IR);
    size_t maxparts = 1024;
    for (size_t l = 0; l < h->L.size(); ++l) {
        Level &lv = h->L[l];
        size_t N = lv.g.N();
        maxparts = std::max<size_t>(maxparts, stencil_blocks(lv.g));
        maxparts = std::max<size_t>(maxparts, fused2d_blocks(lv.g));
        TRY(dalloc(h, &lv.q, N * sizeof(cd)));
        TRY(dalloc(h, &lv.r, N * sizeof(cd)));
        TRY(dalloc(h, &lv.t, N * sizeof(cd)));
        if (l > 0) {
            TRY(dalloc(h, &lv.u, N * sizeof(cd)));
            TRY(dalloc(h, &lv.b, N * sizeof(cd)));
        }
        if (h->opt.smoother == FFMG_SMOOTH_GMRES && l + 1 < h->L.size()) {
            const int mk = h->opt.krylov_m > 0 ? h->opt.krylov_m : 3;
            TRY(dalloc(h, &lv.gz, (size_t)(mk + 2) * N * sizeof(cd)));
            if (ir) TRY(dalloc(h, &lv.gz32, (size_t)(mk + 2) * N * sizeof(cf)));
        }
        if (ir) {
            TRY(dalloc(h, &lv.q32, N * sizeof(cf)));
            TRY(dalloc(h, &lv.u32, N * sizeof(cf)));
            TRY(dalloc(h, &lv.b32, N * sizeof(cf)));
            TRY(dalloc(h, &lv.r32, N * sizeof(cf)));
            TRY(dalloc(h, &lv.t32, N * sizeof(cf)));
        }
    }
    h->nparts = (int)maxparts;
    // FP32 cycles of a fused 3D hierarchy: the pre-smoothing pair, residual and
    // restriction in one pass (the fastest variant measured at 511^3)
    if (h->prob.dim == 3 && ir && h->opt.tile_config != TILE_REFERENCE) h->sweep3d_variant = 4;
    if (h->opt.smoother == FFMG_SMOOTH_GMRES) {
        h->krylov_m = h->opt.krylov_m > 0 ? h->opt.krylov_m : 3;
        TRY(dalloc(h, &h->d_gm, GM_S * sizeof(double)));
        TRY(dalloc(h, &h->d_gm_parts, GM_PARTS * sizeof(double)));
    }
    TRY(dalloc(h, &h->d_parts, maxparts * sizeof(double)));
    TRY(dalloc(h, &h->d_scalar, sizeof(double)));
    {
        const LevelGeom &g0 = h->L[0].g;
        TRY(dalloc(h, &h->pw_f, (size_t)(g0.m[0] + g0.m[1] + g0.m[2]) * sizeof(cd)));
    }
    TRY(dalloc(h, &h->d_info, sizeof(int)));
    TRY(dalloc(h, &h->d_ctl, sizeof(SolveCtl)));
    HIPCHK(h, hipHostMalloc((void **)&h->h_scalar, sizeof(double), hipHostMallocDefault));
    HIPCHK(h, hipHostMalloc((void **)&h->h_ctl, sizeof(SolveCtl), hipHostMallocDefault));

    // contrast on the finest level (q = coef, or q = -2 V), non-finite check
    Level &l0 = h->L[0];
    const double scale = (p.kind == FFMG_SCHRODINGER) ? -2.0 : 1.0;
    launch_make_q((const cd *)p.coef, l0.q, l0.g.N(), scale, h->d_parts, 1024, h->stream);
    HIPCHK(h, hipGetLastError());
    double nbad;
    TRY(reduce_to_host(h, 1024, &nbad));
    if (nbad != 0.0) return fail(h, FFMG_ENAN, "coef holds %.0f non-finite values", nbad);
    for (size_t l = 1; l < h->L.size(); ++l) launch_inject<double>(h->L[l - 1].g, h->L[l - 1].q, h->L[l].q, h->stream);
    if (ir)
        for (auto &lv : h->L) launch_convert<float, double>(lv.q, lv.q32, lv.g.N(), h->stream);
    // exact inverse of the coarsest operator (FP64)
    Level &lc = h->L.back();
    TRY(dalloc(h, &h->aug, (size_t)h->nc * 2 * h->nc * sizeof(cd)));
    launch_build_coarse(lc.g, lc.P64, lc.q, h->aug, h->stream);
    cd *gjws = nullptr;
    if (h->nc > GJ_ONE_BLOCK_MAX) TRY(dalloc(h, &gjws, gauss_jordan_ws(h->nc) * sizeof(cd)));
    launch_gauss_jordan(h->aug, h->nc, h->d_info, h->stream, gjws);
    HIPCHK(h, hipGetLastError());
    int info = 0;
    HIPCHK(h, hipMemcpyAsync(&info, h->d_info, sizeof(int), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    if (info != 0) return fail(h, FFMG_EINVAL, "coarsest operator is singular (zero pivot in column %d)", info - 1);
    plan_tail<double>(h, h->tail64, h->tail_lds[0]);
    if (ir) plan_tail<float>(h, h->tail32, h->tail_lds[1]);
    if (h->opt.smoother == FFMG_SMOOTH_LEARNED) TRY(setup_learned(h));
    return FFMG_OK;
}

// Enqueue one cycle of the solve loop (V-cycle, residual / refinement step,
// control update).  ucur/ualt: FP64 iterate ping-pong of the fused
// refinement step (swapped by the caller).
// start_ec: the 3D start s P e_c was not stored; this (first) step forms it
// from e_c in its refinement pass.
void enqueue_step(ffmg_handle *h, const cd *b, cd *ucur, cd *ualt, const int *stop, const cf *start_ec = nullptr)
{
    Level &l0 = h->L[0];
    if (h->opt.precision == FFMG_FP64) {
        vcycle<double>(h, 0, b, ucur, false, stop);
        launch_stencil<double>(MODE_RNORM, l0.g, l0.P64, ucur, b, l0.q, (cd *)nullptr, h->d_parts, h->stream, false,
                               stop);
        launch_ctl_update(h->d_ctl, h->d_parts, stencil_blocks(l0.g), h->stream);
        return;
    }
    const int inner = h->opt.inner_cycles > 0 ? h->opt.inner_cycles : DEFAULT_INNER_CYCLES;
    for (int c = 0; c < inner; ++c) vcycle<float>(h, 0, l0.b32, l0.u32, c == 0, stop);
    if (l0.g.dim == 2 && h->opt.tile_config != TILE_REFERENCE) {
        int pi = prof_kernel_begin(h, PROF_REFINE);
        launch_refine2d(l0.g, l0.P64, ucur, l0.u32, b, l0.q, ualt, l0.b32, h->d_ctl, h->d_parts, h->stream, stop,
                        h->pw_f);
        prof_kernel_end(h, PROF_REFINE, pi);
        launch_ctl_update(h->d_ctl, h->d_parts, fused2d_blocks(l0.g), h->stream);
    } else if (l0.g.dim == 3 && h->opt.tile_config != TILE_REFERENCE) {
        if (start_ec) {   // (not bracketed: PROF_REFINE times the 64-byte-per-point pass)
            launch_refine3d_start(l0.g, l0.P64, start_ec, l0.u32, b, l0.q, ualt, l0.b32, h->d_ctl, h->d_parts,
                                  h->stream, stop, h->pw_f, h->d_scalar);
        } else {
            int pi = prof_begin(h, PROF_REFINE);
            launch_refine3d(l0.g, l0.P64, ucur, l0.u32, b, l0.q, ualt, l0.b32, h->d_ctl, h->d_parts, h->stream, stop,
                            h->pw_f);
            prof_end(h, PROF_REFINE, pi);
        }
        launch_ctl_update(h->d_ctl, h->d_parts, stencil_blocks(l0.g), h->stream);
    } else {
        launch_refine_update(l0.u32, ucur, h->d_ctl, l0.g.N(), h->stream, stop);
        launch_resid_to_f32_ctl(l0.g, l0.P64, ucur, b, l0.q, l0.b32, h->d_ctl, h->d_parts, h->stream, stop);
        launch_ctl_update(h->d_ctl, h->d_parts, stencil_blocks(l0.g), h->stream);
    }
}

}  // namespace

namespace ffmg {

// Levels that smooth with the network: bit l of learned_levels (0: the
// finest level only), never the levels of the LDS tail or the coarsest.
bool learned_level(const ffmg_handle *h, int l)
{
    if (h->opt.smoother != FFMG_SMOOTH_LEARNED) return false;
    const int nl = (int)h->L.size();
    const int first_tail = (h->opt.tile_config == TILE_FUSED && h->tail64.nt > 0) ? nl - h->tail64.nt : nl - 1;
    if (l >= first_tail) return false;
    const int mask = h->opt.learned_levels ? h->opt.learned_levels : 1;
    return l < 31 && ((mask >> l) & 1);
}

// One learned smoothing step on level l: r = b - A u (FP64), then
// u += h^2 N(r, kappa h^2).
void learned_step(ffmg_handle *h, int l, const cd *b, cd *u, const int *stop)
{
    Level &lv = h->L[l];
    launch_stencil<double>(MODE_RESID, lv.g, lv.P64, u, b, lv.q, lv.r, (double *)nullptr, h->stream, false, stop);
    const int pi = (l == 0) ? prof_begin(h, PROF_NET) : -1;
    launch_net_apply(lv.r, h->d_kh2[l], u, lv.g.m[0], lv.g.m[1], h->d_wfrag, lv.g.h[0] * lv.g.h[1], h->stream,
                     stop);
    prof_end(h, PROF_NET, pi);
}

// One level of a V-cycle with the learned smoother: nu learned steps,
// residual + restriction, the coarse correction, interpolation, nu learned
// steps.
template <typename T>
void vcycle(ffmg_handle *h, int l, const cx<T> *b, cx<T> *u, bool zero_guess, const int *stop);

static void vcycle_learned(ffmg_handle *h, int l, const cd *b, cd *u, bool zero_guess, const int *stop)
{
    Level &lv = h->L[l];
    Level &lc = h->L[l + 1];
    if (zero_guess) launch_zero<double>(u, lv.g.N(), h->stream, stop);
    for (int s = 0; s < nu_pre(h, l); ++s) learned_step(h, l, b, u, stop);
    launch_resid_restrict2d<double>(lv.g, lv.P64, u, b, lv.q, lc.b, h->stream, stop);
    const TailParams<double> &tp = h->tail64;
    if (h->opt.tile_config == TILE_FUSED && tp.nt > 0 && l + 1 == (int)h->L.size() - tp.nt)
        launch_tail2d<double>(tp, h->tail_lds[0], lc.b, lc.u, h->stream, stop);
    else
        vcycle<double>(h, l + 1, lc.b, lc.u, true, stop);
    launch_prolong_add<double>(lv.g, lc.u, u, h->stream, stop);
    for (int s = 0; s < nu_post(h, l); ++s) learned_step(h, l, b, u, stop);
}

// One smoothing step of the GMRES(m) or red-black Gauss-Seidel smoother
// (Sec. 3.3) in place on a level (zero: u is 0 on entry).
template <typename T>
static void other_smooth_step(ffmg_handle *h, Level &lv, const cx<T> *b, cx<T> *u, bool zero, const int *stop)
{
    using LP = LvlPtr<T>;
    if (h->opt.smoother == FFMG_SMOOTH_GMRES) {
        launch_gmres_step<T>(lv.g, LP::P(lv), b, LP::q(lv), u, zero, h->krylov_m, LP::gz(lv), h->d_gm, h->d_gm_parts,
                             h->stream, stop, h->opt.tile_config != TILE_REFERENCE);
    } else {
        if (zero) launch_zero<T>(u, lv.g.N(), h->stream, stop);
        launch_rbgs_sweep<T>(lv.g, LP::P(lv), b, LP::q(lv), u, h->stream, stop);
    }
}

// One level of a V-cycle with GMRES(m) steps or red-black Gauss-Seidel
// sweeps (Sec. 3.3): nu1 steps, residual + restriction, the coarse
// correction, interpolation, nu2 steps.
template <typename T>
static void vcycle_other(ffmg_handle *h, int l, const cx<T> *b, cx<T> *u, bool zero_guess, const int *stop)
{
    using LP = LvlPtr<T>;
    Level &lv = h->L[l];
    Level &lc = h->L[l + 1];
    const int nu1 = nu_pre(h, l), nu2 = nu_post(h, l);
    bool zero = zero_guess;
    if (nu1 == 0 && zero) launch_zero<T>(u, lv.g.N(), h->stream, stop);
    for (int s = 0; s < nu1; ++s, zero = false) other_smooth_step<T>(h, lv, b, u, zero, stop);
    if (h->opt.tile_config == TILE_REFERENCE) {
        launch_stencil<T>(MODE_RESID, lv.g, LP::P(lv), u, b, LP::q(lv), LP::r(lv), nullptr, h->stream, false, stop);
        launch_restrict<T>(lv.g, LP::r(lv), LP::b(lc), h->stream, stop);
    } else if (lv.g.dim == 2) {
        launch_resid_restrict2d<T>(lv.g, LP::P(lv), u, b, LP::q(lv), LP::b(lc), h->stream, stop);
    } else {
        launch_resid_restrict3d<T>(lv.g, LP::P(lv), u, b, LP::q(lv), LP::b(lc), h->stream, stop);
    }
    vcycle<T>(h, l + 1, LP::b(lc), LP::u(lc), true, stop);
    launch_prolong_add<T>(lv.g, LP::u(lc), u, h->stream, stop);
    for (int s = 0; s < nu2; ++s) other_smooth_step<T>(h, lv, b, u, false, stop);
}

template <typename T>
void vcycle(ffmg_handle *h, int l, const cx<T> *b, cx<T> *u, bool zero_guess, const int *stop)
{
    using LP = LvlPtr<T>;
    Level &lv = h->L[l];
    const int last = (int)h->L.size() - 1;
    if (l == last) {
        launch_coarse_apply<T>(h->aug, h->nc, b, u, h->stream, stop);
        return;
    }
    if (h->opt.smoother == FFMG_SMOOTH_GMRES || h->opt.smoother == FFMG_SMOOTH_RBGS) {
        vcycle_other<T>(h, l, b, u, zero_guess, stop);
        return;
    }
    if constexpr (sizeof(T) == 8) {
        if (h->learned_on && learned_level(h, l)) {
            vcycle_learned(h, l, b, u, zero_guess, stop);
            return;
        }
    }
    if (lv.g.dim == 2 && h->opt.tile_config != TILE_REFERENCE) {
        vcycle_fused2d<T>(h, l, b, u, zero_guess, stop);
        return;
    }
    const int nu1 = nu_pre(h, l), nu2 = nu_post(h, l);
    Level &lc = h->L[l + 1];
    if (lv.g.dim == 3 && h->opt.tile_config != TILE_REFERENCE) {
        // fused 3D level: pre-smoothing u -> t, residual + restriction from
        // t, coarse correction, interpolation fused into post-smoothing t -> u
        cx<T> *t = LP::t(lv), *scratch = LP::r(lv);
        cx<T> *cur = u;
        bool restricted = false;
        if (nu1 > 0) {
            if constexpr (sizeof(T) == 4) {
                // variant 4: the two pre-smoothing sweeps, the residual and its
                // full weighting in one pass
                if (nu1 == 2 && h->sweep3d_variant == 4 && sweep2rr_3d_fits(lv.g)) {
                    const int pk = zero_guess ? PROF_SRR0 : PROF_SRR;
                    const int pi = (l == 0) ? prof_begin(h, pk) : -1;
                    launch_sweep2rr_3d<T>(lv.g, LP::P(lv), zero_guess ? nullptr : u, b, LP::q(lv), t, LP::b(lc),
                                          h->stream, l == 0, stop);
                    prof_end(h, pk, pi);
                    restricted = true;
                }
            }
            if (!restricted) smooth_chain3d<T>(h, lv, b, u, t, scratch, nu1, zero_guess, nullptr, PROF_PRE, stop);
            cur = t;
        } else if (zero_guess) {
            launch_zero<T>(u, lv.g.N(), h->stream, stop);
        }
        if (!restricted) {
            const int pr = (l == 0) ? prof_begin(h, PROF_RR) : -1;
            launch_resid_restrict3d<T>(lv.g, LP::P(lv), cur, b, LP::q(lv), LP::b(lc), h->stream, stop);
            prof_end(h, PROF_RR, pr);
        }
        vcycle<T>(h, l + 1, LP::b(lc), LP::u(lc), true, stop);
        if (nu2 > 0) {
            smooth_chain3d<T>(h, lv, b, cur, u, scratch, nu2, false, LP::u(lc), PROF_POST, stop);
        } else {
            if (cur != u) launch_copy<T>(cur, u, lv.g.N(), h->stream, stop);
            launch_prolong_add<T>(lv.g, LP::u(lc), u, h->stream, stop);
        }
        return;
    }
    if (nu1 > 0) smooth<T>(h, lv, b, u, nu1, zero_guess, stop);
    else if (zero_guess) launch_zero<T>(u, lv.g.N(), h->stream, stop);
    launch_stencil<T>(MODE_RESID, lv.g, LP::P(lv), u, b, LP::q(lv), LP::r(lv), nullptr, h->stream, false, stop);
    launch_restrict<T>(lv.g, LP::r(lv), LP::b(lc), h->stream, stop);
    vcycle<T>(h, l + 1, LP::b(lc), LP::u(lc), true, stop);
    launch_prolong_add<T>(lv.g, LP::u(lc), u, h->stream, stop);
    if (nu2 > 0) smooth<T>(h, lv, b, u, nu2, false, stop);
}
template void vcycle<double>(ffmg_handle *, int, const cd *, cd *, bool, const int *);
template void vcycle<float>(ffmg_handle *, int, const cf *, cf *, bool, const int *);

// Full multigrid start on the stream: the finest right-hand side injected
// level by level into the coarse right-hand-side buffers, exact solve on the
// coarsest level, then, finest-ward, each level's solution buffer set to the
// interpolated coarser solution and improved by k V-cycles; u = P u_1.  A
// V-cycle on level l uses only the buffers of levels >= l + 1 besides its
// own temporaries, so the hierarchy's coarse buffers hold the start too.
// With the LDS tail (2D fused kernels) the levels it covers (from level 1 at
// the finest) run their whole part of the nested iteration in one launch.
// T = float works on b / s, s = sqrt(*bnorm2 / N) (unit RMS).
// defer_last: leave out the final interpolation into u (the caller fuses it
// into the initial residual pass).
template <typename T>
void fmg_start(ffmg_handle *h, const cd *b, cd *u, int k, const double *bnorm2, bool defer_last = false)
{
    using LP = LvlPtr<T>;
    const int last = (int)h->L.size() - 1;
    Level &l0 = h->L[0];
    if (last == 0) {
        launch_coarse_apply<double>(h->aug, h->nc, b, u, h->stream, nullptr);
        return;
    }
    const TailParams<T> &tp = LP::tail(h);
    const bool tail = (l0.g.dim == 2 && h->opt.tile_config == TILE_FUSED && tp.nt >= 2);
    const int t0 = tail ? last + 1 - tp.nt : last + 1;   // first tail level
    const int s0 = (t0 == 0) ? 1 : 0;                      // its first level the start runs on
    const int top = tail ? t0 + s0 : last;                 // right-hand sides injected down to here
    const bool tail_fmg = tail && top < last;
    launch_inject_rhs<T>(l0.g, b, LP::b(h->L[1]), bnorm2, h->stream, l0.q, h->pw_f);
    for (int l = 1; l < top; ++l) launch_inject<T>(h->L[l].g, LP::b(h->L[l]), LP::b(h->L[l + 1]), h->stream);
    int from;
    if (tail_fmg) {
        launch_tail2d_fmg<T>(tp, LP::tail_lds(h), LP::b(h->L[top]), LP::u(h->L[top]), s0, k, h->stream);
        from = top - 1;
    } else {
        for (int l = top; l < last; ++l) launch_inject<T>(h->L[l].g, LP::b(h->L[l]), LP::b(h->L[l + 1]), h->stream);
        launch_coarse_apply<T>(h->aug, h->nc, LP::b(h->L[last]), LP::u(h->L[last]), h->stream, nullptr);
        from = last - 1;
    }
    for (int l = from; l >= 1; --l) {
        Level &lv = h->L[l];
        launch_prolong_set<T, T>(lv.g, LP::u(h->L[l + 1]), LP::u(lv), nullptr, 1.0, h->stream);
        for (int c = 0; c < k; ++c) vcycle<T>(h, l, LP::b(lv), LP::u(lv), false, nullptr);
    }
    if (!defer_last)
        launch_prolong_set<T, double>(l0.g, LP::u(h->L[1]), u, bnorm2, 1.0 / sqrt((double)l0.g.N()), h->stream);
}

// The FMG start in the handle's precision; bnorm2: ||b||^2 on the device
// (read by the FP32 form only).
void fmg_enqueue(ffmg_handle *h, const cd *b, cd *u, int k, const double *bnorm2, bool defer_last = false)
{
    if (h->opt.precision == FFMG_FP32_IR) fmg_start<float>(h, b, u, k, bnorm2, defer_last);
    else fmg_start<double>(h, b, u, k, nullptr);
}

// The FP32-in-FP64 3D solve with the fused kernels writes the start's last
// interpolation in its initial residual pass.
bool fmg_fused_resid(const ffmg_handle *h)
{
    return h->opt.fmg_cycles > 0 && h->opt.precision == FFMG_FP32_IR && h->opt.tile_config != TILE_REFERENCE &&
           h->prob.dim == 3 && h->L.size() > 1;
}

// The fused FP32 2D refinement step writes the new iterate into the other of
// two buffers (u and l0.t).
bool fp32_pingpong(const ffmg_handle *h)
{
    return h->opt.precision == FFMG_FP32_IR && h->opt.tile_config != TILE_REFERENCE;
}

// Queue nb steps (V-cycles, or FP32_IR refinement steps) of the pending solve,
// each skipped on the device once the control block has stopped the solve,
// then the copy of the control block into pinned host memory.
ffmg_status enqueue_batch(ffmg_handle *h, int nb)
{
    PendingSolve &p = h->pend;
    const int *stop = &h->d_ctl->done;
    for (int i = 0; i < nb; ++i) {
        enqueue_step(h, p.b, p.ua, p.ub, stop, p.start_ec);
        p.start_ec = nullptr;
        if (fp32_pingpong(h)) std::swap(p.ua, p.ub);
    }
    p.queued += nb;
    HIPCHK(h, hipGetLastError());
    HIPCHK(h, hipMemcpyAsync(h->h_ctl, h->d_ctl, sizeof(SolveCtl), hipMemcpyDeviceToHost, h->stream));
    return FFMG_OK;
}

// Cycle counts, relative residual and rate of a finished solve.
void fill_info(ffmg_handle *h, const SolveCtl &c, double bn2, int k_before_restart, ffmg_solve_info *inf)
{
    inf->cycles = std::max(c.k, 0) + k_before_restart;
    inf->vcycles = inf->cycles * ((h->opt.precision == FFMG_FP32_IR)
                                      ? (h->opt.inner_cycles > 0 ? h->opt.inner_cycles : DEFAULT_INNER_CYCLES) : 1);
    const double bn = sqrt(bn2), rk = sqrt(c.rk2), r0 = sqrt(c.r0_2);
    inf->rel_residual = rk / bn;
    inf->conv_factor = (inf->cycles > 0 && r0 > 0) ? pow(rk / r0, 1.0 / inf->cycles) : 0.0;
    h->last_cycles = inf->cycles;
}

ffmg_status done_status(ffmg_handle *h, const SolveCtl &c, int maxc)
{
    switch (c.done) {
    case 1: return FFMG_OK;
    case 2: return fail(h, FFMG_ENOCONV, "residual grew on 3 consecutive cycles");
    case 4: return fail(h, FFMG_ENOCONV, "residual became non-finite at cycle %d", c.k);
    default: return fail(h, FFMG_ENOCONV, "no convergence in %d cycles", maxc);
    }
}

}  // namespace ffmg

// =========================================================================
extern "C" {

void ffmg_default_options(ffmg_options *o)
{
    if (!o) return;
    memset(o, 0, sizeof *o);
    o->nu1 = 2;
    o->nu2 = 2;
    o->omega = 0.8;
    o->coarsest_n = 8;
    o->max_cycles = 200;
    o->precision = FFMG_FP64;
    o->smoother = FFMG_SMOOTH_JACOBI;
    o->ff_precision = FFMG_FF_FP64;
    o->fmg_cycles = 0;
}

const char *ffmg_strerror(ffmg_status s)
{
    switch (s) {
    case FFMG_OK: return "ok";
    case FFMG_EINVAL: return "invalid argument";
    case FFMG_ENOMEM: return "out of device memory";
    case FFMG_EDEVICE: return "HIP device error";
    case FFMG_ENOCONV: return "no convergence";
    case FFMG_ERANGE: return "exponent range exceeded";
    case FFMG_ENAN: return "non-finite input";
    }
    return "unknown status";
}

const char *ffmg_last_error(const ffmg_handle *h) { return h ? h->err.c_str() : "null handle"; }

ffmg_status mg_setup(const ffmg_problem *p, const ffmg_options *o, ffmg_handle **out)
{
    if (!out) return FFMG_EINVAL;
    *out = nullptr;
    ffmg_handle *h = new ffmg_handle();
    h->serial = next_handle_serial();
    ffmg_status st = validate_problem(p, o, h);
    if (st == FFMG_OK) {
        h->prob = *p;
        h->opt = *o;
        h->stream = (hipStream_t)o->stream;
        if (p->kind == FFMG_SCHRODINGER) {
            // kappa = 2(E - V) = k02 + q for any E; k0 (the incoming plane
            // wave's wavenumber) exists only above the breakup threshold
            h->k02 = 2.0 * p->energy;
            h->k0 = (p->energy > 0.0) ? sqrt(h->k02) : 0.0;
        } else {
            h->k0 = p->k0;
            h->k02 = p->k0 * p->k0;
        }
        st = setup_impl(h);
    }
    if (st != FFMG_OK) {
        mg_destroy(h);
        return st;
    }
    *out = h;
    return FFMG_OK;
}

ffmg_status mg_profile_enable(ffmg_handle *h, int enable)
{
    if (!h) return FFMG_EINVAL;
    h->profile_mask = enable & ((1 << PROF_N) - 1);
    return FFMG_OK;
}

ffmg_status mg_profile_read(ffmg_handle *h, int kernel, double *total_ms, int64_t *count)
{
    if (!h || kernel < 0 || kernel >= PROF_N || !total_ms || !count) return fail(h, FFMG_EINVAL, "bad argument");
    HIPCHK(h, hipStreamSynchronize(h->stream));
    double tot = 0.0;
    for (auto &e : h->ev[kernel]) {
        float ms = 0.f;
        HIPCHK(h, hipEventElapsedTime(&ms, e.first, e.second));
        tot += ms;
        h->ev_free.push_back(e);
    }
    *total_ms = tot;
    *count = (int64_t)h->ev[kernel].size();
    h->ev[kernel].clear();
    return FFMG_OK;
}

ffmg_status mg_profile_durations(ffmg_handle *h, int kernel, double *ms, int64_t cap, int64_t *count)
{
    if (!h || kernel < 0 || kernel >= PROF_N || !count || cap < 0 || (cap > 0 && !ms))
        return fail(h, FFMG_EINVAL, "bad argument");
    HIPCHK(h, hipStreamSynchronize(h->stream));
    int64_t n = 0;
    for (auto &e : h->ev[kernel]) {
        float t = 0.f;
        HIPCHK(h, hipEventElapsedTime(&t, e.first, e.second));
        if (n < cap) ms[n] = t;
        ++n;
        h->ev_free.push_back(e);
    }
    *count = n;
    h->ev[kernel].clear();
    return FFMG_OK;
}

void mg_destroy(ffmg_handle *h)
{
    if (!h) return;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    else (void)hipDeviceSynchronize();
    for (int k = 0; k < PROF_N; ++k)
        for (auto &e : h->ev[k]) h->ev_free.push_back(e);
    for (auto &e : h->ev_free) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    if (h->pend.e0) (void)hipEventDestroy(h->pend.e0);
    if (h->pend.e1) (void)hipEventDestroy(h->pend.e1);
    if (h->ff) ff_plan_destroy(h->ff);
    if (h->batch) batch_destroy(h->batch);
    if (h->ffbatch) ff_batch_destroy(h->ffbatch);
    for (void *p : h->allocs) (void)hipFree(p);
    for (void *p : h->ion_buf)
        if (p) (void)hipFree(p);
    if (h->h_scalar) (void)hipHostFree(h->h_scalar);
    if (h->h_ctl) (void)hipHostFree(h->h_ctl);
    delete h;
}

int mg_num_levels(const ffmg_handle *h) { return h ? (int)h->L.size() : 0; }

ffmg_status mg_level_shape(const ffmg_handle *h, int level, int64_t m[3])
{
    if (!h || !m || level < 0 || level >= (int)h->L.size()) return FFMG_EINVAL;
    for (int k = 0; k < 3; ++k) m[k] = h->L[level].g.m[k];
    return FFMG_OK;
}

ffmg_status mg_rhs_plane_wave(ffmg_handle *h, const double eta[3], void *b)
{
    NOT_PENDING(h);
    if (!h || !eta) return fail(h, FFMG_EINVAL, "null argument");
    if (!(h->k0 > 0.0)) return fail(h, FFMG_EINVAL, "a plane wave needs E > 0");
    double e[3] = {0, 0, 0};
    for (int k = 0; k < h->prob.dim; ++k) {
        if (!isfinite(eta[k])) return fail(h, FFMG_EINVAL, "eta is not finite");
        e[k] = eta[k];
    }
    if (exponent_budget(h) > 700.0) return fail(h, FFMG_ERANGE, "exp(i k0 eta.z) overflows double on this box");
    launch_pw_factors(h->L[0].g, h->prob.gamma, h->k0, e, h->pw_f, h->stream);
    h->pw_set = true;
    if (b) launch_rhs_plane_wave(h->L[0].g, h->L[0].q, h->pw_f, (cd *)b, h->stream);
    HIPCHK(h, hipGetLastError());
    return FFMG_OK;
}

// Solves with b = NULL take the plane wave of the last mg_rhs_plane_wave.
// The FP32-in-FP64 solve with the fused kernels forms it where its FP64
// kernels need it (the norm, the start's injection, the residuals of the
// refinement); every other path gets it stored once in the handle.
static bool pw_implicit(const ffmg_handle *h)
{
    return h->opt.precision == FFMG_FP32_IR && h->opt.tile_config != TILE_REFERENCE &&
           h->opt.smoother == FFMG_SMOOTH_JACOBI && h->L.size() > 1;
}

static ffmg_status pw_resolve(ffmg_handle *h, const cd **b)
{
    if (*b) return FFMG_OK;
    if (!h->pw_set)
        return fail(h, FFMG_EINVAL, "b is NULL but no plane wave was set on this handle (mg_rhs_plane_wave)");
    if (pw_implicit(h)) return FFMG_OK;
    if (!h->pw_b) TRY(dalloc(h, &h->pw_b, h->L[0].g.N() * sizeof(cd)));
    launch_rhs_plane_wave(h->L[0].g, h->L[0].q, h->pw_f, h->pw_b, h->stream);
    HIPCHK(h, hipGetLastError());
    *b = h->pw_b;
    return FFMG_OK;
}

ffmg_status mg_rhs_phase(ffmg_handle *h, const double eta[3], void *b)
{
    NOT_PENDING(h);
    if (!h || !eta || !b) return fail(h, FFMG_EINVAL, "null argument");
    if (!(h->k0 > 0.0)) return fail(h, FFMG_EINVAL, "a plane wave needs E > 0");
    double e[3] = {0, 0, 0};
    for (int k = 0; k < h->prob.dim; ++k) e[k] = eta[k];
    launch_rhs_phase(h->L[0].g, h->prob.gamma, h->k0, e, h->L[0].q, (cd *)b, h->stream);
    HIPCHK(h, hipGetLastError());
    return FFMG_OK;
}

ffmg_status mg_residual(ffmg_handle *h, const void *b, const void *u, void *r)
{
    NOT_PENDING(h);
    if (!h || !b || !u || !r || r == u || r == b) return fail(h, FFMG_EINVAL, "null or aliased argument");
    Level &l0 = h->L[0];
    launch_stencil<double>(MODE_RESID, l0.g, l0.P64, (const cd *)u, (const cd *)b, l0.q, (cd *)r, nullptr, h->stream,
                           false, nullptr);
    HIPCHK(h, hipGetLastError());
    return FFMG_OK;
}

ffmg_status mg_apply(ffmg_handle *h, const void *u, void *Au)
{
    if (!h || !u || !Au) return fail(h, FFMG_EINVAL, "null argument");
    Level &l0 = h->L[0];
    launch_stencil<double>(MODE_APPLY, l0.g, l0.P64, (const cd *)u, nullptr, l0.q, (cd *)Au, nullptr, h->stream);
    HIPCHK(h, hipGetLastError());
    return FFMG_OK;
}

ffmg_status mg_smooth(ffmg_handle *h, const void *b, const void *u, void *u_out)
{
    NOT_PENDING(h);
    if (!h || !b || !u || !u_out || u == u_out) return fail(h, FFMG_EINVAL, "null or aliased argument");
    Level &l0 = h->L[0];
    if (h->opt.smoother == FFMG_SMOOTH_GMRES || h->opt.smoother == FFMG_SMOOTH_RBGS) {
        if (h->L.size() < 2) return fail(h, FFMG_EINVAL, "a one-level hierarchy is solved exactly, not smoothed");
        HIPCHK(h, hipMemcpyAsync(u_out, u, l0.g.N() * sizeof(cd), hipMemcpyDeviceToDevice, h->stream));
        other_smooth_step<double>(h, l0, (const cd *)b, (cd *)u_out, false, nullptr);
        HIPCHK(h, hipGetLastError());
        return FFMG_OK;
    }
    launch_stencil<double>(MODE_JACOBI, l0.g, l0.P64, (const cd *)u, (const cd *)b, l0.q, (cd *)u_out, nullptr,
                           h->stream);
    HIPCHK(h, hipGetLastError());
    return FFMG_OK;
}

ffmg_status mg_learned_smooth(ffmg_handle *h, const void *b, void *u)
{
    NOT_PENDING(h);
    if (!h || !b || !u) return fail(h, FFMG_EINVAL, "null argument");
    if (h->opt.smoother != FFMG_SMOOTH_LEARNED) return fail(h, FFMG_EINVAL, "the handle has no learned smoother");
    if (!learned_level(h, 0)) return fail(h, FFMG_EINVAL, "the finest level does not use the learned smoother");
    learned_step(h, 0, (const cd *)b, (cd *)u, nullptr);
    HIPCHK(h, hipGetLastError());
    return FFMG_OK;
}

ffmg_status mg_gmres_smooth(ffmg_handle *h, const void *b, void *u)
{
    NOT_PENDING(h);
    if (!h || !b || !u) return fail(h, FFMG_EINVAL, "null argument");
    if (h->opt.smoother != FFMG_SMOOTH_GMRES) return fail(h, FFMG_EINVAL, "the handle does not smooth with GMRES(m)");
    if (h->L.size() < 2) return fail(h, FFMG_EINVAL, "a one-level hierarchy is solved exactly, not smoothed");
    Level &l0 = h->L[0];
    launch_gmres_step<double>(l0.g, l0.P64, (const cd *)b, l0.q, (cd *)u, false, h->krylov_m, l0.gz, h->d_gm,
                              h->d_gm_parts, h->stream, nullptr, h->opt.tile_config != TILE_REFERENCE);
    HIPCHK(h, hipGetLastError());
    return FFMG_OK;
}

double mg_jacobi_factor(const ffmg_handle *h) { return h ? h->rho_jacobi : 0.0; }

ffmg_status mg_residual_norm(ffmg_handle *h, const void *b, const void *u, double *rnorm)
{
    NOT_PENDING(h);
    if (!h || !b || !u || !rnorm) return fail(h, FFMG_EINVAL, "null argument");
    return resid_norm(h, (const cd *)b, (const cd *)u, rnorm);
}

ffmg_status mg_vcycle(ffmg_handle *h, const void *b, void *u)
{
    NOT_PENDING(h);
    if (!h || !b || !u) return fail(h, FFMG_EINVAL, "null argument");
    vcycle<double>(h, 0, (const cd *)b, (cd *)u, false, nullptr);
    HIPCHK(h, hipGetLastError());
    return FFMG_OK;
}

ffmg_status mg_fmg(ffmg_handle *h, const void *bv, void *uv, int k)
{
    NOT_PENDING(h);
    if (!h || !bv || !uv) return fail(h, FFMG_EINVAL, "null argument");
    if (k < 0 || k > 64) return fail(h, FFMG_EINVAL, "k must be in [0, 64]");
    const cd *b = (const cd *)bv;
    cd *u = (cd *)uv;
    h->learned_on = (h->opt.smoother == FFMG_SMOOTH_LEARNED);
    double bn2 = 0.0;
    if (h->opt.precision == FFMG_FP32_IR) {
        TRY(norm2_of(h, b, h->L[0].g.N(), &bn2));   // leaves ||b||^2 in h->d_scalar
        if (!isfinite(bn2)) return fail(h, FFMG_ENAN, "right-hand side holds non-finite values");
    }
    fmg_enqueue(h, b, u, k, h->d_scalar);
    HIPCHK(h, hipGetLastError());
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return FFMG_OK;
}

// The learned smoother's solve: the host reads the control block after each
// batch of cycles and may switch the rest of the solve to Jacobi.
static ffmg_status solve_host_controlled(ffmg_handle *h, const void *bv, void *uv, double tol,
                                         ffmg_solve_info *info)
{
    if (!h || !uv) return fail(h, FFMG_EINVAL, "null argument");
    if (!(tol > 0.0) || !(tol < 1.0)) return fail(h, FFMG_EINVAL, "tol must lie in (0, 1)");
    const cd *b = (const cd *)bv;
    TRY(pw_resolve(h, &b));
    cd *u = (cd *)uv;
    ffmg_solve_info inf{};
    hipEvent_t e0, e1;
    HIPCHK(h, hipEventCreate(&e0));
    HIPCHK(h, hipEventCreate(&e1));
    HIPCHK(h, hipEventRecord(e0, h->stream));
    Level &l0 = h->L[0];
    const size_t N = l0.g.N();
    double bn2 = 0.0;
    auto finish = [&](ffmg_status s) {
        (void)hipEventRecord(e1, h->stream);
        (void)hipEventSynchronize(e1);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        inf.status = s;
        inf.t_solve_ms = ms;
        if (info) *info = inf;
        return s;
    };
    ffmg_status st = norm2_of(h, b, N, &bn2);   // leaves ||b||^2 in h->d_scalar
    if (st != FFMG_OK) return finish(st);
    if (bn2 == 0.0) {
        (void)hipMemsetAsync(u, 0, N * sizeof(cd), h->stream);
        return finish(FFMG_OK);
    }
    if (!isfinite(bn2)) return finish(fail(h, FFMG_ENAN, "right-hand side holds non-finite values"));
    const int maxc = h->opt.max_cycles;
    launch_ctl_init(h->d_ctl, h->d_scalar, tol, N, maxc, h->stream);
    const int *stop = &h->d_ctl->done;
    h->learned_on = (h->opt.smoother == FFMG_SMOOTH_LEARNED);
    if (h->opt.fmg_cycles > 0) fmg_enqueue(h, b, u, h->opt.fmg_cycles, h->d_scalar);
    // initial residual (cycle 0)
    if (h->opt.precision == FFMG_FP64) {
        launch_stencil<double>(MODE_RNORM, l0.g, l0.P64, u, b, l0.q, (cd *)nullptr, h->d_parts, h->stream);
        launch_ctl_update(h->d_ctl, h->d_parts, stencil_blocks(l0.g), h->stream);
    } else {
        launch_resid_to_f32_ctl(l0.g, l0.P64, u, b, l0.q, l0.b32, h->d_ctl, h->d_parts, h->stream, nullptr);
        launch_ctl_update(h->d_ctl, h->d_parts, stencil_blocks(l0.g), h->stream);
    }
    // cycles in batches; the control block decides on the device.  With the
    // learned smoother the first cycle runs alone (its reduction from u = 0
    // is a transient) and the mean reduction factor of every later batch of
    // two cycles is compared with the asymptotic factor of the Jacobi V-cycle
    // (measured at setup): two batches in a row more than 10% worse, or
    // residual growth, switch the rest of the solve to Jacobi; a non-finite
    // iterate or a residual ten times the initial one restarts it with Jacobi
    // from u = 0.
    cd *ua = u, *ub = l0.t;
    int queued = 0;
    int batch = h->last_cycles > 0 ? h->last_cycles : 4;
    if (h->learned_on) batch = 1;
    SolveCtl c{};
    int k_prev = 0, bad = 0, k_before_restart = 0;
    double r2_prev = -1.0;
    for (;;) {
        int nb = std::min(batch, maxc - queued);
        for (int i = 0; i < nb; ++i) {
            enqueue_step(h, b, ua, ub, stop);
            if (fp32_pingpong(h)) std::swap(ua, ub);
        }
        queued += nb;
        HIPCHK(h, hipGetLastError());
        HIPCHK(h, hipMemcpyAsync(h->h_ctl, h->d_ctl, sizeof(SolveCtl), hipMemcpyDeviceToHost, h->stream));
        HIPCHK(h, hipStreamSynchronize(h->stream));
        c = *h->h_ctl;
        if (h->learned_on && (c.done == 4 || !(c.rk2 <= 100.0 * c.r0_2))) {
            // a non-finite iterate, or a residual up tenfold from the start:
            // start again from u = 0 with Jacobi
            h->learned_on = false;
            inf.fell_back = 1;
            k_before_restart = c.k;
            launch_zero<double>(u, N, h->stream, nullptr);
            launch_ctl_init(h->d_ctl, h->d_scalar, tol, N, maxc, h->stream);
            launch_stencil<double>(MODE_RNORM, l0.g, l0.P64, u, b, l0.q, (cd *)nullptr, h->d_parts, h->stream);
            launch_ctl_update(h->d_ctl, h->d_parts, stencil_blocks(l0.g), h->stream);
            queued = 0;
            k_prev = 0;
            r2_prev = -1.0;
            batch = 2;
            continue;
        }
        if (h->learned_on && c.done == 2) {
            // the learned cycles made the residual grow: continue with Jacobi
            // from the current iterate instead of failing
            c.done = 0;
            c.grow = 0;
            *h->h_ctl = c;
            HIPCHK(h, hipMemcpyAsync(h->d_ctl, h->h_ctl, sizeof(SolveCtl), hipMemcpyHostToDevice, h->stream));
            h->learned_on = false;
            inf.fell_back = 1;
        } else if (h->learned_on && c.done == 0 && k_prev >= 1 && c.k > k_prev && r2_prev > 0.0) {
            const double rho = pow(c.rk2 / r2_prev, 0.5 / (c.k - k_prev));
            bad = (rho <= 1.10 * h->rho_jacobi) ? 0 : bad + 1;
            if (bad >= 2) {
                h->learned_on = false;
                inf.fell_back = 1;
            }
        }
        k_prev = c.k;
        r2_prev = c.rk2;
        if (c.done || queued >= maxc) break;
        batch = 2;
    }
    // the fused refinement step alternates u between u and l0.t: after an odd
    // number of completed steps the iterate is in l0.t
    if (fp32_pingpong(h) && (c.k % 2) == 1) HIPCHK(h, hipMemcpyAsync(u, l0.t, N * sizeof(cd), hipMemcpyDeviceToDevice, h->stream));
    h->learned_on = (h->opt.smoother == FFMG_SMOOTH_LEARNED);   // the fallback lasts for this solve only
    fill_info(h, c, bn2, k_before_restart, &inf);
    return finish(done_status(h, c, maxc));
}


ffmg_status mg_solve_begin(ffmg_handle *h, const void *bv, void *uv, double tol)
{
    if (!h || !uv) return fail(h, FFMG_EINVAL, "null argument");
    NOT_PENDING(h);
    if (!(tol > 0.0) || !(tol < 1.0)) return fail(h, FFMG_EINVAL, "tol must lie in (0, 1)");
    if (h->opt.smoother == FFMG_SMOOTH_LEARNED)
        return fail(h, FFMG_EINVAL, "the learned smoother's fallback is decided on the host between cycles: use mg_solve");
    const cd *b = (const cd *)bv;
    TRY(pw_resolve(h, &b));
    cd *u = (cd *)uv;
    PendingSolve &p = h->pend;
    Level &l0 = h->L[0];
    const size_t N = l0.g.N();
    if (!p.e0) {
        HIPCHK(h, hipEventCreate(&p.e0));
        HIPCHK(h, hipEventCreate(&p.e1));
    }
    HIPCHK(h, hipEventRecord(p.e0, h->stream));
    enqueue_norm2(h, b, N);   // ||b||^2 -> h->d_scalar; b = 0 or non-finite sets the stop code 5 in the control block
    launch_ctl_init(h->d_ctl, h->d_scalar, tol, N, h->opt.max_cycles, h->stream);
    h->learned_on = false;
    // The fused FP32 step alternates the iterate between u and l0.t.  The
    // full multigrid start overwrites u, so it may as well be written into
    // l0.t: when the previous solve took an odd number of steps, starting
    // there makes the iterate of a solve with the same count end in u, with
    // no copy at the end.
    p.flip = h->opt.fmg_cycles > 0 && fp32_pingpong(h) && (h->last_cycles % 2) == 1;
    cd *u0 = p.flip ? l0.t : u;
    const bool fused_start = fmg_fused_resid(h);
    if (h->opt.fmg_cycles > 0) fmg_enqueue(h, b, u0, h->opt.fmg_cycles, h->d_scalar, fused_start);
    // initial residual (cycle 0)
    if (h->opt.precision == FFMG_FP64)
        launch_stencil<double>(MODE_RNORM, l0.g, l0.P64, u0, b, l0.q, (cd *)nullptr, h->d_parts, h->stream);
    else if (fused_start) {
        // the start's first-level solution is kept (the first step's V-cycles
        // reuse the level's buffers); u0 is formed again by that step's
        // refinement pass, so it is stored only if no step completes
        const size_t n1 = h->L[1].g.N();
        if (!h->fmg_e1) TRY(dalloc(h, &h->fmg_e1, n1 * sizeof(cf)));
        HIPCHK(h, hipMemcpyAsync(h->fmg_e1, h->L[1].u32, n1 * sizeof(cf), hipMemcpyDeviceToDevice, h->stream));
        launch_fmg_resid3d(l0.g, l0.P64, h->fmg_e1, b, l0.q, nullptr, l0.b32, h->d_ctl, h->d_parts, h->d_scalar,
                           h->pw_f, h->stream);
    }
    else if (!b)
        launch_resid_pw(l0.g, l0.P64, u0, l0.q, l0.b32, h->d_ctl, h->d_parts, h->pw_f, h->stream);
    else
        launch_resid_to_f32_ctl(l0.g, l0.P64, u0, b, l0.q, l0.b32, h->d_ctl, h->d_parts, h->stream, nullptr);
    launch_ctl_update(h->d_ctl, h->d_parts, stencil_blocks(l0.g), h->stream);
    HIPCHK(h, hipGetLastError());
    p.b = b;
    p.u = u;
    p.ua = u0;
    p.ub = p.flip ? u : l0.t;
    p.queued = 0;
    p.start_ec = fused_start ? h->fmg_e1 : nullptr;
    p.start_unstored = fused_start;
    // the first batch: as many steps as the previous solve took (4 at first)
    const int batch = std::min(h->last_cycles > 0 ? h->last_cycles : 4, h->opt.max_cycles);
    TRY(enqueue_batch(h, batch));
    p.active = true;
    return FFMG_OK;
}

ffmg_status mg_solve_end(ffmg_handle *h, ffmg_solve_info *info)
{
    if (!h) return FFMG_EINVAL;
    PendingSolve &p = h->pend;
    if (!p.active) return fail(h, FFMG_EINVAL, "no solve begun by mg_solve_begin is pending on this handle");
    p.active = false;
    ffmg_solve_info inf{};
    auto finish = [&](ffmg_status s) {
        (void)hipEventRecord(p.e1, h->stream);
        (void)hipEventSynchronize(p.e1);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, p.e0, p.e1);
        inf.status = s;
        inf.t_solve_ms = ms;
        if (info) *info = inf;
        return s;
    };
    Level &l0 = h->L[0];
    const size_t N = l0.g.N();
    HIPCHK(h, hipStreamSynchronize(h->stream));
    SolveCtl c = *h->h_ctl;
    if (c.done == 5) {
        if (c.b2 == 0.0) {   // b = 0: u = 0 after 0 cycles
            launch_zero<double>(p.u, N, h->stream, nullptr);
            HIPCHK(h, hipGetLastError());
            return finish(FFMG_OK);
        }
        return finish(fail(h, FFMG_ENAN, "right-hand side holds non-finite values"));
    }
    // further batches of two steps until the control block stops the solve
    const int maxc = h->opt.max_cycles;
    while (!c.done && p.queued < maxc) {
        TRY(enqueue_batch(h, std::min(2, maxc - p.queued)));
        HIPCHK(h, hipStreamSynchronize(h->stream));
        c = *h->h_ctl;
    }
    // a start formed only inside the refinement passes, with no step
    // completed: store it in the start buffer
    if (p.start_unstored && c.k <= 0)
        launch_prolong_set<float, double>(l0.g, h->fmg_e1, p.flip ? l0.t : p.u, h->d_scalar,
                                          1.0 / sqrt((double)l0.g.N()), h->stream);
    // the fused refinement step alternates the iterate between the start
    // buffer and the other one: after an odd number of completed steps it is
    // in the other
    if (fp32_pingpong(h) && ((c.k % 2) == 1) != p.flip)
        HIPCHK(h, hipMemcpyAsync(p.u, l0.t, N * sizeof(cd), hipMemcpyDeviceToDevice, h->stream));
    fill_info(h, c, c.b2, 0, &inf);
    return finish(done_status(h, c, maxc));
}

ffmg_status mg_solve(ffmg_handle *h, const void *bv, void *uv, double tol, ffmg_solve_info *info)
{
    if (!h || !uv) return fail(h, FFMG_EINVAL, "null argument");
    NOT_PENDING(h);
    if (h->opt.smoother == FFMG_SMOOTH_LEARNED) return solve_host_controlled(h, bv, uv, tol, info);
    TRY(mg_solve_begin(h, bv, uv, tol));
    return mg_solve_end(h, info);
}

// Validation, the plane-wave factors and the far-field plan for n_dirs
// directions; then the integrand (inside the PROF_FF bracket started here).
static ffmg_status ff_check_args(ffmg_handle *h, const double eta[3], int n_dirs, const double *dirs, int ff_prec)
{
    if (!h || !eta || !dirs || n_dirs < 1) return fail(h, FFMG_EINVAL, "null argument or n_dirs < 1");
    if (!(h->k0 > 0.0)) return fail(h, FFMG_EINVAL, "the far field needs an incoming plane wave (E > 0)");
    const int d = h->prob.dim;
    for (int i = 0; i < n_dirs; ++i) {
        double s = 0.0;
        for (int k = 0; k < d; ++k) {
            double a = dirs[(size_t)i * d + k];
            if (!isfinite(a)) return fail(h, FFMG_EINVAL, "direction %d is not finite", i);
            s += a * a;
        }
        if (fabs(s - 1.0) > 1e-6) return fail(h, FFMG_EINVAL, "direction %d is not a unit vector", i);
    }
    // the integrand multiplies exp(+k0 sin g alpha.x) by exp(-k0 sin g eta.x);
    // the split BF16 contraction forms that product in FP32
    if (2.0 * exponent_budget(h) > 700.0)
        return fail(h, FFMG_ERANGE, "contour exponentials exceed the FP64 range on this box");
    if (ff_prec != FFMG_FF_FP64 && 2.0 * exponent_budget(h) > 60.0)
        return fail(h, FFMG_ERANGE, "contour exponentials exceed the FP32 range of the split BF16 contraction");
    return FFMG_OK;
}

static ffmg_status ff_begin(ffmg_handle *h, const double eta[3], const void *u, int n_dirs, const double *dirs,
                            int *prof_idx)
{
    TRY(ff_check_args(h, eta, n_dirs, dirs, h ? h->opt.ff_precision : FFMG_FF_FP64));
    const int d = h->prob.dim;
    Level &l0 = h->L[0];
    const LevelGeom &g = l0.g;
    if (!h->d_E) TRY(dalloc(h, &h->d_E, (size_t)(g.m[0] + g.m[1] + g.m[2]) * sizeof(cd)));
    if (!h->ff) {
        h->ff = ff_plan_create();
        ff_plan_set_variant(h->ff, h->ff_variant);
    }
    // plane-wave axis factors exp(i k0 e^{ig} eta_k x): c = -k0 sin g eta_k + i k0 cos g eta_k
    int off = 0;
    for (int k = 0; k < 3; ++k) {
        double ek = (k < d) ? eta[k] : 0.0;
        launch_axis_exp(h->d_E + off, g.m[k], g.lo[k], g.h[k], -(h->k0 * sin(h->prob.gamma)) * ek,
                        (h->k0 * cos(h->prob.gamma)) * ek, h->stream);
        off += g.m[k];
    }
    HIPCHK(h, hipGetLastError());
    HIPCHK(h, ff_plan_prepare(h->ff, g, h->k0, h->prob.gamma, n_dirs, dirs, h->opt.ff_precision, h->stream));
    *prof_idx = prof_begin(h, PROF_FF);
    HIPCHK(h, ff_plan_integrand(h->ff, g, l0.q, (const cd *)u, h->d_E, h->stream));
    return FFMG_OK;
}

}  // extern "C"

namespace ffmg {

// Validation and the plan for the directions, without the map (the batched
// far field runs the stages itself).
ffmg_status farfield_prepare(ffmg_handle *h, const double eta[3], int n_dirs, const double *dirs)
{
    TRY(ff_check_args(h, eta, n_dirs, dirs, h ? h->opt.ff_precision : FFMG_FF_FP64));
    if (!h->ff) {
        h->ff = ff_plan_create();
        ff_plan_set_variant(h->ff, h->ff_variant);
    }
    HIPCHK(h, ff_plan_prepare(h->ff, h->L[0].g, h->k0, h->prob.gamma, n_dirs, dirs, h->opt.ff_precision, h->stream));
    return FFMG_OK;
}

ffmg_status farfield_enqueue(ffmg_handle *h, const double eta[3], const void *u, int n_dirs, const double *dirs,
                             cd *Fd)
{
    int pi = -1;
    TRY(ff_begin(h, eta, u, n_dirs, dirs, &pi));
    const LevelGeom &g = h->L[0].g;
    int pg = prof_begin(h, PROF_FFGEMM);
    HIPCHK(h, ff_plan_contract(h->ff, g, h->stream));
    prof_end(h, PROF_FFGEMM, pg);
    HIPCHK(h, ff_plan_finish(h->ff, g, h->prob.gamma, Fd, h->stream));
    prof_end(h, PROF_FF, pi);
    return FFMG_OK;
}

}  // namespace ffmg

extern "C" {

ffmg_status farfield_map(ffmg_handle *h, const double eta[3], const void *u, int n_dirs, const double *dirs,
                         void *F)
{
    NOT_PENDING(h);
    if (!F) return fail(h, FFMG_EINVAL, "F is null");
    // output: device pointer directly, host pointer through a staging buffer
    hipPointerAttribute_t attr;
    bool on_device = false;
    if (hipPointerGetAttributes(&attr, F) == hipSuccess)
        on_device = (attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged);
    else
        (void)hipGetLastError();
    cd *Fd = (cd *)F;
    if (!on_device && h && n_dirs > 0) {
        if (h->d_F_cap < n_dirs) {
            TRY(dalloc(h, &h->d_F, (size_t)n_dirs * sizeof(cd)));
            h->d_F_cap = n_dirs;
        }
        Fd = h->d_F;
    }
    TRY(farfield_enqueue(h, eta, u, n_dirs, dirs, Fd));
    if (!on_device) {
        HIPCHK(h, hipMemcpyAsync(F, Fd, (size_t)n_dirs * sizeof(cd), hipMemcpyDeviceToHost, h->stream));
        HIPCHK(h, hipStreamSynchronize(h->stream));
    } else {
        HIPCHK(h, hipGetLastError());   // device output: the work stays queued on the handle's stream
    }
    return FFMG_OK;
}

ffmg_status farfield_map_noalloc(ffmg_handle *h, const double eta[3], const void *u, int n_dirs,
                                 const double *dirs, void *F)
{
    NOT_PENDING(h);
    if (!F) return fail(h, FFMG_EINVAL, "F is null");
    TRY(ff_check_args(h, eta, n_dirs, dirs, FFMG_FF_FP64));
    if (n_dirs > FFMG_NOALLOC_MAX_DIRS)
        return fail(h, FFMG_EINVAL, "n_dirs = %d exceeds FFMG_NOALLOC_MAX_DIRS (%d)", n_dirs, FFMG_NOALLOC_MAX_DIRS);
    hipPointerAttribute_t attr;
    bool on_device = false;
    if (hipPointerGetAttributes(&attr, F) == hipSuccess)
        on_device = (attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged);
    else
        (void)hipGetLastError();
    const Level &l0 = h->L[0];
    size_t need = 0;
    hipError_t he = hipSuccess;
    const int rc = ff_noalloc_map(l0.g, h->k0, h->prob.gamma, eta, l0.q, (const cd *)u, n_dirs, dirs, (cd *)F,
                                  on_device, h->device, h->stream, &need, &he);
    switch (rc) {
    case 0: return FFMG_OK;
    case 1:
        return fail(h, FFMG_EINVAL, "the map needs %zu bytes of scratch, more than FFMG_NOALLOC_SCRATCH_BYTES (%zu)",
                    need, (size_t)FFMG_NOALLOC_SCRATCH_BYTES);
    case 2: return fail(h, FFMG_EDEVICE, "the scratch array was not set up on device %d", h->device);
    case 3: return fail(h, FFMG_EINVAL, "n_dirs out of range");
    default:
        return fail(h, he == hipErrorOutOfMemory ? FFMG_ENOMEM : FFMG_EDEVICE, "farfield_map_noalloc: %s",
                    hipGetErrorString(he));
    }
}

}  // extern "C"

namespace {
// Re-plans both tails for variant v; batched workspaces built for the old
// tail are rebuilt (they are keyed by the handle serial).
void set_tail_variant(ffmg_handle *h, int v)
{
    if (v == h->tail_variant) return;
    h->tail_variant = v;
    plan_tail<double>(h, h->tail64, h->tail_lds[0]);
    if (h->opt.precision == FFMG_FP32_IR) plan_tail<float>(h, h->tail32, h->tail_lds[1]);
    h->serial = next_handle_serial();
}
}  // namespace

extern "C" {

int mg_tune_variants(const ffmg_handle *h, int tunable)
{
    if (!h) return 0;
    switch (tunable) {
    case FFMG_TUNE_FF_GEMM: return (h->opt.ff_precision == FFMG_FF_FP64) ? 1 : ff_plan_variants();
    case FFMG_TUNE_TAIL:
        return (h->prob.dim == 2 && h->opt.tile_config == TILE_FUSED && h->opt.smoother != FFMG_SMOOTH_LEARNED &&
                h->tail64.nt > 0)
                   ? TAIL_VARIANTS
                   : 1;
    case FFMG_TUNE_SMOOTH:
        return (h->prob.dim == 2 && h->opt.tile_config != TILE_REFERENCE) ? SMOOTH_VARIANTS : 1;
    case FFMG_TUNE_PRE: return (h->prob.dim == 2 && h->opt.tile_config != TILE_REFERENCE) ? 3 : 1;
    case FFMG_TUNE_SMOOTH_COARSE:
        return (h->prob.dim == 2 && h->opt.tile_config != TILE_REFERENCE) ? SMOOTH_VARIANTS : 1;
    case FFMG_TUNE_SWEEP3D: return (h->prob.dim == 3 && h->opt.tile_config != TILE_REFERENCE) ? 5 : 1;
    case FFMG_TUNE_BATCH:
        return (h->prob.dim == 2 && h->opt.precision == FFMG_FP32_IR && h->opt.tile_config == TILE_FUSED)
                   ? BATCH_TUNE_VARIANTS
                   : 1;
    default: return 0;
    }
}

ffmg_status mg_tune_get(const ffmg_handle *h, int tunable, int *variant)
{
    if (!h || !variant) return FFMG_EINVAL;
    switch (tunable) {
    case FFMG_TUNE_FF_GEMM:
        *variant = (h->opt.ff_precision == FFMG_FF_FP64) ? 0
                   : (h->ff_variant < 0)                 ? ff_plan_default_variant()
                                                         : h->ff_variant;
        return FFMG_OK;
    case FFMG_TUNE_TAIL: *variant = h->tail_variant; return FFMG_OK;
    case FFMG_TUNE_SMOOTH: *variant = h->smooth_variant; return FFMG_OK;
    case FFMG_TUNE_PRE: *variant = h->pre_variant; return FFMG_OK;
    case FFMG_TUNE_SMOOTH_COARSE: *variant = h->smooth_coarse_variant; return FFMG_OK;
    case FFMG_TUNE_SWEEP3D: *variant = h->sweep3d_variant; return FFMG_OK;
    case FFMG_TUNE_BATCH: *variant = h->batch_variant; return FFMG_OK;
    default: return FFMG_EINVAL;
    }
}

ffmg_status mg_tune_set(ffmg_handle *h, int tunable, int variant)
{
    NOT_PENDING(h);
    if (!h) return FFMG_EINVAL;
    if (variant < 0 || variant >= mg_tune_variants(h, tunable))
        return fail(h, FFMG_EINVAL, "variant %d out of range for tunable %d", variant, tunable);
    switch (tunable) {
    case FFMG_TUNE_FF_GEMM:
        if (h->opt.ff_precision == FFMG_FF_FP64) return FFMG_OK;
        h->ff_variant = variant;
        if (h->ff) ff_plan_set_variant(h->ff, variant);
        return FFMG_OK;
    case FFMG_TUNE_TAIL: set_tail_variant(h, variant); return FFMG_OK;
    case FFMG_TUNE_SMOOTH: h->smooth_variant = variant; return FFMG_OK;
    case FFMG_TUNE_PRE: h->pre_variant = variant; return FFMG_OK;
    case FFMG_TUNE_SMOOTH_COARSE: h->smooth_coarse_variant = variant; return FFMG_OK;
    case FFMG_TUNE_SWEEP3D: h->sweep3d_variant = variant; return FFMG_OK;
    case FFMG_TUNE_BATCH: h->batch_variant = variant; return FFMG_OK;
    default: return fail(h, FFMG_EINVAL, "unknown tunable %d", tunable);
    }
}

ffmg_status mg_tune_farfield(ffmg_handle *h, const double eta[3], const void *u, int n_dirs, const double *dirs,
                             int reps, double *times_ms, int n_times, int *best)
{
    NOT_PENDING(h);
    if (!h || reps < 1) return fail(h, FFMG_EINVAL, "null handle or reps < 1");
    int pi = -1;
    TRY(ff_begin(h, eta, u, n_dirs, dirs, &pi));
    prof_end(h, PROF_FF, pi);
    const LevelGeom &g = h->L[0].g;
    const int nv = mg_tune_variants(h, FFMG_TUNE_FF_GEMM);
    hipEvent_t e0, e1;
    HIPCHK(h, hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(h, FFMG_EDEVICE, "hipEventCreate failed");
    }
    int arg = 0;
    double tbest = 0.0;
    ffmg_status st = FFMG_OK;
    for (int v = 0; v < nv && st == FFMG_OK; ++v) {
        ff_plan_set_variant(h->ff, v);
        hipError_t e = ff_plan_contract(h->ff, g, h->stream);   // warm-up
        if (e == hipSuccess) e = hipEventRecord(e0, h->stream);
        for (int r = 0; r < reps && e == hipSuccess; ++r) e = ff_plan_contract(h->ff, g, h->stream);
        if (e == hipSuccess) e = hipEventRecord(e1, h->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) {
            st = fail(h, FFMG_EDEVICE, "variant %d: %s", v, hipGetErrorString(e));
            break;
        }
        double t = ms / reps;
        if (times_ms && v < n_times) times_ms[v] = t;
        if (v == 0 || t < tbest) {
            tbest = t;
            arg = v;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != FFMG_OK) return st;
    if (nv > 1) {
        h->ff_variant = arg;
        ff_plan_set_variant(h->ff, arg);
    }
    if (best) *best = arg;
    return FFMG_OK;
}

ffmg_status mg_tune_solve(ffmg_handle *h, int tunable, const void *b, void *u, double tol, int reps, double *times_ms,
                          int n_times, int *best)
{
    NOT_PENDING(h);
    if (!h || !b || !u || reps < 1) return fail(h, FFMG_EINVAL, "null argument or reps < 1");
    if (tunable != FFMG_TUNE_TAIL && tunable != FFMG_TUNE_SMOOTH && tunable != FFMG_TUNE_PRE &&
        tunable != FFMG_TUNE_SMOOTH_COARSE && tunable != FFMG_TUNE_SWEEP3D)
        return fail(h, FFMG_EINVAL, "mg_tune_solve tunes the solve's tunables (got %d)", tunable);
    const int nv = mg_tune_variants(h, tunable);
    const size_t bytes = h->L[0].g.N() * sizeof(cd);
    int arg = 0;
    TRY(mg_tune_get(h, tunable, &arg));
    double tbest = 0.0;
    for (int v = 0; v < nv; ++v) {
        TRY(mg_tune_set(h, tunable, v));
        double t = 0.0;
        for (int r = 0; r <= reps; ++r) {
            HIPCHK(h, hipMemsetAsync(u, 0, bytes, h->stream));
            ffmg_solve_info inf{};
            ffmg_status st = mg_solve(h, b, u, tol, &inf);
            if (st != FFMG_OK) return st;
            if (r > 0) t += inf.t_solve_ms;
        }
        t /= reps;
        if (times_ms && v < n_times) times_ms[v] = t;
        if (v == 0 || t < tbest) {
            tbest = t;
            arg = v;
        }
    }
    TRY(mg_tune_set(h, tunable, arg));
    if (best) *best = arg;
    return FFMG_OK;
}

}  // extern "C"
