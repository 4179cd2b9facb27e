// ffmg_capi.hip -- the handle, the multigrid driver and the C ABI declared in
// include/ffmg.h.  Every arithmetic step runs in the library's HIP kernels;
// the host only sequences launches, reads back one residual norm per cycle
// and decides when to stop (Sec. 4: V-cycles to a residual-reduction
// tolerance).
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/ffmg.h"
#include "ffmg_internal.hpp"

using namespace ffmg;

namespace {

struct Level {
    LevelGeom g;
    Stencil<double> P64;
    Stencil<float> P32;
    cd *q = nullptr;                 // contrast on this level
    cd *u = nullptr, *b = nullptr;   // coarse correction / rhs (levels >= 1)
    cd *r = nullptr, *t = nullptr;   // residual, ping-pong buffer
    cf *q32 = nullptr;               // FP32 copies for the refinement inner cycle
    cf *u32 = nullptr, *b32 = nullptr, *r32 = nullptr, *t32 = nullptr;
};

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

}  // namespace

struct ffmg_handle {
    ffmg_problem prob{};
    ffmg_options opt{};
    double k0 = 0.0, k02 = 0.0;
    std::vector<Level> L;
    cd *aug = nullptr;               // [A_c | A_c^{-1}] of the coarsest level
    int nc = 0;
    int *d_info = nullptr;
    double *d_parts = nullptr;       // per-block partial sums
    int nparts = 0;
    double *d_scalar = nullptr;
    double *h_scalar = nullptr;      // pinned
    hipStream_t stream = nullptr;
    FarFieldPlan *ff = nullptr;
    cd *d_s = nullptr;               // far-field integrand
    cd *d_E = nullptr;               // plane-wave axis factors
    cd *d_F = nullptr;               // far-field staging
    int d_F_cap = 0;
    std::vector<void *> allocs;
    std::string err;
    // optional event timing of selected kernels (benchmark instrumentation)
    bool profile = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[2];
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_free;
};

namespace {

// Record the start of a timed launch of kernel id k (no-op unless enabled).
int prof_begin(ffmg_handle *h, int k)
{
    if (!h->profile) return -1;
    std::pair<hipEvent_t, hipEvent_t> e;
    if (!h->ev_free.empty()) {
        e = h->ev_free.back();
        h->ev_free.pop_back();
    } else {
        if (hipEventCreate(&e.first) != hipSuccess || hipEventCreate(&e.second) != hipSuccess) return -1;
    }
    (void)hipEventRecord(e.first, h->stream);
    h->ev[k].push_back(e);
    return (int)h->ev[k].size() - 1;
}

void prof_end(ffmg_handle *h, int k, int idx)
{
    if (idx < 0) return;
    (void)hipEventRecord(h->ev[k][idx].second, h->stream);
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

#define HIPCHK(h, x)                                                                                               \
    do {                                                                                                           \
        hipError_t e_ = (x);                                                                                       \
        if (e_ != hipSuccess)                                                                                      \
            return fail((h), e_ == hipErrorOutOfMemory ? FFMG_ENOMEM : FFMG_EDEVICE, "%s: %s (%s:%d)", #x,         \
                        hipGetErrorString(e_), __FILE__, __LINE__);                                                \
    } while (0)

template <typename P>
ffmg_status dalloc(ffmg_handle *h, P **p, size_t bytes)
{
    void *v = nullptr;
    hipError_t e = hipMalloc(&v, bytes ? bytes : 16);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(h, FFMG_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    }
    h->allocs.push_back(v);
    *p = (P *)v;
    return FFMG_OK;
}

#define TRY(x)                                                                                                     \
    do {                                                                                                           \
        ffmg_status s_ = (x);                                                                                      \
        if (s_ != FFMG_OK) return s_;                                                                              \
    } while (0)

// Sum of the first n partials -> host double (synchronises the stream).
ffmg_status reduce_to_host(ffmg_handle *h, int n, double *out)
{
    launch_sum(h->d_parts, n, h->d_scalar, h->stream);
    HIPCHK(h, hipMemcpyAsync(h->h_scalar, h->d_scalar, sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    *out = *h->h_scalar;
    return FFMG_OK;
}

__global__ __launch_bounds__(256) void k_norm2(const cd *__restrict__ v, size_t N, double *__restrict__ parts)
{
    __shared__ double red[4];
    double acc = 0.0;
    for (size_t j = (size_t)blockIdx.x * 256 + threadIdx.x; j < N; j += (size_t)gridDim.x * 256) acc += abs2(v[j]);
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) parts[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

ffmg_status norm2_of(ffmg_handle *h, const cd *v, size_t N, double *out)
{
    int nb = (int)std::min<size_t>((N + 255) / 256, 1024);
    hipLaunchKernelGGL(k_norm2, dim3(nb), dim3(256), 0, h->stream, v, N, h->d_parts);
    HIPCHK(h, hipGetLastError());
    double s2;
    TRY(reduce_to_host(h, nb, &s2));
    *out = sqrt(s2);
    return FFMG_OK;
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
};
template <>
struct LvlPtr<float> {
    static cf *q(Level &l) { return l.q32; }
    static cf *u(Level &l) { return l.u32; }
    static cf *b(Level &l) { return l.b32; }
    static cf *r(Level &l) { return l.r32; }
    static cf *t(Level &l) { return l.t32; }
    static const Stencil<float> &P(Level &l) { return l.P32; }
};

// nu weighted-Jacobi sweeps in place on u (ping-pong through t).  With
// zero_guess the incoming u is taken as 0 without being read.
template <typename T>
void smooth(ffmg_handle *h, Level &lv, const cx<T> *b, cx<T> *u, int nu, bool zero_guess)
{
    using LP = LvlPtr<T>;
    cx<T> *t = LP::t(lv);
    const cx<T> *q = LP::q(lv);
    const Stencil<T> &P = LP::P(lv);
    cx<T> *src = u, *dst = t;
    const bool finest = (&lv == &h->L[0]);
    for (int s = 0; s < nu; ++s) {
        int mode = (s == 0 && zero_guess) ? MODE_JACOBI0 : MODE_JACOBI;
        int pi = (finest && mode == MODE_JACOBI) ? prof_begin(h, 0) : -1;
        launch_stencil<T>(mode, lv.g, P, src, b, q, dst, nullptr, h->stream, finest);
        prof_end(h, 0, pi);
        std::swap(src, dst);
    }
    if (src != u) (void)hipMemcpyAsync(u, src, lv.g.N() * sizeof(cx<T>), hipMemcpyDeviceToDevice, h->stream);
}

// One V(nu1, nu2) cycle on level l (Sec. 4): smoothing, restriction of the
// residual, coarse correction (exact on the coarsest level), interpolation,
// smoothing.
template <typename T>
void vcycle(ffmg_handle *h, int l, const cx<T> *b, cx<T> *u, bool zero_guess)
{
    using LP = LvlPtr<T>;
    Level &lv = h->L[l];
    const int last = (int)h->L.size() - 1;
    if (l == last) {
        launch_coarse_apply<T>(h->aug, h->nc, b, u, h->stream);
        return;
    }
    const int nu1 = h->opt.nu1, nu2 = h->opt.nu2;
    if (nu1 > 0) smooth<T>(h, lv, b, u, nu1, zero_guess);
    else if (zero_guess) (void)hipMemsetAsync(u, 0, lv.g.N() * sizeof(cx<T>), h->stream);
    launch_stencil<T>(MODE_RESID, lv.g, LP::P(lv), u, b, LP::q(lv), LP::r(lv), nullptr, h->stream);
    Level &lc = h->L[l + 1];
    launch_restrict<T>(lv.g, LP::r(lv), LP::b(lc), h->stream);
    vcycle<T>(h, l + 1, LP::b(lc), LP::u(lc), true);
    launch_prolong_add<T>(lv.g, LP::u(lc), u, h->stream);
    if (nu2 > 0) smooth<T>(h, lv, b, u, nu2, false);
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
        if (!(p->energy > 0.0) || !isfinite(p->energy))
            return fail(tmp, FFMG_EINVAL, "energy must be positive (scattering regime)");
    } else {
        return fail(tmp, FFMG_EINVAL, "unknown problem kind %d", p->kind);
    }
    if (!p->coef) return fail(tmp, FFMG_EINVAL, "coef is null");
    if (o->nu1 < 0 || o->nu2 < 0 || o->nu1 + o->nu2 < 1 || o->nu1 > 64 || o->nu2 > 64)
        return fail(tmp, FFMG_EINVAL, "need 0 <= nu1, nu2 <= 64 and nu1 + nu2 >= 1");
    if (!(o->omega > 0.0 && o->omega <= 1.0)) return fail(tmp, FFMG_EINVAL, "omega must lie in (0, 1]");
    if (o->max_cycles < 1) return fail(tmp, FFMG_EINVAL, "max_cycles must be >= 1");
    if (o->precision != FFMG_FP64 && o->precision != FFMG_FP32_IR)
        return fail(tmp, FFMG_EINVAL, "unknown precision %d", o->precision);
    if (o->smoother != FFMG_SMOOTH_JACOBI) return fail(tmp, FFMG_EINVAL, "unsupported smoother %d", o->smoother);
    if (o->ff_precision != FFMG_FF_FP64)
        return fail(tmp, FFMG_EINVAL, "unsupported far-field precision %d", o->ff_precision);
    return FFMG_OK;
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

ffmg_status setup_impl(ffmg_handle *h)
{
    const ffmg_problem &p = h->prob;
    HIPCHK(h, hipGetLastError());
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
        TRY(dalloc(h, &lv.q, N * sizeof(cd)));
        TRY(dalloc(h, &lv.r, N * sizeof(cd)));
        TRY(dalloc(h, &lv.t, N * sizeof(cd)));
        if (l > 0) {
            TRY(dalloc(h, &lv.u, N * sizeof(cd)));
            TRY(dalloc(h, &lv.b, N * sizeof(cd)));
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
    TRY(dalloc(h, &h->d_parts, maxparts * sizeof(double)));
    TRY(dalloc(h, &h->d_scalar, sizeof(double)));
    TRY(dalloc(h, &h->d_info, sizeof(int)));
    HIPCHK(h, hipHostMalloc((void **)&h->h_scalar, sizeof(double), hipHostMallocDefault));

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
    launch_gauss_jordan(h->aug, h->nc, h->d_info, h->stream);
    HIPCHK(h, hipGetLastError());
    int info = 0;
    HIPCHK(h, hipMemcpyAsync(&info, h->d_info, sizeof(int), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    if (info != 0) return fail(h, FFMG_EINVAL, "coarsest operator is singular (zero pivot in column %d)", info - 1);
    return FFMG_OK;
}

}  // namespace

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
    ffmg_status st = validate_problem(p, o, h);
    if (st == FFMG_OK) {
        h->prob = *p;
        h->opt = *o;
        h->stream = (hipStream_t)o->stream;
        if (p->kind == FFMG_SCHRODINGER) {
            h->k02 = 2.0 * p->energy;
            h->k0 = sqrt(h->k02);
        } else {
            h->k0 = p->k0;
            h->k02 = p->k0 * p->k0;
        }
        st = setup_impl(h);
    }
    if (st != FFMG_OK) {
        // keep the message on stderr-free path: the caller gets only the code
        mg_destroy(h);
        return st;
    }
    *out = h;
    return FFMG_OK;
}

ffmg_status mg_profile_enable(ffmg_handle *h, int enable)
{
    if (!h) return FFMG_EINVAL;
    h->profile = enable != 0;
    return FFMG_OK;
}

ffmg_status mg_profile_read(ffmg_handle *h, int kernel, double *total_ms, int64_t *count)
{
    if (!h || kernel < 0 || kernel > 1 || !total_ms || !count) return fail(h, FFMG_EINVAL, "bad argument");
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

void mg_destroy(ffmg_handle *h)
{
    if (!h) return;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    else (void)hipDeviceSynchronize();
    for (int k = 0; k < 2; ++k)
        for (auto &e : h->ev[k]) h->ev_free.push_back(e);
    for (auto &e : h->ev_free) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    if (h->ff) ff_plan_destroy(h->ff);
    for (void *p : h->allocs) (void)hipFree(p);
    if (h->h_scalar) (void)hipHostFree(h->h_scalar);
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
    if (!h || !eta || !b) return fail(h, FFMG_EINVAL, "null argument");
    double e[3] = {0, 0, 0};
    for (int k = 0; k < h->prob.dim; ++k) e[k] = eta[k];
    if (exponent_budget(h) > 700.0) return fail(h, FFMG_ERANGE, "exp(i k0 eta.z) overflows double on this box");
    launch_rhs_plane_wave(h->L[0].g, h->prob.gamma, h->k0, e, h->L[0].q, (cd *)b, h->stream);
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
    if (!h || !b || !u || !u_out || u == u_out) return fail(h, FFMG_EINVAL, "null or aliased argument");
    Level &l0 = h->L[0];
    launch_stencil<double>(MODE_JACOBI, l0.g, l0.P64, (const cd *)u, (const cd *)b, l0.q, (cd *)u_out, nullptr,
                           h->stream);
    HIPCHK(h, hipGetLastError());
    return FFMG_OK;
}

ffmg_status mg_residual_norm(ffmg_handle *h, const void *b, const void *u, double *rnorm)
{
    if (!h || !b || !u || !rnorm) return fail(h, FFMG_EINVAL, "null argument");
    return resid_norm(h, (const cd *)b, (const cd *)u, rnorm);
}

ffmg_status mg_vcycle(ffmg_handle *h, const void *b, void *u)
{
    if (!h || !b || !u) return fail(h, FFMG_EINVAL, "null argument");
    vcycle<double>(h, 0, (const cd *)b, (cd *)u, false);
    HIPCHK(h, hipGetLastError());
    return FFMG_OK;
}

ffmg_status mg_solve(ffmg_handle *h, const void *bv, void *uv, double tol, ffmg_solve_info *info)
{
    if (!h || !bv || !uv) return fail(h, FFMG_EINVAL, "null argument");
    if (!(tol > 0.0) || !(tol < 1.0)) return fail(h, FFMG_EINVAL, "tol must lie in (0, 1)");
    const cd *b = (const cd *)bv;
    cd *u = (cd *)uv;
    ffmg_solve_info inf{};
    hipEvent_t e0, e1;
    HIPCHK(h, hipEventCreate(&e0));
    HIPCHK(h, hipEventCreate(&e1));
    HIPCHK(h, hipEventRecord(e0, h->stream));
    Level &l0 = h->L[0];
    const size_t N = l0.g.N();
    ffmg_status st = FFMG_OK;
    double bn = 0.0, r0 = 0.0, rk = 0.0;
    auto finish = [&](ffmg_status s) {
        (void)hipEventRecord(e1, h->stream);
        (void)hipEventSynchronize(e1);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        inf.status = s;
        inf.t_solve_ms = ms;
        inf.rel_residual = bn > 0 ? rk / bn : 0.0;
        inf.conv_factor = (inf.cycles > 0 && r0 > 0) ? pow(rk / r0, 1.0 / inf.cycles) : 0.0;
        if (info) *info = inf;
        return s;
    };
    if ((st = norm2_of(h, b, N, &bn)) != FFMG_OK) return finish(st);
    if (bn == 0.0) {
        (void)hipMemsetAsync(u, 0, N * sizeof(cd), h->stream);
        return finish(FFMG_OK);
    }
    if (!isfinite(bn)) return finish(fail(h, FFMG_ENAN, "right-hand side holds non-finite values"));
    int grow = 0;
    if (h->opt.precision == FFMG_FP64) {
        if ((st = resid_norm(h, b, u, &r0)) != FFMG_OK) return finish(st);
        rk = r0;
        double prev = r0;
        if (r0 / bn <= tol) return finish(FFMG_OK);
        for (int k = 1; k <= h->opt.max_cycles; ++k) {
            vcycle<double>(h, 0, b, u, false);
            if ((st = resid_norm(h, b, u, &rk)) != FFMG_OK) return finish(st);
            inf.cycles = k;
            if (!isfinite(rk)) return finish(fail(h, FFMG_ENOCONV, "residual became non-finite at cycle %d", k));
            if (rk / bn <= tol) return finish(FFMG_OK);
            grow = (rk >= prev) ? grow + 1 : 0;
            if (grow >= 3) return finish(fail(h, FFMG_ENOCONV, "residual grew on 3 consecutive cycles"));
            prev = rk;
        }
        return finish(fail(h, FFMG_ENOCONV, "no convergence in %d cycles", h->opt.max_cycles));
    }
    // FP32 V-cycles inside FP64 iterative refinement.  The FP64 residual is
    // written as FP32 scaled by the previous residual's rms value, the FP32
    // cycle solves for the scaled correction, the update is applied in FP64.
    const double sqN = sqrt((double)N);
    double scale = bn / sqN;
    double s2;
    launch_resid_to_f32(l0.g, l0.P64, u, b, l0.q, l0.b32, 1.0 / scale, h->d_parts, h->stream);
    if ((st = reduce_to_host(h, stencil_blocks(l0.g), &s2)) != FFMG_OK) return finish(st);
    r0 = rk = sqrt(s2);
    if (r0 / bn <= tol) return finish(FFMG_OK);
    double prev = r0;
    for (int k = 1; k <= h->opt.max_cycles; ++k) {
        vcycle<float>(h, 0, l0.b32, l0.u32, true);
        launch_refine_update(l0.u32, u, scale, N, h->stream);
        scale = rk / sqN;
        launch_resid_to_f32(l0.g, l0.P64, u, b, l0.q, l0.b32, 1.0 / scale, h->d_parts, h->stream);
        if ((st = reduce_to_host(h, stencil_blocks(l0.g), &s2)) != FFMG_OK) return finish(st);
        rk = sqrt(s2);
        inf.cycles = k;
        if (!isfinite(rk)) return finish(fail(h, FFMG_ENOCONV, "residual became non-finite at step %d", k));
        if (rk / bn <= tol) return finish(FFMG_OK);
        grow = (rk >= prev) ? grow + 1 : 0;
        if (grow >= 3) return finish(fail(h, FFMG_ENOCONV, "residual grew on 3 consecutive steps"));
        prev = rk;
    }
    return finish(fail(h, FFMG_ENOCONV, "no convergence in %d refinement steps", h->opt.max_cycles));
}

ffmg_status farfield_map(ffmg_handle *h, const double eta[3], const void *u, int n_dirs, const double *dirs,
                         void *F)
{
    if (!h || !eta || !dirs || !F || n_dirs < 1) return fail(h, FFMG_EINVAL, "null argument or n_dirs < 1");
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
    // the integrand multiplies exp(+k0 sin g alpha.x) by exp(-k0 sin g eta.x)
    if (2.0 * exponent_budget(h) > 700.0)
        return fail(h, FFMG_ERANGE, "contour exponentials exceed the FP64 range on this box");
    Level &l0 = h->L[0];
    const LevelGeom &g = l0.g;
    const size_t N = g.N();
    if (!h->d_s) TRY(dalloc(h, &h->d_s, N * sizeof(cd)));
    if (!h->d_E) TRY(dalloc(h, &h->d_E, (size_t)(g.m[0] + g.m[1] + g.m[2]) * sizeof(cd)));
    if (!h->ff) h->ff = ff_plan_create();
    // plane-wave axis factors exp(i k0 e^{ig} eta_k x): c = -k0 sin g eta_k + i k0 cos g eta_k
    int off = 0;
    for (int k = 0; k < 3; ++k) {
        double ek = (k < d) ? eta[k] : 0.0;
        launch_axis_exp(h->d_E + off, g.m[k], g.lo[k], g.h[k], -(h->k0 * sin(h->prob.gamma)) * ek,
                        (h->k0 * cos(h->prob.gamma)) * ek, h->stream);
        off += g.m[k];
    }
    launch_ff_integrand(g, l0.q, (const cd *)u, h->d_E, h->d_s, h->stream);
    HIPCHK(h, hipGetLastError());
    HIPCHK(h, ff_plan_prepare(h->ff, g, h->k0, h->prob.gamma, n_dirs, dirs, h->d_s, h->stream));
    // output: device pointer directly, host pointer through a staging buffer
    hipPointerAttribute_t attr;
    bool on_device = false;
    if (hipPointerGetAttributes(&attr, F) == hipSuccess)
        on_device = (attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged);
    else
        (void)hipGetLastError();
    cd *Fd = (cd *)F;
    if (!on_device) {
        if (h->d_F_cap < n_dirs) {
            TRY(dalloc(h, &h->d_F, (size_t)n_dirs * sizeof(cd)));
            h->d_F_cap = n_dirs;
        }
        Fd = h->d_F;
    }
    int pi = prof_begin(h, 1);
    HIPCHK(h, ff_plan_execute(h->ff, g, h->prob.gamma, Fd, h->stream));
    prof_end(h, 1, pi);
    if (!on_device)
        HIPCHK(h, hipMemcpyAsync(F, Fd, (size_t)n_dirs * sizeof(cd), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return FFMG_OK;
}

}  // extern "C"
