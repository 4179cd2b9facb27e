// ffmg_learned.hip -- the learned smoother: a three-layer 3x3 complex
// convolutional network that replaces the weighted-Jacobi sweeps of the
// finest level (the paper smooths with weighted Jacobi, Sec. 4, and notes
// that other smoothers can take its place).  One smoothing step is
//
//   u <- u + s h^2 N(r / s, kappa h^2) = u + h^2 N(r, kappa h^2),
//   r = b - A u,  s = RMS(r) (the training data are scaled by s),
//   N:  a = W1[., ., 0] * r~,  m = W1[., ., 1] * kappa~,  x1 = a (1 + m),
//       x2 = W2 * x1,  N = W3 * x2,
//
// with 1 + 1 -> 16 -> 16 -> 1 complex channels and 3x3 taps (tap t =
// 3 (dy + 1) + (dx + 1) reads the point (y + dy, x + dx); zero outside the
// grid).  N is complex-linear in r~ (a learned radius-3 stencil whose weights
// the coefficient gate 1 + m adapts), so the smoothing step is a linear
// iteration.  Weights and activations are stored in BF16, products are
// accumulated in FP32.
//
// Training (on patches of (residual, error) pairs from plain V-cycle
// iterates): loss = mean over the patch interior of |L5 (e~ - N)|^2 +
// LOSS_ALPHA max(0, ||e~ - N||^2 / ||e~||^2 - 1) with e~ = e / (s h^2) and
// L5 the 5-point Laplacian stencil (4, -1, -1, -1, -1): the high-frequency
// part of the error left by the smoothing step, plus a penalty on growth of
// the patch's error (smooth error, which L5 does not see, must not be
// amplified).  One
// workgroup per 32 x 32 patch runs the forward pass, the loss and the whole
// backward pass in LDS and writes that patch's weight gradient; a second
// kernel averages them over the minibatch in a fixed order; Adam updates the
// FP32 master weights and refreshes the BF16 copies.
//
// Complex gradients use g = dL/dRe + i dL/dIm; for y = W x this gives
// dL/dW = g_y conj(x) and g_x = conj(W) g_y.
#include <math.h>

#include "ffmg_internal.hpp"
#include "ffmg_learned.hpp"

#include <algorithm>

namespace ffmg {

typedef float f4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// BF16 helpers: round-to-nearest-even of a finite FP32, and complex values
// packed as (bf16 re) | (bf16 im) << 16.
__host__ __device__ __forceinline__ unsigned bf16_bits(float f)
{
    unsigned u = __builtin_bit_cast(unsigned, f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return u >> 16;
}
__host__ __device__ __forceinline__ float bf16_round(float f)
{
    return __builtin_bit_cast(float, bf16_bits(f) << 16);
}
__device__ __forceinline__ unsigned pack_c(float re, float im) { return bf16_bits(re) | (bf16_bits(im) << 16); }
__device__ __forceinline__ float2 unpack_c(unsigned v)
{
    return make_float2(__builtin_bit_cast(float, v << 16), __builtin_bit_cast(float, v & 0xFFFF0000u));
}

__device__ __forceinline__ void cmac(float2 &acc, float2 w, float2 x)
{
    acc.x = fmaf(w.x, x.x, acc.x);
    acc.x = fmaf(-w.y, x.y, acc.x);
    acc.y = fmaf(w.x, x.y, acc.y);
    acc.y = fmaf(w.y, x.x, acc.y);
}
// acc += conj(w) x
__device__ __forceinline__ void cmac_cw(float2 &acc, float2 w, float2 x)
{
    acc.x = fmaf(w.x, x.x, acc.x);
    acc.x = fmaf(w.y, x.y, acc.x);
    acc.y = fmaf(w.x, x.y, acc.y);
    acc.y = fmaf(-w.y, x.x, acc.y);
}
// acc += g conj(x)
__device__ __forceinline__ void cmac_cx(float2 &acc, float2 g, float2 x)
{
    acc.x = fmaf(g.x, x.x, acc.x);
    acc.x = fmaf(g.y, x.y, acc.x);
    acc.y = fmaf(g.y, x.x, acc.y);
    acc.y = fmaf(-g.x, x.y, acc.y);
}

__device__ __forceinline__ constexpr int tap_dy(int t) { return t / 3 - 1; }
__device__ __forceinline__ constexpr int tap_dx(int t) { return t % 3 - 1; }

// ---------------------------------------------------------------------------
// Training: one 256-thread workgroup per 32 x 32 patch.
constexpr float LOSS_ALPHA = 1.f;   // weight of the error-growth penalty
constexpr int TP = 32;              // patch side
constexpr int TPP = TP * TP;        // points per patch
constexpr int TPT = TPP / 256;      // points per thread

struct TrainLds {
    unsigned x0[TPP][2];            // inputs (r~, kappa~), BF16 complex
    unsigned x1[TPP][16];           // layer-1 output, later its gradient
    unsigned x2[TPP][16];           // layer-2 output, later its gradient
    float2 d[TPP];                  // e~ - N, later g_N
    float2 z[TPP];                  // mask L5 (e~ - N)
};

static_assert(offsetof(TrainLds, z) == offsetof(TrainLds, d) + sizeof(float2) * TPP,
              "d and z must be contiguous (used together as a partial-sum buffer)");

__device__ __forceinline__ bool in_patch(int y, int x) { return y >= 0 && y < TP && x >= 0 && x < TP; }

// a_o = sum_t W1[t][o][0] r~(p + d_t), m_o = sum_t W1[t][o][1] kappa~(p + d_t)
__device__ __forceinline__ void layer1_point(const TrainLds &S, const float2 *__restrict__ W1, int p, float2 (&a)[16],
                                             float2 (&m)[16])
{
    const int py = p / TP, px = p % TP;
    float2 x[9][2];
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        const int yy = py + tap_dy(t), xx = px + tap_dx(t);
        const bool in = in_patch(yy, xx);
        const int q = in ? yy * TP + xx : 0;
#pragma unroll
        for (int i = 0; i < 2; ++i) x[t][i] = in ? unpack_c(S.x0[q][i]) : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int o = 0; o < 16; ++o) {
        a[o] = make_float2(0.f, 0.f);
        m[o] = make_float2(0.f, 0.f);
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            cmac(a[o], W1[(t * 16 + o) * 2 + 0], x[t][0]);
            cmac(m[o], W1[(t * 16 + o) * 2 + 1], x[t][1]);
        }
    }
}

__global__ __launch_bounds__(256) void k_train_patch(const float2 *__restrict__ rt, const float2 *__restrict__ kt,
                                                     const float2 *__restrict__ et,
                                                     const float2 *__restrict__ W, float2 *__restrict__ dW_part,
                                                     float *__restrict__ loss_part, int border)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
    TrainLds &S = *reinterpret_cast<TrainLds *>(lds_raw);
    const float2 *W1 = W + NET_W1, *W2 = W + NET_W2, *W3 = W + NET_W3;
    const size_t base = (size_t)blockIdx.x * TPP;
    const int tid = threadIdx.x;
    // inputs, rounded to BF16
    for (int p = tid; p < TPP; p += 256) {
        float2 r = rt[base + p], k = kt[base + p];
        S.x0[p][0] = pack_c(r.x, r.y);
        S.x0[p][1] = pack_c(k.x, k.y);
    }
    __syncthreads();
    // layer 1: a (from r~) gated by 1 + m (from kappa~)
    for (int k = 0; k < TPT; ++k) {
        const int p = tid + 256 * k;
        float2 a[16], m[16];
        layer1_point(S, W1, p, a, m);
#pragma unroll
        for (int o = 0; o < 16; ++o) {
            const float cr = 1.f + m[o].x, ci = m[o].y;
            S.x1[p][o] = pack_c(a[o].x * cr - a[o].y * ci, a[o].x * ci + a[o].y * cr);
        }
    }
    __syncthreads();
    // layer 2: 16 -> 16
    {
        float2 acc[TPT][16];
#pragma unroll
        for (int k = 0; k < TPT; ++k)
#pragma unroll
            for (int o = 0; o < 16; ++o) acc[k][o] = make_float2(0.f, 0.f);
        for (int t = 0; t < 9; ++t) {
            float2 x[TPT][16];
#pragma unroll
            for (int k = 0; k < TPT; ++k) {
                const int p = tid + 256 * k, py = p / TP + tap_dy(t), px = p % TP + tap_dx(t);
                const bool in = in_patch(py, px);
                const int q = in ? py * TP + px : 0;
#pragma unroll
                for (int i = 0; i < 16; ++i) x[k][i] = in ? unpack_c(S.x1[q][i]) : make_float2(0.f, 0.f);
            }
#pragma unroll
            for (int o = 0; o < 16; ++o)
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    const float2 w = W2[(t * 16 + o) * 16 + i];
#pragma unroll
                    for (int k = 0; k < TPT; ++k) cmac(acc[k][o], w, x[k][i]);
                }
        }
#pragma unroll
        for (int k = 0; k < TPT; ++k) {
            const int p = tid + 256 * k;
#pragma unroll
            for (int o = 0; o < 16; ++o) S.x2[p][o] = pack_c(acc[k][o].x, acc[k][o].y);
        }
    }
    __syncthreads();
    // layer 3: 16 -> 1; d = e~ - N
    for (int k = 0; k < TPT; ++k) {
        const int p = tid + 256 * k, py = p / TP, px = p % TP;
        float2 y = make_float2(0.f, 0.f);
        for (int t = 0; t < 9; ++t) {
            const int yy = py + tap_dy(t), xx = px + tap_dx(t);
            if (!in_patch(yy, xx)) continue;
            const int q = yy * TP + xx;
#pragma unroll
            for (int i = 0; i < 16; ++i) cmac(y, W3[t * 16 + i], unpack_c(S.x2[q][i]));
        }
        const float2 e = et[base + p];
        S.d[p] = make_float2(e.x - y.x, e.y - y.y);
    }
    __syncthreads();
    // z = mask L5 d; loss; patch sums of |e~|^2 and |d|^2 for the growth penalty
    const int lo = border, hi = TP - border;
    const float cnt = (float)((hi - lo) * (hi - lo));
    float lsum = 0.f, esum = 0.f, dsum = 0.f;
    for (int k = 0; k < TPT; ++k) {
        const int p = tid + 256 * k, py = p / TP, px = p % TP;
        float2 z = make_float2(0.f, 0.f);
        if (py >= lo && py < hi && px >= lo && px < hi) {
            float2 c = S.d[p];
            z.x = 4.f * c.x;
            z.y = 4.f * c.y;
            const int nb[4][2] = {{0, -1}, {0, 1}, {-1, 0}, {1, 0}};
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const int yy = py + nb[m][0], xx = px + nb[m][1];
                if (in_patch(yy, xx)) {
                    float2 v = S.d[yy * TP + xx];
                    z.x -= v.x;
                    z.y -= v.y;
                }
            }
            lsum += z.x * z.x + z.y * z.y;
            const float2 e = et[base + p];
            esum += e.x * e.x + e.y * e.y;
            dsum += c.x * c.x + c.y * c.y;
        }
        S.z[p] = z;
    }
    __shared__ float red[3][4];
    __shared__ float tot[3];
    {
        float v[3] = {lsum, esum, dsum};
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            for (int off = 32; off > 0; off >>= 1) v[q] += __shfl_down(v[q], off, 64);
            if ((tid & 63) == 0) red[q][tid >> 6] = v[q];
        }
        __syncthreads();
        if (tid < 3) tot[tid] = (red[tid][0] + red[tid][1]) + (red[tid][2] + red[tid][3]);
        __syncthreads();
    }
    const float E = tot[1], D = tot[2];
    const bool grow = E > 0.f && D > E;
    if (tid == 0) loss_part[blockIdx.x] = tot[0] / cnt + (grow ? LOSS_ALPHA * (D / E - 1.f) : 0.f);
    // g_N = -(2 / cnt) L5 z - (growth) 2 LOSS_ALPHA mask d / E  (into d)
    for (int k = 0; k < TPT; ++k) {
        const int p = tid + 256 * k, py = p / TP, px = p % TP;
        float2 c = S.z[p];
        float2 g = make_float2(4.f * c.x, 4.f * c.y);
        const int nb[4][2] = {{0, -1}, {0, 1}, {-1, 0}, {1, 0}};
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int yy = py + nb[m][0], xx = px + nb[m][1];
            if (in_patch(yy, xx)) {
                float2 v = S.z[yy * TP + xx];
                g.x -= v.x;
                g.y -= v.y;
            }
        }
        const float sc = -2.f / cnt;
        float2 gn = make_float2(sc * g.x, sc * g.y);
        if (grow && py >= lo && py < hi && px >= lo && px < hi) {
            const float2 dv = S.d[p];
            const float f = -2.f * LOSS_ALPHA / E;
            gn.x += f * dv.x;
            gn.y += f * dv.y;
        }
        S.d[p] = gn;
    }
    __syncthreads();
    float2 *dW = dW_part + (size_t)blockIdx.x * NET_NW;
    // dW3[t][i] = sum_p g_N(p) conj(x2_i(p + d_t))
    if (tid < 144) {
        const int t = tid / 16, i = tid % 16, dy = tap_dy(t), dx = tap_dx(t);
        float2 acc = make_float2(0.f, 0.f);
        for (int py = 0; py < TP; ++py) {
            const int yy = py + dy;
            if (yy < 0 || yy >= TP) continue;
            for (int px = 0; px < TP; ++px) {
                const int xx = px + dx;
                if (xx < 0 || xx >= TP) continue;
                cmac_cx(acc, S.d[py * TP + px], unpack_c(S.x2[yy * TP + xx][i]));
            }
        }
        dW[NET_W3 + tid] = acc;
    }
    __syncthreads();
    // g_x2 = (conj(W3) * g_N, transposed), in place of x2
    for (int k = 0; k < TPT; ++k) {
        const int q = tid + 256 * k, qy = q / TP, qx = q % TP;
        float2 g[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) g[i] = make_float2(0.f, 0.f);
        for (int t = 0; t < 9; ++t) {
            const int py = qy - tap_dy(t), px = qx - tap_dx(t);
            if (!in_patch(py, px)) continue;
            const float2 gn = S.d[py * TP + px];
#pragma unroll
            for (int i = 0; i < 16; ++i) cmac_cw(g[i], W3[t * 16 + i], gn);
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) S.x2[q][i] = pack_c(g[i].x, g[i].y);
    }
    __syncthreads();
    // dW2[t][o][i] = sum_p g_x2_o(p) conj(x1_i(p + d_t)); thread = (o, i)
    {
        const int o = tid / 16, i = tid % 16;
        float2 acc[9];
#pragma unroll
        for (int t = 0; t < 9; ++t) acc[t] = make_float2(0.f, 0.f);
        for (int py = 0; py < TP; ++py)
            for (int px = 0; px < TP; ++px) {
                const float2 g = unpack_c(S.x2[py * TP + px][o]);
#pragma unroll
                for (int t = 0; t < 9; ++t) {
                    const int yy = py + tap_dy(t), xx = px + tap_dx(t);
                    if (in_patch(yy, xx)) cmac_cx(acc[t], g, unpack_c(S.x1[yy * TP + xx][i]));
                }
            }
#pragma unroll
        for (int t = 0; t < 9; ++t) dW[NET_W2 + (t * 16 + o) * 16 + i] = acc[t];
    }
    __syncthreads();
    // g_x1 = (conj(W2) * g_x2, transposed), in place of x1
    for (int k = 0; k < TPT; ++k) {
        const int q = tid + 256 * k, qy = q / TP, qx = q % TP;
        float2 g[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) g[i] = make_float2(0.f, 0.f);
        for (int t = 0; t < 9; ++t) {
            const int py = qy - tap_dy(t), px = qx - tap_dx(t);
            if (!in_patch(py, px)) continue;
            float2 ga[16];
#pragma unroll
            for (int o = 0; o < 16; ++o) ga[o] = unpack_c(S.x2[py * TP + px][o]);
#pragma unroll
            for (int o = 0; o < 16; ++o)
#pragma unroll
                for (int i = 0; i < 16; ++i) cmac_cw(g[i], W2[(t * 16 + o) * 16 + i], ga[o]);
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) S.x1[q][i] = pack_c(g[i].x, g[i].y);
    }
    __syncthreads();
    // through the gate x1 = a c, c = 1 + m (a, m recomputed from the
    // inputs): g_a = conj(c) g_x1 into x1, g_m = conj(a) g_x1 into x2
    for (int k = 0; k < TPT; ++k) {
        const int p = tid + 256 * k;
        float2 a[16], m[16];
        layer1_point(S, W1, p, a, m);
#pragma unroll
        for (int o = 0; o < 16; ++o) {
            const float2 g = unpack_c(S.x1[p][o]);
            const float2 c = make_float2(1.f + m[o].x, m[o].y);
            float2 ga = make_float2(0.f, 0.f), gm = make_float2(0.f, 0.f);
            cmac_cw(ga, c, g);
            cmac_cw(gm, a[o], g);
            S.x1[p][o] = pack_c(ga.x, ga.y);
            S.x2[p][o] = pack_c(gm.x, gm.y);
        }
    }
    __syncthreads();
    // dW1[t][o][0] = sum_p g_a_o(p) conj(r~(p + d_t)), dW1[t][o][1] likewise
    // from g_m and kappa~; thread = (o, i) x 4 groups of 8 rows, then a
    // fixed-order sum of the 4 partials (kept in the d / z buffers)
    {
        float2 *part = &S.d[0];   // 2 x 1024 float2, d and z are contiguous
        const int pr = tid % 32, grp = tid / 32, o = pr / 2, i = pr % 2;
        if (grp < 4) {
            float2 acc[9];
#pragma unroll
            for (int t = 0; t < 9; ++t) acc[t] = make_float2(0.f, 0.f);
            for (int py = grp * 8; py < grp * 8 + 8; ++py)
                for (int px = 0; px < TP; ++px) {
                    const float2 g = unpack_c(i == 0 ? S.x1[py * TP + px][o] : S.x2[py * TP + px][o]);
#pragma unroll
                    for (int t = 0; t < 9; ++t) {
                        const int yy = py + tap_dy(t), xx = px + tap_dx(t);
                        if (in_patch(yy, xx)) cmac_cx(acc[t], g, unpack_c(S.x0[yy * TP + xx][i]));
                    }
                }
#pragma unroll
            for (int t = 0; t < 9; ++t) part[(grp * 9 + t) * 32 + pr] = acc[t];
        }
        __syncthreads();
        for (int e = tid; e < 288; e += 256) {
            const int t = e / 32, pe = e % 32;
            float2 s = make_float2(0.f, 0.f);
            for (int gg = 0; gg < 4; ++gg) {
                float2 v = part[(gg * 9 + t) * 32 + pe];
                s.x += v.x;
                s.y += v.y;
            }
            const int oo = pe / 2, ii = pe % 2;
            dW[NET_W1 + (t * 16 + oo) * 2 + ii] = s;
        }
    }
}

// Mean of the per-patch gradients (fixed order) and of the losses.
__global__ __launch_bounds__(256) void k_reduce_grads(const float2 *__restrict__ dW_part, int count,
                                                      float2 *__restrict__ grad)
{
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= NET_NW) return;
    float2 s = make_float2(0.f, 0.f);
    for (int p = 0; p < count; ++p) {
        float2 v = dW_part[(size_t)p * NET_NW + k];
        s.x += v.x;
        s.y += v.y;
    }
    const float inv = 1.f / (float)count;
    grad[k] = make_float2(s.x * inv, s.y * inv);
}

__global__ __launch_bounds__(256) void k_reduce_loss(const float *__restrict__ part, int count, float *__restrict__ out)
{
    __shared__ float red[256];
    float s = 0.f;
    for (int p = threadIdx.x; p < count; p += 256) s += part[p];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0] / (float)count;
}

// Adam on the real and imaginary parts (step >= 1); refreshes the BF16-rounded
// copy used by the training forward pass.
__global__ __launch_bounds__(256) void k_adam(float2 *__restrict__ Wm, float2 *__restrict__ Wq,
                                              const float2 *__restrict__ grad, float2 *__restrict__ m,
                                              float2 *__restrict__ v, float lr, float b1, float b2, float eps,
                                              float c1, float c2)
{
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= NET_NW) return;
    float2 g = grad[k], mk = m[k], vk = v[k], w = Wm[k];
    mk.x = b1 * mk.x + (1.f - b1) * g.x;
    mk.y = b1 * mk.y + (1.f - b1) * g.y;
    vk.x = b2 * vk.x + (1.f - b2) * g.x * g.x;
    vk.y = b2 * vk.y + (1.f - b2) * g.y * g.y;
    w.x -= lr * (mk.x / c1) / (sqrtf(vk.x / c2) + eps);
    w.y -= lr * (mk.y / c1) / (sqrtf(vk.y / c2) + eps);
    m[k] = mk;
    v[k] = vk;
    Wm[k] = w;
    Wq[k] = make_float2(bf16_round(w.x), bf16_round(w.y));
}

__global__ __launch_bounds__(256) void k_round_weights(const float2 *__restrict__ Wm, float2 *__restrict__ Wq)
{
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k < NET_NW) Wq[k] = make_float2(bf16_round(Wm[k].x), bf16_round(Wm[k].y));
}

size_t train_lds_bytes() { return sizeof(TrainLds); }

void launch_train_patches(const float2 *rt, const float2 *kt, const float2 *et, const float2 *Wq, float2 *dW_part,
                          float *loss_part, int count, int border, hipStream_t s)
{
    // once (a thread-safe static initialisation)
    static const bool attr = [] {
        (void)hipFuncSetAttribute((const void *)k_train_patch, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)sizeof(TrainLds));
        return true;
    }();
    (void)attr;
    hipLaunchKernelGGL(k_train_patch, dim3(count), dim3(256), sizeof(TrainLds), s, rt, kt, et, Wq, dW_part,
                       loss_part, border);
}

void launch_reduce_grads(const float2 *dW_part, int count, float2 *grad, const float *loss_part, float *loss,
                         hipStream_t s)
{
    hipLaunchKernelGGL(k_reduce_grads, dim3((NET_NW + 255) / 256), dim3(256), 0, s, dW_part, count, grad);
    hipLaunchKernelGGL(k_reduce_loss, dim3(1), dim3(256), 0, s, loss_part, count, loss);
}

void launch_adam(float2 *Wm, float2 *Wq, const float2 *grad, float2 *m, float2 *v, float lr, float b1, float b2,
                 float eps, int step, hipStream_t s)
{
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3((NET_NW + 255) / 256), dim3(256), 0, s, Wm, Wq, grad, m, v, lr, b1, b2, eps,
                       c1, c2);
}

void launch_round_weights(const float2 *Wm, float2 *Wq, hipStream_t s)
{
    hipLaunchKernelGGL(k_round_weights, dim3((NET_NW + 255) / 256), dim3(256), 0, s, Wm, Wq);
}



// ---------------------------------------------------------------------------
// Inference on a grid with the BF16 MFMA v_mfma_f32_16x16x32_bf16 (A[i][k]
// from lane i + 16 (k / 8), element k % 8; B[k][j] likewise with j; D[i][j]
// in lane j + 16 (i / 4), register i % 4).  Each convolution is an implicit
// GEMM over points: rows are 16 points of a region, columns the real output
// channels (Re / Im of each complex channel), K the (tap, real input
// channel) pairs.  A complex weight w acts on (Re x, Im x) as the real 2 x 2
// block [[Re w, -Im w], [Im w, Re w]].
//   layer 1: K = 9 taps x 2 (Re / Im), padded to 32, one k-step.  For the
//            column of part p of channel c, four products give
//            A = p of a, A' = (-Im a, Re a)[p], M = 1 + Re m (accumulator
//            started at 1), M' = Im m, and the gate is x1 = A M + A' M'
//            (Re: a_re (1 + m_re) - a_im m_im; Im: a_im (1 + m_re) +
//            a_re m_im) without any exchange between lanes
//   layer 2: K = 32 channels per tap, one k-step per tap; N = 32
//   layer 3: one output channel, so the 9 taps go to the columns instead:
//            Z_t = W3[t] x2 per point (K = 32, columns 2 t + part, 18 of 32
//            used), then N(p) = sum_t Z_t(p + d_t) by a gather from LDS
// A 16 x 16 output tile needs layer-2 values on 18 x 18 points, layer-1
// values on 20 x 20 and the inputs on 22 x 22 (zero outside the grid); the
// activations live in LDS as BF16 [point][channel].  The weight fragments
// (prepared on the host by pack_net_mfma) stay in registers.
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned short us8 __attribute__((ext_vector_type(8)));

constexpr int IT = 16;                       // output tile side
constexpr int R1 = IT + 4, R2 = IT + 2;      // layer-1 / layer-2 region sides
constexpr int R0 = IT + 6;                   // input region side
constexpr int NR1 = (R1 * R1 + 15) / 16;     // row tiles of the layer-1 region
constexpr int NR2 = (R2 * R2 + 15) / 16;
constexpr int IN_PER_THREAD = (R0 * R0 + 255) / 256;

// Activations: 32 BF16 channel slots per point, padded to 40 (80 bytes): the
// 8 lanes a 128-bit LDS read serves together then start 20 dwords apart and
// cover all 32 banks once.  Slot s holds accumulator column
// 16 (s & 1) + (s >> 1) of the producing layer, so that the lane owning
// column li of both column tiles writes slots 2 li and 2 li + 1 as one dword;
// column j is Re (j even) or Im (j odd) of channel j / 2.
constexpr int XS = 40;
// Per-tap layer-3 products: 18 floats per point, rows of 20 (80 bytes).
constexpr int ZS = 20;
struct alignas(16) InferLds {
    unsigned short x0[R0 * R0][4];           // r~ re, r~ im, kappa~ re, kappa~ im
    union {
        unsigned short x1[NR1 * 16][XS];
        float z[NR2 * 16][ZS];               // layer-3 per-tap products (after layer 2)
    };
    unsigned short x2[NR2 * 16][XS];         // rows past R2 * R2 take unused writes
};

__device__ __forceinline__ bf8 as_bf8(us8 v) { return __builtin_bit_cast(bf8, v); }

// Hardware round-to-nearest-even FP32 -> BF16 (v_cvt_pk_bf16_f32 on gfx950).
__device__ __forceinline__ unsigned short to_bf16(float f) { return __builtin_bit_cast(unsigned short, (__bf16)f); }
typedef float fv2 __attribute__((ext_vector_type(2)));
typedef __bf16 bv2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ unsigned pack_bf16(float lo, float hi)
{
    return __builtin_bit_cast(unsigned, __builtin_convertvector(fv2{lo, hi}, bv2));
}

// Point (y, x) of row-major region of width R for index p.
struct RegionPos {
    int y, x;
};
template <int R>
__device__ __forceinline__ RegionPos region_pos(int p)
{
    return RegionPos{p / R, p - (p / R) * R};
}
template <int R>
__device__ __forceinline__ void region_next(RegionPos &q)
{
    const bool wrap = q.x == R - 1;
    q.x = wrap ? 0 : q.x + 1;
    q.y += wrap ? 1 : 0;
}

// Inputs of one tile's 22 x 22 region (origin oy - 3, ox - 3), held in
// registers between their global load and their LDS store so that the next
// tile's loads overlap the current tile's layers.
struct TileInput {
    cd r[IN_PER_THREAD];
    unsigned k[IN_PER_THREAD];
};

__device__ __forceinline__ bool input_in_grid(int p, int mx, int my, int oy, int ox)
{
    const RegionPos q = region_pos<R0>(p < R0 * R0 ? p : 0);
    const int gy = oy - 3 + q.y, gx = ox - 3 + q.x;
    return p < R0 * R0 && gy >= 0 && gy < my && gx >= 0 && gx < mx;
}

// Issues the loads only (points outside the grid read element 0 and are
// zeroed when stored), so that nothing waits for them before the store.
__device__ __forceinline__ void load_tile_input(TileInput &in, const cd *__restrict__ r,
                                                const unsigned *__restrict__ kh2, int mx, int my, int oy, int ox)
{
#pragma unroll
    for (int i = 0; i < IN_PER_THREAD; ++i) {
        const int p = threadIdx.x + 256 * i;
        const RegionPos q = region_pos<R0>(p < R0 * R0 ? p : 0);
        const size_t j = input_in_grid(p, mx, my, oy, ox) ? (size_t)(oy - 3 + q.y) * mx + (ox - 3 + q.x) : 0;
        in.r[i] = r[j];
        in.k[i] = kh2[j];
    }
}

__device__ __forceinline__ void store_tile_input(InferLds &S, const TileInput &in, int mx, int my, int oy, int ox)
{
#pragma unroll
    for (int i = 0; i < IN_PER_THREAD; ++i) {
        const int p = threadIdx.x + 256 * i;
        const bool ok = input_in_grid(p, mx, my, oy, ox);
        if (p < R0 * R0)
            *reinterpret_cast<uint2 *>(&S.x0[p][0]) =
                ok ? make_uint2(pack_bf16((float)in.r[i].re, (float)in.r[i].im), in.k[i]) : make_uint2(0u, 0u);
    }
}

// Layers of one 16 x 16 output tile (origin oy, ox) whose inputs are in
// S.x0; leaves layer 3's per-tap products in S.z.  The weight fragments stay
// in registers.  In layer 2 each wave takes two row tiles at a time so that
// four independent MFMA accumulation chains interleave.  EDGE: the tile's layer-1 region reaches
// outside the grid, so activations there are set to zero (interior tiles
// skip the test).
template <bool EDGE>
__device__ __forceinline__ void net_layers(InferLds &S, int mx, int my, int oy, int ox, const bf8 (&w1)[4][2],
                                           const bf8 (&w2)[9][2], const bf8 (&w3)[2], int wave)
{
    const int lane = threadIdx.x & 63;
    const int li = lane & 15, lg = lane >> 4;
    // layer-1 operand: lane group lg holds taps 4 lg .. 4 lg + 3; taps 9 ..
    // 15 are zero padding whose weights are zero, so they may read any
    // (finite) slot: the point itself
    int off1[4];
#pragma unroll
    for (int hh = 0; hh < 4; ++hh) {
        const int t = 4 * lg + hh;
        off1[hh] = t < 9 ? 2 * ((t / 3 - 1) * R0 + (t % 3 - 1)) : 0;
    }
    // layer 1 on the 20 x 20 region (origin -2), one row tile per iteration,
    // two iterations interleaved
#pragma unroll 2
    for (int rt = wave; rt < NR1; rt += 4) {
        const int p = rt * 16 + li;
        const RegionPos P = region_pos<R1>(p);
        const uint2 *base = reinterpret_cast<const uint2 *>(&S.x0[(P.y + 1) * R0 + P.x + 1][0]);
        us8 ar, ak;   // the r~ and kappa~ operands
#pragma unroll
        for (int hh = 0; hh < 4; ++hh) {
            const uint2 v = base[off1[hh] / 2];
            ar[2 * hh] = (unsigned short)(v.x & 0xFFFFu);
            ar[2 * hh + 1] = (unsigned short)(v.x >> 16);
            ak[2 * hh] = (unsigned short)(v.y & 0xFFFFu);
            ak[2 * hh + 1] = (unsigned short)(v.y >> 16);
        }
        float x[2][4];
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
            const f4 z = f4{0.f, 0.f, 0.f, 0.f}, one = f4{1.f, 1.f, 1.f, 1.f};
            const f4 A = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf8(ar), w1[0][nt], z, 0, 0, 0);
            const f4 Ap = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf8(ar), w1[1][nt], z, 0, 0, 0);
            const f4 M = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf8(ak), w1[2][nt], one, 0, 0, 0);
            const f4 Mp = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf8(ak), w1[3][nt], z, 0, 0, 0);
#pragma unroll
            for (int v = 0; v < 4; ++v) x[nt][v] = fmaf(A[v], M[v], Ap[v] * Mp[v]);
        }
        const int pp = rt * 16 + 4 * lg;
        RegionPos Q = region_pos<R1>(pp);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            unsigned val = pack_bf16(x[0][v], x[1][v]);
            if (EDGE) {
                const int gy = oy - 2 + Q.y, gx = ox - 2 + Q.x;
                const bool in = gy >= 0 && gy < my && gx >= 0 && gx < mx;
                val = in ? val : 0u;
                region_next<R1>(Q);
            }
            *reinterpret_cast<unsigned *>(&S.x1[pp + v][2 * li]) = val;
        }
    }
    __syncthreads();
    // layer 2 on the 18 x 18 region (origin -1)
    for (int rt0 = wave; rt0 < NR2; rt0 += 8) {
        f4 acc[2][2];
        const us8 *base[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            int p = (rt0 + 4 * q) * 16 + li;
            if (p >= R2 * R2) p = 0;
            const RegionPos P = region_pos<R2>(p);
            base[q] = reinterpret_cast<const us8 *>(&S.x1[(P.y + 1) * R1 + P.x + 1][8 * lg]);
#pragma unroll
            for (int nt = 0; nt < 2; ++nt) acc[q][nt] = f4{0.f, 0.f, 0.f, 0.f};
        }
        us8 a[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) a[q] = base[q][(tap_dy(0) * R1 + tap_dx(0)) * (XS / 8)];
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            us8 an[2];
            if (t + 1 < 9) {
#pragma unroll
                for (int q = 0; q < 2; ++q) an[q] = base[q][(tap_dy(t + 1) * R1 + tap_dx(t + 1)) * (XS / 8)];
            }
#pragma unroll
            for (int q = 0; q < 2; ++q)
#pragma unroll
                for (int nt = 0; nt < 2; ++nt)
                    acc[q][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf8(a[q]), w2[t][nt], acc[q][nt], 0, 0, 0);
            if (t + 1 < 9) {
#pragma unroll
                for (int q = 0; q < 2; ++q) a[q] = an[q];
            }
        }
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int rt = rt0 + 4 * q;
            if (rt >= NR2) break;
            const int pp = rt * 16 + 4 * lg;
            RegionPos P = region_pos<R2>(pp);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                unsigned val = pack_bf16(acc[q][0][v], acc[q][1][v]);
                if (EDGE) {
                    const int gy = oy - 1 + P.y, gx = ox - 1 + P.x;
                    const bool in = gy >= 0 && gy < my && gx >= 0 && gx < mx;
                    val = in ? val : 0u;
                    region_next<R2>(P);
                }
                *reinterpret_cast<unsigned *>(&S.x2[pp + v][2 * li]) = val;
            }
        }
    }
    __syncthreads();
    // layer 3, first part: per-tap products Z_t(q) = W3[t] x2(q) at every
    // point q of the 18 x 18 region (one k-step, columns 2 t + part; taps
    // 0..7 in column tile 0, tap 8 in column tile 1), written to S.z, which
    // reuses the layer-1 storage (dead once layer 2 has been read).  The
    // second part, the 9-point gather N(p) = sum_t Z_t(p + d_t), follows the
    // next barrier (layer3_gather).
#pragma unroll 2
    for (int rt = wave; rt < NR2; rt += 4) {
        int p = rt * 16 + li;
        if (p >= R2 * R2) p = 0;
        const us8 a = *reinterpret_cast<const us8 *>(&S.x2[p][8 * lg]);
        const f4 z = f4{0.f, 0.f, 0.f, 0.f};
        const f4 Z0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf8(a), w3[0], z, 0, 0, 0);
        const f4 Z1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf8(a), w3[1], z, 0, 0, 0);
        const int pp = rt * 16 + 4 * lg;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            S.z[pp + v][li] = Z0[v];
            if (li < 2) S.z[pp + v][16 + li] = Z1[v];
        }
    }
}

// Layer 3, second part, for this thread's output point (py, px) of the tile:
// N = sum over the 9 taps of Z_t at the neighbour p + d_t (region origin -1).
__device__ __forceinline__ float2 layer3_gather(const InferLds &S, int py, int px)
{
    float2 y = make_float2(0.f, 0.f);
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        const int q = (py + 1 + tap_dy(t)) * R2 + (px + 1 + tap_dx(t));
        const float2 zt = *reinterpret_cast<const float2 *>(&S.z[q][2 * t]);
        y.x += zt.x;
        y.y += zt.y;
    }
    return y;
}

// N is complex-linear in its residual input, so s h^2 N(r / s) = h^2 N(r)
// for any scale s; BF16 has the exponent range of FP32, so the residual is
// fed unscaled and no global reduction precedes the step.  Persistent
// workgroups: each loads the weight fragments once and works through a
// contiguous range of tiles (ranges of neighbouring workgroups sit on one
// XCD); the inputs of the next tile are loaded while the current one is
// computed, and u is updated by all threads, one point each.
__global__ __launch_bounds__(256) void k_net_apply(const cd *__restrict__ r, const unsigned *__restrict__ kh2,
                                                   cd *__restrict__ u, int mx, int my, int tiles_x, int ntiles,
                                                   int per_block, const us8 *__restrict__ wfrag, double h2,
                                                   const int *__restrict__ stop)
{
    if (stop && *stop) return;
    __shared__ InferLds S;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    bf8 w1[4][2], w2[9][2], w3[2];
#pragma unroll
    for (int ty = 0; ty < 4; ++ty)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) w1[ty][nt] = as_bf8(wfrag[(ty * 2 + nt) * 64 + lane]);
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) w2[t][nt] = as_bf8(wfrag[512 + (t * 2 + nt) * 64 + lane]);
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) w3[nt] = as_bf8(wfrag[512 + 1152 + nt * 64 + lane]);
    const int first = xcd_tile(blockIdx.x, gridDim.x) * per_block;
    const int last = min(first + per_block, ntiles);
    if (first >= last) return;
    TileInput in;
    load_tile_input(in, r, kh2, mx, my, (first / tiles_x) * IT, (first % tiles_x) * IT);
    // this thread's output point of the tile
    const int py = tid >> 4, px = tid & 15;
    for (int tile = first; tile < last; ++tile) {
        const int oy = (tile / tiles_x) * IT, ox = (tile % tiles_x) * IT;
        store_tile_input(S, in, mx, my, oy, ox);
        __syncthreads();
        if (tile + 1 < last)
            load_tile_input(in, r, kh2, mx, my, ((tile + 1) / tiles_x) * IT, ((tile + 1) % tiles_x) * IT);
        const int gy = oy + py, gx = ox + px;
        const bool mine = gy < my && gx < mx;
        const size_t j = mine ? (size_t)gy * mx + gx : 0;
        const cd uv = u[j];
        // the layer-1 region (origin -2, side 20) lies inside the grid
        const bool interior = oy >= 2 && ox >= 2 && oy + IT + 2 <= my && ox + IT + 2 <= mx;
        if (interior)
            net_layers<false>(S, mx, my, oy, ox, w1, w2, w3, wave);
        else
            net_layers<true>(S, mx, my, oy, ox, w1, w2, w3, wave);
        __syncthreads();
        if (mine) {
            const float2 yv = layer3_gather(S, py, px);
            u[j] = cd{uv.re + h2 * (double)yv.x, uv.im + h2 * (double)yv.y};
        }
        // the next tile's layers start after its input barrier, so S.z (the
        // layer-1 storage) is not overwritten before it is read here
    }
}

// Channel and Re / Im part held in activation slot s (see InferLds).
static int slot_channel(int s) { return (16 * (s & 1) + (s >> 1)) / 2; }
static int slot_part(int s) { return (s >> 1) & 1; }

// MFMA B-operand fragments of the three layers from the complex weights
// (rounded to BF16): 64 lanes x 8 values per fragment, in the order read by
// k_net_apply.
void pack_net_mfma(const float *w, unsigned short *out)
{
    auto W = [&](int off, int idx, int part) { return w[2 * (off + idx) + part]; };
    // real weight of complex weight (re, im) from real input part pi to output part po
    auto real_block = [](float re, float im, int po, int pi) {
        return po == 0 ? (pi == 0 ? re : -im) : (pi == 0 ? im : re);
    };
    auto bf = [](float f) { return (unsigned short)bf16_bits(f); };
    size_t o = 0;
    // layer 1, k = 2 tap + part (k < 18); four products per column j (part
    // po of channel j / 2): type 0 A = part po of a, type 1
    // A' = (-Im a, Re a)[po] (both from the r~ weights), type 2 Re m, type 3
    // Im m (both from the kappa~ weights)
    for (int ty = 0; ty < 4; ++ty)
        for (int nt = 0; nt < 2; ++nt)
            for (int lane = 0; lane < 64; ++lane)
                for (int e = 0; e < 8; ++e) {
                    const int k = 8 * (lane / 16) + e, j = 16 * nt + lane % 16;
                    float v = 0.f;
                    if (k < 18) {
                        const int t = k / 2, pi = k % 2, oc = j / 2, po = j % 2;
                        const int idx = (t * 16 + oc) * 2 + (ty < 2 ? 0 : 1);
                        const float re = W(NET_W1, idx, 0), im = W(NET_W1, idx, 1);
                        switch (ty) {
                        case 0: v = real_block(re, im, po, pi); break;
                        case 1: v = po == 0 ? -real_block(re, im, 1, pi) : real_block(re, im, 0, pi); break;
                        case 2: v = real_block(re, im, 0, pi); break;
                        default: v = real_block(re, im, 1, pi); break;
                        }
                    }
                    out[o++] = bf(v);
                }
    for (int t = 0; t < 9; ++t)
        for (int nt = 0; nt < 2; ++nt)
            for (int lane = 0; lane < 64; ++lane)
                for (int e = 0; e < 8; ++e) {
                    const int slot = 8 * (lane / 16) + e, j = 16 * nt + lane % 16;
                    const int i = slot_channel(slot), pi = slot_part(slot), oc = j / 2, po = j % 2;
                    const int idx = (t * 16 + oc) * 16 + i;
                    out[o++] = bf(real_block(W(NET_W2, idx, 0), W(NET_W2, idx, 1), po, pi));
                }
    // layer 3: column c = 16 nt + lane % 16 is part c % 2 of tap c / 2 (< 9)
    for (int nt = 0; nt < 2; ++nt)
        for (int lane = 0; lane < 64; ++lane)
            for (int e = 0; e < 8; ++e) {
                const int slot = 8 * (lane / 16) + e, c = 16 * nt + lane % 16;
                const int t = c / 2, po = c % 2;
                float v = 0.f;
                if (t < 9) {
                    const int i = slot_channel(slot), pi = slot_part(slot);
                    const int idx = t * 16 + i;
                    v = real_block(W(NET_W3, idx, 0), W(NET_W3, idx, 1), po, pi);
                }
                out[o++] = bf(v);
            }
}

size_t net_mfma_frag_count() { return (size_t)(8 + 18 + 2) * 64 * 8; }

// kappa h^2 as packed BF16 complex
__global__ __launch_bounds__(256) void k_kappa_h2(const cd *__restrict__ q, double k02, double h2, size_t N,
                                                  unsigned *__restrict__ out)
{
    for (size_t j = (size_t)blockIdx.x * 256 + threadIdx.x; j < N; j += (size_t)gridDim.x * 256) {
        const cd qj = q[j];
        out[j] = pack_c((float)((k02 + qj.re) * h2), (float)(qj.im * h2));
    }
}

void launch_kappa_h2(const cd *q, double k02, double h2, size_t N, unsigned *out, hipStream_t s)
{
    size_t nb = std::min<size_t>((N + 255) / 256, 65536);
    hipLaunchKernelGGL(k_kappa_h2, dim3((unsigned)nb), dim3(256), 0, s, q, k02, h2, N, out);
}

void launch_net_apply(const cd *r, const unsigned *kh2, cd *u, int mx, int my, const unsigned short *wfrag,
                      double h2, hipStream_t st, const int *stop)
{
    const int tx = (mx + IT - 1) / IT, ty = (my + IT - 1) / IT, nt = tx * ty;
    const int blocks = std::min(nt, 256 * 2);   // two resident workgroups per CU
    const int per = (nt + blocks - 1) / blocks;
    const int nb = (nt + per - 1) / per;
    hipLaunchKernelGGL(k_net_apply, dim3(nb), dim3(256), 0, st, r, kh2, u, mx, my, tx, nt, per,
                       reinterpret_cast<const us8 *>(wfrag), h2, stop);
}

}  // namespace ffmg

// ===========================================================================
// C ABI: the network object (weights, Adam state, training buffers).
#include <stdarg.h>
#include <stdio.h>

#include <string>
#include <vector>

#include "../../include/ffmg.h"

struct ffmg_net {
    hipStream_t stream = nullptr;
    float2 *Wm = nullptr, *Wq = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr;
    float2 *dW_part = nullptr;
    float *loss_part = nullptr, *d_loss = nullptr, *h_loss = nullptr;
    int part_cap = 0;
    int step = 0;
    std::string err;
    std::vector<void *> allocs;
};

namespace {

ffmg_status net_fail(ffmg_net *n, ffmg_status s, const char *fmt, ...)
{
    if (n) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        n->err = buf;
    }
    return s;
}

#define NCHK(n, x)                                                                                                   \
    do {                                                                                                             \
        hipError_t e_ = (x);                                                                                         \
        if (e_ != hipSuccess)                                                                                        \
            return net_fail((n), e_ == hipErrorOutOfMemory ? FFMG_ENOMEM : FFMG_EDEVICE, "%s: %s", #x,              \
                            hipGetErrorString(e_));                                                                  \
    } while (0)

template <typename P>
ffmg_status net_alloc(ffmg_net *n, P **p, size_t bytes)
{
    void *q = nullptr;
    NCHK(n, hipMalloc(&q, bytes));
    n->allocs.push_back(q);
    *p = (P *)q;
    return FFMG_OK;
}

ffmg_status check_finite(ffmg_net *n, const float *w)
{
    for (int k = 0; k < 2 * ffmg::NET_NW; ++k)
        if (!isfinite(w[k])) return net_fail(n, FFMG_ENAN, "weight %d is not finite", k / 2);
    return FFMG_OK;
}

ffmg_status train_common(ffmg_net *n, const void *rt, const void *kt, const void *et, int count, int border)
{
    if (!rt || !kt || !et || count < 1) return net_fail(n, FFMG_EINVAL, "null patches or count < 1");
    if (border < 1 || border > 12) return net_fail(n, FFMG_EINVAL, "border must lie in [1, 12]");
    if (n->part_cap < count) {
        if (n->dW_part) {
            (void)hipFree(n->dW_part);
            (void)hipFree(n->loss_part);
            n->allocs.erase(std::remove(n->allocs.begin(), n->allocs.end(), (void *)n->dW_part), n->allocs.end());
            n->allocs.erase(std::remove(n->allocs.begin(), n->allocs.end(), (void *)n->loss_part), n->allocs.end());
            n->dW_part = nullptr;
            n->loss_part = nullptr;
            n->part_cap = 0;
        }
        ffmg_status s = net_alloc(n, &n->dW_part, (size_t)count * ffmg::NET_NW * sizeof(float2));
        if (s != FFMG_OK) return s;
        s = net_alloc(n, &n->loss_part, (size_t)count * sizeof(float));
        if (s != FFMG_OK) return s;
        n->part_cap = count;
    }
    ffmg::launch_train_patches((const float2 *)rt, (const float2 *)kt, (const float2 *)et, n->Wq, n->dW_part,
                               n->loss_part, count, border, n->stream);
    ffmg::launch_reduce_grads(n->dW_part, count, n->grad, n->loss_part, n->d_loss, n->stream);
    NCHK(n, hipGetLastError());
    return FFMG_OK;
}

}  // namespace

extern "C" {

ffmg_status ml_net_create(const float *w, void *stream, ffmg_net **out)
{
    if (!out || !w) return FFMG_EINVAL;
    *out = nullptr;
    ffmg_net *n = new ffmg_net();
    n->stream = (hipStream_t)stream;
    ffmg_status s = check_finite(n, w);
    const size_t bytes = ffmg::NET_NW * sizeof(float2);
    if (s == FFMG_OK) s = net_alloc(n, &n->Wm, bytes);
    if (s == FFMG_OK) s = net_alloc(n, &n->Wq, bytes);
    if (s == FFMG_OK) s = net_alloc(n, &n->m, bytes);
    if (s == FFMG_OK) s = net_alloc(n, &n->v, bytes);
    if (s == FFMG_OK) s = net_alloc(n, &n->grad, bytes);
    if (s == FFMG_OK) s = net_alloc(n, &n->d_loss, sizeof(float));
    if (s == FFMG_OK && hipHostMalloc((void **)&n->h_loss, sizeof(float), hipHostMallocDefault) != hipSuccess)
        s = net_fail(n, FFMG_ENOMEM, "hipHostMalloc failed");
    if (s == FFMG_OK) s = ml_net_set_weights(n, w);
    if (s != FFMG_OK) {
        ml_net_destroy(n);
        return s;
    }
    *out = n;
    return FFMG_OK;
}

ffmg_status ml_net_set_weights(ffmg_net *n, const float *w)
{
    if (!n || !w) return FFMG_EINVAL;
    ffmg_status s = check_finite(n, w);
    if (s != FFMG_OK) return s;
    const size_t bytes = ffmg::NET_NW * sizeof(float2);
    NCHK(n, hipMemcpyAsync(n->Wm, w, bytes, hipMemcpyHostToDevice, n->stream));
    ffmg::launch_round_weights(n->Wm, n->Wq, n->stream);
    NCHK(n, hipMemsetAsync(n->m, 0, bytes, n->stream));
    NCHK(n, hipMemsetAsync(n->v, 0, bytes, n->stream));
    n->step = 0;
    NCHK(n, hipStreamSynchronize(n->stream));
    return FFMG_OK;
}

ffmg_status ml_net_get_weights(ffmg_net *n, float *w)
{
    if (!n || !w) return FFMG_EINVAL;
    NCHK(n, hipMemcpyAsync(w, n->Wm, ffmg::NET_NW * sizeof(float2), hipMemcpyDeviceToHost, n->stream));
    NCHK(n, hipStreamSynchronize(n->stream));
    return FFMG_OK;
}

ffmg_status ml_loss_grad(ffmg_net *n, const void *rt, const void *kt, const void *et, int count, int border,
                         float *loss, float *grad)
{
    if (!n) return FFMG_EINVAL;
    ffmg_status s = train_common(n, rt, kt, et, count, border);
    if (s != FFMG_OK) return s;
    if (loss) NCHK(n, hipMemcpyAsync(n->h_loss, n->d_loss, sizeof(float), hipMemcpyDeviceToHost, n->stream));
    if (grad) NCHK(n, hipMemcpyAsync(grad, n->grad, ffmg::NET_NW * sizeof(float2), hipMemcpyDeviceToHost, n->stream));
    NCHK(n, hipStreamSynchronize(n->stream));
    if (loss) *loss = *n->h_loss;
    return FFMG_OK;
}

ffmg_status ml_train_step(ffmg_net *n, const void *rt, const void *kt, const void *et, int count, int border,
                          float lr, float *loss)
{
    if (!n) return FFMG_EINVAL;
    if (!(lr > 0.f) || !isfinite(lr)) return net_fail(n, FFMG_EINVAL, "lr must be positive");
    ffmg_status s = train_common(n, rt, kt, et, count, border);
    if (s != FFMG_OK) return s;
    n->step += 1;
    ffmg::launch_adam(n->Wm, n->Wq, n->grad, n->m, n->v, lr, 0.9f, 0.999f, 1e-8f, n->step, n->stream);
    NCHK(n, hipGetLastError());
    if (loss) {
        NCHK(n, hipMemcpyAsync(n->h_loss, n->d_loss, sizeof(float), hipMemcpyDeviceToHost, n->stream));
        NCHK(n, hipStreamSynchronize(n->stream));
        *loss = *n->h_loss;
    }
    return FFMG_OK;
}

const char *ml_net_last_error(const ffmg_net *n) { return n ? n->err.c_str() : "null network"; }

void ml_net_destroy(ffmg_net *n)
{
    if (!n) return;
    if (n->stream) (void)hipStreamSynchronize(n->stream);
    else (void)hipDeviceSynchronize();
    for (void *p : n->allocs) (void)hipFree(p);
    if (n->h_loss) (void)hipHostFree(n->h_loss);
    delete n;
}

}  // extern "C"
