// ffmg_device.hpp -- device-side building blocks shared by the library's HIP
// kernels: interleaved complex numbers, the contour stencil at one point, and
// the XCD-aware block-to-tile map.  gfx950 (CDNA4) only.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace ffmg {

// Interleaved complex value; 16 B (double) / 8 B (float) aligned so that one
// element is one 128-bit / 64-bit vector load.
template <typename T>
struct alignas(2 * sizeof(T)) cx {
    T re, im;
};
using cd = cx<double>;
using cf = cx<float>;

template <typename T>
__host__ __device__ __forceinline__ cx<T> mk(T r, T i) { return cx<T>{r, i}; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator*(cx<T> a, cx<T> b)
{
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator*(T s, cx<T> a) { return {s * a.re, s * a.im}; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> recip(cx<T> a)
{
    T d = a.re * a.re + a.im * a.im;
    T inv = T(1) / d;
    return {a.re * inv, -a.im * inv};
}
template <typename T>
__host__ __device__ __forceinline__ T abs2(cx<T> a) { return a.re * a.re + a.im * a.im; }

template <typename To, typename Ti>
__host__ __device__ __forceinline__ cx<To> cvt(cx<Ti> a) { return {To(a.re), To(a.im)}; }

// Parameters of the contour operator on one grid level:
//   (A u)_j = sum_k c_k (2u_j - u_{j-e_k} - u_{j+e_k}) - (k0^2 + q_j) u_j,
//   c_k = e^{-2 i gamma} / h_k^2,  D_j = 2 sum_k c_k - k0^2 - q_j.
template <typename T>
struct Stencil {
    int mx, my, mz;     // interior extents (mz = 1 in 2D)
    cx<T> c[3];         // c_k = rot / h_k^2
    cx<T> rot;          // e^{-2 i gamma}
    T ih2[3];           // 1 / h_k^2 (0 for unused axes)
    cx<T> csum2;        // 2 sum_k c_k
    T k02;              // k0^2
    T omega;            // Jacobi damping
    T omc;              // 1 - omega
};

// p[j] where `in` holds, 0 elsewhere.  The load always goes to a valid
// address (j or 0) and the value is selected afterwards: written as
// `in ? p[j] : zero` the compiler may turn it into a load through a select of
// the two addresses, which puts the zero on the stack and makes every load a
// flat (generic) access.
template <typename T>
__device__ __forceinline__ cx<T> ld_masked(const cx<T> *__restrict__ p, size_t j, bool in)
{
    cx<T> v = p[in ? j : 0];
    return in ? v : cx<T>{T(0), T(0)};
}

// Loads through a buffer resource (a base address and a byte range held in
// scalar registers): a load whose byte offset lies outside the range returns
// zeros instead of touching memory, so a kernel can issue every load of a
// tile unconditionally (no branch around it, no wait right after it) and get
// the zero values of points outside the grid for free.  BUF_OOB is an offset
// outside every range the kernels build (arrays are addressed per plane).
constexpr unsigned BUF_OOB = 0x80000000u;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void *base, unsigned bytes)
{
    // dword 3: raw (stride 0) 32-bit data format, range-checked by offset
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), 0, (int)bytes, 0x00020000);
}

template <typename T>
__device__ __forceinline__ cx<T> ld_buf(__amdgpu_buffer_rsrc_t r, unsigned off)
{
    if constexpr (sizeof(T) == 4)
        return __builtin_bit_cast(cx<T>, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
    else
        return __builtin_bit_cast(cx<T>, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
}

// Barrier of a workgroup whose threads exchange data through LDS only: the
// fences order LDS accesses around it and leave global loads in flight (a
// full __syncthreads also waits for every outstanding global load, which
// defeats loads issued a plane ahead).  Not for data passed through global
// memory.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Block index -> tile index such that each XCD (blocks are dispatched
// round-robin over the 8 XCDs) receives a contiguous run of tiles, so halo
// rows shared by neighbouring tiles are served by the same L2.
__host__ __device__ __forceinline__ int xcd_tile(int b, int nb)
{
    const int X = 8;
    int xcd = b % X, local = b / X;
    int q = nb / X, r = nb % X;
    return (xcd < r) ? xcd * (q + 1) + local : r * (q + 1) + (xcd - r) * q + local;
}

// The block index that xcd_tile maps to tile t.
__host__ __device__ __forceinline__ int xcd_tile_inv(int t, int nb)
{
    const int X = 8;
    int q = nb / X, r = nb % X;
    int xcd, local;
    if (t < r * (q + 1)) {
        xcd = t / (q + 1);
        local = t - xcd * (q + 1);
    } else {
        int t2 = t - r * (q + 1);
        xcd = r + t2 / q;
        local = t2 - (xcd - r) * q;
    }
    return local * X + xcd;
}

// The incoming plane wave exp(i k0 e^{i gamma} eta.x) of the right-hand side
// (Sec. 2.1) is a product of one factor per axis on the tensor grid:
// E_k[i] = exp(c_k x_i), c_k = cr_k + i ci_k = i k0 e^{i gamma} eta_k, at
// x_i = lo_k + (i + 1) h_k.  A level's factors are stored [E_x | E_y | E_z]
// (mx + my + mz values).
__device__ __forceinline__ cd pw_factor(int i, double lo, double h, double cr, double ci)
{
    const double x = lo + (double)(i + 1) * h;
    const double mag = exp(cr * x), ph = ci * x;
    return cd{mag * cos(ph), mag * sin(ph)};
}

// (x, y, z) of flat index j = x + mx (y + my z), in 32-bit arithmetic when j
// fits (a 64-bit division costs several times a 32-bit one).
__device__ __forceinline__ void split3(size_t j, int mx, int my, int &x, int &y, int &z)
{
    if (j <= 0xffffffffull) {
        const unsigned u = (unsigned)j, r = u / (unsigned)mx;
        x = (int)(u - r * (unsigned)mx);
        y = (int)(r % (unsigned)my);
        z = (int)(r / (unsigned)my);
    } else {
        const size_t r = j / mx;
        x = (int)(j - r * mx);
        y = (int)(r % my);
        z = (int)(r / my);
    }
}

// (x, y, z) of flat index j = x + mx (y + my z) stepped by a fixed stride
// without a division per step (grid-stride loops): the stride's own digits
// are added with carries.
struct GridWalk {
    int x, y, z, sx, sy, sz, mx, my;
    __device__ __forceinline__ GridWalk(size_t j, size_t stride, int mx_, int my_) : mx(mx_), my(my_)
    {
        const size_t pl = (size_t)mx_ * my_;
        x = (int)(j % mx_);
        y = (int)((j / mx_) % my_);
        z = (int)(j / pl);
        sx = (int)(stride % mx_);
        sy = (int)((stride / mx_) % my_);
        sz = (int)(stride / pl);
    }
    __device__ __forceinline__ void step()
    {
        x += sx;
        int c = 0;
        if (x >= mx) {
            x -= mx;
            c = 1;
        }
        y += sy + c;
        c = 0;
        if (y >= my) {
            y -= my;
            c = 1;
        }
        z += sz + c;
    }
};

// The plane wave at interior point (ix, iy, iz): (E_x E_y) E_z, or E_x E_y in
// 2D.  Every kernel that forms the right-hand side q u_in takes it from here,
// in this order, so a stored and a recomputed right-hand side agree bit for
// bit.
__device__ __forceinline__ cd pw_uin(const cd *__restrict__ f, int ix, int iy, int iz, int mx, int my, int dim)
{
    const cd v = f[ix] * f[mx + iy];
    return dim == 3 ? v * f[mx + my + iz] : v;
}

}  // namespace ffmg
