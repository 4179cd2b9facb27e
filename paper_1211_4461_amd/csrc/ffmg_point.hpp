// ffmg_point.hpp -- the per-point arithmetic of the contour operator, shared
// by every kernel that applies it (one-operation, fused and LDS-tail
// kernels), so that all of them produce the same bits for the same inputs.
//
//   (A u)_j = e^{-2 i gamma} sum_k (2 u_j - u_{j-e_k} - u_{j+e_k}) / h_k^2
//             - (k0^2 + q_j) u_j                                 (Sec. 3.2, eq. csg)
//   D_j     = e^{-2 i gamma} sum_k 2 / h_k^2 - (k0^2 + q_j)        (Jacobi diagonal)
//   (A u)_j = D_j u_j - e^{-2 i gamma} N_j,  N_j = sum_k (u_{j-e_k} + u_{j+e_k}) / h_k^2
//
// The rotation e^{-2 i gamma} is common to every axis, so the real weighted
// second differences are summed first and multiplied by it once.  Products
// use explicit fused multiply-adds (the library is compiled without implicit
// contraction, so the rounding is the same in every kernel).  The reciprocal
// of D is the hardware reciprocal in FP32 (the FP32 cycle is the inner
// solver of the FP64 refinement) and a correctly rounded division in FP64.
#pragma once

#include "ffmg_device.hpp"

namespace ffmg {

__device__ __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float rcp_(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp_(double x) { return 1.0 / x; }

template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b)
{
    return {fma_(a.re, b.re, -(a.im * b.im)), fma_(a.re, b.im, a.im * b.re)};
}

template <typename T>
__device__ __forceinline__ cx<T> crecip(cx<T> a)
{
    T inv = rcp_(fma_(a.re, a.re, a.im * a.im));
    return {a.re * inv, -(a.im * inv)};
}

// sum_k (2 u - u_- - u_+) / h_k^2 for the x and y axes (real weights).
template <typename T>
__device__ __forceinline__ cx<T> lap_xy(const Stencil<T> &P, cx<T> uc, cx<T> w, cx<T> e, cx<T> s, cx<T> n)
{
    T tr = uc.re + uc.re, ti = uc.im + uc.im;
    T xr = (tr - w.re) - e.re, xi = (ti - w.im) - e.im;
    T yr = (tr - s.re) - n.re, yi = (ti - s.im) - n.im;
    return {fma_(yr, P.ih2[1], xr * P.ih2[0]), fma_(yi, P.ih2[1], xi * P.ih2[0])};
}

// adds the z-axis term
template <typename T>
__device__ __forceinline__ cx<T> lap_add_z(const Stencil<T> &P, cx<T> L, cx<T> uc, cx<T> d, cx<T> u_)
{
    T tr = uc.re + uc.re, ti = uc.im + uc.im;
    T zr = (tr - d.re) - u_.re, zi = (ti - d.im) - u_.im;
    return {fma_(zr, P.ih2[2], L.re), fma_(zi, P.ih2[2], L.im)};
}

// A u at a point from the weighted second differences L.
template <typename T>
__device__ __forceinline__ cx<T> apply_point(const Stencil<T> &P, cx<T> L, cx<T> uc, cx<T> qj)
{
    cx<T> kap = {P.k02 + qj.re, qj.im};
    cx<T> a = cmul(P.rot, L), k = cmul(kap, uc);
    return {a.re - k.re, a.im - k.im};
}

template <typename T>
__device__ __forceinline__ cx<T> resid_from(const Stencil<T> &P, cx<T> L, cx<T> uc, cx<T> bj, cx<T> qj)
{
    cx<T> Au = apply_point(P, L, uc, qj);
    return {bj.re - Au.re, bj.im - Au.im};
}

// The Jacobi weight omega / D_j of a point (a function of q_j only: kernels
// that sweep a point several times form it once).
template <typename T>
__device__ __forceinline__ cx<T> jweight(const Stencil<T> &P, cx<T> qj)
{
    cx<T> D = {P.csum2.re - (P.k02 + qj.re), P.csum2.im - qj.im};
    cx<T> r = crecip(D);
    return {P.omega * r.re, P.omega * r.im};
}

// N = sum_k (u_- + u_+) / h_k^2 for the x and y axes (real weights), and the
// z-axis term added to it.
template <typename T>
__device__ __forceinline__ cx<T> nsum_xy(const Stencil<T> &P, cx<T> w, cx<T> e, cx<T> s, cx<T> n)
{
    return {fma_(s.re + n.re, P.ih2[1], (w.re + e.re) * P.ih2[0]),
            fma_(s.im + n.im, P.ih2[1], (w.im + e.im) * P.ih2[0])};
}

template <typename T>
__device__ __forceinline__ cx<T> nsum_add_z(const Stencil<T> &P, cx<T> N, cx<T> d, cx<T> u_)
{
    return {fma_(d.re + u_.re, P.ih2[2], N.re), fma_(d.im + u_.im, P.ih2[2], N.im)};
}

// One omega-Jacobi update u + omega (b - A u) / D.  Since A u = D u - rot N
// (N the weighted neighbour sum), it equals (1 - omega) u + (omega / D)
// (b + rot N), which needs neither the residual nor a division per sweep.
// The rounding of the new iterate is of the order of eps |u| either way; the
// residual itself (restriction, norms, refinement) keeps the
// second-difference form, whose rounding does not grow with 1 / h^2.
template <typename T>
__device__ __forceinline__ cx<T> jacobi_n(const Stencil<T> &P, cx<T> N, cx<T> uc, cx<T> bj, cx<T> wj)
{
    cx<T> rn = cmul(P.rot, N);
    cx<T> t = {bj.re + rn.re, bj.im + rn.im};
    cx<T> v = cmul(wj, t);
    return {fma_(P.omc, uc.re, v.re), fma_(P.omc, uc.im, v.im)};
}

// first sweep from a zero guess: (omega / D) b
template <typename T>
__device__ __forceinline__ cx<T> jacobi0_w(cx<T> bj, cx<T> wj)
{
    return cmul(wj, bj);
}

// 2D sweep from the five stencil values and the point's weight
template <typename T>
__device__ __forceinline__ cx<T> jacobi_point(const Stencil<T> &P, cx<T> uc, cx<T> w, cx<T> e, cx<T> s, cx<T> n,
                                              cx<T> bj, cx<T> wj)
{
    return jacobi_n(P, nsum_xy(P, w, e, s, n), uc, bj, wj);
}

template <typename T>
__device__ __forceinline__ cx<T> resid_point(const Stencil<T> &P, cx<T> uc, cx<T> w, cx<T> e, cx<T> s, cx<T> n,
                                             cx<T> bj, cx<T> qj)
{
    return resid_from(P, lap_xy(P, uc, w, e, s, n), uc, bj, qj);
}

}  // namespace ffmg
