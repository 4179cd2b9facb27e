// ffmg_internal.hpp -- host-side declarations shared by the library's
// translation units (kernel launchers and the handle).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "ffmg_device.hpp"

namespace ffmg {

enum StencilMode { MODE_APPLY = 0, MODE_RESID = 1, MODE_JACOBI = 2, MODE_RNORM = 3, MODE_JACOBI0 = 4 };

// Geometry of one level (interior extents, spacings, origin).
struct LevelGeom {
    int dim;
    int m[3];        // interior points per axis (1 for unused axes)
    double h[3];
    double lo[3];
    size_t N() const { return (size_t)m[0] * m[1] * m[2]; }
};

template <typename T>
Stencil<T> make_stencil(const LevelGeom &g, double gamma, double k02, double omega);

// Number of per-block partial sums a MODE_RESID / MODE_RNORM launch writes.
int stencil_blocks(const LevelGeom &g);

// out = f(u, b, q) per mode; partial[blocks] receives sum |r|^2 per block in
// MODE_RESID and MODE_RNORM (may be null in MODE_RESID).
// finest = true gives MODE_JACOBI launches their own kernel symbol.
template <typename T>
void launch_stencil(int mode, const LevelGeom &g, const Stencil<T> &P, const cx<T> *u,
                    const cx<T> *b, const cx<T> *q, cx<T> *out, double *partial, hipStream_t s,
                    bool finest = false);

template <typename T>
void launch_restrict(const LevelGeom &fine, const cx<T> *rf, cx<T> *bc, hipStream_t s);

template <typename T>
void launch_prolong_add(const LevelGeom &fine, const cx<T> *ec, cx<T> *uf, hipStream_t s);

// sum of nparts doubles -> *out (device), deterministic single-block reduce.
void launch_sum(const double *parts, int nparts, double *out, hipStream_t s);

// Setup kernels.
void launch_make_q(const cd *coef, cd *q, size_t N, double scale, double *bad_parts, int nparts,
                   hipStream_t s);
template <typename T>
void launch_inject(const LevelGeom &fine, const cx<T> *qf, cx<T> *qc, hipStream_t s);
template <typename To, typename Ti>
void launch_convert(const cx<Ti> *in, cx<To> *out, size_t N, hipStream_t s);
void launch_build_coarse(const LevelGeom &g, const Stencil<double> &P, const cd *q, cd *aug, hipStream_t s);
void launch_gauss_jordan(cd *aug, int n, int *info, hipStream_t s);
template <typename T>
void launch_coarse_apply(const cd *Ainv, int n, const cx<T> *b, cx<T> *u, hipStream_t s);
void launch_rhs_plane_wave(const LevelGeom &g, double gamma, double k0, const double eta[3],
                           const cd *q, cd *b, hipStream_t s);

// Mixed-precision refinement: u64 += s * d32; r64 = b - A u64 -> r32 = r64 / scale.
void launch_refine_update(const cf *d, cd *u, double scale, size_t N, hipStream_t s);
void launch_resid_to_f32(const LevelGeom &g, const Stencil<double> &P, const cd *u, const cd *b,
                         const cd *q, cf *r32, double inv_scale, double *partial, hipStream_t s);

// Far field (ffmg_farfield.hip).
struct FarFieldPlan;
FarFieldPlan *ff_plan_create();
void ff_plan_destroy(FarFieldPlan *p);
hipError_t ff_plan_prepare(FarFieldPlan *p, const LevelGeom &g, double k0, double gamma, int M, const double *dirs,
                           const cd *s_field, hipStream_t s);
hipError_t ff_plan_execute(FarFieldPlan *p, const LevelGeom &g, double gamma, cd *F_out, hipStream_t s);
void launch_ff_integrand(const LevelGeom &g, const cd *q, const cd *u, const cd *E, cd *s, hipStream_t st);
void launch_axis_exp(cd *out, int m, double lo, double h, double cr, double ci, hipStream_t s);
}  // namespace ffmg
