// ffmg_internal.hpp -- host-side declarations shared by the library's
// translation units (kernel launchers and the handle).
//
// Every launcher that runs inside the solve loop takes `stop`, a device int
// (or null): when it is non-zero the kernel returns at entry.  The solve loop
// enqueues several V-cycles ahead; once the control kernel (k_ctl_update)
// has decided to stop, the cycles already queued cost only empty launches
// and leave every result untouched.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "ffmg_device.hpp"

namespace ffmg {

enum StencilMode { MODE_APPLY = 0, MODE_RESID = 1, MODE_JACOBI = 2, MODE_RNORM = 3, MODE_JACOBI0 = 4 };

// Kernels timed by the optional event instrumentation (mg_profile_*).
enum ProfKernel {
    PROF_PRE = 0,      // finest-level pre-smoothing (fused 2-sweep kernel, or each sweep)
    PROF_FF = 1,       // far-field contraction
    PROF_POST = 2,     // finest-level interpolation + post-smoothing (fused)
    PROF_REFINE = 3,   // FP64 update + residual of the refinement loop (fused)
    PROF_FFGEMM = 4,   // far-field GEMM stages alone
    PROF_NET = 5,      // learned-smoother network application (finest level)
    PROF_RR = 6,       // finest-level residual + full-weighting restriction (3D)
    PROF_SRR = 7,      // finest-level pre-smoothing pair from a guess + residual + restriction in one pass (3D)
    PROF_SRR0 = 8,     // the same from a zero guess
    PROF_N = 9
};

// Device-resident state of one solve (residual-reduction stopping test of
// Sec. 4, growth test, and the scales of the mixed-precision refinement).
// Timing of one launch for the library's profiling.  While set, the next
// launch made through launch_maybe_timed() carries these two events, which the
// runtime stamps when that kernel itself starts and ends; the interval leaves
// out the time the kernel waits in its queue behind other streams' work.
struct KernelTiming {
    hipEvent_t start = nullptr, stop = nullptr;
    bool used = false;
};
extern thread_local KernelTiming tl_kernel_timing;

template <typename F, typename... Args>
inline void launch_maybe_timed(F kernel, dim3 grid, dim3 block, uint32_t shm, hipStream_t s, Args... args)
{
    KernelTiming &t = tl_kernel_timing;
    if (t.start && !t.used) {
        t.used = true;
        hipExtLaunchKernelGGL(kernel, grid, block, shm, s, t.start, t.stop, 0u, args...);
    } else {
        hipLaunchKernelGGL(kernel, grid, block, shm, s, args...);
    }
}

struct SolveCtl {
    double tol2b2;     // (tol ||b||)^2
    double inv_sqN;    // 1 / sqrt(N)
    double r0_2;       // ||r_0||^2
    double rk2;        // latest ||r_k||^2
    double prev2;      // ||r_{k-1}||^2
    double scale_cur;  // the FP32 right-hand side now in use is r / scale_cur
    double scale_next; // the next one is written as r / scale_next
    int done;          // 0 running, 1 converged, 2 residual grew 3 times, 3 cycle limit, 4 non-finite,
                       // 5 b = 0 or non-finite (set at init: nothing runs)
    int k;             // completed cycles / refinement steps
    int grow;
    int max_cycles;
    double b2;         // ||b||^2
};

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
void launch_stencil(int mode, const LevelGeom &g, const Stencil<T> &P, const cx<T> *u, const cx<T> *b,
                    const cx<T> *q, cx<T> *out, double *partial, hipStream_t s, bool finest = false,
                    const int *stop = nullptr);

// 3D residual + full weighting in one pass: bc = FW(b - A u) on the coarse
// level (bit for bit the MODE_RESID launch followed by launch_restrict).
template <typename T>
void launch_resid_restrict3d(const LevelGeom &fine, const Stencil<T> &P, const cx<T> *u, const cx<T> *b,
                             const cx<T> *q, cx<T> *bc, hipStream_t s, const int *stop = nullptr);
// 3D Jacobi sweep with its input formed on the fly: zero2 = the two sweeps
// from a zero guess in one pass (u unused), else u + P ec (the coarse-grid
// correction fused into the sweep).  u and ec are not written.
template <typename T>
void launch_sweep3d_fused(bool zero2, const LevelGeom &g, const Stencil<T> &P, const cx<T> *u, const cx<T> *ec,
                          const cx<T> *b, const cx<T> *q, cx<T> *out, hipStream_t s, bool finest,
                          const int *stop = nullptr);
template <typename T>
void launch_restrict(const LevelGeom &fine, const cx<T> *rf, cx<T> *bc, hipStream_t s, const int *stop = nullptr);

template <typename T>
void launch_prolong_add(const LevelGeom &fine, const cx<T> *ec, cx<T> *uf, hipStream_t s,
                        const int *stop = nullptr);

template <typename T>
void launch_copy(const cx<T> *src, cx<T> *dst, size_t N, hipStream_t s, const int *stop);
template <typename T>
void launch_zero(cx<T> *dst, size_t N, hipStream_t s, const int *stop);

// sum of nparts doubles -> *out (device), deterministic single-block reduce.
void launch_sum(const double *parts, int nparts, double *out, hipStream_t s);

// Solve control: init from ||b||^2 (device scalar), update from per-block
// partial sums of ||r||^2 (same reduction order as launch_sum).
void launch_ctl_init(SolveCtl *ctl, const double *bnorm2, double tol, size_t N, int max_cycles, hipStream_t s);
void launch_ctl_update(SolveCtl *ctl, const double *parts, int nparts, hipStream_t s);

// Setup kernels.
void launch_make_q(const cd *coef, cd *q, size_t N, double scale, double *bad_parts, int nparts, hipStream_t s);
template <typename T>
void launch_inject(const LevelGeom &fine, const cx<T> *qf, cx<T> *qc, hipStream_t s);
template <typename To, typename Ti>
void launch_convert(const cx<Ti> *in, cx<To> *out, size_t N, hipStream_t s);
// GMRES(m) smoothing (ffmg_krylov.hip).  Scalars of one step (doubles):
// n_i = |Z_i|^2 at [0, GMRES_MAX_M], d_ij = <Z_i, A Z_j> at GM_D + 2 (j
// GMRES_MAX_M + i) (re, im), the coefficients at GM_C + 2 j.
constexpr int GMRES_MAX_M = 8;
constexpr int GM_D = 16;
constexpr int GM_C = GM_D + 2 * GMRES_MAX_M * GMRES_MAX_M;
constexpr int GM_S = GM_C + 2 * GMRES_MAX_M;
constexpr int GM_PARTS = (GMRES_MAX_M + 1 + 2 * GMRES_MAX_M * GMRES_MAX_M) * 1024;
// One GMRES(m) smoothing step in place on a level (zero: u is 0 on entry);
// Z: m + 2 vectors of the level, S: GM_S doubles, parts: GM_PARTS doubles;
// fused: m + 3 launches, else the reference 4 m + 3.
template <typename T>
void launch_gmres_step(const LevelGeom &g, const Stencil<T> &P, const cx<T> *b, const cx<T> *q, cx<T> *u, bool zero,
                       int m, cx<T> *Z, double *S, double *parts, hipStream_t s, const int *stop, bool fused);

// One red-black Gauss-Seidel sweep in place on a level (red points, then
// black; ffmg_rbgs.hip).
template <typename T>
void launch_rbgs_sweep(const LevelGeom &g, const Stencil<T> &P, const cx<T> *b, const cx<T> *q, cx<T> *u,
                       hipStream_t s, const int *stop);

// Full multigrid transfers: the finest right-hand side at the first coarse
// level's nodes, divided by s = sqrt(*bnorm2 / N) (s = 1 when bnorm2 is
// null), and uf = s P ec overwriting uf (inv_sqN = 1 / sqrt(N) of the finest
// level; s = 1 when bnorm2 is null).  bf = null: the finest right-hand side
// is the plane wave's q u_in, from the finest q (qf) and its factors (pwf).
template <typename TO>
void launch_inject_rhs(const LevelGeom &fine, const cd *bf, cx<TO> *bc, const double *bnorm2, hipStream_t s,
                       const cd *qf = nullptr, const cd *pwf = nullptr);
template <typename TC, typename TF>
void launch_prolong_set(const LevelGeom &fine, const cx<TC> *ec, cx<TF> *uf, const double *bnorm2, double inv_sqN,
                        hipStream_t s);
void launch_build_coarse(const LevelGeom &g, const Stencil<double> &P, const cd *q, cd *aug, hipStream_t s);
// Gauss-Jordan inverse of the coarsest operator: one block up to
// GJ_ONE_BLOCK_MAX unknowns, above that blocked over the whole device (ws:
// gauss_jordan_ws(n) complex values of workspace).
constexpr int GJ_ONE_BLOCK_MAX = 256;
void launch_gauss_jordan(cd *aug, int n, int *info, hipStream_t s, cd *ws);
size_t gauss_jordan_ws(int n);
template <typename T>
void launch_coarse_apply(const cd *Ainv, int n, const cx<T> *b, cx<T> *u, hipStream_t s, const int *stop = nullptr);
// The incoming plane wave's per-axis factors on g into f (g.m[0] + g.m[1] +
// g.m[2] values, the layout of pw_uin), and b = q u_in from them.
void launch_pw_factors(const LevelGeom &g, double gamma, double k0, const double eta[3], cd *f, hipStream_t s);
void launch_rhs_plane_wave(const LevelGeom &g, const cd *q, const cd *f, cd *b, hipStream_t s);
void launch_rhs_phase(const LevelGeom &g, double gamma, double k0, const double eta[3], const cd *q, cd *b,
                      hipStream_t s);

// Mixed-precision refinement (one-operation form): u64 += s * d32 with
// s = ctl->scale_cur; r64 = b - A u64 written as r64 / ctl->scale_next.
void launch_refine_update(const cf *d, cd *u, const SolveCtl *ctl, size_t N, hipStream_t s, const int *stop);
// 3D refinement step in one pass: unew = u + s d, r32 = (b - A unew) / scale_next, block sums of |b - A unew|^2
// (stencil_blocks(g) partials); b = null: the plane-wave right-hand side q u_in from the factors pwf
void launch_refine3d(const LevelGeom &g, const Stencil<double> &P, const cd *u, const cf *d, const cd *b,
                     const cd *q, cd *unew, cf *r32, const SolveCtl *ctl, double *partial, hipStream_t s,
                     const int *stop, const cd *pwf = nullptr);
// The FP32 full multigrid start's last interpolation fused with the initial
// residual (3D): u = s P ec (s from bnorm2, as launch_prolong_set<float,
// double>; u = null: not stored) and r32 = (b - A u) / ctl->scale_next with
// the block sums of launch_resid_to_f32_ctl (b = null: the plane wave's q u_in
// from pwf).
void launch_fmg_resid3d(const LevelGeom &g, const Stencil<double> &P, const cf *ec, const cd *b, const cd *q, cd *u,
                        cf *r32, const SolveCtl *ctl, double *partial, const double *bnorm2, const cd *pwf,
                        hipStream_t s);
// The first refinement step after that fused start (3D): the iterate
// s P ec formed from the staged FP32 coarse planes instead of read, then as
// launch_refine3d (unew = s P ec + scale d, its scaled residual and sums).
void launch_refine3d_start(const LevelGeom &g, const Stencil<double> &P, const cf *ec, const cf *d, const cd *b,
                           const cd *q, cd *unew, cf *r32, const SolveCtl *ctl, double *partial, hipStream_t s,
                           const int *stop, const cd *pwf, const double *bnorm2);
// r32 = (q u_in - A u) / ctl->scale_next with block sums of its FP64 square
// (the blocks of launch_resid_to_f32_ctl)
void launch_resid_pw(const LevelGeom &g, const Stencil<double> &P, const cd *u, const cd *q, cf *r32,
                     const SolveCtl *ctl, double *partial, const cd *pwf, hipStream_t s);
// two Jacobi sweeps in one 3D pass from u (ec: from u + P ec; zero: from a zero guess, u not read);
// shape: the tile, as FFMG_TUNE_SWEEP3D variants 0, 2, 3 and 4 (the same bits with every tile)
template <typename T>
void launch_sweep2_3d(const LevelGeom &g, const Stencil<T> &P, const cx<T> *u, const cx<T> *ec, const cx<T> *b,
                      const cx<T> *q, cx<T> *out, hipStream_t s, bool finest, const int *stop, bool zero = false,
                      int shape = 0);
// two Jacobi sweeps from u (null: from a zero guess) into out, then the
// residual of the result and its full weighting into bc, in one 3D pass (FP32;
// the bits of launch_sweep2_3d followed by launch_resid_restrict3d)
bool sweep2rr_3d_fits(const LevelGeom &g);
template <typename T>
void launch_sweep2rr_3d(const LevelGeom &g, const Stencil<T> &P, const cx<T> *u, const cx<T> *b, const cx<T> *q,
                        cx<T> *out, cx<T> *bc, hipStream_t s, bool finest, const int *stop);
void launch_resid_to_f32(const LevelGeom &g, const Stencil<double> &P, const cd *u, const cd *b, const cd *q,
                         cf *r32, double inv_scale, double *partial, hipStream_t s);
void launch_resid_to_f32_ctl(const LevelGeom &g, const Stencil<double> &P, const cd *u, const cd *b, const cd *q,
                             cf *r32, const SolveCtl *ctl, double *partial, hipStream_t s, const int *stop);

// Fused 2D level kernels (ffmg_fused2d.hip).  launch_smooth2d runs 1 or 2
// sweeps from u (or from 0 when zero) into out; with ec != null the coarse
// correction P ec is added to u first; th: tile height (4, 8 or 16 rows).
int fused2d_blocks(const LevelGeom &g);
template <typename T>
void launch_smooth2d(const LevelGeom &g, const Stencil<T> &P, int nsweeps, bool zero, const cx<T> *u,
                     const cx<T> *ec, const cx<T> *b, const cx<T> *q, cx<T> *out, hipStream_t s, bool finest,
                     const int *stop, int th);
template <typename T>
void launch_resid_restrict2d(const LevelGeom &g, const Stencil<T> &P, const cx<T> *u, const cx<T> *b,
                             const cx<T> *q, cx<T> *bc, hipStream_t s, const int *stop);
// Two Jacobi sweeps (zero: from u = 0, u not read) into out, the residual of
// the smoothed iterate and its full weighting into bc, in one pass (the same
// bits as launch_smooth2d with two sweeps followed by launch_resid_restrict2d);
// fh: tile height, 8 or 16 rows (0: 16 for FP32, 8 for FP64).
template <typename T>
void launch_smooth_rr2d(const LevelGeom &g, const Stencil<T> &P, bool zero, const cx<T> *u, const cx<T> *b,
                        const cx<T> *q, cx<T> *out, cx<T> *bc, hipStream_t s, bool finest, const int *stop, int fh);
void launch_refine2d(const LevelGeom &g, const Stencil<double> &P, const cd *u, const cf *d, const cd *b,
                     const cd *q, cd *u_out, cf *r32, const SolveCtl *ctl, double *partial, hipStream_t st,
                     const int *stop, const cd *pwf = nullptr);

// The coarse end of a 2D V-cycle in one workgroup, all fields in LDS: the
// levels lt .. L-1 of the hierarchy (small enough for LDS) and the exact
// coarsest solve.  Reads b of level lt, writes its correction u (zero guess).
constexpr int TAIL_MAX_LEVELS = 6;
template <typename T>
struct TailLevel {
    int mx, my;
    int off;               // element offset of this level's fields in LDS
    Stencil<T> P;
    const cx<T> *q;
};
template <typename T>
struct TailParams {
    int nt;                // tail levels including the coarsest
    int nu1, nu2;
    const cd *aug;         // [A | A^{-1}] of the coarsest level, row stride 2 nc
    int nc;
    TailLevel<T> lv[TAIL_MAX_LEVELS];
};
// LDS bytes the tail needs for the given levels (0 if it does not fit).
template <typename T>
size_t tail2d_lds_bytes(const int *mx, const int *my, int nt);
template <typename T>
void launch_tail2d(const TailParams<T> &tp, size_t lds_bytes, const cx<T> *b_top, cx<T> *u_top, hipStream_t s,
                   const int *stop);
// Full multigrid start on tail levels s0 .. nt - 1 (b_top: level s0's
// right-hand side; u_top: its solution after k V-cycles there).
template <typename T>
void launch_tail2d_fmg(const TailParams<T> &tp, size_t lds_bytes, const cx<T> *b_top, cx<T> *u_top, int s0, int k,
                       hipStream_t s);

// Batched fused 2D kernels (one launch for many instances).  Each job is one
// instance's level; a launch's tiles are the jobs' tiles back to back
// (job j owns tiles [tile0, tile0 + its tile count)), tile_job maps a tile to
// its job.  A job whose stop flag is set is skipped.
template <typename T>
struct SmoothJob {
    const cx<T> *u, *ec, *b, *q;
    cx<T> *out;
    Stencil<T> P;
    int tiles_x, tile0;
    const int *stop;
};
template <typename T>
struct RRJob {
    const cx<T> *u, *b, *q;
    cx<T> *bc;
    Stencil<T> P;
    int ctiles_x, tile0;
    const int *stop;
};
template <typename T>
struct SRRJob {             // one-pass pre-smoothing + residual + restriction
    const cx<T> *u, *b, *q;
    cx<T> *out, *bc;
    Stencil<T> P;
    int tiles_x, tile0;
    const int *stop;
};
struct RefineJob {
    const cd *u;
    const cf *d;
    const cd *b, *q;       // b = null: the plane wave's q u_in from f
    const cd *f;
    cd *u_out;
    cf *r32;
    const SolveCtl *ctl;
    Stencil<double> P;
    int tiles_x, tile0, ntiles;
    double *partial;
    const int *stop;
};
template <typename T>
struct TailJob {
    TailParams<T> tp;
    const cx<T> *b_top;
    cx<T> *u_top;
    const int *stop;
};
// Tile counts (and tiles per row) of the fused kernels on a level, for a
// tile height th (the batched path's heights: batch_tiles of its variant).
template <typename T>
int smooth2d_tiles(const LevelGeom &g, int *tiles_x, int th);
int resid_restrict2d_tiles(const LevelGeom &g, int *ctiles_x);
template <typename T>
int smooth_rr2d_tiles(const LevelGeom &g, int *tiles_x, int th);
int refine2d_tiles(const LevelGeom &g, int *tiles_x);
constexpr int BATCH_TUNE_VARIANTS = 4;
void batch_tiles(int variant, int *th_smooth, int *th_srr);
template <typename T>
void launch_smooth2d_batch(int nsweeps, bool zero, bool prol, const SmoothJob<T> *jobs, const int *tile_job,
                           int ntiles, hipStream_t s, int th);
template <typename T>
void launch_smooth_rr2d_batch(bool zero, const SRRJob<T> *jobs, const int *tile_job, int ntiles, hipStream_t s,
                              int th);
template <typename T>
void launch_resid_restrict2d_batch(const RRJob<T> *jobs, const int *tile_job, int ntiles, hipStream_t s);
void launch_refine2d_batch(const RefineJob *jobs, const int *tile_job, int ntiles, hipStream_t s);
template <typename T>
void launch_tail2d_batch(const TailJob<T> *jobs, int njobs, size_t lds_bytes, hipStream_t s);
// the full multigrid start of each job's tail (from its first level), k
// V-cycles per level
template <typename T>
void launch_tail2d_fmg_batch(const TailJob<T> *jobs, int njobs, int k, size_t lds_bytes, hipStream_t s);

// Per-instance setup of a batched solve (ffmg_stencil.hip): the plane wave's
// factors, zero guess, ||b||^2, control init and the initial scaled FP32
// residual, in the block structure of the single-instance kernels (b = q u_in
// formed where it is read).
struct InitJob {
    const cd *q;
    cd *u;
    cd *f;                 // the plane wave's per-axis factors (mx + my values); b = q u_in is not stored
    cf *r32;
    SolveCtl *ctl;
    double *partial;
    Stencil<double> P;
    LevelGeom g;
    double eta[3];
    double ar_s, ai_s;     // i k0 e^{i gamma} = ar_s + i ai_s
    double tol, inv_sqN;   // inv_sqN = 1 / sqrt(N), formed on the host as in the single solve
    int max_cycles;
    int nb_norm, nb_res, tiles_x;
};
struct CtlJob {
    SolveCtl *ctl;
    const double *parts;
    int n;
};
struct FinishJob {
    const cd *t;           // the other buffer of the FP64 iterate
    cd *u;
    const SolveCtl *ctl;
    size_t N;
};
// One 2D grid transfer of the batched full multigrid start (ffmg_stencil.hip),
// with the arithmetic of the single-instance k_inject_rhs / k_inject /
// k_prolong_set: injection of a right-hand side onto the next coarser level
// (from the FP64 finest level: divided by the RMS scale), or the coarse
// solution interpolated onto the next finer level (into the FP64 finest
// level: multiplied by it).
struct XferJob {
    const void *src;          // kind 0 with src = null: the plane wave's q u_in (qf, pwf)
    void *dst;
    const cd *qf, *pwf;
    int mxf, myf, mxc, myc;   // fine and coarse interior extents
    const double *bnorm2;     // ||b||^2 of the finest level when an FP64 end is involved, else null
    double inv_sqN;           // 1 / sqrt(N) of the finest level
    const int *stop;          // the instance's control flag: nonzero skips the job
};
// kind 0: FP64 -> FP32 right-hand-side injection; 1: FP32 injection;
// 2: FP32 -> FP32 interpolation; 3: FP32 -> FP64 interpolation.  max_n: the
// largest output grid among the jobs.
void launch_xfer_batch(int kind, const XferJob *jobs, int njobs, size_t max_n, hipStream_t s);
int norm2_blocks(size_t N);
void launch_hash_fill(cd *out, size_t N, unsigned long long seed, hipStream_t s);
void stencil_grid2d(const LevelGeom &g, int *nb, int *tiles_x);   // blocks and tiles per row of k_stencil2d
// the plane wave's factors, u = 0 (zero), ||b||^2 and the control block
// (max_m: the largest grid extent among the instances)
void launch_init_batch(const InitJob *jobs, int n, int max_nb_norm, int max_m, bool zero, hipStream_t s);
// the initial residual b - A u as the scaled FP32 right-hand side
void launch_init_resid_batch(const InitJob *jobs, int n, int max_nb_res, hipStream_t s);
void launch_ctl_update_batch(const CtlJob *jobs, int n, hipStream_t s);
void launch_count_done(const CtlJob *jobs, int n, int *ndone, hipStream_t s);
void launch_finish_batch(const FinishJob *jobs, int n, hipStream_t s);

// Far field (ffmg_farfield.hip).
struct FarFieldPlan;
FarFieldPlan *ff_plan_create();
void ff_plan_destroy(FarFieldPlan *p);
// prec: ffmg_ff_precision (0 FP64 MFMA, 1 split BF16 x3, 2 split BF16 x6).
hipError_t ff_plan_prepare(FarFieldPlan *p, const LevelGeom &g, double k0, double gamma, int M, const double *dirs,
                           int prec, hipStream_t s);
hipError_t ff_plan_integrand(FarFieldPlan *p, const LevelGeom &g, const cd *q, const cd *u, const cd *E,
                             hipStream_t s);
hipError_t ff_plan_contract(FarFieldPlan *p, const LevelGeom &g, hipStream_t s);
hipError_t ff_plan_finish(FarFieldPlan *p, const LevelGeom &g, double gamma, cd *F_out, hipStream_t s);
// Batched 2D split-BF16 far fields (farfield_map_batched): instance i has
// its operator's plan (prepared for the same M directions), grid, finest q,
// solution u (null: the Born term), output row F (device), direction eta and
// the operator's k0 and gamma.  The workspace is cached in *cache for the
// list key and rebuilt when it changes; everything is queued on s.
struct FFBInst {
    const FarFieldPlan *plan;
    const LevelGeom *g;
    const cd *q, *u;
    cd *F;
    double eta[3];
    double k0, gamma;
};
struct FFBatch;
void ff_batch_destroy(FFBatch *b);
hipError_t ff_batch_run(FFBatch **cache, const std::vector<uint64_t> &key, const std::vector<FFBInst> &in, int M,
                        hipStream_t s);
// split-GEMM tile variants (autotuning)
int ff_plan_variants();
int ff_plan_default_variant();
void ff_plan_set_variant(FarFieldPlan *p, int v);
int ff_plan_variant(const FarFieldPlan *p);
// Number of times the plan was rebuilt (its buffers freed and reallocated):
// a workspace that keeps pointers into the plan is valid for one generation.
uint64_t ff_plan_generation(const FarFieldPlan *p);
void launch_axis_exp(cd *out, int m, double lo, double h, double cr, double ci, hipStream_t s);
// FP64 MFMA contraction C[m][n] = sum_k A[m][k] S[k][n] for a complex table A
// (M x K, row stride K) and S (K x Nc), C (M x Nc); ws: table_gemm_ws_bytes.
size_t table_gemm_ws_bytes(int M, int K);
void table_gemm_f64(const cd *A, int M, int K, const cd *S, int Nc, cd *C, void *ws, hipStream_t s);
// F[m] = pre sum_k P[m][k] T[m][k] (one block per row, fixed summation order).
void launch_rows_dot(const cd *P, const cd *T, int M, int K, cd pre, cd *F, hipStream_t s);
// No-allocation far field: take the scratch array's address on `device` (the
// current device; once per device), then run the FP64 map from it.  Returns 0
// on success, 1 if the problem needs more than the scratch array (*need set),
// 2 if the scratch was not set up on this device, 3 for n_dirs out of range,
// 4 for a HIP error (*herr).
hipError_t ff_scratch_init(int device);
int ff_noalloc_map(const LevelGeom &g, double k0, double gamma, const double eta[3], const cd *q, const cd *u,
                   int M, const double *dirs, cd *F_out, bool out_on_device, int device, hipStream_t s,
                   size_t *need, hipError_t *herr);
}  // namespace ffmg
