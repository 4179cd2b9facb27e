// ffmg_handle.hpp -- the handle behind the C ABI and the driver entry points
// shared by the library's translation units (single solve, batched solve,
// learned smoother).
#pragma once

#include <string>
#include <utility>
#include <vector>

#include "../../include/ffmg.h"
#include "ffmg_internal.hpp"

namespace ffmg {

struct Level {
    LevelGeom g;
    Stencil<double> P64;
    Stencil<float> P32;
    cd *q = nullptr;                 // contrast on this level
    cd *u = nullptr, *b = nullptr;   // coarse correction / rhs (levels >= 1)
    cd *r = nullptr, *t = nullptr;   // residual / scratch, ping-pong buffer
    cf *q32 = nullptr;               // FP32 copies for the refinement inner cycle
    cf *u32 = nullptr, *b32 = nullptr, *r32 = nullptr, *t32 = nullptr;
    cd *gz = nullptr;                // GMRES(m) smoother: m + 1 basis vectors (FP64)
    cf *gz32 = nullptr;              // and their FP32 copies for the inner cycle
};

// tile_config values
enum { TILE_FUSED = 0, TILE_REFERENCE = 1, TILE_FUSED_NO_TAIL = 2 };

// FP32 V-cycles per FP64 refinement step when options.inner_cycles is 0:
// three cycles reduce the scaled residual by about 60 (V(2,2), Jacobi), far
// above the FP32 floor, and measured fastest to 1e-10 on 2047^2 (2: 9 steps,
// 3: 6 steps, 4 and 5: 5 and 4 steps of more cycles in total).
constexpr int DEFAULT_INNER_CYCLES = 3;

struct Batch;   // batched-solve workspace (ffmg_batch.hip)

}  // namespace ffmg

namespace ffmg {
// A solve started by mg_solve_begin and not yet finished by mg_solve_end.
struct PendingSolve {
    bool active = false;
    const cd *b = nullptr;
    cd *u = nullptr;
    cd *ua = nullptr, *ub = nullptr; // current iterate / the other buffer of the FP32 2D step
    int queued = 0;                  // steps queued so far
    bool flip = false;               // the start was written into l0.t instead of u
    const ffmg::cf *start_ec = nullptr; // the 3D start s P e_c not stored: its first step forms it from e_c
    bool start_unstored = false;     // that start is stored at the end if no step completed
    hipEvent_t e0 = nullptr, e1 = nullptr;
};
}  // namespace ffmg

struct ffmg_handle {
    uint64_t serial = 0;             // unique per handle of this process
    ffmg_problem prob{};
    ffmg_options opt{};
    double k0 = 0.0, k02 = 0.0;
    std::vector<ffmg::Level> L;
    ffmg::cd *aug = nullptr;         // [A_c | A_c^{-1}] of the coarsest level
    int nc = 0;
    int *d_info = nullptr;
    double *d_parts = nullptr;       // per-block partial sums
    int nparts = 0;
    double *d_scalar = nullptr;
    double *h_scalar = nullptr;      // pinned
    ffmg::SolveCtl *d_ctl = nullptr; // device solve control
    ffmg::SolveCtl *h_ctl = nullptr; // pinned copy
    int last_cycles = 0;             // cycles of the previous solve (batch sizing)
    ffmg::PendingSolve pend;         // mg_solve_begin .. mg_solve_end
    int krylov_m = 0;                // GMRES(m) smoother: m
    double *d_gm = nullptr;          // its per-step scalars (GM_S doubles)
    double *d_gm_parts = nullptr;    // and partial sums (GM_PARTS doubles)
    hipStream_t stream = nullptr;
    int device = 0;                  // HIP device current at setup (owns every buffer)
    // coarse end of the 2D cycle run by one workgroup in LDS (levels >= tail_l)
    int tail_l = -1;
    size_t tail_lds[2] = {0, 0};     // [FP64, FP32]
    int tail_variant = 0;            // index into TAIL_POINTS (autotuned)
    int smooth_variant = 0;          // index into SMOOTH_TH, finest level (autotuned)
    int smooth_coarse_variant = 0;   // index into SMOOTH_TH, coarser levels (autotuned)
    int pre_variant = 0;             // FFMG_TUNE_PRE: 0 fused pre-smoothing + residual + restriction (autotuned)
    int batch_variant = 0;           // FFMG_TUNE_BATCH: tile heights of batched solves led by this handle
    int sweep3d_variant = 0;         // FFMG_TUNE_SWEEP3D: 0/2/3 two sweeps per 3D pass (tile shapes), 1 one, 4 the
                                     // FP32 pre-smoothing pair fused with residual + restriction (4 for 3D FP32_IR
                                     // handles at setup; autotuned)
    ffmg::TailParams<double> tail64{};
    ffmg::TailParams<float> tail32{};
    ffmg::FarFieldPlan *ff = nullptr;
    int ff_variant = -1;             // split-GEMM tile variant (-1: default; autotuned)
    ffmg::cd *d_E = nullptr;         // plane-wave axis factors (far field)
    // the plane wave of the last mg_rhs_plane_wave: its per-axis factors on the
    // finest level (the right-hand side q u_in of mg_solve(h, NULL, ...)), and
    // that right-hand side stored for the paths that read b (on first use)
    ffmg::cd *pw_f = nullptr;
    bool pw_set = false;
    ffmg::cd *pw_b = nullptr;
    ffmg::cf *fmg_e1 = nullptr;      // the FP32 start's first-level solution, kept for the first 3D step
    ffmg::cd *d_F = nullptr;         // far-field staging
    int d_F_cap = 0;
    // ionisation observables: workspace slots grown on demand, freed at destroy
    void *ion_buf[6] = {};
    size_t ion_cap[6] = {};
    // learned smoother on the finest level (smoother FFMG_SMOOTH_LEARNED)
    unsigned short *d_wfrag = nullptr;   // MFMA weight fragments (BF16)
    std::vector<unsigned *> d_kh2;       // kappa h^2 per level, BF16 complex (learned levels)
    double rho_jacobi = 0.0;             // Jacobi V-cycle convergence factor (the reference)
    bool learned_on = false;             // learned smoother in use
    ffmg::Batch *batch = nullptr;    // batched-solve workspace for a list of handles starting with this one
    ffmg::FFBatch *ffbatch = nullptr; // batched far-field workspace, likewise
    std::vector<void *> allocs;
    std::string err;
    // optional event timing of selected kernels (benchmark instrumentation)
    int profile_mask = 0;            // bit k: time kernel k (ffmg::ProfKernel)
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[ffmg::PROF_N];
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_free;
};

namespace ffmg {

ffmg_status fail(ffmg_handle *h, ffmg_status s, const char *fmt, ...);
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

// One V(nu1, nu2) cycle on level l; every launch carries `stop`.
template <typename T>
void vcycle(ffmg_handle *h, int l, const cx<T> *b, cx<T> *u, bool zero_guess, const int *stop);

int prof_begin(ffmg_handle *h, int k);
void prof_end(ffmg_handle *h, int k, int idx);
// log of the largest magnitude of exp(+-i k0 e^{i gamma} a.x) over the box
double exponent_budget(const ffmg_handle *h);
// far-field map into device memory F on the handle's stream, no synchronisation
ffmg_status farfield_enqueue(ffmg_handle *h, const double eta[3], const void *u, int n_dirs, const double *dirs,
                             cd *F);
// the checks and the plan of farfield_enqueue without the map
ffmg_status farfield_prepare(ffmg_handle *h, const double eta[3], int n_dirs, const double *dirs);
void batch_destroy(Batch *b);
// one learned smoothing step on level l, in place on u
void learned_step(ffmg_handle *h, int l, const cd *b, cd *u, const int *stop);
bool learned_level(const ffmg_handle *h, int l);

}  // namespace ffmg

#define HIPCHK(h, x)                                                                                                \
    do {                                                                                                            \
        hipError_t e_ = (x);                                                                                        \
        if (e_ != hipSuccess)                                                                                       \
            return ffmg::fail((h), e_ == hipErrorOutOfMemory ? FFMG_ENOMEM : FFMG_EDEVICE, "%s: %s (%s:%d)", #x,    \
                              hipGetErrorString(e_), __FILE__, __LINE__);                                           \
    } while (0)

// Entry points that touch a handle's buffers refuse to run while a solve
// begun by mg_solve_begin is still pending on it.
#define NOT_PENDING(h)                                                                                              \
    do {                                                                                                            \
        if ((h) && (h)->pend.active)                                                                                \
            return ffmg::fail((h), FFMG_EINVAL,                                                                     \
                              "a solve begun by mg_solve_begin is pending on this handle: call mg_solve_end first"); \
    } while (0)

#define TRY(x)                                                                                                      \
    do {                                                                                                            \
        ffmg_status s_ = (x);                                                                                       \
        if (s_ != FFMG_OK) return s_;                                                                               \
    } while (0)
