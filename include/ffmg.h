/*
 * ffmg.h -- C ABI of the MI355X (gfx950) complex-contour multigrid far-field
 * library.
 *
 * Method: Cools, Reps & Vanroose, "An efficient multigrid calculation of the
 * Far Field map for Helmholtz and Schroedinger equations" (arXiv 1211.4461).
 * The far-field map F(alpha) (Sec. 2.2, eq. FFmap) of a scattering problem is
 * computed in two steps:
 *   1. the scattered wave u is solved on the rotated grid z = e^{i gamma} x
 *      (Sec. 3.1, eq. helmholtz_cc), a damped system that multigrid solves
 *      (Sec. 3.2, eq. csg and eq. csl);
 *   2. F is the quadrature of the source plus scattered wave against
 *      exp(-i k0 alpha.z) over the same contour grid (Sec. 3.1,
 *      eq. I2complex, together with eq. i1).
 *
 * Discrete problem (all entry points share it):
 *   - grid: n[k] intervals per axis on [lo[k], hi[k]], h_k = (hi-lo)/n,
 *     interior nodes x_i = lo + i h_k, i = 1..n[k]-1; N = prod (n[k]-1)
 *     unknowns, stored x fastest (then y, then z), no padding; homogeneous
 *     Dirichlet values outside the interior (Sec. 4, n^d mesh on the box).
 *   - operator: (A u)_j = sum_k c_k (2u_j - u_{j-e_k} - u_{j+e_k}) - kappa_j u_j
 *     with c_k = e^{-2 i gamma}/h_k^2 (Sec. 3.2, eq. csg) and
 *     kappa_j = k0^2 + q_j.
 *   - contrast q_j = k^2(z_j) - k0^2 = k0^2 chi(z_j) (Sec. 2.1); for the
 *     Schroedinger form (Sec. 5) k^2 = 2(E - V), k0 = sqrt(2E), q_j = -2 V(z_j).
 *   - right-hand side for an incoming plane wave along eta:
 *     b_j = q_j exp(i k0 eta.z_j) (Sec. 2.1, eq. helmholtz_in on the contour).
 *   - far field: F(alpha) = e^{i d gamma} prod_k h_k
 *                 sum_j exp(-i k0 alpha.z_j) q_j (u_in(z_j) + u_j).
 *
 * Numbers: every array crossing this ABI is complex128, interleaved (re, im)
 * pairs of IEEE doubles.  FP32 is internal only (FFMG_FP32_IR).
 *
 * Device pointers are HIP device allocations on the current device; the
 * library never frees caller memory.  One handle is used by one host thread
 * and one stream at a time; different handles (each with its own stream and
 * workspace) may be used from different host threads at once, so that the
 * solves of several maps overlap on the GPU.  No C++ exception crosses this ABI: every call
 * returns a status, and ffmg_last_error() gives the text of the last failure
 * on a handle.
 */
#ifndef FFMG_H
#define FFMG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FFMG_OK = 0,
    FFMG_EINVAL = 1,      /* invalid argument; nothing was written            */
    FFMG_ENOMEM = 2,      /* a device allocation failed                       */
    FFMG_EDEVICE = 3,     /* a HIP call failed; the handle must be destroyed  */
    FFMG_ENOCONV = 4,     /* no convergence; u holds the last iterate         */
    FFMG_ERANGE = 5,      /* contour exponentials exceed the working range    */
    FFMG_ENAN = 6         /* NaN or Inf in an input array                     */
} ffmg_status;

typedef enum { FFMG_HELMHOLTZ = 0, FFMG_SCHRODINGER = 1 } ffmg_kind;
typedef enum { FFMG_FP64 = 0, FFMG_FP32_IR = 1 } ffmg_precision;
typedef enum {
    FFMG_SMOOTH_JACOBI = 0,
    FFMG_SMOOTH_LEARNED = 1,
    FFMG_SMOOTH_GMRES = 2,
    FFMG_SMOOTH_RBGS = 3
} ffmg_smoother;
typedef enum { FFMG_FF_FP64 = 0, FFMG_FF_BF16X3 = 1, FFMG_FF_BF16X6 = 2 } ffmg_ff_precision;

/* The scattering problem (Sec. 2.1 Helmholtz; Sec. 5 Schroedinger). */
typedef struct ffmg_problem {
    int dim;              /* 2 or 3                                            */
    int64_t n[3];         /* intervals per axis: power of two, >= coarsest_n   */
    double lo[3], hi[3];  /* box, lo < hi                                      */
    double gamma;         /* contour angle (rad), 0 < gamma < pi/2 (Sec. 3.3)  */
    int kind;             /* ffmg_kind                                         */
    double k0;            /* Helmholtz: outer wavenumber (> 0); Schroedinger: ignored */
    double energy;        /* Schroedinger: total energy E, any finite value;
                             k0 = sqrt(2E) for E > 0 (the plane-wave right-
                             hand sides, far field and batch need E > 0);
                             Helmholtz: ignored                             */
    const void *coef;     /* DEVICE complex128[N], x fastest:
                             Helmholtz: contrast k^2(z_j) - k0^2 = k0^2 chi(z_j);
                             Schroedinger: V(z_j).  Copied at setup; the caller
                             may free it afterwards.                          */
} ffmg_problem;

/* Solver options.  ffmg_default_options() fills V(2,2), omega = 0.8,
 * coarsest n = 8 (7^d unknowns, solved exactly), 200 cycles, FP64. */
typedef struct ffmg_options {
    int nu1, nu2;         /* pre / post smoothing sweeps (>= 0, sum >= 1)      */
    double omega;         /* Jacobi damping, 0 < omega <= 1                    */
    int coarsest_n;       /* intervals per axis on the coarsest grid (>= 4)    */
    int max_cycles;       /* mg_solve cycle limit (>= 1)                       */
    int precision;        /* ffmg_precision                                    */
    int smoother;         /* ffmg_smoother: weighted Jacobi (Sec. 4), the
                             learned network, GMRES(krylov_m) steps or
                             red-black Gauss-Seidel sweeps (Sec. 3.3) on
                             every level above the coarsest                  */
    const float *smoother_weights; /* HOST, learned smoother parameters, or NULL */
    int ff_precision;     /* ffmg_ff_precision                                 */
    int tile_config;      /* 0 = fused kernels (default; 2D: two sweeps per
                             pass, residual + restriction, interpolation +
                             sweeps, LDS tail; 3D: the two sweeps from a zero
                             guess in one pass, interpolation fused into the
                             first post-smoothing sweep), 1 = one operation
                             per launch (reference), 2 = fused without the
                             LDS tail                                          */
    int inner_cycles;     /* FP32_IR: V-cycles per FP64 refinement step
                             (0 = default 3)                                   */
    int nu_coarse;        /* sweeps before and after the coarse correction on
                             the levels below the finest (0 = nu1 / nu2)       */
    int learned_levels;   /* FFMG_SMOOTH_LEARNED: bit l = level l smooths with
                             the network (0 = the finest level only; levels of
                             the LDS tail never do); the others use weighted
                             Jacobi                                            */
    int krylov_m;         /* FFMG_SMOOTH_GMRES: the m of GMRES(m), 1..8
                             (0 = 3); nu1 / nu2 then count GMRES(m) steps    */
    int fmg_cycles;       /* mg_solve starts from the full multigrid guess of
                             mg_fmg with this many V-cycles per coarse level
                             (0 = off: start from the caller's u)            */
    void *stream;         /* hipStream_t; NULL = the null stream               */
} ffmg_options;

typedef struct ffmg_solve_info {
    int cycles;           /* V-cycles (FP64) or refinement steps (FP32_IR)     */
    int vcycles;          /* V-cycles in total (FP32_IR: steps x inner_cycles) */
    int status;           /* ffmg_status of the solve                          */
    double rel_residual;  /* ||b - A u||_2 / ||b||_2 in FP64 at return         */
    double conv_factor;   /* (||r_k|| / ||r_0||)^(1/k)  (Sec. 5.5/5.7 rate)   */
    int fell_back;        /* learned smoother replaced by Jacobi (1) or not    */
    double t_solve_ms;    /* wall time of the solve on the stream              */
} ffmg_solve_info;

typedef struct ffmg_handle ffmg_handle;

void ffmg_default_options(ffmg_options *o);

/* Build the multigrid hierarchy for one problem (Sec. 4; coarse grids
 * n/2^l down to coarsest_n, coefficients injected, coarse operators
 * rediscretised at 2^l h; the coarsest system is inverted exactly, as the
 * 7^3 grid of the F(5) cycle in Sec. 5.7).  Copies coef; allocates all device
 * workspace.  EINVAL on bad sizes or angles; ENAN if coef holds NaN/Inf;
 * ENOMEM / EDEVICE on HIP failures.  *out is NULL on failure. */
ffmg_status mg_setup(const ffmg_problem *p, const ffmg_options *o, ffmg_handle **out);

/* b_j = q_j exp(i k0 eta.z_j): the plane-wave right-hand side of
 * eq. helmholtz_cc, with exp(i k0 eta.z) formed as the product of one factor
 * per axis (the grid is a tensor grid).  eta: HOST double[3] unit vector
 * (first dim entries used, finite).  b: DEVICE complex128[N], written; or
 * NULL.  Either way the call records eta as the handle's plane wave, the
 * right-hand side of mg_solve / mg_solve_begin with b = NULL.  ERANGE if
 * |exp(i k0 eta.z)| would overflow double. */
ffmg_status mg_rhs_plane_wave(ffmg_handle *h, const double eta[3], void *b);

/* b_j = q_j exp(i k0 cos(gamma) eta.x_j): the incoming wave's phase along
 * eta on the real coordinates, without the factor exp(-k0 sin(gamma) eta.x)
 * that the contour adds to it.  It oscillates like the right-hand side of
 * eq. helmholtz_cc and stays bounded where that one leaves the double range
 * (k0 h = 1/2 on the large boxes), so it serves to time and check solves at
 * such wavenumbers; far fields need the true plane wave (mg_rhs_plane_wave).
 * eta: HOST double[3]; b: DEVICE complex128[N], written. */
ffmg_status mg_rhs_phase(ffmg_handle *h, const double eta[3], void *b);

/* One V(nu1, nu2) cycle in place (Sec. 4): omega-Jacobi smoothing,
 * full-weighting restriction of the residual, recursive coarse correction,
 * bilinear/trilinear interpolation, exact coarsest solve.  b: DEVICE
 * complex128[N], read; u: DEVICE complex128[N], updated.  Always FP64. */
ffmg_status mg_vcycle(ffmg_handle *h, const void *b, void *u);

/* Full multigrid start (Sec. 4 with Tables 3 and 4: the nested iteration of
 * V-cycles; Sec. 5.7: the F(k) cycle).  u <- the initial guess for A u = b on
 * the finest grid: b sampled at the nodes of every coarser level
 * (injection: the same problem discretised on the coarse grid, like the
 * coefficients), exact solve on the coarsest level, then on each level
 * between, from the interpolated coarser solution, k V-cycles; u is the
 * interpolated solution of the first coarse level (no cycle runs on the
 * finest level).  Computed in FP64, or, when the handle's precision is
 * FFMG_FP32_IR, in FP32 on b scaled to unit RMS (scaled back in FP64).
 * b: DEVICE complex128[N], read; u: DEVICE complex128[N], overwritten (not
 * read).  0 <= k <= 64 (EINVAL otherwise).  A one-level hierarchy gives the
 * exact solve.  Synchronises. */
ffmg_status mg_fmg(ffmg_handle *h, const void *b, void *u, int k);

/* Solve A u = b by V-cycles (FP64) or by FP32 V-cycles inside FP64
 * iterative refinement (FP32_IR: FP64 outer residual, FP64 update, FP64
 * coarsest solve), from the guess in u (or, with options.fmg_cycles > 0,
 * from the mg_fmg guess, which overwrites u first), until
 * ||b - A u||_2 <= tol ||b||_2 (residual-reduction tolerance, Sec. 4).
 * u: DEVICE complex128[N], in: guess, out: solution.  ENOCONV after max_cycles or when the residual grows
 * on 3 consecutive cycles; u then holds the last iterate and info is filled.
 * b = 0 returns u = 0 after 0 cycles.  info may be NULL.  Synchronises.
 * b: DEVICE complex128[N], read; or NULL for the plane-wave right-hand side
 * of the eta last given to mg_rhs_plane_wave on this handle (EINVAL if
 * none), with the same result, bit for bit, as passing what
 * mg_rhs_plane_wave writes.  The FP32_IR solve with the fused kernels and
 * the Jacobi smoother never stores that b: its FP64 kernels form
 * q exp(i k0 eta.z) where they read it, which saves 16 bytes per point in
 * each FP64 residual pass; other configurations store it once in the handle
 * (N complex128, allocated on first use). */
ffmg_status mg_solve(ffmg_handle *h, const void *b, void *u, double tol, ffmg_solve_info *info);

/* mg_solve in two halves, for callers that keep several solves in flight from
 * one host thread (one handle and stream each).  mg_solve_begin queues, on the
 * handle's stream, everything mg_solve would run up to the end of its first
 * batch of cycles (||b|| is formed and tested on the device), then returns
 * without waiting for the GPU.  mg_solve_end waits for that batch, queues and
 * waits for further batches until the stopping test holds, and returns what
 * mg_solve would: the same u, bit for bit, the same status and info.  Until
 * mg_solve_end returns, b and u must stay allocated and unmodified by the
 * caller, and every other entry point that works on the handle's buffers
 * (mg_solve, mg_vcycle, mg_fmg, the smoothers, mg_residual_norm,
 * mg_rhs_plane_wave, farfield_map, mg_tune_*, mg_solve_batched) returns
 * EINVAL for it.  mg_solve_begin: EINVAL for a null argument, tol outside
 * (0, 1), a solve already pending, or the learned smoother (its fallback is
 * decided on the host between cycles: use mg_solve).  b = NULL: the handle's
 * plane wave, as in mg_solve.  mg_solve_end: EINVAL
 * if no solve is pending; for a non-finite b it returns ENAN with u
 * unspecified.  info may be NULL. */
ffmg_status mg_solve_begin(ffmg_handle *h, const void *b, void *u, double tol);
ffmg_status mg_solve_end(ffmg_handle *h, ffmg_solve_info *info);

/* Far-field map (eq. FFmap moved onto the contour, eq. I2complex):
 *   F_m = e^{i d gamma} prod h_k sum_j exp(-i k0 alpha_m.z_j) q_j (u_in,j + u_j)
 * for n_dirs directions alpha_m (HOST double[n_dirs][dim], unit vectors).
 * The kernel factorises over the axes, so the sum runs as a chain of
 * MFMA contractions; directions sharing their last component share the first
 * contraction (3D azimuth x polar grids).  eta: HOST double[3]; u: DEVICE
 * complex128[N] (NULL = zero scattered wave: the Born term); F: complex128
 * [n_dirs], HOST or DEVICE memory.  ff_precision selects FP64 MFMA or split
 * BF16 MFMA with FP32 accumulation.  With F in HOST memory the call
 * synchronises; with F in DEVICE memory it returns once the work is queued
 * on the handle's stream (later work on that stream sees F; other streams
 * must wait for it).  The first call for a set of directions synchronises
 * while it builds the plan. */
ffmg_status farfield_map(ffmg_handle *h, const double eta[3], const void *u, int n_dirs,
                         const double *dirs, void *F);

/* ---- Ionisation observables of the 2D radial partial-wave Schroedinger
 * model (Sec. 5.1-5.4; eq. partialwave2d solved on the contour grid of a
 * handle of kind FFMG_SCHRODINGER with lo = 0 on both axes, whose Dirichlet
 * boundary is the condition u = 0 at x = 0 and y = 0).  1D arrays along an
 * axis are DEVICE complex128[n[axis] - 1] at the interior contour nodes
 * z_i = lo + i h e^{i gamma}; h~ = h e^{i gamma}. */

/* Source right-hand side of (-1/2 Lap + V - E) u = phi: the library solves
 * the Helmholtz form (-Lap - 2(E - V)) u = 2 phi (Sec. 5, introduction), so
 * b = 2 src for FFMG_SCHRODINGER and b = src for FFMG_HELMHOLTZ.  src, b:
 * DEVICE complex128[N] (may alias).  Queued on the handle's stream. */
ffmg_status mg_rhs_source(ffmg_handle *h, const void *src, void *b);

/* eq. boundstate on axis `axis`: the eigenpair of the rotated 1D Hamiltonian
 * -1/2 e^{-2i gamma} D2/h^2 + diag(v) (Sec. 5.2) nearest to the real `shift`,
 * by inverse iteration and Rayleigh-quotient shifts.  v: the one-body
 * potential at the axis nodes.  Outputs lambda (HOST double[2], re/im) and
 * phi (DEVICE complex128[m]) normalised by sum phi^2 h~ = 1 (the contour
 * continuation of int phi^2 dx = 1), sign with Re phi_1 > 0.  ENOCONV when
 * the iteration does not converge in 60 steps.  Synchronises. */
ffmg_status ion_bound_state(ffmg_handle *h, int axis, const void *v, double shift, double lambda[2], void *phi);

/* Channel wavenumbers at total energy E (HOST arrays): *kn = sqrt(2(E - Re
 * lambda)) for the single-ionisation channel of the bound state lambda (0 if
 * E <= Re lambda: closed); for E > 0 the M midpoint nodes of the
 * double-ionisation integral over eps in [0, E] (eq. double-ionization):
 * k1 = sqrt(2 eps_i), k2 = sqrt(2(E - eps_i)), eps_i = (i + 1/2) E / M, and
 * weights w = E/M (all zero for E <= 0).  Host arithmetic, no handle. */
ffmg_status ion_wavenumbers(double energy, const double lambda[2], int M, double *kn, double *k1, double *k2,
                            double *w);

/* eq. testfunction on axis `axis` for the M wavenumbers k (HOST double[M],
 * > 0): the regular solution of (-1/2 d^2/dz^2 + v - k^2/2) phi = 0 with
 * phi = 0 at the axis' lower end, by the recurrence of the rotated
 * three-point stencil, normalised to free-wave amplitude 1/sqrt(k): at the
 * first node r past the last one with |v| > 1e-13, A^2 = (p_r^2 + p_{r+1}^2
 * - 2c p_r p_{r+1})/(1 - c^2), c = 1 - h~^2 k^2/2, is the squared amplitude
 * of the free recurrence, and phi = p/(A sqrt k) with Re A > 0.
 * out: DEVICE complex128[M][m] (row per wavenumber).  EINVAL if v does not
 * die out before the last two nodes.  Synchronises. */
ffmg_status ion_test_functions(ffmg_handle *h, int axis, const void *v, int M, const double *k, void *out);

/* eq. single-ionization / eq. double-ionization on the contour (2D):
 *   amp_m = h~x h~y sum_{y,x} tx[m][x] ty[m][y] (src - v12 u)[y][x]
 * for M pairs of DEVICE tables tx (complex128[M][nx-1]) and ty
 * (complex128[M][ny-1]), and the optical-theorem product
 *   opt = h~x h~y sum src u
 * (src: the source phi, v12: the two-body potential, u: the solution; DEVICE
 * complex128[N]).  The y contraction runs on the FP64 MFMA GEMM of the far
 * field.  amp: HOST complex128[M]; opt: HOST double[2].  Synchronises. */
ffmg_status ion_amplitudes(ffmg_handle *h, const void *src, const void *v12, const void *u, int M, const void *tx,
                           const void *ty, double *amp, double opt[2]);

/* Cross sections (Fig. single_and_double) from the amplitudes, as half the
 * outgoing probability flux of each kind of channel (the scale of the
 * printed points): sigma[0] = 4 |s0|^2 (single; 0 if !open_single),
 * sigma[1] = (4/pi) sum_i w_i |f_i|^2 (double), sigma[2] = Im opt (total,
 * the optical theorem).  s0: HOST double[2]; f: HOST complex128[M]; w: the
 * weights of ion_wavenumbers.  Host arithmetic, no handle. */
ffmg_status ion_cross_sections(int open_single, const double s0[2], int M, const double *f, const double *w,
                               const double opt[2], double sigma[3]);

/* Far-field map that allocates nothing, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  It computes what farfield_map computes
 * on a handle with ff_precision FFMG_FF_FP64 (the FP64 MFMA contraction,
 * whatever the handle's ff_precision), bit for bit, with the same arguments:
 * eta HOST double[3]; u DEVICE complex128[N] or NULL (Born term); dirs HOST
 * double[n_dirs][dim] unit vectors; F complex128[n_dirs] in HOST memory (the
 * call synchronises) or DEVICE memory (returns once queued on the handle's
 * stream).  Every work buffer (axis factors, direction table, packed factors,
 * integrand, stage results) lives in one static device array of
 * FFMG_NOALLOC_SCRATCH_BYTES per GPU, held from the library's load until the
 * process ends; it calls no hipMalloc/hipFree and builds no plan.  The array
 * is shared by every call on that GPU: calls that overlap on one GPU (other
 * streams or host threads) race and must be serialised by the caller; the
 * next call on the handle's stream may start as soon as this one's work is
 * queued.  Limits (EINVAL, nothing written): n_dirs <= FFMG_NOALLOC_MAX_DIRS,
 * and the buffers must fit the array, roughly
 * 16 (N + 3 n_dirs (n_x - 1) + NG (n_x - 1)(n_y - 1)) bytes with NG the
 * number of distinct last components in 3D (e.g. a 1023^2 grid with 360
 * directions, or a 63^3 grid with 128 x 64 directions); the message states
 * the bytes needed.  Other errors as farfield_map. */
#define FFMG_NOALLOC_SCRATCH_BYTES (64u << 20)
#define FFMG_NOALLOC_MAX_DIRS 8192
ffmg_status farfield_map_noalloc(ffmg_handle *h, const double eta[3], const void *u, int n_dirs,
                                 const double *dirs, void *F);

/* Batched solve: count instances, instance i being the plane wave of
 * direction etas[3i..3i+2] (the right-hand side of Sec. 2.1, built on the
 * device) scattered by the operator of handle hs[i]; handles may repeat
 * (several directions of one energy and grid) and may differ in grid size
 * (e.g. the Schroedinger maps of Sec. 5 at several energies on 255^2 ..
 * 1023^2 grids).  Every instance is solved to ||b - A u||_2 <= tol ||b||_2
 * with the FP32-in-FP64 refinement of mg_solve, from u = 0 or, with
 * options.fmg_cycles = k > 0, from the full multigrid start F(k) (Sec. 4;
 * the batch runs every instance's start together, level by level),
 * and its result u[i] (DEVICE complex128[N_i], output) and info (infos[i],
 * may be NULL) equal those of mg_solve on that handle bit for bit.  All
 * instances advance together: one launch per kernel for the whole batch, the
 * refinement step captured once in a HIP graph and replayed until every
 * instance has met its stopping test on the device.  Requirements (EINVAL
 * otherwise): 2D handles set up with precision FFMG_FP32_IR and tile_config
 * 0, all with the same nu1 >= 1, nu2 >= 1, inner cycles and fmg_cycles and
 * the same coarse-level shapes (grids n = 2^k on one coarsest_n).  The workspace and
 * graph are owned by hs[0] (freed by mg_destroy(hs[0])) and reused while the
 * same list of handles is passed; the call is ordered after work on hs[0]'s
 * stream and synchronises.  Returns ENOCONV if an instance did not converge
 * (infos tells which), ENAN if a right-hand side is not finite. */
ffmg_status mg_solve_batched(ffmg_handle *const *hs, int count, const double *etas, void *const *u, double tol,
                             ffmg_solve_info *infos);

/* Far-field maps of count instances (hs[i], etas[3i..], u[i]; u may be NULL:
 * Born terms) at the same n_dirs directions, into F (complex128
 * [count][n_dirs], HOST or DEVICE) without synchronising between instances;
 * each row equals farfield_map on that instance.  2D split-precision handles
 * run each stage of all instances in one launch (per grid size for the
 * contraction); their workspace is owned by hs[0] and rebuilt whenever the
 * handle list, a handle's direction plan (other directions or precision) or
 * its tile variant changed since the last call.  Synchronises. */
ffmg_status farfield_map_batched(ffmg_handle *const *hs, int count, const double *etas, void *const *u, int n_dirs,
                                 const double *dirs, void *F);

/* ---- Learned smoother (a replacement of the weighted-Jacobi sweeps of
 * the finest level; the paper smooths with weighted Jacobi, Sec. 4).  One
 * smoothing step is u += s h^2 N(r / s, kappa h^2), r = b - A u, s = RMS(r),
 * where N is a three-layer 3x3 complex convolutional network with 2 -> 16 ->
 * 16 -> 1 complex channels, no activation function and no biases, stored in
 * BF16 and accumulated in FP32.  Layer 1 is a gate: with
 * a = W1[:, :, 0] * r~ and m = W1[:, :, 1] * kappa~ (3x3 convolutions of
 * the two inputs), its output is x1 = a (1 + m); then x2 = W2 * x1 and
 * N = W3 * x2.  N is complex-linear in r~, so the step is a linear iteration
 * whose stencil (radius 3) adapts to the local coefficient, and weighted
 * Jacobi is one point of the weight space.  Weights: FFMG_NET_WEIGHTS complex values as
 * interleaved (re, im) floats: W1 [9][16][2], W2 [9][16][16], W3 [9][1][16],
 * indexed (tap, output channel, input channel), tap 3 (dy + 1) + (dx + 1)
 * reading the point (y + dy, x + dx).
 *
 * Training patches: count patches of 32 x 32 points, DEVICE complex64
 * [count][32][32] each: the scaled residual r / s, kappa h^2 and the scaled
 * error e / (s h^2).  The loss of a patch is the mean over its points at
 * least `border` from the patch edge of |L5 (e~ - N)|^2 (L5 the 5-point
 * Laplacian stencil), plus the growth penalty
 * max(0, ||e~ - N||^2 / ||e~||^2 - 1) over the same points (the error left
 * after the step must not be larger than the error before it); the
 * minibatch loss is the mean over patches.
 * ml_loss_grad returns the loss and its gradient (host, 2 * FFMG_NET_WEIGHTS
 * floats, may be NULL) at the current weights; ml_train_step also applies
 * one Adam step (beta1 0.9, beta2 0.999, eps 1e-8) to the FP32 master
 * weights and, if loss is not NULL, returns the minibatch loss (before the
 * step; this synchronises).  The network object owns its device memory and
 * works on the stream given at creation. */
#define FFMG_NET_WEIGHTS 2736
typedef struct ffmg_net ffmg_net;
ffmg_status ml_net_create(const float *w, void *stream, ffmg_net **out);
ffmg_status ml_net_set_weights(ffmg_net *net, const float *w);   /* also resets the Adam state */
ffmg_status ml_net_get_weights(ffmg_net *net, float *w);
ffmg_status ml_loss_grad(ffmg_net *net, const void *rt, const void *kt, const void *et, int count, int border,
                         float *loss, float *grad);
ffmg_status ml_train_step(ffmg_net *net, const void *rt, const void *kt, const void *et, int count, int border,
                          float lr, float *loss);
const char *ml_net_last_error(const ffmg_net *net);
void ml_net_destroy(ffmg_net *net);

/* Au = A u (the operator of eq. csg), DEVICE complex128[N] each. */
ffmg_status mg_apply(ffmg_handle *h, const void *u, void *Au);

/* r = b - A u in FP64, DEVICE complex128[N] each (r must not alias b or u). */
ffmg_status mg_residual(ffmg_handle *h, const void *b, const void *u, void *r);

/* One smoothing step on the finest level, FP64, out of place: an
 * omega-Jacobi sweep u_out = u + omega D^{-1} (b - A u) (smoothers Jacobi and
 * learned), a red-black Gauss-Seidel sweep (FFMG_SMOOTH_RBGS) or a GMRES(m)
 * step (FFMG_SMOOTH_GMRES) from u into u_out.  u, u_out must not alias. */
ffmg_status mg_smooth(ffmg_handle *h, const void *b, const void *u, void *u_out);

/* One learned smoothing step on the finest level, in place on u (DEVICE
 * complex128[N]): u += s h^2 N(r / s, kappa h^2) with r = b - A u and
 * s = RMS(r) (N is linear in r, so this is h^2 N(r, kappa h^2)).  The handle must use FFMG_SMOOTH_LEARNED on the finest level.
 * With that smoother the levels selected by learned_levels take nu1 / nu2
 * (nu_coarse) such steps instead of Jacobi sweeps, and mg_solve
 * compares each batch of cycles with the convergence factor of the Jacobi
 * V-cycle on the same operator (measured at setup, mg_jacobi_factor): a
 * learned cycle that reduces the residual less makes the solve continue
 * with Jacobi (info.fell_back = 1). */
ffmg_status mg_learned_smooth(ffmg_handle *h, const void *b, void *u);
double mg_jacobi_factor(const ffmg_handle *h);

/* One GMRES(m) smoothing step on the finest level, in place, FP64 (Sec. 3.3:
 * the Krylov smoother that keeps the V-cycle stable near 10 degrees): with
 * r0 = b - A u, u becomes the u + z, z in span{r0, A r0, ..., A^{m-1} r0}, of
 * least residual norm (one restart cycle of GMRES, m = options.krylov_m).
 * b: DEVICE complex128[N], read; u: DEVICE complex128[N], updated.  EINVAL
 * unless the handle was set up with smoother FFMG_SMOOTH_GMRES and has more
 * than one level.  Queued on the handle's stream. */
ffmg_status mg_gmres_smooth(ffmg_handle *h, const void *b, void *u);

/* ||b - A u||_2 (FP64 accumulation) into *rnorm (host). */
ffmg_status mg_residual_norm(ffmg_handle *h, const void *b, const void *u, double *rnorm);

/* Kernel timing (instrumentation for benchmarks).  Bit k of mask enables a
 * pair of HIP events on the handle's stream around every launch of kernel k:
 * 0 finest-level pre-smoothing (the fused two-sweep kernel, or each sweep),
 * 1 far-field map (integrand, contraction, final sum), 2 finest-level
 * interpolation + post-smoothing, 3 FP64 update + residual of the
 * mixed-precision refinement, 4 the far-field GEMM stages alone, 5 the
 * learned smoother's network on the finest level, 6 the finest-level
 * residual + restriction (3D), 7 and 8 the finest-level pass of two
 * pre-smoothing sweeps, the residual and its full weighting (3D,
 * FFMG_TUNE_SWEEP3D variant 4; 7 from a guess, 8 from a zero guess, whose
 * launches are then not counted under 0 and 6).  mask = 0 disables.  mg_profile_read
 * synchronises, returns the summed duration (ms) and launch count of one
 * kernel, and clears its record.  mg_profile_durations does the same but
 * writes each launch's duration (ms, in launch order) into ms[0 .. cap - 1]
 * (HOST) and the number of launches into *count (which may exceed cap). */
ffmg_status mg_profile_enable(ffmg_handle *h, int mask);
ffmg_status mg_profile_read(ffmg_handle *h, int kernel, double *total_ms, int64_t *count);
ffmg_status mg_profile_durations(ffmg_handle *h, int kernel, double *ms, int64_t cap, int64_t *count);

/* Autotuning of kernel tile shapes.  A tunable is a family of kernel
 * variants that compute the same result (bit for bit) with different tile
 * shapes; the best one depends on the device, the grid and the number of
 * directions.  FFMG_TUNE_FF_GEMM: the split-BF16 far-field GEMM (row tiles x
 * column tiles per wave, or a block tile staged in LDS and shared by its four
 * waves); with ff_precision FP64 it has one variant.
 * FFMG_TUNE_TAIL: the largest coarse level (4096, 1024 or 256 interior
 * points for variants 0, 1, 2) run inside the one-workgroup LDS tail of the
 * fused 2D cycle; the levels above it run as grid-wide launches.  It has one
 * variant for handles without the LDS tail (3D, tile_config != 0) and for the
 * learned smoother.  FFMG_TUNE_SMOOTH: the tile height of the fused 2D
 * smoothing kernel on the finest level (8, 16 or 4 rows of 64 points for
 * variants 0, 1, 2; the batched path has its own, FFMG_TUNE_BATCH); FFMG_TUNE_SMOOTH_COARSE: the
 * same on the coarser levels, where the one-pass pre-smoothing follows it
 * (16 rows with the 16-row variant, else 8); one variant each for 3D and
 * tile_config 1.
 * FFMG_TUNE_PRE: the pre-smoothing of a fused 2D level with nu1 = 2 as one
 * pass of two sweeps, residual and full weighting (variant 0: 16-row tiles on
 * the finest level for FP32 cycles, 8-row for FP64; 2: the other height) or
 * as the two-sweep launch followed by the residual + restriction launch (1);
 * one variant for 3D and tile_config 1.
 * FFMG_TUNE_SWEEP3D: the weighted-Jacobi sweeps of a fused 3D level as one
 * z-marching pass per pair of sweeps (the first sweep's planes held in LDS,
 * the interpolation of the coarse correction formed inside the first pass)
 * with 64-point-wide tiles of 8 rows in FP32 and 4 in FP64 (variant 0) or 16
 * and 8 (variant 2), 32-point-wide tiles of 16 and 8 rows for the pass that
 * interpolates the coarse correction and the variant-0 tiles for the others
 * (variant 3), variant 3 with the two FP32 pre-smoothing sweeps, the residual
 * and its full weighting in one pass (variant 4, the default of FFMG_FP32_IR
 * handles; FP64 levels as variant 3), or one pass per sweep (variant 1); one
 * variant for 2D and tile_config 1.
 * FFMG_TUNE_BATCH (set on the first handle of a batch, 2D FFMG_FP32_IR fused
 * handles): the tile heights of mg_solve_batched's smoothing and one-pass
 * pre-smoothing launches, (8, 16) rows (variant 0), (4, 16) (1), (16, 16) (2)
 * or (8, 8) (3); the same bits with every variant; a batch built with another
 * variant is rebuilt.  Tuned by timing mg_solve_batched (the autotuner).
 * mg_tune_variants returns the number of variants (0 for an unknown
 * tunable); mg_tune_get / mg_tune_set read and select one (a cached choice).
 * mg_tune_farfield builds the integrand of (eta, u) for the n_dirs
 * directions, times every variant of the contraction `reps` times with HIP
 * events on the handle's stream, selects the fastest and returns its index in
 * *best and the mean time of variant v in times_ms[v] (v < n_times; times_ms
 * may be NULL).  Synchronises.
 * mg_tune_solve times `reps` solves of b from u = 0 to tol per variant of
 * `tunable` (FFMG_TUNE_TAIL, FFMG_TUNE_SMOOTH, FFMG_TUNE_PRE,
 * FFMG_TUNE_SMOOTH_COARSE or FFMG_TUNE_SWEEP3D; after one untimed solve),
 * selects the fastest and reports like mg_tune_farfield; u is the caller's
 * workspace and holds the last solution on return.  Synchronises. */
typedef enum {
    FFMG_TUNE_FF_GEMM = 0,
    FFMG_TUNE_TAIL = 1,
    FFMG_TUNE_SMOOTH = 2,
    FFMG_TUNE_PRE = 3,
    FFMG_TUNE_SMOOTH_COARSE = 4,
    FFMG_TUNE_SWEEP3D = 5,
    FFMG_TUNE_BATCH = 6
} ffmg_tunable;
int mg_tune_variants(const ffmg_handle *h, int tunable);
ffmg_status mg_tune_get(const ffmg_handle *h, int tunable, int *variant);
ffmg_status mg_tune_set(ffmg_handle *h, int tunable, int variant);
ffmg_status mg_tune_farfield(ffmg_handle *h, const double eta[3], const void *u, int n_dirs, const double *dirs,
                             int reps, double *times_ms, int n_times, int *best);
ffmg_status mg_tune_solve(ffmg_handle *h, int tunable, const void *b, void *u, double tol, int reps, double *times_ms,
                          int n_times, int *best);

/* Number of levels and the interior sizes of level l (n[k] - 1 per axis). */
int mg_num_levels(const ffmg_handle *h);
ffmg_status mg_level_shape(const ffmg_handle *h, int level, int64_t m[3]);

void mg_destroy(ffmg_handle *h);
const char *ffmg_strerror(ffmg_status s);
const char *ffmg_last_error(const ffmg_handle *h);

#ifdef __cplusplus
}
#endif
#endif /* FFMG_H */
