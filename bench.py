#!/usr/bin/env python3
"""Far-field maps per second on one MI355X.

One step = one far-field map of the 3D Gaussian workload (512 intervals per
axis on [-6,6]^3, 133.4 M unknowns, chi = 0.5 exp(-z.z/2) continued onto the
contour, k0 = 1, contour angle 30 deg, eta = +x): plane-wave right-hand side,
multigrid solve to ||r|| <= 1e-6 ||b|| (the paper's residual-reduction
tolerance; the line reports the map's measured error against the FP64 map
converged to 1e-10) and the far field on a 128 (azimuth) x 64 (polar)
direction grid, with every input already in HBM.  `value` is the
mixed-precision path (FP32 V(2,2) cycles inside FP64 refinement, far field as
a split-BF16 MFMA contraction with FP32 accumulation); the plain FP64 path
(FP64 V-cycles, FP64 MFMA far field) is timed beside it on the same maps at
the same tolerance (equal accuracy), and both are timed again at 1e-10.
Both start from the full multigrid guess (FMG_3D V-cycles per coarse level)
and keep `--lanes` solves in flight from this one host thread: consecutive
maps cycle through that many handles, each on its own stream, and each map's
solve is begun (mg_solve_begin) before the map begun lanes - 1 steps earlier
is finished (mg_solve_end) and its far field queued.

Also reported:
  * the roofline of the dominant kernel: the finest-level kernels the library
    brackets with HIP events (interpolation + post-smoothing, residual +
    restriction, refinement step) are timed launch by launch in a
    one-solve-in-flight pass of the same maps, early-exit launches of an
    already converged solve dropped; the one with the largest total time is
    the dominant kernel (the committed rocprofv3 kernel trace of the same
    command ranks every kernel of a map, coarse levels included);
  * the same kernel rates for the plain FP64 path (its own one-solve pass);
  * the solve-only stress points at k0 h = 1/2 (2048^2 and 512^3) with the
    bounded phase right-hand side;
  * the 2D 2048^2 bumps workload (the former headline) with its pipelined
    mixed and plain rates and its four directions as one batched solve, the
    GMRES(3) smoother, the batched Schroedinger workload (full multigrid
    start), the learned smoother and the ionisation cross-section sweep of
    the partial-wave model;
  * the FP64 CPU oracle on the host cores, on a bounded sample of the
    headline workload (run in a child process).
"""
from __future__ import annotations

import argparse
import collections
import hashlib
import json
import math
import os
import subprocess
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# V-cycles per coarse level of the full multigrid start (the F(k) cycle): 2 for
# the 2D workloads, 3 for the 512^3 headline (both paths), where it lets two
# refinement steps of three FP32 V-cycles reach MAP_TOL (F(2): two steps of
# four; measured per solve 28.8 vs 34.8 ms, residual 7.5e-7 vs 1.0e-7, maps
# 4.8e-8 vs 6.5e-9 from the FP64 map)
FMG_K = 2
FMG_3D = 3
# the 2048^2 bumps maps: F(1) and one refinement step of four FP32 V-cycles
# (measured per solve 1.03 ms, residual 3.8e-7, against 1.34 ms for F(2) and
# two steps of two); the plain path keeps F(2) (with four solves in flight
# its maps ran 818/s from F(2) against 768/s from F(1))
FMG_2D = 1
INNER_2D = 4
# Residual-reduction tolerance of the headline maps (the paper's own Sec. 4
# tolerance): the metric asks for maps within 1e-6 of the FP64 map, which
# this reaches with two orders of magnitude to spare (the line reports the
# measured map error against the FP64 map converged to FP64_TOL)
MAP_TOL = 1e-6
FP64_TOL = 1e-10
# FP32 V-cycles per FP64 refinement step of the 3D mixed path (with F(3): two
# steps of three reach MAP_TOL; two of two take a third step)
INNER_3D = 3
# the literal Schroedinger wells (GMRES smoother): maps within 1e-6 need a
# smaller residual there (measured: 1e-6 leaves map errors up to 3e-6)
LITERAL_TOL = 1e-8
# the batched maps: F(2) and three FP32 V-cycles per refinement step
# (measured solve-only 7.7 ms per batch at 1e-6 and 14.0 at 1e-10, against
# 8.8 / 15.8 for F(1) and two)
BATCH_FMG = 2
BATCH_INNER = 3
CSRC = os.path.join(ROOT, "paper_1211_4461_amd", "csrc")
# committed rocprofv3 FETCH_SIZE / WRITE_SIZE records, keyed by kernel source
TRAFFIC = {3: (os.path.join(ROOT, "profiles", "traffic_gauss3d_512.json"), os.path.join(CSRC, "ffmg_stencil.hip")),
           2: (os.path.join(ROOT, "profiles", "traffic_bumps2d_2048.json"), os.path.join(CSRC, "ffmg_fused2d.hip"))}
# the 2D record predates the per-dimension keys
TRAFFIC_FILE, STENCIL_SRC = TRAFFIC[2]

# PROF_* ids of the kernels the library brackets (mg_profile_*)
KERNELS = {"pre": 0, "ff": 1, "post": 2, "refine": 3, "ffgemm": 4, "net": 5, "rr": 6, "srr": 7, "srr0": 8}
# Algorithmic bytes per finest-level point of the bracketed kernels (complex
# values: FP32 8 B, FP64 16 B; the coarse level has 1/8 (3D) or 1/4 (2D) of
# the points):
#   post    interpolation + two Jacobi sweeps: read u, b, q, e_c; write u
#   rr      residual + full weighting: read u, b, q; write b_c
#   refine  FP64 update + residual: read u, b, q (16 each), d (8); write u (16), r (8)
# "pre" brackets two passes (two sweeps from a zero guess, 3e; two sweeps
# from a guess, 4e) and is reported, not ranked.
# (the refinement pass forms the plane-wave right-hand side from q instead of
# reading it: read u, q (16 B each), d (8); write u, r (16 + 8))
BPP = {3: {"mixed": {"post": 33.0, "rr": 25.0, "refine": 64.0, "srr": 33.0, "srr0": 25.0},
           "plain": {"post": 66.0, "rr": 50.0}},
       2: {"mixed": {"post": 34.0, "refine": 64.0}, "plain": {"post": 68.0}}}
KERNEL_NAMES = {
    3: {"post": "k_sweep2_3d<%s, SRC_PROL> (finest level: interpolation of the coarse correction + two Jacobi sweeps "
                "in one z-marching pass)",
        "rr": "k_resid_restrict3d<%s> (finest level: residual + full weighting in one pass)",
        "srr": "k_sweep2rr_3d<%s, from a guess> (finest level: two Jacobi sweeps + residual + full weighting in one "
               "z-marching pass)",
        "srr0": "k_sweep2rr_3d<%s, from zero> (finest level: two Jacobi sweeps from a zero guess + residual + full "
                "weighting in one z-marching pass)",
        "refine": "k_refine3d<true> (FP64 update + residual of the refinement step, one pass; the plane-wave "
                  "right-hand side formed from q)",
        "pre": "k_sweep2_3d<%s, SRC_ZERO2 / SRC_MEM> (finest level: two Jacobi sweeps per pass)"},
    2: {"post": "k_smooth2d<%s, 2, false, true, 1, TH> (finest level: interpolation + two fused Jacobi sweeps)",
        "refine": "k_refine2d (FP64 update + residual; the plane-wave right-hand side formed from q)",
        "pre": "k_smooth_rr2d<%s, *, 1, *> (finest level: two sweeps + residual + full weighting)"},
}
# Useful flops of one learned-smoother application per point: 2736 complex
# multiply-adds (one per complex weight), 8 real flops each.
NET_FLOP_PER_POINT = 8 * 2736


def src_hash(path=STENCIL_SRC):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(kernel, key, dim=2):
    """HBM bytes per launch of `kernel` (variant `key`) from committed
    rocprofv3 --pmc counters, or None if absent or taken on a different
    kernel source."""
    path, src = TRAFFIC[dim]
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("src_sha") != src_hash(src):
        return None
    if "per_kernel" in t:   # records of several kernels of one source
        v = t["per_kernel"].get(kernel, {}).get(str(key))
    elif t.get("kernel") == kernel:
        v = t.get("per_tile_rows", {}).get(str(key))
    else:
        v = None
    return None if v is None else v.get("bytes_per_launch")


# ---------------------------------------------------------------------------
# tuning and the timed map loop

def tune_handle(ff, torch, h, w, precision, ff_precision):
    """Apply the autotuner's choices (from the cache, or by timing every
    variant, then cached) to handle h; returns what was chosen."""
    from paper_1211_4461_amd import autotune
    tune = {}
    b = torch.empty(w.shape, dtype=torch.complex128, device="cuda")
    u = torch.empty_like(b)
    if ff.mg_tune_variants(h, ff.TUNE_FF_GEMM) > 1:
        tune["ff_gemm"] = autotune.tune_farfield(h, w.eta, None, w.dirs, ff_precision)
    for name, tn in (("smooth_coarse", ff.TUNE_SMOOTH_COARSE), ("smooth", ff.TUNE_SMOOTH), ("pre", ff.TUNE_PRE),
                     ("tail", ff.TUNE_TAIL), ("sweep3d", ff.TUNE_SWEEP3D)):
        if ff.mg_tune_variants(h, tn) > 1:
            ff.mg_rhs_plane_wave(h, w.eta, b)
            tune[name] = autotune.tune_solve(h, b, u, precision, tol=w.tol, tunable=tn)
    del b, u
    return tune


def copy_tuning(ff, src, dst):
    for tn in (ff.TUNE_FF_GEMM, ff.TUNE_SMOOTH, ff.TUNE_SMOOTH_COARSE, ff.TUNE_PRE, ff.TUNE_TAIL, ff.TUNE_SWEEP3D):
        if ff.mg_tune_variants(dst, tn) > 1:
            ff.mg_tune_set(dst, ff.mg_tune_get(src, tn), tn)


def run_path(ff, torch, w, precision, ff_precision, steps, warmup, fmg_cycles=FMG_K, lanes=1, pipelined=False,
             etas=None, tol=None, inner=0):
    """Time `steps` maps (right-hand side, solve, far field into device
    memory) after `warmup` rounds.  lanes = D > 1: maps cycle through D
    handles, each on its own stream; pipelined: each step begins its map's
    solve (mg_solve_begin) before it finishes the map begun D - 1 steps
    earlier (mg_solve_end, far field queued), so D solves are in flight from
    this host thread; the timed region ends when every map begun in it is
    finished.  etas: incoming directions cycled through map by map (default
    the workload's)."""
    etas = [w.eta] if etas is None else etas
    tol = w.tol if tol is None else tol
    opts = dict(precision=precision, ff_precision=ff_precision, fmg_cycles=fmg_cycles, inner_cycles=inner)
    ln_ = []
    for i in range(lanes):
        s_ = torch.cuda.Stream() if lanes > 1 else torch.cuda.current_stream()
        with torch.cuda.stream(s_):
            h_ = ff.setup_workload(w, options=ff.default_options(**opts))[0]
            u_ = torch.empty(w.shape, dtype=torch.complex128, device="cuda")
            F_ = torch.empty(len(w.dirs), dtype=torch.complex128, device="cuda")
        # the right-hand side is the handle's plane wave (b = None): not stored
        # where the solve forms it in its kernels
        ln_.append([h_, None, u_, F_, s_, None])
    tune = tune_handle(ff, torch, ln_[0][0], w, precision, ff_precision)
    for ln in ln_[1:]:
        copy_tuning(ff, ln_[0][0], ln[0])
    torch.cuda.synchronize()
    info = None
    last = []
    nstep = [0]
    pending = collections.deque()

    def begin_map():
        ln = ln_[nstep[0] % lanes]
        ln[5] = etas[nstep[0] % len(etas)]
        nstep[0] += 1
        ff.mg_rhs_plane_wave(ln[0], ln[5], ln[1])
        if fmg_cycles == 0:
            with torch.cuda.stream(ln[4]):
                ln[2].zero_()
        return ln

    def finish_map(info_, ln):
        nonlocal info
        info = info_
        ff.farfield_map(ln[0], ln[5], ln[2], w.dirs, out=ln[3])   # device output: queued, not waited for
        last.append(ln)

    def step():
        ln = begin_map()
        if not pipelined:
            finish_map(ff.mg_solve(ln[0], ln[1], ln[2], tol=tol), ln)
            return
        ff.mg_solve_begin(ln[0], ln[1], ln[2], tol=tol)
        pending.append(ln)
        if len(pending) == lanes:   # the oldest lane is next: finish its map
            old = pending.popleft()
            finish_map(ff.mg_solve_end(old[0]), old)

    def drain():
        while pending:
            old = pending.popleft()
            finish_map(ff.mg_solve_end(old[0]), old)

    for _ in range(max(warmup, 1) * lanes):
        step()
    drain()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    drain()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # the reference map for the accuracy figures: the first direction, solved
    # once more on lane 0 after the timed region (the same bits as any map of
    # that direction in it), so that maps of different runs compare alike
    ln = ln_[0]
    with torch.cuda.stream(ln[4]):
        ff.mg_rhs_plane_wave(ln[0], etas[0], ln[1])
        if fmg_cycles == 0:
            ln[2].zero_()
        ff.mg_solve(ln[0], ln[1], ln[2], tol=tol)
        ff.farfield_map(ln[0], etas[0], ln[2], w.dirs, out=ln[3])
    torch.cuda.synchronize()
    F = ln[3].cpu().numpy()
    out = {"ms_per_step": 1e3 * dt / steps, "maps_per_s": steps / dt, "cycles": info.cycles,
           "vcycles": info.vcycles, "rel_residual": info.rel_residual, "conv_factor": info.conv_factor, "F": F,
           "eta": etas[0], "tune": tune, "lanes": lanes, "pipelined": pipelined, "directions": len(etas)}
    for ln in ln_:
        ln[0].destroy()
    del ln_
    torch.cuda.empty_cache()
    return out


def kernel_pass(ff, torch, w, precision, ff_precision, maps, fmg_cycles, bpp, tol=None, inner=0):
    """The same maps one at a time (one handle, one stream) with HIP events
    around every launch of the finest-level kernels the library brackets:
    per-launch durations, early-exit launches (a batch step queued after the
    solve had stopped: under a fifth of the median) dropped, GB/s from the
    algorithmic bytes.  Returns per-kernel statistics and the dominant
    kernel among `bpp` (the largest total time per map)."""
    h = ff.setup_workload(w, options=ff.default_options(precision=precision, ff_precision=ff_precision,
                                                        fmg_cycles=fmg_cycles, inner_cycles=inner))[0]
    tune_handle(ff, torch, h, w, precision, ff_precision)
    u = torch.empty(w.shape, dtype=torch.complex128, device="cuda")
    F = torch.empty(len(w.dirs), dtype=torch.complex128, device="cuda")

    def one():
        ff.mg_rhs_plane_wave(h, w.eta, None)
        if fmg_cycles == 0:
            u.zero_()
        inf = ff.mg_solve(h, None, u, tol=w.tol if tol is None else tol)
        ff.farfield_map(h, w.eta, u, w.dirs, out=F)
        return inf

    one()
    torch.cuda.synchronize()
    mask = 0
    for k in ("pre", "post", "refine", "rr", "srr", "srr0", "ff", "ffgemm"):
        mask |= 1 << KERNELS[k]
    ff.mg_profile_enable(h, mask)
    for k in KERNELS.values():
        ff.mg_profile_durations(h, k)
    for _ in range(maps):
        info = one()
    torch.cuda.synchronize()
    stats = {}
    for name in ("pre", "post", "refine", "rr", "srr", "srr0", "ff", "ffgemm"):
        d = ff.mg_profile_durations(h, KERNELS[name])
        if d.size == 0:
            continue
        med = float(sorted(d)[d.size // 2])
        keep = d[d >= 0.2 * med]
        st = {"launches": int(keep.size), "early_exit_launches_dropped": int(d.size - keep.size),
              "avg_us": round(1e3 * float(keep.mean()), 2), "min_us": round(1e3 * float(keep.min()), 2),
              "max_us": round(1e3 * float(keep.max()), 2), "ms_per_map": round(float(keep.sum()) / maps, 3)}
        if name in bpp:
            gbs = bpp[name] * w.N / (keep.mean() * 1e-3) / 1e9
            st.update({"bytes_per_point": bpp[name], "bytes_per_launch": int(bpp[name] * w.N),
                       "GB_s": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)})
        stats[name] = st
    ff.mg_profile_enable(h, 0)
    dominant = max((k for k in bpp if k in stats), key=lambda k: stats[k]["ms_per_map"])
    out = {"kernels": stats, "dominant": dominant, "cycles": info.cycles, "vcycles": info.vcycles, "maps": maps}
    h.destroy()
    del u, F
    torch.cuda.empty_cache()
    return out


def gemm_report(stats, w, prec):
    """MFMA rate of the far-field GEMM stages (useful flops: 2D 8 M N; 3D the
    separable chain 8 N M_pol + 8 M (n-1)^2; a split precision issues
    `products` times as many)."""
    g = stats.get("ffgemm")
    if not g:
        return None
    t = g["avg_us"] * 1e-6
    M = len(w.dirs)
    m = w.n - 1
    if w.dim == 2:
        flop = 8.0 * M * w.N
    else:
        n_pol = len(set(round(float(z), 12) for z in w.dirs[:, 2]))
        flop = 8.0 * w.N * n_pol + 8.0 * M * m * m
    products, peak = {"bf16x6": (6, 2500.0), "bf16x3": (3, 2500.0), "fp64": (1, 78.6)}[prec]
    issued = products * flop / t / 1e12
    return {"us": g["avg_us"], "useful_flop_per_map": flop, "products": products,
            "useful_TFLOPs": round(flop / t / 1e12, 2), "mfma_TFLOPs": round(issued, 1), "peak_TFLOPs": peak,
            "mfma_frac": round(issued / peak, 4)}


# ---------------------------------------------------------------------------
# extra workloads

def run_stress(ff, torch, W, reps=3):
    """Solve-only at k0 h = 1/2 (the workloads' literal wavenumbers) with the
    bounded phase right-hand side: cycles, time per solve and the
    mixed-versus-plain speedup, and the finest post-smoothing kernel's rate."""
    out = {}
    for name, w, bpp in (("bumps_2d_2048", W.bumps_2d(k0=None, M=8), BPP[2]),
                         ("gauss_3d_512", W.gauss_3d(k0=None, n_az=4, n_pol=2), BPP[3])):
        r = {"k0": round(w.k0, 4), "k0h": 0.5, "rhs": "q exp(i k0 cos(gamma) eta.x) (mg_rhs_phase)",
             "start": f"full multigrid, {FMG_K} V(2,2) per coarse level"}
        for form, prec in (("mixed", ff.FP32_IR), ("plain_fp64", ff.FP64)):
            h = ff.setup_workload(w, options=ff.default_options(precision=prec, fmg_cycles=FMG_K))[0]
            b = ff.mg_rhs_phase(h, w.eta, torch.empty(w.shape, dtype=torch.complex128, device="cuda"))
            u = torch.empty_like(b)
            info = ff.mg_solve(h, b, u, tol=w.tol)
            torch.cuda.synchronize()
            ts = []
            for _ in range(reps):
                t0 = time.perf_counter()
                info = ff.mg_solve(h, b, u, tol=w.tol)
                ts.append(time.perf_counter() - t0)
            ff.mg_profile_enable(h, 1 << KERNELS["post"])
            ff.mg_profile_durations(h, KERNELS["post"])
            ff.mg_solve(h, b, u, tol=w.tol)
            d = ff.mg_profile_durations(h, KERNELS["post"])
            ff.mg_profile_enable(h, 0)
            d = d[d >= 0.2 * float(sorted(d)[d.size // 2])] if d.size else d
            bp = bpp["mixed" if form == "mixed" else "plain"]["post"]
            gbs = bp * w.N / (d.mean() * 1e-3) / 1e9 if d.size else None
            r[form] = {"ms_per_solve": round(1e3 * min(ts), 3), "steps": info.cycles, "vcycles": info.vcycles,
                       "rel_residual": info.rel_residual, "conv_factor": round(info.conv_factor, 4),
                       "post_smoothing_GB_s": None if gbs is None else round(gbs, 1)}
            h.destroy()
            del b, u
            torch.cuda.empty_cache()
        r["speedup_vs_plain"] = round(r["plain_fp64"]["ms_per_solve"] / r["mixed"]["ms_per_solve"], 3)
        out[name] = r
    return out


def run_ionization(ff, torch, W, lanes=4):
    """The ionisation cross sections of the Sec. 5.2 model over the 20
    energies of Fig. single_and_double (255^2 contour grid, h = 0.05,
    coarsest level 31^2, V(1,1) from a zero start to 1e-10): per energy
    mg_setup (coarsest inverse), the source right-hand side, the solve, the
    test functions of both axes, one contraction of 65 amplitudes and the
    cross sections; the bound state once per sweep (it depends on the
    potential only).  Whole-sweep wall time, so energies/s, with one energy
    at a time and with `lanes` energies in flight (one host thread, stream
    and handle each)."""
    import concurrent.futures as cf
    golden = {}
    gp = os.path.join(ROOT, "tests", "golden", "fig_single_and_double.txt")
    with open(gp) as f:
        for line in f:
            t = line.split("#", 1)[0].split()
            if t:
                golden[round(float(t[0]), 6)] = tuple(float(v) for v in t[1:])
    ws = [W.ionization_2d(E, n=256) for E in W.ION_ENERGIES]
    w0 = ws[0]
    src, v12, v1 = (torch.from_numpy(w0.params[k]).cuda() for k in ("src", "v12", "v1"))
    coefs = [torch.from_numpy(w.coef).cuda() for w in ws]
    M = 64
    out = {"workload": f"ionization_2d n=256 box=[0,12.8]^2 h=0.05 gamma={math.degrees(w0.gamma):.3f}deg, "
                       f"{len(ws)} energies {W.ION_ENERGIES[0]:.4f}..{W.ION_ENERGIES[-1]:.4f}, "
                       f"{M} double-ionisation nodes", "energies": [round(w.energy, 6) for w in ws], "lanes": lanes}

    def one(i, prec, stream, lam, phi0, tt):
        w, coef = ws[i], coefs[i]
        with torch.cuda.stream(stream):
            t0 = time.perf_counter()
            o = ff.default_options(nu1=w.nu1, nu2=w.nu2, coarsest_n=w.params["coarsest_n"], max_cycles=200,
                                   precision=prec)
            h = ff.mg_setup(2, [w.n] * 2, [0.0] * 2, [w.hi] * 2, w.gamma, coef, kind=ff.SCHRODINGER,
                            energy=w.energy, options=o, stream=stream)
            t1 = time.perf_counter()
            b = ff.mg_rhs_source(h, src, torch.empty_like(src))
            u = torch.zeros_like(b)
            info = ff.mg_solve(h, b, u, tol=w.tol)
            t2 = time.perf_counter()
            r = ff.ion_observables(h, src, v12, u, v1, v1, w.energy, M, lam, phi0)
            t3 = time.perf_counter()
            h.destroy()
        if tt is not None:
            tt["setup"] += t1 - t0
            tt["solve"] += t2 - t1
            tt["observables"] += t3 - t2
        return info.cycles, (r["single"], r["double"], r["total"])

    for form, prec in (("mixed", ff.FP32_IR), ("plain_fp64", ff.FP64)):
        rec = {}
        for nl in (1, lanes):
            best = None
            streams = [torch.cuda.Stream() for _ in range(nl)]
            for rep in range(2):
                tt = {"setup": 0.0, "solve": 0.0, "observables": 0.0} if nl == 1 else None
                torch.cuda.synchronize()
                t_all = time.perf_counter()
                # the bound state of the y axis: once per sweep
                h0 = ff.mg_setup(2, [w0.n] * 2, [0.0] * 2, [w0.hi] * 2, w0.gamma, coefs[0], kind=ff.SCHRODINGER,
                                 energy=w0.energy, options=ff.default_options(coarsest_n=w0.params["coarsest_n"]))
                lam, phi0 = ff.ion_bound_state(h0, 1, v1, -1.0)
                h0.destroy()
                if nl == 1:
                    res = [one(i, prec, streams[0], lam, phi0, tt) for i in range(len(ws))]
                else:
                    def lane(k):
                        return [(i, one(i, prec, streams[k], lam, phi0, None)) for i in range(k, len(ws), nl)]
                    with cf.ThreadPoolExecutor(nl) as ex:
                        parts = list(ex.map(lane, range(nl)))
                    res = [r for _, r in sorted(x for p in parts for x in p)]
                torch.cuda.synchronize()
                wall = time.perf_counter() - t_all
                if best is None or wall < best[0]:
                    best = (wall, tt, res)
            rec[nl] = best
        wall, tt, res = rec[1]
        cyc = [c for c, _ in res]
        xs = [x for _, x in res]
        dev = []
        for E, (s1, d1, t1) in zip(W.ION_ENERGIES, xs):
            g = golden[round(E, 6)]
            if E > -0.7:
                dev.append(max(abs(s1 - g[0]) / g[0], abs(t1 - g[2]) / g[2], abs(d1 - g[1]) / g[1] if g[1] > 0 else 0))
        wl = rec[lanes][0]
        out[form] = {"energies_per_s": round(len(ws) / wall, 2), "ms_per_energy": round(1e3 * wall / len(ws), 3),
                     "ms_per_energy_by_phase": {k: round(1e3 * v / len(ws), 3) for k, v in tt.items()},
                     f"energies_per_s_{lanes}_lanes": round(len(ws) / wl, 2),
                     "lanes_same_results": [x for _, x in rec[lanes][2]] == xs,
                     "cycles": cyc, "lambda0": [round(lam.real, 9), round(lam.imag, 9)],
                     "cross_sections": [[round(v, 9) for v in x] for x in xs],
                     "max_rel_dev_from_printed_points_E_gt_-0.7": round(max(dev), 4)}
    out["speedup_vs_plain"] = round(out["plain_fp64"]["ms_per_energy"] / out["mixed"]["ms_per_energy"], 3)
    out["note"] = ("cross sections: [single, double, total] per energy, half the outgoing flux per kind of channel; "
                   "the setup phase is dominated by the blocked Gauss-Jordan inverse of the 31^2 coarsest level")
    return out


def run_bumps2d(ff, torch, W, steps, warmup, lanes, ff_prec):
    """The 2048^2 bumps workload (k0 = 1, 360 angles): pipelined mixed and
    plain maps over four incoming directions, and the dominant kernel of its
    one-solve pass.  Its FP32 working set (about 142 MB per launch of the
    dominant kernel) fits the 256 MB Infinity Cache, so that rate is
    cache-assisted, not an HBM figure."""
    import numpy as np
    w = W.bumps_2d(n=2048, seed=1, k0=1.0, M=360)
    etas = [np.array([math.cos(a), math.sin(a)]) for a in (0.0, 0.5 * math.pi, math.pi, 1.5 * math.pi)]
    ffp = {"bf16x6": ff.FF_BF16X6, "bf16x3": ff.FF_BF16X3, "fp64": ff.FF_FP64}[ff_prec]
    m = run_path(ff, torch, w, ff.FP32_IR, ffp, steps, warmup, fmg_cycles=FMG_2D, lanes=lanes, pipelined=lanes > 1,
                 etas=etas, tol=MAP_TOL, inner=INNER_2D)
    p = run_path(ff, torch, w, ff.FP64, ff.FF_FP64, max(steps // 2, 2), warmup, fmg_cycles=FMG_K, lanes=lanes,
                 pipelined=lanes > 1, etas=etas, tol=MAP_TOL)
    bt = run_bumps2d_batched(ff, torch, w, etas, steps, ffp, m)
    km = kernel_pass(ff, torch, w, ff.FP32_IR, ffp, 8, FMG_2D, BPP[2]["mixed"], tol=MAP_TOL, inner=INNER_2D)
    kp = kernel_pass(ff, torch, w, ff.FP64, ff.FF_FP64, 4, FMG_K, BPP[2]["plain"], tol=MAP_TOL)
    dom = km["dominant"]
    th = (8, 16, 4)[m["tune"].get("smooth", 0)]
    return {"workload": "bumps_2d n=2048 box=[-10,10]^2 k0=1 gamma=30deg 8 bumps seed=1, 360 angles, "
                        "4 incoming directions cycled map by map", "tol": MAP_TOL,
            "start": f"mixed F({FMG_2D}), plain F({FMG_K})", "inner_cycles": INNER_2D,
            "lanes": lanes, "mixed": {"maps_per_s": round(m["maps_per_s"], 3), "ms_per_step": round(m["ms_per_step"], 3),
                                      "refinement_steps": m["cycles"], "vcycles": m["vcycles"],
                                      "rel_residual": m["rel_residual"], "tune": m["tune"]},
            "plain_fp64": {"maps_per_s": round(p["maps_per_s"], 3), "ms_per_step": round(p["ms_per_step"], 3),
                           "cycles": p["cycles"], "rel_residual": p["rel_residual"], "tune": p["tune"]},
            "speedup_vs_plain": round(m["maps_per_s"] / p["maps_per_s"], 3),
            "batched_directions": bt,
            "mixed_vs_plain_farfield_rel_err": float(np.linalg.norm(m["F"] - p["F"]) / np.linalg.norm(p["F"])),
            "kernels_mixed_one_solve": km["kernels"], "kernels_plain_one_solve": kp["kernels"],
            "dominant_kernel_roofline": {
                "kernel": KERNEL_NAMES[2][dom] % "float", "frac_of_hbm": km["kernels"][dom]["hbm_frac"],
                "GB_s": km["kernels"][dom]["GB_s"], "traffic": measured_traffic(dom, th, 2),
                "note": "cache-assisted: one launch moves about 142 MB, which fits the 256 MB Infinity Cache; "
                        "the HBM roofline is judged on the 512^3 headline"},
            "farfield_gemm": gemm_report(km["kernels"], w, ff_prec)}


def run_bumps2d_batched(ff, torch, w, etas, steps, ffp, m):
    """The same mixed maps with the incoming directions solved together: one
    mg_solve_batched over the directions of one operator (full multigrid
    start, FP32 V-cycles in FP64 refinement: every level of every direction
    in one launch) and one farfield_map_batched.  Each map equals the
    single-solve map of its direction bit for bit (checked on the direction
    the pipelined run `m` ended with)."""
    import numpy as np
    from paper_1211_4461_amd import autotune
    h = ff.setup_workload(w, options=ff.default_options(precision=ff.FP32_IR, ff_precision=ffp,
                                                        fmg_cycles=FMG_2D, inner_cycles=INNER_2D))[0]
    tune = tune_handle(ff, torch, h, w, ff.FP32_IR, ffp)
    hs = [h] * len(etas)
    us = [torch.empty(w.shape, dtype=torch.complex128, device="cuda") for _ in etas]
    tune["batch_tiles"] = autotune.tune_batch(hs, etas, us, tol=MAP_TOL)
    F = torch.empty((len(etas), len(w.dirs)), dtype=torch.complex128, device="cuda")
    infos = None

    def batch():
        nonlocal infos
        infos = ff.mg_solve_batched(hs, etas, us, tol=MAP_TOL)
        ff.farfield_map_batched(hs, etas, us, w.dirs, out=F)

    batch()
    batch()
    torch.cuda.synchronize()
    nb = max(steps // len(etas), 2)
    t0 = time.perf_counter()
    for _ in range(nb):
        batch()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / nb
    j = [i for i, e in enumerate(etas) if np.array_equal(np.asarray(e), np.asarray(m["eta"]))][0]
    same = bool(np.array_equal(F[j].cpu().numpy(), m["F"]))
    h.destroy()
    return {"directions": len(etas), "maps_per_s": round(len(etas) / dt, 3), "ms_per_batch": round(1e3 * dt, 3),
            "refinement_steps": [min(i.cycles for i in infos), max(i.cycles for i in infos)],
            "max_rel_residual": max(i.rel_residual for i in infos), "map_equal_to_single_solve": same,
            "tune": tune}


def run_gmres(ff, torch, W, n, steps=6):
    """The 2048^2 bumps workload solved with GMRES(3) smoothing steps (V(1,1),
    Sec. 3.3) from the full multigrid start, FP32 cycles in FP64 refinement,
    on contours of 10 and 30 degrees; weighted Jacobi is tried at 10 degrees
    (below its stability limit of about 13) with a cycle budget."""
    out = {"workload": f"bumps_2d n={n} box=[-10,10]^2 k0=1 8 bumps seed=1, 360 angles",
           "cycle": "V(1,1), GMRES(3) smoothing steps", "start": f"full multigrid, {FMG_K} V per coarse level"}
    for deg in (10, 30):
        w = W.bumps_2d(n=n, seed=1, k0=1.0, M=360)
        w.gamma = math.radians(deg)
        h = ff.setup_workload(w, options=ff.default_options(precision=ff.FP32_IR, ff_precision=ff.FF_BF16X6,
                                                            smoother=ff.SMOOTH_GMRES, krylov_m=3, nu1=1, nu2=1,
                                                            fmg_cycles=FMG_K))[0]
        b = torch.empty(w.shape, dtype=torch.complex128, device="cuda")
        u = torch.empty_like(b)
        F = torch.empty(len(w.dirs), dtype=torch.complex128, device="cuda")
        info = None

        def step():
            nonlocal info
            ff.mg_rhs_plane_wave(h, w.eta, b)
            info = ff.mg_solve(h, b, u, tol=w.tol)
            ff.farfield_map(h, w.eta, u, w.dirs, out=F)

        step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        r = {"maps_per_s": round(1.0 / dt, 3), "ms_per_map": round(1e3 * dt, 3), "refinement_steps": info.cycles,
             "vcycles": info.vcycles, "rel_residual": info.rel_residual, "conv_factor": round(info.conv_factor, 4)}
        h.destroy()
        if deg == 10:
            hj = ff.setup_workload(w, options=ff.default_options(precision=ff.FP32_IR, max_cycles=30))[0]
            ff.mg_rhs_plane_wave(hj, w.eta, b)
            u.zero_()
            ij = ff.mg_solve(hj, b, u, tol=w.tol, raise_on_noconv=False)
            r["jacobi_v22_status"] = {"status": ij.status, "steps": ij.cycles, "rel_residual": ij.rel_residual,
                                      "converged": ij.status == 0}
            hj.destroy()
        out[f"gamma_{deg}deg"] = r
    return out


def run_batched(ff, torch, W, steps):
    """The batched Schroedinger workload: 32 incoming directions x 3 energies
    on seed-drawn 255^2 / 511^2 / 1023^2 grids, all solved in one batched,
    graph-replayed solve and mapped at 360 angles; beside it the same 96 maps
    one after another through mg_solve / farfield_map."""
    from paper_1211_4461_amd import autotune
    insts = W.schrodinger_batch(seed=3)
    cache = {}
    hs = []
    for w in insts:
        key = (w.energy, w.n)
        if key not in cache:
            o = ff.default_options(precision=ff.FP32_IR, ff_precision=ff.FF_BF16X6, fmg_cycles=BATCH_FMG,
                                   inner_cycles=BATCH_INNER)
            h = ff.setup_workload(w, options=o)[0]
            autotune.tune_farfield(h, w.eta, None, w.dirs, ff.FF_BF16X6)
            cache[key] = h
        hs.append(cache[key])
    us = [torch.empty(w.shape, dtype=torch.complex128, device="cuda") for w in insts]
    etas = [w.eta for w in insts]
    dirs = insts[0].dirs
    tile_variant = autotune.tune_batch(hs, etas, us, tol=MAP_TOL)
    F = torch.empty((len(insts), len(dirs)), dtype=torch.complex128, device="cuda")
    infos = None

    def batch(tol):
        nonlocal infos
        infos = ff.mg_solve_batched(hs, etas, us, tol=tol)
        ff.farfield_map_batched(hs, etas, us, dirs, out=F)

    def timed(tol):
        batch(tol)
        batch(tol)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            batch(tol)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    # at the maps' tolerance (the value), then converged to 1e-10 (the
    # reference maps and the comparison with sequential solves)
    tm = timed(MAP_TOL)
    info_m = infos
    Fm = F.clone()
    tb = timed(FP64_TOL)
    Fb = F.clone()
    err_m = float(max((torch.linalg.vector_norm(Fm[i] - Fb[i]) / torch.linalg.vector_norm(Fb[i])).item()
                      for i in range(len(insts))))
    bs = [torch.empty_like(u) for u in us]

    def sequential():
        for i, w in enumerate(insts):
            ff.mg_rhs_plane_wave(hs[i], w.eta, bs[i])
            us[i].zero_()
            ff.mg_solve(hs[i], bs[i], us[i], tol=w.tol)
            ff.farfield_map(hs[i], w.eta, us[i], dirs, out=F[i])

    sequential()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sequential()
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    same = bool(torch.equal(F, Fb))
    sizes = {}
    for w in insts:
        sizes[f"{w.n - 1}^2"] = sizes.get(f"{w.n - 1}^2", 0) + 1
    out = {"workload": "schrodinger_batch seed=3: 32 directions x E in {0.5,1,2}, grids drawn from "
                       "{255^2, 511^2, 1023^2}, box [-10,10]^2, gamma=30deg, 360 angles; wells at 1/10 of the "
                       "literal depths (weighted-Jacobi V-cycles diverge on the literal bound states)",
           "instances": len(insts), "grids": sizes, "operators": len(cache),
           "start": f"F({BATCH_FMG})" if BATCH_FMG else "u = 0", "inner_cycles": BATCH_INNER,
           "tol": MAP_TOL, "maps_per_s": round(len(insts) / tm, 2), "ms_per_batch": round(1e3 * tm, 2),
           "refinement_steps": [min(i.cycles for i in info_m), max(i.cycles for i in info_m)],
           "max_map_rel_err_vs_tol_1e-10": err_m,
           "at_tol_1e-10": {"maps_per_s": round(len(insts) / tb, 2), "ms_per_batch": round(1e3 * tb, 2),
                            "refinement_steps": [min(i.cycles for i in infos), max(i.cycles for i in infos)],
                            "max_rel_residual": max(i.rel_residual for i in infos),
                            "sequential_maps_per_s": round(len(insts) / ts, 2),
                            "speedup_vs_sequential": round(ts / tb, 3),
                            "maps_equal_to_sequential": same},
           "tune": {"batch_tiles": tile_variant},
           "form": "FP32 V-cycles in FP64 refinement, batched + graph-replayed; split-BF16 (x6) far field"}
    for h in cache.values():
        h.destroy()
    return out


def run_literal_gmres(ff, torch, W, reps=2):
    """The batched workload's literal potential (wells of depth U[0.5, 2],
    where weighted-Jacobi V-cycles diverge on the bound states) solved with
    GMRES(3) V(1,1) smoothing (Sec. 5.5) as single solves, one per energy
    and grid size of the batch, mixed precision; each map against the plain
    FP64 GMRES map at 1e-10.  These operators are worse conditioned than the
    others (bound states): at the residual reduction 1e-6 their maps miss
    the 1e-6 bar by up to 3x (measured), so they solve to LITERAL_TOL."""
    import numpy as np
    out = {"workload": "schrodinger_batch law with the literal depths (B = 2, D ~ U[0.5, 2], seed 3), E in "
                       "{0.5, 1, 2} x grids {255^2, 511^2, 1023^2}, box [-10,10]^2, gamma = 30 deg, eta = +x, "
                       "360 angles; GMRES(3) V(1,1) smoothing, single solves (the batched path has "
                       "weighted-Jacobi kernels only)", "tol": LITERAL_TOL, "cases": []}
    dirs = W.directions_2d(360)
    tot_t, nmaps = 0.0, 0
    for n in (256, 512, 1024):
        V = W.schrodinger_potential(n, seed=3, deep=True)
        coef = torch.from_numpy(V).cuda()
        for E in (0.5, 1.0, 2.0):
            maps = {}
            for form, prec, ffp, tol in (("mixed", ff.FP32_IR, ff.FF_BF16X6, LITERAL_TOL),
                                         ("plain_fp64", ff.FP64, ff.FF_FP64, FP64_TOL)):
                o = ff.default_options(smoother=ff.SMOOTH_GMRES, krylov_m=3, nu1=1, nu2=1, precision=prec,
                                       ff_precision=ffp, fmg_cycles=FMG_K)
                h = ff.mg_setup(2, [n, n], [-10.0] * 2, [10.0] * 2, math.pi / 6, coef, kind=ff.SCHRODINGER,
                                energy=E, options=o)
                b = ff.mg_rhs_plane_wave(h, [1.0, 0.0], torch.empty((n - 1, n - 1), dtype=torch.complex128,
                                                                     device="cuda"))
                u = torch.empty_like(b)
                F = torch.empty(len(dirs), dtype=torch.complex128, device="cuda")
                info = ff.mg_solve(h, b, u, tol=tol)
                ff.farfield_map(h, [1.0, 0.0], u, dirs, out=F)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(reps):
                    ff.mg_rhs_plane_wave(h, [1.0, 0.0], b)
                    info = ff.mg_solve(h, b, u, tol=tol)
                    ff.farfield_map(h, [1.0, 0.0], u, dirs, out=F)
                torch.cuda.synchronize()
                dt = (time.perf_counter() - t0) / reps
                maps[form] = (F.cpu().numpy(), info, dt)
                h.destroy()
            Fm, im, tm = maps["mixed"]
            Fp, ip, tp = maps["plain_fp64"]
            tot_t += tm
            nmaps += 1
            out["cases"].append({"grid": f"{n - 1}^2", "E": E, "mixed_ms": round(1e3 * tm, 3),
                                 "mixed_steps": im.cycles, "mixed_vcycles": im.vcycles,
                                 "plain_ms_at_1e-10": round(1e3 * tp, 3), "plain_cycles_at_1e-10": ip.cycles,
                                 "map_rel_err_vs_fp64": float(np.linalg.norm(Fm - Fp) / np.linalg.norm(Fp))})
    out["mixed_maps_per_s"] = round(nmaps / tot_t, 2)
    return out


def run_literal_batch(ff, torch, W, lanes_per_op=1, reps=2):
    """The batched workload as written, with its literal potential: the 96
    instances of the schrodinger_batch law (32 directions x 3 energies, each
    on a seed-drawn 255^2 / 511^2 / 1023^2 grid, seed 3) with the deep wells
    (B = 2, D ~ U[0.5, 2]), solved with GMRES(3) V(1,1) smoothing in mixed
    precision to LITERAL_TOL.  The batched kernels are weighted Jacobi only,
    so the instances are single solves kept in flight: one handle (and
    stream) per operator, solves begun on every free handle before the oldest
    is finished (mg_solve_begin / mg_solve_end), then one farfield_map_batched
    for all 96 maps.  Beside it the same maps one after another; every map of
    the two runs is compared bit for bit."""
    import numpy as np
    insts = W.schrodinger_batch(seed=3)
    dirs = insts[0].dirs
    pots = {n: torch.from_numpy(W.schrodinger_potential(n, seed=3, deep=True)).cuda() for n in sorted({w.n for w in insts})}
    ops, streams = {}, {}
    for w in insts:
        for lane in range(lanes_per_op):
            key = (w.energy, w.n, lane)
            if key in ops:
                continue
            st = torch.cuda.Stream()
            with torch.cuda.stream(st):
                o = ff.default_options(smoother=ff.SMOOTH_GMRES, krylov_m=3, nu1=1, nu2=1, precision=ff.FP32_IR,
                                       ff_precision=ff.FF_BF16X6, fmg_cycles=FMG_K)
                ops[key] = ff.mg_setup(2, [w.n, w.n], [w.lo] * 2, [w.hi] * 2, w.gamma, pots[w.n],
                                       kind=ff.SCHRODINGER, energy=w.energy, options=o)
            streams[key] = st
    torch.cuda.synchronize()
    # instances interleaved over the operators (and lanes), so that consecutive solves use different handles
    by_op = {}
    for i, w in enumerate(insts):
        by_op.setdefault((w.energy, w.n), []).append(i)
    slots = []
    for k, idx in by_op.items():
        for j, i in enumerate(idx):
            slots.append((j // lanes_per_op, i, (k[0], k[1], j % lanes_per_op)))
    order = [(i, key) for _, i, key in sorted(slots)]
    us = [torch.empty(w.shape, dtype=torch.complex128, device="cuda") for w in insts]
    etas = [w.eta for w in insts]
    hs = [None] * len(insts)
    for i, key in order:
        hs[i] = ops[key]
    F = torch.empty((len(insts), len(dirs)), dtype=torch.complex128, device="cuda")
    infos = [None] * len(insts)

    def in_flight():
        pending = []   # (handle key, instance), oldest first
        busy = set()
        for i, key in order:
            while key in busy:
                k0, i0 = pending.pop(0)
                infos[i0] = ff.mg_solve_end(ops[k0])
                busy.discard(k0)
            h = ops[key]
            ff.mg_rhs_plane_wave(h, etas[i], None)
            ff.mg_solve_begin(h, None, us[i], tol=LITERAL_TOL)
            pending.append((key, i))
            busy.add(key)
        for k0, i0 in pending:
            infos[i0] = ff.mg_solve_end(ops[k0])
        ff.farfield_map_batched(hs, etas, us, dirs, out=F)

    def one_by_one(Fs):
        for i, key in order:
            h = ops[key]
            ff.mg_rhs_plane_wave(h, etas[i], None)
            ff.mg_solve(h, None, us[i], tol=LITERAL_TOL)
            ff.farfield_map(h, etas[i], us[i], dirs, out=Fs[i])

    in_flight()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        in_flight()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    F_fl = F.clone()
    F1 = torch.empty_like(F)
    one_by_one(F1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    one_by_one(F1)
    torch.cuda.synchronize()
    dt1 = time.perf_counter() - t0
    same = bool(torch.equal(F_fl, F1))
    steps = [i.cycles for i in infos]
    for h in ops.values():
        h.destroy()
    ns = [w.n - 1 for w in insts]
    return {"workload": "schrodinger_batch law (96 instances: 32 directions x E in {0.5, 1, 2}, grids drawn by "
                        "seed 3 from 255^2 / 511^2 / 1023^2) with the literal depths (B = 2, D ~ U[0.5, 2]), "
                        "360 angles; GMRES(3) V(1,1) smoothing, FP32 cycles in FP64 refinement, full multigrid "
                        f"start, residual reduction {LITERAL_TOL}",
            "grids": {f"{m}^2": ns.count(m) for m in sorted(set(ns))},
            "maps_per_s": round(len(insts) / dt, 2), "ms_per_batch": round(1e3 * dt, 3),
            "one_after_another_maps_per_s": round(len(insts) / dt1, 2),
            "operators": len({(w.energy, w.n) for w in insts}), "handles_per_operator": lanes_per_op,
            "refinement_steps": [min(steps), max(steps)],
            "max_rel_residual": max(i.rel_residual for i in infos),
            "maps_equal_to_one_after_another": same}


def run_learned(ff, torch, W, reps=3):
    """The learned-smoother workload: a network trained on the GPU (the
    library's kernels) from weighted Jacobi on (error, residual) patches of
    plain V-cycle iterates and white noise on 255^2 fields (k0 h in
    [0.02, 0.6]); then on a 1023^2 random bump field (seed 4) the finest
    level's smoother is the network or weighted Jacobi in V(2,2) cycles to
    1e-8: cycles and wall time at the stress point k0 h = 0.5 and at 0.2, and
    the far field at k0 = 1 (360 angles) against the plain FP64 map."""
    import numpy as np
    from paper_1211_4461_amd import learned as LS
    t0 = time.perf_counter()
    data = LS.make_patches(torch, n_fields=48, n=256, seed=1000)
    net = ff.Net(LS.jacobi_init(7))
    sub = [t[:1024].contiguous() for t in (data.rt, data.kt, data.et)]
    L0, _ = net.loss_grad(*sub)
    t1 = time.perf_counter()
    LS.train(torch, net, data, steps=4000, batch=256, lr=1e-3, lr_final=1e-5, seed=1)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    L1, _ = net.loss_grad(*sub)
    Ws = net.weights()
    net.destroy()
    out = {"workload": "random bump field seed 4 on 1023^2, box [-10,10]^2, gamma=30deg, V(2,2) to 1e-8; "
                       "finest-level smoother: trained network vs omega=0.8 Jacobi",
           "training": {"patches": int(data.count), "steps": 4000, "data_s": round(t1 - t0, 2),
                        "train_s": round(t2 - t1, 2), "loss_jacobi_start": round(L0, 4), "loss_trained": round(L1, 4)}}

    def solve(w, b, learned, tol=1e-8):
        o = ff.default_options(smoother=ff.SMOOTH_LEARNED, smoother_weights=Ws) if learned else ff.default_options()
        h = ff.setup_workload(w, options=o)[0]
        u = torch.zeros_like(b)
        info = ff.mg_solve(h, b, u, tol=tol)
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            u.zero_()
            torch.cuda.synchronize()
            t = time.perf_counter()
            info = ff.mg_solve(h, b, u, tol=tol)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t)
        net_ = None
        if learned:   # the network kernel alone, bracketed by HIP events in one more solve
            ff.mg_profile_enable(h, 1 << ff.PROF_NET)
            ff.mg_profile_read(h, ff.PROF_NET)
            u.zero_()
            ff.mg_solve(h, b, u, tol=tol)
            ms, cnt = ff.mg_profile_read(h, ff.PROF_NET)
            ff.mg_profile_enable(h, 0)
            us = 1e3 * ms / max(cnt, 1)
            useful = NET_FLOP_PER_POINT * w.N
            net_ = {"applications": cnt, "avg_us": round(us, 2), "useful_flop": useful,
                    "useful_TFLOPs": round(useful / (us * 1e-6) / 1e12, 1),
                    "mfma_frac_useful": round(useful / (us * 1e-6) / 1e12 / 2500.0, 4)}
        return h, u, info, 1e3 * min(ts), net_

    for kh in (0.5, 0.2):
        w = W.random_field(1024, 4, kh)
        b = LS.phase_rhs(w, torch)
        hj, uj, ij, tj, _ = solve(w, b, False)
        hl, ul, il, tl, net_ = solve(w, b, True)
        out[f"k0h={kh}"] = {"jacobi": {"cycles": ij.cycles, "conv_factor": round(ij.conv_factor, 4), "ms": round(tj, 3)},
                            "learned": {"cycles": il.cycles, "conv_factor": round(il.conv_factor, 4), "ms": round(tl, 3),
                                        "fell_back": il.fell_back, "network_kernel": net_},
                            "solution_rel_diff": float(torch.linalg.norm(ul - uj) / torch.linalg.norm(uj))}
        hj.destroy()
        hl.destroy()
    w = W.random_field(1024, 4, 20.0 / 1024)
    maps = {}
    for learned in (False, True):
        o = ff.default_options(smoother=ff.SMOOTH_LEARNED, smoother_weights=Ws) if learned else ff.default_options()
        h = ff.setup_workload(w, options=o)[0]
        b = ff.mg_rhs_plane_wave(h, w.eta, torch.empty(w.shape, dtype=torch.complex128, device="cuda"))
        u = torch.zeros_like(b)
        ff.mg_solve(h, b, u, tol=1e-8 if learned else 1e-10)
        maps[learned] = ff.farfield_map(h, w.eta, u, w.dirs)
        h.destroy()
    out["k0=1"] = {"farfield_rel_err_vs_plain_fp64": float(np.linalg.norm(maps[True] - maps[False]) /
                                                             np.linalg.norm(maps[False]))}
    return out


# ---------------------------------------------------------------------------
# A plain device copy on the same GPU: what streaming HBM traffic reaches here

def copy_rate(torch, gib=1, reps=5):
    """Bytes read + written per second (GB/s, best of reps) by a device copy
    of `gib` GiB (torch y.copy_(x)), timed with events on the current stream."""
    n = (gib << 30) // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        y.copy_(x)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del x, y
    torch.cuda.empty_cache()
    return 2.0 * (gib << 30) / (best * 1e-3) / 1e9


# ---------------------------------------------------------------------------
# CPU baseline (child process: the oracle, built for this host)

def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_sample(n, plain_cycles, n_dirs_sample, out_path):
    """Child process: the FP64 oracle as it stands, built -O3 -march=native
    for this host, on a bounded sample of the 3D workload at n intervals:
    setup, the full multigrid start, one V(2,2)-cycle and the far field of
    n_dirs_sample of the 128 x 64 directions, each timed; the map time is
    estimated as start + plain_cycles V-cycles + the far field scaled to all
    directions (the cycle count is the plain FP64 GPU path's, which equals
    the oracle's iteration: parity tests)."""
    import numpy as np
    from oracle import oracle as orc
    from paper_1211_4461_amd import workloads as W
    lib = orc.build(force=True, native=True, path=os.path.join(tempfile.gettempdir(), "libffmg_oracle_native.so"))
    orc.load(lib)
    w = W.gauss_3d(n=n)
    g = orc.Grid(w.dim, w.n, w.lo, w.hi)
    kappa, q, k0 = orc.problem(w.kind, w.k0, w.energy, w.coef)
    t0 = time.perf_counter()
    mg = orc.Multigrid(g, w.gamma, kappa, nu1=w.nu1, nu2=w.nu2, omega=w.omega)
    b = orc.rhs_plane_wave(g, w.gamma, k0, q, w.eta)
    t1 = time.perf_counter()
    u = mg.fmg(b, FMG_3D)
    t2 = time.perf_counter()
    u = mg.vcycle(b, u)
    t3 = time.perf_counter()
    idx = np.linspace(0, len(w.dirs) - 1, n_dirs_sample).astype(int)
    orc.farfield(g, w.gamma, k0, q, w.eta, u, w.dirs[idx])
    t4 = time.perf_counter()
    t_ff = (t4 - t3) * len(w.dirs) / n_dirs_sample
    est = (t2 - t1) + plain_cycles * (t3 - t2) + t_ff
    res = {"threads": orc.num_threads(), "setup_s": round(t1 - t0, 3), "fmg_start_s": round(t2 - t1, 3),
           "vcycle_s": round(t3 - t2, 3), "farfield_sample_s": round(t4 - t3, 3), "farfield_est_s": round(t_ff, 2),
           "map_est_s": round(est, 2), "map_est_zero_start_s": None}
    with open(out_path, "w") as f:
        json.dump(res, f)


def cpu_baseline(plain_cycles_fmg, plain_cycles_zero):
    """The oracle on the host cores (all of them, then one thread on a
    smaller instance of the same law), in child processes."""
    out = {}
    runs = {}
    for tag, n, threads, ndir in (("all", 512, None, 16), ("one", 128, 1, 8)):
        env = dict(os.environ)
        if threads:
            env["OMP_NUM_THREADS"] = str(threads)
        path = os.path.join(tempfile.gettempdir(), f"ffmg_cpu_{tag}.json")
        cmd = [sys.executable, os.path.abspath(__file__), "--cpu-sample", str(n), str(plain_cycles_fmg), str(ndir),
               path]
        subprocess.check_call(cmd, env=env, stdout=subprocess.DEVNULL)
        with open(path) as f:
            runs[tag] = json.load(f)
    a = runs["all"]
    zero_est = a["map_est_s"] - a["fmg_start_s"] + (plain_cycles_zero - plain_cycles_fmg) * a["vcycle_s"]
    return {"value": round(1.0 / a["map_est_s"], 5), "unit": "maps/s", "cores": a["threads"], "kind": "oracle",
            "sample": (f"512^3 (the headline workload), the oracle built -O3 -march=native on this host: setup, the "
                       f"full multigrid start and one V(2,2)-cycle timed, the far field timed on 16 of the 8192 "
                       f"directions; map = start + {plain_cycles_fmg} V-cycles (the plain FP64 count from that start) "
                       f"+ far field scaled to 8192 directions"),
            "cpu_model": cpu_model(), "measured": a,
            "map_est_zero_start_s": round(zero_est, 2),
            "one_thread": {"instance": "gauss_3d n=128 (the same law, 1/64 of the points)", **runs["one"]}}


# ---------------------------------------------------------------------------

def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=16, help="timed maps of the headline")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--lanes", type=int, default=2, help="solves in flight (handles and streams) of the headline")
    ap.add_argument("--ff-precision", choices=("bf16x6", "bf16x3", "fp64"), default="bf16x6",
                    help="far-field contraction of the mixed path")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain FP64 path of the headline")
    ap.add_argument("--no-stress", action="store_true", help="skip the k0h = 1/2 solve-only points")
    ap.add_argument("--no-2d", action="store_true", help="skip the 2048^2 bumps workload")
    ap.add_argument("--no-gmres", action="store_true", help="skip the GMRES(3)-smoother workload")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched Schroedinger workload")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-smoother workload")
    ap.add_argument("--no-ion", action="store_true", help="skip the ionisation cross-section sweep")
    ap.add_argument("--no-3d", action="store_true",
                    help="profiling aid: skip the 512^3 headline and report the 2048^2 workload alone")
    ap.add_argument("--tune-only", action="store_true", help="fill the autotuning cache for the headline and exit")
    ap.add_argument("--tune-in-process", action="store_true",
                    help="run the autotuning sweeps in this process instead of a child process")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one 1 GiB device copy (counter calibration for rocprofv3 --pmc)")
    ap.add_argument("--cpu-sample", nargs=4, metavar=("N", "CYCLES", "NDIRS", "OUT"), help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multigrid sweeps and the far-field contraction are measured on one MI355X.", file=sys.stderr)
        sys.exit(2)
    if args.cpu_sample:
        n, cyc, nd, outp = args.cpu_sample
        cpu_sample(int(n), int(cyc), int(nd), outp)
        return

    if not args.tune_only and not args.tune_in_process:
        # the autotuning sweeps run in a child process that fills the cache
        # before this process touches the GPU; this one reads the cache
        cmd = [sys.executable, os.path.abspath(__file__), "--tune-only", "--ff-precision", args.ff_precision] + (
            ["--no-2d"] if args.no_2d else [])
        rc = subprocess.call(cmd, stdout=subprocess.DEVNULL)
        if rc != 0:
            print(f"bench.py: the autotuning child process failed ({rc}); tuning in this process", file=sys.stderr)

    import numpy as np
    import torch

    from paper_1211_4461_amd import ffmg
    from paper_1211_4461_amd import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    ffmg.lib()
    ffp_name = args.ff_precision
    ffp = {"bf16x6": ffmg.FF_BF16X6, "bf16x3": ffmg.FF_BF16X3, "fp64": ffmg.FF_FP64}[ffp_name]
    w = W.gauss_3d()
    if args.tune_only:
        wl = [w] + ([] if args.no_2d else [W.bumps_2d(n=2048, seed=1, k0=1.0, M=360)])
        for wk in wl:
            for prec, fp in ((ffmg.FP32_IR, ffp), (ffmg.FP64, ffmg.FF_FP64)):
                inner = (INNER_3D if wk.dim == 3 else INNER_2D) if prec == ffmg.FP32_IR else 0
                fk = FMG_3D if wk.dim == 3 else (FMG_2D if prec == ffmg.FP32_IR else FMG_K)
                h = ffmg.setup_workload(wk, options=ffmg.default_options(precision=prec, ff_precision=fp,
                                                                         fmg_cycles=fk, inner_cycles=inner))[0]
                tune_handle(ffmg, torch, h, wk, prec, fp)
                h.destroy()
                torch.cuda.empty_cache()
        return
    if args.calib_copy:
        x = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        del x, y

    lanes = max(args.lanes, 1)
    pipe = lanes > 1
    if args.no_3d:
        # profiling aid: the 2D workload alone (its maps/s in "value")
        b2 = run_bumps2d(ffmg, torch, W, 40, 3, 4, ffp_name)
        line = {"metric": "far-field maps/sec at 1e-6 rel error: plain FP64 MG vs mixed-prec/learned MG",
                "value": b2["mixed"]["maps_per_s"], "unit": "maps/s", "n_gpus": 1, "steps": 40, "warmup": 3,
                "ms_per_step": b2["mixed"]["ms_per_step"], "higher_is_better": True, "scaling": "weak",
                "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
                "config": {"workload": b2["workload"]}, "bumps_2d": b2}
        args.no_2d = True
        args.no_plain = True
    else:
        # consecutive maps take four incoming directions in turn (+x, +y, -x, -y:
        # equivalent for this scatterer, so every map does the same work), so
        # that no lane can pass on another lane's data unnoticed
        etas3 = [np.array(e, dtype=np.float64) for e in ((1, 0, 0), (0, 1, 0), (-1, 0, 0), (0, -1, 0))]
        mixed = run_path(ffmg, torch, w, ffmg.FP32_IR, ffp, args.steps, args.warmup, fmg_cycles=FMG_3D, lanes=lanes,
                         pipelined=pipe, etas=etas3, tol=MAP_TOL, inner=INNER_3D)
        # the dominant kernel and the finest-level kernel rates: one solve in flight
        km = kernel_pass(ffmg, torch, w, ffmg.FP32_IR, ffp, 4, FMG_3D, BPP[3]["mixed"], tol=MAP_TOL,
                         inner=INNER_3D)
        dom = km["dominant"]
        dk = km["kernels"][dom]
        roof = {"kernel": KERNEL_NAMES[3][dom] % "float", "bound": "hbm", "achieved": dk["GB_s"], "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": dk["hbm_frac"], "traffic": measured_traffic(dom, "float", 3),
                "bytes_per_launch": dk["bytes_per_launch"], "bytes_per_point": dk["bytes_per_point"],
                "avg_launch_us": dk["avg_us"], "launches": dk["launches"],
                "early_exit_launches_dropped": dk["early_exit_launches_dropped"],
                "timed_in": "a one-solve-in-flight pass of the same maps after the headline: HIP events around every "
                            "launch of the finest-level kernels the library brackets",
                "ranked_by": "largest time per map among the bracketed finest-level kernels; "
                             "profiles/kernels_gauss3d_512_mixed.md ranks every kernel of a map (rocprofv3)",
                "working_set": "HBM-resident: one FP32 field is 1.07 GB, far above the 256 MB Infinity Cache"}
        cr = copy_rate(torch)
        roof["device_copy_GBs"] = round(cr, 1)
        roof["frac_of_device_copy"] = round(dk["GB_s"] / cr, 4)
        roof["device_copy"] = "1 GiB torch copy on this GPU, read + write bytes over the best of 5 event-timed copies"
        line = {
            "metric": "far-field maps/sec at 1e-6 rel error: plain FP64 MG vs mixed-prec/learned MG",
            "value": round(mixed["maps_per_s"], 3),
            "unit": "maps/s",
            "n_gpus": 1,
            "steps": args.steps,
            "warmup": args.warmup,
            "ms_per_step": round(mixed["ms_per_step"], 3),
            "higher_is_better": True,
            "scaling": "weak",
            "vs_baseline": None,
            "dtype": "f32+f64",
            "data": "synthetic",
            "config": {"workload": f"gauss_3d n=512 box=[-6,6]^3 chi=0.5exp(-z.z/2) k0=1 gamma=30deg, "
                                   f"incoming directions +x, +y, -x, -y cycled map by map, "
                                   f"128 azimuth x 64 polar outgoing directions",
                       "unknowns": w.N, "directions": len(w.dirs), "tol": MAP_TOL,
                       "accuracy": "maps within 1e-6 relative of the FP64 map converged to 1e-10 (measured: "
                                   "map_rel_err_vs_fp64)", "cycle": "V(2,2) omega=0.8 Jacobi",
                       "start": f"full multigrid: {FMG_3D} V(2,2) per coarse level, then the finest-level iteration",
                       "lanes": (f"{lanes} solves in flight from one host thread (one handle and stream each, "
                                 "mg_solve_begin / mg_solve_end)" if pipe else "1"),
                       "inner_cycles": INNER_3D,
                       "form": "FP32 V-cycles in FP64 refinement + "
                               + {"bf16x6": "split-BF16 (3 parts, 6 products) MFMA far field, FP32 accumulation",
                                  "bf16x3": "split-BF16 (2 parts, 3 products) MFMA far field, FP32 accumulation",
                                  "fp64": "FP64 MFMA far field"}[ffp_name]},
            "mixed": {"refinement_steps": mixed["cycles"], "vcycles": mixed["vcycles"],
                      "rel_residual": mixed["rel_residual"], "conv_factor": round(mixed["conv_factor"], 4),
                      "tune": mixed["tune"], "kernels_one_solve": km["kernels"],
                      "farfield_gemm": gemm_report(km["kernels"], w, ffp_name)},
            "roofline": roof,
        }
        if not args.no_plain:
            def map_err(F, Fr):
                return {"norm": float(np.linalg.norm(F - Fr) / np.linalg.norm(Fr)),
                        "elementwise": float(np.abs(F - Fr).max() / np.abs(Fr).max())}
            # plain FP64 at the same tolerance (equal accuracy), and converged to 1e-10 (the FP64 path's own
            # tolerance, and the reference map of the accuracy figures)
            plain = run_path(ffmg, torch, w, ffmg.FP64, ffmg.FF_FP64, max(args.steps // 2, 2), args.warmup,
                             fmg_cycles=FMG_3D, lanes=lanes, pipelined=pipe, etas=etas3, tol=MAP_TOL)
            kp = kernel_pass(ffmg, torch, w, ffmg.FP64, ffmg.FF_FP64, 2, FMG_3D, BPP[3]["plain"], tol=MAP_TOL)
            p10 = run_path(ffmg, torch, w, ffmg.FP64, ffmg.FF_FP64, max(args.steps // 4, 2), 1, fmg_cycles=FMG_3D,
                           lanes=lanes, pipelined=pipe, etas=etas3, tol=FP64_TOL)
            m10 = run_path(ffmg, torch, w, ffmg.FP32_IR, ffp, max(args.steps // 2, 2), 1, fmg_cycles=FMG_3D,
                           lanes=lanes, pipelined=pipe, etas=etas3, tol=FP64_TOL, inner=INNER_3D)
            line["map_rel_err_vs_fp64"] = map_err(mixed["F"], p10["F"])
            line["plain_fp64"] = {"value": round(plain["maps_per_s"], 3), "ms_per_step": round(plain["ms_per_step"], 3),
                                  "tol": MAP_TOL, "cycles": plain["cycles"], "rel_residual": plain["rel_residual"],
                                  "map_rel_err_vs_fp64": map_err(plain["F"], p10["F"]), "tune": plain["tune"],
                                  "kernels_one_solve": kp["kernels"], "farfield_gemm": gemm_report(kp["kernels"], w, "fp64")}
            line["speedup_vs_plain"] = round(mixed["maps_per_s"] / plain["maps_per_s"], 3)
            line["at_tol_1e-10"] = {
                "plain_fp64": {"value": round(p10["maps_per_s"], 3), "ms_per_step": round(p10["ms_per_step"], 3),
                               "cycles": p10["cycles"], "rel_residual": p10["rel_residual"]},
                "mixed": {"value": round(m10["maps_per_s"], 3), "ms_per_step": round(m10["ms_per_step"], 3),
                          "refinement_steps": m10["cycles"], "vcycles": m10["vcycles"],
                          "rel_residual": m10["rel_residual"], "map_rel_err_vs_fp64": map_err(m10["F"], p10["F"])},
                "speedup_vs_plain": round(m10["maps_per_s"] / p10["maps_per_s"], 3)}
            # the plain iteration from u = 0, for the CPU baseline's zero-start estimate
            h0 = ffmg.setup_workload(w, options=ffmg.default_options())[0]
            b0 = ffmg.mg_rhs_plane_wave(h0, w.eta, torch.empty(w.shape, dtype=torch.complex128, device="cuda"))
            u0 = torch.zeros_like(b0)
            zero_cycles = ffmg.mg_solve(h0, b0, u0, tol=MAP_TOL).cycles
            h0.destroy()
            del b0, u0
            torch.cuda.empty_cache()
            line["plain_fp64"]["cycles_zero_start"] = zero_cycles
    if not args.no_stress:
        line["stress_k0h_half"] = run_stress(ffmg, torch, W)
    if not args.no_2d:
        line["bumps_2d"] = run_bumps2d(ffmg, torch, W, 40, 3, 4, ffp_name)
    if not args.no_gmres:
        line["gmres_smoother"] = run_gmres(ffmg, torch, W, 2048)
    if not args.no_batch:
        line["batched"] = run_batched(ffmg, torch, W, 4)
    if not args.no_learned:
        line["learned"] = run_learned(ffmg, torch, W)
    if not args.no_batch:
        line["literal_batch_potential_gmres"] = run_literal_gmres(ffmg, torch, W)
        line["literal_batch_as_written"] = run_literal_batch(ffmg, torch, W, lanes_per_op=2)
    if not args.no_ion:
        line["ionization"] = run_ionization(ffmg, torch, W)
    if not args.no_cpu_baseline:
        pc = line.get("plain_fp64", {}).get("cycles", 14)
        pz = line.get("plain_fp64", {}).get("cycles_zero_start", 21)
        line["cpu_baseline"] = cpu_baseline(pc, pz)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
