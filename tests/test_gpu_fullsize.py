"""Parity at the workloads' full sizes, in the configuration the benchmark
times, on outputs the FP64 oracle can afford there:

* 2048^2 bumps, FP32 V-cycles in FP64 refinement + split-BF16 far field: the
  right-hand side element by element, the residual of the GPU solution under
  the oracle's operator, and the map against the oracle's map of the GPU
  solution and of its own converged solution (1e-6, the mixed forms' bar),
  also for the benchmark's maps (full multigrid start, residual reduction
  1e-6, mixed and plain);
  and the benchmark's pipelined form (full multigrid start, four solves in
  flight), every map bit for bit the map solved alone;
* 512^3 Gaussian (3D, 7-point stencil), same form: right-hand side, residual
  under the oracle's operator, and 16 sampled directions of the 128 x 64 map
  against the oracle's quadrature of the GPU solution, and the benchmark's
  map (full multigrid start, residual reduction 1e-6) against that map;
* the 96-instance batched Schroedinger workload: sampled instances of every
  grid size bit for bit equal to their single solves, residual under the
  oracle's operator and far field against the oracle;
* 1023^2 learned smoothing step: sampled output points against the oracle
  network evaluated on the window each point depends on.
"""
import numpy as np
import pytest

from paper_1211_4461_amd import workloads as W
from tests.compare import rel as relerr

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ff():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1211_4461_amd import ffmg
    ffmg.lib()
    return ffmg




def check_solution(orc, w, b_gpu, u_gpu, info, tol):
    """RHS against the oracle element by element; the GPU solution's residual
    under the oracle's FP64 operator meets the tolerance and agrees with the
    residual the library reported."""
    g = orc.Grid(w.dim, w.n, w.lo, w.hi)
    kappa, q, k0 = orc.problem(w.kind, w.k0, w.energy, w.coef)
    bo = orc.rhs_plane_wave(g, w.gamma, k0, q, w.eta)
    bg = b_gpu.cpu().numpy().reshape(g.shape)
    assert np.max(np.abs(bg - bo)) <= 1e-12 * np.max(np.abs(bo))
    u = u_gpu.cpu().numpy().reshape(g.shape)
    r = orc.residual(g, w.gamma, kappa, bo, u)
    rel = float(np.linalg.norm(r) / np.linalg.norm(bo))
    assert rel <= 1.01 * tol, rel
    assert abs(rel - info.rel_residual) <= 1e-2 * rel, (rel, info.rel_residual)
    return g, kappa, q, k0, bo, u


def test_bumps_2048_mixed_map(ff, orc):
    w = W.bumps_2d()
    o = ff.default_options(precision=ff.FP32_IR, ff_precision=ff.FF_BF16X6)
    h = ff.setup_workload(w, options=o)[0]
    b = ff.mg_rhs_plane_wave(h, w.eta, torch.empty(w.shape, dtype=torch.complex128, device="cuda"))
    u = torch.zeros_like(b)
    info = ff.mg_solve(h, b, u, tol=w.tol)
    assert info.status == 0
    F = ff.farfield_map(h, w.eta, u, w.dirs)
    g, kappa, q, k0, bo, ug = check_solution(orc, w, b, u, info, w.tol)
    Fu = orc.farfield(g, w.gamma, k0, q, w.eta, ug, w.dirs)
    assert relerr(F, Fu) < 1e-6
    uo, st, k, _ = orc.Multigrid(g, w.gamma, kappa).solve(bo, tol=1e-11)
    assert st == 0
    Fo = orc.farfield(g, w.gamma, k0, q, w.eta, uo, w.dirs)
    print(f"2048^2: {info.cycles} refinement steps, residual {info.rel_residual:.2e}; map vs oracle "
          f"{relerr(F, Fo):.2e} (oracle {k} cycles)")
    assert relerr(F, Fo) < 1e-6
    h.destroy()
    # the benchmark's form: full multigrid start (mixed: F(1) and one
    # refinement step of four FP32 V-cycles; plain FP64: F(2)), residual
    # reduction 1e-6, the handle's plane wave as the right-hand side; both
    # maps within 1e-6 of the oracle's converged map
    for prec, ffp, fk, inner in ((ff.FP32_IR, ff.FF_BF16X6, 1, 4), (ff.FP64, ff.FF_FP64, 2, 0)):
        h = ff.setup_workload(w, options=ff.default_options(precision=prec, ff_precision=ffp, fmg_cycles=fk,
                                                            inner_cycles=inner))[0]
        ff.mg_rhs_plane_wave(h, w.eta, None)
        ih = ff.mg_solve(h, None, u, tol=1e-6)
        assert ih.status == 0 and ih.rel_residual <= 1e-6
        Fh = ff.farfield_map(h, w.eta, u, w.dirs)
        print(f"2048^2 at tol 1e-6 (precision {prec}): {ih.cycles} steps, map vs oracle {relerr(Fh, Fo):.2e}")
        assert relerr(Fh, Fo) < 1e-6
        h.destroy()


def test_bumps_2048_pipelined_headline_configuration(ff, orc):
    """The pipelined launch configuration of the 2D workload: F(1) start,
    four FP32 V-cycles per refinement step, four handles on four streams, each
    map begun before the map three steps earlier is finished, every map with
    an incoming direction of its own (four directions) given as the handle's
    plane wave.  Every map equals, bit for bit, the map of its direction
    solved alone with mg_solve from the stored right-hand side (so no lane
    reads another lane's buffers); the last solution meets the tolerance under the oracle's
    operator and its map matches the oracle's quadrature of it."""
    import math
    w = W.bumps_2d()
    etas = [np.array([math.cos(a), math.sin(a)]) for a in (0.0, 0.5 * math.pi, 0.25 * math.pi, math.pi)]
    opts = dict(precision=ff.FP32_IR, ff_precision=ff.FF_BF16X6, fmg_cycles=1, inner_cycles=4)
    lanes = []
    for _ in range(4):
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            h = ff.setup_workload(w, options=ff.default_options(**opts))[0]
            b = torch.empty(w.shape, dtype=torch.complex128, device="cuda")
            u = torch.empty_like(b)
            F = torch.empty(len(w.dirs), dtype=torch.complex128, device="cuda")
        lanes.append((h, b, u, F))
    # each direction alone (on lane 0)
    h, b, u, F = lanes[0]
    solo = []
    for e in etas:
        ff.mg_rhs_plane_wave(h, e, b)
        inf = ff.mg_solve(h, b, u, tol=w.tol)
        ff.farfield_map(h, e, u, w.dirs, out=F)
        torch.cuda.synchronize()
        assert inf.status == 0
        solo.append((inf, F.clone(), u.clone()))
    # eight maps, four in flight, map k along etas[(k + 1) % 4] (a lane never repeats its last direction)
    pend, done = [], []
    for k in range(8):
        ln = lanes[k % 4]
        d = (k + 1) % 4
        ff.mg_rhs_plane_wave(ln[0], etas[d], None)   # the handle's plane wave, as the benchmark
        ff.mg_solve_begin(ln[0], None, ln[2], tol=w.tol)
        pend.append((ln, d))
        if len(pend) == 4 or k == 7:
            while pend and (len(pend) == 4 or k == 7):
                o, do = pend.pop(0)
                inf = ff.mg_solve_end(o[0])
                ff.farfield_map(o[0], etas[do], o[2], w.dirs, out=o[3])
                torch.cuda.synchronize()
                done.append((do, inf, o[3].clone(), o[2].clone(), None))
    assert len(done) == 8
    for i, (d, inf, Fk, uk, bk) in enumerate(done):
        s_inf, s_F, s_u = solo[d]
        assert inf.status == 0 and (inf.cycles, inf.rel_residual) == (s_inf.cycles, s_inf.rel_residual), i
        assert torch.equal(Fk, s_F) and torch.equal(uk, s_u), i
    d, inf, Fk, uk, _ = done[-1]
    w.eta = etas[d]
    # the lanes solved for the handles' plane waves: the stored right-hand
    # side of that direction for the check against the oracle
    bk = ff.mg_rhs_plane_wave(lanes[0][0], etas[d], lanes[0][1])
    g, kappa, q, k0, bo, ug = check_solution(orc, w, bk, uk, inf, w.tol)
    Fu = orc.farfield(g, w.gamma, k0, q, w.eta, ug, w.dirs)
    assert relerr(Fk.cpu().numpy(), Fu) < 1e-6
    for ln in lanes:
        ln[0].destroy()


def test_gauss3d_512_mixed(ff, orc):
    w = W.gauss_3d()
    o = ff.default_options(precision=ff.FP32_IR, ff_precision=ff.FF_BF16X6)
    h = ff.setup_workload(w, options=o)[0]
    b = ff.mg_rhs_plane_wave(h, w.eta, torch.empty(w.shape, dtype=torch.complex128, device="cuda"))
    u = torch.zeros_like(b)
    info = ff.mg_solve(h, b, u, tol=w.tol)
    assert info.status == 0
    F = ff.farfield_map(h, w.eta, u, w.dirs)
    h.destroy()
    g, kappa, q, k0, bo, ug = check_solution(orc, w, b, u, info, w.tol)
    del b, u, kappa, bo
    # 16 sampled directions on two polar angles (the oracle contracts each
    # direction over the whole grid)
    rng = np.random.default_rng(7)
    n_az = 128
    idx = np.concatenate([p * n_az + rng.choice(n_az, 8, replace=False) for p in (5, 40)])
    Fs = orc.farfield(g, w.gamma, k0, q, w.eta, ug, w.dirs[idx])
    print(f"512^3: {info.cycles} refinement steps, residual {info.rel_residual:.2e}; sampled map vs oracle "
          f"{relerr(F[idx], Fs):.2e}")
    assert relerr(F[idx], Fs) < 1e-6
    # the benchmark's headline form: F(3) start, three FP32 V-cycles per
    # refinement step, the handle's plane wave as the right-hand side (never
    # stored), stopped at the residual reduction 1e-6; its map within 1e-6 of
    # the map of the solution converged to 1e-10 (Fs: the oracle's quadrature
    # of that solution, whose residual was checked under the oracle's operator
    # above)
    del ug
    h = ff.setup_workload(w, options=ff.default_options(precision=ff.FP32_IR, ff_precision=ff.FF_BF16X6,
                                                        fmg_cycles=3, inner_cycles=3))[0]
    ff.mg_rhs_plane_wave(h, w.eta, None)
    u = torch.empty(w.shape, dtype=torch.complex128, device="cuda")
    ih = ff.mg_solve(h, None, u, tol=1e-6)
    assert ih.status == 0 and ih.rel_residual <= 1e-6
    Fh = ff.farfield_map(h, w.eta, u, w.dirs)
    h.destroy()
    del u
    torch.cuda.empty_cache()
    print(f"512^3 at tol 1e-6: {ih.cycles} refinement steps, residual {ih.rel_residual:.2e}; sampled map vs the "
          f"converged map {relerr(Fh[idx], Fs):.2e}")
    assert relerr(Fh[idx], Fs) < 1e-6


def test_schrodinger_batch_full(ff, orc):
    insts = W.schrodinger_batch(seed=3)
    hs, cache = [], {}
    for w in insts:
        key = (w.energy, w.n)
        if key not in cache:
            o = ff.default_options(precision=ff.FP32_IR, ff_precision=ff.FF_BF16X6)
            cache[key] = ff.setup_workload(w, options=o)[0]
        hs.append(cache[key])
    us = [torch.empty(w.shape, dtype=torch.complex128, device="cuda") for w in insts]
    infos = ff.mg_solve_batched(hs, [w.eta for w in insts], us)
    dirs = insts[0].dirs
    Fb = ff.farfield_map_batched(hs, [w.eta for w in insts], us, dirs)
    assert all(i.status == 0 and i.rel_residual <= 1e-10 for i in infos)
    # two sampled instances of every grid size
    rng = np.random.default_rng(11)
    picks = []
    for n in (256, 512, 1024):
        ids = [i for i, w in enumerate(insts) if w.n == n]
        picks += list(rng.choice(ids, min(2, len(ids)), replace=False))
    Fos = {}
    for i in picks:
        w = insts[i]
        b = ff.mg_rhs_plane_wave(hs[i], w.eta, torch.empty(w.shape, dtype=torch.complex128, device="cuda"))
        u = torch.zeros_like(b)
        info = ff.mg_solve(hs[i], b, u, tol=w.tol)
        assert torch.equal(u, us[i]), i
        assert info.cycles == infos[i].cycles and info.rel_residual == infos[i].rel_residual
        F1 = ff.farfield_map(hs[i], w.eta, u, dirs)
        np.testing.assert_array_equal(Fb[i], F1)
        g, kappa, q, k0, bo, ug = check_solution(orc, w, b, u, info, w.tol)
        Fo = orc.farfield(g, w.gamma, k0, q, w.eta, ug, dirs)
        assert relerr(F1, Fo) < 1e-6, (i, relerr(F1, Fo))
        Fos[i] = Fo
    for h in cache.values():
        h.destroy()
    # the benchmark's form: F(2) start, three FP32 V-cycles per refinement
    # step, residual reduction 1e-6; sampled instances equal single solves of
    # that form bit for bit and their maps lie within 1e-6 of the maps above
    hs, cache = [], {}
    for w in insts:
        key = (w.energy, w.n)
        if key not in cache:
            o = ff.default_options(precision=ff.FP32_IR, ff_precision=ff.FF_BF16X6, fmg_cycles=2, inner_cycles=3)
            cache[key] = ff.setup_workload(w, options=o)[0]
        hs.append(cache[key])
    infos = ff.mg_solve_batched(hs, [w.eta for w in insts], us, tol=1e-6)
    Fb = ff.farfield_map_batched(hs, [w.eta for w in insts], us, dirs)
    assert all(i.status == 0 and i.rel_residual <= 1e-6 for i in infos)
    for i in picks:
        w = insts[i]
        ff.mg_rhs_plane_wave(hs[i], w.eta, None)
        u = torch.empty(w.shape, dtype=torch.complex128, device="cuda")
        info = ff.mg_solve(hs[i], None, u, tol=1e-6)
        assert torch.equal(u, us[i]), i
        assert info.cycles == infos[i].cycles and info.rel_residual == infos[i].rel_residual
        assert relerr(Fb[i], Fos[i]) < 1e-6, (i, relerr(Fb[i], Fos[i]))
    for h in cache.values():
        h.destroy()


def test_learned_step_1023_sampled_points(ff, orc):
    """One learned smoothing step on the 1023^2 grid of the learned workload:
    the update at sampled points (corners, edges, interior) against the oracle
    network on the window of radius 6 around each point (the output depends on
    the residual within radius 3, the window keeps the grid's zero padding
    where it reaches the boundary)."""
    from oracle import convnet as cn
    from paper_1211_4461_amd import learned as LS
    w = W.random_field(1024, 4, 0.5)
    Ws = [Wl.astype(np.complex64).astype(np.complex128) for Wl in LS.jacobi_init(3, noise=0.5)]
    h = ff.setup_workload(w, options=ff.default_options(smoother=ff.SMOOTH_LEARNED, smoother_weights=Ws))[0]
    g = orc.Grid(2, w.n, w.lo, w.hi)
    kappa, q, k0 = orc.problem(w.kind, w.k0, w.energy, w.coef)
    b = LS.phase_rhs(w, torch)
    rng = np.random.default_rng(12)
    u0 = (rng.standard_normal(g.shape) + 1j * rng.standard_normal(g.shape)) * 0.1
    ud = torch.from_numpy(u0).cuda()
    ff.mg_learned_smooth(h, b, ud)
    upd = ud.cpu().numpy() - u0
    r = orc.residual(g, w.gamma, kappa, b.cpu().numpy(), u0)
    hh = (w.hi - w.lo) / w.n
    kh2 = kappa * hh * hh
    m = g.shape[0]
    pts = [(0, 0), (0, m - 1), (m - 1, 0), (m - 1, m - 1), (0, 500), (m - 1, 17), (3, 3), (511, 511)]
    pts += [tuple(int(v) for v in rng.integers(0, m, 2)) for _ in range(24)]
    R = 6
    errs = []
    for (y, x) in pts:
        y0, y1, x0, x1 = max(y - R, 0), min(y + R + 1, m), max(x - R, 0), min(x + R + 1, m)
        # the window is cut only at the grid boundary, so the oracle's zero
        # padding at its edges is the grid's Dirichlet boundary there and at
        # distance >= R > 3 elsewhere
        ref = cn.smooth_step(Ws, r[y0:y1, x0:x1], kh2[y0:y1, x0:x1], hh * hh, quant=True)
        # smooth_step scales by the window's RMS; N is linear in r, so the
        # scale cancels
        errs.append(abs(upd[y, x] - ref[y - y0, x - x0]) / (np.max(np.abs(ref)) + 1e-300))
    h.destroy()
    assert max(errs) < 1e-2, max(errs)
