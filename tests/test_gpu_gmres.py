"""GPU parity of the GMRES(m) smoother (Sec. 3.3) against the FP64 oracle.

Bars: one smoothing step and V-cycle iterates to 1e-10 (the GPU builds the
Krylov basis by classical Gram-Schmidt with FP64 partial sums, the oracle by
modified Gram-Schmidt: equal in exact arithmetic); converged solves and far
fields as for weighted Jacobi (1e-10 FP64, the mixed bars for FP32_IR); at a
10-degree contour, where Jacobi V-cycles diverge on both sides, GMRES(3)
V(1,1) cycles converge on both sides in the same number of cycles.
"""
import math

import numpy as np
import pytest

from paper_1211_4461_amd import workloads as W
from tests.compare import rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ff():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1211_4461_amd import ffmg
    ffmg.lib()
    return ffmg


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()




def crand(seed, shape):
    r = np.random.default_rng(seed)
    return r.standard_normal(shape) + 1j * r.standard_normal(shape)


def at_angle(w, deg):
    """The workload on a contour of another rotation angle."""
    w.gamma = math.radians(deg)
    return w


CASES = [
    ("2d-63", lambda: W.small_2d(n=64)),
    ("2d-127-ragged", lambda: W.bumps_2d(n=128, seed=5, k0=1.3, M=40)),
    ("3d-31", lambda: W.radial_3d(32, L=6.0, n_az=8, n_pol=5)),
]


def problem(ff, orc, w, **opt):
    h, _ = ff.setup_workload(w, options=ff.default_options(smoother=ff.SMOOTH_GMRES, **opt))
    g = orc.Grid(w.dim, w.n, w.lo, w.hi)
    kappa, q, k0 = orc.problem(w.kind, w.k0, w.energy, w.coef)
    b = orc.rhs_plane_wave(g, w.gamma, k0, q, w.eta)
    return h, g, kappa, q, k0, b


@pytest.mark.parametrize("m", [2, 3])
@pytest.mark.parametrize("name,mk", CASES)
def test_gmres_step_matches_oracle(ff, orc, name, mk, m):
    w = mk()
    h, g, kappa, q, k0, b = problem(ff, orc, w, krylov_m=m)
    u0 = crand(3, g.shape)
    ud = dev(u0)
    ff.mg_gmres_smooth(h, dev(b), ud)
    ref = orc.gmres_step(g, w.gamma, kappa, b, u0, m)
    assert rel(host(ud) - u0, ref - u0) < 1e-10
    h.destroy()


@pytest.mark.parametrize("tile", [0, 1])
@pytest.mark.parametrize("name,mk", CASES)
def test_gmres_vcycle_iterates_match_oracle(ff, orc, name, mk, tile):
    w = mk()
    h, g, kappa, q, k0, b = problem(ff, orc, w, nu1=1, nu2=1, tile_config=tile)
    mg = orc.Multigrid(g, w.gamma, kappa, nu1=1, nu2=1, smoother="gmres", krylov_m=3)
    assert h.num_levels() == mg.nlev
    ud = torch.zeros(g.shape, dtype=torch.complex128, device="cuda")
    bd = dev(b)
    uo = np.zeros(g.shape, dtype=np.complex128)
    for k in range(3):
        ff.mg_vcycle(h, bd, ud)
        uo = mg.vcycle(b, uo)
        assert rel(host(ud), uo) < 1e-10, f"cycle {k + 1}"
    h.destroy()


BIG = [
    ("2d-255", lambda: at_angle(W.bumps_2d(n=256, seed=2, M=24), 10)),
    ("3d-63", lambda: W.radial_3d(64, L=6.0, n_az=8, n_pol=5)),
]


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("m", [1, 2, 3])
@pytest.mark.parametrize("name,mk", BIG, ids=[c[0] for c in BIG])
def test_fused_gmres_passes_equal_reference_passes(ff, orc, name, mk, m, prec):
    """The m + 3-launch GMRES(m) step (the orthogonalisation formed inside the
    next application of A, each pass summing the previous passes' partials
    itself) and the reference passes (4 m + 3 launches)
    give the same bits: two FP64 steps on the finest level, V-cycle iterates,
    and a solve (cycles, residual, iterate).  The levels above 4096 points
    take the multi-block passes, the smaller ones the one-workgroup step."""
    w = mk()
    hs = [problem(ff, orc, w, krylov_m=m, nu1=1, nu2=1, precision=prec, tile_config=t)[0] for t in (0, 1)]
    g = orc.Grid(w.dim, w.n, w.lo, w.hi)
    kappa, q, k0 = orc.problem(w.kind, w.k0, w.energy, w.coef)
    bd = dev(orc.rhs_plane_wave(g, w.gamma, k0, q, w.eta))
    u0 = dev(crand(5, g.shape))
    us = [u0.clone() for _ in hs]
    for h, u in zip(hs, us):
        ff.mg_gmres_smooth(h, bd, u)
        ff.mg_gmres_smooth(h, bd, u)
    torch.cuda.synchronize()
    assert torch.equal(us[0], us[1])
    vs = [torch.zeros_like(bd) for _ in hs]
    for k in range(2):
        for h, v in zip(hs, vs):
            ff.mg_vcycle(h, bd, v)
        torch.cuda.synchronize()
        assert torch.equal(vs[0], vs[1]), f"cycle {k + 1}"
    infos = []
    for h, v in zip(hs, vs):
        v.zero_()
        infos.append(ff.mg_solve(h, bd, v, tol=1e-9))
    torch.cuda.synchronize()
    assert infos[0].status == 0 and infos[0].cycles == infos[1].cycles
    assert infos[0].rel_residual == infos[1].rel_residual
    assert torch.equal(vs[0], vs[1])
    for h in hs:
        h.destroy()


@pytest.mark.parametrize("deg", [10, 30])
def test_gmres_solve_below_the_jacobi_angle(ff, orc, deg):
    """At 10 degrees Jacobi V(2,2) diverges (ENOCONV on both sides) and
    GMRES(3) V(1,1) converges, in FP64 and in FP32-in-FP64; far fields match
    the oracle's converged map."""
    w = at_angle(W.small_2d(n=128), deg)
    h, g, kappa, q, k0, b = problem(ff, orc, w, nu1=1, nu2=1)
    mg = orc.Multigrid(g, w.gamma, kappa, nu1=1, nu2=1, smoother="gmres", krylov_m=3)
    uo, st, k, _ = mg.solve(b, tol=1e-10, max_cycles=100)
    assert st == 0
    ud = torch.zeros(g.shape, dtype=torch.complex128, device="cuda")
    info = ff.mg_solve(h, dev(b), ud, tol=1e-10)
    assert info.status == 0 and info.cycles == k and info.rel_residual <= 1e-10
    assert rel(host(ud), uo) < 1e-10
    Fo = orc.farfield(g, w.gamma, k0, q, w.eta, uo, w.dirs)
    assert rel(ff.farfield_map(h, w.eta, ud, w.dirs), Fo) < 1e-9
    h.destroy()
    h32, *_ = problem(ff, orc, w, nu1=1, nu2=1, precision=ff.FP32_IR, ff_precision=ff.FF_BF16X6)
    u32 = torch.zeros_like(ud)
    info = ff.mg_solve(h32, dev(b), u32, tol=1e-10)
    assert info.status == 0 and info.rel_residual <= 1e-10
    assert rel(host(u32), uo) < 1e-8
    assert rel(ff.farfield_map(h32, w.eta, u32, w.dirs), Fo) < 1e-6
    h32.destroy()
    if deg == 10:
        hj, _ = ff.setup_workload(w, options=ff.default_options(max_cycles=60))
        uj = torch.zeros_like(ud)
        ij = ff.mg_solve(hj, dev(b), uj, tol=1e-10, raise_on_noconv=False)
        _, stj, _, _ = orc.Multigrid(g, w.gamma, kappa).solve(b, tol=1e-10, max_cycles=60)
        assert ij.status == ff.FFMG_ENOCONV and stj == orc.ENOCONV
        hj.destroy()


def test_gmres_fmg_start_matches_oracle(ff, orc):
    w = at_angle(W.bumps_2d(n=256, seed=2, M=24), 10)
    h, g, kappa, q, k0, b = problem(ff, orc, w, nu1=1, nu2=1)
    ud = torch.empty(g.shape, dtype=torch.complex128, device="cuda")
    ff.mg_fmg(h, dev(b), ud, 2)
    mg = orc.Multigrid(g, w.gamma, kappa, nu1=1, nu2=1, smoother="gmres", krylov_m=3)
    assert rel(host(ud), mg.fmg(b, 2)) < 1e-10
    h.destroy()


def test_gmres_errors(ff, orc):
    w = W.small_2d(n=64)
    h, _ = ff.setup_workload(w)
    b = torch.zeros((63, 63), dtype=torch.complex128, device="cuda")
    with pytest.raises(ff.FfmgError) as e:
        ff.mg_gmres_smooth(h, b, torch.zeros_like(b))
    assert e.value.status == ff.FFMG_EINVAL
    h.destroy()
    with pytest.raises(ff.FfmgError) as e:
        ff.setup_workload(w, options=ff.default_options(smoother=ff.SMOOTH_GMRES, krylov_m=9))
    assert e.value.status == ff.FFMG_EINVAL
    # a zero right-hand side and a zero guess stay zero
    h, _ = ff.setup_workload(w, options=ff.default_options(smoother=ff.SMOOTH_GMRES))
    u = torch.zeros_like(b)
    ff.mg_gmres_smooth(h, b, u)
    assert torch.count_nonzero(u).item() == 0
    h.destroy()


@pytest.mark.parametrize("E", [0.5, 1.0, 2.0])
def test_literal_batch_potential_with_gmres(ff, orc, E):
    """The batched Schroedinger workload's literal potential (V = -2 e^{-z.z}
    plus wells of depth U[0.5, 2]) holds bound states below -E, where the
    weighted-Jacobi V-cycle diverges (Sec. 5.4); GMRES(3) V(1,1) smoothing
    (Sec. 5.5) converges on it.  255^2 grid: FP64 solves in the oracle's
    cycle count, iterate and map to 1e-9; the mixed solve's map within 1e-6
    of the oracle's."""
    n = 256
    V = W.schrodinger_potential(n, seed=3, deep=True)
    w = W.Workload(f"literal_E{E}", 2, n, -10.0, 10.0, math.pi / 6, W.SCHRODINGER, math.sqrt(2 * E), E, V,
                   np.array([1.0, 0.0]), W.directions_2d(24), tol=1e-10, nu1=1, nu2=1)
    h, g, kappa, q, k0, b = problem(ff, orc, w, nu1=1, nu2=1, krylov_m=3)
    uo, st, k, _ = orc.Multigrid(g, w.gamma, kappa, nu1=1, nu2=1, smoother="gmres", krylov_m=3).solve(b, tol=1e-10)
    assert st == 0
    bd = dev(b)
    ud = torch.zeros_like(bd)
    info = ff.mg_solve(h, bd, ud, tol=1e-10)
    assert info.status == 0 and info.cycles == k, (info.cycles, k)
    assert rel(host(ud), uo) < 1e-9
    Fo = orc.farfield(g, w.gamma, k0, q, w.eta, uo, w.dirs)
    assert rel(ff.farfield_map(h, w.eta, ud, w.dirs), Fo) < 1e-9
    h.destroy()
    hm, _ = ff.setup_workload(w, options=ff.default_options(smoother=ff.SMOOTH_GMRES, nu1=1, nu2=1, krylov_m=3,
                                                           precision=ff.FP32_IR, ff_precision=ff.FF_BF16X6))
    um = torch.zeros_like(bd)
    im = ff.mg_solve(hm, bd, um, tol=1e-10)
    assert im.status == 0
    err = rel(ff.farfield_map(hm, w.eta, um, w.dirs), Fo)
    print(f"literal potential, E = {E}: GMRES(3) V(1,1) {k} cycles (oracle and GPU), mixed {im.cycles} steps, "
          f"map {err:.1e}")
    assert err < 1e-6
    hm.destroy()
