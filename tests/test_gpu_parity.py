"""GPU parity of the HIP library (through the C ABI) against the FP64 oracle.

Bars: kernel-level results agree to a few ulps (relative 1e-13); iterates
after the same number of V-cycles to 1e-12 (the iteration is contractive, so
rounding differences of the two implementations do not grow); converged far
fields to 1e-10 (FP64) and the stated mixed-precision bars.
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


def setup(ff, orc, w, **opt):
    o = ff.default_options(**opt)
    h, coef = ff.setup_workload(w, options=o)
    g = orc.Grid(w.dim, w.n, w.lo, w.hi)
    kappa, q, k0 = orc.problem(w.kind, w.k0, w.energy, w.coef)
    return h, coef, g, kappa, q, k0


CASES = [
    ("2d-63", lambda: W.small_2d(n=64)),
    ("2d-127-ragged", lambda: W.bumps_2d(n=128, seed=5, k0=1.3, M=40)),
    ("3d-15", lambda: W.radial_3d(16, L=4.0, n_az=6, n_pol=4)),
    ("3d-31", lambda: W.radial_3d(32, L=6.0, n_az=8, n_pol=5)),
]


@pytest.mark.parametrize("name,mk", CASES)
def test_apply_and_sweep_match_oracle(ff, orc, name, mk):
    w = mk()
    h, coef, g, kappa, q, k0 = setup(ff, orc, w)
    u = crand(1, g.shape)
    b = crand(2, g.shape)
    Au = ff.mg_apply(h, dev(u), torch.empty(g.shape, dtype=torch.complex128, device="cuda"))
    ref = orc.apply_A(g, w.gamma, kappa)(u)
    assert rel(host(Au), ref) < 1e-13
    uo = ff.mg_smooth(h, dev(b), dev(u), torch.empty(g.shape, dtype=torch.complex128, device="cuda"))
    ref = orc.jacobi(g, w.gamma, kappa, b, u, 0.8)
    assert rel(host(uo), ref) < 1e-13
    rn = ff.mg_residual_norm(h, dev(b), dev(u))
    assert abs(rn - np.linalg.norm(orc.residual(g, w.gamma, kappa, b, u))) <= 1e-12 * rn


@pytest.mark.parametrize("name,mk", CASES)
def test_rhs_matches_oracle(ff, orc, name, mk):
    w = mk()
    h, coef, g, kappa, q, k0 = setup(ff, orc, w)
    b = ff.mg_rhs_plane_wave(h, w.eta, torch.empty(g.shape, dtype=torch.complex128, device="cuda"))
    ref = orc.rhs_plane_wave(g, w.gamma, k0, q, w.eta)
    assert rel(host(b), ref) < 1e-13


@pytest.mark.parametrize("name,mk", CASES)
def test_vcycle_iterates_match_oracle(ff, orc, name, mk):
    """The same number of V(2,2) cycles from u = 0 on both sides."""
    w = mk()
    h, coef, g, kappa, q, k0 = setup(ff, orc, w)
    mg = orc.Multigrid(g, w.gamma, kappa)
    b = orc.rhs_plane_wave(g, w.gamma, k0, q, w.eta)
    assert h.num_levels() == mg.nlev
    ud = torch.zeros(g.shape, dtype=torch.complex128, device="cuda")
    bd = dev(b)
    uo = np.zeros(g.shape, dtype=np.complex128)
    for k in range(4):
        ff.mg_vcycle(h, bd, ud)
        uo = mg.vcycle(b, uo)
        assert rel(host(ud), uo) < 1e-12, f"cycle {k + 1}"


@pytest.mark.parametrize("name,mk", CASES)
def test_solve_and_far_field_match_oracle(ff, orc, name, mk):
    w = mk()
    h, coef, g, kappa, q, k0 = setup(ff, orc, w)
    mg = orc.Multigrid(g, w.gamma, kappa)
    b = orc.rhs_plane_wave(g, w.gamma, k0, q, w.eta)
    uo, st, k, hist = mg.solve(b, tol=1e-10)
    assert st == 0
    ud = torch.zeros(g.shape, dtype=torch.complex128, device="cuda")
    info = ff.mg_solve(h, dev(b), ud, tol=1e-10)
    assert info.status == 0 and info.cycles == k
    assert info.rel_residual <= 1e-10
    assert rel(host(ud), uo) < 1e-12
    Fo = orc.farfield(g, w.gamma, k0, q, w.eta, uo, w.dirs)
    Fg = ff.farfield_map(h, w.eta, ud, w.dirs)
    assert rel(Fg, Fo) < 1e-10
    # device output buffer gives the same numbers
    Fd = torch.empty(len(w.dirs), dtype=torch.complex128, device="cuda")
    ff.farfield_map(h, w.eta, ud, w.dirs, out=Fd)
    np.testing.assert_array_equal(host(Fd), Fg)


@pytest.mark.parametrize("dim", [2, 3])
def test_far_field_contraction_random_field(ff, orc, dim):
    """The MFMA contraction alone, on a random u and a ragged direction set."""
    w = W.bumps_2d(n=64, seed=3, k0=1.7, M=37) if dim == 2 else W.radial_3d(16, L=3.0, k0=1.2, n_az=7, n_pol=3)
    h, coef, g, kappa, q, k0 = setup(ff, orc, w)
    u = crand(7, g.shape) * 0.1
    Fo = orc.farfield(g, w.gamma, k0, q, w.eta, u, w.dirs, method="dense")
    Fg = ff.farfield_map(h, w.eta, dev(u), w.dirs)
    assert rel(Fg, Fo) < 1e-12


def test_far_field_born_closed_form(ff, orc):
    """GPU Born term (u = 0) against the Gaussian's Fourier transform."""
    from tests import refs
    w = W.radial_2d(256, L=10.0, k0=2.0, amp=0.5, width=1.0)
    h, coef, g, kappa, q, k0 = setup(ff, orc, w)
    Fg = ff.farfield_map(h, w.eta, None, w.dirs)
    ref = refs.born_2d(2.0, 0.5, 1.0, w.dirs, w.eta)
    assert rel(Fg, ref) < 1e-13


def test_zero_contrast(ff, orc):
    w = W.small_2d()
    w.coef = np.zeros_like(w.coef)
    h, coef, g, kappa, q, k0 = setup(ff, orc, w)
    b = ff.mg_rhs_plane_wave(h, w.eta, torch.empty(g.shape, dtype=torch.complex128, device="cuda"))
    assert torch.count_nonzero(b).item() == 0
    u = torch.ones(g.shape, dtype=torch.complex128, device="cuda")
    info = ff.mg_solve(h, b, u)
    assert info.cycles == 0 and torch.count_nonzero(u).item() == 0
    F = ff.farfield_map(h, w.eta, u, w.dirs)
    assert np.all(F == 0)


def test_reciprocity_on_gpu(ff, orc):
    w = W.bumps_2d(n=128, seed=11, k0=1.5, M=8)
    h, coef, g, kappa, q, k0 = setup(ff, orc, w)

    def F_of(e, a):
        b = ff.mg_rhs_plane_wave(h, e, torch.empty(g.shape, dtype=torch.complex128, device="cuda"))
        u = torch.zeros_like(b)
        ff.mg_solve(h, b, u, tol=1e-14)
        return ff.farfield_map(h, e, u, a[None, :])[0]

    eta, alpha = np.array([1.0, 0.0]), np.array([0.0, 1.0])
    f1, f2 = F_of(eta, alpha), F_of(-alpha, -eta)
    assert abs(f1 - f2) <= 1e-11 * abs(f1)


@pytest.mark.parametrize("name,mk", CASES[:3])
def test_mixed_precision_solve(ff, orc, name, mk):
    """FP32 V-cycles inside FP64 refinement reach the FP64 tolerance; the far
    field matches the oracle's converged one to 1e-8."""
    w = mk()
    h, coef, g, kappa, q, k0 = setup(ff, orc, w, precision=ff.FP32_IR)
    mg = orc.Multigrid(g, w.gamma, kappa)
    b = orc.rhs_plane_wave(g, w.gamma, k0, q, w.eta)
    uo, st, k, hist = mg.solve(b, tol=1e-13)
    ud = torch.zeros(g.shape, dtype=torch.complex128, device="cuda")
    info = ff.mg_solve(h, dev(b), ud, tol=1e-10)
    assert info.status == 0 and info.rel_residual <= 1e-10
    assert info.cycles <= k + 3
    assert rel(host(ud), uo) < 1e-8
    Fo = orc.farfield(g, w.gamma, k0, q, w.eta, uo, w.dirs)
    Fg = ff.farfield_map(h, w.eta, ud, w.dirs)
    assert rel(Fg, Fo) < 1e-8


def test_schrodinger_instance(ff, orc):
    n, E = 128, 1.0
    V = W.schrodinger_potential(n)
    w = W.Workload("s", 2, n, -10.0, 10.0, math.pi / 6, W.SCHRODINGER, math.sqrt(2 * E), E, V,
                   np.array([0.6, 0.8]), W.directions_2d(24))
    h, coef, g, kappa, q, k0 = setup(ff, orc, w)
    mg = orc.Multigrid(g, w.gamma, kappa)
    b = orc.rhs_plane_wave(g, w.gamma, k0, q, w.eta)
    bd = ff.mg_rhs_plane_wave(h, w.eta, torch.empty(g.shape, dtype=torch.complex128, device="cuda"))
    assert rel(host(bd), b) < 1e-13
    uo, st, k, _ = mg.solve(b, tol=1e-10)
    ud = torch.zeros_like(bd)
    info = ff.mg_solve(h, bd, ud, tol=1e-10)
    assert st == 0 and info.cycles == k
    Fo = orc.farfield(g, w.gamma, k0, q, w.eta, uo, w.dirs)
    assert rel(ff.farfield_map(h, w.eta, ud, w.dirs), Fo) < 1e-10


def test_deep_wells_diverge_on_both_sides(ff, orc):
    """Bound states below -E break the plain V-cycle (Sec. 5.4): the oracle
    and the library both report no convergence."""
    n, E = 128, 1.0
    V = W.schrodinger_potential(n, deep=True)
    w = W.Workload("s", 2, n, -10.0, 10.0, math.pi / 6, W.SCHRODINGER, math.sqrt(2 * E), E, V,
                   np.array([0.6, 0.8]), W.directions_2d(4))
    h, coef, g, kappa, q, k0 = setup(ff, orc, w)
    b = orc.rhs_plane_wave(g, w.gamma, k0, q, w.eta)
    uo, st, k, _ = orc.Multigrid(g, w.gamma, kappa).solve(b, tol=1e-10)
    ud = torch.zeros(g.shape, dtype=torch.complex128, device="cuda")
    info = ff.mg_solve(h, dev(b), ud, tol=1e-10, raise_on_noconv=False)
    assert st == orc.ENOCONV and info.status == ff.FFMG_ENOCONV and info.cycles == k


def test_errors(ff, orc):
    w = W.small_2d()
    coef = dev(w.coef)
    with pytest.raises(ff.FfmgError) as e:
        ff.mg_setup(2, [60, 64], -5, 5, w.gamma, coef, k0=2.0)
    assert e.value.status == ff.FFMG_EINVAL
    with pytest.raises(ff.FfmgError) as e:
        ff.mg_setup(2, 64, -5, 5, 0.0, coef, k0=2.0)
    assert e.value.status == ff.FFMG_EINVAL
    bad = w.coef.copy()
    bad[3, 7] = np.nan
    with pytest.raises(ff.FfmgError) as e:
        ff.mg_setup(2, 64, -5, 5, w.gamma, dev(bad), k0=2.0)
    assert e.value.status == ff.FFMG_ENAN
    h = ff.mg_setup(2, 64, -500, 500, w.gamma, coef, k0=5.0)
    with pytest.raises(ff.FfmgError) as e:
        ff.mg_rhs_plane_wave(h, w.eta, torch.empty((63, 63), dtype=torch.complex128, device="cuda"))
    assert e.value.status == ff.FFMG_ERANGE
    h2 = ff.mg_setup(2, 64, -5, 5, w.gamma, coef, k0=2.0)
    with pytest.raises(ff.FfmgError) as e:
        ff.farfield_map(h2, w.eta, None, np.array([[1.0, 1.0]]))
    assert e.value.status == ff.FFMG_EINVAL


def test_no_convergence_reported(ff, orc):
    """A tiny cycle budget ends in ENOCONV with the iterate left in u."""
    w = W.small_2d()
    h, coef, g, kappa, q, k0 = setup(ff, orc, w, max_cycles=2)
    b = ff.mg_rhs_plane_wave(h, w.eta, torch.empty(g.shape, dtype=torch.complex128, device="cuda"))
    u = torch.zeros_like(b)
    info = ff.mg_solve(h, b, u, raise_on_noconv=False)
    assert info.status == ff.FFMG_ENOCONV and info.cycles == 2
    assert torch.count_nonzero(u).item() > 0


@pytest.mark.parametrize("n", [64, 128, 256])
def test_fused_2d_path_is_bitwise_identical(ff, orc, n):
    """The fused 2D level kernels (two sweeps per launch, interpolation fused
    into post-smoothing, residual fused with restriction, fused refinement
    step) perform the same per-point arithmetic as the one-operation kernels:
    iterates agree bit for bit, for FP64 V-cycles and FP32-in-FP64 solves,
    on grids with ragged tiles."""
    w = W.bumps_2d(n=n, seed=n, k0=1.1, M=8)
    hf, coef, g, kappa, q, k0 = setup(ff, orc, w)
    hr, _, _, _, _, _ = setup(ff, orc, w, tile_config=1)
    b = ff.mg_rhs_plane_wave(hf, w.eta, torch.empty(g.shape, dtype=torch.complex128, device="cuda"))
    uf, ur = torch.zeros_like(b), torch.zeros_like(b)
    for _ in range(3):
        ff.mg_vcycle(hf, b, uf)
        ff.mg_vcycle(hr, b, ur)
    torch.cuda.synchronize()
    assert torch.equal(uf, ur)
    for nu1, nu2 in [(1, 1), (3, 0), (0, 3), (0, 2), (0, 1), (2, 0)]:
        hf2, _, _, _, _, _ = setup(ff, orc, w, nu1=nu1, nu2=nu2)
        hr2, _, _, _, _, _ = setup(ff, orc, w, nu1=nu1, nu2=nu2, tile_config=1)
        uf, ur = torch.zeros_like(b), torch.zeros_like(b)
        for _ in range(2):
            ff.mg_vcycle(hf2, b, uf)
            ff.mg_vcycle(hr2, b, ur)
        torch.cuda.synchronize()
        assert torch.equal(uf, ur), (nu1, nu2)
    for tc in (0, 2):   # fused with and without the one-workgroup LDS tail
        hf3, _, _, _, _, _ = setup(ff, orc, w, precision=ff.FP32_IR, tile_config=tc)
        hr3, _, _, _, _, _ = setup(ff, orc, w, precision=ff.FP32_IR, tile_config=1)
        uf, ur = torch.zeros_like(b), torch.zeros_like(b)
        i1 = ff.mg_solve(hf3, b, uf)
        i2 = ff.mg_solve(hr3, b, ur)
        assert i1.cycles == i2.cycles and i1.rel_residual == i2.rel_residual, tc
        assert torch.equal(uf, ur), tc
        hf4, _, _, _, _, _ = setup(ff, orc, w, tile_config=tc)
        uf, ur = torch.zeros_like(b), torch.zeros_like(b)
        for _ in range(2):
            ff.mg_vcycle(hf4, b, uf)
            ff.mg_vcycle(hr, b, ur) if tc == 0 else None
        if tc == 0:
            torch.cuda.synchronize()
            ur2 = torch.zeros_like(b)
            for _ in range(2):
                ff.mg_vcycle(hr, b, ur2)
            torch.cuda.synchronize()
            assert torch.equal(uf, ur2)


@pytest.mark.parametrize("n", [32, 64, 128])
def test_fused_3d_path_is_bitwise_identical(ff, orc, n):
    """The fused 3D sweeps (two sweeps from a zero guess in one pass; two
    sweeps from a nonzero guess in one pass with the first sweep's planes in
    LDS with any of three tile shapes, or one pass per sweep; the
    interpolation formed inside the first post-smoothing pass; the FP32
    pre-smoothing pair, residual and full weighting in one pass) and the
    one-pass FP64 refinement step (update +
    residual, iterate ping-ponged between two buffers) perform the per-point
    arithmetic of the one-operation kernels: iterates agree bit for bit with
    the reference path, for FP64 V-cycles with several (nu1, nu2) and for
    FP32-in-FP64 solves from u = 0 and from the full multigrid start (odd and
    even step counts), on grids with ragged x, y and z tiles."""
    w = W.radial_3d(n, L=5.0, k0=1.3, n_az=4, n_pol=3)
    for nu1, nu2 in [(2, 2), (1, 1), (3, 1), (0, 2), (0, 1), (0, 3), (2, 0), (4, 3)]:
        hr, _, g, _, _, _ = setup(ff, orc, w, nu1=nu1, nu2=nu2, tile_config=1)
        b = ff.mg_rhs_plane_wave(hr, w.eta, torch.empty(g.shape, dtype=torch.complex128, device="cuda"))
        ur = torch.zeros_like(b)
        for _ in range(2):
            ff.mg_vcycle(hr, b, ur)
        for v in range(5):
            hf, _, _, _, _, _ = setup(ff, orc, w, nu1=nu1, nu2=nu2)
            assert ff.mg_tune_variants(hf, ff.TUNE_SWEEP3D) == 5
            ff.mg_tune_set(hf, v, ff.TUNE_SWEEP3D)
            uf = torch.zeros_like(b)
            for _ in range(2):
                ff.mg_vcycle(hf, b, uf)
            torch.cuda.synchronize()
            assert torch.equal(uf, ur), (nu1, nu2, v)
    for fk in (0, 1, 2):
        hr, _, _, _, _, _ = setup(ff, orc, w, precision=ff.FP32_IR, tile_config=1, fmg_cycles=fk)
        ur = torch.zeros_like(b)
        i2 = ff.mg_solve(hr, b, ur)
        for v in range(5):
            hf, _, _, _, _, _ = setup(ff, orc, w, precision=ff.FP32_IR, fmg_cycles=fk)
            ff.mg_tune_set(hf, v, ff.TUNE_SWEEP3D)
            for rep in range(2):          # the second solve starts from the other buffer when the count is odd
                uf = torch.zeros_like(b)
                i1 = ff.mg_solve(hf, b, uf)
                assert i1.cycles == i2.cycles and i1.rel_residual == i2.rel_residual, (fk, v, rep)
                assert torch.equal(uf, ur), (fk, v, rep)


def test_fused_3d_path_on_an_anisotropic_grid(ff):
    """Every 3D kernel variant on a grid of 63 x 31 x 31 interior points (x
    over two ragged tiles, y and z over one; a 15 x 7 x 7 coarsest level): FP64
    V-cycles and FP32-in-FP64 solves (the default variant: the pre-smoothing
    pair, residual and restriction in one pass) equal the reference kernels'
    bit for bit."""
    n = [64, 32, 32]
    shape = (n[2] - 1, n[1] - 1, n[0] - 1)
    z = [np.linspace(-4.0, 4.0, m + 1)[1:-1] for m in n]
    Z, Y, X = np.meshgrid(z[2], z[1], z[0], indexing="ij")
    coef = torch.from_numpy(0.6 * np.exp(-(X * X + Y * Y + Z * Z) / 3.0) + 0.0j).cuda()

    def handle(**opt):
        return ff.mg_setup(3, n, [-4.0] * 3, [4.0] * 3, math.pi / 6, coef, k0=1.1,
                           options=ff.default_options(**opt))

    eta = [0.6, 0.0, 0.8]
    hr = handle(tile_config=1)
    b = ff.mg_rhs_plane_wave(hr, eta, torch.empty(shape, dtype=torch.complex128, device="cuda"))
    ur = torch.zeros_like(b)
    for _ in range(2):
        ff.mg_vcycle(hr, b, ur)
    for v in range(5):
        hf = handle()
        ff.mg_tune_set(hf, v, ff.TUNE_SWEEP3D)
        uf = torch.zeros_like(b)
        for _ in range(2):
            ff.mg_vcycle(hf, b, uf)
        torch.cuda.synchronize()
        assert torch.equal(uf, ur), v
        hf.destroy()
    hr.destroy()
    hr = handle(tile_config=1, precision=ff.FP32_IR, fmg_cycles=2)
    ur = torch.zeros_like(b)
    ir = ff.mg_solve(hr, b, ur, tol=1e-9)
    hf = handle(precision=ff.FP32_IR, fmg_cycles=2)
    assert ff.mg_tune_get(hf, ff.TUNE_SWEEP3D) == 4
    for v in (4, 3, 0):
        ff.mg_tune_set(hf, v, ff.TUNE_SWEEP3D)
        uf = torch.zeros_like(b)
        i1 = ff.mg_solve(hf, b, uf, tol=1e-9)
        torch.cuda.synchronize()
        assert ir.status == 0 and i1.cycles == ir.cycles and i1.rel_residual == ir.rel_residual, v
        assert torch.equal(uf, ur), v
    hf.destroy()
    hr.destroy()


@pytest.mark.parametrize("n", [256, 512])
def test_tail_variants_are_bitwise_identical_and_tuned(ff, orc, n, tmp_path):
    """The LDS tail runs the per-point arithmetic of the grid-wide kernels, so
    every tail size gives the same iterates bit for bit (FP64 V-cycles and
    FP32-in-FP64 solves); the solve-timing sweep selects one of them and the
    cached choice is applied to a second handle; a batch built before a tail
    change is rebuilt and still equals the single solve."""
    from paper_1211_4461_amd import autotune
    w = W.bumps_2d(n=n, seed=n + 1, k0=1.2, M=8)
    h64, _, g, _, _, _ = setup(ff, orc, w)
    nv = ff.mg_tune_variants(h64, ff.TUNE_TAIL)
    assert nv == 3
    b = ff.mg_rhs_plane_wave(h64, w.eta, torch.empty(g.shape, dtype=torch.complex128, device="cuda"))
    ref = None
    for v in range(nv):
        ff.mg_tune_set(h64, v, ff.TUNE_TAIL)
        assert ff.mg_tune_get(h64, ff.TUNE_TAIL) == v
        u = torch.zeros_like(b)
        for _ in range(3):
            ff.mg_vcycle(h64, b, u)
        torch.cuda.synchronize()
        if ref is None:
            ref = u.clone()
        assert torch.equal(u, ref), v
    h32, _, _, _, _, _ = setup(ff, orc, w, precision=ff.FP32_IR)
    sols = []
    for v in range(nv):
        ff.mg_tune_set(h32, v, ff.TUNE_TAIL)
        u = torch.zeros_like(b)
        info = ff.mg_solve(h32, b, u)
        sols.append((info.cycles, info.rel_residual, u))
    for c, r, u in sols[1:]:
        assert c == sols[0][0] and r == sols[0][1] and torch.equal(u, sols[0][2])
    ub = [torch.zeros_like(b)]
    ff.mg_solve_batched([h32], [w.eta], ub)
    assert torch.equal(ub[0], sols[0][2])
    ws = torch.zeros_like(b)
    best, times = ff.mg_tune_solve(h32, b, ws, tol=1e-10, reps=1)
    assert 0 <= best < nv and len(times) == nv and times[best] == min(times)
    assert ff.mg_tune_get(h32, ff.TUNE_TAIL) == best
    assert torch.equal(ws, sols[0][2])
    ub = [torch.zeros_like(b)]
    ff.mg_solve_batched([h32], [w.eta], ub)
    assert torch.equal(ub[0], sols[0][2])
    cache = str(tmp_path / "tune.json")
    v1 = autotune.tune_solve(h32, b, ws, ff.FP32_IR, path=cache, reps=1)
    h2, _, _, _, _, _ = setup(ff, orc, w, precision=ff.FP32_IR)
    assert autotune.tune_solve(h2, b, ws, ff.FP32_IR, path=cache) == v1
    assert ff.mg_tune_get(h2, ff.TUNE_TAIL) == v1
    with pytest.raises(ff.FfmgError):
        ff.mg_tune_set(h2, nv, ff.TUNE_TAIL)
    h3, _, _, _, _, _ = setup(ff, orc, w, tile_config=1)
    assert ff.mg_tune_variants(h3, ff.TUNE_TAIL) == 1
    assert ff.mg_tune_variants(h3, ff.TUNE_SMOOTH) == 1


@pytest.mark.parametrize("n", [128, 512])
def test_smoothing_tile_variants_are_bitwise_identical_and_tuned(ff, orc, n, tmp_path):
    """Every tile height of the fused smoothing kernel (8, 16, 4 rows), on the
    finest level and on the coarser ones (two tunables), does the same
    per-point arithmetic: FP64 V-cycles and FP32-in-FP64 solves agree bit for
    bit (ragged last tiles included); the solve-timing sweep selects one and
    the cache applies it to a second handle."""
    from paper_1211_4461_amd import autotune
    w = W.bumps_2d(n=n, seed=n + 3, k0=1.1, M=8)
    for prec in (ff.FP64, ff.FP32_IR):
        h, _, g, _, _, _ = setup(ff, orc, w, precision=prec)
        nv = ff.mg_tune_variants(h, ff.TUNE_SMOOTH)
        assert nv == 3 and ff.mg_tune_variants(h, ff.TUNE_SMOOTH_COARSE) == 3
        b = ff.mg_rhs_plane_wave(h, w.eta, torch.empty(g.shape, dtype=torch.complex128, device="cuda"))
        ref = None
        for v, vc in ((0, 0), (1, 1), (2, 2), (0, 2), (2, 1)):
            ff.mg_tune_set(h, v, ff.TUNE_SMOOTH)
            ff.mg_tune_set(h, vc, ff.TUNE_SMOOTH_COARSE)
            assert ff.mg_tune_get(h, ff.TUNE_SMOOTH) == v and ff.mg_tune_get(h, ff.TUNE_SMOOTH_COARSE) == vc
            u = torch.zeros_like(b)
            if prec == ff.FP64:
                for _ in range(3):
                    ff.mg_vcycle(h, b, u)
                key = None
            else:
                info = ff.mg_solve(h, b, u)
                key = (info.cycles, info.rel_residual)
            torch.cuda.synchronize()
            if ref is None:
                ref = (key, u.clone())
            assert key == ref[0] and torch.equal(u, ref[1]), (prec, v, vc)
    ws = torch.zeros_like(b)
    best, times = ff.mg_tune_solve(h, b, ws, reps=1, tunable=ff.TUNE_SMOOTH_COARSE)
    assert 0 <= best < 3 and times[best] == min(times) and ff.mg_tune_get(h, ff.TUNE_SMOOTH_COARSE) == best
    assert torch.equal(ws, ref[1])
    best, times = ff.mg_tune_solve(h, b, ws, reps=1, tunable=ff.TUNE_SMOOTH)
    assert 0 <= best < 3 and times[best] == min(times) and ff.mg_tune_get(h, ff.TUNE_SMOOTH) == best
    assert torch.equal(ws, ref[1])
    cache = str(tmp_path / "tune.json")
    v1 = autotune.tune_solve(h, b, ws, ff.FP32_IR, path=cache, reps=1, tunable=ff.TUNE_SMOOTH)
    h2, _, _, _, _, _ = setup(ff, orc, w, precision=ff.FP32_IR)
    assert autotune.tune_solve(h2, b, ws, ff.FP32_IR, path=cache, tunable=ff.TUNE_SMOOTH) == v1
    assert ff.mg_tune_get(h2, ff.TUNE_SMOOTH) == v1


@pytest.mark.parametrize("n", [64, 128, 512])
def test_pre_pass_variants_are_bitwise_identical_and_tuned(ff, orc, n, tmp_path):
    """The one-pass pre-smoothing (two sweeps, residual, full weighting; 16-
    or 8-row tiles on the finest level, FP32 and FP64) and the two launches it replaces agree
    bit for bit: FP64 V-cycles from zero and
    from a nonzero guess, FP32-in-FP64 solves and the full multigrid start
    (ragged last tiles and the grid border included); the solve-timing sweep
    selects one and the cache applies it to a second handle."""
    from paper_1211_4461_amd import autotune
    w = W.bumps_2d(n=n, seed=n + 7, k0=1.2, M=8)
    for prec in (ff.FP64, ff.FP32_IR):
        h, _, g, _, _, _ = setup(ff, orc, w, precision=prec)
        assert ff.mg_tune_variants(h, ff.TUNE_PRE) == 3
        assert ff.mg_tune_get(h, ff.TUNE_PRE) == 0
        b = ff.mg_rhs_plane_wave(h, w.eta, torch.empty(g.shape, dtype=torch.complex128, device="cuda"))
        u0 = dev(0.3 * crand(n, g.shape))
        outs = []
        for v in (0, 1, 2):
            ff.mg_tune_set(h, v, ff.TUNE_PRE)
            if prec == ff.FP64:
                u = torch.zeros_like(b)
                for _ in range(2):
                    ff.mg_vcycle(h, b, u)
                u2 = u0.clone()
                ff.mg_vcycle(h, b, u2)
                key = None
            else:
                u = torch.zeros_like(b)
                info = ff.mg_solve(h, b, u)
                key = (info.cycles, info.rel_residual)
                u2 = torch.empty_like(b)
                ff.mg_fmg(h, b, u2, 2)
            torch.cuda.synchronize()
            outs.append((key, u.clone(), u2.clone()))
        for o in outs[1:]:
            assert o[0] == outs[0][0]
            assert torch.equal(o[1], outs[0][1]) and torch.equal(o[2], outs[0][2]), prec
    ws = torch.zeros_like(b)
    best, times = ff.mg_tune_solve(h, b, ws, reps=1, tunable=ff.TUNE_PRE)
    assert best in (0, 1, 2) and times[best] == min(times) and ff.mg_tune_get(h, ff.TUNE_PRE) == best
    assert torch.equal(ws, outs[0][1])
    cache = str(tmp_path / "tune.json")
    v1 = autotune.tune_solve(h, b, ws, ff.FP32_IR, path=cache, reps=1, tunable=ff.TUNE_PRE)
    h2, _, _, _, _, _ = setup(ff, orc, w, precision=ff.FP32_IR)
    assert autotune.tune_solve(h2, b, ws, ff.FP32_IR, path=cache, tunable=ff.TUNE_PRE) == v1
    assert ff.mg_tune_get(h2, ff.TUNE_PRE) == v1
    h3, _, _, _, _, _ = setup(ff, orc, w, tile_config=1)
    assert ff.mg_tune_variants(h3, ff.TUNE_PRE) == 1


def test_repeated_solves_and_batches(ff, orc):
    """The device-side stopping test with batched enqueueing: repeated solves
    (whose batch size follows the previous cycle count) and a solve from a
    converged guess give the oracle's cycle counts."""
    w = W.small_2d(n=128)
    h, coef, g, kappa, q, k0 = setup(ff, orc, w)
    mg = orc.Multigrid(g, w.gamma, kappa)
    b = orc.rhs_plane_wave(g, w.gamma, k0, q, w.eta)
    bd = dev(b)
    for tol in (1e-6, 1e-10, 1e-8, 1e-12):
        uo, st, k, _ = mg.solve(b, tol=tol)
        ud = torch.zeros_like(bd)
        info = ff.mg_solve(h, bd, ud, tol=tol)
        assert info.cycles == k, tol
        assert rel(host(ud), uo) < 1e-12
    # a converged guess: zero cycles, u unchanged
    before = ud.clone()
    info = ff.mg_solve(h, bd, ud, tol=1e-6)
    torch.cuda.synchronize()
    assert info.cycles == 0 and torch.equal(ud, before)
