"""Solves whose right-hand side is the handle's plane wave (b = NULL): the
same bits as solving for the stored right-hand side that mg_rhs_plane_wave
writes, on the path that never stores it (3D, FP32 V-cycles in FP64
refinement, fused kernels) and on the paths that store it once in the
handle (2D, FP64, the reference kernels).  The stored right-hand side itself
is compared with the oracle's exp(i k0 eta.z) in test_gpu_parity.py and
test_gpu_fullsize.py.
"""
import numpy as np
import pytest

from paper_1211_4461_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ff():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1211_4461_amd import ffmg
    ffmg.lib()
    return ffmg


def explicit_and_implicit(ff, h, w, eta, tol, begin=False):
    b = ff.mg_rhs_plane_wave(h, eta, torch.empty(w.shape, dtype=torch.complex128, device="cuda"))
    u1 = torch.zeros_like(b)
    i1 = ff.mg_solve(h, b, u1, tol=tol)
    ff.mg_rhs_plane_wave(h, eta, None)
    u2 = torch.zeros_like(b)
    if begin:
        ff.mg_solve_begin(h, None, u2, tol=tol)
        i2 = ff.mg_solve_end(h)
    else:
        i2 = ff.mg_solve(h, None, u2, tol=tol)
    torch.cuda.synchronize()
    return u1, i1, u2, i2


CASES = [
    ("3d-63-ir-fmg", lambda: W.gauss_3d(n=64, n_az=4, n_pol=2), dict(precision=1, fmg_cycles=1)),
    ("3d-63-ir-zero", lambda: W.gauss_3d(n=64, n_az=4, n_pol=2), dict(precision=1)),
    ("3d-127-ir-inner4", lambda: W.gauss_3d(n=128, n_az=4, n_pol=2), dict(precision=1, fmg_cycles=1,
                                                                            inner_cycles=4)),
    ("3d-31-fp64-fmg", lambda: W.radial_3d(32, L=6.0, n_az=8, n_pol=5), dict(precision=0, fmg_cycles=1)),
    ("3d-31-ir-reference", lambda: W.radial_3d(32, L=6.0, n_az=8, n_pol=5), dict(precision=1, tile_config=1)),
    ("2d-255-ir-fmg", lambda: W.bumps_2d(n=256, seed=2, M=24), dict(precision=1, fmg_cycles=1)),
    ("2d-127-fp64", lambda: W.bumps_2d(n=128, seed=5, k0=1.3, M=40), dict(precision=0)),
]


@pytest.mark.parametrize("name,mk,opt", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("begin", [False, True])
def test_plane_wave_solve_equals_stored_rhs(ff, name, mk, opt, begin):
    w = mk()
    h = ff.setup_workload(w, options=ff.default_options(**opt))[0]
    for eta in (w.eta, -np.asarray(w.eta)):
        u1, i1, u2, i2 = explicit_and_implicit(ff, h, w, eta, 1e-9, begin)
        assert i1.status == 0 and i2.status == 0
        assert i2.cycles == i1.cycles and i2.rel_residual == i1.rel_residual, (i1.cycles, i2.cycles)
        assert torch.equal(u1, u2)
    h.destroy()


def test_plane_wave_solve_needs_a_plane_wave(ff):
    w = W.gauss_3d(n=32, n_az=4, n_pol=2)
    h = ff.setup_workload(w, options=ff.default_options(precision=1))[0]
    u = torch.zeros(w.shape, dtype=torch.complex128, device="cuda")
    with pytest.raises(ff.FfmgError) as e:
        ff.mg_solve(h, None, u)
    assert e.value.status == ff.FFMG_EINVAL
    with pytest.raises(ff.FfmgError) as e:
        ff.mg_rhs_plane_wave(h, [float("nan"), 0.0, 0.0], None)
    assert e.value.status == ff.FFMG_EINVAL
    # a pending solve keeps its plane wave: a new one is refused until it ends
    ff.mg_rhs_plane_wave(h, w.eta, None)
    ff.mg_solve_begin(h, None, u, tol=1e-8)
    with pytest.raises(ff.FfmgError) as e:
        ff.mg_rhs_plane_wave(h, -np.asarray(w.eta), None)
    assert e.value.status == ff.FFMG_EINVAL
    assert ff.mg_solve_end(h).status == 0
    h.destroy()


def test_start_met_at_once_is_stored(ff):
    """The 3D FP32-in-FP64 solve forms its full multigrid start inside the
    first refinement pass instead of storing it; when the start already meets
    the tolerance no step runs and the start is stored at the end: u equals
    mg_fmg's start bit for bit, after an even and an odd previous step count
    (the start buffer alternates between u and the handle's other buffer)."""
    w = W.gauss_3d(n=64, n_az=4, n_pol=2)
    h = ff.setup_workload(w, options=ff.default_options(precision=1, fmg_cycles=2))[0]
    b = ff.mg_rhs_plane_wave(h, w.eta, torch.empty(w.shape, dtype=torch.complex128, device="cuda"))
    u0 = torch.empty_like(b)
    ff.mg_fmg(h, b, u0, 2)
    bn = float(torch.linalg.vector_norm(b).item())
    rel0 = ff.mg_residual_norm(h, b, u0) / bn
    assert 0 < rel0 < 0.99, rel0
    for prev_tol in (1e-3, 1e-6, 1e-9):   # previous solves with different step counts
        u = torch.zeros_like(b)
        ff.mg_solve(h, b, u, tol=prev_tol)
        u = torch.full_like(b, 3.0)
        info = ff.mg_solve(h, b, u, tol=min(0.999, 1.01 * rel0))
        torch.cuda.synchronize()
        assert info.status == 0 and info.cycles == 0, (prev_tol, info.cycles)
        assert torch.equal(u, u0), prev_tol
    h.destroy()
