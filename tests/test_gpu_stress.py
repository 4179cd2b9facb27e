"""Full-size parity of the plain FP64 path and of the literal wavenumbers.

* 2048^2 bumps, plain FP64 (the benchmark's plain form: full multigrid start,
  fused kernels with every tuned tile variant): every variant bit for bit the
  same; the iterate against the oracle's nested iteration and V-cycles of
  the same count (element-wise 1e-12); the map against the oracle's map of
  its own solution converged to its FP64 residual floor (2e-12; 1e-10, norm-
  and element-wise).
* The stress points the workloads name, k0 h = 1/2: 2048^2 (k0 = 51.2) and
  512^3 (k0 = 21.33), solve only, with the bounded phase right-hand side
  q exp(i k0 cos(gamma) eta.x) (the contour plane wave leaves the double range
  there): the right-hand side against the oracle element by element, the
  residual of the mixed and of the plain solution under the oracle's
  operator, and the two solutions against each other.
"""
import numpy as np
import pytest

from paper_1211_4461_amd import workloads as W
from tests.compare import elementwise, rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ff():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1211_4461_amd import ffmg
    ffmg.lib()
    return ffmg


def residual_under_oracle(orc, g, w, kappa, b, u):
    r = orc.residual(g, w.gamma, kappa, b, u)
    return float(np.linalg.norm(r) / np.linalg.norm(b))


def test_bumps_2048_plain_fp64(ff, orc):
    w = W.bumps_2d()
    g = orc.Grid(2, w.n, w.lo, w.hi)
    kappa, q, k0 = orc.problem(w.kind, w.k0, w.energy, w.coef)
    h = ff.setup_workload(w, options=ff.default_options(fmg_cycles=2))[0]
    b = ff.mg_rhs_plane_wave(h, w.eta, torch.empty(w.shape, dtype=torch.complex128, device="cuda"))
    u = torch.empty_like(b)
    info = ff.mg_solve(h, b, u, tol=w.tol)
    assert info.status == 0
    F = ff.farfield_map(h, w.eta, u, w.dirs)
    u_ref = u.clone()
    # every variant of every tunable of the plain path: the same bits
    for tn in (ff.TUNE_SMOOTH, ff.TUNE_SMOOTH_COARSE, ff.TUNE_PRE, ff.TUNE_TAIL):
        v0 = ff.mg_tune_get(h, tn)
        for v in range(ff.mg_tune_variants(h, tn)):
            ff.mg_tune_set(h, v, tn)
            uv = torch.empty_like(b)
            iv = ff.mg_solve(h, b, uv, tol=w.tol)
            assert iv.cycles == info.cycles and torch.equal(uv, u_ref), (tn, v)
        ff.mg_tune_set(h, v0, tn)
    # iterate parity: the oracle's nested iteration and as many V-cycles
    bo = orc.rhs_plane_wave(g, w.gamma, k0, q, w.eta)
    assert elementwise(b.cpu().numpy(), bo) <= 1e-12
    mg = orc.Multigrid(g, w.gamma, kappa)
    u0 = mg.fmg(bo, 2)
    uo, st, k, _ = mg.solve(bo, u0=u0, tol=w.tol)
    assert st == 0 and k == info.cycles, (k, info.cycles)
    ug = u.cpu().numpy()
    err_it = rel(ug, uo)
    assert err_it <= 1e-12, err_it
    # converged parity of the map: the oracle's solution taken to its FP64
    # residual floor (about 1.4e-12 relative on 2047^2; 1e-13 is out of reach)
    uc, st, kc, _ = mg.solve(bo, u0=uo, tol=2e-12)
    assert st == 0
    Fo = orc.farfield(g, w.gamma, k0, q, w.eta, uc, w.dirs)
    print(f"2048^2 plain FP64: {info.cycles} cycles from the full multigrid start, iterate vs oracle {err_it:.2e}, "
          f"map vs oracle at 2e-12: {rel(F, Fo):.2e}")
    assert rel(F, Fo) <= 1e-10
    h.destroy()


@pytest.mark.parametrize("dim", [2, 3])
def test_stress_k0h_half(ff, orc, dim):
    w = W.bumps_2d(k0=None, M=8) if dim == 2 else W.gauss_3d(k0=None, n_az=4, n_pol=2)
    g = orc.Grid(dim, w.n, w.lo, w.hi)
    kappa, q, k0 = orc.problem(w.kind, w.k0, w.energy, w.coef)
    assert abs(k0 * g.h[0] - 0.5) < 1e-12
    sols = {}
    for name, prec in (("mixed", ff.FP32_IR), ("plain", ff.FP64)):
        h = ff.setup_workload(w, options=ff.default_options(precision=prec, fmg_cycles=2))[0]
        b = ff.mg_rhs_phase(h, w.eta, torch.empty(w.shape, dtype=torch.complex128, device="cuda"))
        u = torch.empty_like(b)
        info = ff.mg_solve(h, b, u, tol=w.tol)
        assert info.status == 0, name
        sols[name] = (info, u.cpu().numpy())
        if name == "mixed":
            bg = b.cpu().numpy()
        h.destroy()
        del b, u
        torch.cuda.empty_cache()
    bo = orc.rhs_phase(g, w.gamma, k0, q, w.eta)
    assert elementwise(bg, bo) <= 1e-12
    for name, (info, ug) in sols.items():
        rr = residual_under_oracle(orc, g, w, kappa, bo, ug)
        assert rr <= 1.01 * w.tol and abs(rr - info.rel_residual) <= 1e-2 * rr, (name, rr, info.rel_residual)
    d = rel(sols["mixed"][1], sols["plain"][1])
    print(f"{dim}D k0 h = 1/2 (k0 = {k0:.2f}): mixed {sols['mixed'][0].cycles} steps "
          f"({sols['mixed'][0].vcycles} V-cycles), plain {sols['plain'][0].cycles} V-cycles; "
          f"solutions differ by {d:.2e}")
    assert d <= 1e-7
