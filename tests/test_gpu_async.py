"""mg_solve_begin / mg_solve_end: a solve queued without waiting, finished
later.  Several solves in flight from one host thread (one handle and stream
each) give, bit for bit, the solutions, cycle counts and residuals of the
same solves run one at a time with mg_solve; one of them matches the oracle's
far field.  Edge cases: b = 0, a non-finite b, the cycle limit, and calls on
a handle with a pending solve."""
import math

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


def _lanes(ff, w, n, **opt):
    lanes = []
    for _ in range(n):
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            h, coef = ff.setup_workload(w, options=ff.default_options(**opt))
            b = torch.empty(w.shape, dtype=torch.complex128, device="cuda")
            u = torch.zeros_like(b)
        lanes.append([h, b, u, s, coef])
    return lanes


def _etas(n):
    return [np.array([math.cos(2 * math.pi * i / n), math.sin(2 * math.pi * i / n), 0.0]) for i in range(n)]


# (workload, options): FP32 refinement with the fused 2D kernels and the full
# multigrid start, the one-operation-per-launch kernels, plain FP64, 3D, and
# the GMRES(3) and red-black Gauss-Seidel smoothers
CASES = [
    ("2d-fp32-fmg", lambda: W.bumps_2d(n=256, seed=9, M=24), dict(precision=1, fmg_cycles=2)),
    ("2d-fp32-reference-tiles", lambda: W.bumps_2d(n=128, seed=9, M=24), dict(precision=1, tile_config=1)),
    ("2d-fp64", lambda: W.small_2d(n=128, M=24), dict(precision=0)),
    ("3d-fp32-fmg", lambda: W.gauss_3d(n=32, n_az=8, n_pol=4), dict(precision=1, fmg_cycles=2)),
    ("2d-gmres", lambda: W.small_2d(n=128, M=24), dict(precision=0, smoother=2, krylov_m=3, nu1=1, nu2=1)),
    ("2d-gmres-fp32-fmg", lambda: W.bumps_2d(n=256, seed=9, M=24),
     dict(precision=1, smoother=2, krylov_m=3, nu1=1, nu2=1, fmg_cycles=2)),
    ("2d-rbgs", lambda: W.small_2d(n=128, M=24), dict(precision=1, smoother=3, nu1=1, nu2=1)),
]


@pytest.mark.parametrize("name,wl,opt", CASES, ids=[c[0] for c in CASES])
def test_interleaved_solves_match_one_at_a_time(ff, name, wl, opt):
    w = wl()
    n = 3
    etas = _etas(n)
    lanes = _lanes(ff, w, n, **opt)
    # one at a time, with mg_solve
    ref = []
    for i, (h, b, u, s, _) in enumerate(lanes):
        ff.mg_rhs_plane_wave(h, etas[i], b)
        with torch.cuda.stream(s):
            u.zero_()
        info = ff.mg_solve(h, b, u, tol=1e-10)
        torch.cuda.synchronize()
        assert info.status == 0, (name, i)
        ref.append((info.cycles, info.vcycles, info.rel_residual, info.conv_factor, u.clone()))
    # all begun before any is finished, twice in a row (the second round
    # starts its first batch from the cycle count of the first)
    for rep in range(2):
        for i, (h, b, u, s, _) in enumerate(lanes):
            with torch.cuda.stream(s):
                u.zero_()
            ff.mg_solve_begin(h, b, u, tol=1e-10)
        infos = [ff.mg_solve_end(h) for (h, _, _, _, _) in lanes]
        torch.cuda.synchronize()
        for i, info in enumerate(infos):
            assert info.status == 0, (name, rep, i)
            assert (info.cycles, info.vcycles, info.rel_residual, info.conv_factor) == ref[i][:4], (name, rep, i)
            assert torch.equal(lanes[i][2], ref[i][4]), (name, rep, i)
    for ln in lanes:
        ln[0].destroy()


def test_pipelined_maps_match_oracle(ff, orc):
    """The bench's pattern: the next map is begun before the previous one is
    finished and its far field queued."""
    w = W.bumps_2d(n=256, seed=9, M=24)
    lanes = _lanes(ff, w, 2, precision=1, fmg_cycles=2, ff_precision=ff.FF_BF16X6)
    F = [torch.empty(len(w.dirs), dtype=torch.complex128, device="cuda") for _ in lanes]
    etas = _etas(4)
    outs = []
    pending = None
    for k in range(4):
        h, b, u, s, _ = lanes[k % 2]
        ff.mg_rhs_plane_wave(h, etas[k], b)
        ff.mg_solve_begin(h, b, u, tol=1e-10)
        if pending is not None:
            kp = pending
            hp, _, up, _, _ = lanes[kp % 2]
            assert ff.mg_solve_end(hp).status == 0
            ff.farfield_map(hp, etas[kp], up, w.dirs, out=F[kp % 2])
            torch.cuda.synchronize()
            outs.append((kp, F[kp % 2].cpu().numpy()))
        pending = k
    h, _, u, _, _ = lanes[pending % 2]
    assert ff.mg_solve_end(h).status == 0
    ff.farfield_map(h, etas[pending], u, w.dirs, out=F[pending % 2])
    torch.cuda.synchronize()
    outs.append((pending, F[pending % 2].cpu().numpy()))
    g = orc.Grid(2, w.n, w.lo, w.hi)
    kappa, q, k0 = orc.problem(w.kind, w.k0, w.energy, w.coef)
    for k, Fg in outs[1:3]:
        bo = orc.rhs_plane_wave(g, w.gamma, k0, q, etas[k])
        uo, st, _, _ = orc.Multigrid(g, w.gamma, kappa).solve(bo, tol=1e-12)
        Fo = orc.farfield(g, w.gamma, k0, q, etas[k], uo, w.dirs)
        assert np.linalg.norm(Fg - Fo) / np.linalg.norm(Fo) < 1e-6, k
    for ln in lanes:
        ln[0].destroy()


@pytest.mark.parametrize("prec,fmg", [(0, 0), (1, 0), (1, 2)])
def test_zero_and_nonfinite_rhs(ff, prec, fmg):
    w = W.small_2d(n=64, M=8)
    (h, b, u, s, _), = _lanes(ff, w, 1, precision=prec, fmg_cycles=fmg)
    with torch.cuda.stream(s):
        b.zero_()
        u.fill_(1.0 + 2.0j)
    ff.mg_solve_begin(h, b, u, tol=1e-10)
    info = ff.mg_solve_end(h)
    torch.cuda.synchronize()
    assert info.status == 0 and info.cycles == 0 and info.rel_residual == 0.0
    assert torch.count_nonzero(u).item() == 0
    # mg_solve takes the same path
    with torch.cuda.stream(s):
        u.fill_(1.0 + 2.0j)
    info = ff.mg_solve(h, b, u, tol=1e-10)
    torch.cuda.synchronize()
    assert info.status == 0 and info.cycles == 0 and torch.count_nonzero(u).item() == 0
    # a non-finite b
    ff.mg_rhs_plane_wave(h, [1.0, 0.0, 0.0], b)
    with torch.cuda.stream(s):
        b[3, 5] = complex(float("nan"), 0.0)
    ff.mg_solve_begin(h, b, u, tol=1e-10)
    with pytest.raises(ff.FfmgError) as e:
        ff.mg_solve_end(h)
    assert e.value.status == ff.FFMG_ENAN
    with pytest.raises(ff.FfmgError) as e:
        ff.mg_solve(h, b, u, tol=1e-10)
    assert e.value.status == ff.FFMG_ENAN
    # the handle still solves afterwards
    ff.mg_rhs_plane_wave(h, [1.0, 0.0, 0.0], b)
    with torch.cuda.stream(s):
        u.zero_()
    assert ff.mg_solve(h, b, u, tol=1e-10).status == 0
    h.destroy()


@pytest.mark.parametrize("max_cycles", [1, 5])
def test_cycle_limit_matches_mg_solve(ff, max_cycles):
    """max_cycles below the first batch (1) and above it (5, more batches)."""
    w = W.small_2d(n=128, M=8)
    (h, b, u, s, _), = _lanes(ff, w, 1, precision=1, max_cycles=max_cycles)
    ff.mg_rhs_plane_wave(h, [1.0, 0.0, 0.0], b)
    with torch.cuda.stream(s):
        u.zero_()
    ref = ff.mg_solve(h, b, u, tol=1e-14, raise_on_noconv=False)
    uref = u.clone()
    with torch.cuda.stream(s):
        u.zero_()
    ff.mg_solve_begin(h, b, u, tol=1e-14)
    info = ff.mg_solve_end(h, raise_on_noconv=False)
    torch.cuda.synchronize()
    assert ref.status == ff.FFMG_ENOCONV and info.status == ff.FFMG_ENOCONV
    assert info.cycles == ref.cycles == max_cycles
    assert info.rel_residual == ref.rel_residual and torch.equal(u, uref)
    h.destroy()


def test_pending_solve_guards(ff):
    w = W.small_2d(n=64, M=8)
    (h, b, u, s, _), = _lanes(ff, w, 1, precision=1)
    ff.mg_rhs_plane_wave(h, [1.0, 0.0, 0.0], b)
    with pytest.raises(ff.FfmgError) as e:
        ff.mg_solve_end(h)                      # nothing pending
    assert e.value.status == ff.FFMG_EINVAL
    with pytest.raises(ff.FfmgError) as e:
        ff.mg_solve_begin(h, b, u, tol=2.0)     # tol outside (0, 1)
    assert e.value.status == ff.FFMG_EINVAL
    ff.mg_solve_begin(h, b, u, tol=1e-10)
    t = torch.empty_like(u)
    for call in (lambda: ff.mg_solve_begin(h, b, u, tol=1e-10),
                 lambda: ff.mg_solve(h, b, u, tol=1e-10),
                 lambda: ff.mg_vcycle(h, b, t),
                 lambda: ff.mg_rhs_plane_wave(h, [1.0, 0.0, 0.0], t),
                 lambda: ff.farfield_map(h, [1.0, 0.0, 0.0], t, w.dirs)):
        with pytest.raises(ff.FfmgError) as e:
            call()
        assert e.value.status == ff.FFMG_EINVAL
    info = ff.mg_solve_end(h)                   # the pending solve is unharmed
    assert info.status == 0 and info.rel_residual <= 1e-10
    assert ff.mg_solve(h, b, u, tol=1e-10).status == 0
    h.destroy()


def test_start_buffer_parity_matches_a_fresh_handle(ff):
    """With the full multigrid start the first buffer of the FP32 ping-pong
    follows the previous solve's step count; a solve whose count differs from
    the previous one's (the iterate then ends in the work buffer and is
    copied) and one whose count agrees give the bits of a fresh handle."""
    w = W.bumps_2d(n=256, seed=9, M=8)
    opt = dict(precision=1, fmg_cycles=2)

    def fresh(tol):
        (h, b, u, s, _), = _lanes(ff, w, 1, **opt)
        ff.mg_rhs_plane_wave(h, w.eta, b)
        info = ff.mg_solve(h, b, u, tol=tol)
        torch.cuda.synchronize()
        out = (info.cycles, info.rel_residual, u.clone())
        h.destroy()
        return out

    ref, odd, even = {}, None, None
    for tol in (1e-10, 1e-9, 1e-8, 1e-7, 1e-6, 1e-5, 1e-4, 1e-11):
        r = fresh(tol)
        if r[0] % 2 == 1 and odd is None:
            odd, ref[tol] = tol, r
        elif r[0] % 2 == 0 and r[0] > 0 and even is None:
            even, ref[tol] = tol, r
        if odd is not None and even is not None:
            break
    assert odd is not None and even is not None, ref
    (h, b, u, s, _), = _lanes(ff, w, 1, **opt)
    ff.mg_rhs_plane_wave(h, w.eta, b)
    # (start flipped, count agrees): (no, -), (yes, yes), (yes, no), (no, no),
    # (yes, no), (no, yes)
    for tol in (odd, odd, even, odd, even, even):
        info = ff.mg_solve(h, b, u, tol=tol)
        torch.cuda.synchronize()
        c, rr, uref = ref[tol]
        assert (info.cycles, info.rel_residual) == (c, rr), tol
        assert torch.equal(u, uref), tol
    h.destroy()
