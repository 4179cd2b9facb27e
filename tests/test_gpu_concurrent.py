"""Several handles driven from several host threads at once (each handle with
its own stream and workspace): every map equals, bit for bit, the same map
computed alone, and one of them matches the oracle's far field."""
import math
import threading

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


@pytest.mark.parametrize("prec,fmg", [(1, 2), (0, 0)])
def test_threads_match_sequential(ff, orc, prec, fmg):
    w = W.bumps_2d(n=256, seed=9, M=24)
    nt = 4
    etas = [np.array([math.cos(2 * math.pi * i / nt), math.sin(2 * math.pi * i / nt), 0.0]) for i in range(nt)]
    lanes = []
    for i in range(nt):
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            h, coef = ff.setup_workload(w, options=ff.default_options(precision=prec, fmg_cycles=fmg,
                                                                      ff_precision=ff.FF_BF16X6 if prec else 0))
            b = torch.empty(w.shape, dtype=torch.complex128, device="cuda")
            u = torch.zeros_like(b)
            F = torch.empty(len(w.dirs), dtype=torch.complex128, device="cuda")
        lanes.append([h, b, u, F, s, coef])

    def one_map(i):
        h, b, u, F, s, _ = lanes[i]
        ff.mg_rhs_plane_wave(h, etas[i], b)
        if not fmg:
            with torch.cuda.stream(s):
                u.zero_()
        info = ff.mg_solve(h, b, u, tol=1e-10)
        ff.farfield_map(h, etas[i], u, w.dirs, out=F)
        return info

    # alone, one after another
    ref = []
    for i in range(nt):
        info = one_map(i)
        torch.cuda.synchronize()
        ref.append((info.cycles, info.rel_residual, lanes[i][2].clone(), lanes[i][3].clone()))
    # all at once, three maps per thread
    infos = [None] * nt
    errors = []

    def worker(i):
        try:
            for _ in range(3):
                infos[i] = one_map(i)
        except Exception as e:
            errors.append(e)

    threads = [threading.Thread(target=worker, args=(i,)) for i in range(nt)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    torch.cuda.synchronize()
    assert not errors, errors
    for i in range(nt):
        assert infos[i].status == 0 and (infos[i].cycles, infos[i].rel_residual) == ref[i][:2], i
        assert torch.equal(lanes[i][2], ref[i][2]) and torch.equal(lanes[i][3], ref[i][3]), i
    # direction 1 against the oracle
    g = orc.Grid(2, w.n, w.lo, w.hi)
    kappa, q, k0 = orc.problem(w.kind, w.k0, w.energy, w.coef)
    bo = orc.rhs_plane_wave(g, w.gamma, k0, q, etas[1])
    uo, st, _, _ = orc.Multigrid(g, w.gamma, kappa).solve(bo, tol=1e-12)
    Fo = orc.farfield(g, w.gamma, k0, q, etas[1], uo, w.dirs)
    Fg = lanes[1][3].cpu().numpy()
    assert np.linalg.norm(Fg - Fo) / np.linalg.norm(Fo) < (1e-6 if prec else 1e-10)
    for ln in lanes:
        ln[0].destroy()
