"""Batched persistent solve (one launch per kernel for all instances, the
refinement step replayed as a HIP graph) against the single-instance solve
and the oracle.

Every instance of a batch must reproduce mg_solve on its handle bit for bit
(the batched kernels keep each instance's block structure and reduction
order); the single-instance solve is itself pinned to the oracle in
test_gpu_parity.py, and one instance per batch is checked against the oracle
here as well.
"""
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




def operators(ff, insts, **opt):
    """One handle per (energy, grid); returns (handles per instance, cache)."""
    cache = {}
    hs = []
    for w in insts:
        key = (w.energy, w.n)
        if key not in cache:
            o = ff.default_options(precision=ff.FP32_IR, **opt)
            cache[key] = ff.setup_workload(w, options=o)[0]
        hs.append(cache[key])
    return hs, cache


def single(ff, h, w, tol):
    b = ff.mg_rhs_plane_wave(h, w.eta, torch.empty(w.shape, dtype=torch.complex128, device="cuda"))
    u = torch.zeros_like(b)
    info = ff.mg_solve(h, b, u, tol=tol)
    return u, info


@pytest.mark.parametrize("sizes", [(128, 256), (256,), (128, 256, 512)])
def test_batch_equals_single_solves(ff, orc, sizes):
    insts = W.schrodinger_batch(seed=3, n_dirs=4, sizes=sizes, M=24)
    hs, cache = operators(ff, insts)
    us = [torch.full(w.shape, 7.0, dtype=torch.complex128, device="cuda") for w in insts]   # overwritten
    infos = ff.mg_solve_batched(hs, [w.eta for w in insts], us, tol=1e-10)
    for i, w in enumerate(insts):
        u1, i1 = single(ff, hs[i], w, 1e-10)
        torch.cuda.synchronize()
        assert infos[i].status == 0 and infos[i].cycles == i1.cycles, (i, infos[i].cycles, i1.cycles)
        assert infos[i].rel_residual == i1.rel_residual and infos[i].rel_residual <= 1e-10
        assert torch.equal(us[i], u1), i
    # one instance against the oracle's converged solution
    w = insts[-1]
    g = orc.Grid(2, w.n, w.lo, w.hi)
    kappa, q, k0 = orc.problem(w.kind, w.k0, w.energy, w.coef)
    b = orc.rhs_plane_wave(g, w.gamma, k0, q, w.eta)
    uo, st, k, _ = orc.Multigrid(g, w.gamma, kappa).solve(b, tol=1e-13)
    assert st == 0
    assert rel(us[-1].cpu().numpy(), uo) < 1e-8


@pytest.mark.parametrize("sizes,k", [((128, 256, 512), 1), ((256,), 2), ((128, 512), 1)])
def test_batch_fmg_start_equals_single_solves(ff, orc, sizes, k):
    """With the full multigrid start F(k) every instance of a batch (grids of
    different depths: the starts of all instances run level by level
    together) equals mg_solve with the same start bit for bit and converges
    to the solution of the batch from u = 0."""
    insts = W.schrodinger_batch(seed=4, n_dirs=3, sizes=sizes, M=24)
    hs, cache = operators(ff, insts, fmg_cycles=k)
    etas = [w.eta for w in insts]
    us = [torch.full(w.shape, 5.0, dtype=torch.complex128, device="cuda") for w in insts]   # overwritten
    infos = ff.mg_solve_batched(hs, etas, us, tol=1e-10)
    hz, cz = operators(ff, insts)
    uz = [torch.empty(w.shape, dtype=torch.complex128, device="cuda") for w in insts]
    iz = ff.mg_solve_batched(hz, etas, uz, tol=1e-10)
    for i, w in enumerate(insts):
        u1, i1 = single(ff, hs[i], w, 1e-10)
        torch.cuda.synchronize()
        assert infos[i].status == 0 and infos[i].cycles == i1.cycles, (i, infos[i].cycles, i1.cycles)
        assert infos[i].rel_residual == i1.rel_residual and infos[i].rel_residual <= 1e-10
        assert torch.equal(us[i], u1), i
        assert iz[i].status == 0 and rel(us[i].cpu().numpy(), uz[i].cpu().numpy()) < 1e-8
    for h in list(cache.values()) + list(cz.values()):
        h.destroy()


def test_batch_tile_variants_and_tuning(ff, orc, tmp_path):
    """Every FFMG_TUNE_BATCH variant (tile heights of the batched smoothing
    launches) gives the same bits (the batch is rebuilt when the variant
    changes); the autotuner times them, keeps one and applies the cached
    choice to another batch led by the same operator."""
    from paper_1211_4461_amd import autotune
    insts = W.schrodinger_batch(seed=3, n_dirs=4, sizes=(128, 256, 512), M=24)
    hs, cache = operators(ff, insts)
    etas = [w.eta for w in insts]
    nv = ff.mg_tune_variants(hs[0], ff.TUNE_BATCH)
    assert nv == 4
    ref = None
    for v in range(nv):
        ff.mg_tune_set(hs[0], v, ff.TUNE_BATCH)
        us = [torch.full(w.shape, 3.0, dtype=torch.complex128, device="cuda") for w in insts]
        infos = ff.mg_solve_batched(hs, etas, us, tol=1e-10)
        if ref is None:
            ref = ([u.clone() for u in us], [i.cycles for i in infos])
        else:
            assert [i.cycles for i in infos] == ref[1], v
            assert all(torch.equal(a, b) for a, b in zip(us, ref[0])), v
    path = str(tmp_path / "tune.json")
    us = [torch.empty(w.shape, dtype=torch.complex128, device="cuda") for w in insts]
    best = autotune.tune_batch(hs, etas, us, tol=1e-6, path=path, reps=2)
    assert 0 <= best < nv and ff.mg_tune_get(hs[0], ff.TUNE_BATCH) == best
    ff.mg_tune_set(hs[0], (best + 1) % nv, ff.TUNE_BATCH)
    assert autotune.tune_batch(hs, etas, us, tol=1e-6, path=path) == best
    assert ff.mg_tune_get(hs[0], ff.TUNE_BATCH) == best
    for h in cache.values():
        h.destroy()


def test_batch_reuse_and_far_fields(ff, orc):
    """A second call with new directions reuses the graph; batched far fields
    equal per-instance maps; a different handle list rebuilds the batch."""
    insts = W.schrodinger_batch(seed=5, n_dirs=3, sizes=(128, 256), M=30)
    hs, cache = operators(ff, insts, ff_precision=2)
    us = [torch.empty(w.shape, dtype=torch.complex128, device="cuda") for w in insts]
    etas = [w.eta for w in insts]
    ff.mg_solve_batched(hs, etas, us)
    etas2 = [-np.asarray(e) for e in etas]
    infos = ff.mg_solve_batched(hs, etas2, us)
    for i, w in enumerate(insts):
        u1, i1 = single(ff, hs[i], W.Workload(w.name, 2, w.n, w.lo, w.hi, w.gamma, w.kind, w.k0, w.energy, w.coef,
                                              etas2[i], w.dirs), 1e-10)
        torch.cuda.synchronize()
        assert infos[i].cycles == i1.cycles and torch.equal(us[i], u1)
    dirs = insts[0].dirs
    F = ff.farfield_map_batched(hs, etas2, us, dirs)
    for i in range(len(insts)):
        np.testing.assert_array_equal(F[i], ff.farfield_map(hs[i], etas2[i], us[i], dirs))
    Fd = torch.empty((len(insts), len(dirs)), dtype=torch.complex128, device="cuda")
    ff.farfield_map_batched(hs, etas2, us, dirs, out=Fd)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(Fd.cpu().numpy(), F)
    # the Born terms (u = None), and a second direction set (the batched
    # workspace is rebuilt for it), equal the per-instance maps too
    F0 = ff.farfield_map_batched(hs, etas2, None, dirs)
    for i in range(len(insts)):
        np.testing.assert_array_equal(F0[i], ff.farfield_map(hs[i], etas2[i], None, dirs))
    dirs2 = dirs[::3]
    F2 = ff.farfield_map_batched(hs, etas2, us, dirs2)
    for i in range(len(insts)):
        np.testing.assert_array_equal(F2[i], ff.farfield_map(hs[i], etas2[i], us[i], dirs2))
    # another direction set of the same size rebuilds every plan: the batched
    # workspace, which points into the plans, is rebuilt with them (also when
    # the plans were rebuilt in between by single maps of other directions)
    t3 = np.arctan2(dirs2[:, 1], dirs2[:, 0]) + 0.01
    dirs3 = np.stack([np.cos(t3), np.sin(t3)], axis=1)
    for D in (dirs3, dirs2):
        FB = ff.farfield_map_batched(hs, etas2, us, D)
        for i in range(len(insts)):
            np.testing.assert_array_equal(FB[i], ff.farfield_map(hs[i], etas2[i], us[i], D))
        for i in range(len(insts)):
            ff.farfield_map(hs[i], etas2[i], us[i], dirs)
    # a sub-list of the handles: rebuilt workspace, same answers
    sub = [0, 2, 4]
    us2 = [torch.empty_like(us[i]) for i in sub]
    ff.mg_solve_batched([hs[i] for i in sub], [etas2[i] for i in sub], us2)
    torch.cuda.synchronize()
    for j, i in enumerate(sub):
        assert torch.equal(us2[j], us[i])


def test_batch_reports_non_convergence(ff, orc):
    """An instance whose handle allows too few cycles ends in ENOCONV with its
    info filled; the others converge as alone."""
    insts = W.schrodinger_batch(seed=3, n_dirs=2, sizes=(128,), M=8)
    o_ok = ff.default_options(precision=ff.FP32_IR)
    o_short = ff.default_options(precision=ff.FP32_IR, max_cycles=2)
    h_ok = ff.setup_workload(insts[0], options=o_ok)[0]
    h_short = ff.setup_workload(insts[0], options=o_short)[0]
    hs = [h_ok, h_short]
    us = [torch.empty(insts[0].shape, dtype=torch.complex128, device="cuda") for _ in hs]
    infos = ff.mg_solve_batched(hs, [insts[0].eta, insts[1].eta], us, raise_on_noconv=False)
    assert infos[0].status == 0 and infos[1].status == ff.FFMG_ENOCONV and infos[1].cycles == 2
    with pytest.raises(ff.FfmgError) as e:
        ff.mg_solve_batched(hs, [insts[0].eta, insts[1].eta], us)
    assert e.value.status == ff.FFMG_ENOCONV


def test_batch_rejects_unsupported_handles(ff, orc):
    w = W.schrodinger_batch(seed=3, n_dirs=1, sizes=(128,), M=8)[0]
    h64 = ff.setup_workload(w, options=ff.default_options())[0]
    hir = ff.setup_workload(w, options=ff.default_options(precision=ff.FP32_IR))[0]
    hnu = ff.setup_workload(w, options=ff.default_options(precision=ff.FP32_IR, nu1=1, nu2=1))[0]
    hfmg = ff.setup_workload(w, options=ff.default_options(precision=ff.FP32_IR, fmg_cycles=1))[0]
    u = [torch.empty(w.shape, dtype=torch.complex128, device="cuda") for _ in range(2)]
    for hs in ([h64, hir], [hir, hnu], [hir, hfmg]):
        with pytest.raises(ff.FfmgError) as e:
            ff.mg_solve_batched(hs, [w.eta, w.eta], u)
        assert e.value.status == ff.FFMG_EINVAL
