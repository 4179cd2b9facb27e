"""Autotuning of kernel tile shapes, with a JSON cache.

The library exposes tunable kernel families (``mg_tune_variants``); every
variant of a family computes the same bits with a different tile shape, and
which one is fastest depends on the device and on the problem's shapes.  This
module keys a choice by (device architecture, tunable and its number of
variants, dimension, interior extents, number of directions, precision, the
solve options that change the timed work), runs the library's own timing
sweep (``mg_tune_farfield``, ``mg_tune_solve``) on a cache miss, and stores
the winner.

The cache is a flat JSON object ``{key: {"variant": v, "ms": [...]}}``; a
missing or unreadable file is an empty cache.
"""
from __future__ import annotations

import json
import os
from typing import Optional

from . import ffmg

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "ffmg", "autotune.json")


def cache_path() -> str:
    return os.environ.get("FFMG_TUNE_CACHE", DEFAULT_CACHE)


def load(path: Optional[str] = None) -> dict:
    try:
        with open(path or cache_path()) as f:
            c = json.load(f)
        return c if isinstance(c, dict) else {}
    except (OSError, ValueError):
        return {}


def save(cache: dict, path: Optional[str] = None) -> None:
    p = path or cache_path()
    os.makedirs(os.path.dirname(p) or ".", exist_ok=True)
    tmp = p + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, p)


# solve options that change what a tuning sweep times (the cycle, the start,
# the smoother and the kernel configuration)
KEY_OPTIONS = ("nu1", "nu2", "nu_coarse", "inner_cycles", "fmg_cycles", "smoother", "krylov_m", "tile_config",
               "ff_precision")


def key(arch: str, tunable: int, dim: int, shape, n_dirs: int, precision: int, n_variants: int = 0,
        options: Optional[dict] = None) -> str:
    """Cache key: device, tunable and its variant count (a family that gains
    a variant is tuned again), grid, directions, precision and the solve
    options that affect timing."""
    ext = "x".join(str(int(m)) for m in shape)
    opts = ",".join(f"{k}={int((options or {}).get(k, 0))}" for k in KEY_OPTIONS)
    return (f"{arch}|tunable={int(tunable)}|nv={int(n_variants)}|d={int(dim)}|m={ext}|M={int(n_dirs)}"
            f"|prec={int(precision)}|{opts}")


def device_arch() -> str:
    import torch
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return getattr(p, "gcnArchName", p.name).split(":")[0]


def tune_farfield(h: "ffmg.Handle", eta, u, dirs, ff_precision: int, path: Optional[str] = None,
                  reps: int = 5, force: bool = False) -> int:
    """Select the far-field GEMM variant for this handle: from the cache, or
    by timing every variant (then cached).  Returns the variant."""
    nv = ffmg.mg_tune_variants(h, ffmg.TUNE_FF_GEMM)
    if nv <= 1:
        return 0
    shape = [m for m in h.level_shape(0) if m > 1]
    k = key(device_arch(), ffmg.TUNE_FF_GEMM, len(shape), shape, len(dirs), ff_precision, nv,
            getattr(h, "options", None))
    cache = load(path)
    hit = cache.get(k)
    if not force and isinstance(hit, dict) and isinstance(hit.get("variant"), int) and 0 <= hit["variant"] < nv:
        ffmg.mg_tune_set(h, hit["variant"], ffmg.TUNE_FF_GEMM)
        return hit["variant"]
    best, times = ffmg.mg_tune_farfield(h, eta, u, dirs, reps=reps)
    cache[k] = {"variant": best, "ms": [round(t, 5) for t in times]}
    save(cache, path)
    return best


def tune_solve(h: "ffmg.Handle", b, u, precision: int, tol: float = 1e-10, path: Optional[str] = None,
               reps: int = 3, force: bool = False, tunable: int = None) -> int:
    """Select a variant of a solve-level tunable of the fused 2D cycle for
    this handle (the LDS-tail size by default, or the smoothing tile height):
    from the cache, or by timing whole solves per variant (then cached; u is
    overwritten).  Returns the variant."""
    tunable = ffmg.TUNE_TAIL if tunable is None else tunable
    nv = ffmg.mg_tune_variants(h, tunable)
    if nv <= 1:
        return 0
    shape = [m for m in h.level_shape(0) if m > 1]
    k = key(device_arch(), tunable, len(shape), shape, 0, precision, nv, getattr(h, "options", None))
    cache = load(path)
    hit = cache.get(k)
    if not force and isinstance(hit, dict) and isinstance(hit.get("variant"), int) and 0 <= hit["variant"] < nv:
        ffmg.mg_tune_set(h, hit["variant"], tunable)
        return hit["variant"]
    best, times = ffmg.mg_tune_solve(h, b, u, tol=tol, reps=reps, tunable=tunable)
    cache[k] = {"variant": best, "ms": [round(t, 4) for t in times]}
    save(cache, path)
    return best


def tune_batch(hs, etas, us, tol: float = 1e-6, path: Optional[str] = None, reps: int = 3,
               force: bool = False) -> int:
    """Select the tile heights of batched solves led by hs[0]
    (FFMG_TUNE_BATCH): from the cache, or by timing reps batched solves per
    variant after one untimed solve (then cached; us is overwritten).  The
    key holds the instances' grids and the number of instances.  Returns the
    variant."""
    import time
    import torch
    h0 = hs[0]
    nv = ffmg.mg_tune_variants(h0, ffmg.TUNE_BATCH)
    if nv <= 1:
        return 0
    shape = sorted(int(h.level_shape(0)[0]) for h in hs)
    k = key(device_arch(), ffmg.TUNE_BATCH, 2, shape, len(hs), ffmg.FP32_IR, nv, getattr(h0, "options", None))
    cache = load(path)
    hit = cache.get(k)
    if not force and isinstance(hit, dict) and isinstance(hit.get("variant"), int) and 0 <= hit["variant"] < nv:
        ffmg.mg_tune_set(h0, hit["variant"], ffmg.TUNE_BATCH)
        return hit["variant"]
    times = []
    for v in range(nv):
        ffmg.mg_tune_set(h0, v, ffmg.TUNE_BATCH)
        ffmg.mg_solve_batched(hs, etas, us, tol=tol)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            ffmg.mg_solve_batched(hs, etas, us, tol=tol)
        torch.cuda.synchronize()
        times.append(1e3 * (time.perf_counter() - t0) / reps)
    best = int(min(range(nv), key=lambda v: times[v]))
    ffmg.mg_tune_set(h0, best, ffmg.TUNE_BATCH)
    cache[k] = {"variant": best, "ms": [round(t, 4) for t in times]}
    save(cache, path)
    return best
