"""Host logic of the autotuning cache (no GPU)."""
import json

from paper_1211_4461_amd import autotune


def test_key_distinguishes_every_field():
    base = dict(arch="gfx950", tunable=0, dim=2, shape=(2047, 2047), n_dirs=360, precision=2)
    k0 = autotune.key(**base)
    for f, v in [("arch", "gfx942"), ("tunable", 1), ("dim", 3), ("shape", (2047, 1023)), ("n_dirs", 180),
                 ("precision", 1), ("n_variants", 3)]:
        assert autotune.key(**{**base, f: v}) != k0, f


def test_key_distinguishes_solve_options():
    """A family that gains a variant, and every option that changes the timed
    work (start, cycle, smoother, kernel configuration), gets its own entry."""
    opts = {k: 0 for k in autotune.KEY_OPTIONS}
    base = dict(arch="gfx950", tunable=3, dim=2, shape=(2047, 2047), n_dirs=0, precision=1, n_variants=2)
    k0 = autotune.key(**base, options=opts)
    assert autotune.key(**{**base, "n_variants": 3}, options=opts) != k0
    for f in autotune.KEY_OPTIONS:
        assert autotune.key(**base, options={**opts, f: 2}) != k0, f
    assert autotune.key(**base, options=None) == k0


def test_roundtrip_and_bad_files(tmp_path):
    p = str(tmp_path / "sub" / "c.json")
    assert autotune.load(p) == {}
    autotune.save({"a": {"variant": 2, "ms": [0.1]}}, p)
    assert autotune.load(p) == {"a": {"variant": 2, "ms": [0.1]}}
    with open(p, "w") as f:
        f.write("{not json")
    assert autotune.load(p) == {}
    with open(p, "w") as f:
        json.dump([1, 2], f)
    assert autotune.load(p) == {}


def test_env_override(tmp_path, monkeypatch):
    monkeypatch.setenv("FFMG_TUNE_CACHE", str(tmp_path / "x.json"))
    assert autotune.cache_path() == str(tmp_path / "x.json")
