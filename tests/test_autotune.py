"""Host logic of the autotuner (no GPU: the timing function is replaced)."""
import json

from paper_2104_07097_amd import autotune
from paper_2104_07097_amd import instances as inst


def test_shape_key_buckets():
    assert autotune.shape_key(100, 2000, 0, 1024) == "n128_m2048_e0_z1024"
    assert autotune.shape_key(500, 5500, 5, 4096) == "n512_m8192_e1_z4096"


def test_tune_picks_fastest_and_caches(tmp_path, monkeypatch):
    monkeypatch.setenv("MHAR_AUTOTUNE_CACHE", str(tmp_path / "cache.json"))
    fake = {("fp32", 25): 3.0, ("fp32", 50): 2.0, ("bf16x3", 50): 1.0}
    calls = []

    def timer(p, opts, steps=200, warmup=20):
        calls.append(opts)
        return fake[(opts["precision"], opts["recompute_every"])]

    monkeypatch.setattr(autotune, "time_options", timer)
    cands = [{"precision": p, "recompute_every": r, "steps_per_launch": 0} for p, r in fake]
    p = inst.randpoly(n=10, m=40, z=16, seed=1)
    best = autotune.tune(p, candidates=cands)
    assert best["precision"] == "bf16x3" and best["recompute_every"] == 50
    assert len(calls) == 3
    again = autotune.tune(p, candidates=cands)   # served from the cache
    assert again == best and len(calls) == 3
    data = json.load(open(tmp_path / "cache.json"))
    assert list(data) == [autotune.shape_key(10, 40, 0, 16)]


def test_tune_skips_paths_that_do_not_fit(tmp_path, monkeypatch):
    from paper_2104_07097_amd import mhar
    monkeypatch.setenv("MHAR_AUTOTUNE_CACHE", str(tmp_path / "cache.json"))

    def timer(p, opts, steps=200, warmup=20):
        if opts.get("path") == "resident":
            raise mhar.MharError(mhar.E_UNSUPPORTED, "does not fit")
        return 1.0 if opts.get("path") == "tiled" else 2.0

    monkeypatch.setattr(autotune, "time_options", timer)
    cands = [{"precision": "fp32", "recompute_every": 50, "steps_per_launch": 0, "path": q}
             for q in ("resident", "general", "tiled")]
    best = autotune.tune(inst.randpoly(n=10, m=40, z=16, seed=1), candidates=cands)
    assert best["path"] == "tiled"
