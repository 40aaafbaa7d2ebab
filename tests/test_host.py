"""Host-side logic that needs no GPU: the tile-shape cache lookup and the bench helpers."""
import json

from paper_2407_19689_amd import autotune


def test_tiles_for_picks_the_nearest_tuned_bucket(tmp_path, monkeypatch):
    cache = {
        "gfx950/p1/points_euclid/5x5": {"vec": 1, "rows": 16},
        "gfx950/p1/points_euclid/11x11": {"vec": 4, "rows": 64},
        "gfx950/p0/points_euclid/11x11": {"vec": 2, "rows": 32},
    }
    f = tmp_path / "cache.json"
    f.write_text(json.dumps(cache))
    monkeypatch.setattr(autotune, "CACHE", str(f))
    monkeypatch.setattr(autotune, "_cache", None)
    assert autotune.tiles_for(40, 30, 1, "points_euclid") == (1, 16)
    assert autotune.tiles_for(2000, 1500, 1, "points_euclid") == (4, 64)
    assert autotune.tiles_for(2000, 1500, 0, "points_euclid") == (2, 32)
    # nothing tuned for this kind: (0, 0) selects the library's built-in shape
    assert autotune.tiles_for(2000, 1500, 1, "grid_sqeuclid") == (0, 0)
    # instances solved together: the widest lane n allows, the tuned rows
    assert autotune.tiles_for(2000, 1500, 0, "points_euclid", shared=True) == (4, 32)
    assert autotune.tiles_for(2000, 200, 0, "points_euclid", shared=True) == (2, 32)
    assert autotune.tiles_for(40, 30, 1, "points_euclid", shared=True) == (1, 16)
    assert autotune.tiles_for(2000, 1500, 1, "grid_sqeuclid", shared=True) == (4, 0)


def test_tiles_for_without_a_cache(tmp_path, monkeypatch):
    monkeypatch.setattr(autotune, "CACHE", str(tmp_path / "missing.json"))
    monkeypatch.setattr(autotune, "_cache", None)
    assert autotune.tiles_for(100, 100, 1, "points_sqeuclid") == (0, 0)


def test_committed_cache_holds_valid_shapes():
    cache = autotune.load_cache()
    for k, v in cache.items():
        assert k.startswith("gfx950/p")
        assert v["vec"] in (1, 2, 4) and v["rows"] >= 16 and v["rows"] % 16 == 0


def test_committed_cache_covers_every_kind_and_precision():
    """Both plan precisions and every cost kind the bench, batch and server use have tuned
    shapes (images: every size bucket of the tuner)."""
    cache = autotune.load_cache()
    for prec in (0, 1):
        for kind in autotune.KINDS:
            keys = [k for k in cache if k.startswith(f"gfx950/p{prec}/{kind}/")]
            assert keys, (prec, kind)
            if kind in autotune.GRID_KINDS:
                assert len(keys) == len(autotune.EXPS[kind])


def test_bucket():
    assert autotune.bucket(32, 2048) == (5, 11)
    assert autotune.bucket(1, 1) == (0, 0)


def test_synthetic_image_classes_are_distributions():
    """The stand-in image classes give nonnegative images summing to 1; the suite's costs
    are the raw pixel distances of Section 5.1."""
    import numpy as np
    from workloads import generators as gen
    for cls in gen.IMAGE_CLASSES:
        inst = gen.suite_pair(3, 8, cls, "l1")
        assert inst.m == inst.n == 64
        for w in (inst.f, inst.g):
            assert np.all(w > 0) and abs(w.sum() - 1.0) <= 1e-12
    a = gen.suite_pair(3, 4, "blobs", "l1").dense_cost()
    b = gen.suite_pair(3, 4, "blobs", "l2").dense_cost()
    c = gen.suite_pair(3, 4, "blobs", "linf").dense_cost()
    # pixels 0 = (0, 0) and 5 = (1, 1): distances 2, sqrt(2), 1
    assert a[0, 5] == 2.0 and b[0, 5] == np.sqrt(2.0) and c[0, 5] == 1.0
    assert a.max() == 6.0 and c.max() == 3.0
