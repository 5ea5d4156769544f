"""Autotune cache keys and lookups (host only)."""
import json

from paper_1705_09366_amd import Desc, FLAG_KAHAN, Tuning, autotune


def test_buckets_and_density_classes():
    assert [autotune._bucket(v) for v in (0.3, 1, 1.5, 2, 3, 4, 5, 8, 9, 50)] == [0, 0, 1, 1, 2, 2, 3, 3, 4, 6]
    d = Desc(gx=1024, gy=1024, gt=256, hs=10.0, ht=7.0)
    # 1e6 points covering pi 10^2 * 14 voxels each over 2^28 voxels: about 16 per voxel
    assert 15 < autotune.density(d, 1_000_000) < 18
    assert autotune.density_class(d, 1_000_000) == 2
    assert autotune.key(d, 1_000_000) == "gfx950/hs4/ht3/d2/g14/plain"
    dk = Desc(**{**d.__dict__, "flags": FLAG_KAHAN})
    assert autotune.key(dk, 1_000_000).endswith("/kahan")
    # domain units: the buckets use hs/sres, ht/tres
    d2 = Desc(gx=512, gy=512, gt=128, hs=20.0, ht=14.0, sres=2.0, tres=2.0)
    assert autotune.key(d2, 1_000_000).startswith("gfx950/hs4/ht3/")
    assert autotune.grid_class(Desc(gx=256, gy=256, gt=64, hs=1.0, ht=1.0)) == 11


def test_lookup_prefers_explicit_cache_and_caps_kahan(tmp_path):
    d = Desc(gx=256, gy=256, gt=64, hs=5.0, ht=4.0)
    k_plain = autotune.key(d, 20_000)
    dk = Desc(**{**d.__dict__, "flags": FLAG_KAHAN})
    k_kahan = autotune.key(dk, 20_000)
    path = tmp_path / "c.json"
    path.write_text(json.dumps({"version": 1, "arch": "gfx950", "entries": {
        k_plain: {"tuning": [64, 16, 8, 512]}, k_kahan: {"tuning": [64, 0, 0, 0]}}}))
    assert autotune.lookup(d, 20_000, str(path)) == Tuning(64, 16, 8, 512)
    assert autotune.lookup(dk, 20_000, str(path)) == Tuning(32, 0, 0, 0)
    other = tmp_path / "other.json"
    other.write_text(json.dumps({"version": 1, "arch": "gfx942", "entries": {
        k_plain: {"tuning": [16, 0, 0, 0]}}}))
    # another architecture's cache is ignored
    assert autotune.lookup(d, 20_000, str(other)) == autotune.lookup(d, 20_000, None)


def test_shipped_cache_is_well_formed():
    import os
    if not os.path.exists(autotune.SHIPPED_CACHE):
        return
    data = json.load(open(autotune.SHIPPED_CACHE))
    assert data["version"] == autotune.CACHE_VERSION and data["arch"] == autotune.ARCH
    for k, e in data["entries"].items():
        assert k.startswith("gfx950/hs")
        tt, cxy, ct, ss = e["tuning"]
        assert tt in (16, 32, 64) and (cxy == 0 or 4 <= cxy <= 256) and (ct == 0 or 4 <= ct <= 256)
        assert ss == 0 or 64 <= ss <= 65536
        if "/kahan" in k:
            assert tt <= 32
        assert k.count("/") == 5 or k.endswith("/fp32")


def test_resolve_prefers_own_key_then_nearest(tmp_path):
    import json
    from paper_1705_09366_amd import Desc, FLAG_KAHAN, autotune
    d = Desc(gx=1024, gy=1024, gt=256, hs=10.0, ht=7.0, flags=FLAG_KAHAN)
    k = autotune.key(d, 1_000_000)
    far = Desc(gx=1781, gy=3601, gt=2435, hs=30.0, ht=5.0, flags=FLAG_KAHAN)
    kf = autotune.key(far, 291_990_435)
    near_key = "gfx950/hs5/ht3/d5/g16/kahan"  # distance 0.5 from kf
    other = "gfx950/hs5/ht3/d5/g17/plain"     # same place, other mode: never used
    cache = {"version": autotune.CACHE_VERSION, "arch": "gfx950", "entries": {
        k: {"tuning": [32, 24, 8, 0]},
        near_key: {"tuning": [16, 16, 8, 512]},
        other: {"tuning": [64, 16, 8, 0]}}}
    path = tmp_path / "c.json"
    path.write_text(json.dumps(cache))
    t, src = autotune.resolve(d, 1_000_000, str(path))
    assert (t.tile_t, t.cell_xy, t.cell_t) == (32, 24, 8) and src == f"autotune {k}"
    t, src = autotune.resolve(far, 291_990_435, str(path))
    assert (t.tile_t, t.cell_xy, t.cell_t, t.split_share) == (16, 16, 8, 512) and near_key in src
    # the same answer every time
    assert autotune.resolve(far, 291_990_435, str(path))[1] == src
    # nothing within reach: the library default
    tiny = Desc(gx=8, gy=8, gt=8, hs=1.0, ht=1.0, flags=FLAG_KAHAN)
    empty = tmp_path / "e.json"
    empty.write_text(json.dumps({**cache, "entries": {near_key: {"tuning": [16, 16, 8, 0]}}}))
    t, src = autotune.resolve(tiny, 10, str(empty), max_distance=0.0)
    assert t is None and src.startswith("default")


def test_operand_form_keys_are_separate(tmp_path):
    """Gathers with FP32 operands (asked for, per-point bandwidths) have keys
    of their own and never take the default form's entries, also through the
    nearest-entry search."""
    from paper_1705_09366_amd import FLAG_ADAPTIVE, kernel_flag
    d = Desc(gx=1024, gy=1024, gt=256, hs=10.0, ht=7.0, flags=FLAG_KAHAN)
    k = autotune.key(d, 1_000_000)
    assert k == "gfx950/hs4/ht3/d2/g14/kahan"
    assert autotune.key(d, 1_000_000, fp32=True) == k + "/fp32"
    dq = Desc(**{**d.__dict__, "flags": FLAG_KAHAN | FLAG_ADAPTIVE})
    assert autotune.key(dq, 1_000_000) == k + "/fp32"
    for fl in (kernel_flag(1), kernel_flag(3)):  # the other pairs have two-term operands too
        dq = Desc(**{**d.__dict__, "flags": FLAG_KAHAN | fl})
        assert autotune.key(dq, 1_000_000) == k
    # a grid class the shipped cache does not cover, so that only this cache answers
    big = Desc(gx=4096, gy=4096, gt=1024, hs=10.0, ht=7.0, flags=FLAG_KAHAN)
    kb = autotune.key(big, 4_000_000)
    kb_near_fp32 = autotune.key(big, 16_000_000, fp32=True)  # one density class away
    assert kb_near_fp32 != kb + "/fp32"
    path = tmp_path / "c.json"
    path.write_text(json.dumps({"version": 1, "arch": "gfx950", "entries": {
        kb: {"tuning": [32, 24, 8, 512]}, kb_near_fp32: {"tuning": [32, 16, 8, 0]}}}))
    t, src = autotune.resolve(big, 4_000_000, str(path))
    assert (t.tile_t, t.cell_xy, t.operand_form) == (32, 24, 0) and src.endswith(kb)
    t, src = autotune.resolve(big, 4_000_000, str(path), fp32=True)
    assert (t.cell_xy, t.operand_form) == (16, 1) and f"nearest {kb_near_fp32}" in src
    bq = Desc(**{**big.__dict__, "flags": FLAG_KAHAN | FLAG_ADAPTIVE})
    t, src = autotune.resolve(bq, 4_000_000, str(path))
    assert t.cell_xy == 16 and "/fp32" in src
    # an FP32-form cache alone never serves a default-form plan
    only = tmp_path / "o.json"
    only.write_text(json.dumps({"version": 1, "arch": "gfx950", "entries": {
        kb_near_fp32: {"tuning": [32, 16, 8, 0]}}}))
    t, src = autotune.resolve(big, 4_000_000, str(only))
    assert t is None or "/fp32" not in src


def test_tune_searches_rows_and_bins_together(monkeypatch):
    """The best (tile rows, bin edges) pair is found even where the best rows
    with default bins differ from the best rows overall."""
    d = Desc(gx=512, gy=512, gt=365, hs=50.0, ht=30.0, flags=FLAG_KAHAN)

    def fake_measure(points, desc, t, reps=5):
        if t.tile_t == 0:
            return 10.0
        if (t.tile_t, t.cell_xy, t.cell_t) == (16, 20, 8):
            return 7.0
        # 32-row tiles win with the default bins and with every other edge pair
        return {16: 9.0, 32: 8.0}[t.tile_t] + (0.5 if t.cell_xy else 0.0)

    monkeypatch.setattr(autotune, "measure", fake_measure)
    best, ms, table = autotune.tune(None, d)
    assert (best.tile_t, best.cell_xy, best.cell_t, best.split_share) == (16, 20, 8, 0)
    assert ms == 7.0
    # every pair was measured: both row counts with the default and each edge pair
    measured = {tuple(e[0][:3]) for e in table}
    assert (32, 0, 0) in measured and (16, 20, 8) in measured and (32, 20, 8) in measured
