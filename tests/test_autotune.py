"""Host-side checks of the autotuner: the encoding of its choices into the library's
options, the parameters it explores per workload kind, and the cache round trip."""
import json

from paper_2605_25346_amd import autotune as A
from paper_2605_25346_amd import binding as B
from paper_2605_25346_amd.workloads import config_workload


def test_encoding_of_choices():
    cfg, fuse = A._encode(dict(bound_cap=3, dual_cap=2, reach_cap=1, bound_weights_global=1, bound_paired_tiles=1,
                               dual_no_cache=1, fuse_spec=0))
    assert cfg & 0xF == 3 and (cfg >> 8) & 0xF == 2 and (cfg >> 12) & 0xF == 1 and (cfg >> 4) & 0xF == 0
    assert cfg & B.DR_TILE_GLOBAL_WEIGHTS and cfg & B.DR_TILE_PAIRED_TILES and cfg & B.DR_TILE_NO_ITEM_CACHE
    assert fuse is False
    assert A._encode({}) == (0, True)


def test_parameters_per_workload_kind():
    names = lambda i: [n for n, _ in A._params(config_workload(i, n_sub=4))]
    assert names(2) == ["bound_cap", "bound_weights_global", "bound_paired_tiles", "fuse_spec"]   # 64-wide
    assert names(3) == ["bound_cap", "fuse_spec", "dual_cap", "dual_no_cache"]                     # 128-wide, ascent
    assert names(4) == ["reach_cap"]                                                                 # reach
    for i in (2, 3, 4):
        assert all(len(v) >= 2 for _, v in A._params(config_workload(i, n_sub=4)))


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "cache.json")
    wl = config_workload(2, n_sub=4)
    assert A.lookup(wl.nets, "f32", path) == (0, True)          # not tuned: defaults
    cfg, fuse = A._encode(dict(bound_cap=2, bound_paired_tiles=1, fuse_spec=0))
    with open(path, "w") as f:
        json.dump({A.key_of(wl.nets, "f32"): dict(tile_cfg=cfg, fuse_spec=fuse)}, f)
    assert A.lookup(wl.nets, "f32", path) == (cfg, False)
    assert A.lookup(wl.nets, "f64", path) == (0, True)          # keyed by precision
