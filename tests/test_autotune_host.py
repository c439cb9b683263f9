"""Host side of the timing autotuner and of the gridding split it tunes:
candidate shares, cache keys and files, the split's validation and its effect
on the device memory a context would hold (no GPU needed)."""
import json

import numpy as np
import pytest

import paper_1305_3162_amd as slp
from paper_1305_3162_amd import autotune as at
from synth.workloads import cube_random
from slp_testlib import es_for


def test_share_candidates_bracket_the_automatic_share():
    c = at.share_candidates(600, 147456)
    assert c == sorted(set(c)) and 600 in c and 147456 in c
    assert min(c) == 150 and 1200 in c
    # clamped to the valid range of slp_params.seg_share
    c = at.share_candidates(100, 50)
    assert min(c) == at.MIN_SHARE and all(at.MIN_SHARE <= s <= at.MAX_SHARE for s in c)
    assert max(at.share_candidates(1 << 24, 1 << 30)) == at.MAX_SHARE


def test_cache_key_separates_every_input():
    info = {"n_src": 3840, "tiles": [4, 4, 4], "n_targets": 642}
    base = at.cache_key(info, (64, 64, 64), 8, slp.WINDOW_GAUSS, slp.FP64, "dev")
    others = [at.cache_key(info, (64, 64, 64), 8, slp.WINDOW_KB, slp.FP64, "dev"),
              at.cache_key(info, (64, 64, 64), 8, slp.WINDOW_GAUSS, slp.FP32, "dev"),
              at.cache_key(info, (64, 64, 64), 7, slp.WINDOW_GAUSS, slp.FP64, "dev"),
              at.cache_key(info, (64, 64, 128), 8, slp.WINDOW_GAUSS, slp.FP64, "dev"),
              at.cache_key(info, (64, 64, 64), 8, slp.WINDOW_GAUSS, slp.FP64, "dev2"),
              at.cache_key(dict(info, n_src=3841), (64, 64, 64), 8, slp.WINDOW_GAUSS, slp.FP64, "dev"),
              at.cache_key(dict(info, tiles=[4, 4, 5]), (64, 64, 64), 8, slp.WINDOW_GAUSS, slp.FP64, "dev"),
              at.cache_key(dict(info, n_targets=1), (64, 64, 64), 8, slp.WINDOW_GAUSS, slp.FP64, "dev")]
    assert len(set(others + [base])) == len(others) + 1


def test_cache_file_round_trip(tmp_path):
    p = tmp_path / "tune.json"
    assert at.load_cache(str(p)) == {}
    at.store_cache(str(p), {"k": {"seg_share": 300, "us": 1.5}})
    assert at.load_cache(str(p)) == {"k": {"seg_share": 300, "us": 1.5}}
    assert list(tmp_path.iterdir()) == [p]          # no temporary left behind
    p.write_text(json.dumps([1, 2]))
    with pytest.raises(ValueError):
        at.load_cache(str(p))
    at.store_cache(None, {"k": 1})                 # no path: nothing written


def test_seg_share_validation_and_device_bytes():
    wl = cube_random(16, 2, 64, 4)
    w, g = es_for(wl)
    args = (wl.nodes, wl.tris, wl.grid, 4, w, g, wl.alpha, slp.FP64)
    auto = slp.geometry_device_bytes(*args)
    # one piece per tile whatever the share once it exceeds every tile's sources
    assert slp.geometry_device_bytes(*args, seg_share=1 << 24) == slp.geometry_device_bytes(
        *args, seg_share=1 << 20)
    # the smallest share cuts tiles into more pieces, each with its own block
    assert slp.geometry_device_bytes(*args, seg_share=64) > auto
    for bad in (1, 63, (1 << 24) + 1, -5):
        with pytest.raises(slp.SlpError, match="seg_share"):
            slp.geometry_device_bytes(*args, seg_share=bad)


def test_reduce_cells_validation():
    """The block-sum form (slp_params.reduce_cells): 0 automatic, 1 or 2 cells
    per thread; it changes no buffer, so the device bytes are the same."""
    wl = cube_random(16, 2, 64, 4)
    w, g = es_for(wl)
    args = (wl.nodes, wl.tris, wl.grid, 4, w, g, wl.alpha, slp.FP64)
    auto = slp.geometry_device_bytes(*args)
    for cells in (1, 2):
        assert slp.geometry_device_bytes(*args, reduce_cells=cells) == auto
    for bad in (-1, 3, 4):
        with pytest.raises(slp.SlpError, match="reduce_cells"):
            slp.geometry_device_bytes(*args, reduce_cells=bad)
