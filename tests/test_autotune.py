"""Autotuner host logic: geometry keys, candidate sets and the JSON cache
(CPU); a small tuning run on the GPU."""
import numpy as np
import pytest

from sharp_data import gen


def test_candidates_and_keys(tmp_path):
    from paper_1602_01448_amd import autotune as at
    c = at._merge_candidates(2048)
    assert {x["tile"] for x in c} == {16, 32, 64}
    assert all(x["merge_split"] >= 1 for x in c)
    assert any(x["merge_split"] > 1 for x in at._merge_candidates(128))
    f = at._frame_candidates(256)
    assert {"frame_launch": 2, "strip_rows": 2} in f and {"frame_launch": 1, "fft_block": 512} in f
    assert not at._uses_tile_merge(256, {"frame_launch": 2, "strip_rows": 1})
    assert at._uses_tile_merge(256, {"frame_launch": 1, "fft_block": 256})
    assert at._frame_candidates(128) == [{"frame_launch": 2}, {"frame_launch": 1}]
    assert at._uses_tile_merge(128, {"frame_launch": 2})
    assert at._frame_candidates(64) == [{}]
    pos = gen.raster_positions(5, 10, 80, 32)
    k1 = at.geometry_key("raar", 80, 80, 32, pos, False)
    k2 = at.geometry_key("raar", 80, 80, 32, pos[::-1], False)
    assert k1 != k2 and k1.startswith(at._arch())
    path = str(tmp_path / "t.json")
    at.save_cache({k1: {"options": {"tile": 64}}}, path)
    assert at.lookup("raar", 80, 80, 32, pos, False, path=path) == {"tile": 64}
    assert at.lookup("raar", 80, 80, 32, pos[::-1], False, path=path) == {}


@pytest.mark.gpu
def test_tune_small_geometry(tmp_path):
    from paper_1602_01448_amd import Plan, autotune as at
    pos = gen.raster_positions(6, 16, 160, 64, jitter=2, rng=np.random.default_rng(0))
    path = str(tmp_path / "t.json")
    best = at.tune_raar(160, 160, 64, pos, iters=1, reps=1, path=path)
    assert best["tile"] in (16, 32, 64)
    p = Plan.tuned(160, 160, 64, pos)          # default cache: unaffected, library defaults
    assert p.info()["tile"] in (16, 32, 64)
    assert at.lookup("raar", 160, 160, 64, pos, path=path) == best
