"""Host logic of the autotuner (no GPU): candidate generation, scoring, cache."""
import os

from paper_1305_4196_amd import tune


def test_candidates_are_valid_and_ranked():
    for occ in (5.3, 6.6, 19.1, 30.0):
        cands = tune.candidates(occ, top=8)
        assert 1 <= len(cands) <= 8
        scores = [tune.score(s, t, occ) for s, t in cands]
        assert scores == sorted(scores, reverse=True) and scores[0] > 0
        for (bx, by, bz), t in cands:
            assert 1 <= min(bx, by, bz) and max(bx, by, bz) <= 4
            assert bx * by * bz <= 64 and (bx + 2) * (by + 2) * (bz + 2) <= 512
            assert t % 64 == 0 and 128 <= t <= 512


def test_score_rejects_stages_beyond_the_lds():
    # ~80 atoms per cell: a 4x4x4 brick stages ~17k candidates, far beyond 160 KiB
    assert tune.score((4, 4, 4), 512, 80.0) == 0.0
    assert tune.score((1, 1, 1), 128, 80.0) > 0.0


def test_lane_efficiency_accounts_for_spread():
    # a brick whose mean fills the workgroup exactly needs a second round at +2 sd
    s_tight = tune.score((2, 2, 2), 128, 16.0)      # 128 atoms on 128 lanes
    s_room = tune.score((2, 2, 2), 192, 16.0)       # same brick on 192 lanes
    assert s_room > s_tight


def test_cache_round_trip(tmp_path):
    path = os.path.join(str(tmp_path), "sub", "cache.json")
    assert tune.load_cache(path) == {}
    entry = {"shape": [4, 3, 2], "threads": 512, "ms": 0.25}
    tune.save_cache({"k": entry}, path)
    assert tune.load_cache(path) == {"k": entry}


def test_candidate_set_adds_the_fixed_shapes():
    for occ in (6.6, 19.1):
        cs = tune.candidate_set(occ, top=4)
        assert cs[:4] == tune.candidates(occ, top=4)
        assert len(set(cs)) == len(cs)
        for shape, t in tune.EXTRA_SHAPES:
            assert ((shape, t) in cs) == (tune.score(shape, t, occ) > 0)
