"""Launch-schedule tuner without a GPU: the candidate list and the choice
from timings (median, default kept within the noise margin, ties to the
earlier schedule)."""
import pytest

from paper_1810_12163_amd import (SCHEDULE_FAST_WAVES, SCHEDULE_IPT, SCHEDULE_LDS_LEVELS, SCHEDULE_SCORE_WINDOWS,
                                  autotune)


def test_candidates_cover_every_accepted_schedule_default_first():
    c = autotune.candidates()
    assert c[0] == autotune.DEFAULT
    assert sorted(c) == sorted((i, f, l, w) for i in SCHEDULE_IPT for f in SCHEDULE_FAST_WAVES
                               for l in SCHEDULE_LDS_LEVELS for w in SCHEDULE_SCORE_WINDOWS)
    assert len(set(c)) == len(c) == 36
    assert autotune.candidates(ipts=(2,), fast_waves=(4,), lds_levels=(6,), windows=(2,)) == [(2, 4, 6, 2)]
    assert autotune.candidates(ipts=(4,), fast_waves=(1,), lds_levels=(8,), windows=(2, 0)) == [(4, 1, 8, 0), (4, 1, 8, 2)]
    assert autotune.candidates(first=autotune.BATCH_DEFAULT)[0] == autotune.BATCH_DEFAULT
    assert sorted(autotune.candidates(first=autotune.BATCH_DEFAULT)) == sorted(c)


def test_pick_uses_the_median():
    t = {(4, 1, 8, 0): [10.0, 10.0, 10.0], (2, 1, 8, 0): [1.0, 9.0, 9.0], (8, 1, 6, 2): [20.0, 8.0, 8.0]}
    assert autotune.pick(t) == (8, 1, 6, 2)         # medians 10, 9, 8


def test_pick_keeps_the_default_within_the_margin():
    t = {(4, 1, 8, 0): [10.0], (8, 2, 6, 2): [9.9]}
    assert autotune.pick(t) == (4, 1, 8, 0)
    assert autotune.pick(t, margin=0.0) == (8, 2, 6, 2)
    t = {(4, 1, 8, 0): [10.0], (8, 2, 6, 2): [9.7]}
    assert autotune.pick(t) == (8, 2, 6, 2)


def test_pick_ties_go_to_the_earlier_schedule_and_empty_is_an_error():
    assert autotune.pick({(2, 2): [5.0], (8, 4): [5.0]}) == (2, 2)
    assert autotune.pick({(8, 4): [5.0], (2, 2): [5.0]}) == (8, 4)
    with pytest.raises(ValueError):
        autotune.pick({})
