"""Host logic of the stage-5 autotuner: which timed setting is kept."""

from paper_2011_13861_amd.autotune import pick


def test_pick_prefers_xcd_aligned_fewer_splits_within_noise():
    timed = [(2, 10, 100.0), (2, 8, 101.0), (2, 16, 100.5), (2, 3, 140.0)]
    assert pick(timed) == (2, 8, 101.0)             # within 1.5 %, a multiple of 8, fewest


def test_pick_keeps_the_fastest_beyond_noise():
    assert pick([(2, 10, 100.0), (2, 8, 110.0)]) == (2, 10, 100.0)
    assert pick([(4, 7, 50.0)]) == (4, 7, 50.0)


def test_pick_one_split_has_no_partials():
    assert pick([(2, 1, 100.0), (2, 8, 100.2)]) == (2, 1, 100.0)
    assert pick([(2, 1, 100.5), (2, 8, 100.0), (2, 24, 99.9)]) == (2, 1, 100.5)
