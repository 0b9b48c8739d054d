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


def test_size_buckets_of_the_cache():
    """An exact entry wins; otherwise the nearest tuned padded size within 25 % with the
    same architecture, dimension, kind, precision and objective."""
    from paper_2011_13861_amd.autotune import lookup
    data = {"gfx950|d3|exp|f64|Np17664|apply": {"nsplit": 10},
            "gfx950|d3|exp|f64|Np16384|apply": {"nsplit": 8},
            "gfx950|d3|exp|f64|Np4608|apply": {"nsplit": 6},
            "gfx950|d3|exp|f32|Np18176|apply": {"nsplit": 12},
            "gfx950|d2|exp|f64|Np17920|apply": {"nsplit": 14},
            "gfx950|d3|exp|f64|Np17920": {"nsplit": 3}}
    assert lookup(data, "gfx950|d3|exp|f64|Np16384|apply") == {"nsplit": 8}
    assert lookup(data, "gfx950|d3|exp|f64|Np17920|apply") == {"nsplit": 10}     # nearest, not d2 / f32 / stage5
    assert lookup(data, "gfx950|d3|exp|f64|Np15360|apply") == {"nsplit": 8}
    assert lookup(data, "gfx950|d3|exp|f64|Np9216|apply") is None                 # beyond 25 %
    assert lookup(data, "gfx950|d3|sqexp|f64|Np17664|apply") is None
    assert lookup(data, "gfx942|d3|exp|f64|Np17664|apply") is None
