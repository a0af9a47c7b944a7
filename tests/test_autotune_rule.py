"""The autotuner's choice rule (CPU): a candidate displaces the best so far
only when it is more than 1% faster, so the first candidate (the default
tuning) keeps its place against differences within run-to-run noise."""
from paper_2303_12980_amd.autotune import choose


def test_default_kept_within_one_percent():
    assert choose([{"ms": 1.000}, {"ms": 0.995}, {"ms": 1.200}]) == 0


def test_clear_winner_displaces_the_default():
    assert choose([{"ms": 1.000}, {"ms": 0.950}]) == 1


def test_later_candidate_must_beat_the_current_best_by_the_margin():
    # 0.946 is within 1% of 0.950 (the best so far), 0.93 is not
    assert choose([{"ms": 1.000}, {"ms": 0.950}, {"ms": 0.946}]) == 1
    assert choose([{"ms": 1.000}, {"ms": 0.950}, {"ms": 0.946}, {"ms": 0.930}]) == 3


def test_margin_zero_is_the_plain_minimum():
    times = [{"ms": t} for t in (1.0, 0.999, 1.3, 0.998, 1.1)]
    assert choose(times, margin=0.0) == 3
