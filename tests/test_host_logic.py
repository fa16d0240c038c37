"""Host-side logic of the batching layer (no GPU): the autotuner's choice
between the library's default setting and a timed candidate."""
import pytest

from paper_2401_13708_amd.batch import pick_setting


def test_default_kept_within_the_noise_margin():
    # every candidate within 2 % of the default: timing noise, keep the default
    t = {128: 2.6353, 256: 2.6448, 512: 2.6553, 1024: 2.6419, 2048: 2.6336}
    assert pick_setting(t, 256, 0.02) == 256


def test_clear_winner_replaces_the_default():
    t = {(0, 1): 2.632, (16384, 4): 2.6298, (32768, 1): 2.4672, (65536, 1): 2.3875}
    assert pick_setting(t, (0, 1), 0.02) == (65536, 1)


def test_margin_zero_takes_the_fastest():
    assert pick_setting({1: 1.0, 2: 0.999}, 1, 0.0) == 2


@pytest.mark.parametrize("times", [{}, {512: 1.0}])
def test_default_untimed_or_nothing_timed(times):
    # nothing timed: the default; a default that was not timed cannot be kept
    assert pick_setting(times, 256, 0.02) == (256 if not times else 512)


def test_attract_launch_rule_mirrors_the_library():
    # the library's threshold (k_bh.hip, kAttractWithTopAt) and the binding's
    import re
    from pathlib import Path
    from paper_2401_13708_amd import hts
    src = (Path(__file__).resolve().parents[1] / "paper_2401_13708_amd" / "csrc" / "k_bh.hip").read_text()
    assert int(re.search(r"kAttractWithTopAt = (\d+);", src).group(1)) == hts.ATTRACT_WITH_TOP_AT
    assert hts.attract_in_items(0, 70000) and not hts.attract_in_items(0, 200000)
    assert hts.attract_in_items(2, 10 ** 6) and not hts.attract_in_items(1, 1000)
