"""Host-side logic of the autotuner (no GPU)."""
from paper_2106_12802_amd import autotune


def test_choose_median_and_ties():
    t = [((1, 1), [5.0, 1.0, 9.0]), ((2, 2), [4.0, 4.0, 4.0]), ((3, 3), [4.0, 3.0, 100.0])]
    (cand, med) = autotune.choose(t)
    assert cand == (2, 2) and med == 4.0  # medians 5, 4, 4: first of the tie
    assert autotune.choose([((7, 7), [2.0])]) == ((7, 7), 2.0)
