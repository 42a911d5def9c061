"""Pins for the metric oracle: Eq. 3 breakpoints and the paper's spp_avg tables."""
import math
import os

import numpy as np
import pytest

from oracle import metrics as M

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "spp_avg_tables.txt")


def test_srgb_eq3_pieces():
    assert M.srgb(-1.0) == 0.0 and M.srgb(0.0) == 0.0
    assert M.srgb(0.001) == pytest.approx(0.01292, rel=1e-12)
    # continuity at the linear/power breakpoint (the two branches meet to 4 digits)
    lo = 12.92 * 0.0031308
    hi = 1.055 * 0.0031308 ** (1 / 2.4) - 0.055
    assert M.srgb(0.0031308) == pytest.approx(lo, rel=1e-15)
    assert abs(lo - hi) < 1e-6
    assert M.srgb(0.5) == pytest.approx(1.055 * 0.5 ** (1 / 2.4) - 0.055, rel=1e-15)
    assert M.srgb(1.0) == 1.0 and M.srgb(123.0) == 1.0
    assert M.srgb(1.0 - 1e-12) == pytest.approx(1.0, abs=1e-11)  # continuous at 1
    x = np.linspace(-1, 2, 10001)
    assert np.all(np.diff(M.srgb(x)) >= 0)  # monotone


def test_psnr_and_relmse_closed_forms():
    ref = np.full((4, 4, 3), 0.5)
    img = ref.copy()
    img[0, 0, 0] = 1.0  # one sRGB value off by s(1) - s(0.5)
    d = 1.0 - M.srgb(0.5)
    assert M.psnr(img, ref) == pytest.approx(10 * math.log10(48 / d ** 2), rel=1e-12)
    assert M.psnr(ref, ref) == np.inf
    assert M.relmse(img, ref) == pytest.approx(0.5 * 0.25 / (0.25 + 0.01) / 48, rel=1e-12)
    assert M.relmse(img, ref, 1.0, 1e-4) == pytest.approx(0.25 / (0.25 + 1e-4) / 48, rel=1e-12)


def test_spp_avg_matches_paper_tables():
    rows = [list(map(int, l.split())) for l in open(GOLDEN) if l.strip() and l[0] != "#"]
    assert len(rows) == 18
    for table, s, lrhs, hrls, column in rows:
        v = M.spp_avg(lrhs, hrls, s)
        # every printed pair lands on its column (250 / 64 + 4 = 7.9 rounds to 8)
        assert round(v) == column, (table, s, lrhs, hrls, v)
        assert abs(v - column) <= 0.5
