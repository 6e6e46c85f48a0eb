"""Pins for the oracle's sRGB -> CIELAB conversion and CIEDE2000 (CPU only).

Sources outside the oracle: the CIELAB definition (CIE 15) fixes white at
L* = 100, a* = b* = 0 and L* = 116 cbrt(Y) - 16 for Y above (6/29)^3; the
sRGB standard (IEC 61966-2-1) fixes the luminance weights 0.2126 / 0.7152 /
0.0722 of the primaries; the sRGB primaries' CIELAB coordinates under D65 are
tabulated in colour-science references as red (53.24, 80.09, 67.20), green
(87.73, -86.18, 83.18), blue (32.30, 79.19, -107.86) and mid-grey 128 has
L* = 53.59.  CIEDE2000 (Sharma, Wu, Dalal 2005) reduces in special cases to
closed forms checked below: neutral pairs (only the lightness term), pairs on
the +a* axis (only the chroma term, the rotation term vanishes at hue 0), and
mirror pairs (a, b) / (a, -b) (only the hue term, mean hue 0 or 180).  The rotation term R_T is parity
unpinned beyond these limits and symmetry.
"""
import math

import numpy as np
import pytest

import oracle


def test_white_black_greys():
    assert np.allclose(oracle.srgb_to_lab64([255, 255, 255]), [100, 0, 0], atol=1e-9)
    assert np.allclose(oracle.srgb_to_lab64([0, 0, 0]), [0, 0, 0], atol=1e-12)
    for v in range(0, 256, 5):
        lab = oracle.srgb_to_lab64([v, v, v])
        assert abs(lab[1]) < 1e-9 and abs(lab[2]) < 1e-9
    assert abs(oracle.srgb_to_lab64([128, 128, 128])[0] - 53.59) < 0.01


@pytest.mark.parametrize("rgb,Y", [((255, 0, 0), 0.2126), ((0, 255, 0), 0.7152), ((0, 0, 255), 0.0722)])
def test_primary_lightness_closed_form(rgb, Y):
    L = oracle.srgb_to_lab64(rgb)[0]
    assert abs(L - (116 * Y ** (1 / 3) - 16)) < 1e-9


@pytest.mark.parametrize("rgb,lab", [((255, 0, 0), (53.24, 80.09, 67.20)),
                                     ((0, 255, 0), (87.73, -86.18, 83.18)),
                                     ((0, 0, 255), (32.30, 79.19, -107.86))])
def test_primaries_tabulated(rgb, lab):
    assert np.allclose(oracle.srgb_to_lab64(rgb), lab, atol=0.05)


def test_lab32_matches_lab64():
    rng = np.random.default_rng(3)
    for _ in range(2000):
        c = rng.integers(0, 256, size=3).astype(np.uint8)
        assert np.max(np.abs(oracle.srgb_to_lab32(c) - oracle.srgb_to_lab64(c))) < 2e-4


def test_ciede2000_zero_and_symmetry():
    rng = np.random.default_rng(4)
    for _ in range(500):
        a = np.array([rng.uniform(0, 100), rng.uniform(-120, 120), rng.uniform(-120, 120)])
        b = np.array([rng.uniform(0, 100), rng.uniform(-120, 120), rng.uniform(-120, 120)])
        assert oracle.ciede2000_64(a, a) == 0.0
        assert abs(oracle.ciede2000_64(a, b) - oracle.ciede2000_64(b, a)) < 1e-9
        assert oracle.ciede2000_64(a, b) >= 0


@pytest.mark.parametrize("L1,L2", [(50, 60), (20, 25), (90, 70), (0, 100), (50, 50.5)])
def test_ciede2000_neutral_pairs(L1, L2):
    Lm = (L1 + L2) / 2
    SL = 1 + 0.015 * (Lm - 50) ** 2 / math.sqrt(20 + (Lm - 50) ** 2)
    assert abs(oracle.ciede2000_64([L1, 0, 0], [L2, 0, 0]) - abs(L2 - L1) / SL) < 1e-12


@pytest.mark.parametrize("a1,a2", [(10, 20), (30, 31), (5, 60), (80, 40)])
def test_ciede2000_chroma_only_on_a_axis(a1, a2):
    # same L, b = 0, a > 0: hue 0 for both, so dH = 0 and R_T ~ 30 exp(-121) ~ 0
    Cm = (a1 + a2) / 2
    G = 0.5 * (1 - math.sqrt(Cm ** 7 / (Cm ** 7 + 25.0 ** 7)))
    c1, c2 = a1 * (1 + G), a2 * (1 + G)
    expect = abs(c2 - c1) / (1 + 0.045 * (c1 + c2) / 2)
    assert abs(oracle.ciede2000_64([50, a1, 0], [50, a2, 0]) - expect) < 1e-9


def _T(h):
    r = math.radians
    return 1 - 0.17 * math.cos(r(h - 30)) + 0.24 * math.cos(r(2 * h)) + 0.32 * math.cos(r(3 * h + 6)) - 0.20 * math.cos(r(4 * h - 63))


@pytest.mark.parametrize("a,b,mean_hue", [(30, 8, 0), (12, 3, 0), (60, 25, 0), (-30, 8, 180), (-45, 20, 180)])
def test_ciede2000_hue_only_mirror_pairs(a, b, mean_hue):
    # (a, b) and (a, -b): equal L, equal C' (a' = a (1 + G) is shared), so only
    # the hue term survives and the mean hue lies on the a* axis (0 or 180).
    C = math.hypot(a, b)
    G = 0.5 * (1 - math.sqrt(C ** 7 / (C ** 7 + 25.0 ** 7)))
    ap = a * (1 + G)
    Cp = math.hypot(ap, b)
    half = math.atan2(abs(b), abs(ap))  # half the hue angle between the two
    if ap < 0:
        half = math.atan2(abs(b), -ap)
    dH = 2 * Cp * math.sin(half)
    SH = 1 + 0.015 * Cp * _T(mean_hue)
    expect = dH / SH
    got = oracle.ciede2000_64([50, a, b], [50, a, -b])
    assert abs(got - expect) < 1e-9


def test_ciede2000_hue_wraparound_short_arc():
    # (350, 10) and (10, 350) are 20 degrees apart, never 340
    C = 40.0
    x = [60, C * math.cos(math.radians(350)), C * math.sin(math.radians(350))]
    y = [60, C * math.cos(math.radians(10)), C * math.sin(math.radians(10))]
    d = oracle.ciede2000_64(x, y)
    far = [60, C * math.cos(math.radians(190)), C * math.sin(math.radians(190))]
    assert d < oracle.ciede2000_64(x, far) / 3
    assert abs(d - oracle.ciede2000_64(y, x)) < 1e-12


def test_ciede2000_32_matches_64():
    rng = np.random.default_rng(5)
    worst = 0.0
    for _ in range(5000):
        a = np.array([rng.uniform(0, 100), rng.uniform(-110, 110), rng.uniform(-110, 110)])
        b = a + rng.normal(0, 15, size=3)
        d64 = oracle.ciede2000_64(a, b)
        d32 = oracle.ciede2000_32(a.astype(np.float32), b.astype(np.float32))
        worst = max(worst, abs(d64 - d32))
    assert worst < 1e-3
