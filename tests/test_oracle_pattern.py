"""Pins of the oracle's subray pattern (Sec. 3.4, Eq. 1, Fig. 6)."""
import math
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "fig6_subray_counts.txt")


def _golden_counts():
    rows = []
    for line in open(GOLDEN):
        line = line.split("#")[0].strip()
        if line:
            q, s, _ = line.split(None, 2)
            rows.append((int(q), int(s)))
    return rows


def test_printed_counts_fig6(orc):
    rows = _golden_counts()
    assert rows == [(5, 93), (9, 279)]
    for q, s in rows:
        assert orc.pattern_size(0, q) == s
        a, p, w = orc.pattern(dict(divergence_rad=0.3e-3, n_subrays=0, beam_quality=q,
                                   pulse_width_ns=4.0, bin_ns=1.0, n_bins=16))
        assert a.size == s


def test_small_qualities(orc):
    # quality 1 -> 1 + 6 and quality 2 -> 1 + 6 + 12: a single ray for quality 0
    assert orc.pattern_size(0, 0) == 1
    assert orc.pattern_size(0, 1) == 7
    assert orc.pattern_size(0, 2) == 19
    assert orc.pattern_size(0, 3) == 37


def test_ring_fill_counts(orc):
    # counts between ring totals: complete rings, then the remainder on the last ring
    assert list(orc.ring_layout(31)) == [6, 12, 12]
    assert list(orc.ring_layout(61)) == [6, 12, 18, 24]
    assert list(orc.ring_layout(19)) == [6, 12]
    assert list(orc.ring_layout(1)) == []
    assert list(orc.ring_layout(2)) == [1]
    for s in range(1, 300):
        assert orc.pattern_size(s, 0) == s


def _sc(S, div=0.5e-3, kappa=1.0):
    return dict(divergence_rad=div, n_subrays=S, pattern_extent=kappa, pulse_width_ns=4.0, bin_ns=1.0, n_bins=16)


@pytest.mark.parametrize("S", [7, 19, 31, 37, 61, 93])
def test_weights_and_symmetry(orc, S):
    a, p, w = orc.pattern(_sc(S))
    assert abs(w.sum() - 1.0) < 1e-14
    # every ring with >= 2 evenly spaced members has zero weighted centroid
    cx = np.sum(w * np.sin(a) * np.cos(p))
    cy = np.sum(w * np.sin(a) * np.sin(p))
    assert abs(cx) < 1e-18 and abs(cy) < 1e-18
    # the weight falls with the angle from the axis
    order = np.argsort(a, kind="stable")
    assert np.all(np.diff(w[order]) <= 1e-18)


@pytest.mark.parametrize("S", [7, 19, 31, 61, 279])
def test_outer_ring_at_one_over_e_squared(orc, S):
    # Fig. 6 caption: the divergence is quoted at the 1/e^2 points; with the
    # outer ring on that cone (kappa = 1) its intensity is e^-2 of the centre.
    a, p, w = orc.pattern(_sc(S, div=0.3e-3))
    outer = a.max()
    assert abs(outer - 0.15e-3) < 1e-18
    assert abs(w[np.argmax(a)] / w[0] - math.exp(-2.0)) < 1e-12


def test_equal_angular_spacing(orc):
    # Sec. 3.4: adjacent subrays are about equally far apart, along and across rings
    a, p, w = orc.pattern(_sc(279))
    rings = np.unique(a[a > 0])
    dr = rings[0]
    for r in rings:
        n_i = np.count_nonzero(a == r)
        along = 2.0 * math.pi * r / n_i
        assert 1.0 <= along / dr < 1.05


@pytest.mark.parametrize("d", [(0, 0, -1), (0, 0, 1), (1, 0, 0), (0.3, -0.4, -0.866), (-0.7, 0.1, 0.2)])
def test_subray_directions(orc, d):
    sc = _sc(31, div=2e-2)   # wide beam so angles are resolved well
    d = np.asarray(d, dtype=np.float64)
    dh = d / np.linalg.norm(d)
    a, p, w = orc.pattern(sc)
    D = orc.subray_directions(d, sc)
    assert np.allclose(np.linalg.norm(D, axis=1), 1.0, atol=1e-15)
    # angle to the beam axis equals alpha (via the sine, well conditioned)
    s = np.linalg.norm(np.cross(D, dh[None, :]), axis=1)
    assert np.allclose(s, np.sin(a), atol=1e-15)
    assert np.all(D @ dh > 0)
    # weighted mean direction is the beam axis
    m = (w[:, None] * D).sum(0)
    assert np.linalg.norm(np.cross(m / np.linalg.norm(m), dh)) < 1e-15
    # on each ring, neighbours are 2*pi/n_i apart in azimuth around the axis
    proj = D - (D @ dh)[:, None] * dh[None, :]
    for r in np.unique(a[a > 0]):
        idx = np.nonzero(a == r)[0]
        n_i = idx.size
        for q in range(n_i):
            u = proj[idx[q]]
            v = proj[idx[(q + 1) % n_i]]
            ang = math.atan2(np.linalg.norm(np.cross(u, v)), u @ v)
            assert abs(ang - 2.0 * math.pi / n_i) < 1e-9
        # and they turn in one sense about the axis
        assert np.cross(proj[idx[0]], proj[idx[1]]) @ dh > 0
