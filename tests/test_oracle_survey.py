"""Pins of the oracle's pulse generation from a survey (Sec. 3.2: a LinearPath
platform moves at constant speed from waypoint to waypoint, facing the next one;
Sec. 3.3 and Fig. 7: a polygon mirror gives parallel lines of even density, a
fibre array a similar pattern from fixed directions, a swinging mirror a
zig-zag denser at its extremes, a Palmer scanner a cone at a constant angle off
nadir), and of its counter-based SplitMix64 (Steele, Lea & Flood 2014)."""
import numpy as np
import pytest

from synth.rng import splitmix64 as synth_splitmix64

WP = [[0.0, 0.0, 500.0], [1200.0, 0.0, 500.0], [1200.0, 300.0, 520.0], [-100.0, 300.0, 520.0],
      [500.0, 900.0, 480.0]]


def _survey(**kw):
    sv = dict(waypoints=WP, deflector="polygon", speed_mps=60.0, pulse_rate_hz=2000.0, scan_freq_hz=20.0,
              scan_angle_rad=0.4, n_fibres=0, t0=0.0, platform_noise_m=0.0, seed=1)
    sv.update(kw)
    return sv


def _legs():
    wp = np.array(WP)
    seg = np.diff(wp, axis=0)
    return wp, seg, np.concatenate([[0.0], np.cumsum(np.linalg.norm(seg, axis=1))])


def test_splitmix64_published_sequence(orc):
    # the first outputs of the reference generator seeded with 0
    assert [orc.splitmix64(0, c) for c in range(3)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4,
                                                        0x06C45D188009454F]
    # and an independent implementation of the same definition
    gamma = 0x9E3779B97F4A7C15
    rng = np.random.default_rng(3)
    for seed, c in zip(rng.integers(0, 2**63, 20), rng.integers(0, 2**40, 20)):
        state = (int(seed) + int(c) * gamma) & 0xFFFFFFFFFFFFFFFF   # the finaliser adds one more gamma
        assert orc.splitmix64(int(seed), int(c)) == int(synth_splitmix64(np.uint64(state)))


def test_linear_path_kinematics(orc):
    wp, seg, cum = _legs()
    sv = _survey()
    n = int(cum[-1] / 60.0 * 2000.0) + 4000          # past the end of the path
    o, d = orc.generate_pulses(sv, 0, n)
    t = np.arange(n) / 2000.0
    s = np.minimum(60.0 * t, cum[-1])
    # every origin lies on the polyline at arc length s (constant speed)
    for i in range(len(seg)):
        m = (s >= cum[i]) & (s <= cum[i + 1])
        f = (s[m] - cum[i]) / (cum[i + 1] - cum[i])
        assert np.allclose(o[m], wp[i] + f[:, None] * seg[i], atol=1e-9)
    # at the waypoints' times the platform is at the waypoints
    for i in range(1, len(wp)):
        k = int(round(cum[i] / 60.0 * 2000.0))
        assert np.linalg.norm(o[k] - wp[i]) <= 60.0 / 2000.0 + 1e-9
    # the platform faces the current leg: line directions are across-track, and
    # a positive scan angle points to the platform's left
    ph = (2000.0 * 0.0 + 20.0 * t) % 1.0
    ang = -0.4 + 0.8 * ph
    for i in range(len(seg)):
        m = (s > cum[i] + 1.0) & (s < cum[i + 1] - 1.0)
        h = seg[i][:2] / np.linalg.norm(seg[i][:2])
        assert np.max(np.abs(d[m, :2] @ h)) <= 1e-12
        left = np.array([-h[1], h[0]])
        assert np.allclose(d[m, :2] @ left, np.sin(ang[m]), atol=1e-9)
    # after the end it stays at the last waypoint
    assert np.allclose(o[-100:], wp[-1], atol=1e-9)
    assert np.allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-14)


def _across_angle(d, heading):
    left = np.array([-np.sin(heading), np.cos(heading), 0.0])
    return np.arctan2(d @ left, -d[:, 2])


def test_polygon_mirror_sawtooth(orc):
    sv = _survey(waypoints=[[0.0, 0.0, 300.0]], pulse_rate_hz=1000.0, scan_freq_hz=10.0, scan_angle_rad=0.35)
    _, d = orc.generate_pulses(sv, 0, 3000)
    a = _across_angle(d, 0.0)
    assert a.min() >= -0.35 - 1e-12 and a.max() < 0.35
    step = np.diff(a)
    inline = step > 0
    assert np.allclose(step[inline], 2 * 0.35 * 10.0 / 1000.0, atol=1e-12)   # even spacing along a line
    assert np.sum(~inline) == 29                                           # a new line every 1/f
    assert np.allclose(d[:, 0], 0.0)


def test_swing_mirror_zigzag(orc):
    sv = _survey(waypoints=[[0.0, 0.0, 300.0]], deflector="swing", pulse_rate_hz=5000.0, scan_freq_hz=7.0,
                 scan_angle_rad=0.3)
    _, d = orc.generate_pulses(sv, 0, 50000)
    a = _across_angle(d, 0.0)
    t = np.arange(50000) / 5000.0
    assert np.allclose(a, 0.3 * np.sin(2 * np.pi * 7.0 * t), atol=1e-12)
    h, _ = np.histogram(a, bins=10, range=(-0.3, 0.3))
    assert h[0] > 2 * h[4] and h[-1] > 2 * h[5]      # denser at the extremes


def test_conic_constant_off_nadir(orc):
    sv = _survey(deflector="conic", scan_angle_rad=0.26, scan_freq_hz=15.0, speed_mps=400.0)
    o, d = orc.generate_pulses(sv, 0, 20000)
    assert np.allclose(-d[:, 2], np.cos(0.26), atol=1e-14)
    az = np.arctan2(d[:, 1], d[:, 0])
    # a full circle of azimuths over one revolution
    k = int(2000.0 / 15.0)
    assert np.ptp(np.unwrap(az[:k])) > 2 * np.pi * (1 - 2.0 / k)
    # in the platform frame the azimuth turns from forward towards left at 15 Hz
    wp, seg, cum = _legs()
    t = np.arange(20000) / 2000.0
    s = 400.0 * t
    p = 2 * np.pi * ((15.0 * t) % 1.0)
    assert s[-1] > cum[-2] + 1.0            # every leg, the diagonal one included
    for i in range(len(seg)):
        m = (s > cum[i] + 1.0) & (s < cum[i + 1] - 1.0)
        if not m.any():
            continue
        h = seg[i][:2] / np.linalg.norm(seg[i][:2])
        fwd = d[m, :2] @ h
        left = d[m, :2] @ np.array([-h[1], h[0]])
        assert np.allclose(fwd, np.sin(0.26) * np.cos(p[m]), atol=1e-9)
        assert np.allclose(left, np.sin(0.26) * np.sin(p[m]), atol=1e-9)


def test_fibre_array_fixed_directions(orc):
    sv = _survey(waypoints=[[0.0, 0.0, 300.0]], deflector="fibre", n_fibres=7, scan_angle_rad=0.2)
    _, d = orc.generate_pulses(sv, 0, 700)
    a = _across_angle(d, 0.0)
    assert np.allclose(a[:7], np.linspace(-0.2, 0.2, 7), atol=1e-14)
    assert np.allclose(a.reshape(-1, 7), a[:7][None, :], atol=0.0)


def test_platform_noise(orc):
    sv0 = _survey()
    sv = _survey(platform_noise_m=0.05, seed=12345)
    o0, d0 = orc.generate_pulses(sv0, 0, 40000)
    o, d = orc.generate_pulses(sv, 0, 40000)
    assert np.array_equal(d, d0)                      # noise moves origins only
    e = o - o0
    assert np.all(np.abs(e.mean(axis=0)) < 0.05 * 4 / np.sqrt(40000))
    assert np.allclose(e.std(axis=0), 0.05, rtol=0.03)
    c = np.corrcoef(e.T)
    assert np.max(np.abs(c - np.eye(3))) < 0.03
    # independent across pulses too (no draw is shared with a neighbour)
    lag = np.corrcoef(np.hstack([e[:-1], e[1:]]).T)[:3, 3:]
    assert np.max(np.abs(lag)) < 0.03
    # Gaussian: about 68.3 % within one sigma
    assert abs(np.mean(np.abs(e) < 0.05) - 0.6827) < 0.01
    # counter-based: any chunk equals the same pulses of the whole run
    o2, _ = orc.generate_pulses(sv, 12345, 1000)
    assert np.array_equal(o2, o[12345:13345])
    o3, _ = orc.generate_pulses(_survey(platform_noise_m=0.05, seed=12346), 0, 1000)
    assert not np.any(o3 == o[:1000])
