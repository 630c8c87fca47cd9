"""Pins of the oracle's Multicopter smooth turn mode (Sec. 3.2: the platform
banks to turn smoothly at the waypoints instead of stopping and turning on the
spot).  Reading: a coordinated turn on a circular arc tangent to both legs, of
radius v^2 / (g tan b), flown at the cruise speed and banked by b toward the
turn's centre; level, straight flight elsewhere; the ramps from rest and to
rest at the first and last waypoints.  The checks are independent of the
oracle's construction: a least-squares circle through the sampled turn, the
closest approach to the corner, speeds and headings read off the origins,
the beam's tilt and the flight time from the path length."""
import numpy as np
import pytest

G = 9.80665
V, A, PRF, BANK = 8.0, 2.0, 100.0, np.radians(20.0)
LAWN = [[0.0, 0.0, 60.0], [300.0, 0.0, 60.0], [300.0, 60.0, 60.0], [0.0, 60.0, 60.0]]
R = V * V / (G * np.tan(BANK))


def _survey(wp=LAWN, **kw):
    # a fibre array with angle 0 fires straight down the platform's z axis
    sv = dict(waypoints=wp, deflector="fibre", n_fibres=2, scan_angle_rad=0.0, speed_mps=V, pulse_rate_hz=PRF,
              platform="multicopter_smooth", accel_mps2=A, bank_angle_rad=BANK, t0=0.0, platform_noise_m=0.0,
              seed=1)
    sv.update(kw)
    return sv


def _fit_circle(xy):
    """Algebraic least-squares circle (Kasa): centre and radius."""
    x, y = xy[:, 0], xy[:, 1]
    M = np.stack([x, y, np.ones_like(x)], 1)
    b = x * x + y * y
    c, *_ = np.linalg.lstsq(M, b, rcond=None)
    cx, cy = c[0] / 2, c[1] / 2
    return np.array([cx, cy]), np.sqrt(c[2] + cx * cx + cy * cy)


def _flight(orc, wp=LAWN, n=None, **kw):
    L = np.linalg.norm(np.diff(np.array(wp), axis=0), axis=1).sum()
    n = n or int((L / V + V / A + 5.0) * PRF)
    return orc.generate_pulses(_survey(wp, **kw), 0, n)


def test_turn_is_a_circle_of_the_bank_radius(orc):
    o, d = _flight(orc)
    # the first corner (300, 0): its arc lies in the square [300 - R, 300] x [0, R]
    m = (o[:, 0] > 300.0 - R + 1e-3) & (o[:, 1] > 1e-3) & (o[:, 1] < R - 1e-3)
    assert m.sum() > 100
    c, r = _fit_circle(o[m, :2])
    assert abs(r - R) < 1e-6 * R, (r, R)
    assert np.allclose(c, [300.0 - R, R], atol=1e-6)
    assert np.allclose(o[m, 2], 60.0)
    # closest approach to the corner: R (1 / cos(45 deg) - 1)
    dmin = np.linalg.norm(o[:, :2] - [300.0, 0.0], axis=1).min()
    assert abs(dmin - R * (np.sqrt(2.0) - 1.0)) < V / PRF


def test_speed_and_heading_are_continuous_through_turns(orc):
    o, d = _flight(orc)
    step = np.linalg.norm(np.diff(o, axis=0), axis=1) * PRF
    assert step.max() <= V * (1 + 1e-9)
    # cruise speed everywhere between the ramps, the turns included (no stop)
    t = np.arange(o.shape[0]) / PRF
    L = 300.0 + 60.0 + 300.0 - 2 * (2 * R - R * np.pi / 2)
    T = L / V + V / A
    cruise = (t[1:] > V / A + 0.02) & (t[1:] < T - V / A - 0.02)
    assert np.allclose(step[cruise], V, rtol=1e-5)
    # the heading of motion turns by at most v dt / R per pulse
    h = np.unwrap(np.arctan2(np.diff(o[:, 1]), np.diff(o[:, 0]))[cruise])
    assert np.abs(np.diff(h)).max() <= V / (R * PRF) * (1 + 1e-6)
    assert abs(h[-1] - h[0] - np.pi) < 1e-3   # two left turns of 90 degrees
    # the flight ends at the last waypoint at T = L / v + v / a and stays there
    done = t > T + 1e-6
    assert np.allclose(o[done], LAWN[-1], atol=1e-9)
    late = (t > T - 0.5) & (t < T - 1e-3)
    assert np.all(np.linalg.norm(o[late] - LAWN[-1], axis=1) > 0)


def test_bank_tilts_the_beam_outward_in_turns_only(orc):
    for wp, sign in ((LAWN, 1.0), ([[0.0, 0.0, 60.0], [300.0, 0.0, 60.0], [300.0, -60.0, 60.0]], -1.0)):
        o, d = _flight(orc, wp)
        off = np.degrees(np.arccos(np.clip(-d[:, 2], -1, 1)))
        m = (o[:, 0] > 300.0 - R + 1e-3) & (np.abs(o[:, 1]) > 1e-3) & (np.abs(o[:, 1]) < R - 1e-3)
        straight = (o[:, 0] < 300.0 - R - 1e-3) & (np.abs(o[:, 1]) < 1e-9)
        assert m.sum() > 100 and straight.sum() > 100
        # straight flight: level, the beam straight down
        assert np.allclose(d[straight], [0.0, 0.0, -1.0], atol=1e-15)
        # in the turn: tilted by the bank angle, away from the turn's centre
        assert np.allclose(off[m], np.degrees(BANK), atol=1e-9)
        centre = np.array([300.0 - R, sign * R])
        out = o[m, :2] - centre
        assert np.all(np.einsum("ij,ij->i", out, d[m, :2]) > 0)


def test_climbing_turn_stays_in_the_legs_plane(orc):
    wp = [[0.0, 0.0, 50.0], [200.0, 0.0, 70.0], [200.0, 150.0, 90.0]]
    o, d = _flight(orc, wp)
    a, w, b = (np.array(x) for x in wp)
    u = (w - a) / np.linalg.norm(w - a)
    v = (b - w) / np.linalg.norm(b - w)
    nrm = np.cross(u, v)
    nrm /= np.linalg.norm(nrm)
    th = np.arccos(u @ v)
    s = R * np.tan(th / 2)
    # points of the arc: past the arc's start along the first leg and before its end on the second
    along_in = (o - w) @ u
    along_out = (o - w) @ v
    m = (along_in > -s + 1e-3) & (along_out < s - 1e-3)
    assert m.sum() > 50
    assert np.abs((o[m] - w) @ nrm).max() < 1e-9      # in the plane of the two legs
    # equidistant (R) from one centre: the point at distance R from both tangent points
    nin = v - (u @ v) * u
    nin /= np.linalg.norm(nin)
    c = w - s * u + R * nin
    assert np.allclose(np.linalg.norm(o[m] - c, axis=1), R, rtol=1e-9)


def test_straight_through_waypoints_is_one_leg(orc):
    # a waypoint on the line between its neighbours adds no turn
    o1, d1 = _flight(orc, [[0.0, 0.0, 40.0], [120.0, 0.0, 40.0], [300.0, 0.0, 40.0]])
    o2, d2 = _flight(orc, [[0.0, 0.0, 40.0], [300.0, 0.0, 40.0]], n=o1.shape[0])
    assert np.allclose(o1, o2, atol=1e-9) and np.allclose(d1, d2, atol=1e-12)


def test_smooth_rejections(orc):
    with pytest.raises(ValueError):   # bank outside (0, 90) degrees
        orc.generate_pulses(_survey(bank_angle_rad=0.0), 0, 10)
    with pytest.raises(ValueError):
        orc.generate_pulses(_survey(bank_angle_rad=np.pi / 2), 0, 10)
    with pytest.raises(ValueError):   # a 60 m cross leg cannot hold two arcs of 2 R > 60 m
        orc.generate_pulses(_survey(bank_angle_rad=np.radians(5.0)), 0, 10)
    with pytest.raises(ValueError):   # a turn that reverses the leg
        orc.generate_pulses(_survey([[0.0, 0.0, 60.0], [300.0, 0.0, 60.0], [0.0, 0.1, 60.0]]), 0, 10)
    with pytest.raises(ValueError):   # the first leg cannot hold the ramp and the arc
        orc.generate_pulses(_survey([[0.0, 0.0, 60.0], [20.0, 0.0, 60.0], [20.0, 100.0, 60.0]]), 0, 10)
    with pytest.raises(ValueError):   # leg yaws belong to the stop-and-turn mode
        orc.generate_pulses(_survey(leg_yaw=[[0.0, 0.0]] * 3), 0, 10)
