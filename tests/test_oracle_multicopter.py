"""Pins of the oracle's Multicopter platform (Sec. 3.2: unlike the LinearPath
platform it speeds up and slows down; without banked turns it stops at every
waypoint and turns there; start and end yaw of each leg may be given).  The
kinematics are checked against a time-stepped controller that knows only the
rules (accelerate up to the cruise speed, brake as late as still stops at the
waypoint), against the LinearPath platform in the limit of a huge
acceleration, and through speeds and accelerations read off the origins."""
import numpy as np
import pytest

WP = [[0.0, 0.0, 80.0], [400.0, 0.0, 80.0], [400.0, 16.0, 84.0], [100.0, 300.0, 70.0]]
V, A, PRF = 10.0, 2.0, 200.0


def _survey(**kw):
    sv = dict(waypoints=WP, deflector="fibre", n_fibres=2, scan_angle_rad=0.3, speed_mps=V, pulse_rate_hz=PRF,
              platform="multicopter", accel_mps2=A, t0=0.0, platform_noise_m=0.0, seed=1)
    sv.update(kw)
    return sv


def _controller(wp, v, a, dt):
    """Positions at the times k dt of a point that flies the legs one after the
    other, each from rest to rest: it brakes at `a` once its stopping distance
    reaches what is left of the leg, else speeds up at `a` to `v`.  Sub-steps of
    dt / 200 with the speed held over each; returns positions and the times the
    waypoints were reached."""
    h = dt / 200.0
    out, arrive = [np.array(wp[0], float)], [0.0]
    t, n_sub = 0.0, 0
    for i in range(len(wp) - 1):
        p0, p1 = np.array(wp[i], float), np.array(wp[i + 1], float)
        L = np.linalg.norm(p1 - p0)
        u = (p1 - p0) / L
        s, sp = 0.0, 0.0
        while True:
            left = L - s
            if left <= 1e-12 or (sp <= 0.0 and s > 0.0):
                break
            if sp * sp / (2.0 * a) >= left:
                acc = -a
            elif sp < v:
                acc = a
            else:
                acc = 0.0
            sp_new = min(max(sp + acc * h, 0.0), v)
            s = min(s + 0.5 * (sp + sp_new) * h, L)
            sp = sp_new
            t += h
            n_sub += 1
            if n_sub % 200 == 0:
                out.append(p0 + s * u)
        arrive.append(t)
    return np.array(out), np.array(arrive)


def test_legs_follow_the_controller(orc):
    wp = np.array(WP)
    n = 9000
    o, _ = orc.generate_pulses(_survey(), 0, n)
    ref, arrive = _controller(WP, V, A, 1.0 / PRF)
    m = min(len(ref), n)
    # braking decisions fall on the sub-step grid: a few centimetres at most
    err = np.linalg.norm(o[:m] - ref[:m], axis=1)
    assert err.max() < 0.03, err.max()
    # the long first leg reaches the cruise speed; the short second one does not
    L = np.linalg.norm(np.diff(wp, axis=0), axis=1)
    t_leg = np.diff(arrive)
    # (braking up to a sub-step late, the controller reaches a waypoint with up
    # to sqrt(2 a v dt / 200) left over and arrives that / a early: 0.016 s)
    assert abs(t_leg[0] - (L[0] / V + V / A)) < 0.03
    assert abs(t_leg[1] - 2.0 * np.sqrt(L[1] / A)) < 0.03
    # afterwards it stays at the last waypoint
    t = np.arange(n) / PRF
    assert np.array_equal(o[t > arrive[-1] + 0.01], np.tile(wp[-1], ((t > arrive[-1] + 0.01).sum(), 1)))


def test_speeds_and_accelerations(orc):
    n = 12000
    o, _ = orc.generate_pulses(_survey(), 0, n)
    dt = 1.0 / PRF
    vel = np.linalg.norm(np.diff(o, axis=0), axis=1) / dt
    assert vel.max() <= V + 1e-9
    assert abs(vel.max() - V) < 1e-9                           # the cruise of the first leg
    acc = np.diff(vel) / dt
    assert np.abs(acc).max() <= A * (1.0 + 1e-6)
    # the platform is at rest at each waypoint it turns at: the pulse closest to
    # the arrival is within a braking step of it, and the steps on either side
    # of that pulse (each within 2 dt of the stop) cover at most 2 a dt^2
    wp = np.array(WP)
    for i in (1, 2):
        k = np.argmin(np.linalg.norm(o - wp[i], axis=1))
        assert np.linalg.norm(o[k] - wp[i]) <= 0.5 * A * dt * dt + 1e-9
        assert vel[k - 1] <= 2 * A * dt + 1e-9 and vel[k] <= 2 * A * dt + 1e-9
    # the short leg tops out at sqrt(a L) half way along it
    L1 = np.linalg.norm(wp[2] - wp[1])
    seg = (o[:-1, 1] > 0.0) & (o[:-1, 1] < 16.0) & (np.abs(o[:-1, 0] - 400.0) < 1e-9)
    assert abs(vel[seg].max() - np.sqrt(A * L1)) < A * dt
    mid = np.argmax(np.where(seg, vel, 0.0))
    assert abs(o[mid, 1] - 8.0) < np.sqrt(A * L1) * dt


def test_huge_acceleration_is_the_linear_path(orc):
    n = 12000
    lin = orc.generate_pulses(_survey(platform="linear", accel_mps2=0.0), 0, n)
    cop = orc.generate_pulses(_survey(accel_mps2=1e9), 0, n)
    assert np.abs(cop[0] - lin[0]).max() < 1e-6
    # the headings agree except on a pulse that falls on a waypoint, which the
    # multicopter reaches 2 v / a later (still facing the leg it ends)
    wp = np.array(WP)
    change = np.cumsum(np.linalg.norm(np.diff(wp, axis=0), axis=1)) / V
    t = np.arange(n) / PRF
    away = np.min(np.abs(t[:, None] - change[None, :]), axis=1) > 1e-6
    assert (~away).sum() <= len(change)
    assert np.abs(cop[1][away] - lin[1][away]).max() < 1e-12


def test_leg_yaw(orc):
    ly = np.array([[0.0, 1.0], [1.0, 1.0], [2.5, -0.5]])
    n = 20000                                   # the path takes 97 s
    o, d = orc.generate_pulses(_survey(leg_yaw=ly), 0, n)
    _, d0 = orc.generate_pulses(_survey(), 0, n)
    # fibres at +-0.3: the direction is (-sin y sin a, cos y sin a, -cos a)
    a = np.where(np.arange(n) % 2 == 0, -0.3, 0.3)
    yaw = np.arctan2(-d[:, 0] / np.sin(a), d[:, 1] / np.sin(a))
    assert np.allclose(-d[:, 2], np.cos(0.3), atol=1e-12)
    wp = np.array(WP)
    L0 = np.linalg.norm(wp[1] - wp[0])
    T0 = L0 / V + V / A
    t = np.arange(n) / PRF
    first = t < T0 - 1e-9
    # the first leg turns from 0 to 1 rad at a constant rate in time (not in
    # distance, which would bend the yaw during the ramps)
    rate = np.diff(yaw[first]) * PRF
    assert np.allclose(rate, 1.0 / T0, rtol=1e-6)
    assert abs(yaw[0]) < 1e-12
    # the second leg holds 1 rad; the third ends at -0.5 and then stays
    k1 = np.searchsorted(t, T0 + 0.01)
    assert abs(yaw[k1] - 1.0) < 1e-12
    assert np.allclose(yaw[-50:], -0.5, atol=1e-12)
    # without leg yaws the platform faces each leg
    h = np.arctan2(-d0[:, 0] / np.sin(a), d0[:, 1] / np.sin(a))
    assert np.allclose(h[first], 0.0, atol=1e-12)
    assert abs(h[k1] - np.pi / 2) < 1e-12
    # the yaws do not move the platform
    _o0, _ = orc.generate_pulses(_survey(), 0, n)
    assert np.array_equal(o, _o0)


def test_multicopter_rejects(orc):
    with pytest.raises(ValueError):
        orc.generate_pulses(_survey(accel_mps2=0.0), 0, 10)
    with pytest.raises(ValueError):
        orc.generate_pulses(_survey(speed_mps=0.0), 0, 10)
    with pytest.raises(ValueError):
        orc.generate_pulses(_survey(platform="linear", leg_yaw=np.zeros((3, 2))), 0, 10)
    with pytest.raises(ValueError):
        orc.generate_pulses(_survey(leg_yaw=np.zeros((2, 2))), 0, 10)
    with pytest.raises(ValueError):
        orc.generate_pulses(_survey(waypoints=[WP[0], WP[1], WP[1], WP[2]]), 0, 10)   # a leg of length 0
    # one waypoint: static whatever the acceleration
    o, _ = orc.generate_pulses(_survey(waypoints=WP[:1], accel_mps2=0.0), 0, 5)
    assert np.array_equal(o, np.tile(WP[0], (5, 1)))
