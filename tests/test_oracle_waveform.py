"""Pins of the oracle's radiometry, pulse shape, waveform and returns
(Sec. 3.4 Eq. 1 and Eq. 3; Sec. 5.2 Eq. 7; Sec. 5.4 waveform length cap)."""
import math

import numpy as np
import pytest
from scipy.optimize import brentq

import synth
from synth import configs

C = 0.299792458  # m/ns, Sec. 3.4


def _big_plane(z=0.0, rho=0.5):
    return synth.flat_quad(-1e4, 1e4, -1e4, 1e4, z, reflectance=rho)


def test_gaussian_pulse_shape(orc):
    sc = configs.scanner(1e-3, 1, pulse_width_ns=4.0)
    assert orc.pulse_value(sc, 0.0) == 1.0
    assert abs(orc.pulse_value(sc, 2.0) - 0.5) < 1e-15      # FWHM 4 ns
    assert abs(orc.pulse_value(sc, -2.0) - 0.5) < 1e-15
    h = 1e-5
    for s in (-3.0, -0.7, 0.4, 2.5):
        fd = (orc.pulse_value(sc, s + h) - orc.pulse_value(sc, s - h)) / (2 * h)
        assert abs(orc.pulse_derivative(sc, s) - fd) < 1e-9


def test_eq3_pulse_shape(orc):
    # Eq. 3 with tau = pulse length / 1.75: peak 4 e^-2 at s = 2 tau
    L = 4.0
    tau = L / 1.75
    sc = configs.scanner(1e-3, 1, pulse_shape="eq3", pulse_width_ns=L)
    assert abs(orc.pulse_value(sc, 2 * tau) - 4 * math.exp(-2)) < 1e-15
    assert orc.pulse_value(sc, 0.0) == 0.0 and orc.pulse_value(sc, -1.0) == 0.0
    assert abs(orc.pulse_derivative(sc, 2 * tau)) < 1e-15
    # half-maximum points of x^2 e^-x, solved independently
    f = lambda x: x * x * math.exp(-x) - 2 * math.exp(-2)
    x1, x2 = brentq(f, 1e-6, 2.0), brentq(f, 2.0, 20.0)
    assert abs(orc.pulse_value(sc, x1 * tau) - 2 * math.exp(-2)) < 1e-14
    assert abs(orc.pulse_value(sc, x2 * tau) - 2 * math.exp(-2)) < 1e-14
    assert abs((x2 - x1) - 3.3947) < 1e-4
    h = 1e-5
    for s in (0.3, 2.0, 9.0):
        fd = (orc.pulse_value(sc, s + h) - orc.pulse_value(sc, s - h)) / (2 * h)
        assert abs(orc.pulse_derivative(sc, s) - fd) < 1e-9


def test_energy_conservation_perpendicular_facet(orc):
    # every subray hits one facet perpendicular to the beam at distance R0:
    # the summed power equals the single-ray value up to O(alpha_max^2)
    R0 = 250.0
    rho = 0.37
    m = _big_plane(0.0, rho)
    sc = configs.scanner(0.5e-3, 61, peak_power_w=2.0, receiver_diameter_m=0.3, efficiency=0.8)
    p = synth.Pulses(np.array([[3.0, 4.0, R0]]), np.array([[0, 0, -1]], np.float32))
    r = orc.simulate(m, p, sc)
    single = 2.0 * 0.8 * 0.3 ** 2 / 4.0 * rho / R0 ** 2
    amax = 0.25e-3
    assert np.all(r.sub_tri >= 0)
    assert abs(r.sub_power.sum() / single - 1.0) <= 2 * amax ** 2
    assert r.sub_power.sum() < single


def test_incidence_angle(orc):
    # a plane tilted by theta to the beam returns cos(theta) of the normal-incidence power
    R0 = 100.0
    theta = math.radians(60.0)
    m = _big_plane(0.0, 0.5)
    sc = configs.scanner(0.3e-3, 19)
    d = np.array([[math.sin(theta), 0.0, -math.cos(theta)]], np.float32)
    p = synth.Pulses(np.array([[0.0, 0.0, R0 * math.cos(theta)]]), d)
    r = orc.simulate(m, p, sc)
    single = 0.25 * 0.5 * math.cos(theta) / R0 ** 2
    assert abs(r.sub_power.sum() / single - 1.0) < 1e-6


def test_radar_equation_form(orc):
    # Eq. 7, I ~ lambda sigma P alpha^2 / (4 pi d^4 beta^2), with an extended
    # Lambertian target sigma = pi rho cos(theta) d^2 beta^2 (beta = divergence)
    mesh, pulses, sc = configs.small_tls()
    sc = dict(sc, peak_power_w=3.0, receiver_diameter_m=0.1, efficiency=0.6)
    r = orc.simulate(mesh, pulses.subset(np.arange(0, 10000, 97)), sc)
    a, phi, w = orc.pattern(sc)
    beta = sc["divergence_rad"]
    hit = r.sub_tri >= 0
    d = np.where(hit, r.sub_range, 1.0)
    rho = mesh.reflectance[np.where(hit, r.sub_tri, 0)].astype(np.float64)
    sigma = math.pi * rho * r.sub_cos * d ** 2 * beta ** 2
    I = 0.6 * sigma * (3.0 * w[None, :]) * 0.1 ** 2 / (4 * math.pi * d ** 4 * beta ** 2)
    assert np.allclose(r.sub_power[hit], I[hit], rtol=1e-13)
    assert np.all(r.sub_power[~hit] == 0)


@pytest.mark.parametrize("shape,width,bin_ns,tol", [("gaussian", 4.0, 1.0, 1e-9), ("gaussian", 4.0, 0.5, 1e-9),
                                                   ("eq3", 4.0, 0.25, 2e-4)])
def test_waveform_integral(orc, shape, width, bin_ns, tol):
    # sum_j wf_j * bin = sum_k P_k * integral of the pulse (whole pulse inside the window)
    m = _big_plane(0.0, 0.5)
    sc = configs.scanner(0.5e-3, 31, pulse_shape=shape, pulse_width_ns=width, bin_ns=bin_ns, n_bins=400)
    p = synth.Pulses(np.array([[0.0, 0.0, 80.0]]), np.array([[0.2, 0.1, -1.0]], np.float32) / np.float32(1.0247))
    r = orc.simulate(m, p, sc)
    if shape == "gaussian":
        sg = width / (2 * math.sqrt(2 * math.log(2)))
        integral = sg * math.sqrt(2 * math.pi)
    else:
        integral = 2.0 * width / 1.75    # Gamma(3) tau
    assert abs(r.waveform.sum() * bin_ns / (r.sub_power.sum() * integral) - 1.0) < tol


@pytest.mark.parametrize("shape", ["gaussian", "eq3"])
@pytest.mark.parametrize("beta_deg", [0.0, 25.0])
def test_single_plane_single_echo(orc, shape, beta_deg):
    h = 212.0
    m = _big_plane(0.0)
    bin_ns = 0.5
    sc = configs.scanner(0.5e-3, 31, pulse_shape=shape, bin_ns=bin_ns, n_bins=128)
    b = math.radians(beta_deg)
    p = synth.Pulses(np.array([[0.0, 0.0, h]]), np.array([[math.sin(b), 0.0, -math.cos(b)]], np.float32))
    r = orc.simulate(m, p, sc)
    assert r.n_returns[0] == 1
    assert abs(r.ret_range[0, 0] - h / math.cos(b)) <= bin_ns * C / 2
    assert r.ret_tri[0, 0] in (0, 1)
    assert r.ret_amp[0, 0] == r.waveform[0].max()
    # the window starts t_pre before the first return
    tmin = 2 * r.sub_range[0].min() / C
    assert abs(r.t0[0] - (tmin - orc.window_pre(sc))) < 1e-9


def test_two_planes_two_echoes(orc):
    # a half-plane occluder H above the ground, edge through the beam axis:
    # two echoes, separated by H within a bin, attributed to the right surfaces
    H = 6.0
    ground = _big_plane(0.0)
    occl = synth.flat_quad(-1e3, 0.0, -1e3, 1e3, H, reflectance=0.5)
    m = synth.merge_meshes([ground, occl])
    bin_ns = 0.5
    sc = configs.scanner(0.5e-3, 61, bin_ns=bin_ns, n_bins=256)
    p = synth.Pulses(np.array([[0.0, 0.3, 150.0]]), np.array([[0, 0, -1]], np.float32))
    r = orc.simulate(m, p, sc)
    assert r.n_returns[0] == 2
    r1, r2 = r.ret_range[0, :2]
    assert abs((r2 - r1) - H) <= bin_ns * C / 2
    assert abs(r1 - (150.0 - H)) <= bin_ns * C / 2
    assert r.ret_tri[0, 0] in (2, 3) and r.ret_tri[0, 1] in (0, 1)


def test_no_hit_pulse(orc):
    m = synth.flat_quad(0, 1, 0, 1, 0.0)
    sc = configs.scanner(0.5e-3, 19, n_bins=64)
    p = synth.Pulses(np.array([[10.0, 10.0, 5.0]]), np.array([[0, 0, -1]], np.float32))
    r = orc.simulate(m, p, sc)
    assert np.all(r.sub_tri == -1) and np.all(r.sub_power == 0)
    assert np.isnan(r.t0[0]) and np.all(r.waveform == 0) and r.n_returns[0] == 0
    assert np.all(r.ret_tri == -1) and np.all(r.ret_bin == -1)


def test_echoes_beyond_window_are_dropped(orc):
    # Sec. 5.4: the recorded waveform has a maximum length; later echoes are lost
    ground = _big_plane(0.0)
    occl = synth.flat_quad(-1e3, 0.0, -1e3, 1e3, 40.0)
    m = synth.merge_meshes([ground, occl])
    sc = configs.scanner(0.5e-3, 31, bin_ns=1.0, n_bins=64)   # 64 ns window < 2*40 m / c
    p = synth.Pulses(np.array([[0.0, 0.0, 150.0]]), np.array([[0, 0, -1]], np.float32))
    r = orc.simulate(m, p, sc)
    assert r.n_returns[0] == 1 and abs(r.ret_range[0, 0] - 110.0) < 0.5


def test_peak_detector_hand_cases(orc):
    assert list(orc.detect_peaks([0, 1, 0])) == [1]
    assert list(orc.detect_peaks([0, 2, 2, 0])) == [1]          # plateau: leftmost bin
    assert list(orc.detect_peaks([5, 1, 0, 0])) == []            # first bin is never a peak
    assert list(orc.detect_peaks([0, 0, 1, 5])) == []            # nor the last
    assert list(orc.detect_peaks([0, 3, 1, 2, 0, 1, 0])) == [1, 3, 5]
    # a rise onto a shelf counts (> on the left, >= on the right)
    assert list(orc.detect_peaks([0, 1, 1, 2, 0])) == [1, 3]
    assert list(orc.detect_peaks([0, 0, 0, 0])) == []
    assert list(orc.detect_peaks([1, 2, 3, 4])) == []
    # relative threshold: 1e-3 of the maximum
    assert list(orc.detect_peaks([0, 1000, 0, 0.5, 0, 1.0, 0])) == [1, 5]
    # absolute threshold
    assert list(orc.detect_peaks([0, 3, 0, 5, 0], thr_abs=4.0)) == [3]
    # the first K in time order
    wf = np.zeros(40)
    wf[2:40:4] = np.arange(1, 11)
    assert list(orc.detect_peaks(wf, K=8)) == [2, 6, 10, 14, 18, 22, 26, 30]
    assert list(orc.detect_peaks(wf, K=3)) == [2, 6, 10]


def test_attribution_rule(orc):
    # the return goes to the subray contributing most at the peak bin; equal
    # contributions go to the lowest subray index; misses never count
    sc = configs.scanner(0.5e-3, 4, bin_ns=1.0, n_bins=32)
    R = np.array([30.0, 30.0, 30.0, 31.0])
    tj = 2 * 30.0 / C
    assert orc.attribute(sc, [5, 6, 7, 8], R, [1.0, 2.0, 2.0, 9.0], tj) == 1
    assert orc.attribute(sc, [5, 6, 7, 8], R, [3.0, 3.0, 3.0, 0.0], tj) == 0
    assert orc.attribute(sc, [-1, 6, 7, 8], R, [3.0, 3.0, 3.0, 0.0], tj) == 1
    assert orc.attribute(sc, [-1, -1, -1, -1], R, [3.0, 3.0, 3.0, 0.0], tj) == -1
    # far in time from its own echo a strong subray loses to a weak one on time
    assert orc.attribute(sc, [5, 6, 7, 8], R, [1.0, 0.0, 0.0, 100.0], tj) == 0


def test_returns_are_prefix_of_larger_k(orc):
    # Sec. 3.4: the first K local maxima in time order are kept, so the returns
    # of a K-limited run are the first ones of any run with a larger K
    rng = np.random.default_rng(4)
    tiles = []
    for i in range(12):
        for j in range(12):
            x0, y0 = -3 + 0.5 * i, -3 + 0.5 * j
            tiles.append(synth.flat_quad(x0, x0 + 0.5, y0, y0 + 0.5, float(rng.uniform(0, 25)),
                                         float(rng.uniform(0.2, 0.8))))
    m = synth.merge_meshes(tiles)
    n = 6
    o = np.stack([rng.uniform(-1, 1, n), rng.uniform(-1, 1, n), np.full(n, 60.0)], 1)
    p = synth.Pulses(o, np.tile([[0.0, 0.0, -1.0]], (n, 1)).astype(np.float32))
    kw = dict(n_bins=1024, bin_ns=0.25)
    r4 = orc.simulate(m, p, configs.scanner(0.1, 64, max_returns=4, **kw))
    r16 = orc.simulate(m, p, configs.scanner(0.1, 64, max_returns=16, **kw))
    assert (r4.n_returns == 4).all() and (r16.n_returns > 4).all()
    for a, b in ((r4.ret_bin, r16.ret_bin), (r4.ret_range, r16.ret_range), (r4.ret_amp, r16.ret_amp),
                 (r4.ret_tri, r16.ret_tri)):
        assert np.array_equal(a, b[:, :4])
    assert np.array_equal(r4.waveform, r16.waveform)
    # the uncapped list of the waveform's maxima starts with the kept ones
    for q in range(n):
        full = orc.detect_peaks(r16.waveform[q], K=r16.waveform.shape[1])
        assert list(full[:r16.n_returns[q]]) == list(r16.ret_bin[q, :r16.n_returns[q]])
        # ranges of returns past the kept ones come from the same rule
        assert orc.echo_range(configs.scanner(0.1, 64, max_returns=16, **kw), r16.t0[q], int(full[0])) == \
            r16.ret_range[q, 0]


def test_echo_range_of_bin(orc):
    # a return at bin j lies at half the two-way time of the bin, less the
    # pulse's peak offset (0 for the Gaussian, 2 tau for Eq. 3)
    sc = configs.scanner(0.5e-3, 1, bin_ns=0.5)
    assert orc.echo_range(sc, 1000.0, 10) == pytest.approx(0.5 * C * 1005.0, rel=1e-15)
    L = 4.0
    sc3 = configs.scanner(0.5e-3, 1, bin_ns=0.5, pulse_shape="eq3", pulse_width_ns=L)
    assert orc.echo_range(sc3, 1000.0, 10) == pytest.approx(0.5 * C * (1005.0 - 2 * L / 1.75), rel=1e-15)
