"""Pins of the oracle's Phong-type specular response (Sec. 5.1: materials carry
reflectance and specularity): f = (1 - ks) cos theta + ks max(cos 2 theta, 0)^n
for a receiver at the emitter, where the mirror direction makes 2 theta with
the way back."""
import math

import numpy as np
import pytest

import synth
from synth import configs


def test_response_special_cases(orc):
    rng = np.random.default_rng(1)
    for _ in range(200):
        ct, ks, n = rng.uniform(0, 1), rng.uniform(0, 1), rng.uniform(0, 50)
        # no specularity: Lambert's cosine
        assert orc.surface_response(ct, 0.0, n) == ct
        # normal incidence returns everything whatever the split
        assert orc.surface_response(1.0, ks, n) == pytest.approx(1.0, abs=1e-15)
        # beyond 45 degrees the mirror lobe points away: only the diffuse part remains
        c45 = rng.uniform(0, math.sqrt(0.5))
        assert orc.surface_response(c45, ks, n) == pytest.approx((1 - ks) * c45, abs=1e-15)
    # exponent 1: the lobe is cos 2 theta itself; a wider lobe (smaller n) returns more off normal
    th = math.radians(20.0)
    assert orc.surface_response(math.cos(th), 1.0, 1.0) == pytest.approx(math.cos(2 * th), abs=1e-15)
    assert orc.surface_response(math.cos(th), 1.0, 2.0) < orc.surface_response(math.cos(th), 1.0, 1.0)
    # the response falls off monotonically from normal incidence
    cs = np.linspace(0.01, 1.0, 200)
    f = [orc.surface_response(c, 0.6, 12.0) for c in cs]
    assert np.all(np.diff(f) > 0)


def test_specular_power_on_planes(orc):
    # vertical rays on planes tilted by 10 and 60 degrees about x: the first sees
    # (1 - ks) cos 10 + ks cos(20)^n times the diffuse power per unit cos, the
    # second (1 - ks) cos 60 (its mirror lobe points away)
    sc = configs.scanner(1e-4, 1, n_bins=64)
    o = np.array([[0.0, 0.0, 30.0]])
    d = np.array([[0.0, 0.0, -1.0]], np.float32)
    for deg in (10.0, 60.0):
        t = math.radians(deg)
        v = np.array([[-5, -5 * math.cos(t), -5 * math.sin(t)], [5, -5 * math.cos(t), -5 * math.sin(t)],
                      [5, 5 * math.cos(t), 5 * math.sin(t)], [-5, 5 * math.cos(t), 5 * math.sin(t)]], np.float32)
        tri = np.array([[0, 1, 2], [0, 2, 3]], np.int32)
        mesh = synth.Mesh(v, tri, np.full(2, 0.5, np.float32))
        lam = orc.simulate(mesh, synth.Pulses(o, d), sc)
        ks, n = float(np.float32(0.7)), 6.0          # the materials are FP32
        spec = orc.simulate(mesh, synth.Pulses(o, d), sc, specular=(np.full(2, ks), np.full(2, n)))
        ct = lam.sub_cos[0, 0]
        assert ct == pytest.approx(math.cos(t), abs=1e-6)
        ratio = spec.sub_power[0, 0] / lam.sub_power[0, 0]
        want = ((1 - ks) * ct + ks * max(2 * ct * ct - 1, 0.0) ** n) / ct
        assert ratio == pytest.approx(want, rel=1e-12)
        if deg > 45:
            assert ratio == pytest.approx(1 - ks, rel=1e-12)
    # zero specularity is bitwise the Lambertian forward
    mesh, pulses, sc = configs.small_tls(n_az=20, n_el=10)
    a = orc.simulate(mesh, pulses, sc)
    b = orc.simulate(mesh, pulses, sc, specular=(np.zeros(mesh.n_triangles), np.full(mesh.n_triangles, 5.0)))
    assert np.array_equal(a.waveform, b.waveform) and np.array_equal(a.sub_power, b.sub_power)
