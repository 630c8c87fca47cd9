"""Pins of the oracle's analytic gradient: central finite differences on the
FP64 forward (h = 1e-3) with the window origins held fixed and hit selection
discrete.  Parameters whose perturbation changes any subray's hit triangle
are excluded from the comparison (and counted)."""
import numpy as np
import pytest

import synth
from synth import configs


def _case(n=12, spacing=1.0, lines=6, per_line=7, S=7, shape="gaussian"):
    x = np.arange(n, dtype=np.float64) * spacing
    X, Y = np.meshgrid(x, x)
    h = synth.value_noise_field(X, Y, seed=99, octaves=3, base_wavelength=6.0, amplitude=1.5)
    mesh = synth.dtm_mesh(h, spacing, refl_seed=99)
    extent = (n - 1) * spacing
    y = 1.0 + (extent - 2.0) * np.arange(lines) / (lines - 1)
    pulses = synth.als_lines(extent / 2, y, 40.0, per_line, beta_deg=(-6.0, 6.0))
    sc = configs.scanner(2e-3, S, pulse_shape=shape, pulse_width_ns=4.0 if shape == "gaussian" else 3.0,
                         bin_ns=0.5, n_bins=96, peak_power_w=5e3)
    target = configs.diff_target(mesh, seed=5, dz=0.2, drho=0.05)
    return mesh, target, pulses, sc


def _loss(orc, mesh, pulses, sc, t0, tgt, spec=None):
    r = orc.simulate(mesh, pulses, sc, t0=t0, specular=spec)
    return float(np.sum((r.waveform - tgt) ** 2)), r.sub_tri


@pytest.mark.parametrize("shape,specular", [("gaussian", False), ("eq3", False), ("gaussian", True)])
def test_gradient_matches_finite_differences(orc, shape, specular):
    mesh, target, pulses, sc = _case(shape=shape)
    spec = None
    if specular:
        # a Phong-type part on every triangle: specularity 0.2-0.8, exponents 1-8
        rng = np.random.default_rng(17)
        spec = (rng.uniform(0.2, 0.8, mesh.n_triangles), rng.uniform(1.0, 8.0, mesh.n_triangles))
    base = orc.simulate(mesh, pulses, sc, specular=spec)
    t0 = base.t0
    tgt = orc.simulate(target, pulses, sc, t0=t0).waveform
    G = 2.0 * (base.waveform - tgt)
    gr, gz = orc.gradient(mesh, pulses, sc, t0, G, specular=spec)
    # the mirror lobe's higher derivatives are larger: a smaller step keeps the
    # central difference's O(h^2) error under the tolerance
    h = 2.5e-4 if specular else 1e-3
    scale = max(np.abs(gr).max(), np.abs(gz).max())
    excluded = 0
    compared = 0
    for v in range(mesh.n_vertices):
        mp = synth.Mesh(mesh.vertices.copy(), mesh.triangles, mesh.reflectance)
        mm = synth.Mesh(mesh.vertices.copy(), mesh.triangles, mesh.reflectance)
        mp.vertices[v, 2] += np.float32(h)
        mm.vertices[v, 2] -= np.float32(h)
        hh = (float(mp.vertices[v, 2]) - float(mm.vertices[v, 2])) / 2
        lp, tp = _loss(orc, mp, pulses, sc, t0, tgt, spec)
        lm, tm = _loss(orc, mm, pulses, sc, t0, tgt, spec)
        if not (np.array_equal(tp, base.sub_tri) and np.array_equal(tm, base.sub_tri)):
            excluded += 1
            continue
        fd = (lp - lm) / (2 * hh)
        assert abs(fd - gz[v]) <= 1e-4 * abs(gz[v]) + 1e-6 * scale, (v, fd, gz[v])
        compared += 1
    for t in range(mesh.n_triangles):
        rp = mesh.reflectance.astype(np.float64).copy()
        rm = rp.copy()
        rp[t] += h
        rm[t] -= h
        lp, _ = _loss(orc, synth.Mesh(mesh.vertices, mesh.triangles, rp.astype(np.float32)), pulses, sc, t0, tgt,
                      spec)
        lm, _ = _loss(orc, synth.Mesh(mesh.vertices, mesh.triangles, rm.astype(np.float32)), pulses, sc, t0, tgt,
                      spec)
        hh = (float(np.float32(rp[t])) - float(np.float32(rm[t]))) / 2
        fd = (lp - lm) / (2 * hh)
        # L is quadratic in each reflectance: the central difference is exact up to rounding
        assert abs(fd - gr[t]) <= 1e-6 * abs(gr[t]) + 1e-9 * scale, (t, fd, gr[t])
        compared += 1
    assert excluded <= mesh.n_vertices // 4
    assert compared > mesh.n_triangles
    # some gradient must be non-trivial for the comparison to mean anything
    assert np.count_nonzero(gz) > mesh.n_vertices // 4 and np.count_nonzero(gr) > 10


def test_flat_facet_height_gradient(orc):
    # a horizontal facet under a nadir beam: raising its three vertices by dz
    # shortens every range by dz, so sum_i dL/dz_i = -dL/dR for any loss; with
    # L = sum_j wf_j * g_j and a single subray, dL/dR = d/dR [P(R) p(t_j - 2R/c)]
    m = synth.flat_quad(-50, 50, -50, 50, 0.0, reflectance=0.5)
    sc = configs.scanner(1e-3, 1, bin_ns=0.5, n_bins=64, peak_power_w=1e4)
    p = synth.Pulses(np.array([[10.0, 20.0, 30.0]]), np.array([[0, 0, -1]], np.float32))
    base = orc.simulate(m, p, sc)
    g = np.linspace(-1.0, 1.0, 64)
    gr, gz = orc.gradient(m, p, sc, base.t0, g[None, :])
    # direct derivative of the closed form in R
    C = 0.299792458
    t0 = base.t0[0]
    sg = 4.0 / (2 * np.sqrt(2 * np.log(2)))

    def L(R):
        s = t0 + 0.5 * np.arange(64) - 2 * R / C
        return np.sum(g * 1e4 * 0.25 * 0.5 / R ** 2 * np.exp(-s * s / (2 * sg * sg)))

    dLdR = (L(30.0 + 1e-6) - L(30.0 - 1e-6)) / 2e-6
    assert abs(gz.sum() + dLdR) <= 1e-6 * abs(dLdR)
