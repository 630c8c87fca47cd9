"""Pins of the oracle's scene parts placed by affine maps (Sec. 3.5: one part
loaded several times and moved by transforms; Sec. 5.1: primitives rotate,
scale and translate)."""
import math

import numpy as np
import pytest

import synth
from synth import configs


def _aff(A=np.eye(3), t=(0.0, 0.0, 0.0)):
    return np.hstack([np.asarray(A, np.float64), np.asarray(t, np.float64)[:, None]])


def test_exact_maps(orc):
    mesh = configs.small_tls()[0]
    v = mesh.vertices
    # identity, a quarter turn about z, a translation by whole metres and a
    # doubling are exact in FP32 on this grid
    rot = np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    cases = [(_aff(), v), (_aff(rot), np.stack([-v[:, 1], v[:, 0], v[:, 2]], 1)),
             (_aff(t=(64.0, -32.0, 0.0)), v + np.array([64.0, -32.0, 0.0], np.float32)),
             (_aff(2.0 * np.eye(3)), 2.0 * v)]
    for aff, want in cases:
        m = orc.instance_mesh([mesh], [(0, aff)])
        assert np.array_equal(m.vertices, want.astype(np.float32))
        assert np.array_equal(m.triangles, mesh.triangles) and np.array_equal(m.reflectance, mesh.reflectance)


def test_general_map_and_layout(orc):
    rng = np.random.default_rng(2)
    a = synth.flat_quad(-3.0, 3.0, -2.0, 2.0, 1.0, reflectance=0.3)
    b = configs.small_tls()[0]
    insts = []
    for i in range(5):
        th = rng.uniform(0, 2 * np.pi)
        R = np.array([[math.cos(th), -math.sin(th), 0.0], [math.sin(th), math.cos(th), 0.0], [0.0, 0.0, 1.0]])
        s = rng.uniform(0.5, 2.0)
        insts.append((i % 2, _aff(s * R, rng.uniform(-100, 100, 3))))
    m = orc.instance_mesh([a, b], insts)
    parts = [a, b]
    vo = 0
    to = 0
    for p, aff in insts:
        pv = parts[p].vertices.astype(np.float64)
        want = pv @ aff[:, :3].T + aff[:, 3]
        got = m.vertices[vo:vo + pv.shape[0]].astype(np.float64)
        # one rounding to FP32 of the FP64 map (the sum order may differ in the last FP64 bits)
        assert np.all(np.abs(got - want) <= np.spacing(np.abs(want).astype(np.float32)) * 0.5 + 1e-9)
        nt = parts[p].n_triangles
        assert np.array_equal(m.triangles[to:to + nt], parts[p].triangles + vo)
        assert np.array_equal(m.reflectance[to:to + nt], parts[p].reflectance)
        vo += pv.shape[0]
        to += nt
    assert m.n_vertices == vo and m.n_triangles == to


def test_moved_copy_sees_moved_pulses(orc):
    # a copy moved by t, scanned by pulses moved by t, gives the same echoes
    # with ids offset by the first copy's triangles
    mesh, pulses, sc = configs.small_tls(n_az=20, n_el=10)
    t = np.array([512.0, 256.0, 0.0])
    scene = orc.instance_mesh([mesh], [(0, _aff()), (0, _aff(t=t))])
    r0 = orc.simulate(mesh, pulses, sc)
    moved = synth.Pulses(pulses.origins + t, pulses.directions)
    r1 = orc.simulate(scene, moved, sc)
    nt = mesh.n_triangles
    hit = r0.sub_tri >= 0
    assert hit.mean() > 0.5
    assert np.array_equal(r1.sub_tri[hit], r0.sub_tri[hit] + nt) and (r1.sub_tri[~hit] == -1).all()
    assert np.array_equal(r1.sub_range, r0.sub_range)
    assert np.array_equal(r1.waveform, r0.waveform)


def test_mirrored_copy_still_hit(orc):
    # a map with a negative determinant reverses the winding; the test is
    # two-sided, so vertical rays still hit the mirrored quad at its height
    q = synth.flat_quad(-5.0, 5.0, -5.0, 5.0, 2.0, reflectance=0.5)
    m = orc.instance_mesh([q], [(0, _aff(np.diag([-1.0, 1.0, 1.0])))])
    sc = configs.scanner(1e-3, 7, n_bins=64)
    o = np.array([[0.5, 0.25, 10.0], [-3.0, 1.0, 10.0]])
    d = np.tile([[0.0, 0.0, -1.0]], (2, 1)).astype(np.float32)
    r = orc.simulate(m, synth.Pulses(o, d), sc)
    assert (r.sub_tri >= 0).all()
    assert np.allclose(r.sub_range[:, 0], 8.0, atol=1e-12)
