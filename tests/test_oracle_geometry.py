"""Pins of the oracle's ray casting (Sec. 3.4 first hit; Sec. 5.1 minimum distance)."""
import numpy as np
import pytest

import synth
from synth import configs


A = (0.0, 0.0, 0.0)
B = (1.0, 0.0, 0.0)
C = (0.0, 1.0, 0.0)


def test_hand_cases(orc):
    hit, t, u, v = orc.ray_triangle((0.25, 0.25, 1.0), (0, 0, -1), A, B, C)
    assert hit and t == 1.0 and u == 0.25 and v == 0.25
    # from below (back face) still hits: the test is two-sided
    hit, t, u, v = orc.ray_triangle((0.25, 0.5, -2.0), (0, 0, 1), A, B, C)
    assert hit and t == 2.0 and (u, v) == (0.25, 0.5)
    # vertices and edges are inclusive
    for x, y in [(0, 0), (1, 0), (0, 1), (0.5, 0), (0, 0.5), (0.5, 0.5)]:
        hit, t, u, v = orc.ray_triangle((x, y, 3.0), (0, 0, -1), A, B, C)
        assert hit and t == 3.0
    # outside
    for x, y in [(0.6, 0.6), (-0.01, 0.5), (0.5, -0.01), (1.01, 0.0)]:
        assert not orc.ray_triangle((x, y, 3.0), (0, 0, -1), A, B, C)[0]
    # parallel to the plane: no hit
    assert not orc.ray_triangle((0.2, 0.2, 1.0), (1, 0, 0), A, B, C)[0]
    assert not orc.ray_triangle((-1.0, 0.2, 0.0), (1, 0, 0), A, B, C)[0]
    # pointing away, and starting on the plane: only t > 0 counts
    assert not orc.ray_triangle((0.25, 0.25, 1.0), (0, 0, 1), A, B, C)[0]
    assert not orc.ray_triangle((0.25, 0.25, 0.0), (0, 0, -1), A, B, C)[0]
    # oblique: t scales with the path length
    d = np.array([0.6, 0.0, -0.8])
    hit, t, u, v = orc.ray_triangle((0.1 - 0.6 * 5, 0.2, 4.0), d, A, B, C)
    assert hit and abs(t - 5.0) < 1e-14 and abs(u - 0.1) < 1e-14 and abs(v - 0.2) < 1e-14


def test_closest_and_ties(orc):
    m0 = synth.flat_quad(-1, 1, -1, 1, 0.0)
    m1 = synth.flat_quad(-1, 1, -1, 1, 2.0)
    m = synth.merge_meshes([m0, m1])
    h, t, u, v = orc.closest_hit((0.3, 0.1, 5.0), (0, 0, -1), m)
    assert h in (2, 3) and t == 3.0
    h, t, u, v = orc.closest_hit((0.3, 0.1, -5.0), (0, 0, 1), m)
    assert h in (0, 1) and t == 5.0
    # an exact duplicate: the lower index wins
    dup = synth.merge_meshes([m1, m1])
    h, t, u, v = orc.closest_hit((0.3, 0.1, 5.0), (0, 0, -1), dup)
    assert h in (0, 1)
    # on the shared diagonal both triangles hit at the same t: lower index
    h, t, u, v = orc.closest_hit((0.25, 0.25, 5.0), (0, 0, -1), m1)
    assert h == 0
    # miss
    assert orc.closest_hit((3.0, 3.0, 5.0), (0, 0, -1), m)[0] == -1


def test_dtm_vertical_rays_closed_form(orc):
    # heightfield: the covering triangle and its height follow from the grid
    # cell and the side of its diagonal, independently of any ray test
    mesh, _, _ = configs.small_tls()
    n = 64
    z = mesh.vertices[:, 2].astype(np.float64).reshape(n, n)
    rng = np.random.default_rng(5)
    checked = 0
    while checked < 300:
        x, y = rng.uniform(0, n - 1, 2)
        i, j = int(x), int(y)
        fx, fy = x - i, y - j
        if min(fx, fy, 1 - fx, 1 - fy, abs(fx - fy)) < 1e-3:
            continue
        z00, z10, z01, z11 = z[j, i], z[j, i + 1], z[j + 1, i], z[j + 1, i + 1]
        if fx >= fy:
            zz = z00 + fx * (z10 - z00) + fy * (z11 - z10)
            tid = 2 * (j * (n - 1) + i)
        else:
            zz = z00 + fy * (z01 - z00) + fx * (z11 - z01)
            tid = 2 * (j * (n - 1) + i) + 1
        h, t, u, v = orc.closest_hit((x, y, 50.0), (0, 0, -1), mesh)
        assert h == tid
        assert abs(t - (50.0 - zz)) < 1e-12
        checked += 1


@pytest.mark.parametrize("beta_deg", [0.0, 17.0, 41.0])
def test_flat_plane_range(orc, beta_deg):
    # sensor at height h over z = 0: every subray's range is h / |d_k . z|
    h = 123.25
    m = synth.flat_quad(-1e4, 1e4, -1e4, 1e4, 0.0)
    b = np.deg2rad(beta_deg)
    d = np.array([np.sin(b), 0.0, -np.cos(b)], np.float32)
    p = synth.Pulses(np.array([[1.5, -2.0, h]]), d[None, :])
    sc = configs.scanner(5e-3, 37, n_bins=64)
    r = orc.simulate(m, p, sc)
    D = orc.subray_directions(d.astype(np.float64), sc)
    assert np.all(r.sub_tri[0] >= 0)
    assert np.allclose(r.sub_range[0], h / np.abs(D[:, 2]), rtol=1e-14, atol=0)
    # incidence: cos(theta) = |d_k . z|
    assert np.allclose(r.sub_cos[0], np.abs(D[:, 2]), rtol=1e-14)


def test_tilted_plane_range(orc):
    # plane through P0 with normal n: R = ((P0 - O).n) / (d.n)
    n = np.array([0.3, -0.2, 1.0])
    n /= np.linalg.norm(n)
    P0 = np.array([2.0, 3.0, -1.0])
    u = np.cross(n, [1.0, 0, 0])
    u /= np.linalg.norm(u)
    v = np.cross(n, u)
    L = 500.0
    corners = np.array([P0 - L * u - L * v, P0 + L * u - L * v, P0 + L * u + L * v, P0 - L * u + L * v])
    m = synth.Mesh(corners.astype(np.float32), np.array([[0, 1, 2], [0, 2, 3]], np.int32),
                   np.full(2, 0.4, np.float32))
    O = np.array([0.5, 0.25, 60.0])
    d = np.array([0.1, 0.05, -1.0], np.float32)
    p = synth.Pulses(O[None, :], d[None, :])
    sc = configs.scanner(3e-3, 19, n_bins=64)
    r = orc.simulate(m, p, sc)
    D = orc.subray_directions(d.astype(np.float64), sc)
    assert np.all(r.sub_tri[0] >= 0)
    for k in range(D.shape[0]):
        # the plane of the hit triangle, as stored in float32
        V = m.vertices[m.triangles[r.sub_tri[0, k]]].astype(np.float64)
        nf = np.cross(V[1] - V[0], V[2] - V[0])
        expect = ((V[0] - O) @ nf) / (D[k] @ nf)
        assert abs(r.sub_range[0, k] - expect) <= 1e-12 * expect


def test_watertight_shared_edges_and_vertices(orc):
    # Sec. 3.4: a subray that reaches a closed surface produces a return.  Rays
    # along shared edges and through shared vertices of the terrain must hit.
    mesh, pulses, sc = configs.small_tls()
    for x in (17.0, 32.0, 40.0):
        for y in (17.0, 32.0, 40.0):
            for d in ((0.0, 0.0, -1.0), (0.6, 0.0, -0.8), (0.0, -0.6, -0.8), (0.6, 0.6, -0.52915026)):
                h, t, u, v = orc.closest_hit((x, y, 10.0), d, mesh)
                assert h >= 0, (x, y, d)
    # the terrestrial grid looks along grid lines at azimuth 0, 90, 180, 270
    # degrees; its steeper pulses land well inside the terrain
    sel = np.concatenate([a * 100 + np.arange(0, 50) for a in (0, 25, 50, 75)])
    r = orc.simulate(mesh, pulses.subset(sel), sc)
    assert np.all(r.sub_tri >= 0)
