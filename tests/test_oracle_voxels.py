"""Pins of the oracle's transmissive voxels (Sec. 3.5.4 and Sec. 5.2: extinction
from plant area density through a leaf-angle table (Eq. 5, Table 2), a random
depth s = -ln(u) / sigma (Eq. 6), continuation through the voxels along the ray
(Sec. 5.1), echo power by Eq. 7)."""
import math
import os

import numpy as np
import pytest

import synth
from synth import configs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table2_erectophile_lut.txt")


def _table2():
    rows = np.loadtxt(GOLDEN)
    return rows[:, [1, 2]]          # (vertical component, g)


def _grid(pad, size=1.0, origin=(0.0, 0.0, 0.0), lut=None, seed=7):
    return dict(origin=list(origin), size=size, pad=np.asarray(pad, np.float32),
                lut=[[0.0, 0.5], [1.0, 0.5]] if lut is None else lut, seed=seed)


def test_table2_rows_and_interpolation(orc):
    lut = _table2()
    vox = _grid(np.zeros((1, 1, 1)), lut=lut)
    # the printed rows come back exactly; the table is symmetric in the beam's
    # vertical sense; between rows it is linear; beyond the ends it is held
    for v, g in lut:
        assert orc.lut_g(vox, v) == pytest.approx(g, abs=1e-15)
        assert orc.lut_g(vox, -v) == pytest.approx(g, abs=1e-15)
    mid = 0.5 * (lut[1, 0] + lut[2, 0])
    assert orc.lut_g(vox, mid) == pytest.approx(0.5 * (lut[1, 1] + lut[2, 1]), abs=1e-15)
    f = (0.5 - lut[2, 0]) / (lut[3, 0] - lut[2, 0])
    assert orc.lut_g(vox, 0.5) == pytest.approx(lut[2, 1] + f * (lut[3, 1] - lut[2, 1]), abs=1e-15)
    assert orc.lut_g(vox, 1.0) == pytest.approx(0.848822, abs=1e-15)


def test_transmission_through_a_slab(orc):
    # Beer-Lambert: a ray crossing length L of extinction sigma passes with
    # probability exp(-sigma L); the depths of the stops follow the truncated
    # exponential
    pad = np.full((3, 3, 8), 0.6, np.float32)         # 8 voxels along x
    vox = _grid(pad, size=0.5)
    sigma = 0.6 * 0.5
    L = 8 * 0.5
    n = 20000
    hits = [orc.voxel_hit(vox, [-1.0, 0.75, 0.75], [1.0, 0.0, 0.0], math.inf, p, 3) for p in range(n)]
    v = np.array([h[0] for h in hits])
    t = np.array([h[1] for h in hits])
    p_pass = math.exp(-sigma * L)
    frac = (v < 0).mean()
    assert abs(frac - p_pass) < 4 * math.sqrt(p_pass * (1 - p_pass) / n)
    depth = t[v >= 0] - 1.0
    mean_trunc = 1 / sigma - L * p_pass / (1 - p_pass)
    assert abs(depth.mean() - mean_trunc) < 4 * depth.std() / math.sqrt(depth.size)
    # the stopping voxel is the one the depth lies in
    assert np.array_equal(v[v >= 0] % 8, np.minimum(np.floor(depth / 0.5), 7).astype(int))


def _first_wall(pad, origin, size, O, d, t_max):
    """The first voxel with pad > 0 along the ray and its entry distance, by
    dense sampling (independent of the oracle's walk)."""
    nz, ny, nx = pad.shape
    ts = np.arange(0.0, t_max, size * 1e-4)
    p = np.asarray(O)[None, :] + ts[:, None] * np.asarray(d)[None, :]
    idx = np.floor((p - np.asarray(origin)[None, :]) / size).astype(int)
    inside = np.all((idx >= 0) & (idx < np.array([nx, ny, nz])[None, :]), axis=1)
    for k in np.nonzero(inside)[0]:
        ix, iy, iz = idx[k]
        if pad[iz, iy, ix] > 0:
            return ix + nx * (iy + ny * iz), ts[k]
    return -1, None


def test_walk_visits_voxels_in_order(orc):
    # walls of huge density stop every ray at their entry: the voxel reached
    # first along random rays, and the distance, agree with dense sampling
    rng = np.random.default_rng(4)
    pad = np.zeros((6, 7, 9), np.float32)
    walls = rng.random(pad.shape) < 0.08
    pad[walls] = 1e12
    origin, size = (-2.0, 1.0, 0.5), 0.7
    vox = _grid(pad, size=size, origin=origin)
    for q in range(150):
        O = np.array(origin) + rng.uniform(-1.0, 1.0, 3) * np.array([9, 7, 6]) * size
        d = rng.normal(size=3)
        if q % 5 == 0:
            d[q % 3] = 0.0                              # rays parallel to a face
        d /= np.linalg.norm(d)
        vi, t, _ = orc.voxel_hit(vox, O, d, math.inf, q, 0)
        ref, tref = _first_wall(pad, origin, size, O, d, 30.0)
        assert vi == ref, (q, vi, ref)
        if ref >= 0:
            assert abs(t - tref) <= size * 1e-4 + 1e-9
    # rays that start on a voxel boundary and run almost along it, either side
    for q in range(60):
        O = np.array(origin) + (rng.integers(1, 6, 3) + rng.uniform(0.2, 0.8, 3)) * size
        ax = q % 3
        O[ax] = origin[ax] + rng.integers(1, 6) * size            # exactly on a boundary plane
        d = np.zeros(3)
        d[(ax + 1) % 3] = rng.choice([-1.0, 1.0])
        d[ax] = rng.choice([-1e-19, 1e-19])
        d /= np.linalg.norm(d)
        vi, t, _ = orc.voxel_hit(vox, O, d, math.inf, q, 1)
        side = O.copy()
        side[ax] += np.sign(d[ax]) * size * 1e-6                  # the side the ray lies on
        ref, tref = _first_wall(pad, origin, size, side, d, 30.0)
        assert vi == ref, (q, vi, ref)


def test_triangle_in_front_wins(orc):
    pad = np.full((2, 2, 2), 5.0, np.float32)
    vox = _grid(pad, size=1.0)
    # the limit (a triangle hit) before the grid: no voxel
    assert orc.voxel_hit(vox, [-3.0, 0.5, 0.5], [1.0, 0.0, 0.0], 2.5, 0, 0)[0] == -1
    # a limit inside the first voxel cuts its length: stops beyond it are not taken
    for p in range(200):
        vi, t, _ = orc.voxel_hit(vox, [-1.0, 0.5, 0.5], [1.0, 0.0, 0.0], 1.2, p, 0)
        assert vi == -1 or t <= 1.2


def test_voxel_echo_power_and_ids(orc):
    # a scene of one far plane behind a voxel slab: subrays that stop in a voxel
    # report id n_tri + voxel, cos 1 and the power of Eq. 7
    plane = synth.flat_quad(-50.0, 50.0, -50.0, 50.0, 0.0, reflectance=0.5)
    pad = np.full((2, 4, 4), 0.4, np.float32)
    vox = _grid(pad, size=2.0, origin=(-4.0, -4.0, 10.0), lut=[[0.0, 0.3], [1.0, 0.7]], seed=11)
    sc = configs.scanner(2e-3, 19, n_bins=256, bin_ns=0.5)
    o = np.tile([[0.0, 0.0, 40.0]], (200, 1))
    d = np.tile([[0.0, 0.0, -1.0]], (200, 1)).astype(np.float32)
    pulses = synth.Pulses(o, d)
    r = orc.simulate(plane, pulses, sc, voxels=vox)
    n_tri = plane.n_triangles
    vh = r.sub_tri >= n_tri
    assert vh.mean() > 0.3 and (r.sub_tri[~vh] >= 0).all()
    # every subray draws its own depths: within one pulse (whose subrays cross
    # the same voxels) some stop and some pass, as for independent trials
    per_pulse = vh.sum(axis=1)
    assert np.mean((per_pulse > 0) & (per_pulse < vh.shape[1])) > 0.9
    pat_w = orc.pattern(sc)[2]
    beta = sc["divergence_rad"]
    for q, k in zip(*np.nonzero(vh)):
        R = r.sub_range[q, k]
        assert 26.0 <= R <= 30.0 + 1e-9
        sig = float(np.float32(0.4)) * (0.3 + 0.4 * abs(orc.subray_directions(d[q].astype(np.float64), sc)[k][2]))
        P = sc["efficiency"] * sig * sc["peak_power_w"] * pat_w[k] * sc["receiver_diameter_m"] ** 2 / (
            4 * math.pi * R ** 4 * beta ** 2)
        assert r.sub_power[q, k] == pytest.approx(P, rel=1e-12)
        assert r.sub_cos[q, k] == 1.0
    # without voxels (or with empty ones) every subray reaches the plane
    r0 = orc.simulate(plane, pulses, sc)
    re = orc.simulate(plane, pulses, sc, voxels=_grid(np.zeros((2, 4, 4)), size=2.0, origin=(-4.0, -4.0, 10.0)))
    assert np.array_equal(r0.sub_tri, re.sub_tri) and np.array_equal(r0.waveform, re.waveform)
    # the same seed gives the same draws; another seed others
    r2 = orc.simulate(plane, pulses, sc, voxels=vox)
    assert np.array_equal(r.sub_tri, r2.sub_tri)
    r3 = orc.simulate(plane, pulses, sc, voxels=dict(vox, seed=12))
    assert not np.array_equal(r.sub_tri, r3.sub_tri)


def test_degenerate_rays_and_grids(orc):
    vox = _grid(np.full((2, 2, 2), 3.0, np.float32))
    # a ray that is not finite meets nothing
    for O, d in [([np.nan, 0.5, 0.5], [1.0, 0.0, 0.0]), ([-1.0, 0.5, 0.5], [np.nan, 0.0, 0.0]),
                 ([-1.0, 0.5, np.inf], [1.0, 0.0, 0.0])]:
        assert orc.voxel_hit(vox, O, d, math.inf, 0, 0)[0] == -1
    # a ray parallel to a face outside the grid, a ray pointing away, and one
    # starting beyond its far side meet nothing
    assert orc.voxel_hit(vox, [-1.0, 2.5, 0.5], [1.0, 0.0, 0.0], math.inf, 0, 0)[0] == -1
    assert orc.voxel_hit(vox, [-1.0, 0.5, 0.5], [-1.0, 0.0, 0.0], math.inf, 0, 0)[0] == -1
    assert orc.voxel_hit(vox, [3.0, 0.5, 0.5], [1.0, 0.0, 0.0], math.inf, 0, 0)[0] == -1
    # a ray starting inside stops at depths measured from its origin
    ts = [orc.voxel_hit(vox, [0.5, 0.5, 0.5], [1.0, 0.0, 0.0], math.inf, p, 0) for p in range(4000)]
    t = np.array([x[1] for x in ts if x[0] >= 0])
    sigma = 3.0 * 0.5
    assert abs(np.mean(np.array([x[0] for x in ts]) < 0) - math.exp(-1.5 * sigma)) < 0.02
    assert t.min() >= 0.0 and t.max() <= 1.5


def test_voxel_gradient_is_the_triangles_alone(orc):
    # voxel echoes depend on neither reflectance nor heights: with a grid that
    # stops every subray the gradient vanishes; with an empty one it is the
    # gradient without voxels
    mesh = synth.flat_quad(-50.0, 50.0, -50.0, 50.0, 0.0, reflectance=0.5)
    sc = configs.scanner(2e-3, 19, n_bins=128, bin_ns=0.5)
    o = np.tile([[0.3, -0.2, 30.0]], (6, 1))
    d = np.tile([[0.05, 0.02, -1.0]], (6, 1)).astype(np.float32)
    pulses = synth.Pulses(o, d)
    base = orc.simulate(mesh, pulses, sc)
    G = np.random.default_rng(1).normal(size=base.waveform.shape)
    gr0, gz0 = orc.gradient(mesh, pulses, sc, base.t0, G, threads=1)
    assert np.abs(gr0).max() > 0
    empty = _grid(np.zeros((2, 2, 2), np.float32), size=4.0, origin=(-4.0, -4.0, 10.0))
    gr1, gz1 = orc.gradient(mesh, pulses, sc, base.t0, G, threads=1, voxels=empty)
    assert np.array_equal(gr0, gr1) and np.array_equal(gz0, gz1)
    wall = _grid(np.full((2, 2, 2), 1e9, np.float32), size=4.0, origin=(-4.0, -4.0, 10.0))
    assert (orc.simulate(mesh, pulses, sc, voxels=wall).sub_tri >= mesh.n_triangles).all()
    gr2, gz2 = orc.gradient(mesh, pulses, sc, base.t0, G, voxels=wall)
    assert not gr2.any() and not gz2.any()


def test_voxel_forest_workload():
    mesh, vox, pulses, sc = configs.uls_voxels(n_lines=2, per_line=10)
    pad = vox["pad"]
    nz, ny, nx = pad.shape
    assert (nx, ny) == (400, 400) and vox["size"] == 0.5
    assert pad.dtype == np.float32 and pad.min() >= 0.0 and 0.05 < (pad > 0).mean() < 0.8
    # the grid is tight around the crowns: they reach its lowest and highest layers
    assert pad[0].any() and pad[-1].any()
    assert mesh.n_triangles + pad.size < 2**31
