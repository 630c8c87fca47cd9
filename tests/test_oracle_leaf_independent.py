"""The oracle's closest hit against an independent one on real workloads.

The oracle tests triangles with the watertight test of Woop, Benthin & Wald
(2013).  Here a separate brute force in numpy uses the test of Moller &
Trumbore (1997) in FP64 (inclusive edges, a zero determinant misses, t > 0,
the smallest t wins, equal t goes to the lower index) over every triangle of
the small terrestrial workload (a sample of its subrays) and of the ALS scene
with buildings (a few pulses).  The two must give the same triangle except
where the hit lies within 1e-6 (barycentric) of an edge of either triangle,
and the same distance to 1e-12 relative on equal triangles (Sec. 3.4: a hit
ends the subray; Sec. 5.1: the minimum-distance intersection).
"""
import numpy as np

import oracle
import synth
from synth import configs

EDGE = 1e-6


class Tris:
    """FP64 copies of a mesh's triangles, with the edges Moller-Trumbore uses."""

    def __init__(self, mesh):
        V = mesh.vertices.astype(np.float64)[mesh.triangles]
        self.v0 = V[:, 0]
        self.e1 = V[:, 1] - V[:, 0]
        self.e2 = V[:, 2] - V[:, 0]
        lo, hi = V.min(axis=1), V.max(axis=1)
        self.centre = 0.5 * (lo + hi)
        self.radius = 0.5 * np.linalg.norm(hi - lo, axis=1)


def mt_closest(O, d, T, idx=None):
    """Closest hit of the ray O + t d over the triangles `idx` (all by default):
    (index or -1, t, u, v) with the barycentrics of the winner."""
    if idx is None:
        idx = np.arange(T.v0.shape[0])
    v0, e1, e2 = T.v0[idx], T.e1[idx], T.e2[idx]
    p = np.cross(d, e2)
    det = np.einsum("ij,ij->i", e1, p)
    ok = det != 0.0
    inv = np.where(ok, 1.0 / np.where(ok, det, 1.0), 0.0)
    s = O - v0
    u = np.einsum("ij,ij->i", s, p) * inv
    q = np.cross(s, e1)
    v = (q @ d) * inv
    t = np.einsum("ij,ij->i", e2, q) * inv
    hit = ok & (u >= 0.0) & (v >= 0.0) & (u + v <= 1.0) & (t > 0.0)
    if not hit.any():
        return -1, np.inf, 0.0, 0.0
    th = np.where(hit, t, np.inf)
    tmin = th.min()
    cand = idx[th == tmin]
    best = int(cand.min())
    j = int(np.nonzero(idx == best)[0][0])
    return best, float(t[j]), float(u[j]), float(v[j])


def bary_min(O, d, T, i):
    """Smallest barycentric coordinate of the ray's crossing of triangle i's
    plane (no inside test; -inf for a ray parallel to the plane)."""
    p = np.cross(d, T.e2[i])
    det = float(T.e1[i] @ p)
    if det == 0.0:
        return -np.inf
    s = O - T.v0[i]
    u = float(s @ p) / det
    v = float(d @ np.cross(s, T.e1[i])) / det
    return min(u, v, 1.0 - u - v)


def near_ray(O, d, T):
    """Triangles whose bounding sphere the ray's line comes near (a superset of
    every triangle the ray can hit: the distance from the box centre to the line
    is at most the half-diagonal for any triangle the line crosses)."""
    w = T.centre - O
    along = w @ d
    dist2 = np.einsum("ij,ij->i", w, w) - along * along
    r = T.radius * (1.0 + 1e-9) + 1e-9
    return np.nonzero(dist2 <= r * r)[0]


def compare(mesh, pulses, sc, sel, subrays=None):
    T = Tris(mesh)
    r = oracle.simulate(mesh, pulses, sc, select=sel, waveform=False)
    n_eq = n_tot = 0
    for q, p in enumerate(sel):
        O = pulses.origins[p].astype(np.float64)
        dirs = oracle.subray_directions(pulses.directions[p].astype(np.float64), sc)
        ks = range(dirs.shape[0]) if subrays is None else subrays
        for k in ks:
            d = dirs[k]
            idx = near_ray(O, d, T)
            mi, mt, _, _ = mt_closest(O, d, T, idx)
            oi, ot = int(r.sub_tri[q, k]), float(r.sub_range[q, k])
            n_tot += 1
            if mi == oi:
                n_eq += 1
                if mi >= 0:
                    assert abs(mt - ot) <= 1e-12 * ot, (p, k, mt, ot)
                continue
            # a differing triangle: only at an edge of one of the two
            edge = (mi >= 0 and bary_min(O, d, T, mi) <= EDGE) or (oi >= 0 and bary_min(O, d, T, oi) <= EDGE)
            assert edge, (p, k, mi, oi, mt, ot)
    return n_eq, n_tot


def test_small_tls_sample_against_moller_trumbore():
    mesh, pulses, sc = configs.small_tls()
    rng = np.random.default_rng(17)
    sel = np.sort(rng.choice(pulses.n, 100, replace=False))
    n_eq, n_tot = compare(mesh, pulses, sc, sel)
    # the scanner sits on a grid vertex, so subrays along the grid axes run
    # exactly through vertices and edges: a few differing (excused) triangles
    assert n_tot == 1900 and n_eq >= 0.995 * n_tot


def test_small_tls_vertex_and_edge_rays():
    # subrays aimed exactly at grid vertices and cell diagonals: hits on shared
    # edges, where the two tests may pick different (adjacent) triangles
    mesh, _, sc = configs.small_tls()
    T = Tris(mesh)
    V = mesh.vertices.astype(np.float64)
    O = np.array([32.0, 32.0, float(V[:, 2].max()) + 10.0])
    rng = np.random.default_rng(3)
    targets = []
    for _ in range(40):
        i, j = rng.integers(1, 62, 2)
        a, b = V[i * 64 + j], V[(i + 1) * 64 + j + 1]
        targets += [a, 0.5 * (a + b)]
    dirs = np.array([(t - O) / np.linalg.norm(t - O) for t in targets])
    pulses = synth.Pulses(np.tile(O, (len(dirs), 1)), dirs.astype(np.float32))
    one = dict(sc, n_subrays=1)
    sel = np.arange(pulses.n)
    n_eq, n_tot = compare(mesh, pulses, one, sel)
    assert n_tot == len(dirs)


def test_als_buildings_pulses_against_moller_trumbore():
    mesh, pulses, sc = configs.als_buildings()
    n_dtm = 2 * 1023 * 1023
    # one pulse at the swath centre, one near its start, and one whose beam
    # lands on a building (a box triangle: index past the terrain's)
    sel = np.array([499950, 500300, 500500])
    r = oracle.simulate(mesh, pulses, sc, select=sel[1:2], waveform=False)
    assert (r.sub_tri[0] >= n_dtm).any()
    n_eq, n_tot = compare(mesh, pulses, sc, sel)
    assert n_eq >= n_tot - 1
