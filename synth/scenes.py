"""Seeded synthetic triangle scenes: value-noise / fBm terrain, box buildings,
procedural trees.  Output arrays: vertices float32 [V,3] (metres), triangles
int32 [T,3] (vertex indices), reflectance float32 [T].
"""
from dataclasses import dataclass, field

import numpy as np

from .rng import uniform01, stream_uniform


@dataclass
class Mesh:
    vertices: np.ndarray      # float32 [V,3]
    triangles: np.ndarray     # int32 [T,3]
    reflectance: np.ndarray   # float32 [T]
    info: dict = field(default_factory=dict)

    @property
    def n_vertices(self):
        return int(self.vertices.shape[0])

    @property
    def n_triangles(self):
        return int(self.triangles.shape[0])

    def checked(self):
        assert self.vertices.dtype == np.float32 and self.vertices.ndim == 2 and self.vertices.shape[1] == 3
        assert self.triangles.dtype == np.int32 and self.triangles.ndim == 2 and self.triangles.shape[1] == 3
        assert self.reflectance.dtype == np.float32 and self.reflectance.shape == (self.n_triangles,)
        if self.n_triangles:
            assert self.triangles.min() >= 0 and self.triangles.max() < self.n_vertices
        return self


def _fade(t):
    # quintic fade 6t^5 - 15t^4 + 10t^3 (Perlin 2002)
    return t * t * t * (t * (t * 6.0 - 15.0) + 10.0)


def value_noise_field(x, y, *, seed, octaves, base_wavelength, amplitude,
                      lacunarity=2.0, gain=0.5):
    """Multi-octave value noise at world points (x, y), |h| <= amplitude.

    Lattice values come from a counter-based hash of (seed, octave, ix, iy), so
    the field is defined on the whole plane: a larger grid over the same seed
    contains a smaller one as its corner.  The normalisation is the fixed sum
    of octave gains (not data dependent) for the same reason.
    """
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    total = np.zeros(np.broadcast(x, y).shape)
    norm = 0.0
    amp = 1.0
    wl = float(base_wavelength)
    for o in range(octaves):
        gx = x / wl
        gy = y / wl
        ix = np.floor(gx).astype(np.int64)
        iy = np.floor(gy).astype(np.int64)
        fx = _fade(gx - ix)
        fy = _fade(gy - iy)

        def lat(i, j):
            key = (i + (1 << 24)) * (1 << 25) + (j + (1 << 24))
            return 2.0 * uniform01(seed, 1000 + o, key) - 1.0

        v00 = lat(ix, iy)
        v10 = lat(ix + 1, iy)
        v01 = lat(ix, iy + 1)
        v11 = lat(ix + 1, iy + 1)
        a = v00 + fx * (v10 - v00)
        b = v01 + fx * (v11 - v01)
        total += amp * (a + fy * (b - a))
        norm += amp
        amp *= gain
        wl /= lacunarity
    return amplitude * total / norm


def dtm_mesh(heights, spacing, *, x0=0.0, y0=0.0, refl_seed=None, refl_stream=7,
             refl_range=(0.1, 0.6)):
    """Grid heights [ny, nx] -> triangle mesh.

    Vertex (i, j) (i along x, j along y) has index j*nx + i.  Cell (i, j)
    yields triangles (i,j),(i+1,j),(i+1,j+1) and (i,j),(i+1,j+1),(i,j+1);
    cells in row-major order (j outer), two triangles per cell.
    """
    h = np.asarray(heights, dtype=np.float64)
    ny, nx = h.shape
    ii, jj = np.meshgrid(np.arange(nx), np.arange(ny))
    verts = np.stack([x0 + ii * spacing, y0 + jj * spacing, h], axis=-1).reshape(-1, 3)
    ci, cj = np.meshgrid(np.arange(nx - 1), np.arange(ny - 1))
    ci = ci.reshape(-1)
    cj = cj.reshape(-1)
    v00 = cj * nx + ci
    v10 = v00 + 1
    v01 = v00 + nx
    v11 = v01 + 1
    t_a = np.stack([v00, v10, v11], axis=-1)
    t_b = np.stack([v00, v11, v01], axis=-1)
    tris = np.stack([t_a, t_b], axis=1).reshape(-1, 3)
    n_t = tris.shape[0]
    if refl_seed is None:
        refl = np.full(n_t, 0.5)
    else:
        refl = stream_uniform(refl_seed, refl_stream, n_t, *refl_range)
    return Mesh(verts.astype(np.float32), tris.astype(np.int32), refl.astype(np.float32),
                {"kind": "dtm", "nx": nx, "ny": ny, "spacing": spacing, "x0": x0, "y0": y0})


def ground_height(heights, spacing, x, y, *, x0=0.0, y0=0.0):
    """Bilinear ground height at (x, y) (used only to place objects/scanners)."""
    h = np.asarray(heights, dtype=np.float64)
    ny, nx = h.shape
    gx = np.clip((np.asarray(x) - x0) / spacing, 0, nx - 1 - 1e-9)
    gy = np.clip((np.asarray(y) - y0) / spacing, 0, ny - 1 - 1e-9)
    i = np.floor(gx).astype(np.int64)
    j = np.floor(gy).astype(np.int64)
    fx = gx - i
    fy = gy - j
    a = h[j, i] + fx * (h[j, i + 1] - h[j, i])
    b = h[j + 1, i] + fx * (h[j + 1, i + 1] - h[j + 1, i])
    return a + fy * (b - a)


def merge_meshes(meshes):
    verts, tris, refl = [], [], []
    off = 0
    for m in meshes:
        verts.append(m.vertices)
        tris.append(m.triangles.astype(np.int64) + off)
        refl.append(m.reflectance)
        off += m.n_vertices
    return Mesh(np.concatenate(verts).astype(np.float32),
                np.concatenate(tris).astype(np.int32),
                np.concatenate(refl).astype(np.float32), {"kind": "merged"})


# 12 triangles of an axis-aligned box over its 8 corners (corner bit0 = x, bit1 = y, bit2 = z)
_BOX_TRIS = np.array([
    [0, 2, 3], [0, 3, 1],      # bottom z-
    [4, 5, 7], [4, 7, 6],      # top z+
    [0, 1, 5], [0, 5, 4],      # y-
    [2, 6, 7], [2, 7, 3],      # y+
    [0, 4, 6], [0, 6, 2],      # x-
    [1, 3, 7], [1, 7, 5],      # x+
], dtype=np.int64)


def add_boxes(heights, spacing, n_boxes, *, seed, extent, side=(2.0, 6.0),
              height=(4.0, 30.0), base_below=0.5, refl_range=(0.1, 0.6)):
    """``n_boxes`` axis-aligned box buildings over a height grid.

    Centres uniform over [0, extent]^2, sides U(side) per axis, heights
    U(height); the base sits ``base_below`` metres under the lowest ground
    corner of the footprint.  12 triangles per box; overlaps are allowed.
    """
    cx = stream_uniform(seed, 21, n_boxes, 0.0, extent)
    cy = stream_uniform(seed, 22, n_boxes, 0.0, extent)
    sx = stream_uniform(seed, 23, n_boxes, *side)
    sy = stream_uniform(seed, 24, n_boxes, *side)
    hz = stream_uniform(seed, 25, n_boxes, *height)
    x0, x1 = cx - sx / 2, cx + sx / 2
    y0, y1 = cy - sy / 2, cy + sy / 2
    corners_g = np.stack([ground_height(heights, spacing, x0, y0), ground_height(heights, spacing, x1, y0),
                          ground_height(heights, spacing, x0, y1), ground_height(heights, spacing, x1, y1)], 1)
    zb = corners_g.min(axis=1) - base_below
    zt = zb + hz
    c = np.arange(8)
    X = np.where(c[None, :] & 1, x1[:, None], x0[:, None])
    Y = np.where(c[None, :] & 2, y1[:, None], y0[:, None])
    Z = np.where(c[None, :] & 4, zt[:, None], zb[:, None])
    verts = np.stack([X, Y, Z], axis=-1).reshape(-1, 3)
    tris = (_BOX_TRIS[None, :, :] + 8 * np.arange(n_boxes)[:, None, None]).reshape(-1, 3)
    refl = stream_uniform(seed, 26, tris.shape[0], *refl_range)
    m = Mesh(verts.astype(np.float32), tris.astype(np.int32), refl.astype(np.float32),
             {"kind": "boxes", "n": n_boxes})
    m.info["footprints"] = np.stack([x0, x1, y0, y1], axis=1)
    return m


def flat_quad(x0, x1, y0, y1, z, reflectance=0.5):
    """Two triangles covering [x0,x1]x[y0,y1] at height z (for closed-form cases)."""
    v = np.array([[x0, y0, z], [x1, y0, z], [x1, y1, z], [x0, y1, z]], dtype=np.float32)
    t = np.array([[0, 1, 2], [0, 2, 3]], dtype=np.int32)
    return Mesh(v, t, np.full(2, reflectance, np.float32), {"kind": "quad"})


def _frusta(p0, p1, r0, r1, facets):
    """Open frusta (one per row) with ``facets`` sides: returns (verts, tris)."""
    m = p0.shape[0]
    axis = p1 - p0
    axis = axis / np.linalg.norm(axis, axis=1, keepdims=True)
    helper = np.where(np.abs(axis[:, 2:3]) < 0.9, np.array([[0.0, 0.0, 1.0]]), np.array([[1.0, 0.0, 0.0]]))
    u = np.cross(axis, helper)
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    v = np.cross(axis, u)
    ang = 2.0 * np.pi * np.arange(facets) / facets
    ring = np.cos(ang)[None, :, None] * u[:, None, :] + np.sin(ang)[None, :, None] * v[:, None, :]
    a = p0[:, None, :] + r0[:, None, None] * ring          # [m, F, 3]
    b = p1[:, None, :] + r1[:, None, None] * ring
    verts = np.concatenate([a, b], axis=1).reshape(-1, 3)  # per frustum: F bottom then F top
    f = np.arange(facets)
    g = (f + 1) % facets
    local = np.concatenate([np.stack([f, g, facets + g], 1), np.stack([f, facets + g, facets + f], 1)], 0)
    tris = (local[None, :, :] + (2 * facets) * np.arange(m)[:, None, None]).reshape(-1, 3)
    return verts, tris


def _poisson_positions(n, extent, min_dist, seed, margin=5.0):
    """Dart throwing with a grid hash: ``n`` points in [margin, extent-margin]^2."""
    pts = []
    cell = min_dist / np.sqrt(2.0)
    ng = int(np.ceil(extent / cell)) + 1
    grid = -np.ones((ng, ng), dtype=np.int64)
    cand = 0
    while len(pts) < n:
        xs = stream_uniform(seed, 31, cand + 4096, margin, extent - margin)[cand:]
        ys = stream_uniform(seed, 32, cand + 4096, margin, extent - margin)[cand:]
        cand += 4096
        for x, y in zip(xs, ys):
            gi, gj = int(x / cell), int(y / cell)
            ok = True
            for a in range(max(gi - 2, 0), min(gi + 3, ng)):
                for b in range(max(gj - 2, 0), min(gj + 3, ng)):
                    k = grid[a, b]
                    if k >= 0 and (pts[k][0] - x) ** 2 + (pts[k][1] - y) ** 2 < min_dist ** 2:
                        ok = False
                        break
                if not ok:
                    break
            if ok:
                grid[gi, gj] = len(pts)
                pts.append((x, y))
                if len(pts) == n:
                    break
        if cand > 400 * n + 100000:
            raise RuntimeError("could not place %d points with spacing %g" % (n, min_dist))
    return np.array(pts)


def tree_layout(heights, spacing, n_trees, *, seed, extent, min_dist=3.0):
    """Positions, ground heights, heights and crown ellipsoids (horizontal
    semi-axis ca, vertical cc, centre height cz) of the procedural trees."""
    pos = _poisson_positions(n_trees, extent, min_dist, seed)
    tid = np.arange(n_trees)
    gz = ground_height(heights, spacing, pos[:, 0], pos[:, 1])
    H = 10.0 + 15.0 * uniform01(seed, 40, tid)
    ca = 2.0 + 2.0 * uniform01(seed, 45, tid)
    cc = 0.3 * H
    cz = gz + 0.7 * H
    return dict(pos=pos, gz=gz, H=H, ca=ca, cc=cc, cz=cz)


def crown_voxels(layout, *, seed, extent, voxel_size=0.5, pad_range=(0.4, 1.6)):
    """Plant area density (m^2/m^3) of the crowns on a grid over [0, extent]^2
    and the crowns' height range: each tree adds pad_tree (0.5 + 0.5 u) to the
    voxels whose centre lies in its crown ellipsoid, pad_tree uniform in
    ``pad_range`` per tree and u uniform per voxel.  Returns (origin, pad
    [nz, ny, nx] float32)."""
    pos, ca, cc, cz = layout["pos"], layout["ca"], layout["cc"], layout["cz"]
    n = pos.shape[0]
    z0 = np.floor((cz - cc).min() / voxel_size) * voxel_size
    z1 = (cz + cc).max()
    nx = ny = int(np.ceil(extent / voxel_size))
    nz = int(np.ceil((z1 - z0) / voxel_size))
    vary = 0.5 + 0.5 * stream_uniform(seed, 54, nx * ny * nz).reshape(nz, ny, nx)
    pad_tree = pad_range[0] + (pad_range[1] - pad_range[0]) * uniform01(seed, 53, np.arange(n))
    pad = np.zeros((nz, ny, nx), np.float64)
    cx = (np.arange(nx) + 0.5) * voxel_size
    czs = z0 + (np.arange(nz) + 0.5) * voxel_size
    for t in range(n):
        i0 = max(int((pos[t, 0] - ca[t]) / voxel_size), 0)
        i1 = min(int((pos[t, 0] + ca[t]) / voxel_size) + 1, nx)
        j0 = max(int((pos[t, 1] - ca[t]) / voxel_size), 0)
        j1 = min(int((pos[t, 1] + ca[t]) / voxel_size) + 1, ny)
        k0 = max(int((cz[t] - cc[t] - z0) / voxel_size), 0)
        k1 = min(int((cz[t] + cc[t] - z0) / voxel_size) + 1, nz)
        X = ((cx[i0:i1] - pos[t, 0]) / ca[t]) ** 2
        Y = ((cx[j0:j1] - pos[t, 1]) / ca[t]) ** 2
        Z = ((czs[k0:k1] - cz[t]) / cc[t]) ** 2
        inside = (Z[:, None, None] + Y[None, :, None] + X[None, None, :]) <= 1.0
        pad[k0:k1, j0:j1, i0:i1] += np.where(inside, pad_tree[t] * vary[k0:k1, j0:j1, i0:i1], 0.0)
    return (0.0, 0.0, float(z0)), pad.astype(np.float32)


def procedural_trees(heights, spacing, n_trees, *, seed, extent, min_dist=3.0,
                     trunk_segments=8, facets=16, branches=40, branch_segments=2,
                     leaves=2000, leaf_size=0.05, refl_range=(0.1, 0.6)):
    """Procedural trees: tapered trunk of open frusta, branches, equilateral leaves.

    Per tree: ``trunk_segments`` frusta of ``facets`` sides (2*facets triangles
    each), ``branches`` x ``branch_segments`` branch frusta from the upper 60 %
    of the trunk, ``leaves`` equilateral triangles of side ``leaf_size`` placed
    uniformly in a crown ellipsoid with isotropic normals.
    """
    lay = tree_layout(heights, spacing, n_trees, seed=seed, extent=extent, min_dist=min_dist)
    pos, gz, H = lay["pos"], lay["gz"], lay["H"]
    n = n_trees
    tid = np.arange(n)
    r_base = 0.12 + 0.012 * H
    r_top = 0.25 * r_base
    # trunk frusta
    s = np.arange(trunk_segments)
    z0 = (gz[:, None] - 0.3) + (H[:, None] + 0.3) * s[None, :] / trunk_segments
    z1 = (gz[:, None] - 0.3) + (H[:, None] + 0.3) * (s[None, :] + 1) / trunk_segments
    rr0 = r_base[:, None] + (r_top - r_base)[:, None] * s[None, :] / trunk_segments
    rr1 = r_base[:, None] + (r_top - r_base)[:, None] * (s[None, :] + 1) / trunk_segments
    P0 = np.stack([np.repeat(pos[:, 0:1], trunk_segments, 1), np.repeat(pos[:, 1:2], trunk_segments, 1), z0], -1).reshape(-1, 3)
    P1 = np.stack([np.repeat(pos[:, 0:1], trunk_segments, 1), np.repeat(pos[:, 1:2], trunk_segments, 1), z1], -1).reshape(-1, 3)
    tv, tt = _frusta(P0, P1, rr0.reshape(-1), rr1.reshape(-1), facets)
    # branches: start on the trunk axis in the upper 60 %, up-and-out direction
    bid = np.arange(n * branches)
    tree_of_b = bid // branches
    hb = 0.4 + 0.6 * uniform01(seed, 41, bid)
    az = 2.0 * np.pi * uniform01(seed, 42, bid)
    el = np.deg2rad(20.0 + 40.0 * uniform01(seed, 43, bid))
    blen = 1.0 + 3.0 * uniform01(seed, 44, bid)
    start = np.stack([pos[tree_of_b, 0], pos[tree_of_b, 1], gz[tree_of_b] + hb * H[tree_of_b]], -1)
    bdir = np.stack([np.cos(el) * np.cos(az), np.cos(el) * np.sin(az), np.sin(el)], -1)
    rb0 = 0.35 * (r_base[tree_of_b] + (r_top - r_base)[tree_of_b] * hb)
    segs = np.arange(branch_segments)
    bp0 = (start[:, None, :] + bdir[:, None, :] * (blen[:, None] * segs[None, :] / branch_segments)[..., None]).reshape(-1, 3)
    bp1 = (start[:, None, :] + bdir[:, None, :] * (blen[:, None] * (segs[None, :] + 1) / branch_segments)[..., None]).reshape(-1, 3)
    br0 = (rb0[:, None] * (1.0 - 0.4 * segs[None, :] / branch_segments)).reshape(-1)
    br1 = (rb0[:, None] * (1.0 - 0.4 * (segs[None, :] + 1) / branch_segments)).reshape(-1)
    bv, bt = _frusta(bp0, bp1, br0, br1, facets)
    # leaves: uniform in the crown ellipsoid, isotropic normals
    lid = np.arange(n * leaves)
    tree_of_l = lid // leaves
    ca, cc, cz = lay["ca"], lay["cc"], lay["cz"]
    # uniform point in the unit ball by radius cube-root + direction
    u1 = uniform01(seed, 46, lid)
    u2 = uniform01(seed, 47, lid)
    u3 = uniform01(seed, 48, lid)
    rad = np.cbrt(u1)
    cth = 2.0 * u2 - 1.0
    sth = np.sqrt(np.maximum(0.0, 1.0 - cth * cth))
    ph = 2.0 * np.pi * u3
    cen = np.stack([pos[tree_of_l, 0] + ca[tree_of_l] * rad * sth * np.cos(ph),
                    pos[tree_of_l, 1] + ca[tree_of_l] * rad * sth * np.sin(ph),
                    cz[tree_of_l] + cc[tree_of_l] * rad * cth], -1)
    nz = 2.0 * uniform01(seed, 49, lid) - 1.0
    nph = 2.0 * np.pi * uniform01(seed, 50, lid)
    nr = np.sqrt(np.maximum(0.0, 1.0 - nz * nz))
    nrm = np.stack([nr * np.cos(nph), nr * np.sin(nph), nz], -1)
    helper = np.where(np.abs(nrm[:, 2:3]) < 0.9, np.array([[0.0, 0.0, 1.0]]), np.array([[1.0, 0.0, 0.0]]))
    e1 = np.cross(nrm, helper)
    e1 /= np.linalg.norm(e1, axis=1, keepdims=True)
    e2 = np.cross(nrm, e1)
    rot = 2.0 * np.pi * uniform01(seed, 51, lid)
    circ = leaf_size / np.sqrt(3.0)
    lv = []
    for q in range(3):
        a = rot + q * 2.0 * np.pi / 3.0
        lv.append(cen + circ * (np.cos(a)[:, None] * e1 + np.sin(a)[:, None] * e2))
    lverts = np.stack(lv, 1).reshape(-1, 3)
    ltris = np.arange(3 * n * leaves).reshape(-1, 3)
    verts = np.concatenate([tv, bv, lverts])
    tris = np.concatenate([tt, bt + tv.shape[0], ltris + tv.shape[0] + bv.shape[0]])
    refl = stream_uniform(seed, 52, tris.shape[0], *refl_range)
    m = Mesh(verts.astype(np.float32), tris.astype(np.int32), refl.astype(np.float32),
             {"kind": "trees", "n": n_trees, "positions": pos})
    return m
