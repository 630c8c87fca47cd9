"""The seven synthetic workloads, as (scene, pulses, scanner) recipes.

  small_tls      64x64 value-noise DTM at 1 m (7,938 triangles); terrestrial
                 scanner, 100x100 az/el grid; 19 subrays; 256 x 1 ns bins.
  als_buildings  1024x1024 fBm DTM at 0.5 m + 20,000 box buildings
                 (2,333,058 triangles); line scanner at 500 m AGL, 1M pulses;
                 31 subrays; 512 x 0.5 ns bins.
  uls_trees      200x200 m fBm DTM at 0.5 m + 2,000 procedural trees
                 (~9.95M triangles); 60 m AGL, 2M pulses; 61 subrays; 8 returns.
  uls_voxels     the uls_trees terrain and flight; trunks and branches as
                 triangles (5,952,000), crowns as 0.5 m transmissive voxels of
                 plant area density 0.2-1.6 m^2/m^3 per crown (summed where
                 crowns overlap); Table 2's printed rows.
  uls_instanced  the uls_trees terrain and flight; its 2,000 trees are instances
                 of 8 procedural tree models (turned, scaled 0.8-1.2, moved).
  batched_tls    the als_buildings scene; 256 terrestrial positions with
                 log-uniform pulse counts in [1k, 200k]; three scanner types.
  diff_als       the small_tls noise field on 256x256 vertices (130,050
                 triangles); 100k line-scanner pulses; a seeded perturbed target.

A scanner is a plain dict of instrument parameters (no method arithmetic).
"""
import numpy as np

from .rng import stream_uniform, uniform01
from .scenes import (value_noise_field, dtm_mesh, add_boxes, merge_meshes, ground_height, procedural_trees,
                     tree_layout, crown_voxels)
from .pulses import tls_grid, als_lines, concat_pulses


def scanner(divergence_rad, n_subrays, *, pulse_shape="gaussian", pulse_width_ns=4.0,
            bin_ns=1.0, n_bins=256, window_pre_ns=-1.0, max_returns=8,
            min_echo_abs=0.0, min_echo_rel=1e-3, peak_power_w=1.0,
            receiver_diameter_m=1.0, efficiency=1.0, pattern_extent=1.0, beam_quality=0,
            range_noise_m=0.0, noise_seed=0):
    return dict(divergence_rad=float(divergence_rad), n_subrays=int(n_subrays),
                beam_quality=int(beam_quality), pattern_extent=float(pattern_extent),
                pulse_shape=pulse_shape, pulse_width_ns=float(pulse_width_ns),
                bin_ns=float(bin_ns), n_bins=int(n_bins), window_pre_ns=float(window_pre_ns),
                peak_power_w=float(peak_power_w), receiver_diameter_m=float(receiver_diameter_m),
                efficiency=float(efficiency), min_echo_abs=float(min_echo_abs),
                min_echo_rel=float(min_echo_rel), max_returns=int(max_returns),
                range_noise_m=float(range_noise_m), noise_seed=int(noise_seed))


# ---------------------------------------------------------------- small_tls
SMALL_SEED = 20210122


def small_heights(n=64, seed=SMALL_SEED):
    x = np.arange(n, dtype=np.float64)
    X, Y = np.meshgrid(x, x)          # [ny, nx]
    return value_noise_field(X, Y, seed=seed, octaves=4, base_wavelength=32.0, amplitude=5.0)


def small_tls(seed=SMALL_SEED, n_az=100, n_el=100):
    h = small_heights(64, seed)
    mesh = dtm_mesh(h, 1.0, refl_seed=seed)
    origin = (32.0, 32.0, float(h[32, 32]) + 1.5)
    pulses = tls_grid(origin, n_az, n_el, az_deg=(0.0, 360.0), el_deg=(-30.0, -5.0))
    sc = scanner(0.3e-3, 19, pulse_width_ns=4.0, bin_ns=1.0, n_bins=256)
    return mesh, pulses, sc


# ---------------------------------------------------------------- als_buildings
ALS_SEED = 7102021


def als_heights(n=1024, seed=ALS_SEED):
    x = np.arange(n, dtype=np.float64) * 0.5
    X, Y = np.meshgrid(x, x)
    return value_noise_field(X, Y, seed=seed, octaves=6, base_wavelength=256.0, amplitude=30.0)


def als_scene(seed=ALS_SEED, n=1024, n_boxes=20000):
    h = als_heights(n, seed)
    dtm = dtm_mesh(h, 0.5, refl_seed=seed)
    extent = (n - 1) * 0.5
    boxes = add_boxes(h, 0.5, n_boxes, seed=seed, extent=extent)
    mesh = merge_meshes([dtm, boxes])
    mesh.info.update(kind="als_buildings", heights_mean=float(h.mean()), extent=extent,
                     footprints=boxes.info["footprints"], heights=h)
    return mesh


def als_buildings(seed=ALS_SEED, n_lines=1000, per_line=1000, mesh=None):
    mesh = als_scene(seed) if mesh is None else mesh
    extent = mesh.info["extent"]
    z = mesh.info["heights_mean"] + 500.0
    y = extent * np.arange(n_lines) / max(n_lines - 1, 1)
    pulses = als_lines(extent / 2.0, y, z, per_line, beta_deg=(-30.0, 30.0))
    sc = scanner(0.5e-3, 31, pulse_width_ns=4.0, bin_ns=0.5, n_bins=512)
    return mesh, pulses, sc


# ---------------------------------------------------------------- uls_trees
ULS_SEED = 11092021


def uls_scene(seed=ULS_SEED, n_trees=2000):
    x = np.arange(401, dtype=np.float64) * 0.5
    X, Y = np.meshgrid(x, x)
    h = value_noise_field(X, Y, seed=seed, octaves=5, base_wavelength=64.0, amplitude=5.0)
    dtm = dtm_mesh(h, 0.5, refl_seed=seed)
    trees = procedural_trees(h, 0.5, n_trees, seed=seed, extent=200.0)
    mesh = merge_meshes([dtm, trees])
    mesh.info.update(kind="uls_trees", heights_mean=float(h.mean()), extent=200.0, heights=h)
    return mesh


def uls_trees(seed=ULS_SEED, strips=4, n_lines=500, per_line=1000, mesh=None):
    mesh = uls_scene(seed) if mesh is None else mesh
    z = mesh.info["heights_mean"] + 60.0
    parts = []
    for s in range(strips):
        xc = 200.0 * (s + 0.5) / strips
        y = 200.0 * np.arange(n_lines) / max(n_lines - 1, 1)
        parts.append(als_lines(xc, y, z, per_line, beta_deg=(-45.0, 45.0)))
    o = np.concatenate([p.origins for p in parts])
    d = np.concatenate([p.directions for p in parts])
    from .pulses import Pulses
    pulses = Pulses(o, d, info={"kind": "uls"})
    sc = scanner(0.25e-3, 61, pulse_width_ns=4.0, bin_ns=0.5, n_bins=512, max_returns=8)
    return mesh, pulses, sc


# ---------------------------------------------------------------- uls_voxels
# The rows of the leaf-angle table the paper prints (Table 2, erectophile):
# (vertical component of the beam, hit probability g).  Its middle rows are
# elided there; between the printed rows the table is taken as linear.
TABLE2_ROWS = [[0.0, 0.424413], [0.025180, 0.424682], [0.050345, 0.425489], [0.999955, 0.848789],
               [1.0, 0.848822]]


def uls_voxels(seed=ULS_SEED, strips=4, n_lines=500, per_line=1000, voxel_size=0.5):
    """The uls_trees terrain and flight, with woody trees (trunks and branches as
    triangles) whose crowns are transmissive voxels of plant area density."""
    x = np.arange(401, dtype=np.float64) * 0.5
    X, Y = np.meshgrid(x, x)
    h = value_noise_field(X, Y, seed=seed, octaves=5, base_wavelength=64.0, amplitude=5.0)
    dtm = dtm_mesh(h, 0.5, refl_seed=seed)
    wood = procedural_trees(h, 0.5, 2000, seed=seed, extent=200.0, leaves=0)
    mesh = merge_meshes([dtm, wood])
    mesh.info.update(kind="uls_voxels", heights_mean=float(h.mean()), extent=200.0)
    lay = tree_layout(h, 0.5, 2000, seed=seed, extent=200.0)
    origin, pad = crown_voxels(lay, seed=seed, extent=200.0, voxel_size=voxel_size)
    voxels = dict(origin=list(origin), size=float(voxel_size), pad=pad, lut=TABLE2_ROWS, seed=seed)
    _, pulses, sc = uls_trees(seed, strips, n_lines, per_line, mesh=mesh)
    return mesh, voxels, pulses, sc


# ---------------------------------------------------------------- uls_instanced
def tree_models(seed=ULS_SEED, n_models=8, leaves=2000):
    """Procedural tree models standing at the origin on flat ground."""
    models = []
    for m in range(n_models):
        t = procedural_trees(np.zeros((3, 3)), 10.0, 1, seed=seed + 101 * (m + 1), extent=20.0, leaves=leaves)
        p = t.info["positions"][0]
        t.vertices = (t.vertices - np.array([p[0], p[1], 0.0], np.float32)).astype(np.float32)
        models.append(t)
    return models


def uls_instanced(seed=ULS_SEED, n_models=8, n_trees=2000, strips=4, n_lines=500, per_line=1000, leaves=2000):
    """The uls_trees terrain and flight with its forest as instances of a few tree
    models: part 0 is the terrain (placed once, unmoved), parts 1..n_models the
    models, each tree a model turned about z by a uniform angle, scaled by
    U(0.8, 1.2) and moved to its position on the ground."""
    x = np.arange(401, dtype=np.float64) * 0.5
    X, Y = np.meshgrid(x, x)
    h = value_noise_field(X, Y, seed=seed, octaves=5, base_wavelength=64.0, amplitude=5.0)
    parts = [dtm_mesh(h, 0.5, refl_seed=seed)] + tree_models(seed, n_models, leaves)
    lay = tree_layout(h, 0.5, n_trees, seed=seed, extent=200.0)
    tid = np.arange(n_trees)
    model = 1 + np.minimum((uniform01(seed, 60, tid) * n_models).astype(np.int64), n_models - 1)
    th = 2.0 * np.pi * uniform01(seed, 61, tid)
    sc_ = 0.8 + 0.4 * uniform01(seed, 62, tid)
    instances = [(0, np.hstack([np.eye(3), np.zeros((3, 1))]))]
    for i in range(n_trees):
        c, s_ = np.cos(th[i]) * sc_[i], np.sin(th[i]) * sc_[i]
        A = np.array([[c, -s_, 0.0], [s_, c, 0.0], [0.0, 0.0, sc_[i]]])
        t = np.array([lay["pos"][i, 0], lay["pos"][i, 1], lay["gz"][i]])
        instances.append((int(model[i]), np.hstack([A, t[:, None]])))
    info = dict(kind="uls_instanced", heights_mean=float(h.mean()), extent=200.0)
    mesh_for_pulses = parts[0]
    mesh_for_pulses.info.update(info)
    _, pulses, sc = uls_trees(seed, strips, n_lines, per_line, mesh=mesh_for_pulses)
    return parts, instances, pulses, sc


# ---------------------------------------------------------------- batched_tls
BATCH_SEED = 4242

BATCH_SCANNERS = [
    scanner(0.3e-3, 19, bin_ns=1.0, n_bins=256),
    scanner(0.5e-3, 31, bin_ns=1.0, n_bins=256),
    scanner(0.25e-3, 61, bin_ns=1.0, n_bins=256),
]


def batched_tls(seed=BATCH_SEED, n_positions=256, mesh=None, count_range=(1e3, 2e5), max_pulses=None):
    mesh = als_scene() if mesh is None else mesh
    extent = mesh.info["extent"]
    fp = mesh.info["footprints"]
    h = mesh.info["heights"]
    pos = []
    k = 0
    while len(pos) < n_positions:
        x = float(stream_uniform(seed, 61, k + 1, 5.0, extent - 5.0)[k])
        y = float(stream_uniform(seed, 62, k + 1, 5.0, extent - 5.0)[k])
        k += 1
        inside = np.any((fp[:, 0] <= x) & (x <= fp[:, 1]) & (fp[:, 2] <= y) & (y <= fp[:, 3]))
        if not inside:
            pos.append((x, y, float(ground_height(h, 0.5, x, y)) + 1.5))
    lo, hi = np.log(count_range[0]), np.log(count_range[1])
    counts = np.rint(np.exp(lo + (hi - lo) * uniform01(seed, 63, np.arange(n_positions)))).astype(np.int64)
    if max_pulses is not None:
        counts = np.minimum(counts, max_pulses)
    parts = []
    for p in range(n_positions):
        n_p = int(counts[p])
        n_el = max(1, int(round(np.sqrt(n_p / 6.0))))
        n_az = int(np.ceil(n_p / n_el))
        parts.append(tls_grid(pos[p], n_az, n_el, az_deg=(0.0, 360.0), el_deg=(-40.0, 20.0), truncate=n_p))
    pulses = concat_pulses(parts, np.arange(n_positions) % 3)
    pulses.info["positions"] = np.array(pos)
    return mesh, pulses, list(BATCH_SCANNERS)


# ---------------------------------------------------------------- diff_als
def diff_scene(seed=SMALL_SEED, n=256):
    h = small_heights(n, seed)
    mesh = dtm_mesh(h, 1.0, refl_seed=seed)
    mesh.info.update(kind="diff_dtm", heights_mean=float(h.mean()), extent=float(n - 1))
    return mesh


def diff_target(mesh, seed=SMALL_SEED + 1, dz=0.2, drho=0.05):
    v = mesh.vertices.copy()
    v[:, 2] += stream_uniform(seed, 71, v.shape[0], -dz, dz).astype(np.float32)
    r = np.clip(mesh.reflectance + stream_uniform(seed, 72, mesh.n_triangles, -drho, drho), 0.0, 1.0)
    from .scenes import Mesh
    return Mesh(v, mesh.triangles.copy(), r.astype(np.float32), dict(mesh.info, target=True))


def diff_als(seed=SMALL_SEED, n_lines=250, per_line=400, n=256):
    mesh = diff_scene(seed, n)
    target = diff_target(mesh)
    extent = mesh.info["extent"]
    z = mesh.info["heights_mean"] + 200.0
    y = extent * np.arange(n_lines) / max(n_lines - 1, 1)
    pulses = als_lines(extent / 2.0, y, z, per_line, beta_deg=(-30.0, 30.0))
    sc = scanner(0.5e-3, 31, pulse_width_ns=4.0, bin_ns=0.5, n_bins=512)
    return mesh, target, pulses, sc
