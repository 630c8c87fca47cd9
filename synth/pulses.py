"""Seeded pulse sets: origins float64 [n,3] (metres), unit directions float32 [n,3].

Optional batching metadata: ``segment_offsets`` int64 [n_seg+1] and
``segment_scanner`` int32 [n_seg] (index into a list of scanner descriptions).
"""
from dataclasses import dataclass, field
from typing import Optional

import numpy as np


@dataclass
class Pulses:
    origins: np.ndarray                 # float64 [n,3]
    directions: np.ndarray              # float32 [n,3]
    segment_offsets: Optional[np.ndarray] = None   # int64 [n_seg+1]
    segment_scanner: Optional[np.ndarray] = None   # int32 [n_seg]
    info: dict = field(default_factory=dict)

    @property
    def n(self):
        return int(self.origins.shape[0])

    def subset(self, idx):
        idx = np.asarray(idx, dtype=np.int64)
        return Pulses(np.ascontiguousarray(self.origins[idx]), np.ascontiguousarray(self.directions[idx]),
                      info=dict(self.info, subset=True))


def _dirs(az, el):
    d = np.stack([np.cos(el) * np.cos(az), np.cos(el) * np.sin(az), np.sin(el)], -1)
    return d / np.linalg.norm(d, axis=-1, keepdims=True)


def tls_grid(origin, n_az, n_el, az_deg=(0.0, 360.0), el_deg=(-30.0, -5.0), *,
             az_endpoint=False, truncate=None):
    """Terrestrial az/el grid from one position; pulse index = i_az * n_el + j_el.

    Azimuth steps (hi-lo)/n_az (endpoint excluded: a full turn); elevation
    lo + (hi-lo)*j/(n_el-1).
    """
    i = np.arange(n_az)
    j = np.arange(n_el)
    if az_endpoint and n_az > 1:
        az = az_deg[0] + (az_deg[1] - az_deg[0]) * i / (n_az - 1)
    else:
        az = az_deg[0] + (az_deg[1] - az_deg[0]) * i / n_az
    el = el_deg[0] + (el_deg[1] - el_deg[0]) * (j / (n_el - 1) if n_el > 1 else np.zeros(1))
    A, E = np.meshgrid(np.deg2rad(az), np.deg2rad(el), indexing="ij")
    d = _dirs(A.reshape(-1), E.reshape(-1))
    if truncate is not None:
        d = d[:truncate]
    o = np.broadcast_to(np.asarray(origin, dtype=np.float64), d.shape).copy()
    return Pulses(o, d.astype(np.float32), info={"kind": "tls"})


def als_lines(x_center, y_lines, z, n_per_line, beta_deg=(-30.0, 30.0)):
    """Line scanner across +x flying along +y; pulse index = line * n_per_line + m.

    Scan angle beta_m = lo + (hi-lo)*m/(n-1); direction (sin b, 0, -cos b).
    """
    y_lines = np.asarray(y_lines, dtype=np.float64)
    m = np.arange(n_per_line)
    beta = np.deg2rad(beta_deg[0] + (beta_deg[1] - beta_deg[0]) * m / max(n_per_line - 1, 1))
    d1 = np.stack([np.sin(beta), np.zeros_like(beta), -np.cos(beta)], -1)
    d = np.broadcast_to(d1[None, :, :], (y_lines.size, n_per_line, 3)).reshape(-1, 3)
    x_center = np.broadcast_to(np.asarray(x_center, dtype=np.float64), y_lines.shape)
    o = np.stack([np.repeat(x_center, n_per_line), np.repeat(y_lines, n_per_line),
                  np.full(y_lines.size * n_per_line, float(z))], -1)
    return Pulses(o, d.astype(np.float32), info={"kind": "als"})


def concat_pulses(parts, scanner_index):
    """Concatenate pulse sets into one batch with segment metadata."""
    o = np.concatenate([p.origins for p in parts])
    d = np.concatenate([p.directions for p in parts])
    counts = np.array([p.n for p in parts], dtype=np.int64)
    off = np.zeros(len(parts) + 1, dtype=np.int64)
    off[1:] = np.cumsum(counts)
    return Pulses(o, d, off, np.asarray(scanner_index, dtype=np.int32), info={"kind": "batch"})
