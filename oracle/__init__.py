"""FP64 CPU oracle (test infrastructure only).

Thin ctypes wrapper over ``vls_oracle.c``.  Only the tests, the smoke check
and the benchmark's CPU-baseline leg may import this package; the GPU library
never does.  See ``vls_oracle.c`` for what is computed and the readings of
the paper it takes.
"""
import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "vls_oracle.c")
LIB = os.path.join(HERE, "libvls_oracle.so")

C_M_PER_NS = 0.299792458
PULSE_GAUSSIAN = 0
PULSE_EQ3 = 1


def build(force=True):
    """Compile the oracle with gcc (OpenMP)."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-o", tmp,
                           SRC, "-lm"])
    os.replace(tmp, LIB)
    return LIB


class OrcSurvey(ctypes.Structure):
    _fields_ = [("waypoints", ctypes.c_void_p), ("n_waypoints", ctypes.c_int32), ("deflector", ctypes.c_int32),
                ("speed", ctypes.c_double), ("prf", ctypes.c_double), ("scan_freq", ctypes.c_double),
                ("scan_angle", ctypes.c_double), ("n_fibres", ctypes.c_int32), ("platform", ctypes.c_int32),
                ("t0", ctypes.c_double), ("noise_sigma", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("accel", ctypes.c_double), ("leg_yaw", ctypes.c_void_p), ("bank", ctypes.c_double)]


DEFLECTORS = {"polygon": 0, "swing": 1, "conic": 2, "fibre": 3}
PLATFORMS = {"linear": 0, "multicopter": 1, "multicopter_smooth": 2}


class OrcVoxels(ctypes.Structure):
    _fields_ = [("origin", ctypes.c_double * 3), ("size", ctypes.c_double), ("nx", ctypes.c_int32),
                ("ny", ctypes.c_int32), ("nz", ctypes.c_int32), ("n_lut", ctypes.c_int32),
                ("pad", ctypes.c_void_p), ("lut", ctypes.c_void_p), ("seed", ctypes.c_uint64)]


def voxel_struct(vox):
    """ctypes view of a voxel grid dict (origin, size, pad [nz, ny, nx], lut [n, 2], seed); the arrays
    are kept alive in the returned tuple."""
    pad = np.ascontiguousarray(vox["pad"], dtype=np.float32)
    lut = np.ascontiguousarray(vox["lut"], dtype=np.float64).reshape(-1, 2)
    nz, ny, nx = pad.shape
    st = OrcVoxels((ctypes.c_double * 3)(*[float(x) for x in vox["origin"]]), float(vox["size"]), nx, ny, nz,
                   lut.shape[0], pad.ctypes.data, lut.ctypes.data, int(vox.get("seed", 0)) & 0xFFFFFFFFFFFFFFFF)
    return st, (pad, lut)


class OrcScanner(ctypes.Structure):
    _fields_ = [("divergence_rad", ctypes.c_double), ("pattern_extent", ctypes.c_double),
                ("pulse_width_ns", ctypes.c_double), ("bin_ns", ctypes.c_double),
                ("window_pre_ns", ctypes.c_double), ("peak_power_w", ctypes.c_double),
                ("receiver_diameter_m", ctypes.c_double), ("efficiency", ctypes.c_double),
                ("min_echo_abs", ctypes.c_double), ("min_echo_rel", ctypes.c_double),
                ("n_subrays", ctypes.c_int32), ("beam_quality", ctypes.c_int32),
                ("pulse_shape", ctypes.c_int32), ("n_bins", ctypes.c_int32),
                ("max_returns", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("range_noise_m", ctypes.c_double), ("noise_seed", ctypes.c_uint64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        L.orc_ring_layout.argtypes = [ctypes.c_int, ctypes.c_int, P, ctypes.c_int]
        L.orc_pattern_size.argtypes = [ctypes.c_int, ctypes.c_int]
        L.orc_pattern.argtypes = [P, P, P, P, ctypes.c_int]
        L.orc_subray_direction.argtypes = [P, ctypes.c_double, ctypes.c_double, P]
        L.orc_ray_triangle.argtypes = [P] * 8
        L.orc_closest_hit.argtypes = [P, P, P, P, i64, P, P, P]
        L.orc_closest_hit.restype = i64
        L.orc_pulse_value.argtypes = [P, ctypes.c_double]
        L.orc_pulse_value.restype = ctypes.c_double
        L.orc_pulse_derivative.argtypes = [P, ctypes.c_double]
        L.orc_pulse_derivative.restype = ctypes.c_double
        L.orc_window_pre.argtypes = [P]
        L.orc_window_pre.restype = ctypes.c_double
        L.orc_peak_offset.argtypes = [P]
        L.orc_peak_offset.restype = ctypes.c_double
        L.orc_echo_range.argtypes = [P, ctypes.c_double, ctypes.c_int]
        L.orc_echo_range.restype = ctypes.c_double
        L.orc_detect_peaks.argtypes = [P, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int, P]
        L.orc_echo_width_bins.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_double, P]
        L.orc_echo_width_bins.restype = ctypes.c_double
        L.orc_echo_width.argtypes = [P, P, ctypes.c_int, P, ctypes.c_int, P]
        L.orc_splitmix64.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        L.orc_splitmix64.restype = ctypes.c_uint64
        L.orc_generate_pulses.argtypes = [P, i64, i64, P, P]
        L.orc_attribute.argtypes = [P, P, P, P, ctypes.c_int, ctypes.c_double]
        L.orc_simulate.argtypes = [P, i64, P, P, i64, P, P, P, i64, P, i64, P] + [P] * 6 + [P] * 7 + [ctypes.c_int]
        L.orc_gradient.argtypes = [P, i64, P, P, i64, P, P, P, i64, P, P, P, P, ctypes.c_int]
        L.orc_simulate_ext.argtypes = L.orc_simulate.argtypes + [P, P, P]
        L.orc_gradient_ext.argtypes = L.orc_gradient.argtypes + [P, P, P]
        L.orc_surface_response.argtypes = [ctypes.c_double] * 3
        L.orc_surface_response.restype = ctypes.c_double
        L.orc_lut_g.argtypes = [P, ctypes.c_double]
        L.orc_lut_g.restype = ctypes.c_double
        L.orc_voxel_hit.argtypes = [P, P, P, ctypes.c_double, ctypes.c_uint64, P, P]
        L.orc_voxel_hit.restype = i64
        L.orc_instance_vertices.argtypes = [P, i64, P, P]
        L.orc_range_noise.argtypes = [P, i64, ctypes.c_int]
        L.orc_range_noise.restype = ctypes.c_double
        L.orc_max_threads.argtypes = []
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def scanner_struct(sc):
    """Plain scanner dict (see synth.configs.scanner) -> OrcScanner."""
    shape = sc.get("pulse_shape", "gaussian")
    return OrcScanner(divergence_rad=sc["divergence_rad"], pattern_extent=sc.get("pattern_extent", 1.0),
                      pulse_width_ns=sc["pulse_width_ns"], bin_ns=sc["bin_ns"],
                      window_pre_ns=sc.get("window_pre_ns", -1.0), peak_power_w=sc.get("peak_power_w", 1.0),
                      receiver_diameter_m=sc.get("receiver_diameter_m", 1.0), efficiency=sc.get("efficiency", 1.0),
                      min_echo_abs=sc.get("min_echo_abs", 0.0), min_echo_rel=sc.get("min_echo_rel", 1e-3),
                      n_subrays=sc.get("n_subrays", 0), beam_quality=sc.get("beam_quality", 0),
                      pulse_shape=PULSE_EQ3 if shape in ("eq3", PULSE_EQ3) else PULSE_GAUSSIAN,
                      n_bins=sc["n_bins"], max_returns=sc.get("max_returns", 8), pad_=0,
                      range_noise_m=sc.get("range_noise_m", 0.0), noise_seed=int(sc.get("noise_seed", 0)) & (2**64 - 1))


def ring_layout(n_subrays=0, beam_quality=0):
    rc = np.zeros(256, np.int32)
    n = lib().orc_ring_layout(n_subrays, beam_quality, _ptr(rc), 256)
    if n < 0:
        raise ValueError("bad pattern request")
    return rc[:n].copy()


def pattern_size(n_subrays=0, beam_quality=0):
    return int(lib().orc_pattern_size(n_subrays, beam_quality))


def pattern(sc):
    """-> (alpha, phi, weight) float64 arrays of length S."""
    st = scanner_struct(sc)
    a = np.zeros(4096)
    p = np.zeros(4096)
    w = np.zeros(4096)
    s = lib().orc_pattern(ctypes.byref(st), _ptr(a), _ptr(p), _ptr(w), 4096)
    if s < 0:
        raise ValueError("bad pattern request")
    return a[:s].copy(), p[:s].copy(), w[:s].copy()


def subray_directions(d, sc):
    a, p, _ = pattern(sc)
    d = np.ascontiguousarray(d, dtype=np.float64)
    out = np.zeros((a.size, 3))
    for k in range(a.size):
        o = np.zeros(3)
        lib().orc_subray_direction(_ptr(d), float(a[k]), float(p[k]), _ptr(o))
        out[k] = o
    return out


def ray_triangle(O, d, a, b, c):
    args = [np.ascontiguousarray(x, dtype=np.float64) for x in (O, d, a, b, c)]
    t = np.zeros(1)
    u = np.zeros(1)
    v = np.zeros(1)
    hit = lib().orc_ray_triangle(*[_ptr(x) for x in args], _ptr(t), _ptr(u), _ptr(v))
    return bool(hit), float(t[0]), float(u[0]), float(v[0])


def closest_hit(O, d, mesh):
    O = np.ascontiguousarray(O, dtype=np.float64)
    d = np.ascontiguousarray(d, dtype=np.float64)
    t = np.zeros(1)
    u = np.zeros(1)
    v = np.zeros(1)
    h = lib().orc_closest_hit(_ptr(O), _ptr(d), _ptr(mesh.vertices), _ptr(mesh.triangles),
                              mesh.n_triangles, _ptr(t), _ptr(u), _ptr(v))
    return int(h), float(t[0]), float(u[0]), float(v[0])


def pulse_value(sc, s):
    st = scanner_struct(sc)
    return float(lib().orc_pulse_value(ctypes.byref(st), float(s)))


def pulse_derivative(sc, s):
    st = scanner_struct(sc)
    return float(lib().orc_pulse_derivative(ctypes.byref(st), float(s)))


def window_pre(sc):
    st = scanner_struct(sc)
    return float(lib().orc_window_pre(ctypes.byref(st)))


def peak_offset(sc):
    st = scanner_struct(sc)
    return float(lib().orc_peak_offset(ctypes.byref(st)))


def echo_range(sc, t0, j):
    """Range (m) of a return at bin j of a window starting at t0 (ns), without ranging error."""
    st = scanner_struct(sc)
    return float(lib().orc_echo_range(ctypes.byref(st), float(t0), int(j)))


def detect_peaks(wf, thr_abs=0.0, thr_rel=1e-3, K=8):
    """The first K local maxima of a waveform in time order (K >= the number of
    bins gives all of them)."""
    wf = np.ascontiguousarray(wf, dtype=np.float64)
    K = max(0, min(int(K), wf.size))
    bins = np.zeros(max(K, 1), np.int32)
    n = lib().orc_detect_peaks(_ptr(wf), wf.size, float(thr_abs), float(thr_rel), int(K), _ptr(bins))
    return bins[:n].copy()


def echo_width_bins(wf, j, s0):
    """Gaussian fit to the lobe of the return at bin j (Sec. 3.4 echo width):
    (width in bins or NaN, fitted (A, mu, s))."""
    wf = np.ascontiguousarray(wf, dtype=np.float64)
    p = np.zeros(3)
    w = lib().orc_echo_width_bins(_ptr(wf), wf.size, int(j), float(s0), _ptr(p))
    return w, p


def echo_width(sc, wf, bins):
    """Echo widths (ns) of the returns `bins` of one waveform."""
    st = scanner_struct(sc)
    wf = np.ascontiguousarray(wf, dtype=np.float64)
    bins = np.ascontiguousarray(bins, dtype=np.int32)
    out = np.zeros(max(bins.size, 1))
    lib().orc_echo_width(ctypes.byref(st), _ptr(wf), wf.size, _ptr(bins), bins.size, _ptr(out))
    return out[:bins.size].copy()


def splitmix64(seed, c):
    """Output number c of the SplitMix64 sequence seeded with `seed`."""
    return int(lib().orc_splitmix64(int(seed) & 0xFFFFFFFFFFFFFFFF, int(c)))


def generate_pulses(sv, first, count):
    """Pulses [first, first + count) of a survey (Sec. 3.2-3.3 readings):
    origins and unit directions, both float64 [count, 3].  `platform` is
    "linear" (default), "multicopter" (with `accel_mps2` and optionally
    `leg_yaw`, [n_waypoints - 1, 2] start and end yaw of each leg) or
    "multicopter_smooth" (banked turns: `accel_mps2` and `bank_angle_rad`)."""
    wp = np.ascontiguousarray(sv["waypoints"], dtype=np.float64).reshape(-1, 3)
    ly = sv.get("leg_yaw")
    ly = None if ly is None else np.ascontiguousarray(ly, dtype=np.float64).reshape(-1, 2)
    if ly is not None and ly.shape[0] != max(wp.shape[0] - 1, 0):
        raise ValueError("leg_yaw needs one row per leg")
    st = OrcSurvey(wp.ctypes.data, wp.shape[0], DEFLECTORS[sv.get("deflector", "polygon")],
                   float(sv.get("speed_mps", 0.0)), float(sv["pulse_rate_hz"]), float(sv.get("scan_freq_hz", 0.0)),
                   float(sv.get("scan_angle_rad", 0.0)), int(sv.get("n_fibres", 0)),
                   PLATFORMS[sv.get("platform", "linear")], float(sv.get("t0", 0.0)),
                   float(sv.get("platform_noise_m", 0.0)), int(sv.get("seed", 0)) & 0xFFFFFFFFFFFFFFFF,
                   float(sv.get("accel_mps2", 0.0)), None if ly is None else ly.ctypes.data,
                   float(sv.get("bank_angle_rad", 0.0)))
    o = np.zeros((count, 3))
    d = np.zeros((count, 3))
    if lib().orc_generate_pulses(ctypes.byref(st), int(first), int(count), _ptr(o), _ptr(d)) != 0:
        raise ValueError("invalid survey")
    return o, d


def attribute(sc, tri, R, P, tj):
    """Index of the subray contributing most at time tj (ties: lowest index)."""
    st = scanner_struct(sc)
    tri = np.ascontiguousarray(tri, dtype=np.int32)
    R = np.ascontiguousarray(R, dtype=np.float64)
    P = np.ascontiguousarray(P, dtype=np.float64)
    return int(lib().orc_attribute(ctypes.byref(st), _ptr(tri), _ptr(R), _ptr(P), tri.size, float(tj)))


@dataclass
class OracleResult:
    sub_tri: np.ndarray
    sub_range: np.ndarray
    sub_cos: np.ndarray
    sub_power: np.ndarray
    sub_u: np.ndarray
    sub_v: np.ndarray
    waveform: np.ndarray
    t0: np.ndarray
    n_returns: np.ndarray
    ret_range: np.ndarray
    ret_amp: np.ndarray
    ret_tri: np.ndarray
    ret_bin: np.ndarray
    S: int


def _specular(specular):
    if specular is None:
        return None, None
    ks, n = specular
    return np.ascontiguousarray(ks, dtype=np.float32), np.ascontiguousarray(n, dtype=np.float32)


def range_noise(sc, pulse, ret):
    """The ranging error of return slot `ret` of pulse `pulse` (0 without noise)."""
    st = scanner_struct(sc)
    return lib().orc_range_noise(ctypes.byref(st), int(pulse), int(ret))


def surface_response(ct, ks, n):
    """(1 - ks) cos + ks max(cos 2 theta, 0)^n of a triangle seen at incidence cos ct."""
    return lib().orc_surface_response(float(ct), float(ks), float(n))


def simulate(mesh, pulses, sc, select=None, t0=None, threads=0, waveform=True, voxels=None, specular=None):
    """Forward over all pulses, or over the pulse indices in ``select``; ``voxels``: an
    optional transmissive voxel grid (see voxel_struct); ``specular``: optional per-triangle
    (specularity, Phong exponent)."""
    mesh.checked()
    st = scanner_struct(sc)
    S = pattern_size(st.n_subrays, st.beam_quality)
    if S <= 0:
        raise ValueError("bad pattern request")
    sel = None if select is None else np.ascontiguousarray(select, dtype=np.int64)
    n = pulses.n if sel is None else sel.size
    nb, K = st.n_bins, st.max_returns
    r = OracleResult(np.zeros((n, S), np.int32), np.zeros((n, S)), np.zeros((n, S)), np.zeros((n, S)),
                     np.zeros((n, S)), np.zeros((n, S)),
                     np.zeros((n, nb)) if waveform else None, np.zeros(n), np.zeros(n, np.int32),
                     np.zeros((n, K)), np.zeros((n, K)), np.zeros((n, K), np.int32), np.zeros((n, K), np.int32), S)
    t0a = None if t0 is None else np.ascontiguousarray(t0, dtype=np.float64)
    o = np.ascontiguousarray(pulses.origins, dtype=np.float64)
    d = np.ascontiguousarray(pulses.directions, dtype=np.float32)
    vst, keep = voxel_struct(voxels) if voxels is not None else (None, None)
    sk, sn = _specular(specular)
    got = lib().orc_simulate_ext(_ptr(mesh.vertices), mesh.n_vertices, _ptr(mesh.triangles), _ptr(mesh.reflectance),
                                 mesh.n_triangles, ctypes.byref(st), _ptr(o), _ptr(d), pulses.n,
                                 _ptr(sel), n, _ptr(t0a),
                                 _ptr(r.sub_tri), _ptr(r.sub_range), _ptr(r.sub_cos), _ptr(r.sub_power),
                                 _ptr(r.sub_u), _ptr(r.sub_v),
                                 _ptr(r.waveform), _ptr(r.t0), _ptr(r.n_returns), _ptr(r.ret_range), _ptr(r.ret_amp),
                                 _ptr(r.ret_tri), _ptr(r.ret_bin), int(threads),
                                 ctypes.byref(vst) if vst is not None else None, _ptr(sk), _ptr(sn))
    del keep
    if got != S:
        raise RuntimeError("oracle simulate failed")
    return r


def lut_g(voxels, vz):
    """The leaf-angle table's value at vertical component |vz|."""
    vst, keep = voxel_struct(voxels)
    return lib().orc_lut_g(ctypes.byref(vst), float(vz))


def voxel_hit(voxels, O, d, t_limit, pulse, subray):
    """(voxel index or -1, hit distance, sigma) of one ray through the grid."""
    vst, keep = voxel_struct(voxels)
    O = np.ascontiguousarray(O, dtype=np.float64)
    d = np.ascontiguousarray(d, dtype=np.float64)
    n_vox = int(np.asarray(voxels["pad"]).size)
    c0 = ((int(pulse) * 64 + int(subray)) * n_vox) & 0xFFFFFFFFFFFFFFFF
    t = ctypes.c_double(0.0)
    sg = ctypes.c_double(0.0)
    vi = lib().orc_voxel_hit(ctypes.byref(vst), _ptr(O), _ptr(d), float(t_limit), c0, ctypes.byref(t),
                             ctypes.byref(sg))
    return int(vi), t.value, sg.value


def gradient(mesh, pulses, sc, t0, grad_wf, threads=0, voxels=None, specular=None):
    """(grad_reflectance [T], grad_z [V]) of L with dL/dwf = grad_wf at fixed t0; ``voxels``: an
    optional transmissive voxel grid (its echoes are constants); ``specular``: optional
    per-triangle (specularity, Phong exponent)."""
    st = scanner_struct(sc)
    vst, keep = voxel_struct(voxels) if voxels is not None else (None, None)
    sk, sn = _specular(specular)
    gr = np.zeros(mesh.n_triangles)
    gz = np.zeros(mesh.n_vertices)
    o = np.ascontiguousarray(pulses.origins, dtype=np.float64)
    d = np.ascontiguousarray(pulses.directions, dtype=np.float32)
    t0 = np.ascontiguousarray(t0, dtype=np.float64)
    G = np.ascontiguousarray(grad_wf, dtype=np.float64)
    got = lib().orc_gradient_ext(_ptr(mesh.vertices), mesh.n_vertices, _ptr(mesh.triangles),
                                 _ptr(mesh.reflectance), mesh.n_triangles, ctypes.byref(st), _ptr(o), _ptr(d),
                                 pulses.n, _ptr(t0), _ptr(G), _ptr(gr), _ptr(gz), int(threads),
                                 ctypes.byref(vst) if vst is not None else None, _ptr(sk), _ptr(sn))
    del keep
    if got < 0:
        raise RuntimeError("oracle gradient failed")
    return gr, gz


def instance_mesh(parts, instances):
    """The scene of parts placed by affine maps (Sec. 3.5, Sec. 5.1): instance i of part p
    contributes part p's triangles with vertices A x + t (``instances``: (part, affine 3 x 4)),
    in instance order; reflectance is the part's."""
    from synth import Mesh
    vs, ts, rs = [], [], []
    off = 0
    for part, aff in instances:
        m = parts[part]
        a = np.ascontiguousarray(aff, dtype=np.float64).reshape(3, 4)
        v = np.ascontiguousarray(m.vertices, dtype=np.float32)
        w = np.empty_like(v)
        if v.shape[0]:
            lib().orc_instance_vertices(_ptr(v), v.shape[0], _ptr(a), _ptr(w))
        vs.append(w)
        ts.append(m.triangles.astype(np.int64) + off)
        rs.append(m.reflectance)
        off += v.shape[0]
    cat = lambda xs, shape, dt: np.concatenate(xs).astype(dt) if xs else np.zeros(shape, dt)
    return Mesh(cat(vs, (0, 3), np.float32), cat(ts, (0, 3), np.int32), cat(rs, (0,), np.float32))


def max_threads():
    return int(lib().orc_max_threads())
