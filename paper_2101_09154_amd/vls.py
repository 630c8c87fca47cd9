"""Python binding of the C ABI in include/vls.h (argument marshalling only).

Every computation runs in the HIP library ``libvls.so``; torch is used for
device memory and streams.  If the library is missing, every entry point
raises: there is no fallback path.
"""
import ctypes
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
# VLS_LIBRARY may point at another build of the same library (e.g. a tuning variant)
LIB_PATH = os.environ.get("VLS_LIBRARY") or os.path.join(HERE, "libvls.so")

OK = 0
STATUS = {0: "ok", 1: "invalid argument", 2: "out of memory", 3: "device error", 4: "not built",
          5: "unsupported", 6: "internal error"}
MEM_HOST = 0
MAX_CANDIDATES = 255  # VLS_MAX_CANDIDATES: triangles the cone pass lists per pulse
NOALLOC_MAX_PULSES = 32768  # VLS_NOALLOC_MAX_PULSES: pulses per vls_simulate_noalloc call
MEM_DEVICE = 1
PULSE_GAUSSIAN = 0
PULSE_EQ3 = 1


class VlsError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


P = ctypes.c_void_p
i32 = ctypes.c_int32
i64 = ctypes.c_int64
f64 = ctypes.c_double


class MeshDesc(ctypes.Structure):
    _fields_ = [("vertices", P), ("triangles", P), ("reflectance", P), ("n_vertices", i64),
                ("n_triangles", i64), ("memory", i32), ("reserved", i32)]


class SceneStats(ctypes.Structure):
    _fields_ = [("n_vertices", i64), ("n_triangles", i64), ("n_internal_nodes", i64), ("device_bytes", i64),
                ("max_depth", i32), ("max_supported_depth", i32), ("bounds_lo", ctypes.c_float * 3),
                ("bounds_hi", ctypes.c_float * 3), ("box_pad", ctypes.c_float), ("reserved", ctypes.c_float)]


class VoxelDesc(ctypes.Structure):
    _fields_ = [("origin", f64 * 3), ("voxel_size_m", f64), ("nx", i32), ("ny", i32), ("nz", i32), ("n_lut", i32),
                ("pad", P), ("lut", P), ("seed", ctypes.c_uint64)]


class InstanceDesc(ctypes.Structure):
    _fields_ = [("part", i32), ("reserved", i32), ("affine", f64 * 12)]


class ScannerDesc(ctypes.Structure):
    _fields_ = [("divergence_rad", f64), ("pattern_extent", f64), ("pulse_width_ns", f64), ("bin_ns", f64),
                ("window_pre_ns", f64), ("peak_power_w", f64), ("receiver_diameter_m", f64),
                ("efficiency", f64), ("min_echo_abs", f64), ("min_echo_rel", f64), ("n_subrays", i32),
                ("beam_quality", i32), ("pulse_shape", i32), ("n_bins", i32), ("max_returns", i32),
                ("reserved", i32), ("range_noise_m", f64), ("noise_seed", ctypes.c_uint64)]


class PulseBatch(ctypes.Structure):
    _fields_ = [("origins", P), ("directions", P), ("window_t0_ns", P), ("n_pulses", i64),
                ("segment_offsets", P), ("segment_scanner", P), ("n_segments", i32), ("reserved", i32)]


class Outputs(ctypes.Structure):
    _fields_ = [("subray_tri", P), ("subray_range", P), ("subray_cos", P), ("subray_power", P),
                ("waveform", P), ("window_t0_ns", P), ("n_returns", P), ("ret_range", P),
                ("ret_amplitude", P), ("ret_tri", P), ("ret_bin", P)]


class LaunchConfig(ctypes.Structure):
    _fields_ = [("block_waves", i32), ("stack_lds", i32), ("persistent_blocks", i32), ("pack", i32),
                ("cone", i32), ("cover_off", i32), ("grouped", i32), ("reserved", i32)]


class SurveyDesc(ctypes.Structure):
    _fields_ = [("waypoints", P), ("n_waypoints", i32), ("deflector", i32), ("speed_mps", f64),
                ("pulse_rate_hz", f64), ("scan_freq_hz", f64), ("scan_angle_rad", f64), ("n_fibres", i32),
                ("platform", i32), ("t0_s", f64), ("platform_noise_m", f64), ("seed", ctypes.c_uint64),
                ("accel_mps2", f64), ("leg_yaw", P), ("bank_angle_rad", f64)]


DEFLECTORS = {"polygon": 0, "swing": 1, "conic": 2, "fibre": 3}
PLATFORMS = {"linear": 0, "multicopter": 1, "multicopter_smooth": 2}


class Profile(ctypes.Structure):
    _fields_ = [("cone_ms", f64), ("fused_ms", f64), ("cone_launches", ctypes.c_int64),
                ("fused_launches", ctypes.c_int64), ("packet_ms", f64), ("packet_launches", ctypes.c_int64)]


class TuneResult(ctypes.Structure):
    _fields_ = [("best", LaunchConfig), ("best_ms", f64), ("default_ms", f64), ("n_tried", i32),
                ("from_cache", i32)]


_lib = None

_SIGS = {
    "vls_status_string": ([i32], ctypes.c_char_p),
    "vls_last_error": ([], ctypes.c_char_p),
    "vls_version": ([], i32),
    "vls_context_create": ([i32, P], i32),
    "vls_context_destroy": ([P], i32),
    "vls_scene_create": ([P, P, P, P], i32),
    "vls_scene_update_vertices": ([P, P, P], i32),
    "vls_scene_update_reflectance": ([P, P, P], i32),
    "vls_scene_set_voxels": ([P, P, P], i32),
    "vls_scene_set_specular": ([P, P, P, P], i32),
    "vls_scene_create_instanced": ([P, P, i32, P, i32, P, P], i32),
    "vls_scene_create_two_level": ([P, P, i32, P, i32, P, P], i32),
    "vls_scene_stats_get": ([P, P], i32),
    "vls_scene_export": ([P, P, P, P, P], i32),
    "vls_scene_destroy": ([P], i32),
    "vls_scanner_subrays": ([P, P], i32),
    "vls_trace": ([P, P, P, i32, P, P, P], i32),
    "vls_waveform": ([P, P, i32, P, P, P], i32),
    "vls_returns": ([P, P, i32, P, P, P], i32),
    "vls_echo_width": ([P, P, i32, P, P, P, P], i32),
    "vls_generate_pulses": ([P, P, ctypes.c_int64, ctypes.c_int64, P, P, P], i32),
    "vls_simulate": ([P, P, P, i32, P, P, P], i32),
    "vls_simulate_noalloc": ([P, P, P, P, P, P], i32),
    "vls_set_deterministic": ([P, i32], i32),
    "vls_set_launch_config": ([P, P], i32),
    "vls_get_launch_config": ([P, P], i32),
    "vls_synchronize": ([P, P], i32),
    "vls_trace_counts": ([P, P, P, i32, P, P, P], i32),
    "vls_waveform_backward": ([P, P, P, P, P, P, P, P, P], i32),
    "vls_graph_capture": ([P, P, P, i32, P, P, P], i32),
    "vls_cone_candidates": ([P, P, P, i32, P, P, P], i32),
    "vls_graph_launch": ([P, P], i32),
    "vls_graph_destroy": ([P], i32),
    "vls_autotune": ([P, P, P, i32, P, P, ctypes.c_char_p, P, P], i32),
    "vls_profile_enable": ([P, i32], i32),
    "vls_profile_read": ([P, P], i32),
}


def library_path():
    return LIB_PATH


def lib():
    """Load libvls.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libvls.so is not built (run __graft_entry__.build() or "
                               "python -m paper_2101_09154_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def declared_symbols():
    return sorted(_SIGS)


def _check(status):
    if status != OK:
        raise VlsError(status, lib().vls_last_error().decode(errors="replace"))


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _dev(t, dtype, shape=None, name="tensor"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("%s must have shape %s, got %s" % (name, tuple(shape), tuple(t.shape)))
    return t


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def scanner_desc(sc):
    """Scanner dict (keys as in ScannerDesc; pulse_shape 'gaussian' or 'eq3') -> ScannerDesc."""
    shape = sc.get("pulse_shape", "gaussian")
    return ScannerDesc(divergence_rad=sc["divergence_rad"], pattern_extent=sc.get("pattern_extent", 1.0),
                       pulse_width_ns=sc["pulse_width_ns"], bin_ns=sc["bin_ns"],
                       window_pre_ns=sc.get("window_pre_ns", -1.0), peak_power_w=sc.get("peak_power_w", 1.0),
                       receiver_diameter_m=sc.get("receiver_diameter_m", 1.0), efficiency=sc.get("efficiency", 1.0),
                       min_echo_abs=sc.get("min_echo_abs", 0.0), min_echo_rel=sc.get("min_echo_rel", 1e-3),
                       n_subrays=sc.get("n_subrays", 0), beam_quality=sc.get("beam_quality", 0),
                       pulse_shape=PULSE_EQ3 if shape in ("eq3", PULSE_EQ3) else PULSE_GAUSSIAN,
                       n_bins=sc["n_bins"], max_returns=sc.get("max_returns", 8), reserved=0,
                       range_noise_m=sc.get("range_noise_m", 0.0),
                       noise_seed=int(sc.get("noise_seed", 0)) & 0xFFFFFFFFFFFFFFFF)


def n_subrays(sc):
    d = scanner_desc(sc)
    out = i32(0)
    _check(lib().vls_scanner_subrays(ctypes.byref(d), ctypes.byref(out)))
    return int(out.value)


class Scene:
    @classmethod
    def instanced(cls, ctx, parts, instances, stream=None, two_level=False):
        """A scene of parts placed by affine maps: parts = [(vertices, triangles, reflectance)]
        (host numpy arrays or device tensors), instances = [(part, affine 3 x 4)]; two_level keeps
        the parts once under a tree of the instances (vls_scene_create_two_level)."""
        descs = (MeshDesc * max(len(parts), 1))()
        keep = []
        for i, (v, t, r) in enumerate(parts):
            if isinstance(v, np.ndarray):
                v = np.ascontiguousarray(v, dtype=np.float32).reshape(-1, 3)
                t = np.ascontiguousarray(t, dtype=np.int32).reshape(-1, 3)
                r = np.ascontiguousarray(r, dtype=np.float32).reshape(-1)
                descs[i] = MeshDesc(v.ctypes.data, t.ctypes.data, r.ctypes.data, v.shape[0], t.shape[0], MEM_HOST, 0)
            else:
                v = _dev(v, torch.float32, name="vertices")
                t = _dev(t, torch.int32, name="triangles")
                r = _dev(r, torch.float32, name="reflectance")
                descs[i] = MeshDesc(v.data_ptr(), t.data_ptr(), r.data_ptr(), v.shape[0], t.shape[0], MEM_DEVICE, 0)
            keep.append((v, t, r))
        inst = (InstanceDesc * max(len(instances), 1))()
        for j, (part, aff) in enumerate(instances):
            a = np.ascontiguousarray(aff, dtype=np.float64).reshape(12)
            inst[j] = InstanceDesc(int(part), 0, (f64 * 12)(*a.tolist()))
        self = cls.__new__(cls)
        self.ctx = ctx
        self._h = P()
        fn = lib().vls_scene_create_two_level if two_level else lib().vls_scene_create_instanced
        _check(fn(ctx._h, descs, len(parts), inst, len(instances), _stream(stream), ctypes.byref(self._h)))
        del keep
        st = self.stats()
        self.n_vertices = int(st["n_vertices"])
        self.n_triangles = int(st["n_triangles"])
        return self

    def __init__(self, ctx, vertices, triangles, reflectance, stream=None):
        self.ctx = ctx
        self._h = P()
        if isinstance(vertices, np.ndarray):
            v = np.ascontiguousarray(vertices, dtype=np.float32)
            t = np.ascontiguousarray(triangles, dtype=np.int32)
            r = np.ascontiguousarray(reflectance, dtype=np.float32)
            desc = MeshDesc(v.ctypes.data, t.ctypes.data, r.ctypes.data, v.shape[0], t.shape[0], MEM_HOST, 0)
            keep = (v, t, r)
        else:
            v = _dev(vertices, torch.float32, name="vertices")
            t = _dev(triangles, torch.int32, name="triangles")
            r = _dev(reflectance, torch.float32, name="reflectance")
            desc = MeshDesc(v.data_ptr(), t.data_ptr(), r.data_ptr(), v.shape[0], t.shape[0], MEM_DEVICE, 0)
            keep = (v, t, r)
        _check(lib().vls_scene_create(ctx._h, ctypes.byref(desc), _stream(stream), ctypes.byref(self._h)))
        del keep
        self.n_vertices = int(desc.n_vertices)
        self.n_triangles = int(desc.n_triangles)

    def stats(self):
        s = SceneStats()
        _check(lib().vls_scene_stats_get(self._h, ctypes.byref(s)))
        return {f: (list(getattr(s, f)) if f.startswith("bounds") else getattr(s, f)) for f, _ in s._fields_}

    def update_vertices(self, vertices, stream=None):
        v = _dev(vertices, torch.float32, (self.n_vertices, 3), "vertices")
        _check(lib().vls_scene_update_vertices(self._h, _ptr(v), _stream(stream)))

    def update_reflectance(self, reflectance, stream=None):
        r = _dev(reflectance, torch.float32, (self.n_triangles,), "reflectance")
        _check(lib().vls_scene_update_reflectance(self._h, _ptr(r), _stream(stream)))

    def set_specular(self, specularity=None, exponent=None, stream=None):
        """Per-triangle specularity ks and Phong exponent n (device tensors [n_triangles] float32);
        both None turns the specular term off."""
        if specularity is None and exponent is None:
            _check(lib().vls_scene_set_specular(self._h, None, None, _stream(stream)))
            return
        k = _dev(specularity, torch.float32, (self.n_triangles,), "specularity")
        n = _dev(exponent, torch.float32, (self.n_triangles,), "exponent")
        _check(lib().vls_scene_set_specular(self._h, _ptr(k), _ptr(n), _stream(stream)))
        self._spec_keep = (k, n)

    def set_voxels(self, origin, voxel_size_m, pad, lut, seed=0, stream=None):
        """A transmissive voxel grid: pad [nz, ny, nx] plant area density, lut [n, 2] rows of the
        leaf-angle table (vertical component, g); host arrays, copied."""
        pad = np.ascontiguousarray(pad, dtype=np.float32)
        lut = np.ascontiguousarray(lut, dtype=np.float64).reshape(-1, 2)
        if pad.ndim != 3:
            raise ValueError("pad must be [nz, ny, nx]")
        nz, ny, nx = pad.shape
        desc = VoxelDesc((f64 * 3)(*[float(x) for x in origin]), float(voxel_size_m), nx, ny, nz, lut.shape[0],
                         pad.ctypes.data, lut.ctypes.data, int(seed) & 0xFFFFFFFFFFFFFFFF)
        _check(lib().vls_scene_set_voxels(self._h, ctypes.byref(desc), _stream(stream)))
        self.n_voxels = int(pad.size)

    def export(self):
        n = self.n_triangles
        nodes = np.zeros((max(n - 1, 0), 16), np.float32)
        leaf = np.zeros(n, np.int32)
        mort = np.zeros(n, np.uint64)
        root = i32(0)
        _check(lib().vls_scene_export(self._h, nodes.ctypes.data if nodes.size else None,
                                      leaf.ctypes.data if n else None, mort.ctypes.data if n else None,
                                      ctypes.byref(root)))
        return nodes, leaf, mort, int(root.value)

    def close(self):
        if self._h:
            _check(lib().vls_scene_destroy(self._h))
            self._h = P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Graph:
    def __init__(self):
        self._h = P()
        self._keep = None

    def launch(self, stream=None):
        _check(lib().vls_graph_launch(self._h, _stream(stream)))

    def close(self):
        if self._h:
            _check(lib().vls_graph_destroy(self._h))
            self._h = P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Context:
    def __init__(self, device=0):
        self.device = device
        self._h = P()
        _check(lib().vls_context_create(device, ctypes.byref(self._h)))

    def close(self):
        if self._h:
            _check(lib().vls_context_destroy(self._h))
            self._h = P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def scene(self, vertices, triangles, reflectance, stream=None):
        return Scene(self, vertices, triangles, reflectance, stream)

    def scene_instanced(self, parts, instances, stream=None, two_level=False):
        return Scene.instanced(self, parts, instances, stream, two_level)

    def set_launch_config(self, block_waves=1, stack_lds=16, persistent_blocks=0, pack=0, cone=1, cover_off=0,
                          grouped=1):
        c = LaunchConfig(block_waves, stack_lds, persistent_blocks, pack, cone, cover_off, grouped, 0)
        _check(lib().vls_set_launch_config(self._h, ctypes.byref(c)))

    def set_deterministic(self, on=True):
        """Fixed summation order for the adjoint (bitwise repeatable gradients)."""
        _check(lib().vls_set_deterministic(self._h, 1 if on else 0))

    def launch_config(self):
        c = LaunchConfig()
        _check(lib().vls_get_launch_config(self._h, ctypes.byref(c)))
        return {"block_waves": c.block_waves, "stack_lds": c.stack_lds, "persistent_blocks": c.persistent_blocks,
                "pack": c.pack, "cone": c.cone, "cover_off": c.cover_off, "grouped": c.grouped}

    def synchronize(self, stream=None):
        _check(lib().vls_synchronize(self._h, _stream(stream)))

    # -------------------------------------------------------------- marshalling helpers
    @staticmethod
    def _scanners(scanners):
        if isinstance(scanners, dict):
            scanners = [scanners]
        arr = (ScannerDesc * len(scanners))(*[scanner_desc(s) for s in scanners])
        return arr, len(scanners)

    @staticmethod
    def _batch(origins, directions, t0=None, segment_offsets=None, segment_scanner=None):
        n = origins.shape[0]
        _dev(origins, torch.float64, (n, 3), "origins")
        _dev(directions, torch.float32, (n, 3), "directions")
        _dev(t0, torch.float64, (n,), "window_t0_ns")
        keep = []
        b = PulseBatch(origins.data_ptr(), directions.data_ptr(), None if t0 is None else t0.data_ptr(), n,
                       None, None, 0, 0)
        if segment_offsets is not None:
            so = np.ascontiguousarray(segment_offsets, dtype=np.int64)
            ss = np.ascontiguousarray(segment_scanner, dtype=np.int32)
            keep += [so, ss]
            b.segment_offsets = so.ctypes.data
            b.segment_scanner = ss.ctypes.data
            b.n_segments = ss.size
        return b, keep

    @staticmethod
    def _outputs(d):
        return Outputs(*[_ptr(d.get(k)) for k in ("subray_tri", "subray_range", "subray_cos", "subray_power",
                                                   "waveform", "window_t0_ns", "n_returns", "ret_range",
                                                   "ret_amplitude", "ret_tri", "ret_bin")])

    @staticmethod
    def alloc_outputs(n, S, n_bins, K, device, subrays=True, waveform=True, returns=True):
        o = {}
        dev = torch.device("cuda", device) if isinstance(device, int) else device
        if subrays:
            o["subray_tri"] = torch.empty((n, S), dtype=torch.int32, device=dev)
            o["subray_range"] = torch.empty((n, S), dtype=torch.float64, device=dev)
            o["subray_cos"] = torch.empty((n, S), dtype=torch.float32, device=dev)
            o["subray_power"] = torch.empty((n, S), dtype=torch.float32, device=dev)
        if waveform:
            o["waveform"] = torch.empty((n, n_bins), dtype=torch.float32, device=dev)
        o["window_t0_ns"] = torch.empty(n, dtype=torch.float64, device=dev)
        if returns:
            o["n_returns"] = torch.empty(n, dtype=torch.int32, device=dev)
            o["ret_range"] = torch.empty((n, K), dtype=torch.float32, device=dev)
            o["ret_amplitude"] = torch.empty((n, K), dtype=torch.float32, device=dev)
            o["ret_tri"] = torch.empty((n, K), dtype=torch.int32, device=dev)
            o["ret_bin"] = torch.empty((n, K), dtype=torch.int32, device=dev)
        return o

    # -------------------------------------------------------------- the hot path
    def simulate(self, scene, scanners, origins, directions, *, t0=None, out=None, subrays=True, waveform=True,
                 segment_offsets=None, segment_scanner=None, stream=None):
        """Fused trace + power + waveform + returns; returns the output dict."""
        scs = [scanners] if isinstance(scanners, dict) else list(scanners)
        S = max(n_subrays(s) for s in scs)
        if out is None:
            out = self.alloc_outputs(origins.shape[0], S, scs[0]["n_bins"], scs[0].get("max_returns", 8),
                                     origins.device, subrays=subrays, waveform=waveform)
        arr, ns = self._scanners(scs)
        b, keep = self._batch(origins, directions, t0, segment_offsets, segment_scanner)
        o = self._outputs(out)
        _check(lib().vls_simulate(self._h, scene._h, arr, ns, ctypes.byref(b), ctypes.byref(o), _stream(stream)))
        return out

    def simulate_noalloc(self, scene, scanner, origins, directions, out, *, t0=None, stream=None):
        """vls_simulate_noalloc: the fused path on one scanner with the library's
        fixed device scratch; `out` (from alloc_outputs) is required."""
        arr, ns = self._scanners([scanner])
        b, keep = self._batch(origins, directions, t0, None, None)
        o = self._outputs(out)
        _check(lib().vls_simulate_noalloc(self._h, scene._h, arr, ctypes.byref(b), ctypes.byref(o), _stream(stream)))
        return out

    def trace(self, scene, scanners, origins, directions, *, out=None, segment_offsets=None, segment_scanner=None,
              stream=None):
        scs = [scanners] if isinstance(scanners, dict) else list(scanners)
        S = max(n_subrays(s) for s in scs)
        if out is None:
            out = self.alloc_outputs(origins.shape[0], S, 3, 1, origins.device, waveform=False, returns=False)
        arr, ns = self._scanners(scs)
        b, keep = self._batch(origins, directions, None, segment_offsets, segment_scanner)
        o = self._outputs(out)
        _check(lib().vls_trace(self._h, scene._h, arr, ns, ctypes.byref(b), ctypes.byref(o), _stream(stream)))
        return out

    def waveform(self, scanners, origins, directions, out, *, t0=None, segment_offsets=None, segment_scanner=None,
                 stream=None):
        arr, ns = self._scanners(scanners)
        b, keep = self._batch(origins, directions, t0, segment_offsets, segment_scanner)
        o = self._outputs(out)
        _check(lib().vls_waveform(self._h, arr, ns, ctypes.byref(b), ctypes.byref(o), _stream(stream)))
        return out

    def waveform_backward(self, scene, scanner, origins, directions, t0, subray_tri, grad_waveform, *,
                          grad_reflectance=None, grad_z=None, stream=None):
        """(grad_reflectance [n_tri], grad_z [n_vert]) of a waveform loss, hit selection and t0 fixed."""
        n = origins.shape[0]
        dev = origins.device
        if grad_reflectance is None:
            grad_reflectance = torch.empty(scene.n_triangles, dtype=torch.float32, device=dev)
        if grad_z is None:
            grad_z = torch.empty(scene.n_vertices, dtype=torch.float32, device=dev)
        _dev(subray_tri, torch.int32, name="subray_tri")
        _dev(grad_waveform, torch.float32, (n, scanner["n_bins"]), "grad_waveform")
        _dev(grad_reflectance, torch.float32, (scene.n_triangles,), "grad_reflectance")
        _dev(grad_z, torch.float32, (scene.n_vertices,), "grad_z")
        d = scanner_desc(scanner)
        b, keep = self._batch(origins, directions, t0)
        _check(lib().vls_waveform_backward(self._h, scene._h, ctypes.byref(d), ctypes.byref(b), _ptr(subray_tri),
                                           _ptr(grad_waveform), _ptr(grad_reflectance), _ptr(grad_z),
                                           _stream(stream)))
        return grad_reflectance, grad_z

    def capture_graph(self, scene, scanners, origins, directions, out, *, t0=None, segment_offsets=None,
                      segment_scanner=None):
        """HIP graph of one simulate call; `out` and the inputs must outlive it."""
        arr, ns = self._scanners(scanners)
        b, keep = self._batch(origins, directions, t0, segment_offsets, segment_scanner)
        o = self._outputs(out)
        g = Graph()
        _check(lib().vls_graph_capture(self._h, scene._h, arr, ns, ctypes.byref(b), ctypes.byref(o),
                                       ctypes.byref(g._h)))
        g._keep = (origins, directions, t0, out, scene)
        return g

    def autotune(self, scene, scanners, origins, directions, out, *, cache_path=None, segment_offsets=None,
                 segment_scanner=None, stream=None):
        arr, ns = self._scanners(scanners)
        b, keep = self._batch(origins, directions, None, segment_offsets, segment_scanner)
        o = self._outputs(out)
        r = TuneResult()
        _check(lib().vls_autotune(self._h, scene._h, arr, ns, ctypes.byref(b), ctypes.byref(o),
                                  None if cache_path is None else cache_path.encode(), _stream(stream),
                                  ctypes.byref(r)))
        return {"best": {"block_waves": r.best.block_waves, "stack_lds": r.best.stack_lds,
                         "persistent_blocks": r.best.persistent_blocks, "pack": r.best.pack,
                         "cone": r.best.cone, "cover_off": r.best.cover_off, "grouped": r.best.grouped},
                "best_ms": r.best_ms, "default_ms": r.default_ms, "n_tried": r.n_tried,
                "from_cache": bool(r.from_cache)}

    def cone_candidates(self, scene, scanners, origins, directions, *, out=None, segment_offsets=None,
                        segment_scanner=None, stream=None):
        """[n, MAX_CANDIDATES + 1] int32: candidate count (-1 = overflow) then original
        triangle ids, per pulse."""
        n = origins.shape[0]
        if out is None:
            out = torch.empty((n, MAX_CANDIDATES + 1), dtype=torch.int32, device=origins.device)
        arr, ns = self._scanners(scanners)
        b, keep = self._batch(origins, directions, None, segment_offsets, segment_scanner)
        _check(lib().vls_cone_candidates(self._h, scene._h, arr, ns, ctypes.byref(b), _ptr(out), _stream(stream)))
        return out

    def profile(self, enable=True):
        """Record HIP events around the cone pass and the fused kernel of each
        eager simulate call (see profile_read)."""
        _check(lib().vls_profile_enable(self._h, 1 if enable else 0))

    def profile_read(self):
        """Summed kernel times (ms) and launch counts since the last read (waits for them)."""
        p = Profile()
        _check(lib().vls_profile_read(self._h, ctypes.byref(p)))
        return {"cone_ms": p.cone_ms, "fused_ms": p.fused_ms, "packet_ms": p.packet_ms,
                "cone_launches": int(p.cone_launches), "fused_launches": int(p.fused_launches),
                "packet_launches": int(p.packet_launches)}

    def trace_counts(self, scene, scanners, origins, directions, *, segment_offsets=None, segment_scanner=None,
                     stream=None):
        """(subrays, node visits, triangle tests) of tracing the batch (synchronous)."""
        arr, ns = self._scanners(scanners)
        b, keep = self._batch(origins, directions, None, segment_offsets, segment_scanner)
        c = (ctypes.c_uint64 * 3)()
        _check(lib().vls_trace_counts(self._h, scene._h, arr, ns, ctypes.byref(b), c, _stream(stream)))
        return int(c[0]), int(c[1]), int(c[2])

    def returns(self, scanners, origins, directions, out, *, segment_offsets=None, segment_scanner=None,
                stream=None):
        arr, ns = self._scanners(scanners)
        b, keep = self._batch(origins, directions, None, segment_offsets, segment_scanner)
        o = self._outputs(out)
        _check(lib().vls_returns(self._h, arr, ns, ctypes.byref(b), ctypes.byref(o), _stream(stream)))
        return out

    def generate_pulses(self, survey, first, count, *, origins=None, directions=None, device=0, stream=None):
        """Pulses [first, first + count) of a survey (dict: waypoints, deflector, speed_mps,
        pulse_rate_hz, scan_freq_hz, scan_angle_rad, n_fibres, t0_s, platform_noise_m, seed;
        platform "linear" (default), "multicopter" with accel_mps2 and optionally leg_yaw,
        [n_waypoints - 1, 2], or "multicopter_smooth" with accel_mps2 and bank_angle_rad)
        generated on the device: (origins float64 [count, 3],
        directions float32 [count, 3])."""
        wp = np.ascontiguousarray(survey["waypoints"], dtype=np.float64).reshape(-1, 3)
        ly = survey.get("leg_yaw")
        if ly is not None:
            ly = np.ascontiguousarray(ly, dtype=np.float64).reshape(-1, 2)
            if ly.shape[0] != max(wp.shape[0] - 1, 0):
                raise VlsError(1, "leg_yaw needs one row per leg")
        desc = SurveyDesc(wp.ctypes.data, wp.shape[0], DEFLECTORS[survey.get("deflector", "polygon")],
                          float(survey.get("speed_mps", 0.0)), float(survey["pulse_rate_hz"]),
                          float(survey.get("scan_freq_hz", 0.0)), float(survey.get("scan_angle_rad", 0.0)),
                          int(survey.get("n_fibres", 0)), PLATFORMS[survey.get("platform", "linear")],
                          float(survey.get("t0_s", 0.0)), float(survey.get("platform_noise_m", 0.0)),
                          int(survey.get("seed", 0)) & 0xFFFFFFFFFFFFFFFF, float(survey.get("accel_mps2", 0.0)),
                          None if ly is None else ly.ctypes.data, float(survey.get("bank_angle_rad", 0.0)))
        dev = torch.device("cuda", device) if isinstance(device, int) else device
        if origins is None:
            origins = torch.empty((count, 3), dtype=torch.float64, device=dev)
        if directions is None:
            directions = torch.empty((count, 3), dtype=torch.float32, device=dev)
        _dev(origins, torch.float64, (count, 3), "origins")
        _dev(directions, torch.float32, (count, 3), "directions")
        _check(lib().vls_generate_pulses(self._h, ctypes.byref(desc), int(first), int(count), _ptr(origins),
                                         _ptr(directions), _stream(stream)))
        del wp, ly
        return origins, directions

    def echo_width(self, scanners, origins, directions, out, *, width=None, segment_offsets=None,
                   segment_scanner=None, stream=None):
        """Echo width (ns) of every kept return in `out` (waveform, n_returns and ret_bin
        as written by simulate or returns): float32 [n, K], NaN where there is none."""
        arr, ns = self._scanners(scanners)
        b, keep = self._batch(origins, directions, None, segment_offsets, segment_scanner)
        o = self._outputs(out)
        n = origins.shape[0]
        K = out["ret_bin"].shape[1] if out.get("ret_bin") is not None else 1
        if width is None:
            width = torch.empty((n, K), dtype=torch.float32, device=origins.device)
        _dev(width, torch.float32, (n, K), "width")
        _check(lib().vls_echo_width(self._h, arr, ns, ctypes.byref(b), ctypes.byref(o), _ptr(width),
                                    _stream(stream)))
        return width
