"""MI355X-native full-waveform virtual laser scanning (the hot path of HELIOS++,
arXiv 2101.09154): HIP kernels for gfx950 behind the C ABI of include/vls.h,
with a thin ctypes binding."""
from . import vls
from .autograd import WaveformFn
from .vls import NOALLOC_MAX_PULSES, Context, Scene, VlsError, n_subrays, scanner_desc

__all__ = ["vls", "WaveformFn", "NOALLOC_MAX_PULSES", "Context", "Scene", "VlsError", "n_subrays", "scanner_desc"]
