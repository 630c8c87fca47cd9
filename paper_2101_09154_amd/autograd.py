"""torch.autograd.Function over the library's forward and adjoint kernels.

WaveformFn.apply(reflectance [T], heights [V], ...) -> waveform [n, n_bins].
The forward writes the new heights and reflectance into the scene (refitting
its boxes), runs the fused forward with the window origins t0 held fixed and
keeps the per-subray hit triangles; the backward runs the hand-written
adjoint kernel with those hits.  The scene is shared state: call backward
before the next forward on the same scene.
"""
import torch


class WaveformFn(torch.autograd.Function):
    @staticmethod
    def forward(fctx, reflectance, heights, vctx, scene, scanner, origins, directions, t0, base_xy):
        verts = torch.cat([base_xy, heights.detach()[:, None]], dim=1).contiguous()
        scene.update_vertices(verts)
        scene.update_reflectance(reflectance.detach().contiguous())
        out = vctx.simulate(scene, scanner, origins, directions, t0=t0)
        fctx.vctx = vctx
        fctx.scene = scene
        fctx.scanner = scanner
        fctx.save_for_backward(origins, directions, t0, out["subray_tri"])
        return out["waveform"]

    @staticmethod
    def backward(fctx, grad_wf):
        origins, directions, t0, sub_tri = fctx.saved_tensors
        g_refl, g_z = fctx.vctx.waveform_backward(fctx.scene, fctx.scanner, origins, directions, t0, sub_tri,
                                                  grad_wf.contiguous())
        return g_refl, g_z, None, None, None, None, None, None, None
