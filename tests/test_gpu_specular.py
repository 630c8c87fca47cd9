"""GPU parity of specular materials (Sec. 5.1: reflectance and specularity;
the Phong-type response f = (1 - ks) cos + ks max(cos 2 theta, 0)^n) through the
C ABI against the FP64 oracle, at the tolerances of parity_util.  The library
shades in FP32: cos theta carries a few 2^-24 of relative error, and
(2 cos^2 - 1)^n multiplies it by about 4n + 3, so with exponents up to 8 a
subray's power is within 1e-5 relative (the waveform bound)."""
import sys

import numpy as np
import pytest

import oracle
from synth import configs
from parity_util import attribution_excused, check_hits, check_returns, check_waveforms, to_np

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2101_09154_amd as vp
    return vp.Context(0)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _materials(n_tri, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, 0.9, n_tri).astype(np.float32), rng.uniform(1.0, 8.0, n_tri).astype(np.float32)


def test_specular_matches_oracle(ctx):
    mesh, pulses, sc = configs.small_tls()
    ks, n = _materials(mesh.n_triangles, 3)
    scene = ctx.scene(mesh.vertices, mesh.triangles, mesh.reflectance)
    o, d = _dev(pulses.origins), _dev(pulses.directions)
    lam = to_np(ctx.simulate(scene, sc, o, d))
    scene.set_specular(_dev(ks), _dev(n))
    g = to_np(ctx.simulate(scene, sc, o, d))
    torch.cuda.synchronize()
    sel = np.arange(pulses.n)
    r = oracle.simulate(mesh, pulses, sc, specular=(ks, n))
    rep = {}
    ok_h = check_hits(mesh, pulses, sc, sel, g, r, rep)
    ok_w = check_waveforms(g, r, rep)
    ok_r, tri_bad = check_returns(g, r, sc, rep)
    left = attribution_excused(mesh, pulses, sc, sel, g, r, tri_bad)
    hit = r.sub_tri >= 0
    prel = np.abs(g["subray_power"][:, :r.S][hit] - r.sub_power[hit]) / r.sub_power[hit]
    rep["power_rel_worst"] = float(prel.max())
    say("specular small_tls", rep)
    assert ok_h and ok_w and ok_r and not left, rep
    assert rep["power_rel_worst"] <= 1e-5, rep
    # the term changes the echoes
    assert not np.array_equal(lam["subray_power"], g["subray_power"])
    # zero specularity, and the term turned off, are bitwise the Lambertian forward
    scene.set_specular(_dev(np.zeros_like(ks)), _dev(n))
    z = to_np(ctx.simulate(scene, sc, o, d))
    scene.set_specular()
    off = to_np(ctx.simulate(scene, sc, o, d))
    torch.cuda.synchronize()
    for k in lam:
        assert np.array_equal(lam[k], z[k], equal_nan=True), k
        assert np.array_equal(lam[k], off[k], equal_nan=True), k


def test_specular_adjoint_matches_oracle(ctx):
    mesh, target, pulses, sc = configs.diff_als(n_lines=40, per_line=50)
    ks, n = _materials(mesh.n_triangles, 4)
    scene = ctx.scene(mesh.vertices, mesh.triangles, mesh.reflectance)
    scene.set_specular(_dev(ks), _dev(n))
    o, d = _dev(pulses.origins), _dev(pulses.directions)
    base = oracle.simulate(mesh, pulses, sc, specular=(ks, n))
    tgt = oracle.simulate(target, pulses, sc, t0=base.t0).waveform
    G = 2.0 * (base.waveform - tgt)
    gr_o, gz_o = oracle.gradient(mesh, pulses, sc, base.t0, G, specular=(ks, n))
    t0d = _dev(base.t0)
    out = ctx.simulate(scene, sc, o, d, t0=t0d)
    gr, gz = ctx.waveform_backward(scene, sc, o, d, t0d, out["subray_tri"], _dev(G.astype(np.float32)))
    torch.cuda.synchronize()
    assert np.array_equal(out["subray_tri"].cpu().numpy()[:, :base.S], base.sub_tri)
    er = np.linalg.norm(gr.cpu().numpy() - gr_o) / np.linalg.norm(gr_o)
    ez = np.linalg.norm(gz.cpu().numpy() - gz_o) / np.linalg.norm(gz_o)
    say("specular adjoint rel L2: reflectance %.2e heights %.2e" % (er, ez))
    assert er <= 1e-4 and ez <= 1e-4


def test_specular_als_full_sampled(ctx):
    # the ALS workload at full size in the launch configuration bench.py times,
    # a lobe on every triangle; sampled pulses against the oracle
    mesh, pulses, sc = configs.als_buildings()
    ks, n = _materials(mesh.n_triangles, 9)
    scene = ctx.scene(mesh.vertices, mesh.triangles, mesh.reflectance)
    scene.set_specular(_dev(ks), _dev(n))
    prev = ctx.launch_config()
    ctx.set_launch_config(block_waves=2, stack_lds=8)
    try:
        out = ctx.simulate(scene, sc, _dev(pulses.origins), _dev(pulses.directions))
        torch.cuda.synchronize()
    finally:
        ctx.set_launch_config(**{k: prev[k] for k in ("block_waves", "stack_lds", "persistent_blocks", "pack", "cone")})
    rng = np.random.default_rng(12)
    sel = np.sort(rng.choice(pulses.n, 24, replace=False))
    idx = torch.from_numpy(sel).cuda()
    g = {k: v.index_select(0, idx).cpu().numpy() for k, v in out.items()}
    r = oracle.simulate(mesh, pulses, sc, select=sel, specular=(ks, n))
    rep = {}
    ok_h = check_hits(mesh, pulses, sc, sel, g, r, rep)
    ok_w = check_waveforms(g, r, rep)
    ok_r, tri_bad = check_returns(g, r, sc, rep)
    left = attribution_excused(mesh, pulses, sc, sel, g, r, tri_bad)
    say("specular als_buildings", rep)
    assert ok_h and ok_w and ok_r and not left, rep
