"""GPU parity of transmissive voxels (Sec. 3.5.4, Sec. 5.2) through the C ABI
against the FP64 oracle, at the tolerances of parity_util (a voxel echo against
anything else only at a tie in distance; Eq. 7's power to 1e-6 relative).

The draws are addressed by (pulse index in the call's batch, subray, voxel), so
the oracle is always run on the whole batch with a selection, never on a
re-indexed subset.
"""
import ctypes
import sys

import numpy as np
import pytest

import oracle
import synth
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


def _scene(ctx, mesh, vox):
    scene = ctx.scene(mesh.vertices, mesh.triangles, mesh.reflectance)
    if vox is not None:
        scene.set_voxels(vox["origin"], vox["size"], vox["pad"], vox["lut"], vox["seed"])
    return scene


def compare_vox(mesh, vox, pulses, sc, g, sel, label, min_voxel_frac=0.0):
    """g: GPU rows of the selected pulses of the whole batch `pulses`."""
    sel = np.asarray(sel)
    r = oracle.simulate(mesh, pulses, sc, select=sel, voxels=vox)
    rep = {}
    ok_h = check_hits(mesh, pulses, sc, sel, g, r, rep)
    ok_w = check_waveforms(g, r, rep)
    ok_r, tri_bad = check_returns(g, r, sc, rep)
    left = attribution_excused(mesh, pulses, sc, sel, g, r, tri_bad)
    rep["attribution_unexcused"] = left[:10]
    vfrac = float((r.sub_tri >= mesh.n_triangles).mean())
    rep["voxel_fraction"] = vfrac
    say(label, rep)
    assert ok_h, rep
    assert ok_w, rep
    assert ok_r, rep
    assert not left, rep
    assert vfrac >= min_voxel_frac, rep
    return r


def _slab_case(seed=3):
    """A ground plane under a 20 x 20 x 6 grid of 1 m voxels (a quarter empty),
    airborne lines through it, terrestrial pulses from inside it (some exactly
    along the grid's axes) and two pulses without a direction: 1,308 pulses."""
    rng = np.random.default_rng(seed)
    mesh = synth.flat_quad(-60.0, 60.0, -60.0, 60.0, 0.0, reflectance=0.4)
    pad = rng.uniform(0.05, 0.8, (6, 20, 20)).astype(np.float32)
    pad[rng.random(pad.shape) < 0.25] = 0.0
    vox = dict(origin=[-10.0, -10.0, 5.0], size=1.0, pad=pad, lut=configs.TABLE2_ROWS, seed=seed)
    als = synth.als_lines(0.0, np.linspace(-8.0, 8.0, 40), 40.0, 31, beta_deg=(-25.0, 25.0))
    tls = synth.tls_grid((0.3, 0.2, 8.0), 12, 5, el_deg=(-60.0, 40.0))
    axes = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], np.float32)
    o = np.concatenate([als.origins, tls.origins, np.tile([[0.3, 0.2, 8.0]], (6, 1)), np.tile([[1.0, 2.0, 3.0]], (2, 1))])
    d = np.concatenate([als.directions, tls.directions, axes, np.zeros((2, 3), np.float32)]).astype(np.float32)
    return mesh, vox, synth.Pulses(o, d)


SLAB_SC = configs.scanner(3e-3, 19, n_bins=256, bin_ns=0.5, max_returns=6)


def test_voxel_slab_matches_oracle(ctx):
    mesh, vox, pulses = _slab_case()
    scene = _scene(ctx, mesh, vox)
    say("voxel slab: pulses", pulses.n)
    out = to_np(ctx.simulate(scene, SLAB_SC, _dev(pulses.origins), _dev(pulses.directions)))
    torch.cuda.synchronize()
    compare_vox(mesh, vox, pulses, SLAB_SC, out, np.arange(pulses.n), "voxel slab", min_voxel_frac=0.3)
    # the pulses without a direction miss everything
    assert (out["subray_tri"][-2:, :19] == -1).all()


def test_voxel_densities_over_seven_decades(ctx):
    """The slab with densities from 1e-4 to 1e3 per metre: sigma L from far
    below 1 (the FP32 pre-test of the draw rejects nearly every cell) to far
    above 64 (beyond its range: the FP64 test alone), on the same pulses."""
    mesh, vox, pulses = _slab_case(seed=5)
    rng = np.random.default_rng(5)
    pad = (10.0 ** rng.uniform(-4.0, 3.0, vox["pad"].shape)).astype(np.float32)
    pad[vox["pad"] == 0.0] = 0.0
    vox = dict(vox, pad=pad)
    scene = _scene(ctx, mesh, vox)
    say("voxel slab, densities 1e-4..1e3: pulses", pulses.n)
    out = to_np(ctx.simulate(scene, SLAB_SC, _dev(pulses.origins), _dev(pulses.directions)))
    torch.cuda.synchronize()
    compare_vox(mesh, vox, pulses, SLAB_SC, out, np.arange(pulses.n), "voxel slab decades", min_voxel_frac=0.3)


def test_voxels_without_triangles(ctx):
    mesh, vox, pulses = _slab_case(seed=4)
    empty = synth.Mesh(np.zeros((0, 3), np.float32), np.zeros((0, 3), np.int32), np.zeros(0, np.float32))
    scene = _scene(ctx, empty, vox)
    say("voxels alone")
    out = to_np(ctx.simulate(scene, SLAB_SC, _dev(pulses.origins), _dev(pulses.directions)))
    torch.cuda.synchronize()
    compare_vox(empty, vox, pulses, SLAB_SC, out, np.arange(pulses.n), "voxels alone", min_voxel_frac=0.3)


def test_empty_grid_is_bitwise_the_mesh_alone(ctx):
    mesh, vox, pulses = _slab_case()
    zero = dict(vox, pad=np.zeros_like(vox["pad"]))
    o, d = _dev(pulses.origins), _dev(pulses.directions)
    say("empty grid vs no grid")
    a = to_np(ctx.simulate(_scene(ctx, mesh, None), SLAB_SC, o, d))
    b = to_np(ctx.simulate(_scene(ctx, mesh, zero), SLAB_SC, o, d))
    torch.cuda.synchronize()
    for k in a:
        assert np.array_equal(a[k], b[k], equal_nan=True), k


def test_voxel_draws_deterministic_and_seeded(ctx):
    mesh, vox, pulses = _slab_case()
    o, d = _dev(pulses.origins), _dev(pulses.directions)
    say("voxel determinism")
    a = to_np(ctx.simulate(_scene(ctx, mesh, vox), SLAB_SC, o, d))
    b = to_np(ctx.simulate(_scene(ctx, mesh, vox), SLAB_SC, o, d))
    c = to_np(ctx.simulate(_scene(ctx, mesh, dict(vox, seed=vox["seed"] + 1)), SLAB_SC, o, d))
    torch.cuda.synchronize()
    for k in a:
        assert np.array_equal(a[k], b[k], equal_nan=True), k
    assert not np.array_equal(a["subray_tri"], c["subray_tri"])


def test_voxels_split_batched_and_graph(ctx):
    mesh, vox, pulses = _slab_case()
    scene = _scene(ctx, mesh, vox)
    o, d = _dev(pulses.origins), _dev(pulses.directions)
    n = pulses.n
    say("voxels: split entry points")
    fused = to_np(ctx.simulate(scene, SLAB_SC, o, d))
    out = ctx.trace(scene, SLAB_SC, o, d)
    out.update(ctx.alloc_outputs(n, 19, SLAB_SC["n_bins"], SLAB_SC["max_returns"], o.device, subrays=False))
    ctx.waveform(SLAB_SC, o, d, out)
    ctx.returns(SLAB_SC, o, d, out)
    torch.cuda.synchronize()
    g = to_np(out)
    for k in fused:
        assert np.array_equal(fused[k], g[k], equal_nan=True), k
    # a persistent batch of three segments with two scanners: each segment
    # against the oracle on the whole batch
    scs = [SLAB_SC, configs.scanner(1e-3, 31, n_bins=256, bin_ns=0.5, max_returns=6)]
    off = np.array([0, 500, 900, n], np.int64)
    seg = np.array([0, 1, 0], np.int32)
    say("voxels: persistent batch")
    gb = to_np(ctx.simulate(scene, scs, o, d, segment_offsets=off, segment_scanner=seg))
    torch.cuda.synchronize()
    for s in range(3):
        sc = scs[seg[s]]
        S = oracle.pattern(sc)[0].size
        rows = np.arange(off[s], off[s + 1])
        sel = rows[:: 7]
        gs = {k: v[sel] for k, v in gb.items()}
        gs = dict(gs, subray_tri=gs["subray_tri"][:, :S], subray_range=gs["subray_range"][:, :S],
                  subray_cos=gs["subray_cos"][:, :S], subray_power=gs["subray_power"][:, :S])
        compare_vox(mesh, vox, pulses, sc, gs, sel, "batch segment %d" % s)
    # graph replays equal the eager call
    say("voxels: graph")
    out = ctx.alloc_outputs(n, 31, 256, 6, o.device)
    gr = ctx.capture_graph(scene, scs, o, d, out, segment_offsets=off, segment_scanner=seg)
    for rep in range(3):
        for v in out.values():
            v.fill_(-7)
        gr.launch()
        torch.cuda.synchronize()
        got = to_np(out)
        for k in gb:
            if k.startswith("subray_"):
                # a segment's rows hold its scanner's subrays; the tail is untouched
                for s in range(3):
                    S = oracle.pattern(scs[seg[s]])[0].size
                    a, b = gb[k][off[s]:off[s + 1], :S], got[k][off[s]:off[s + 1], :S]
                    assert np.array_equal(a, b, equal_nan=True), (rep, k, s)
            else:
                assert np.array_equal(gb[k], got[k], equal_nan=True), (rep, k)
    gr.close()


def test_voxel_gradient_matches_oracle(ctx):
    mesh = configs.diff_scene()
    rng = np.random.default_rng(8)
    lo = mesh.vertices.min(axis=0)
    hi = mesh.vertices.max(axis=0)
    # one layer of 12 x 12 voxels above the terrain, thin enough that about a
    # third of the subrays stop in it
    pad = rng.uniform(0.0, 0.05, (1, 12, 12)).astype(np.float32)
    size = float((hi[0] - lo[0]) / 12)
    vox = dict(origin=[float(lo[0]), float(lo[1]), float(hi[2]) + 2.0], size=size, pad=pad,
               lut=configs.TABLE2_ROWS, seed=21)
    z = float(hi[2]) + 60.0
    cx = 0.5 * float(lo[0] + hi[0])
    pulses = synth.als_lines(cx, np.linspace(float(lo[1]) + 5, float(hi[1]) - 5, 30), z, 40, beta_deg=(-20.0, 20.0))
    sc = configs.scanner(2e-3, 19, n_bins=256, bin_ns=0.5)
    scene = _scene(ctx, mesh, vox)
    o, d = _dev(pulses.origins), _dev(pulses.directions)
    say("voxel gradient: pulses", pulses.n)
    base = oracle.simulate(mesh, pulses, sc, voxels=vox)
    vf = (base.sub_tri >= mesh.n_triangles).mean()
    say("voxel gradient: voxel echoes per subray %.3f" % vf)
    assert 0.1 < vf < 0.7
    G = rng.normal(size=base.waveform.shape)
    gr_o, gz_o = oracle.gradient(mesh, pulses, sc, base.t0, G, voxels=vox)
    t0d = _dev(base.t0)
    out = ctx.simulate(scene, sc, o, d, t0=t0d)
    gr, gz = ctx.waveform_backward(scene, sc, o, d, t0d, out["subray_tri"], _dev(G.astype(np.float32)))
    torch.cuda.synchronize()
    assert np.array_equal(out["subray_tri"].cpu().numpy()[:, :19], base.sub_tri)
    gr = gr.cpu().numpy().astype(np.float64)
    gz = gz.cpu().numpy().astype(np.float64)
    er = np.linalg.norm(gr - gr_o) / np.linalg.norm(gr_o)
    ez = np.linalg.norm(gz - gz_o) / np.linalg.norm(gz_o)
    say("voxel gradient rel L2: reflectance %.2e heights %.2e" % (er, ez))
    assert er <= 1e-4 and ez <= 1e-4


def test_voxel_api_errors(ctx):
    import paper_2101_09154_amd as vp
    from paper_2101_09154_amd import vls
    mesh, vox, pulses = _slab_case()
    scene = _scene(ctx, mesh, vox)
    with pytest.raises(vp.VlsError):
        scene.set_voxels(vox["origin"], vox["size"], vox["pad"], vox["lut"])        # one grid per scene
    o, d = _dev(pulses.origins[:10]), _dev(pulses.directions[:10])
    with pytest.raises(vp.VlsError):
        ctx.simulate(scene, dict(SLAB_SC, divergence_rad=0.0, n_subrays=1), o, d)  # Eq. 7 needs beta > 0
    bad = [dict(pad=-vox["pad"]), dict(pad=np.full_like(vox["pad"], np.nan)),
           dict(lut=[[0.5, 0.4], [0.2, 0.6]]), dict(lut=[[0.0, -0.1]]), dict(size=0.0),
           dict(pad=np.zeros((0, 3, 3), np.float32))]
    for kw in bad:
        v = dict(vox, **kw)
        s2 = ctx.scene(mesh.vertices, mesh.triangles, mesh.reflectance)
        with pytest.raises(vp.VlsError):
            s2.set_voxels(v["origin"], v["size"], v["pad"], v["lut"])
    # a grid too large for int32 ids is refused before its densities are read
    small = np.zeros(8, np.float32)
    lut = np.asarray(configs.TABLE2_ROWS, np.float64)
    desc = vls.VoxelDesc((ctypes.c_double * 3)(0.0, 0.0, 0.0), 1.0, 1300, 1300, 1300, lut.shape[0],
                         small.ctypes.data, lut.ctypes.data, 0)
    s3 = ctx.scene(mesh.vertices, mesh.triangles, mesh.reflectance)
    assert vls.lib().vls_scene_set_voxels(s3._h, ctypes.byref(desc), None) != 0


def test_voxel_forest_sampled(ctx):
    mesh, vox, pulses, sc = configs.uls_voxels()
    say("uls_voxels: triangles", mesh.n_triangles, "voxels", vox["pad"].size, "pulses", pulses.n)
    scene = _scene(ctx, mesh, vox)
    o, d = _dev(pulses.origins), _dev(pulses.directions)
    out = ctx.simulate(scene, sc, o, d)
    torch.cuda.synchronize()
    tri = out["subray_tri"]
    nt = mesh.n_triangles
    vfrac = float((tri >= nt).float().mean())
    say("uls_voxels: voxel echoes per subray %.3f" % vfrac)
    assert 0.05 < vfrac < 0.95
    assert int(tri.max()) < nt + vox["pad"].size
    pw = out["subray_power"][tri >= nt]
    assert bool(torch.isfinite(pw).all()) and float(pw.min()) > 0.0
    assert bool((out["subray_cos"][tri >= nt] == 1.0).all())
    # pulses whose beam axis lands inside the stand, against the oracle
    rng = np.random.default_rng(6)
    x_land = pulses.origins[:, 0] - pulses.directions[:, 0] / pulses.directions[:, 2] * 60.0
    inside = np.nonzero((x_land > 10) & (x_land < 190))[0]
    sel = np.sort(rng.choice(inside, 10, replace=False))
    idx = torch.from_numpy(sel).cuda()
    g = {k: v.index_select(0, idx).cpu().numpy() for k, v in out.items()}
    compare_vox(mesh, vox, pulses, sc, g, sel, "uls_voxels", min_voxel_frac=0.02)
