"""One context used from two streams at once, graphs of one batch layout
replayed on two streams, and the adjoint in its fixed summation order.

Each stream gets its own workspaces (candidate lists, counters), so
simultaneous calls on two streams give bitwise the results of the same calls
made one after the other; each captured graph owns its workspace and work
counter.  The deterministic adjoint gives bitwise equal gradients on repeated
runs and meets the same bound against the FP64 oracle's gradient as the
atomic form (Sec. 5.2, Eq. 7; Sec. 3.4, Eq. 3 through the chain rule).
"""
import sys

import numpy as np
import pytest

import oracle
import synth
from synth import configs

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


def _equal(a, b, what):
    for k in a:
        assert torch.equal(a[k].nan_to_num(-7.0), b[k].nan_to_num(-7.0)), (what, k)


def test_two_streams_one_context(ctx):
    mesh, pulses, sc = configs.als_buildings()
    scene = ctx.scene(mesh.vertices, mesh.triangles, mesh.reflectance)
    # two different pulse sets, the second larger (its workspace grows on its own stream)
    ia = np.arange(100000, 250000)
    ib = np.arange(600000, 900000)
    oa, da = _dev(pulses.origins[ia]), _dev(pulses.directions[ia])
    ob, db = _dev(pulses.origins[ib]), _dev(pulses.directions[ib])
    say("two streams: reference calls on the current stream")
    ref_a = ctx.simulate(scene, sc, oa, da, subrays=False)
    ref_b = ctx.simulate(scene, sc, ob, db, subrays=False)
    torch.cuda.synchronize()
    import paper_2101_09154_amd as vp
    S = vp.n_subrays(sc)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    outs = []
    for rep in range(2):
        out_a = ctx.alloc_outputs(ia.size, S, sc["n_bins"], sc["max_returns"], oa.device, subrays=False)
        out_b = ctx.alloc_outputs(ib.size, S, sc["n_bins"], sc["max_returns"], ob.device, subrays=False)
        torch.cuda.synchronize()
        for i in range(3):   # interleaved launches on both streams, nothing in between
            ctx.simulate(scene, sc, oa, da, out=out_a, stream=s1)
            ctx.simulate(scene, sc, ob, db, out=out_b, stream=s2)
        torch.cuda.synchronize()
        outs.append((out_a, out_b))
    say("two streams: compare")
    for out_a, out_b in outs:
        _equal(ref_a, out_a, "stream 1")
        _equal(ref_b, out_b, "stream 2")


def _batch_layout():
    mesh, _, _ = configs.small_tls()
    scs = [configs.scanner(0.3e-3, 19, n_bins=256), configs.scanner(0.5e-3, 31, n_bins=256),
           configs.scanner(0.25e-3, 61, n_bins=256)]
    seg_sc = (np.arange(6) % 3).astype(np.int32)
    # two pulse sets with the same segment layout, from different positions
    sets = []
    for shift in (0.0, 6.0):
        parts = [synth.tls_grid((8.0 + 9 * i + shift, 12.0 + 7 * i, 3.0), 40 + 13 * i, 7 + i, el_deg=(-35.0, 15.0))
                 for i in range(6)]
        sets.append(synth.concat_pulses(parts, seg_sc))
    return mesh, scs, sets, seg_sc


def test_two_graphs_one_layout_two_streams(ctx):
    mesh, scs, sets, seg_sc = _batch_layout()
    scene = ctx.scene(mesh.vertices, mesh.triangles, mesh.reflectance)
    eager, graphs, outs = [], [], []
    for b in sets:
        o, d = _dev(b.origins), _dev(b.directions)
        kw = dict(segment_offsets=b.segment_offsets, segment_scanner=b.segment_scanner)
        eager.append(ctx.simulate(scene, scs, o, d, subrays=False, **kw))
        torch.cuda.synchronize()
        out = {k: torch.empty_like(v) for k, v in eager[-1].items()}
        graphs.append(ctx.capture_graph(scene, scs, o, d, out, **kw))
        outs.append(out)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    say("two graphs of one layout on two streams")
    for rep in range(3):
        for out in outs:
            for v in out.values():
                v.fill_(-5)
        torch.cuda.synchronize()
        graphs[0].launch(stream=s1)
        graphs[1].launch(stream=s2)
        torch.cuda.synchronize()
        _equal(eager[0], outs[0], "graph 1, replay %d" % rep)
        _equal(eager[1], outs[1], "graph 2, replay %d" % rep)
    for g in graphs:
        g.close()


def _grad_case(n=48, lines=40, per_line=50):
    mesh = configs.diff_scene(n=n)
    target = configs.diff_target(mesh)
    extent = mesh.info["extent"]
    z = mesh.info["heights_mean"] + 120.0
    y = 4.0 + (extent - 8.0) * np.arange(lines) / (lines - 1)
    pulses = synth.als_lines(extent / 2, y, z, per_line, beta_deg=(-12.0, 12.0))
    sc = configs.scanner(0.5e-3, 31, pulse_width_ns=4.0, bin_ns=0.5, n_bins=512)
    return mesh, target, pulses, sc


def test_deterministic_adjoint(ctx):
    import paper_2101_09154_amd as vp
    mesh, target, pulses, sc = _grad_case()
    base = oracle.simulate(mesh, pulses, sc)
    t0 = base.t0
    tgt = oracle.simulate(target, pulses, sc, t0=t0).waveform
    G = 2.0 * (base.waveform - tgt)
    gr_o, gz_o = oracle.gradient(mesh, pulses, sc, t0, G)
    c2 = vp.Context(0)
    scene = c2.scene(mesh.vertices, mesh.triangles, mesh.reflectance)
    o, d, t0d = _dev(pulses.origins), _dev(pulses.directions), _dev(t0)
    out = c2.simulate(scene, sc, o, d, t0=t0d)
    Gd = _dev(G.astype(np.float32))
    say("adjoint: atomic, then fixed order twice")
    ga = c2.waveform_backward(scene, sc, o, d, t0d, out["subray_tri"], Gd)
    c2.set_deterministic(True)
    g1 = c2.waveform_backward(scene, sc, o, d, t0d, out["subray_tri"], Gd)
    torch.cuda.synchronize()
    g1 = [x.clone() for x in g1]
    g2 = c2.waveform_backward(scene, sc, o, d, t0d, out["subray_tri"], Gd)
    torch.cuda.synchronize()
    c2.set_deterministic(False)
    assert torch.equal(g1[0], g2[0]) and torch.equal(g1[1], g2[1])
    gr, gz = (x.cpu().numpy().astype(np.float64) for x in g1)
    er = np.linalg.norm(gr - gr_o) / np.linalg.norm(gr_o)
    ez = np.linalg.norm(gz - gz_o) / np.linalg.norm(gz_o)
    say("fixed order vs oracle: reflectance %.2e heights %.2e" % (er, ez))
    assert er <= 1e-4 and ez <= 1e-4
    assert np.all(gr[gr_o == 0] == 0) and np.all(gz[gz_o == 0] == 0)
    # the two summation orders agree to float rounding
    ra, za = (x.cpu().numpy().astype(np.float64) for x in ga)
    assert np.linalg.norm(ra - gr) <= 1e-5 * np.linalg.norm(gr)
    assert np.linalg.norm(za - gz) <= 1e-5 * np.linalg.norm(gz)
