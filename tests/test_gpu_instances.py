"""GPU parity of scenes built from parts placed by affine maps (Sec. 3.5,
Sec. 5.1) through the C ABI: the library's placed scene against the oracle's
(`oracle.instance_mesh`), at the tolerances of parity_util."""
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


def _parts(ms):
    return [(m.vertices, m.triangles, m.reflectance) for m in ms]


def compare(mesh, pulses, sc, g, sel, label):
    r = oracle.simulate(mesh, pulses, sc, select=sel)
    rep = {}
    ok_h = check_hits(mesh, pulses, sc, sel, g, r, rep)
    ok_w = check_waveforms(g, r, rep)
    ok_r, tri_bad = check_returns(g, r, sc, rep)
    left = attribution_excused(mesh, pulses, sc, sel, g, r, tri_bad)
    rep["attribution_unexcused"] = left[:10]
    say(label, rep)
    assert ok_h and ok_w and ok_r and not left, rep
    return r


def _small_case(seed=5):
    """The small terrain (unmoved) with 40 copies of three small tree models,
    turned, scaled (one copy mirrored) and moved onto it; terrestrial pulses."""
    rng = np.random.default_rng(seed)
    terrain, pulses, sc = configs.small_tls(n_az=80, n_el=30)
    models = configs.tree_models(seed=77, n_models=3, leaves=60)
    inst = [(0, np.hstack([np.eye(3), np.zeros((3, 1))]))]
    for i in range(40):
        th = rng.uniform(0, 2 * np.pi)
        s = rng.uniform(0.3, 0.6)
        A = s * np.array([[np.cos(th), -np.sin(th), 0.0], [np.sin(th), np.cos(th), 0.0], [0.0, 0.0, 1.0]])
        if i == 7:
            A[0] = -A[0]                    # a mirrored copy
        t = np.array([rng.uniform(4, 60), rng.uniform(4, 60), rng.uniform(-4.0, 2.0)])
        inst.append((1 + i % 3, np.hstack([A, t[:, None]])))
    return [terrain] + models, inst, pulses, sc


def test_instanced_scene_matches_oracle(ctx):
    parts, inst, pulses, sc = _small_case()
    mesh = oracle.instance_mesh(parts, inst)
    say("instanced: parts", [p.n_triangles for p in parts], "instances", len(inst), "triangles", mesh.n_triangles)
    scene = ctx.scene_instanced(_parts(parts), inst)
    assert scene.n_triangles == mesh.n_triangles and scene.n_vertices == mesh.n_vertices
    o, d = _dev(pulses.origins), _dev(pulses.directions)
    g = to_np(ctx.simulate(scene, sc, o, d))
    torch.cuda.synchronize()
    r = compare(mesh, pulses, sc, g, np.arange(pulses.n), "instanced small")
    tree_hits = (r.sub_tri >= parts[0].n_triangles).mean()
    say("instanced: subrays on placed trees %.3f" % tree_hits)
    assert tree_hits > 0.01
    # the same scene uploaded whole from the host: bitwise the same outputs,
    # so the device placement gave the oracle's FP32 vertices
    flat = to_np(ctx.simulate(ctx.scene(mesh.vertices, mesh.triangles, mesh.reflectance), sc, o, d))
    torch.cuda.synchronize()
    for k in g:
        assert np.array_equal(g[k], flat[k], equal_nan=True), k


def test_instanced_parts_on_device_and_edge_cases(ctx):
    parts, inst, pulses, sc = _small_case(seed=6)
    host = ctx.scene_instanced(_parts(parts), inst)
    dev_parts = [(torch.from_numpy(m.vertices).cuda(), torch.from_numpy(m.triangles).cuda(),
                  torch.from_numpy(m.reflectance).cuda()) for m in parts]
    dev = ctx.scene_instanced(dev_parts, inst)
    o, d = _dev(pulses.origins), _dev(pulses.directions)
    a = to_np(ctx.simulate(host, sc, o, d))
    b = to_np(ctx.simulate(dev, sc, o, d))
    torch.cuda.synchronize()
    for k in a:
        assert np.array_equal(a[k], b[k], equal_nan=True), k
    # no instances: an empty scene; an unused part is fine
    empty = ctx.scene_instanced(_parts(parts), [])
    assert empty.n_triangles == 0
    out = to_np(ctx.simulate(empty, sc, o[:10], d[:10]))
    assert (out["subray_tri"] == -1).all()
    one = ctx.scene_instanced(_parts(parts), [(2, inst[1][1])])
    assert one.n_triangles == parts[2].n_triangles


def test_instanced_errors(ctx):
    import paper_2101_09154_amd as vp
    parts, inst, _, _ = _small_case()
    with pytest.raises(vp.VlsError):
        ctx.scene_instanced(_parts(parts), [(len(parts), inst[1][1])])        # part out of range
    bad_aff = inst[1][1].copy()
    bad_aff[1, 2] = np.nan
    with pytest.raises(vp.VlsError):
        ctx.scene_instanced(_parts(parts), [(1, bad_aff)])                    # non-finite map
    m = parts[1]
    broken = (m.vertices, np.where(m.triangles == 0, m.vertices.shape[0], m.triangles).astype(np.int32),
              m.reflectance)
    # an index past the part's own vertices, though inside the placed scene's
    with pytest.raises(vp.VlsError):
        ctx.scene_instanced([(parts[0].vertices, parts[0].triangles, parts[0].reflectance), broken],
                            [(1, inst[1][1]), (0, inst[0][1])])
    huge = inst[1][1].copy()
    huge[:, :3] *= 1e300
    with pytest.raises(vp.VlsError):
        ctx.scene_instanced(_parts(parts), [(1, huge)])                       # placed vertices overflow


def test_instanced_forest_sampled(ctx):
    parts, inst, pulses, sc = configs.uls_instanced()
    mesh = oracle.instance_mesh(parts, inst)
    say("uls_instanced: instances", len(inst), "triangles", mesh.n_triangles)
    scene = ctx.scene_instanced(_parts(parts), inst)
    assert scene.n_triangles == mesh.n_triangles
    o, d = _dev(pulses.origins), _dev(pulses.directions)
    out = ctx.simulate(scene, sc, o, d)
    torch.cuda.synchronize()
    rng = np.random.default_rng(7)
    x_land = pulses.origins[:, 0] - pulses.directions[:, 0] / pulses.directions[:, 2] * 60.0
    inside = np.nonzero((x_land > 10) & (x_land < 190))[0]
    sel = np.sort(rng.choice(inside, 8, replace=False))
    idx = torch.from_numpy(sel).cuda()
    g = {k: v.index_select(0, idx).cpu().numpy() for k, v in out.items()}
    compare(mesh, pulses, sc, g, sel, "uls_instanced")
    tri = out["subray_tri"]
    say("uls_instanced: subrays on trees %.3f" % float((tri >= parts[0].n_triangles).float().mean()))


# ------------------------------------------------------------------ two levels


def test_two_level_bitwise_equals_expanded(ctx):
    # the two-level scene tests the same placed triangles with the same
    # arithmetic: every output equals the expanded scene's bit for bit
    for seed in (5, 6):
        parts, inst, pulses, sc = _small_case(seed=seed)
        flat = ctx.scene_instanced(_parts(parts), inst)
        two = ctx.scene_instanced(_parts(parts), inst, two_level=True)
        st = two.stats()
        say("two-level stats", st)
        assert two.n_triangles == flat.n_triangles
        assert st["device_bytes"] < flat.stats()["device_bytes"]
        o, d = _dev(pulses.origins), _dev(pulses.directions)
        a = to_np(ctx.simulate(flat, sc, o, d))
        b = to_np(ctx.simulate(two, sc, o, d))
        tr = to_np(ctx.trace(two, sc, o, d))
        torch.cuda.synchronize()
        for k in a:
            assert np.array_equal(a[k], b[k], equal_nan=True), (seed, k)
        for k in tr:
            assert np.array_equal(a[k], tr[k], equal_nan=True), (seed, k)
        assert (a["subray_tri"] >= parts[0].n_triangles).mean() > 0.01
        # a ranging error (Sec. 3.7) is drawn alike on both forms
        scn = dict(sc, range_noise_m=0.03, noise_seed=seed)
        an = to_np(ctx.simulate(flat, scn, o, d))
        bn = to_np(ctx.simulate(two, scn, o, d))
        torch.cuda.synchronize()
        for k in an:
            assert np.array_equal(an[k], bn[k], equal_nan=True), (seed, "noise", k)
        assert not np.array_equal(an["ret_range"], a["ret_range"], equal_nan=True)


def test_two_level_batches_and_limits(ctx):
    import paper_2101_09154_amd as vp
    parts, inst, pulses, sc = _small_case(seed=8)
    two = ctx.scene_instanced(_parts(parts), inst, two_level=True)
    flat = ctx.scene_instanced(_parts(parts), inst)
    o, d = _dev(pulses.origins), _dev(pulses.directions)
    # a batch of two scanners, fixed window origins, and outputs without subrays
    scs = [sc, configs.scanner(1e-3, 7, n_bins=256)]
    off = np.array([0, 900, pulses.n], np.int64)
    seg = np.array([1, 0], np.int32)
    a = to_np(ctx.simulate(flat, scs, o, d, segment_offsets=off, segment_scanner=seg))
    b = to_np(ctx.simulate(two, scs, o, d, segment_offsets=off, segment_scanner=seg))
    t0 = _dev(a["window_t0_ns"])
    c = to_np(ctx.simulate(two, sc, o, d, t0=t0, subrays=False))
    e = to_np(ctx.simulate(flat, sc, o, d, t0=t0, subrays=False))
    torch.cuda.synchronize()
    for k in a:
        if k.startswith("subray_"):
            for q in range(2):
                S = oracle.pattern(scs[seg[q]])[0].size
                assert np.array_equal(a[k][off[q]:off[q + 1], :S], b[k][off[q]:off[q + 1], :S], equal_nan=True), k
        else:
            assert np.array_equal(a[k], b[k], equal_nan=True), k
    for k in c:
        assert np.array_equal(c[k], e[k], equal_nan=True), k
    # no instances, and calls without a two-level form
    empty = ctx.scene_instanced(_parts(parts), [], two_level=True)
    assert (to_np(ctx.simulate(empty, sc, o[:5], d[:5]))["subray_tri"] == -1).all()
    with pytest.raises(vp.VlsError):
        two.update_reflectance(torch.zeros(two.n_triangles, device="cuda"))
    with pytest.raises(vp.VlsError):
        ctx.capture_graph(two, sc, o, d, ctx.alloc_outputs(pulses.n, 19, 256, 8, o.device))
    sing = inst[1][1].copy()
    sing[2, :3] = 0.0
    with pytest.raises(vp.VlsError):
        ctx.scene_instanced(_parts(parts), [(1, sing)], two_level=True)      # a map that is not invertible


def test_two_level_forest_sampled(ctx):
    parts, inst, pulses, sc = configs.uls_instanced()
    two = ctx.scene_instanced(_parts(parts), inst, two_level=True)
    flat = ctx.scene_instanced(_parts(parts), inst)
    say("uls_instanced two-level stats", two.stats(), "expanded bytes", flat.stats()["device_bytes"])
    o, d = _dev(pulses.origins), _dev(pulses.directions)
    rng = np.random.default_rng(11)
    sel = np.sort(rng.choice(pulses.n, 20000, replace=False))
    idx = torch.from_numpy(sel).cuda()
    os_, ds_ = o.index_select(0, idx).contiguous(), d.index_select(0, idx).contiguous()
    a = to_np(ctx.simulate(flat, sc, os_, ds_))
    b = to_np(ctx.simulate(two, sc, os_, ds_))
    torch.cuda.synchronize()
    for k in a:
        assert np.array_equal(a[k], b[k], equal_nan=True), k
