"""vls_simulate_noalloc through the C ABI against vls_simulate: the same
outputs, bit for bit, on two calls in a row with the second smaller, on the
small terrestrial workload and on the ALS workload at the largest batch the
entry point takes; its limits are checked on the host before anything runs."""
import sys

import numpy as np
import pytest

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


def _same(a, b, what):
    for k in a:
        x, y = a[k].cpu(), b[k].cpu()
        if x.dtype.is_floating_point:
            assert torch.equal(x.nan_to_num(-7.0), y.nan_to_num(-7.0)), (what, k)
        else:
            assert torch.equal(x, y), (what, k)


def _run_pair(ctx, scene, sc, pulses, sel, what):
    import paper_2101_09154_amd as vp
    o = _dev(pulses.origins[sel])
    d = _dev(pulses.directions[sel])
    n = len(sel)
    S = vp.n_subrays(sc)
    ref = ctx.simulate(scene, sc, o, d)
    out = ctx.alloc_outputs(n, S, sc["n_bins"], sc["max_returns"], o.device)
    for v in out.values():
        v.fill_(-3)   # every output element must be written by the call
    ctx.simulate_noalloc(scene, sc, o, d, out)
    torch.cuda.synchronize()
    _same(ref, out, what)
    return int((out["n_returns"] > 0).sum().item())


def test_noalloc_matches_simulate_small_tls(ctx):
    mesh, pulses, sc = configs.small_tls()
    scene = ctx.scene(mesh.vertices, mesh.triangles, mesh.reflectance)
    say("noalloc small_tls: 10000 pulses, then 1201")
    h1 = _run_pair(ctx, scene, sc, pulses, np.arange(pulses.n), "small_tls all")
    h2 = _run_pair(ctx, scene, sc, pulses, np.arange(3, pulses.n, 8)[:1201], "small_tls second, smaller")
    assert h1 > 5000 and h2 > 600


def test_noalloc_matches_simulate_als_at_the_limit(ctx):
    import paper_2101_09154_amd as vp
    mesh, pulses, sc = configs.als_buildings()
    scene = ctx.scene(mesh.vertices, mesh.triangles, mesh.reflectance)
    lim = vp.NOALLOC_MAX_PULSES
    say("noalloc als_buildings: %d pulses, then 5000" % lim)
    h1 = _run_pair(ctx, scene, sc, pulses, np.arange(400000, 400000 + lim), "als at the limit")
    # a second, smaller call: the device memory in use does not change
    o = _dev(pulses.origins[600000:605000])
    d = _dev(pulses.directions[600000:605000])
    out = ctx.alloc_outputs(5000, vp.n_subrays(sc), sc["n_bins"], sc["max_returns"], o.device)
    ref = ctx.simulate(scene, sc, o, d)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    ctx.simulate_noalloc(scene, sc, o, d, out)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0
    _same(ref, out, "als second, smaller")
    assert h1 > 0.8 * lim


def test_noalloc_limits(ctx):
    import paper_2101_09154_amd as vp
    mesh, pulses, sc = configs.small_tls()
    scene = ctx.scene(mesh.vertices, mesh.triangles, mesh.reflectance)
    lim = vp.NOALLOC_MAX_PULSES
    # one pulse over the limit: rejected on the host before anything is enqueued
    o = torch.zeros((lim + 1, 3), dtype=torch.float64, device="cuda")
    d = torch.zeros((lim + 1, 3), dtype=torch.float32, device="cuda")
    d[:, 2] = -1.0
    out = ctx.alloc_outputs(lim + 1, vp.n_subrays(sc), sc["n_bins"], sc["max_returns"], o.device)
    with pytest.raises(vp.VlsError, match="invalid argument"):
        ctx.simulate_noalloc(scene, sc, o, d, out)
    # zero pulses: nothing to do
    e = {k: v[:0] for k, v in out.items()}
    ctx.simulate_noalloc(scene, sc, o[:0], d[:0], e)
    torch.cuda.synchronize()
