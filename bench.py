"""Benchmark of the fused laser-scanning hot path on one GPU.

Workload (default): the ALS scene with buildings -- a 1024x1024 fBm terrain at
0.5 m plus 20,000 box buildings (2,333,058 triangles), 1,000,000 line-scanner
pulses from 500 m above ground, 31 subrays per pulse, 512 bins of 0.5 ns, up
to 8 returns.  One step: subrays, traversal, power, waveform write and
returns for every pulse, inputs resident in HBM.

Prints one JSON line.  A step is three launches: the cone pass (one traversal
per pulse collecting candidate triangles), the packet walk of the pulses whose
candidate list overflowed (one wavefront per pulse; few on this workload) and
the fused kernel (subray tests, power, waveform, returns).  The roofline is
reported for the fused kernel, the dominant one, with its algorithmic bytes:
per pulse 36 B in, the candidate count (4 B), 52 B per candidate (its id and
its 48 B leaf record) and 4*n_bins + 8 + 4 + 16*K B out, plus 4 B of
reflectance per subray; the cone pass is reported beside it with 112 B per
four-wide record visited.  Record visits and triangle tests are counted by the
library (vls_trace_counts).
"""
import argparse
import hashlib
import re
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# launch configurations the autotuner chose on MI355X for these workloads (JSON
# lines keyed by scene size, subrays, bins, pulse count and segments); a key not
# in the file is tuned on the spot (and appended when the file is writable)
TUNE_CACHE = os.path.join(ROOT, "paper_2101_09154_amd", "tuning", "mi355x.jsonl")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_hash():
    """Hash of the device code (the .hip sources and the headers they include),
    comments left out and white space collapsed: an edit of a comment does not
    change the code the profiles were taken on."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2101_09154_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".h")):
            with open(os.path.join(csrc, f), "r") as fh:
                text = fh.read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            text = re.sub(r"//[^\n]*", "", text)
            h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def traffic_record(workload, kernel_hash):
    """The traffic-json record of the committed PMC summary of a workload, if it
    was taken on this device code (else None)."""
    path = os.path.join(ROOT, "profiles", "simulate_%s_pmc.md" % workload)
    if not os.path.exists(path):
        return None
    rec = None
    for line in open(path):
        if line.startswith("traffic-json:"):
            rec = json.loads(line.split(":", 1)[1])
    if not rec or rec.get("source_hash") != kernel_hash:
        return None
    return rec


def measured_traffic(kernel_hash):
    """HBM bytes per launch of the fused kernel on the ALS workload, from its PMC summary."""
    rec = traffic_record("als_buildings", kernel_hash)
    return rec.get("bytes_per_launch") if rec else None


def input_digest(mesh, pulses, sc, seed):
    """SHA-256 of the arrays a step reads (scene, pulses, segments) and of the
    scanner descriptions, with the generator seed they came from."""
    h = hashlib.sha256()
    arrays = [mesh.vertices, mesh.triangles, mesh.reflectance, pulses.origins, pulses.directions]
    if getattr(pulses, "segment_offsets", None) is not None:
        arrays += [pulses.segment_offsets, pulses.segment_scanner]
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    h.update(json.dumps(sc, sort_keys=True).encode())
    return {"sha256": h.hexdigest(), "seed": seed}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def copy_bandwidth(mib=1024, reps=5):
    """A plain device-to-device copy of `mib` MiB, timed with events: bytes read
    plus bytes written per second (the measured counterpart of the 8 TB/s peak)."""
    import torch
    n = (mib << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    ms = time_ms(lambda: dst.copy_(src), reps, 2, torch.cuda.current_stream())
    del src, dst
    return {"bytes_per_copy": 2 * 4 * n, "ms": ms, "GBps": 2 * 4 * n / (ms * 1e-3) / 1e9,
            "what": "torch copy_ of %d MiB on the device, read + write, mean of %d" % (mib, reps)}


def candidate_census(ctx, scene, sc, o, d, chunk=131072):
    """Per-pulse candidate lists of the cone pass, in chunks: (candidates summed
    over the pulses with a list, pulses whose list overflowed)."""
    import torch
    total = 0
    over = 0
    rows = None
    for a in range(0, o.shape[0], chunk):
        b = min(a + chunk, o.shape[0])
        if rows is None or rows.shape[0] != b - a:
            rows = torch.empty((b - a, 256), dtype=torch.int32, device=o.device)
        ctx.cone_candidates(scene, sc, o[a:b], d[a:b], out=rows)
        c = rows[:, 0]
        total += int(c.clamp(min=0).sum().item())
        over += int((c < 0).sum().item())
    return total, over


def bench_plain(ctx, name, label, mesh, pulses, sc, steps, seed, hbm=True):
    """One scanner's step on a whole workload: step time and rates, the kernels'
    times, the fused kernel's algorithmic bytes (candidate records once per
    pulse), and, when a PMC summary of this workload was taken on this device
    code, each kernel's measured HBM traffic and rate."""
    import torch
    import paper_2101_09154_amd as vp
    dev = torch.device("cuda", 0)
    scene = ctx.scene(mesh.vertices, mesh.triangles, mesh.reflectance)
    o = torch.from_numpy(pulses.origins).to(dev)
    d = torch.from_numpy(pulses.directions).to(dev)
    n = pulses.n
    S = vp.n_subrays(sc)
    K = sc["max_returns"]
    nb = sc["n_bins"]
    out = ctx.alloc_outputs(n, S, nb, K, dev, subrays=False)
    stream = torch.cuda.current_stream()
    cand, n_over = candidate_census(ctx, scene, sc, o, d)
    visits = None
    if hbm:
        # the cone pass's four-wide records visited (a counting pass, untimed)
        _, visits, _ = ctx.trace_counts(scene, sc, o, d)
    ms = time_ms(lambda: ctx.simulate(scene, sc, o, d, out=out), steps, 2, stream)
    ctx.profile(True)
    for _ in range(steps):
        ctx.simulate(scene, sc, o, d, out=out)
    prof = ctx.profile_read()
    ctx.profile(False)
    fused_ms = prof["fused_ms"] / max(prof["fused_launches"], 1)
    cone_ms = prof["cone_ms"] / max(prof["cone_launches"], 1)
    packet_ms = prof["packet_ms"] / max(prof["packet_launches"], 1)
    per_pulse_io = 36.0 + 4.0 * nb + 8.0 + 4.0 + 16.0 * K
    # fused kernel: pulse in, count, each listed candidate's id and 48 B record
    # once per pulse; a pulse that overflowed reads one leaf per subray (the
    # packet walk's result); a reflectance per subray; outputs out
    fused_bytes = n * (per_pulse_io + 4.0) + 52.0 * cand + 52.0 * S * n_over + 4.0 * n * S
    scene_bytes = 112.0 * max(mesh.n_triangles - 1, 1) + 52.0 * mesh.n_triangles
    res = {"workload": label, "pulses": n, "subrays_per_pulse": S, "n_bins": nb, "max_returns": K,
           "triangles": mesh.n_triangles, "inputs": input_digest(mesh, pulses, sc, seed),
           "ms": ms, "subrays_per_s": n * S / (ms * 1e-3), "pulses_per_s": n / (ms * 1e-3),
           "candidates_per_listed_pulse": cand / max(n - n_over, 1), "overflowed_pulses": n_over,
           "kernels": {"cone_ms": cone_ms, "packet_ms": packet_ms, "fused_ms": fused_ms},
           "fused": {"algorithmic_bytes_per_launch": fused_bytes,
                     "achieved_GBps": fused_bytes / (fused_ms * 1e-3) / 1e9},
           "scene_bytes": scene_bytes,
           "timing": "HIP events: step = mean of %d simulate calls; kernels recorded by the library around "
                     "each launch on its stream" % steps}
    if hbm:
        res["fused"]["frac"] = res["fused"]["achieved_GBps"] / HBM_PEAK_GBS
        # cone pass: 112 B per four-wide record visited, pulse in (36 B), count
        # and basis out (4 + 40 B), 52 B per listed candidate (id out, triangle
        # read by the cover test)
        cone_bytes = 112.0 * visits + n * (36.0 + 4.0 + 40.0) + 52.0 * cand
        res["cone"] = {"node_visits_per_pulse": visits / n, "algorithmic_bytes_per_launch": cone_bytes,
                       "achieved_GBps": cone_bytes / (cone_ms * 1e-3) / 1e9,
                       "level": "records re-read by neighbouring pulses are served by L2 and the last-level "
                                "cache: the counters' traffic (below) is what reaches HBM"}
        rec = traffic_record(name, source_hash())
        if rec:
            for kern, t in (("fused", fused_ms), ("cone", cone_ms), ("packet", packet_ms)):
                b = rec.get(kern + "_bytes_per_launch")
                if b:
                    res.setdefault("traffic", {})[kern] = {
                        "bytes_per_launch": b, "GBps": b / (t * 1e-3) / 1e9,
                        "frac": b / (t * 1e-3) / 1e9 / HBM_PEAK_GBS}
    else:
        res["fused"]["level"] = "L2: the scene and the candidate records stay in the caches"
    scene.close()
    return res


def cpu_baseline(mesh, pulses, sc, target_s):
    import oracle
    threads = oracle.max_threads()
    rng = np.random.default_rng(123)
    probe = np.sort(rng.choice(pulses.n, 2 * threads, replace=False))
    t = time.perf_counter()
    oracle.simulate(mesh, pulses, sc, select=probe)
    per = (time.perf_counter() - t) / probe.size
    n = int(np.clip(target_s / max(per, 1e-6), 8, 20000))
    sel = np.sort(rng.choice(pulses.n, n, replace=False))
    t = time.perf_counter()
    r = oracle.simulate(mesh, pulses, sc, select=sel)
    dt = time.perf_counter() - t
    return {"value": n * r.S / dt, "unit": "subrays/s", "cores": threads, "kind": "oracle",
            "pulses_per_s": n / dt,
            "sample": "%d seeded random pulses of the same workload (%d subrays), FP64 brute force over all "
                      "%d triangles, %.1f s" % (n, n * r.S, mesh.n_triangles, dt)}


def time_ms(fn, steps, warmup, stream):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def bench_batched(ctx, scene, mesh, steps, tune_cache=None):
    """256 terrestrial positions on the same scene: per-segment launches vs one
    persistent launch vs one launch per scanner over its segments (grouped) vs a
    replayed HIP graph of the autotuned choice."""
    import torch
    from synth import configs
    import paper_2101_09154_amd as vp
    _, pulses, scs = configs.batched_tls(mesh=mesh)
    off = pulses.segment_offsets
    seg = pulses.segment_scanner
    S = [vp.n_subrays(sc) for sc in scs]
    n = pulses.n
    subrays = int(sum((off[i + 1] - off[i]) * S[seg[i]] for i in range(seg.size)))
    dev = torch.device("cuda", 0)
    o = torch.from_numpy(pulses.origins).to(dev)
    d = torch.from_numpy(pulses.directions).to(dev)
    out = ctx.alloc_outputs(n, max(S), scs[0]["n_bins"], scs[0]["max_returns"], dev, subrays=False)
    stream = torch.cuda.current_stream()
    views = []
    for i in range(seg.size):
        a, b = int(off[i]), int(off[i + 1])
        views.append((scs[seg[i]], o[a:b], d[a:b], {k: v[a:b] for k, v in out.items()}))

    def per_segment():
        for sc, oo, dd, oo_out in views:
            ctx.simulate(scene, sc, oo, dd, out=oo_out)

    kw = dict(segment_offsets=off, segment_scanner=seg)
    cfg0 = ctx.launch_config()
    t_seg = time_ms(per_segment, max(1, steps // 4), 1, stream)
    ctx.set_launch_config(**dict(cfg0, grouped=0))
    t_pers = time_ms(lambda: ctx.simulate(scene, scs, o, d, out=out, **kw), steps, 1, stream)
    ctx.set_launch_config(**dict(cfg0, grouped=1))
    t_grp = time_ms(lambda: ctx.simulate(scene, scs, o, d, out=out, **kw), steps, 1, stream)
    ctx.set_launch_config(**cfg0)
    tune = ctx.autotune(scene, scs, o, d, out, cache_path=tune_cache, **kw)
    t_tuned = time_ms(lambda: ctx.simulate(scene, scs, o, d, out=out, **kw), steps, 1, stream)
    g = ctx.capture_graph(scene, scs, o, d, out, **kw)
    t_graph = time_ms(lambda: g.launch(), steps, 1, stream)
    cfg_tuned = ctx.launch_config()
    g.close()
    ctx.set_launch_config(**cfg0)
    return {"workload": "batched_tls: %d positions on the als_buildings scene, %d pulses, %d subrays, "
                        "scanners S=19/31/61, 256 x 1 ns bins" % (seg.size, n, subrays),
            "pulses": n, "subrays": subrays,
            "per_segment_launches_ms": t_seg, "persistent_ms": t_pers, "grouped_ms": t_grp, "tuned_ms": t_tuned,
            "graph_tuned_ms": t_graph, "subrays_per_s_graph": subrays / (t_graph * 1e-3),
            "pulses_per_s_graph": n / (t_graph * 1e-3),
            "subrays_per_s_per_segment": subrays / (t_seg * 1e-3),
            "speedup_vs_per_segment": t_seg / t_graph, "tuned_launch": cfg_tuned, "autotune": tune}


def bench_grad(ctx, steps):
    """Differentiation workload: forward = new heights and reflectance into the
    scene (refit) + fused forward with fixed window origins + L2 loss against a
    perturbed target; backward = loss gradient + the adjoint kernel."""
    import torch
    from synth import configs
    import paper_2101_09154_amd as vp
    mesh, target, pulses, sc = configs.diff_als()
    dev = torch.device("cuda", 0)
    scene = ctx.scene(mesh.vertices, mesh.triangles, mesh.reflectance)
    tscene = ctx.scene(target.vertices, target.triangles, target.reflectance)
    o = torch.from_numpy(pulses.origins).to(dev)
    d = torch.from_numpy(pulses.directions).to(dev)
    t0 = ctx.simulate(scene, sc, o, d)["window_t0_ns"].clone()
    tgt = ctx.simulate(tscene, sc, o, d, t0=t0)["waveform"].clone()
    base_xy = torch.from_numpy(mesh.vertices[:, :2].copy()).to(dev)
    heights = torch.from_numpy(mesh.vertices[:, 2].copy()).to(dev).requires_grad_(True)
    refl = torch.from_numpy(mesh.reflectance.copy()).to(dev).requires_grad_(True)
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    fwd = bwd = 0.0
    for it in range(steps + 2):
        heights.grad = None
        refl.grad = None
        torch.cuda.synchronize()
        ev[0].record(stream)
        wf = vp.WaveformFn.apply(refl, heights, ctx, scene, sc, o, d, t0, base_xy)
        loss = ((wf - tgt) ** 2).sum()
        ev[1].record(stream)
        loss.backward()
        ev[2].record(stream)
        torch.cuda.synchronize()
        if it >= 2:
            fwd += ev[0].elapsed_time(ev[1])
            bwd += ev[1].elapsed_time(ev[2])
    fwd /= steps
    bwd /= steps
    # the adjoint in its fixed summation order (bitwise repeatable)
    ctx.set_deterministic(True)
    bwd_det = 0.0
    for it in range(steps + 2):
        heights.grad = None
        refl.grad = None
        wf = vp.WaveformFn.apply(refl, heights, ctx, scene, sc, o, d, t0, base_xy)
        loss = ((wf - tgt) ** 2).sum()
        torch.cuda.synchronize()
        ev[1].record(stream)
        loss.backward()
        ev[2].record(stream)
        torch.cuda.synchronize()
        if it >= 2:
            bwd_det += ev[1].elapsed_time(ev[2])
    ctx.set_deterministic(False)
    bwd_det /= steps
    S = vp.n_subrays(sc)
    return {"workload": "diff_als: 256x256 value-noise DTM (130,050 triangles), 100,000 ALS pulses at 200 m, "
                        "31 subrays, 512 x 0.5 ns bins; L2 loss to a target with heights +-0.2 m and "
                        "reflectance +-0.05",
            "forward_ms": fwd, "backward_ms": bwd, "bwd_fwd_ratio": bwd / fwd,
            "backward_deterministic_ms": bwd_det, "bwd_fwd_ratio_deterministic": bwd_det / fwd,
            "forward_subrays_per_s": pulses.n * S / (fwd * 1e-3), "loss": float(loss.item()),
            "grad_norm_reflectance": float(refl.grad.norm().item()),
            "grad_norm_heights": float(heights.grad.norm().item())}


def bench_voxels(ctx, steps, tune_cache=None):
    """Transmissive voxels (Sec. 3.5.4, Sec. 5.2): the uls_voxels forest, crowns
    as a voxel grid of plant area density over woody trees and terrain (launch
    configuration from the autotuner's cache)."""
    import torch
    from synth import configs
    import paper_2101_09154_amd as vp
    mesh, vox, pulses, sc = configs.uls_voxels()
    dev = torch.device("cuda", 0)
    scene = ctx.scene(mesh.vertices, mesh.triangles, mesh.reflectance)
    scene.set_voxels(vox["origin"], vox["size"], vox["pad"], vox["lut"], vox["seed"])
    o = torch.from_numpy(pulses.origins).to(dev)
    d = torch.from_numpy(pulses.directions).to(dev)
    n = pulses.n
    S = vp.n_subrays(sc)
    out = ctx.alloc_outputs(n, S, sc["n_bins"], sc["max_returns"], dev)
    stream = torch.cuda.current_stream()
    cfg0 = ctx.launch_config()
    tune = ctx.autotune(scene, sc, o, d, out, cache_path=tune_cache)
    ctx.simulate(scene, sc, o, d, out=out)
    torch.cuda.synchronize()
    vfrac = float((out["subray_tri"] >= mesh.n_triangles).float().mean().item())
    ms = time_ms(lambda: ctx.simulate(scene, sc, o, d, out=out), steps, 1, stream)
    ctx.profile(True)
    for _ in range(steps):
        ctx.simulate(scene, sc, o, d, out=out)
    prof = ctx.profile_read()
    ctx.profile(False)
    nz, ny, nx = vox["pad"].shape
    res = {"workload": "uls_voxels: uls_trees terrain and flight (2,000,000 pulses, 61 subrays, 512 x 0.5 ns bins), "
                       "trunks and branches as %d triangles, crowns as %d x %d x %d voxels of 0.5 m"
                       % (mesh.n_triangles, nx, ny, nz),
           "ms": ms, "subrays_per_s": n * S / (ms * 1e-3), "pulses_per_s": n / (ms * 1e-3),
           "voxel_echo_fraction": vfrac,
           "fused_ms": prof["fused_ms"] / max(prof["fused_launches"], 1),
           "cone_ms": prof["cone_ms"] / max(prof["cone_launches"], 1),
           "packet_ms": prof["packet_ms"] / max(prof["packet_launches"], 1),
           "launch": ctx.launch_config(), "autotune": tune}
    ctx.set_launch_config(**cfg0)
    scene.close()
    return res


def bench_instanced(ctx, steps):
    """Scene parts placed by affine maps (Sec. 3.5, Sec. 5.1): the uls_instanced
    forest, 2,000 trees as instances of 8 models, built from the parts on the
    device, then one step per timed iteration."""
    import torch
    from synth import configs
    import paper_2101_09154_amd as vp
    parts, inst, pulses, sc = configs.uls_instanced()
    ps = [(m.vertices, m.triangles, m.reflectance) for m in parts]
    ctx.scene_instanced(ps, inst).close()       # code objects and first allocations
    torch.cuda.synchronize()
    t = time.perf_counter()
    scene = ctx.scene_instanced(ps, inst)
    build_ms = (time.perf_counter() - t) * 1e3
    dev = torch.device("cuda", 0)
    o = torch.from_numpy(pulses.origins).to(dev)
    d = torch.from_numpy(pulses.directions).to(dev)
    n = pulses.n
    S = vp.n_subrays(sc)
    out = ctx.alloc_outputs(n, S, sc["n_bins"], sc["max_returns"], dev, subrays=False)
    ms = time_ms(lambda: ctx.simulate(scene, sc, o, d, out=out), steps, 1, torch.cuda.current_stream())
    res = {"workload": "uls_instanced: uls_trees terrain and flight, 2,000 trees as instances of 8 procedural models "
                       "(turned, scaled 0.8-1.2, moved); %d placed triangles" % scene.n_triangles,
           "instances": len(inst), "placed_triangles": scene.n_triangles,
           "part_triangles": int(sum(m.n_triangles for m in parts)),
           "build_from_parts_ms": build_ms, "ms": ms, "subrays_per_s": n * S / (ms * 1e-3),
           "device_bytes": scene.stats()["device_bytes"]}
    scene.close()
    # the same scene in two levels: the parts once, a tree of the instances
    ctx.scene_instanced(ps, inst, two_level=True).close()
    torch.cuda.synchronize()
    t = time.perf_counter()
    two = ctx.scene_instanced(ps, inst, two_level=True)
    tl_build = (time.perf_counter() - t) * 1e3
    tl_ms = time_ms(lambda: ctx.simulate(two, sc, o, d, out=out), max(steps // 4, 1), 1, torch.cuda.current_stream())
    res["two_level"] = {"build_ms": tl_build, "ms": tl_ms, "subrays_per_s": n * S / (tl_ms * 1e-3),
                        "device_bytes": two.stats()["device_bytes"]}
    two.close()
    return res


def run_leg(ctx, leg, steps, tune=True, tune_cache=None):
    """The vegetation workload (2,000 trees, ~10M triangles, 2M ULS pulses, 61
    subrays, K = 8; scene larger than the caches, so HBM-level figures) or the
    small terrestrial one (7,938 triangles, 10,000 pulses, 19 subrays; the scene
    stays in L2, so L2-level figures), each with its own tuned launch."""
    import torch
    from synth import configs
    import paper_2101_09154_amd as vp
    cfg0 = ctx.launch_config()
    if leg == "uls_trees":
        mesh, pulses, sc = configs.uls_trees()
        label = ("uls_trees: 2,000 procedural trees on a 200 x 200 m fBm DTM (%d triangles), 2,000,000 ULS "
                 "pulses at 60 m AGL, 61 subrays, 512 x 0.5 ns bins, K=8" % mesh.n_triangles)
        seed, hbm = configs.ULS_SEED, True
    else:
        mesh, pulses, sc = configs.small_tls()
        label = ("small_tls: 64 x 64 value-noise DTM at 1 m (7,938 triangles), 10,000 TLS pulses on a 100 x 100 "
                 "grid, 19 subrays, 256 x 1 ns bins, K=8")
        seed, hbm = configs.SMALL_SEED, False
    tuned = None
    if tune:
        scene = ctx.scene(mesh.vertices, mesh.triangles, mesh.reflectance)
        o = torch.from_numpy(pulses.origins).cuda()
        d = torch.from_numpy(pulses.directions).cuda()
        out = ctx.alloc_outputs(pulses.n, vp.n_subrays(sc), sc["n_bins"], sc["max_returns"], o.device,
                                subrays=False)
        tuned = ctx.autotune(scene, sc, o, d, out, cache_path=tune_cache)
        scene.close()
        del o, d, out
    res = bench_plain(ctx, leg, label, mesh, pulses, sc, steps, seed, hbm=hbm)
    res["launch"] = ctx.launch_config()
    res["autotune"] = tuned
    ctx.set_launch_config(**cfg0)
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--block-waves", type=int, default=1)
    ap.add_argument("--stack-lds", type=int, default=16)
    ap.add_argument("--only-plain", action="store_true", help="skip the batched and gradient workloads")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (three times), to scale HBM counters")
    ap.add_argument("--tune-cache", default=TUNE_CACHE,
                    help="autotuner cache (JSON lines); '' tunes every workload afresh")
    ap.add_argument("--leg", choices=["uls_trees", "small_tls", "batched_tls", "uls_voxels"], default=None,
                    help="only run this workload's leg and print its record (for profiling)")
    args = ap.parse_args()
    args.tune_cache = args.tune_cache or None
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU form "
              "(pulses would shard across GPUs with no exchange)", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_calibration:
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": nbytes}))
        return
    from synth import configs
    import paper_2101_09154_amd as vp

    if args.leg:
        ctx = vp.Context(0)
        if args.leg == "batched_tls":
            # the 256 positions on the als_buildings scene, launch from the cache
            log("batched workload")
            mesh, _, _ = configs.als_buildings()
            scene = ctx.scene(mesh.vertices, mesh.triangles, mesh.reflectance)
            rec = bench_batched(ctx, scene, mesh, args.steps, tune_cache=args.tune_cache)
        elif args.leg == "uls_voxels":
            log("voxel workload")
            rec = bench_voxels(ctx, args.steps, tune_cache=args.tune_cache)
        else:
            if not args.no_tune:
                log("autotune (%s)" % args.leg)
            rec = run_leg(ctx, args.leg, args.steps, tune=not args.no_tune, tune_cache=args.tune_cache)
        print(json.dumps(rec), flush=True)
        return
    log("generating scene and pulses")
    mesh, pulses, sc = configs.als_buildings()
    dev = torch.device("cuda", 0)
    ctx = vp.Context(0)
    ctx.set_launch_config(block_waves=args.block_waves, stack_lds=args.stack_lds)
    # the first build of a process also pays for loading the code objects and
    # the first device allocations; the build time reported is a second build
    torch.cuda.synchronize()
    t = time.perf_counter()
    scene = ctx.scene(mesh.vertices, mesh.triangles, mesh.reflectance)
    first_build_ms = (time.perf_counter() - t) * 1e3
    scene.close()
    torch.cuda.synchronize()
    t = time.perf_counter()
    scene = ctx.scene(mesh.vertices, mesh.triangles, mesh.reflectance)
    build_ms = (time.perf_counter() - t) * 1e3
    stats = scene.stats()
    log("scene built in %.1f ms: %s" % (build_ms, stats))
    o = torch.from_numpy(pulses.origins).to(dev)
    d = torch.from_numpy(pulses.directions).to(dev)
    n = pulses.n
    S = vp.n_subrays(sc)
    K = sc["max_returns"]
    nb = sc["n_bins"]
    out = ctx.alloc_outputs(n, S, nb, K, dev, subrays=False)

    log("traversal counters")
    n_sub, visits, tests = ctx.trace_counts(scene, sc, o, d)
    v_node = visits / n_sub   # node fetches per subray (the cone pass fetches once per pulse)
    v_tri = tests / n_sub
    hit_frac = None

    stream = torch.cuda.current_stream()
    tune = None
    if not args.no_tune:
        log("autotune (plain)")
        tune = ctx.autotune(scene, sc, o, d, out, cache_path=args.tune_cache)
    for _ in range(args.warmup):
        ctx.simulate(scene, sc, o, d, out=out)
    torch.cuda.synchronize()
    hit_frac = float((out["n_returns"] > 0).float().mean().item())
    log("timing %d steps" % args.steps)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        ctx.simulate(scene, sc, o, d, out=out)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall
    ms = ev0.elapsed_time(ev1) / args.steps
    sub_per_s = n * S / (ms * 1e-3)
    pulse_per_s = n / (ms * 1e-3)

    # per-kernel times: the library records HIP events on the launch stream
    # around the cone pass and around the fused kernel of each call
    ctx.profile(True)
    for _ in range(args.steps):
        ctx.simulate(scene, sc, o, d, out=out)
    prof = ctx.profile_read()
    ctx.profile(False)
    cone_ms = prof["cone_ms"] / max(prof["cone_launches"], 1)
    packet_ms = prof["packet_ms"] / max(prof["packet_launches"], 1)
    sim_ms = prof["fused_ms"] / max(prof["fused_launches"], 1)
    per_pulse_io = 36.0 + 4.0 * nb + 8.0 + 4.0 + 16.0 * K
    cand_per_pulse = tests / n_sub   # every subray tests its pulse's candidates
    # fused kernel: pulse in, candidate count and ids and the candidate
    # triangles (48 B each) per pulse, a reflectance per subray, outputs out
    sim_bytes = n * (per_pulse_io + 4.0 + 52.0 * cand_per_pulse) + 4.0 * n_sub
    # cone pass: 112 B per four-wide record visited (six coordinate rows and the
    # refs), 48 B per leaf reached, pulse in, list out
    cone_bytes = 112.0 * visits + n * (36.0 + 4.0 + 52.0 * cand_per_pulse)
    alg_bytes = sim_bytes + cone_bytes
    achieved = sim_bytes / (sim_ms * 1e-3) / 1e9
    # bytes the whole step must move at least once: the scene as the step reads it
    # (112 B of each four-wide record, the leaf records, reflectances), pulses in,
    # outputs out
    scene_bytes = 112.0 * max(mesh.n_triangles - 1, 1) + 48.0 * mesh.n_triangles + 4.0 * mesh.n_triangles
    compulsory = scene_bytes + n * per_pulse_io
    khash = source_hash()
    traffic = measured_traffic(khash)

    res = {
        "metric": "subrays/s & pulses/s w/ full waveform, plain vs batched; bwd/fwd time ratio",
        "value": sub_per_s,
        "unit": "subrays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "als_buildings: 1024x1024 fBm DTM at 0.5 m + 20,000 boxes (2,333,058 triangles), "
                               "1,000,000 ALS pulses at 500 m AGL, 31 subrays, 512 x 0.5 ns bins, K=8",
                   "pulses": n, "subrays_per_pulse": S, "n_bins": nb, "max_returns": K,
                   "triangles": mesh.n_triangles, "parallelism": "single GPU",
                   "launch": ctx.launch_config()},
        "pulses_per_s": pulse_per_s,
        "scene_build_ms": build_ms,
        "scene_build_first_ms": first_build_ms,
        "scene_depth": stats["max_depth"],
        "node_visits_per_subray": v_node,
        "tri_tests_per_subray": v_tri,
        "cone_node_visits_per_pulse": visits / n,
        "candidates_per_pulse": cand_per_pulse,
        "pulses_with_returns": hit_frac,
        "wall_s_timed": wall,
        "roofline": {"bound": "hbm", "kernel": "k_simulate (fused subray tests, power, waveform, returns)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "algorithmic_bytes_per_launch": sim_bytes, "kernel_ms": sim_ms,
                     "source_hash": khash,
                     "cone_pass": {"kernel_ms": cone_ms, "algorithmic_bytes_per_launch": cone_bytes,
                                   "achieved": cone_bytes / (cone_ms * 1e-3) / 1e9},
                     "packet_walk": {"kernel_ms": packet_ms},
                     "timing": "HIP events recorded by the library on the launch stream around each kernel, "
                               "mean of %d launches" % prof["fused_launches"],
                     "step": {"ms": ms, "algorithmic_bytes": alg_bytes,
                              "achieved": alg_bytes / (ms * 1e-3) / 1e9,
                              "compulsory_bytes": compulsory,
                              "compulsory_frac": compulsory / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}},
    }
    # echo width (Sec. 3.4, optional): a Gaussian fitted to each kept return
    log("echo width")
    width = torch.empty((n, K), dtype=torch.float32, device=dev)
    ctx.echo_width(sc, o, d, out, width=width)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        ctx.echo_width(sc, o, d, out, width=width)
    e1.record(stream)
    torch.cuda.synchronize()
    ew_ms = e0.elapsed_time(e1) / args.steps
    n_ret = int(out["n_returns"].sum().item())
    res["echo_width"] = {"ms": ew_ms, "returns": n_ret, "returns_per_s": n_ret / (ew_ms * 1e-3),
                         "fitted": int(torch.isfinite(width).sum().item()),
                         "step_with_echo_width_over_step": (ms + ew_ms) / ms,
                         "paper_runtime_factor": 1.3}
    # pulses generated on the device from a survey (Sec. 3.2, 3.3): a flight
    # line 500 m above the terrain with a polygon mirror of +-30 deg, 1,000 pulses
    # per line, as many pulses as the workload; then one step on them
    log("pulse generation")
    ext = mesh.info["extent"]
    z = mesh.info["heights_mean"] + 500.0
    survey = dict(waypoints=[[0.05 * ext, 0.5 * ext, z], [0.95 * ext, 0.5 * ext, z]], deflector="polygon",
                  speed_mps=60.0, pulse_rate_hz=1.0e6, scan_freq_hz=1.0e3, scan_angle_rad=math.radians(30.0),
                  platform_noise_m=0.02, seed=2021)
    go = torch.empty((n, 3), dtype=torch.float64, device=dev)
    gd = torch.empty((n, 3), dtype=torch.float32, device=dev)
    ctx.generate_pulses(survey, 0, n, origins=go, directions=gd)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        ctx.generate_pulses(survey, 0, n, origins=go, directions=gd)
    e1.record(stream)
    torch.cuda.synchronize()
    gen_ms = e0.elapsed_time(e1) / args.steps
    gstep_ms = None
    if not args.only_plain:   # (kept out of the profiled runs: a different pulse set)
        e0.record(stream)
        for _ in range(args.steps):
            ctx.generate_pulses(survey, 0, n, origins=go, directions=gd)
            ctx.simulate(scene, sc, go, gd, out=out)
        e1.record(stream)
        torch.cuda.synchronize()
        gstep_ms = e0.elapsed_time(e1) / args.steps
    res["pulse_generation"] = {"survey": "LinearPath 500 m above mean ground across the scene, polygon mirror "
                                         "+-30 deg, 1e6 pulses/s, 1e3 lines/s, platform noise 2 cm",
                               "ms": gen_ms, "pulses_per_s": n / (gen_ms * 1e-3),
                               "bytes_written_per_pulse": 36,
                               "achieved_GBps": 36.0 * n / (gen_ms * 1e-3) / 1e9,
                               "step_with_generation_ms": gstep_ms,
                               "subrays_per_s_with_generation": n * S / (gstep_ms * 1e-3) if gstep_ms else None}
    if not args.only_plain:   # (kept out of the profiled runs: other surveys and scanners)
        # a Multicopter (Sec. 3.2) flying three legs 100 m above the terrain with
        # ramps at every waypoint and turning yaws, a Palmer scanner; and the
        # step with a 2 cm ranging error on every return (Sec. 3.7)
        log("multicopter generation, ranging error")
        zc = mesh.info["heights_mean"] + 100.0
        mc = dict(waypoints=[[0.1 * ext, 0.1 * ext, zc], [0.9 * ext, 0.1 * ext, zc], [0.9 * ext, 0.2 * ext, zc],
                             [0.1 * ext, 0.2 * ext, zc]],
                  platform="multicopter", speed_mps=8.0, accel_mps2=2.0,
                  leg_yaw=[[0.0, 0.3], [1.57, 1.57], [3.14, 2.9]], deflector="conic", pulse_rate_hz=2.0e4,
                  scan_freq_hz=50.0, scan_angle_rad=math.radians(15.0), platform_noise_m=0.02, seed=7)
        ctx.generate_pulses(mc, 0, n, origins=go, directions=gd)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(args.steps):
            ctx.generate_pulses(mc, 0, n, origins=go, directions=gd)
        e1.record(stream)
        torch.cuda.synchronize()
        mc_ms = e0.elapsed_time(e1) / args.steps
        res["pulse_generation"]["multicopter"] = {
            "survey": "Multicopter 100 m above mean ground, three legs from rest to rest (8 m/s, 2 m/s^2, "
                      "turning yaws), Palmer scanner 15 deg, 2e4 pulses/s, platform noise 2 cm",
            "ms": mc_ms, "pulses_per_s": n / (mc_ms * 1e-3)}
        scn = dict(sc, range_noise_m=0.02, noise_seed=11)
        ctx.simulate(scene, scn, o, d, out=out)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(args.steps):
            ctx.simulate(scene, scn, o, d, out=out)
        e1.record(stream)
        torch.cuda.synchronize()
        rn_ms = e0.elapsed_time(e1) / args.steps
        res["ranging_error"] = {"sigma_m": 0.02, "ms": rn_ms, "step_with_ranging_error_over_step": rn_ms / ms}
    if not args.only_plain:   # (kept out of the profiled runs: the same kernel with the lobe on)
        # specular materials (Sec. 5.1): the same step with a Phong-type part on every triangle
        log("specular materials")
        g = torch.Generator(device="cpu").manual_seed(5)
        ks = torch.rand(mesh.n_triangles, generator=g).mul_(0.9).to(dev)
        ne = torch.rand(mesh.n_triangles, generator=g).mul_(7.0).add_(1.0).to(dev)
        scene.set_specular(ks, ne)
        spec_ms = time_ms(lambda: ctx.simulate(scene, sc, o, d, out=out), args.steps, 1, stream)
        scene.set_specular()
        res["specular"] = {"ms": spec_ms, "step_with_specular_over_step": spec_ms / ms,
                           "materials": "specularity U(0, 0.9), exponent U(1, 8) per triangle"}
    res["autotune"] = tune
    if not args.only_plain:
        log("batched workload")
        res["batched"] = bench_batched(ctx, scene, mesh, args.steps // 2 if args.steps > 2 else 1,
                                       tune_cache=args.tune_cache)
        log("gradient workload")
        res["gradient"] = bench_grad(ctx, max(args.steps // 2, 2))
        log("voxel workload")
        res["voxels"] = bench_voxels(ctx, max(args.steps // 2, 2), tune_cache=args.tune_cache)
        log("instanced workload")
        res["instanced"] = bench_instanced(ctx, max(args.steps // 2, 2))
    if not args.only_plain:
        for leg in ("uls_trees", "small_tls"):
            log("%s workload" % leg)
            res[leg] = run_leg(ctx, leg, max(args.steps // 2, 2), tune=not args.no_tune, tune_cache=args.tune_cache)
        log("copy bandwidth")
        res["copy_bandwidth"] = copy_bandwidth()
    res["inputs"] = input_digest(mesh, pulses, sc, configs.ALS_SEED)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        res["cpu_baseline"] = cpu_baseline(mesh, pulses, sc, args.cpu_seconds)
        res["cpu_baseline"]["cpu_model"] = cpu_model()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
