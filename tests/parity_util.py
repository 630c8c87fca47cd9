"""Comparison of GPU outputs with the oracle at the stated tolerances.

Hit triangle ids: >= 99.99 % equal, and every mismatch excused: in FP64 the
subray hits the GPU's triangle (when the GPU reports one) and the hit lies
within 1e-6 (barycentric) of an edge of either triangle, or the two hit
distances agree to 1e-6 relative (a depth tie).  A miss against a hit is
excused only at an edge of the hit triangle.  A voxel echo (id >= n_triangles)
against anything else is excused only where the two distances agree to 1e-6
relative; equal voxel echoes carry Eq. 7's power to 1e-6 relative and cos 1.
Range: <= 1e-4 m on equal ids.
Waveform: per-pulse relative L2 <= 1e-5 for pulses whose ids all match;
all-miss pulses are all zero.
Returns: the GPU's bins are the oracle's first bins in time order (all of them
when the GPU kept fewer than K) except where the oracle's waveform has a near
tie (|wf[j] - wf[j +- 1]| or |wf[j] - thr| <= 1e-5 max wf) at a differing bin;
range, amplitude and attribution on every bin both sides report.
"""
import numpy as np

import oracle

C = oracle.C_M_PER_NS
EDGE = 1e-6
RANGE_TOL = 1e-4
WF_TOL = 1e-5
ID_FRACTION = 0.9999


def to_np(out):
    return {k: v.detach().cpu().numpy() for k, v in out.items()}


def _bary_min(O, d, mesh, tri):
    """Plane hit of the ray on triangle `tri` in FP64 without any inside test:
    (hit within 1e-6 of the triangle, t, smallest barycentric coordinate)."""
    V = mesh.vertices[mesh.triangles[tri]].astype(np.float64)
    e1 = V[1] - V[0]
    e2 = V[2] - V[0]
    n = np.cross(e1, e2)
    dn = float(d @ n)
    if dn == 0.0:
        return False, np.inf, -np.inf
    t = float((V[0] - O) @ n) / dn
    X = O + t * d
    nn = float(n @ n)
    u = float(np.cross(X - V[0], e2) @ n) / nn
    v = float(np.cross(e1, X - V[0]) @ n) / nn
    b = min(u, v, 1.0 - u - v)
    return (t > 0 and b >= -EDGE), t, b


def check_hits(mesh, pulses, sc, sel, g, r, report):
    """g: GPU dict (numpy) rows for the selected pulses; r: oracle result."""
    S = r.S
    nt = mesh.n_triangles
    gt = g["subray_tri"][:, :S]
    eq = gt == r.sub_tri
    frac = float(eq.mean())
    report["id_fraction"] = frac
    bad = np.argwhere(~eq)
    unexcused = []
    for q, k in bad:
        p = sel[q]
        go, oo = int(gt[q, k]), int(r.sub_tri[q, k])
        if go >= nt or oo >= nt:
            # a voxel echo (id >= n_triangles) against anything else: excused
            # only where the two distances tie
            rg, ro = float(g["subray_range"][q, k]), float(r.sub_range[q, k])
            if not (np.isfinite(rg) and np.isfinite(ro) and abs(rg - ro) <= 1e-6 * ro):
                unexcused.append((int(p), int(k), go, oo))
            continue
        O = pulses.origins[p].astype(np.float64)
        d = oracle.subray_directions(pulses.directions[p].astype(np.float64), sc)[k]
        ok = False
        if go >= 0:
            hg, tg, bg = _bary_min(O, d, mesh, go)
            if hg:
                if oo >= 0:
                    ho, to, bo = _bary_min(O, d, mesh, oo)
                    ok = bg <= EDGE or bo <= EDGE or abs(tg - to) <= 1e-6 * to
                else:
                    ok = bg <= EDGE
        else:
            ho, to, bo = _bary_min(O, d, mesh, oo)
            ok = bo <= EDGE
        if not ok:
            unexcused.append((int(p), int(k), go, oo))
    report["mismatches"] = int(bad.shape[0])
    report["unexcused"] = unexcused
    ranges = np.abs(g["subray_range"][:, :S] - r.sub_range)
    m = eq & (r.sub_tri >= 0)
    report["max_range_err"] = float(ranges[m].max()) if m.any() else 0.0
    miss_ok = bool(np.all(np.isinf(g["subray_range"][:, :S][eq & (r.sub_tri < 0)])))
    report["miss_ok"] = miss_ok
    power_ok = True
    vm = eq & (r.sub_tri >= nt)
    if vm.any() and "subray_power" in g:
        # voxel echoes: Eq. 7's power, rounded once to FP32 by the GPU
        rel = np.abs(g["subray_power"][:, :S][vm] - r.sub_power[vm]) / r.sub_power[vm]
        report["voxel_echoes"] = int(vm.sum())
        report["voxel_power_rel_err"] = float(rel.max())
        power_ok = report["voxel_power_rel_err"] <= 1e-6 and bool(np.all(g["subray_cos"][:, :S][vm] == 1.0))
    return (frac >= ID_FRACTION and not unexcused and report["max_range_err"] <= RANGE_TOL and miss_ok
            and power_ok)


def check_waveforms(g, r, report):
    S = r.S
    allmatch = np.all(g["subray_tri"][:, :S] == r.sub_tri, axis=1)
    wf = g["waveform"].astype(np.float64)
    nrm = np.linalg.norm(r.waveform, axis=1)
    rel = np.linalg.norm(wf - r.waveform, axis=1) / np.where(nrm > 0, nrm, 1.0)
    hit = nrm > 0
    chk = allmatch & hit
    report["wf_checked"] = int(chk.sum())
    report["wf_worst"] = float(rel[chk].max()) if chk.any() else 0.0
    zero = allmatch & ~hit
    zero_ok = bool(np.all(wf[zero] == 0.0))
    report["wf_zero_ok"] = zero_ok
    t0ok = np.all(np.isnan(g["window_t0_ns"][zero]) == np.isnan(r.t0[zero]))
    dt0 = np.abs(g["window_t0_ns"][chk] - r.t0[chk])
    report["t0_max_err_ns"] = float(dt0.max()) if dt0.size else 0.0
    return report["wf_worst"] <= WF_TOL and zero_ok and bool(t0ok) and report["t0_max_err_ns"] <= 1e-6


def _near_tie(w, j, thr, scale):
    eps = 1e-5 * scale
    if j <= 0 or j >= w.size - 1:
        return True
    return abs(w[j] - w[j - 1]) <= eps or abs(w[j] - w[j + 1]) <= eps or abs(w[j] - thr) <= eps


def check_returns(g, r, sc, report):
    """Returns of every pulse whose subray ids all match the oracle's.

    The oracle's complete list of local maxima comes from its own FP64
    waveform (its peak rule with no cap on the count); its K-limited returns
    must be the prefix of that list (first K in time order).  The GPU keeps
    the first K in time order too, so its bins must equal the oracle's bins up
    to the GPU's last kept bin (all of them when it kept fewer than K), except
    at near ties of the oracle's waveform.  Every GPU return whose bin the
    oracle also has is compared, whether or not either side reached K: range
    (1e-4 m), amplitude (1e-5 of the waveform's maximum) and attribution.  With
    a ranging error only slots drawn alike on both sides compare ranges.
    """
    S = r.S
    K = sc.get("max_returns", 8)
    thr_abs, thr_rel = sc.get("min_echo_abs", 0.0), sc.get("min_echo_rel", 1e-3)
    noisy = sc.get("range_noise_m", 0.0) > 0.0
    allmatch = np.all(g["subray_tri"][:, :S] == r.sub_tri, axis=1)
    bad = []
    tri_bad = []
    n_sat = n_cmp = n_pulses = 0
    for q in np.nonzero(allmatch)[0]:
        n_pulses += 1
        ng, no = int(g["n_returns"][q]), int(r.n_returns[q])
        w = r.waveform[q]
        mx = w.max() if w.size else 0.0
        thr = max(thr_abs, thr_rel * mx)
        full = [int(b) for b in oracle.detect_peaks(w, thr_abs, thr_rel, K=w.size)]
        if [int(b) for b in r.ret_bin[q, :no]] != full[:K] or no != min(len(full), K):
            bad.append(int(q))  # the oracle's K-limited list is not its prefix
            continue
        bg = [int(b) for b in g["ret_bin"][q, :ng]]
        if ng < 0 or ng > K or any(bg[i] >= bg[i + 1] for i in range(ng - 1)):
            bad.append(int(q))
            continue
        if ng == K or no == K:
            n_sat += 1
        ref = full if ng < K else [b for b in full if b <= bg[-1]]
        diff = set(bg) ^ set(ref)
        if not all(_near_tie(w, j, thr, mx) for j in diff):
            bad.append(int(q))
        pos = {b: i for i, b in enumerate(full)}
        for s in range(ng):
            j = bg[s]
            so = pos.get(j)
            if so is None:
                continue  # a near-tie bin the oracle does not have
            n_cmp += 1
            if abs(float(g["ret_amplitude"][q, s]) - w[j]) > 1e-5 * mx:
                bad.append(int(q))
            if so < no:
                rr = None if noisy and so != s else float(r.ret_range[q, so])
            else:
                rr = None if noisy else oracle.echo_range(sc, r.t0[q], j)
            if rr is not None and abs(float(g["ret_range"][q, s]) - rr) > RANGE_TOL:
                bad.append(int(q))
            if so < no:
                to = int(r.ret_tri[q, so])
            else:
                kb = oracle.attribute(sc, r.sub_tri[q], r.sub_range[q], r.sub_power[q], r.t0[q] + j * sc["bin_ns"])
                to = int(r.sub_tri[q, kb]) if kb >= 0 else -1
            if int(g["ret_tri"][q, s]) != to:
                tri_bad.append((int(q), s, j))
        if np.any(g["ret_bin"][q, ng:K] != -1) or np.any(g["ret_tri"][q, ng:K] != -1):
            bad.append(int(q))
    report["returns_pulses"] = n_pulses
    report["returns_saturated"] = n_sat
    report["returns_compared"] = n_cmp
    report["returns_bad"] = sorted(set(bad))[:20]
    report["returns_bad_n"] = len(set(bad))
    report["ret_tri_mismatch"] = len(tri_bad)
    return not bad, tri_bad


def attribution_excused(mesh, pulses, sc, sel, g, r, tri_bad):
    """A differing return attribution is excused when the GPU's triangle carries a
    subray whose contribution at the bin is within 1e-5 of the largest.
    tri_bad: (row, GPU slot, bin) of each differing attribution."""
    left = []
    for q, s, j in tri_bad:
        tj = r.t0[q] + j * sc["bin_ns"]
        contrib = np.array([r.sub_power[q, k] * oracle.pulse_value(sc, tj - 2 * r.sub_range[q, k] / C)
                            if r.sub_tri[q, k] >= 0 else -1.0 for k in range(r.S)])
        best = contrib.max()
        cand = [k for k in range(r.S) if r.sub_tri[q, k] == g["ret_tri"][q, s]]
        if not cand or max(contrib[k] for k in cand) < (1 - 1e-5) * best:
            left.append((int(sel[q]), s))
    return left
