"""Per-workload parity figures collected by the GPU tests and printed at the end
of the run: pulses and subrays compared, hit-id agreement, id mismatches and
how many of them are not excused, worst range error, worst waveform relative
L2, and the returns compared."""

_rows = []


def record(label, n_pulses, S, rep):
    _rows.append((label, int(n_pulses), int(n_pulses) * int(S), rep))


def lines():
    if not _rows:
        return []
    out = ["%-28s %7s %9s %10s %6s %9s %10s %10s %8s %8s" %
           ("workload", "pulses", "subrays", "id_frac", "mism", "unexcused", "range_m", "wf_L2", "ret_cmp", "ret_bad")]
    for label, n, ns, rep in _rows:
        out.append("%-28s %7d %9d %10.6f %6d %9d %10.2e %10.2e %8d %8d" % (
            label[:28], n, ns, rep.get("id_fraction", float("nan")), rep.get("mismatches", 0),
            len(rep.get("unexcused", [])), rep.get("max_range_err", 0.0), rep.get("wf_worst", 0.0),
            rep.get("returns_compared", 0), rep.get("returns_bad_n", 0)))
    return out
