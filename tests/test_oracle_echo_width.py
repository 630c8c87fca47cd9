"""Pins of the oracle's echo width (Sec. 3.4: an optional Gaussian fitted by
non-linear least squares to the waveform around each return; its standard
deviation is the echo width).  The fit is pinned to closed forms (exact
Gaussian samples), to an independent solver (scipy's Levenberg-Marquardt run
to convergence on the same samples), and to invariances of the least-squares
problem."""
import numpy as np
import pytest
from scipy.optimize import least_squares

from synth import configs

HALF = 31  # lobe half-width cap, in bins


def _lobe(wf, j):
    """The samples the fit must use: from j outward while the waveform keeps
    falling strictly and stays at or above 2^-10 of wf[j], at most HALF bins to
    each side (written here from the reading, independently of the oracle)."""
    floor = wf[j] / 1024.0
    L = j
    while L > 0 and j - L < HALF and wf[L - 1] < wf[L] and wf[L - 1] >= floor:
        L -= 1
    R = j
    while R < len(wf) - 1 and R - j < HALF and wf[R + 1] < wf[R] and wf[R + 1] >= floor:
        R += 1
    return np.arange(L, R + 1)


def _scipy_fit(wf, j, p0):
    idx = _lobe(wf, j)
    x = (idx - j).astype(np.float64)
    y = wf[idx]

    def res(p):
        return p[0] * np.exp(-(x - p[1]) ** 2 / (2 * p[2] ** 2)) - y

    r = least_squares(res, p0, method="lm", xtol=1e-15, ftol=1e-15, gtol=1e-15, max_nfev=20000)
    return np.array([r.x[0], r.x[1], abs(r.x[2])])  # only s^2 enters the model


def _gauss(x, A, mu, s):
    return A * np.exp(-(x - mu) ** 2 / (2 * s * s))


@pytest.mark.parametrize("A,mu,s", [(2.5, 0.3, 3.1), (1e-3, -0.45, 0.8), (7.0, 0.1, 12.0), (1.0, 0.0, 40.0)])
def test_exact_gaussian_recovered(orc, A, mu, s):
    # noise-free Gaussian samples: the least-squares optimum is the generator
    # itself (cost 0), also when the lobe is cut at 31 bins (s = 40) or at
    # 2^-10 of the peak (the others)
    x = np.arange(160, dtype=np.float64)
    j = 80
    wf = _gauss(x, A, j + mu, s)
    assert int(np.argmax(wf)) == j
    w, p = orc.echo_width_bins(wf, j, 4.0)
    assert abs(w - s) <= 1e-9 * s
    assert abs(p[0] - A) <= 1e-9 * A and abs(p[1] - mu) <= 1e-9


def _cases():
    x = np.arange(128, dtype=np.float64)
    rng = np.random.default_rng(7)
    two = _gauss(x, 1.0, 60.0, 3.0) + _gauss(x, 0.45, 65.5, 2.2)           # overlapping echoes
    tau = 2.0
    u = np.maximum(x - 55.0, 0.0) / tau
    eq3 = u * u * np.exp(-u)                                                # Eq. 3 pulse, not a Gaussian
    noisy = _gauss(x, 2.0, 64.2, 4.0) * (1.0 + 0.02 * rng.standard_normal(x.size))
    flat_top = np.minimum(_gauss(x, 1.0, 70.0, 6.0), 0.97) + 1e-3 * _gauss(x, 1.0, 70.3, 1.0)
    return {"two": two, "eq3": eq3, "noisy": noisy, "flat_top": flat_top}


@pytest.mark.parametrize("name", ["two", "eq3", "noisy", "flat_top"])
def test_matches_independent_solver(orc, name):
    # non-Gaussian lobes: the oracle's twelve iterations reach the optimum that
    # scipy's Levenberg-Marquardt finds when run to convergence on the same
    # samples, from two starts (within 1e-6 relative: far below what an FP32
    # fit resolves)
    wf = _cases()[name]
    j = int(np.argmax(wf))
    w, p = orc.echo_width_bins(wf, j, 4.0)
    ref = _scipy_fit(wf, j, p)
    ref2 = _scipy_fit(wf, j, np.array([wf[j], 0.0, 4.0]))
    assert np.allclose(ref, ref2, rtol=1e-6, atol=1e-6), (ref, ref2)   # one optimum
    assert abs(w - ref[2]) <= 1e-6 * ref[2], (w, ref)
    assert abs(p[0] - ref[0]) <= 1e-6 * ref[0] and abs(p[1] - ref[1]) <= 1e-6


def test_invariances(orc):
    wf = _cases()["two"]
    j = int(np.argmax(wf))
    w, p = orc.echo_width_bins(wf, j, 4.0)
    # scaling the waveform scales A only
    w7, p7 = orc.echo_width_bins(7.0 * wf, j, 4.0)
    assert abs(w7 - w) <= 1e-9 * w and abs(p7[0] - 7.0 * p[0]) <= 1e-9 * p7[0]
    # mirroring the waveform mirrors mu
    n = wf.size
    wm, pm = orc.echo_width_bins(wf[::-1].copy(), n - 1 - j, 4.0)
    assert abs(wm - w) <= 1e-9 * w and abs(pm[1] + p[1]) <= 1e-9


def test_each_return_uses_its_own_lobe(orc):
    x = np.arange(200, dtype=np.float64)
    a = _gauss(x, 1.0, 50.0, 3.0)
    b = _gauss(x, 0.6, 120.0, 5.5)
    both = a + b
    assert orc.echo_width_bins(both, 50, 4.0)[0] == pytest.approx(3.0, rel=1e-9)
    assert orc.echo_width_bins(both, 120, 4.0)[0] == pytest.approx(5.5, rel=1e-9)


def test_lobe_floor(orc):
    # bins below 2^-10 of the return bin's value are left out: a pedestal far
    # below the echo does not widen it
    x = np.arange(200, dtype=np.float64)
    wf = _gauss(x, 1.0, 100.0, 3.0) + 2e-4 * _gauss(x, 1.0, 100.0, 60.0)
    L, R = _lobe(wf, 100)[[0, -1]]
    assert R - L + 1 < 2 * HALF + 1 and wf[L] >= wf[100] / 1024 and wf[L - 1] < wf[100] / 1024
    w, _ = orc.echo_width_bins(wf, 100, 4.0)
    idx = _lobe(wf, 100)
    ref = _scipy_fit(wf, 100, np.array([1.0, 0.0, 3.0]))
    assert abs(w - ref[2]) <= 1e-6 * ref[2]


@pytest.mark.parametrize("side", [-1, 1])
def test_lobe_stops_at_a_plateau(orc, side):
    # the lobe ends where the waveform stops falling strictly: two equal bins
    # on one flank end it there, and the fit uses only the bins before them
    x = np.arange(128, dtype=np.float64)
    wf = _gauss(x, 1.0, 64.2, 3.0) + 0.3 * _gauss(x, 1.0, 64.0 + side * 9.0, 4.0)
    j = int(np.argmax(wf))
    k = j + side * 4
    wf[k + side] = wf[k]          # a plateau four bins out
    idx = _lobe(wf, j)
    assert (idx[0] if side < 0 else idx[-1]) == k
    w, p = orc.echo_width_bins(wf, j, 3.0)
    ref = _scipy_fit(wf, j, p)
    assert abs(w - ref[2]) <= 1e-6 * ref[2], (w, ref)


def test_no_fit_cases(orc):
    # a lobe of two bins (a dip before the peak, a plateau after it) has no fit
    wf = np.zeros(16)
    wf[2], wf[3], wf[4], wf[5] = 0.5, 0.4, 1.0, 1.0
    w, _ = orc.echo_width_bins(wf, 4, 2.0)
    assert np.isnan(w)
    # three bins do: the Gaussian through them
    wf[2] = 0.01
    w3, p3 = orc.echo_width_bins(wf, 4, 2.0)
    assert np.isfinite(w3) and p3[0] > 0.0
    # out of range
    assert np.isnan(orc.echo_width_bins(wf, -1, 2.0)[0]) and np.isnan(orc.echo_width_bins(wf, 16, 2.0)[0])


def test_widths_in_ns(orc):
    # per-waveform form: widths in ns, starting from the pulse's own sigma
    sc = configs.scanner(1e-3, 1, pulse_width_ns=4.0, bin_ns=0.5, n_bins=256)
    x = np.arange(256, dtype=np.float64)
    wf = _gauss(x, 1.0, 80.0, 3.4) + _gauss(x, 0.5, 170.2, 4.4)
    bins = np.array([80, 170], np.int32)
    w = orc.echo_width(sc, wf, bins)
    assert w[0] == pytest.approx(3.4 * 0.5, rel=1e-9) and w[1] == pytest.approx(4.4 * 0.5, rel=1e-9)
