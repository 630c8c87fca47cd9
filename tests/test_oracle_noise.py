"""Pins of the oracle's ranging error (Sec. 3.7: each distance measurement
carries a normally distributed error with the scanner's parameters): mean 0,
the scanner's standard deviation, Gaussian, independent across returns and
pulses, fixed by the seed and the pulse, and on the distances alone."""
import numpy as np

import synth
from synth import configs


def _pairs(orc, sigma, seed):
    mesh, pulses, sc = configs.small_tls()
    clean = orc.simulate(mesh, pulses, sc)
    noisy = orc.simulate(mesh, pulses, dict(sc, range_noise_m=sigma, noise_seed=seed))
    return mesh, pulses, sc, clean, noisy


def test_noise_only_moves_ranges(orc):
    mesh, pulses, sc, clean, noisy = _pairs(orc, 0.05, 77)
    assert np.array_equal(clean.waveform, noisy.waveform)
    assert np.array_equal(clean.n_returns, noisy.n_returns) and np.array_equal(clean.ret_bin, noisy.ret_bin)
    assert np.array_equal(clean.ret_amp, noisy.ret_amp) and np.array_equal(clean.ret_tri, noisy.ret_tri)
    zero = orc.simulate(mesh, pulses, dict(sc, range_noise_m=0.0, noise_seed=77))
    assert np.array_equal(zero.ret_range, clean.ret_range)


def test_noise_statistics(orc):
    sigma = 0.05
    _, pulses, sc, clean, noisy = _pairs(orc, sigma, 77)
    K = sc["max_returns"]
    has = np.arange(K)[None, :] < clean.n_returns[:, None]
    e = (noisy.ret_range - clean.ret_range)[has]
    n = e.size
    assert n > 5000
    assert abs(e.mean()) < 4 * sigma / np.sqrt(n)
    assert abs(e.std() / sigma - 1.0) < 0.03
    assert abs(np.mean(np.abs(e) < sigma) - 0.6827) < 0.015          # Gaussian: one sigma
    assert abs(np.mean(np.abs(e) < 2 * sigma) - 0.9545) < 0.01
    # independent across neighbouring pulses (first returns)
    E = noisy.ret_range[:, 0] - clean.ret_range[:, 0]
    m = clean.n_returns > 0
    both = m[:-1] & m[1:]
    assert abs(np.corrcoef(E[:-1][both], E[1:][both])[0, 1]) < 0.05
    # the slots of one pulse draw their own errors: the error of slot r is the
    # one the pulse's counter gives, whatever other returns the pulse has
    q = np.nonzero(clean.n_returns > 1)[0][:50]
    for p in q:
        for r in range(clean.n_returns[p]):
            want = orc.range_noise(dict(sc, range_noise_m=sigma, noise_seed=77), p, r)
            assert abs(noisy.ret_range[p, r] - clean.ret_range[p, r] - want) < 1e-12



def test_noise_independent_within_a_pulse(orc):
    # pulses aimed at a 3 m step between two planes: two returns each, whose
    # errors are drawn apart
    lo = synth.flat_quad(-20.0, 0.0, -50.0, 50.0, 0.0, reflectance=0.5)
    hi = synth.flat_quad(0.0, 20.0, -50.0, 50.0, 3.0, reflectance=0.5)
    mesh = synth.merge_meshes([lo, hi])
    n = 3000
    o = np.stack([np.zeros(n), np.linspace(-40.0, 40.0, n), np.full(n, 60.0)], 1)
    d = np.tile([[0.0, 0.0, -1.0]], (n, 1)).astype(np.float32)
    sc = configs.scanner(0.03, 19, n_bins=256, bin_ns=0.5)
    clean = orc.simulate(mesh, synth.Pulses(o, d), sc)
    noisy = orc.simulate(mesh, synth.Pulses(o, d), dict(sc, range_noise_m=0.05, noise_seed=5))
    two = clean.n_returns == 2
    assert two.mean() > 0.9
    D = noisy.ret_range - clean.ret_range
    assert abs(np.corrcoef(D[two, 0], D[two, 1])[0, 1]) < 4 / np.sqrt(two.sum())
    assert abs(D[two, 1].std() / 0.05 - 1.0) < 0.05


def test_noise_seeded_and_selectable(orc):
    mesh, pulses, sc, clean, noisy = _pairs(orc, 0.05, 77)
    again = orc.simulate(mesh, pulses, dict(sc, range_noise_m=0.05, noise_seed=77))
    assert np.array_equal(again.ret_range, noisy.ret_range)
    other = orc.simulate(mesh, pulses, dict(sc, range_noise_m=0.05, noise_seed=78))
    hit = clean.n_returns > 0
    assert not np.any(other.ret_range[hit, 0] == noisy.ret_range[hit, 0])
    # a pulse's errors depend on its index, not on which pulses are simulated with it
    sel = np.array([5, 777, 4321, 9999])
    part = orc.simulate(mesh, pulses, dict(sc, range_noise_m=0.05, noise_seed=77), select=sel)
    assert np.array_equal(part.ret_range, noisy.ret_range[sel])
