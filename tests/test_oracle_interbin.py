"""Pins of the interbinning of Sec. VI B, Eq. (intbin):
X(k + 1/2) ~ [X(k+1) - X(k)] / sqrt(2)."""
import json
import math
import os

import numpy as np

from oracle import method, sums
from paper_1003_0844_amd import synth
from tests.common import DET, EPH

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def _best_amplitude(n, offset, ib=method.interbin):
    # a unit complex tone offset (in bins) above Fourier bin q of an unpadded
    # N-point DFT: the largest amplitude among X(q), X(q+1) and the interbinned
    # value between them, relative to the matched amplitude N
    q = 40
    j = np.arange(n)
    z = np.exp(2j * math.pi * (q + offset) * j / n)
    X = sums.dft_bins(z, n, np.array([q, q + 1]))
    return max(abs(X[0]), abs(X[1]), abs(ib(X[0], X[1]))) / n


def test_worst_loss_with_interbinning_is_the_papers():
    n = 2048
    offs = np.linspace(0.0, 1.0, 201)
    best = np.array([_best_amplitude(n, d) for d in offs])
    loss = 1.0 - best.min()
    g = GOLD["interbinning_max_loss"]
    assert abs(loss - g["value"]) < g["tol"], loss
    # the worst offsets sit about 0.29 bin from a Fourier frequency (symmetric),
    # and half way between bins interbinning recovers 2 sqrt(2)/pi of the amplitude
    worst = offs[np.argmin(best)]
    assert min(abs(worst - 0.293), abs(worst - 0.707)) < 0.02, worst
    assert abs(_best_amplitude(n, 0.5) - 2 * math.sqrt(2) / math.pi) < 1e-3
    # a sum instead of the difference, or no interbinning, miss the paper's number
    bad = [_best_amplitude(n, d, ib=lambda a, b: (a + b) / math.sqrt(2)) for d in offs]
    assert abs(1.0 - min(bad) - g["value"]) > 0.1
    assert abs((1 - 2 / math.pi) - g["value"]) > 0.2  # no interbinning: 36.3 %


def test_interbinned_noise_has_the_bin_variance():
    # for white noise and an unpadded DFT the bins are independent with equal
    # variance; the 1/sqrt(2) keeps that variance half way between them
    g = synth.rng(71)
    n = 4096
    X = np.fft.fft(g.normal(size=(64, n)) + 1j * g.normal(size=(64, n)), axis=1)
    Xh = method.interbin(X[:, :-1], X[:, 1:])
    ratio = np.mean(np.abs(Xh[:, ::2]) ** 2) / np.mean(np.abs(X) ** 2)
    assert abs(ratio - 1.0) < 0.02, ratio
    # without the 1/sqrt(2) the variance doubles
    assert abs(2.0 * ratio - 1.0) > 0.9


def _unpadded_segment(seed, signal=None):
    # 4096 samples over one sidereal day: nfft = N, no zero padding
    from tests.common import small_segment
    dt = synth.SIDEREAL_DAY / 4096
    return small_segment(days=1, dt=dt, seed=seed, signal=signal, nfft=4096)


def test_interbinned_F_on_noise_is_chi2_4():
    # 2F half way between independent bins follows the same chi-square law
    # with 4 degrees of freedom (mean 4, variance 8); every other half bin
    twoF = []
    for s in range(6):
        seg = _unpadded_segment(300 + s)
        al, de = synth.sky_uniform(synth.rng(400 + s), 1)
        _, Fh = method.fstat_bins_interbinned(seg, 0.0, al[0], de[0], DET, EPH, method.NEAREST,
                                              k=np.arange(0, 2047, 2), dft="fft")
        twoF.append(2.0 * Fh)
    v = np.concatenate(twoF)
    assert abs(v.mean() - 4.0) < 0.25, v.mean()
    assert abs(v.var() - 8.0) < 1.5, v.var()


def test_integer_bins_are_fstat_bins():
    seg = _unpadded_segment(310)
    k = np.array([0, 5, 100, 2046])
    F0, _ = method.fstat_bins_interbinned(seg, -3e-10, 1.0, 0.4, DET, EPH, method.LINEAR_UP2, k=k)
    ref = method.fstat_bins(seg, -3e-10, 1.0, 0.4, DET, EPH, method.LINEAR_UP2, k=k)
    assert np.array_equal(F0, ref)
