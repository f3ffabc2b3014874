"""Pins of the oracle's barycentric resampling (Sec. VI A, Eqs. Bt, ia) and its
DFT stage (Sec. VI B, Eq. DFT)."""
import json
import math
import os

import numpy as np
import pytest
from scipy.interpolate import CubicSpline

from oracle import method, model, sums
from tests.common import DET, EPH, small_segment, one_signal

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def test_ssb_time_inversion_residual():
    seg = small_segment(days=2, dt=13.0)
    for al, de in [(0.1, 0.2), (3.0, -1.2), (5.5, 0.9)]:
        tb0, t = method.ssb_times(seg, al, de, DET, EPH)
        resid = t + model.roemer_delay(seg.t0 + t, al, de, DET, EPH) - (tb0 + np.arange(seg.n) * seg.dt)
        assert np.max(np.abs(resid)) < 1e-9
        assert abs(tb0 - model.roemer_delay(0.0, al, de, DET, EPH)) == 0.0


@pytest.mark.parametrize("n", [1, 2, 7, 64, 301, 1000])
def test_upsample_keeps_samples(n):
    x = np.random.default_rng(n).normal(size=n)
    y = method.fourier_upsample(x)
    assert y.size == 2 * n
    assert np.max(np.abs(y[0::2] - x)) < 1e-13 * max(1.0, np.max(np.abs(x)))


@pytest.mark.parametrize("n", [64, 301, 1000])
def test_upsample_reproduces_fourier_tones(n):
    # a tone at a Fourier frequency of the N-grid is band-limited: its 2x
    # upsampled series is the same tone on the 2N-grid
    m = np.arange(n)
    for q in (0, 1, 5, n // 3, (n - 1) // 2):
        x = np.cos(2 * math.pi * q * m / n + 0.7)
        y = method.fourier_upsample(x)
        ref = np.cos(2 * math.pi * q * (np.arange(2 * n) / 2) / n + 0.7)
        assert np.max(np.abs(y - ref)) < 1e-12


def test_upsample_against_trigonometric_interpolant_brute_force():
    # y(s) = (1/N) sum_k X_k e^{2 pi i k s/N} with k in the symmetric range and
    # the Nyquist term (even N) entering as X_{N/2} cos(pi s), written out term
    # by term for tiny N
    for n in (6, 7, 10):
        x = np.random.default_rng(n).normal(size=n)
        X = np.array([sum(x[l] * np.exp(-2j * math.pi * l * k / n) for l in range(n)) for k in range(n)])
        s = np.arange(2 * n) / 2.0
        y = np.zeros(2 * n)
        for k in range(n):
            kk = k if k < n / 2 else k - n
            if n % 2 == 0 and k == n // 2:
                y += (X[k] * np.cos(math.pi * s)).real / n
            else:
                y += (X[k] * np.exp(2j * math.pi * kk * s / n)).real / n
        assert np.max(np.abs(method.fourier_upsample(x) - y)) < 1e-12


def test_periodic_spline_matches_library():
    y = np.random.default_rng(5).normal(size=400)
    M = method.periodic_spline_m(y)
    p = y.size
    cs = CubicSpline(np.arange(p + 1), np.append(y, y[0]), bc_type="periodic")
    assert np.max(np.abs(M - cs(np.arange(p), 2))) < 1e-10
    # the oracle's evaluation formula against the library's evaluation
    seg = small_segment(days=1, dt=26.0)
    yy, MM = method._upsampled(seg, method.CUBIC_UP2)
    cs = CubicSpline(np.arange(yy.size + 1), np.append(yy, yy[0]), bc_type="periodic")
    u = np.random.default_rng(9).uniform(0, seg.n - 1, 500)
    xr, dxdu = method.interpolate(seg, u, method.CUBIC_UP2)
    assert np.max(np.abs(xr - cs(2 * u))) < 1e-10
    assert np.max(np.abs(dxdu - 2 * cs(2 * u, 1))) < 1e-9


def test_linear_and_nearest_interpolation():
    seg = small_segment(days=1, dt=26.0)
    y, _ = method._upsampled(seg, method.LINEAR_UP2)
    u = np.array([0.0, 0.25, 0.5, 10.75, seg.n - 1.0, -1e-5, seg.n - 1 + 1e-5, -1e-9, seg.n - 1 + 1e-9])
    xr, _ = method.interpolate(seg, u, method.LINEAR_UP2)
    assert xr[0] == y[0] and xr[4] == y[2 * seg.n - 2]
    assert abs(xr[0] - seg.x[0]) < 1e-13 and abs(xr[4] - seg.x[-1]) < 1e-13
    assert abs(xr[1] - 0.5 * (y[0] + y[1])) < 1e-15
    assert xr[2] == y[1]
    assert abs(xr[3] - 0.5 * (y[21] + y[22])) < 1e-15
    assert xr[5] == 0.0 and xr[6] == 0.0              # outside the span
    assert xr[7] == y[0] and xr[8] == y[2 * seg.n - 2]  # within the margin: clamped
    xn, _ = method.interpolate(seg, np.array([0.49, 0.5, 1.49, seg.n - 1.0]), method.NEAREST)
    assert list(xn) == [seg.x[0], seg.x[1], seg.x[1], seg.x[-1]]


def test_no_ephemeris_makes_method_exact():
    # with the detector at the SSB the barycentric time is the detector time:
    # the resampled series is the data itself for every interpolation, and the
    # method equals direct summation
    eph0 = model.Ephemeris(orbit_radius=0.0)
    det0 = model.Detector(lat=DET.lat, lon=DET.lon, gamma=DET.gamma, radius=0.0)
    sig = one_signal(11, band=1 / 52.0)
    seg = small_segment(days=1, dt=26.0, signal=sig, eph=eph0, nfft=8192)
    k = np.arange(0, 4096, 37)
    for mode in (method.NEAREST, method.LINEAR_UP2, method.CUBIC_UP2):
        r = method.resampled(seg, sig["alpha"], sig["delta"], det0, eph0, mode)
        assert np.max(np.abs(r["t"] - np.arange(seg.n) * seg.dt)) == 0.0
        assert np.max(np.abs(r["xr"] - seg.x)) < 1e-12
        Fm = method.fstat_bins(seg, sig["fdot"], sig["alpha"], sig["delta"], det0, eph0, mode, k=k)
        Fe = method.fstat_exact(seg, k / (8192 * seg.dt), sig["fdot"], sig["alpha"], sig["delta"], det0, eph0)
        assert np.max(np.abs(Fm - Fe) / np.maximum(Fe, 1)) < 1e-11


# --------------------------------------------------------------------------
# DFT stage
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n,nfft", [(1, 1), (5, 8), (100, 256), (1000, 1000), (3000, 4096), (4096, 4096)])
def test_direct_dft_matches_library_fft(n, nfft):
    g = np.random.default_rng(n)
    z = g.normal(size=n) + 1j * g.normal(size=n)
    k = np.arange(-3, nfft + 3)
    got = sums.dft_bins(z, nfft, k)
    ref = np.fft.fft(z, nfft)[k % nfft]
    assert np.max(np.abs(got - ref)) < 1e-12 * max(1.0, np.sqrt(n))


def test_continuous_frequency_sum_matches_bins():
    g = np.random.default_rng(2)
    z = g.normal(size=700) + 1j * g.normal(size=700)
    dt, nfft = 0.5, 2048
    k = np.array([0, 1, 17, 1023])
    assert np.max(np.abs(sums.dft_freqs(z, dt, k / (nfft * dt)) - sums.dft_bins(z, nfft, k))) < 1e-11


def _tone_loss(n, nfft, offset_bins):
    # amplitude at the nearest DFT bin of a unit complex tone lying
    # offset_bins (in units of 1/N) away from a Fourier frequency of the N-grid
    q = 40
    j = np.arange(n)
    z = np.exp(2j * math.pi * (q + offset_bins) * j / n)
    p = nfft // n
    k = np.arange(q * p - 2, q * p + 3)
    amp = np.abs(sums.dft_bins(z, nfft, k))
    return 1.0 - np.max(amp) / n


def test_scalloping_losses_of_the_paper():
    # Sec. VI B: worst loss 36.3% at a half bin; 9.97% with N zeros of padding
    n = 2048
    loss = _tone_loss(n, n, 0.5)
    g = GOLD["scalloping_loss_half_bin"]
    assert abs(loss - g["value"]) < g["tol"]
    loss2 = _tone_loss(n, 2 * n, 0.25)
    g = GOLD["scalloping_loss_2x_padding"]
    assert abs(loss2 - g["value"]) < g["tol"]
    # and the worst case really is there
    assert _tone_loss(n, 2 * n, 0.2) < loss2 and _tone_loss(n, 2 * n, 0.3) < loss2


def test_mc_padding_worked_number():
    g = GOLD["mc_points_and_padding"]
    assert g["n_data"] + g["n_zeros"] == g["n_fft"] == 1 << 15
    # the paper pads to the next power of two (about 1.9 N there); an
    # explicit FFT length overrides the default nextpow2(2N)
    seg = method.Segment(x=np.zeros(g["n_data"]), dt=10.0, n_days=2, nfft=g["n_fft"])
    assert seg.fft_len == 1 << int(math.ceil(math.log2(g["n_data"])))
    assert method.Segment(x=np.zeros(g["n_data"]), dt=10.0, n_days=2).fft_len == 2 * g["n_fft"]
