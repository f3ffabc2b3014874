"""Shared helpers for the tests: small seeded segments and signals.

Signals are synthesised by the oracle (test infrastructure); the HIP path
never provides an input or an expected value."""
import math

import numpy as np

from oracle import method, model
from paper_1003_0844_amd import synth

DET = model.default_detector()
EPH = model.Ephemeris()


# For the coarse sampling of the small cases the band edge f_ref must be low
# enough that the Doppler excursion f_ref * v/c (v/c ~ 1e-4) stays well inside
# the band 1/(2 dt); otherwise the sampled signal aliases, which no real
# narrow-band data does.
SMALL_F_REF = 20.0


def small_segment(days=1, dt=26.0, seed=7, sigma=1.0, signal=None, noise=True,
                  mask=None, nfft=0, f_ref=None, t0=0.0, eph=EPH):
    """Whole-sidereal-day segment of white noise (sigma) plus an optional
    injected signal (dict as produced by synth.signal_params)."""
    if f_ref is None:
        f_ref = SMALL_F_REF if dt >= 10.0 else synth.F_REF
    n = int(round(days * synth.SIDEREAL_DAY / dt))
    g = synth.rng(seed)
    x = synth.white_noise(g, n, sigma) if noise else np.zeros(n)
    if signal is not None:
        x = x + model.injection(n, dt, t0, signal, f_ref, sigma * sigma, DET, eph, mask)
    return method.Segment(x=x, dt=dt, n_days=days, t0=t0, mask=mask, f_ref=f_ref,
                          sigma2=sigma * sigma, nfft=nfft)


def one_signal(seed, band, snr=10.0, f=None, fdot=(-1e-9, 0.0)):
    """One random signal with its frequency in the middle half of the band."""
    g = synth.rng(seed)
    p = synth.signal_params(g, 1, band, snr=(snr, snr), fdot=fdot, f=f)[0]
    if f is None:
        p["f"] = band * (0.25 + 0.5 * (p["f"] / band - 0.05) / 0.9)
    return p


def rel_err(got, ref):
    """max |got - ref| / max(|ref|, 1): the error metric for F."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.max(np.abs(got - ref) / np.maximum(np.abs(ref), 1.0)))


def deg(x):
    return math.radians(x)


def inversion_tolerances(e_amp, h0, cosi):
    """Bounds on the errors of h0 (relative) and of cos(iota) that follow from
    an error of at most e_amp in each of the four amplitudes A1..A4, through
    the inversion z1 = A1 + i A2, z2 = A4 - i A3, m+- = |z1 +- z2| =
    h0 (1 +- cos iota)^2 / 2, h0 = (m+ + m-)/2 + sqrt(m+ m-), h0 cos iota =
    (m+ - m-)/2 (Eqs. ampone, h0iota).  |dz1|, |dz2| <= sqrt(2) e_amp, so
    |dm+-| <= E = 2 sqrt(2) e_amp; the first term of h0 moves by at most E, the
    square root (increasing in both factors) by at most its change with both
    factors moved by E the same way; |d(h0 cos iota)| <= E.  The bound grows
    like 1 / (1 - |cos iota|): near circular polarisation m- is small and its
    square root is ill-conditioned."""
    E = 2.0 * math.sqrt(2.0) * e_amp
    big = h0 * (1.0 + abs(cosi)) ** 2 / 2.0
    small = h0 * (1.0 - abs(cosi)) ** 2 / 2.0
    root = math.sqrt(big * small)
    d_root = max(math.sqrt((big + E) * (small + E)) - root,
                 root - math.sqrt(max(big - E, 0.0) * max(small - E, 0.0)))
    d_h0 = E + d_root
    d_cosi = (E + abs(cosi) * d_h0) / max(h0 - d_h0, 1e-300)
    return d_h0 / h0, d_cosi
