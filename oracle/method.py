"""The F-statistic, exact and by the resampling method, in FP64 (oracle; test
infrastructure only -- see the package docstring).

Paper: Sec. III A (Eqs. OS, Fab: the F-statistic), Sec. VI A (Eqs. pham, phas,
Far, Bt, ia: barycentric resampling; nearest-neighbour and two-step Fourier +
spline interpolation), Sec. VI B (Eq. DFT).

Readings of points the paper leaves open:

R-norm   Normalisation.  For white noise of per-sample variance sigma^2 the
         one-sided PSD is S0 = 2 sigma^2 dt and the integrals of Eqs. (Fab) are
         dt times sums, so Eq. (OS) becomes
             F = |S_a|^2/(sigma^2 A) + |S_b|^2/(sigma^2 B),
         with S_a = sum m x a e^{-i phi}, A = sum m a^2, B = sum m b^2 over the
         detector samples (m = gap mask).  Where a gap mask breaks the
         whole-sidereal-day assumption that makes <ab> vanish (Sec. III A), the
         same maximum-likelihood projection with C = sum m a b is used:
             F = (B|S_a|^2 + A|S_b|^2 - 2C Re(S_a S_b*)) / (sigma^2 (AB - C^2)),
         which equals the Eq. (OS) form exactly when C = 0.
R-band   The data are real, narrow-band, heterodyned: band-relative frequency f
         in [0, 1/(2 dt)), physical frequency f_ref + f.  omega_0 = 2 pi (f_ref+f)
         enters the Roemer term of Eq. (pha3).
R-grid   SSB time grid: t_b0 = t_b(0) = phi_m(0), t_b_j = t_b0 + j dt,
         j = 0..N-1 (the same number of points as the data, Sec. VI A).
         The resampled value is 0 where t(t_b) falls outside [0, (N-1) dt],
         with a margin of 1e-6 samples (clamped), because t_0 = 0 exactly and
         its rounding must not decide whether the first sample counts.
R-interp Only x is interpolated; a(t), b(t) and the demodulation phase are
         evaluated exactly at t(t_b_j) (Eq. ia read literally).  Nearest
         neighbour takes x[floor(u + 1/2)], u = t/dt.  The two-step method
         upsamples x by 2 by zero-padding its DFT (the Nyquist bin of an even N
         split equally between +N/2 and -N/2), then interpolates the 2N-point
         series by a degree-1 spline (LINEAR_UP2) or by the periodic cubic
         spline (CUBIC_UP2; the Fourier interpolant is periodic with period 2N
         samples, so the periodic end condition is the consistent one).
R-jac    The Jacobian dt/dt_b is dropped, as in Eq. (ia).
R-f0     The frequency term e^{-2 pi i f t_b0} common to S_a and S_b is
         dropped; it does not change F.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import model, sums

NEAREST, LINEAR_UP2, CUBIC_UP2 = 0, 1, 2


@dataclass
class Segment:
    """One data segment (mirrors the fields of the C-ABI segment description)."""
    x: np.ndarray
    dt: float
    n_days: int
    t0: float = 0.0
    mask: Optional[np.ndarray] = None
    f_ref: float = 435.1875
    sigma2: float = 1.0
    nfft: int = 0
    _cache: dict = field(default_factory=dict, repr=False)

    @property
    def n(self) -> int:
        return int(np.asarray(self.x).size)

    @property
    def m(self) -> np.ndarray:
        return (np.ones(self.n) if self.mask is None
                else (np.asarray(self.mask) != 0).astype(np.float64))

    @property
    def xm(self) -> np.ndarray:
        """Data with gaps zeroed."""
        return np.asarray(self.x, dtype=np.float64) * self.m

    @property
    def fft_len(self) -> int:
        if self.nfft:
            return int(self.nfft)
        return 1 << int(math.ceil(math.log2(2 * self.n)))

    def noise_var(self) -> float:
        """sigma^2: the caller's value, or (if <= 0) the unbiased sample
        variance of the samples outside gaps."""
        if self.sigma2 > 0:
            return float(self.sigma2)
        v = np.asarray(self.x, dtype=np.float64)[self.m != 0]
        return float(np.sum((v - v.mean()) ** 2) / (v.size - 1))


# --------------------------------------------------------------------------
# Barycentric time (Eq. Bt) and its inversion
# --------------------------------------------------------------------------
def ssb_times(seg: Segment, alpha, delta, det, eph, tol=1e-12, max_iter=60):
    """Returns (t_b0, t) with t_j the detector time whose barycentric time
    t + phi_m(t) equals t_b0 + j dt.  Fixed-point iteration
    t <- t_b - phi_m(t), a contraction because |phi_m'| << 1."""
    j = np.arange(seg.n, dtype=np.float64)
    tb0 = float(model.roemer_delay(seg.t0, alpha, delta, det, eph))
    tb = tb0 + j * seg.dt
    t = j * seg.dt
    for _ in range(max_iter):
        t_new = tb - model.roemer_delay(seg.t0 + t, alpha, delta, det, eph)
        done = np.max(np.abs(t_new - t)) < tol
        t = t_new
        if done:
            break
    return tb0, t


def ssb_positions(seg: Segment, alpha, delta, det, eph):
    """Fractional sample positions u_j = t_j / dt of the barycentric grid, in
    extended precision (numpy longdouble).  The FP64 solution of ssb_times is
    refined by one more fixed-point step t <- t_b - phi_m(t) carried out in
    extended precision: the step contracts the error by |phi_m'| ~ 1e-4, so
    the result is exact to extended-precision rounding, whereas t_j / dt in
    FP64 carries the rounding of an absolute time (~1e-10 s at 6 days), which
    moves every interpolation weight by ~5e-10."""
    L = np.longdouble
    _, t = ssb_times(seg, alpha, delta, det, eph)
    T0 = L(seg.t0)
    tb = model.roemer_delay_ext(T0, alpha, delta, det, eph) + np.arange(seg.n, dtype=L) * L(seg.dt)
    tx = tb - model.roemer_delay_ext(T0 + t.astype(L), alpha, delta, det, eph)
    return tx / L(seg.dt)


# --------------------------------------------------------------------------
# Interpolation (Sec. VI A)
# --------------------------------------------------------------------------
def fourier_upsample(x):
    """2x upsampling by zero-padding the DFT: returns y with 2N points,
    y[2m] = x[m] (Sec. VI A, first step of the two-step method)."""
    x = np.asarray(x, dtype=np.float64)
    n = x.size
    X = np.fft.fft(x)
    Y = np.zeros(2 * n, dtype=np.complex128)
    h = n // 2
    if n % 2 == 0:
        Y[:h] = X[:h]
        Y[h] = 0.5 * X[h]
        Y[2 * n - h] = 0.5 * X[h]
        Y[2 * n - h + 1:] = X[h + 1:]
    else:
        Y[:h + 1] = X[:h + 1]
        Y[2 * n - h:] = X[h + 1:]
    return 2.0 * np.fft.ifft(Y).real


def periodic_spline_m(y):
    """Second derivatives M of the periodic cubic spline through (i, y_i),
    i = 0..P-1 with period P: the cyclic system
        M_{i-1} + 4 M_i + M_{i+1} = 6 (y_{i-1} - 2 y_i + y_{i+1})."""
    y = np.asarray(y, dtype=np.float64)
    p = y.size
    i = np.arange(p)
    rows = np.concatenate([i, i, i])
    cols = np.concatenate([i, (i - 1) % p, (i + 1) % p])
    vals = np.concatenate([np.full(p, 4.0), np.ones(p), np.ones(p)])
    A = sp.csc_matrix((vals, (rows, cols)), shape=(p, p))
    rhs = 6.0 * (np.roll(y, 1) - 2.0 * y + np.roll(y, -1))
    return spla.spsolve(A, rhs)


def _upsampled(seg: Segment, mode):
    key = ("up", mode)
    if key not in seg._cache:
        y = fourier_upsample(seg.xm)
        M = periodic_spline_m(y) if mode == CUBIC_UP2 else None
        seg._cache[key] = (y, M)
    return seg._cache[key]


SPAN_EPS = 1e-6  # samples


def interpolate(seg: Segment, u, mode):
    """x at fractional sample positions u (0 outside [0, N-1]), and dx/du.

    The first barycentric sample maps exactly onto the first data sample
    (t_b0 = phi_m(0) gives t_0 = 0), so the span test must not depend on the
    last bit of t: positions within SPAN_EPS samples of the span count as
    inside and are clamped onto it."""
    u = np.asarray(u)
    if u.dtype != np.longdouble:
        u = u.astype(np.float64)
    n = seg.n
    valid = (u >= -SPAN_EPS) & (u <= n - 1 + SPAN_EPS)
    uu = np.where(valid, np.clip(u, 0.0, n - 1.0), 0.0)
    xr = np.zeros(u.shape)
    dxdu = np.zeros(u.shape)
    if mode == NEAREST:
        idx = np.floor(uu + 0.5).astype(np.int64)
        xr = np.where(valid, seg.xm[np.minimum(idx, n - 1)], 0.0)
        return xr, dxdu
    y, M = _upsampled(seg, mode)
    v = 2 * uu
    i = np.minimum(np.floor(v).astype(np.int64), 2 * n - 2)
    s = (v - i).astype(np.float64)
    y0, y1 = y[i], y[i + 1]
    if mode == LINEAR_UP2:
        val = (1.0 - s) * y0 + s * y1
        dv = y1 - y0
    elif mode == CUBIC_UP2:
        m0, m1 = M[i], M[i + 1]
        r = 1.0 - s
        val = r * y0 + s * y1 + ((r ** 3 - r) * m0 + (s ** 3 - s) * m1) / 6.0
        dv = y1 - y0 + ((1.0 - 3.0 * r * r) * m0 + (3.0 * s * s - 1.0) * m1) / 6.0
    else:
        raise ValueError("unknown interpolation mode %r" % (mode,))
    xr = np.where(valid, val, 0.0)
    dxdu = np.where(valid, 2.0 * dv, 0.0)
    return xr, dxdu


# --------------------------------------------------------------------------
# The resampled, demodulated series (Eq. ia) and the F-statistic
# --------------------------------------------------------------------------
def resampled(seg: Segment, alpha, delta, det, eph, mode):
    """Everything the method needs on the uniform SSB grid for one sky point."""
    tb0, t = ssb_times(seg, alpha, delta, det, eph)
    u = ssb_positions(seg, alpha, delta, det, eph)
    xr, dxdu = interpolate(seg, u, mode)
    a, b = model.amplitude_modulation(seg.t0 + t, alpha, delta, det, eph)
    pm = model.roemer_delay(seg.t0 + t, alpha, delta, det, eph)
    return dict(tb0=tb0, t=t, u=u, xr=xr, dxdu=dxdu, a=a, b=b, pm=pm)


def demod_cycles(t, T0, alpha, delta, f_ref, fdot, det, eph):
    """Frequency-independent part of the phase on the resampled grid, turns,
    reduced to [-1/2, 1/2]:
        f_ref (phi_m(t) - phi_m(0)) + fdot (t^2/2 + phi_m(t) t)
    (Eq. phas plus the f_ref part of omega_0 phi_m that the band-relative FFT
    does not absorb; the constant f_ref phi_m(0) is a phase common to S_a and
    S_b and is left out, reading R-f0).  Evaluated in extended precision: the
    f_ref phi_m term alone reaches ~2e5 turns."""
    L = np.longdouble
    tl = np.asarray(t, dtype=L)
    pm = model.roemer_delay_ext(L(T0) + tl, alpha, delta, det, eph)
    pm0 = model.roemer_delay_ext(L(T0), alpha, delta, det, eph)
    cyc = L(f_ref) * (pm - pm0) + L(fdot) * (tl * tl / 2 + pm * tl)
    return (cyc - np.round(cyc)).astype(np.float64)


def demodulated(seg: Segment, fdot, alpha, delta, det, eph, mode):
    """z_a, z_b on the SSB grid: x(t(t_b)) a(t(t_b)) e^{-i phi_s(t(t_b))}."""
    r = resampled(seg, alpha, delta, det, eph, mode)
    cyc = demod_cycles(r["t"], seg.t0, alpha, delta, seg.f_ref, fdot, det, eph)
    e = np.exp(-2j * math.pi * cyc)
    return r["xr"] * r["a"] * e, r["xr"] * r["b"] * e


def abc(seg: Segment, alpha, delta, det, eph):
    """A, B, C = sums of m a^2, m b^2, m a b over the detector samples."""
    t = np.arange(seg.n, dtype=np.float64) * seg.dt
    a, b = model.amplitude_modulation(seg.t0 + t, alpha, delta, det, eph)
    m = seg.m
    return float(np.sum(m * a * a)), float(np.sum(m * b * b)), float(np.sum(m * a * b))


def combine(Sa, Sb, A, B, C, sigma2):
    """F from the two correlations (reading R-norm; Eq. OS when C = 0)."""
    Sa = np.asarray(Sa)
    Sb = np.asarray(Sb)
    num = B * np.abs(Sa) ** 2 + A * np.abs(Sb) ** 2 - 2.0 * C * np.real(Sa * np.conj(Sb))
    return num / (sigma2 * (A * B - C * C))


def shift_bins(z, nfft, bin_offset):
    """z_j e^{-2 pi i off j / nfft}: its DFT at bin k is the transform of z at
    the frequency (k + off) / (nfft dt), so a line of Fourier bins can start a
    fraction of a bin off zero (the frequency lines of the lattice grid of
    Sec. IV, Eq. avec)."""
    if bin_offset == 0.0:
        return z
    j = np.arange(len(z), dtype=np.float64)
    cyc = float(bin_offset) * j / nfft
    return z * np.exp(-2j * math.pi * (cyc - np.round(cyc)))


def fstat_bins(seg: Segment, fdot, alpha, delta, det, eph, mode, k=None, dft="direct", bin_offset=0.0):
    """F on Fourier bins k (default: all of [0, nfft/2)) by the resampling
    method, at the frequencies (k + bin_offset) / (nfft dt).  dft='direct' sums
    the DFT term by term; dft='fft' uses numpy's FP64 FFT of the zero-padded
    series for the same sums."""
    nfft = seg.fft_len
    if k is None:
        k = np.arange(nfft // 2, dtype=np.int64)
    k = np.asarray(k, dtype=np.int64)
    za, zb = demodulated(seg, fdot, alpha, delta, det, eph, mode)
    za, zb = shift_bins(za, nfft, bin_offset), shift_bins(zb, nfft, bin_offset)
    if dft == "direct":
        Sa, Sb = sums.dft_bins(za, nfft, k), sums.dft_bins(zb, nfft, k)
    elif dft == "fft":
        Sa, Sb = np.fft.fft(za, nfft)[k], np.fft.fft(zb, nfft)[k]
    else:
        raise ValueError(dft)
    A, B, C = abc(seg, alpha, delta, det, eph)
    return combine(Sa, Sb, A, B, C, seg.noise_var())


def interbin(S_k, S_k1):
    """Eq. (intbin): the DFT component half way between the Fourier bins k and
    k + 1, approximated by (X(k+1) - X(k)) / sqrt(2) (interbinning, Sec. VI B)."""
    return (np.asarray(S_k1) - np.asarray(S_k)) / math.sqrt(2.0)


def fstat_bins_interbinned(seg: Segment, fdot, alpha, delta, det, eph, mode, k=None, dft="direct",
                           bin_offset=0.0):
    """F at the Fourier bins k and at the half bins k + 1/2: Eq. (intbin)
    applied to S_a and S_b, then the F combination.  Needs k + 1 <= nfft/2.
    Bins start bin_offset off zero as in fstat_bins.  Returns (F at k, F at
    k + 1/2)."""
    nfft = seg.fft_len
    if k is None:
        k = np.arange(nfft // 2, dtype=np.int64)
    k = np.asarray(k, dtype=np.int64)
    if k.size and (k.min() < 0 or k.max() + 1 > nfft // 2):
        raise ValueError("bins k and k + 1 must lie in [0, nfft/2]")
    kk = np.union1d(k, k + 1)
    za, zb = demodulated(seg, fdot, alpha, delta, det, eph, mode)
    za, zb = shift_bins(za, nfft, bin_offset), shift_bins(zb, nfft, bin_offset)
    if dft == "direct":
        Sa, Sb = sums.dft_bins(za, nfft, kk), sums.dft_bins(zb, nfft, kk)
    elif dft == "fft":
        Sa, Sb = np.fft.fft(za, nfft)[kk], np.fft.fft(zb, nfft)[kk]
    else:
        raise ValueError(dft)
    i0, i1 = np.searchsorted(kk, k), np.searchsorted(kk, k + 1)
    A, B, C = abc(seg, alpha, delta, det, eph)
    s2 = seg.noise_var()
    F0 = combine(Sa[i0], Sb[i0], A, B, C, s2)
    Fh = combine(interbin(Sa[i0], Sa[i1]), interbin(Sb[i0], Sb[i1]), A, B, C, s2)
    return F0, Fh


# --------------------------------------------------------------------------
# Amplitude parameters (Sec. III, Eqs. ampone, amle0, h0iota)
# --------------------------------------------------------------------------
def amplitudes_from_parameters(h0, cosi, psi, phi0):
    """The four amplitudes of Eq. (ampone) from h0, cos(iota), psi, phi0, with
    h0+ = h0 (1 + cos^2 iota)/2 and h0x = h0 cos(iota) (Eq. h0iota)."""
    hp, hx = 0.5 * h0 * (1.0 + cosi * cosi), h0 * cosi
    c2, s2, cp, sp_ = math.cos(2 * psi), math.sin(2 * psi), math.cos(phi0), math.sin(phi0)
    return np.array([hp * c2 * cp - hx * s2 * sp_,
                     hp * s2 * cp + hx * c2 * sp_,
                     -hp * c2 * sp_ - hx * s2 * cp,
                     -hp * s2 * sp_ + hx * c2 * cp])


def parameters_from_amplitudes(Ab):
    """Inversion of Eq. (ampone), then of Eq. (h0iota).  With
    z1 = Ab1 + i Ab2 and z2 = Ab4 - i Ab3, Eq. (ampone) reads
    z1 + z2 = (h0+ + h0x) e^{i(2 psi + phi0)} and
    z1 - z2 = (h0+ - h0x) e^{i(2 psi - phi0)}, so h0+ +- h0x = |z1 +- z2| (the
    unique solution of the paper's A = h0+^2 + h0x^2, D = h0+ h0x with h0+ > 0)
    and the two arguments give psi and phi0 with their quadrants (the paper's
    tan(2 phi0), tan(4 psi) relations fix them only modulo pi/2 and pi/4).
    Then h0 = h0+ + sqrt(h0+^2 - h0x^2) and cos iota = h0x / h0.
    Convention: psi in [0, pi/2), phi0 in [0, 2 pi) ((psi + pi/2, phi0 + pi)
    gives the same amplitudes); for cos iota = +-1 only 2 psi +- phi0 is
    determined and the argument of the vanishing combination is taken as 0.
    Returns (h0, cos iota, psi, phi0)."""
    a1, a2, a3, a4 = (float(v) for v in Ab)
    zp = complex(a1 + a4, a2 - a3)
    zm = complex(a1 - a4, a2 + a3)
    sp_, sm = abs(zp), abs(zm)
    hp, hx = 0.5 * (sp_ + sm), 0.5 * (sp_ - sm)
    h0 = hp + math.sqrt(sp_ * sm)
    cosi = hx / h0 if h0 > 0 else 0.0
    ap = math.atan2(zp.imag, zp.real) if sp_ > 0 else 0.0
    am = math.atan2(zm.imag, zm.real) if sm > 0 else 0.0
    psi = 0.25 * (ap + am)
    phi0 = 0.5 * (ap - am)
    shift = math.floor(psi / (math.pi / 2))
    psi -= shift * (math.pi / 2)
    phi0 -= shift * math.pi
    return h0, cosi, psi, phi0 % (2 * math.pi)


def amplitude_estimates(Sa, Sb, A, B, C, theta0, sin_zeta=1.0):
    """ML estimators of the amplitudes (Eq. amle0) from the correlations S_a,
    S_b of the resampling method.  theta0 restores the phase common to S_a and
    S_b that the method leaves out (reading R-f0): S_true = S e^{-i theta0}.
    With h1..h4 = a cos, b cos, a sin, b sin of the phase, the normal equations
    are [A C; C B] (A1, A2) = 2 Re(S_a, S_b) and the same for (A3, A4) with
    -Im; C = 0 gives Eq. (amle0).  Returns the amplitudes divided by sin(zeta)."""
    rot = complex(math.cos(theta0), -math.sin(theta0))
    sa, sb = complex(Sa) * rot, complex(Sb) * rot
    det_ = A * B - C * C
    inv = np.array([[B, -C], [-C, A]]) / det_
    a12 = 2.0 * inv @ np.array([sa.real, sb.real])
    a34 = 2.0 * inv @ np.array([-sa.imag, -sb.imag])
    return np.array([a12[0], a12[1], a34[0], a34[1]]) / sin_zeta


def estimate_parameters(seg: Segment, params, det, eph, mode):
    """Amplitude estimates and (h0, cos iota, psi, phi0) at continuous
    (f, fdot, alpha, delta) by the resampling method (the second step of the
    ML estimation, Sec. III)."""
    f, fdot, alpha, delta = (float(v) for v in params)
    n, dt = seg.n, seg.dt
    j = np.arange(n, dtype=np.float64)
    _, t = ssb_times(seg, alpha, delta, det, eph)
    T = seg.t0 + t
    xr, _ = interpolate(seg, ssb_positions(seg, alpha, delta, det, eph), mode)
    a, b = model.amplitude_modulation(T, alpha, delta, det, eph)
    cyc = demod_cycles(t, seg.t0, alpha, delta, seg.f_ref, fdot, det, eph) + f * j * dt
    e = np.exp(-2j * math.pi * (cyc - np.round(cyc)))
    Sa, Sb = np.sum(xr * a * e), np.sum(xr * b * e)
    A, B, C = abc(seg, alpha, delta, det, eph)
    L = np.longdouble
    turns = (L(seg.f_ref) + L(f)) * model.roemer_delay_ext(L(seg.t0), alpha, delta, det, eph)
    theta0 = 2.0 * math.pi * float(turns - np.round(turns))
    Ab = amplitude_estimates(Sa, Sb, A, B, C, theta0, math.sin(det.zeta))
    return Ab, parameters_from_amplitudes(Ab)


# --------------------------------------------------------------------------
# Candidate selection and fine search (Secs. III B, VI C)
# --------------------------------------------------------------------------
def false_alarm_cell(F0):
    """Eq. (PF): probability that F exceeds F0 in one cell without a signal."""
    return (1.0 + F0) * math.exp(-F0)


def threshold(alpha, n_cells):
    """F0 with false-alarm probability alpha over n_cells cells: Eq. (FP)
    solved for F0 by bisection on Eq. (PF).  P_F = 1 - (1 - alpha)^(1/N_c) is
    formed as -expm1(log1p(-alpha)/N_c): the direct form cancels for small alpha
    and large N_c."""
    pf = -math.expm1(math.log1p(-alpha) / n_cells)
    lo, hi = 0.0, 1.0
    while false_alarm_cell(hi) > pf:
        hi *= 2.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if false_alarm_cell(mid) > pf:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def nelder_mead_max(fun, x0, scale, tol, max_evals):
    """Maximum of fun by the Nelder-Mead simplex method (Nelder & Mead 1965;
    reflection 1, expansion 2, contraction 1/2, shrink 1/2) on -fun in the
    coordinates u = (x - x0)/scale, from the simplex x0 + unit steps; stops
    when all vertices are within tol of the best one (max norm, in u) or after
    max_evals evaluations.  Returns (x, fun(x), evaluations)."""
    x0 = np.asarray(x0, dtype=np.float64)
    scale = np.asarray(scale, dtype=np.float64)
    dim = x0.size
    nev = [0]

    def g(u):
        nev[0] += 1
        return -fun(x0 + u * scale)

    V = [np.zeros(dim)] + [np.eye(dim)[i] for i in range(dim)]
    G = [g(v) for v in V]
    while nev[0] < max_evals:
        order = sorted(range(dim + 1), key=lambda i: G[i])
        V = [V[i] for i in order]
        G = [G[i] for i in order]
        if max(np.max(np.abs(v - V[0])) for v in V[1:]) < tol:
            break
        cen = np.mean(V[:-1], axis=0)
        xr = cen + (cen - V[-1])
        gr = g(xr)
        if gr < G[0]:
            xe = cen + 2.0 * (xr - cen)
            ge = g(xe)
            V[-1], G[-1] = (xe, ge) if ge < gr else (xr, gr)
        elif gr < G[-2]:
            V[-1], G[-1] = xr, gr
        else:
            if gr < G[-1]:
                xc = cen + 0.5 * (xr - cen)
                gc = g(xc)
                ok = gc <= gr
            else:
                xc = cen + 0.5 * (V[-1] - cen)
                gc = g(xc)
                ok = gc < G[-1]
            if ok:
                V[-1], G[-1] = xc, gc
            else:
                for i in range(1, dim + 1):
                    V[i] = V[0] + 0.5 * (V[i] - V[0])
                    G[i] = g(V[i])
    b = int(np.argmin(G))
    return x0 + V[b] * scale, -G[b], nev[0]


def fstat_exact(seg: Segment, f, fdot, alpha, delta, det, eph):
    """F by direct summation of Eqs. (Fab) on the detector samples, at the
    band-relative frequencies f (no resampling, no FFT)."""
    t = np.arange(seg.n, dtype=np.float64) * seg.dt
    pm = model.roemer_delay(seg.t0 + t, alpha, delta, det, eph)
    a, b = model.amplitude_modulation(seg.t0 + t, alpha, delta, det, eph)
    w = seg.xm
    tau = t + pm
    psi = seg.f_ref * pm + fdot * (0.5 * t * t + pm * t)
    Sa, Sb = sums.phase_sums(w * a, w * b, tau, psi, f)
    A, B, C = abc(seg, alpha, delta, det, eph)
    return combine(Sa, Sb, A, B, C, seg.noise_var())


# --------------------------------------------------------------------------
# Continuous frequency and the analytic gradient
# --------------------------------------------------------------------------
def _roemer_partials(T, alpha, delta, det, eph):
    """phi_m and its partials d/dalpha, d/ddelta, d/dT (seconds, s/rad, 1)."""
    xes, yes = model.earth_center(T, eph)
    xe, ye, ze = model.site_vector(T, det, eph)
    ang = eph.orbit_omega * np.asarray(T, dtype=np.float64) + eph.orbit_phase0
    th = model.sidereal_angle(T, det, eph)
    wr = 2.0 * math.pi / eph.sidereal_day
    dxes = -eph.orbit_radius * eph.orbit_omega * np.sin(ang)
    dyes = eph.orbit_radius * eph.orbit_omega * np.cos(ang)
    dxe = -det.radius * math.cos(det.lat) * wr * np.sin(th)
    dye = det.radius * math.cos(det.lat) * wr * np.cos(th)
    ca, sa = math.cos(alpha), math.sin(alpha)
    cd, sd = math.cos(delta), math.sin(delta)
    ce, se = math.cos(eph.obliquity), math.sin(eph.obliquity)
    c = model.C_LIGHT
    pm = (ca * cd * (xes + xe) + (sa * cd * ce + sd * se) * yes + sa * cd * ye + sd * ze) / c
    d_al = (-sa * cd * (xes + xe) + ca * cd * ce * yes + ca * cd * ye) / c
    d_de = (-ca * sd * (xes + xe) + (-sa * sd * ce + cd * se) * yes - sa * sd * ye + cd * ze) / c
    d_T = (ca * cd * (dxes + dxe) + (sa * cd * ce + sd * se) * dyes + sa * cd * dye) / c
    return pm, d_al, d_de, d_T


def _ab_partials(T, alpha, delta, det, eph):
    """a, b and their partials w.r.t. x = alpha - sidereal angle and delta."""
    x = alpha - model.sidereal_angle(T, det, eph)
    ca, cb = model._ab_coeffs(delta, det)
    g2, lam = 2.0 * det.gamma, det.lat
    s2g, c2g = math.sin(g2), math.cos(g2)
    sl, cl = math.sin(lam), math.cos(lam)
    s2l, c2l = math.sin(2 * lam), math.cos(2 * lam)
    sd, cd = math.sin(delta), math.cos(delta)
    s2d, c2d = math.sin(2 * delta), math.cos(2 * delta)
    # d/ddelta of the coefficients
    da = dict(a2c=s2g * (3 - c2l) * 2 * s2d / 16.0, a2s=-c2g * sl * 2 * s2d / 4.0,
              a1c=s2g * s2l * 2 * c2d / 4.0, a1s=-c2g * cl * 2 * c2d / 2.0,
              a0=-0.75 * s2g * cl * cl * s2d)
    db = dict(b2c=c2g * sl * cd, b2s=s2g * (3 - c2l) * cd / 4.0,
              b1c=-c2g * cl * sd, b1s=-s2g * s2l * sd / 2.0)
    c2x, s2x, c1x, s1x = np.cos(2 * x), np.sin(2 * x), np.cos(x), np.sin(x)

    def ev(k, pre):
        v = k[pre + "2c"] * c2x + k[pre + "2s"] * s2x + k[pre + "1c"] * c1x + k[pre + "1s"] * s1x
        return v + k.get(pre + "0", 0.0)

    def evx(k, pre):
        return (-2 * k[pre + "2c"] * s2x + 2 * k[pre + "2s"] * c2x
                - k[pre + "1c"] * s1x + k[pre + "1s"] * c1x)

    return ev(ca, "a"), ev(cb, "b"), evx(ca, "a"), evx(cb, "b"), ev(da, "a"), ev(db, "b")


def fstat_continuous(seg: Segment, params, det, eph, mode, grad=False):
    """F at a continuous band-relative frequency by the resampling method
    (the sum over the SSB grid with e^{-2 pi i f j dt} in place of the FFT
    kernel), and optionally its analytic gradient dF/d(f, fdot, alpha, delta).

    The gradient differentiates every step: t_b0(alpha, delta); t_j through
    the implicit relation t_j + phi_m(t_j) = t_b0 + j dt; the interpolant
    (NEAREST has zero derivative); a(t_j), b(t_j); the demodulation phase; and
    A, B, C."""
    f, fdot, alpha, delta = (float(v) for v in params)
    n, dt = seg.n, seg.dt
    j = np.arange(n, dtype=np.float64)
    tb0, t = ssb_times(seg, alpha, delta, det, eph)
    T = seg.t0 + t
    xr, dxdu = interpolate(seg, ssb_positions(seg, alpha, delta, det, eph), mode)
    pm, pm_al, pm_de, pm_T = _roemer_partials(T, alpha, delta, det, eph)
    a, b, a_x, b_x, a_d, b_d = _ab_partials(T, alpha, delta, det, eph)
    cyc = demod_cycles(t, seg.t0, alpha, delta, seg.f_ref, fdot, det, eph) + f * j * dt
    e = np.exp(-2j * math.pi * (cyc - np.round(cyc)))
    Sa = np.sum(xr * a * e)
    Sb = np.sum(xr * b * e)
    A, B, C = abc(seg, alpha, delta, det, eph)
    s2 = seg.noise_var()
    F = float(combine(Sa, Sb, A, B, C, s2))
    if not grad:
        return F
    # d t_b0 / d(alpha, delta)
    _, tb0_al, tb0_de, _ = _roemer_partials(np.array([seg.t0]), alpha, delta, det, eph)
    wr = 2.0 * math.pi / eph.sidereal_day
    den = 1.0 + pm_T
    dS = {}
    for name in ("f", "fdot", "alpha", "delta"):
        if name in ("alpha", "delta"):
            pm_th = pm_al if name == "alpha" else pm_de
            tb0_th = float((tb0_al if name == "alpha" else tb0_de)[0])
            dt_th = (tb0_th - pm_th) / den                       # d t_j / d theta
            dxr = dxdu * dt_th / dt
            dx = (1.0 if name == "alpha" else 0.0) - wr * dt_th  # d x / d theta
            da = a_x * dx + (a_d if name == "delta" else 0.0)
            db = b_x * dx + (b_d if name == "delta" else 0.0)
            dpm = pm_th + pm_T * dt_th                            # total d phi_m
            dcyc = seg.f_ref * dpm + fdot * (t * dt_th + dpm * t + pm * dt_th)
        else:
            dxr = da = db = 0.0
            dcyc = (j * dt) if name == "f" else (0.5 * t * t + pm * t)
        g = -2j * math.pi * dcyc
        dS[name] = (np.sum((dxr * a + xr * da + xr * a * g) * e),
                    np.sum((dxr * b + xr * db + xr * b * g) * e))
    # d(A, B, C) on the detector grid
    td = seg.t0 + np.arange(n, dtype=np.float64) * dt
    ga, gb, gax, gbx, gad, gbd = _ab_partials(td, alpha, delta, det, eph)
    m = seg.m
    dABC = {"f": (0.0, 0.0, 0.0), "fdot": (0.0, 0.0, 0.0),
            "alpha": (np.sum(m * 2 * ga * gax), np.sum(m * 2 * gb * gbx),
                      np.sum(m * (gax * gb + ga * gbx))),
            "delta": (np.sum(m * 2 * ga * gad), np.sum(m * 2 * gb * gbd),
                      np.sum(m * (gad * gb + ga * gbd)))}
    D = s2 * (A * B - C * C)
    num = B * abs(Sa) ** 2 + A * abs(Sb) ** 2 - 2 * C * np.real(Sa * np.conj(Sb))
    out = []
    for name in ("f", "fdot", "alpha", "delta"):
        dSa, dSb = dS[name]
        dA, dB, dC = dABC[name]
        dnum = (dB * abs(Sa) ** 2 + 2 * B * np.real(np.conj(Sa) * dSa)
                + dA * abs(Sb) ** 2 + 2 * A * np.real(np.conj(Sb) * dSb)
                - 2 * dC * np.real(Sa * np.conj(Sb))
                - 2 * C * np.real(dSa * np.conj(Sb) + Sa * np.conj(dSb)))
        dD = s2 * (dA * B + A * dB - 2 * C * dC)
        out.append(float(dnum / D - num * dD / (D * D)))
    return F, np.array(out)
