"""Interbinning (Sec. VI B, Eq. intbin) in the pass-2 epilogue: F at the Fourier
bins k and the half bins k + 1/2 from (S(k+1) - S(k))/sqrt(2), against the
oracle, on unpadded FFT lengths nfft = nextpow2(N)."""
import math

import numpy as np
import pytest
import torch

from oracle import method
from paper_1003_0844_amd import fstat, synth
from tests.common import DET, EPH, one_signal, small_segment
from tests.gpu_common import PREC_TOL, banner, f_error, make_plan

pytestmark = pytest.mark.gpu


def _segment(seed, days=1, dt=13.0, offset_bins=None):
    n = int(round(days * synth.SIDEREAL_DAY / dt))
    nfft = 1 << int(math.ceil(math.log2(n)))
    sig = one_signal(seed, band=1 / (2 * dt), snr=20.0)
    if offset_bins is not None:
        # put the signal half way between two Fourier frequencies
        df = 1.0 / (nfft * dt)
        sig["f"] = (math.floor(sig["f"] / df) + offset_bins) * df
    seg = small_segment(days=days, dt=dt, seed=seed, signal=sig, nfft=nfft)
    return seg, sig


def _nodes(sig, seed):
    al, de = synth.sky_uniform(synth.rng(seed), 2)
    return fstat.nodes_array(np.r_[sig["alpha"], al], np.r_[sig["delta"], de], [sig["fdot"], -2e-10, -6e-10])


def _interleave(F0, Fh):
    out = np.empty(2 * len(F0))
    out[0::2], out[1::2] = F0, Fh
    return out


@pytest.mark.parametrize("prec", [fstat.FP32, fstat.FP64])
@pytest.mark.parametrize("krange", [(0, None), (37, 2000)])
def test_interbinned_map_matches_oracle(prec, krange):
    # 1 day at dt = 13 s: N = 6628, nfft = 2^13 (no padding beyond the power
    # of two); the full band reaches the last bin, whose neighbour is the
    # Nyquist bin of the next row of the FFT split
    seg, sig = _segment(21)
    banner("interbin map", "prec", prec, "range", krange, "nfft", seg.fft_len)
    plan = make_plan([seg], method.LINEAR_UP2, prec)
    k_lo, k_hi = krange[0], (krange[1] if krange[1] is not None else seg.fft_len // 2)
    nodes = _nodes(sig, 5)
    F = plan.grid_map(nodes, k_lo, k_hi, interbin=True).cpu().numpy()
    assert F.shape == (len(nodes), 2 * (k_hi - k_lo))
    k = np.arange(k_lo, k_hi)
    for i, nd in enumerate(nodes):
        F0, Fh = method.fstat_bins_interbinned(seg, nd["fdot"], nd["alpha"], nd["delta"], DET, EPH,
                                               method.LINEAR_UP2, k=k, dft="fft")
        err = f_error(F[i], _interleave(F0, Fh))
        assert err < PREC_TOL[prec], (i, err)


@pytest.mark.parametrize("prec", [fstat.FP32, fstat.FP64])
def test_interbinned_modes_agree(prec):
    seg, sig = _segment(22)
    banner("interbin modes", "prec", prec)
    plan = make_plan([seg], method.CUBIC_UP2, prec, max_batch=2)
    nodes = _nodes(sig, 6)
    half = seg.fft_len // 2
    # the Fourier bins of the interbinned map are the plain map up to rounding
    # (the two kernels inline the same butterflies in different contexts, and
    # the compiler may fuse multiply-adds differently)
    Fi = plan.grid_map(nodes, 0, half, interbin=True).double().cpu().numpy()
    Fp = plan.grid_map(nodes, 0, half).double().cpu().numpy()
    assert f_error(Fi[:, 0::2], Fp) < (1e-6 if prec == fstat.FP32 else 1e-13)
    # per-node maximum over both kinds of points, in half-bin units
    Fmax, kmax = plan.grid_max(nodes, 0, half, interbin=True)
    Fmax, kmax = Fmax.double().cpu().numpy(), kmax.cpu().numpy()
    assert np.array_equal(Fmax, Fi.max(axis=1))
    assert np.array_equal(kmax, np.argmax(Fi, axis=1))
    # crossings: exactly the map entries above the threshold
    thr = float(np.quantile(Fi, 0.995))
    rec, cnt = plan.grid_crossings(nodes, 0, half, thr, 1 << 16, interbin=True)
    got = fstat.Plan.read_crossings(rec, cnt)
    rows, cols = np.nonzero(Fi > thr)
    assert len(got) == len(rows) == int(cnt.item())
    want = set(zip(rows.tolist(), cols.tolist()))
    assert set(zip(got["node"].tolist(), got["k"].tolist())) == want
    for r in got:
        assert r["F"] == Fi[r["node"], r["k"]]


def test_half_bin_signal_is_recovered():
    # a signal half way between Fourier frequencies: the Fourier bins lose
    # about 1 - (2/pi)^2 of its power, the interbinned point about 1 - 8/pi^2
    seg, sig = _segment(23, offset_bins=0.5)
    banner("interbin half-bin signal")
    plan = make_plan([seg], method.CUBIC_UP2, fstat.FP32)
    node = fstat.nodes_array(sig["alpha"], sig["delta"], sig["fdot"])
    half = seg.fft_len // 2
    Fi = plan.grid_map(node, 0, half, interbin=True)[0].double().cpu().numpy()
    kh = int(np.argmax(Fi))
    k_sig = sig["f"] * seg.fft_len * seg.dt
    assert kh % 2 == 1 and abs(kh / 2 - k_sig) < 0.01, (kh, k_sig)
    assert Fi[kh] > 1.5 * Fi[0::2].max()
