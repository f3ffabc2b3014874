"""The lattice grid of Sec. IV on the GPU: nodes whose lines of Fourier bins are
shifted by a fraction of a bin (Eq. avec), against the oracle, and a search of
a sky patch with the library's constrained lattice."""
import math

import numpy as np
import pytest
import torch

from oracle import method
from paper_1003_0844_amd import fstat, synth
from tests.common import DET, EPH, one_signal, small_segment
from tests.gpu_common import PREC_TOL, banner, f_error, make_plan

pytestmark = pytest.mark.gpu

OFFSETS = [0.0, 0.25, -0.4, 0.999, 0.5]


def _nodes_with_offsets(sig, seed):
    al, de = synth.sky_uniform(synth.rng(seed), 2)
    alpha = np.r_[sig["alpha"], al, sig["alpha"], al[0]]
    delta = np.r_[sig["delta"], de, sig["delta"], de[1]]
    fdot = [sig["fdot"], -2e-10, -6e-10, sig["fdot"], -1e-10]
    return fstat.nodes_array(alpha, delta, fdot, bin_offset=OFFSETS)


@pytest.mark.parametrize("prec", [fstat.FP32, fstat.FP64])
@pytest.mark.parametrize("interbin", [False, True])
def test_bin_offsets_match_oracle(prec, interbin):
    # 1 day at dt = 13 s: N = 6628; nfft = 2^14 (plain) or 2^13 (interbinned)
    dt = 13.0
    n = int(round(synth.SIDEREAL_DAY / dt))
    nfft = (1 << int(math.ceil(math.log2(n)))) * (1 if interbin else 2)
    sig = one_signal(41, band=1 / (2 * dt), snr=20.0)
    seg = small_segment(days=1, dt=dt, seed=41, signal=sig, nfft=nfft)
    banner("lattice bin offsets", "prec", prec, "interbin", interbin, "nfft", nfft)
    plan = make_plan([seg], method.LINEAR_UP2, prec)
    nodes = _nodes_with_offsets(sig, 8)
    half = nfft // 2
    k_lo, k_hi = 3, half - 1
    F = plan.grid_map(nodes, k_lo, k_hi, interbin=interbin).double().cpu().numpy()
    k = np.arange(k_lo, k_hi)
    for i, nd in enumerate(nodes):
        off = float(nd["bin_offset"])
        if interbin:
            F0, Fh = method.fstat_bins_interbinned(seg, nd["fdot"], nd["alpha"], nd["delta"], DET, EPH,
                                                   method.LINEAR_UP2, k=k, dft="fft", bin_offset=off)
            ref = np.empty(2 * len(k))
            ref[0::2], ref[1::2] = F0, Fh
        else:
            ref = method.fstat_bins(seg, nd["fdot"], nd["alpha"], nd["delta"], DET, EPH, method.LINEAR_UP2, k=k,
                                    dft="fft", bin_offset=off)
        err = f_error(F[i], ref)
        assert err < PREC_TOL[prec], (i, off, err)
    # an offset of zero is the plain map, bit for bit
    plain = plan.grid_map(fstat.nodes_array(nodes["alpha"][:1], nodes["delta"][:1], nodes["fdot"][:1]),
                          k_lo, k_hi, interbin=interbin).double().cpu().numpy()
    assert np.array_equal(plain[0], F[0])


def test_bin_offset_is_validated():
    dt = 26.0
    seg = small_segment(days=1, dt=dt, seed=3)
    banner("lattice bin offset validation")
    plan = make_plan([seg], method.LINEAR_UP2, fstat.FP32)
    for bad in (1.0, -1.0, float("nan"), float("inf")):
        nodes = fstat.nodes_array(1.0, 0.2, 0.0, bin_offset=bad)
        with pytest.raises(fstat.FStatError) as e:
            plan.grid_map(nodes, 0, 16)
        assert e.value.status == fstat.EINVAL


@pytest.mark.parametrize("rule", [fstat.NU_DEEP_HOLES, fstat.NU_COVERING])
@pytest.mark.parametrize("seed", [31, 32, 33])
def test_lattice_patch_search_recovers_a_signal(seed, rule):
    # a noise-free signal; the library's lattice nodes over a sky patch of
    # half a sky cell around it and its spindown: the covering (correlation
    # C0 = 3/4 in the linear model) keeps the best node near 3/4 of the
    # perfect template's F in the full model
    dt = 13.0
    band = 1 / (2 * dt)
    sig = one_signal(seed, band=band, snr=20.0, fdot=(-4e-10, 0.0))
    seg = small_segment(days=1, dt=dt, seed=seed, signal=sig, noise=False)
    spec = fstat.SegmentSpec(x=seg.x, dt=dt, n_days=1, t0=seg.t0, f_ref=seg.f_ref, sigma2=seg.sigma2)
    lat = fstat.Lattice.for_segment(spec, fstat.detector_spec(DET), fstat.ephemeris_spec(EPH), rule=rule)
    f_sky = seg.f_ref + band
    om = 2 * math.pi * f_sky
    ce, se = math.cos(EPH.obliquity), math.sin(EPH.obliquity)
    al, de = sig["alpha"], sig["delta"]
    a1 = om * (math.sin(al) * math.cos(de) * ce + math.sin(de) * se)
    a2 = om * math.cos(al) * math.cos(de)
    nz = -math.sin(al) * math.cos(de) * se + math.sin(de) * ce
    cell = math.sqrt(abs(np.linalg.det(lat.basis[2:, 2:])))
    nodes = lat.nodes(f_sky, sig["fdot"], sig["fdot"], fstat.ephemeris_spec(EPH), sky=(a1, a2, 0.5 * cell),
                      hemisphere=1 if nz >= 0 else -1)
    banner("lattice patch search", "seed", seed, "rule", rule, "nodes", len(nodes), "theta", lat.theta)
    assert 8 <= len(nodes) <= 200
    plan = make_plan([seg], method.LINEAR_UP2, fstat.FP32)
    half = seg.fft_len // 2
    F = plan.grid_map(nodes, 0, half).double().cpu().numpy()
    Ftrue = method.fstat_continuous(seg, (sig["f"], sig["fdot"], al, de), DET, EPH, method.LINEAR_UP2)
    best = int(np.argmax(F.max(axis=1)))
    assert F.max() > 0.7 * Ftrue, (F.max(), Ftrue)
    # parity on the best node and two others, whole band
    k = np.arange(half)
    for i in {best, 0, len(nodes) - 1}:
        nd = nodes[i]
        ref = method.fstat_bins(seg, nd["fdot"], nd["alpha"], nd["delta"], DET, EPH, method.LINEAR_UP2, k=k,
                                dft="fft", bin_offset=float(nd["bin_offset"]))
        assert f_error(F[i], ref) < PREC_TOL[fstat.FP32], i


def test_lattice_nodes_at_full_size_sampled_bins():
    # the 2-day segment of the benchmark (N = 344656, nfft = 2^20) with an
    # injection; lattice nodes over a small patch around it, in the benchmark's
    # launch configuration; sampled bins of a few nodes against the oracle
    w = synth.GRID2D
    g, x, sigs = synth.segment_data(w)
    sig = sigs[0]
    from oracle import model
    x = x + model.injection(len(x), w.dt, 0.0, sig, synth.F_REF, 1.0, DET, EPH, None)
    spec = fstat.SegmentSpec(x=x, dt=w.dt, n_days=w.days, nfft=w.nfft)
    lat = fstat.Lattice.for_segment(spec, fstat.detector_spec(DET), fstat.ephemeris_spec(EPH))
    f_sky = synth.F_REF + 1 / (2 * w.dt)
    om = 2 * math.pi * f_sky
    ce, se = math.cos(EPH.obliquity), math.sin(EPH.obliquity)
    al, de = sig["alpha"], sig["delta"]
    a1 = om * (math.sin(al) * math.cos(de) * ce + math.sin(de) * se)
    a2 = om * math.cos(al) * math.cos(de)
    nodes = lat.nodes(f_sky, sig["fdot"] - 2e-10, sig["fdot"] + 2e-10, fstat.ephemeris_spec(EPH),
                      sky=(a1, a2, 60.0))
    banner("lattice full size", w.name, "nodes", len(nodes))
    plan = fstat.Plan([spec], fstat.detector_spec(DET), fstat.ephemeris_spec(EPH), interp=fstat.LINEAR_UP2,
                      prec=fstat.FP32, device=0, autotune=True)
    half = w.nfft // 2
    F = plan.grid_map(nodes, 0, half)
    Fmax, kmax = plan.grid_max(nodes, 0, half)
    Fh = F.double().cpu().numpy()
    assert np.array_equal(Fmax.double().cpu().numpy(), Fh.max(axis=1))
    seg = method.Segment(x=x, dt=w.dt, n_days=w.days, f_ref=synth.F_REF, sigma2=1.0, nfft=w.nfft)
    rng = np.random.default_rng(5)
    best = int(np.argmax(Fh.max(axis=1)))
    for i in sorted({best, *rng.choice(len(nodes), 3, replace=False).tolist()}):
        nd = nodes[i]
        k = np.unique(np.r_[int(np.argmax(Fh[i])), rng.integers(0, half, 32)])
        ref = method.fstat_bins(seg, nd["fdot"], nd["alpha"], nd["delta"], DET, EPH, method.LINEAR_UP2, k=k,
                                bin_offset=float(nd["bin_offset"]))
        assert f_error(Fh[i][k], ref) < PREC_TOL[fstat.FP32], i
    # the SNR-10 injection stands out at the best node (2F ~ 4 in noise)
    assert 2 * Fh.max() > 40


@pytest.mark.parametrize("interbin", [False, True])
def test_graph_replays_of_offset_nodes(interbin):
    # lattice nodes (bin offsets) recorded as a HIP graph: every replay equal to
    # the eager call, with eager work between replays
    dt = 13.0
    sig = one_signal(44, band=1 / (2 * dt), snr=15.0)
    seg = small_segment(days=1, dt=dt, seed=44, signal=sig)
    spec = fstat.SegmentSpec(x=seg.x, dt=dt, n_days=1, t0=seg.t0, f_ref=seg.f_ref, sigma2=seg.sigma2)
    lat = fstat.Lattice.for_segment(spec, fstat.detector_spec(DET), fstat.ephemeris_spec(EPH))
    f_sky = seg.f_ref + 1 / (2 * dt)
    nodes = lat.nodes(f_sky, -3e-10, 0.0, fstat.ephemeris_spec(EPH), sky=(0.2 * 2 * math.pi * f_sky, 0.1, 150.0))
    banner("lattice graph", "interbin", interbin, "nodes", len(nodes))
    assert len(nodes) > 4 and np.any(nodes["bin_offset"] != 0)
    plan = make_plan([seg], method.LINEAR_UP2, fstat.FP32, max_batch=4)
    half = seg.fft_len // 2 - (1 if interbin else 0)
    eager = plan.grid_map(nodes, 0, half, interbin=interbin).clone()
    g = plan.graph_map(nodes, 0, half, interbin=interbin)
    for rep in range(3):
        g.outputs["F"].fill_(float("nan"))
        g.launch()
        torch.cuda.synchronize()
        assert torch.equal(g.outputs["F"], eager), rep
        plan.grid_map(nodes[::-1].copy(), 0, half // 2)
        (torch.randn(1 << 18, device="cuda") * 2).sum().item()
        torch.cuda.synchronize()


@pytest.mark.parametrize("interbin", [False, True])
def test_bin_params_reproduce_the_map(interbin):
    # crossings on lattice nodes -> continuous parameters -> F by the method at
    # that frequency (fstat_eval, FP64 direct sum): the map value at the bin
    dt = 13.0
    sig = one_signal(45, band=1 / (2 * dt), snr=25.0)
    seg = small_segment(days=1, dt=dt, seed=45, signal=sig)
    n = int(round(synth.SIDEREAL_DAY / dt))
    nfft = (1 << int(math.ceil(math.log2(n)))) * (1 if interbin else 2)
    seg.nfft = nfft
    spec = fstat.SegmentSpec(x=seg.x, dt=dt, n_days=1, t0=seg.t0, f_ref=seg.f_ref, sigma2=seg.sigma2, nfft=nfft)
    lat = fstat.Lattice.for_segment(spec, fstat.detector_spec(DET), fstat.ephemeris_spec(EPH))
    f_sky = seg.f_ref + 1 / (2 * dt)
    om = 2 * math.pi * f_sky
    ce, se = math.cos(EPH.obliquity), math.sin(EPH.obliquity)
    al, de = sig["alpha"], sig["delta"]
    a1 = om * (math.sin(al) * math.cos(de) * ce + math.sin(de) * se)
    a2 = om * math.cos(al) * math.cos(de)
    nodes = lat.nodes(f_sky, sig["fdot"], sig["fdot"], fstat.ephemeris_spec(EPH), sky=(a1, a2, 60.0))
    banner("lattice bin params", "interbin", interbin, "nodes", len(nodes))
    plan = make_plan([seg], method.LINEAR_UP2, fstat.FP64)
    half = nfft // 2 - (1 if interbin else 0)
    F = plan.grid_map(nodes, 0, half, interbin=interbin).cpu().numpy()
    thr = float(np.quantile(F, 0.9995))
    rec, cnt = plan.grid_crossings(nodes, 0, half, thr, 1 << 14, interbin=interbin)
    got = fstat.Plan.read_crossings(rec, cnt)
    assert len(got) > 5
    params, segi = plan.bin_params(nodes[got["node"]], got["k"], interbin=interbin)
    Fe, _ = plan.eval(params, segi, want_state=False)
    Fe = Fe.cpu().numpy()
    if interbin:
        # integer bins only: the half bins are Eq. (intbin)'s approximation, not F there
        whole = got["k"] % 2 == 0
        assert np.any(whole)
        assert f_error(Fe[whole], got["F"][whole]) < 1e-9
    else:
        assert f_error(Fe, got["F"]) < 1e-9
