"""The search of Sec. VII on one segment, end to end on the GPU: lattice nodes
over a sky patch (Sec. IV), the F map and its threshold crossings (Eqs. PF, FP),
the strongest crossing turned into continuous parameters, the Nelder-Mead fine
search on exact F (Sec. VI C) and the amplitude estimates (Eqs. amle0,
ampone)."""
import math

import numpy as np
import pytest
import torch

from oracle import method, model
from paper_1003_0844_amd import fstat, synth
from tests.common import DET, EPH, one_signal, small_segment
from tests.gpu_common import banner, make_plan

pytestmark = pytest.mark.gpu


def _patch(lat, seg, sig, dt, radius_cells):
    f_sky = seg.f_ref + 1 / (2 * dt)
    om = 2 * math.pi * f_sky
    ce, se = math.cos(EPH.obliquity), math.sin(EPH.obliquity)
    al, de = sig["alpha"], sig["delta"]
    a1 = om * (math.sin(al) * math.cos(de) * ce + math.sin(de) * se)
    a2 = om * math.cos(al) * math.cos(de)
    cell = math.sqrt(abs(np.linalg.det(lat.basis[2:, 2:])))
    return lat.nodes(f_sky, -4e-10, 0.0, fstat.ephemeris_spec(EPH), sky=(a1, a2, radius_cells * cell))


def _setup(seed, snr):
    dt = 13.0
    sig = one_signal(seed, band=1 / (2 * dt), snr=max(snr, 1.0), fdot=(-4e-10, 0.0))
    seg = small_segment(days=1, dt=dt, seed=seed, signal=sig if snr > 0 else None)
    spec = fstat.SegmentSpec(x=seg.x, dt=dt, n_days=1, t0=seg.t0, f_ref=seg.f_ref, sigma2=seg.sigma2)
    lat = fstat.Lattice.for_segment(spec, fstat.detector_spec(DET), fstat.ephemeris_spec(EPH), rule=fstat.NU_COVERING)
    nodes = _patch(lat, seg, sig, dt, 1.5)
    return dt, sig, seg, nodes


def _cells(seg):
    T = seg.n * seg.dt
    df = 1.0 / (seg.fft_len * seg.dt)
    v_c = 2 * math.pi * 1.495978707e11 / (365.256363004 * 86400.0) / 299792458.0
    return [df, 1.0 / T ** 2, df / (seg.f_ref * v_c), df / (seg.f_ref * v_c)]


@pytest.mark.parametrize("seed", [61, 62])
def test_search_of_one_segment(seed):
    dt, sig, seg, nodes = _setup(seed, snr=15.0)
    half = seg.fft_len // 2
    banner("pipeline", "seed", seed, "nodes", len(nodes))
    plan = make_plan([seg], method.LINEAR_UP2, fstat.FP32)
    # threshold for a 0.1 % false-alarm probability over every grid point
    F0 = fstat.threshold(1e-3, len(nodes) * half)
    rec, cnt = plan.grid_crossings(nodes, 0, half, F0, 1 << 16)
    got = fstat.Plan.read_crossings(rec, cnt)
    assert len(got) > 0
    best = got[np.argmax(got["F"])]
    assert best["F"] > F0
    # coarse candidate -> continuous parameters -> fine search on exact F
    plan64 = make_plan([seg], method.LINEAR_UP2, fstat.FP64)
    p0, segi = plan64.bin_params(nodes[[best["node"]]], [best["k"]])
    Fc = plan64.eval_exact(p0, segi).cpu().numpy()[0]
    pout, Ff, nev = plan64.refine(p0, _cells(seg), tol=1e-3, max_evals=600, exact=True, seg=segi)
    Ff = Ff.cpu().numpy()[0]
    truth = torch.tensor([[sig["f"], sig["fdot"], sig["alpha"], sig["delta"]]], dtype=torch.float64, device="cuda")
    Ft = plan64.eval_exact(truth).cpu().numpy()[0]
    print("pipeline seed %d: %d nodes, F0 %.2f, %d crossings, coarse F %.1f (exact %.1f), refined %.1f in %d "
          "evaluations, F at the injection %.1f" % (seed, len(nodes), F0, len(got), best["F"], Fc, Ff,
                                                     int(nev.cpu().item()), Ft), flush=True)
    assert Ff >= Fc and Ff >= 0.95 * Ft
    # amplitudes at the refined point: the injected h0 (the amplitude that
    # gives the requested SNR) comes back within the noise (SNR 15: ~10 %)
    amp = plan64.amplitudes(pout, segi).cpu().numpy()[0]
    t = np.arange(seg.n) * seg.dt
    h1 = model.signal(t, 0.0, sig["f"], sig["fdot"], sig["alpha"], sig["delta"], 1.0, sig["cosi"], sig["psi"],
                      sig["phi0"], seg.f_ref, DET, EPH)
    h0 = sig["snr"] / math.sqrt(np.sum(h1 * h1) / seg.sigma2)
    assert abs(amp[4] / h0 - 1) < 0.4, (amp[4], h0)


def test_noise_only_segment_has_no_crossing():
    dt, sig, seg, nodes = _setup(63, snr=0.0)
    half = seg.fft_len // 2
    banner("pipeline noise", "nodes", len(nodes))
    plan = make_plan([seg], method.LINEAR_UP2, fstat.FP32)
    F0 = fstat.threshold(1e-3, len(nodes) * half)
    rec, cnt = plan.grid_crossings(nodes, 0, half, F0, 1 << 10)
    assert int(cnt.cpu().item()) == 0
    Fmax, _ = plan.grid_max(nodes, 0, half)
    # and so does the largest F of the map
    assert float(Fmax.max().item()) < F0
