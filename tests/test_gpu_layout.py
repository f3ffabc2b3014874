"""The inter-pass spill in both of its layouts: where a row of pass 2's column
block (B2 elements) is shorter than 512 B the spill is stored blocked,
Z[k2 / B2][r][k2 % B2], otherwise row-major, Z[r][k2].  Splits of nfft = 2^16
are forced through the tuning cache so that both layouts run at a size the
oracle maps in full: plain maps and interbinned maps (Eq. intbin) against the
oracle, at both precisions, and the per-node maxima and threshold crossings of
the same calls against the map."""
import numpy as np
import pytest

from oracle import method, model
from paper_1003_0844_amd import fstat, synth
from tests.common import DET, EPH
from tests.gpu_common import PREC_TOL, banner, f_error, oracle_map

pytestmark = pytest.mark.gpu

# (precision, C): R = 2^16 / C; FP32 B2 = min(4096 / R, 64) of 16 B elements,
# FP64 B2 = min(2048 / R, 32) of 32 B elements
CASES = [
    (fstat.FP32, 64),    # R = 1024, B2 = 4: 64 B rows, blocked
    (fstat.FP32, 256),   # R = 256, B2 = 16: 256 B rows, blocked (the 2-day map's layout)
    (fstat.FP32, 1024),  # R = 64, B2 = 64: 1 KB rows, row-major
    (fstat.FP64, 256),   # R = 256, B2 = 8: 256 B rows, blocked
    (fstat.FP64, 4096),  # R = 16, B2 = 32: 1 KB rows, row-major
]


def _interleave(F0, Fh):
    out = np.empty(2 * len(F0))
    out[0::2], out[1::2] = F0, Fh
    return out


@pytest.mark.parametrize("interbin", [False, True])
@pytest.mark.parametrize("prec,C", CASES)
def test_spill_layouts_against_oracle(prec, C, interbin, tmp_path, monkeypatch):
    w = synth.TINY  # N = 43082, nfft = 2^16 = nextpow2(N): also the interbinned length
    g, x, sigs = synth.segment_data(w)
    p = sigs[0]
    x = x + model.injection(w.n, w.dt, 0.0, p, synth.F_REF, 1.0, DET, EPH)
    seg = method.Segment(x=x, dt=w.dt, n_days=w.days, f_ref=synth.F_REF, sigma2=1.0, nfft=w.nfft)
    cache = tmp_path / "tune.txt"
    cache.write_text("fstat-tune-v3 %d %d %d %d %d 2 1\n" % (prec, w.interp, w.nfft, w.n, C))
    monkeypatch.setenv("FSTAT_TUNE_CACHE", str(cache))
    banner("spill layout", "prec", prec, "C", C, "interbin", interbin)
    specs = [fstat.SegmentSpec(x=seg.x, dt=seg.dt, n_days=seg.n_days, f_ref=seg.f_ref, sigma2=1.0, nfft=w.nfft)]
    plan = fstat.Plan(specs, fstat.detector_spec(DET), fstat.ephemeris_spec(EPH), interp=w.interp, prec=prec,
                      autotune=True)
    sch = plan.schedule()
    assert sch["C"] == C and sch["R"] * C == w.nfft and sch["batch"] == 2
    al, de = synth.sky_uniform(synth.rng(7), 2)
    # three nodes in batches of two: two launches of each pass
    nodes = fstat.nodes_array(np.r_[p["alpha"], al], np.r_[p["delta"], de], [p["fdot"], -3e-10, -8e-10])
    half = w.nfft // 2
    k = np.arange(half)
    F = plan.grid_map(nodes, 0, half, interbin=interbin).cpu().numpy()
    for i, nd in enumerate(nodes):
        if interbin:
            F0, Fh = method.fstat_bins_interbinned(seg, nd["fdot"], nd["alpha"], nd["delta"], DET, EPH, w.interp,
                                                   k=k, dft="fft")
            ref = _interleave(F0, Fh)
        else:
            ref = oracle_map(seg, nd["fdot"], nd["alpha"], nd["delta"], w.interp, k)
        err = f_error(F[i], ref)
        assert err < PREC_TOL[prec], (prec, C, interbin, i, err)
    # the per-node maximum and the threshold crossings read the same spill and
    # round like the map: their values are the map's, exactly
    Fmax, kmax = plan.grid_max(nodes, 0, half, interbin=interbin)
    Fmax, kmax = Fmax.cpu().numpy(), kmax.cpu().numpy()
    assert np.array_equal(Fmax, F.max(axis=1)) and np.array_equal(kmax, F.argmax(axis=1))
    # the kernel compares F, widened to FP64, with the FP64 threshold
    F64 = F.astype(np.float64)
    thr = float(np.quantile(F64, 0.999))
    rec, cnt = plan.grid_crossings(nodes, 0, half, thr, 4 * F.size // 1000 + 16, interbin=interbin)
    got = fstat.Plan.read_crossings(rec, cnt)
    want = np.argwhere(F64 > thr)
    assert int(cnt.cpu().item()) == len(want) == len(got)
    assert sorted(zip(got["node"].tolist(), got["k"].tolist())) == sorted(map(tuple, want.tolist()))
    assert np.array_equal(np.sort(got["F"]), np.sort(F64[F64 > thr]))



def test_sub_bands_and_unaligned_maps_equal_the_full_map(tmp_path, monkeypatch):
    # FP32 with R = 256 (B2 = 16, the 2-day map's pass 2): a band [k_lo, k_hi)
    # is the same columns of the full map, whatever the band's alignment to the
    # column blocks, and a map that starts 4 bytes off 16-byte alignment gets
    # the same values, bit for bit
    import torch
    w = synth.TINY
    g, x, sigs = synth.segment_data(w)
    cache = tmp_path / "tune.txt"
    cache.write_text("fstat-tune-v3 %d %d %d %d %d 2 1\n" % (fstat.FP32, w.interp, w.nfft, w.n, 256))
    monkeypatch.setenv("FSTAT_TUNE_CACHE", str(cache))
    banner("map sub-bands", "nfft", w.nfft)
    plan = fstat.Plan([fstat.SegmentSpec(x=x, dt=w.dt, n_days=w.days, nfft=w.nfft)], fstat.detector_spec(DET),
                      fstat.ephemeris_spec(EPH), interp=w.interp, prec=fstat.FP32, autotune=True)
    assert plan.schedule()["R"] == 256 and plan.schedule()["B2"] == 16
    al, de = synth.sky_uniform(synth.rng(11), 3)
    nodes = fstat.nodes_array(al, de, [0.0, -4e-10, -9e-10])
    half = w.nfft // 2
    full = plan.grid_map(nodes, 0, half).clone()
    for lo, hi in [(0, half - 1), (64, half - 96), (63, half - 96), (17, 4113)]:
        part = plan.grid_map(nodes, lo, hi).clone()
        torch.cuda.synchronize()
        assert torch.equal(part, full[:, lo:hi]), (lo, hi)
    buf = torch.full((len(nodes) * half + 1,), float("nan"), dtype=torch.float32, device="cuda")
    skew = buf[1:].view(len(nodes), half)
    plan.grid_map(nodes, 0, half, skew)
    torch.cuda.synchronize()
    assert torch.equal(skew, full)
