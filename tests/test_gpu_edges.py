"""Edge cases of the grid path: the largest and smallest supported FFT
lengths, sky positions at the poles and at alpha = 0 / 2 pi, zero spindown,
single-bin ranges, and the argument checks that need a plan."""
import math

import numpy as np
import pytest
import torch

from oracle import method
from paper_1003_0844_amd import fstat, synth
from tests.common import DET, EPH, small_segment
from tests.gpu_common import PREC_TOL, banner, f_error, make_plan, oracle_map

pytestmark = pytest.mark.gpu


def test_largest_fft_length():
    # N = 2^21 samples over one sidereal day, nfft = 2^22 (the largest
    # supported): split R = 1024, C = 4096 in both precisions
    n = 1 << 21
    dt = synth.SIDEREAL_DAY / n
    seg = small_segment(days=1, dt=dt, seed=51, nfft=1 << 22)
    banner("largest nfft", seg.n, seg.fft_len)
    nodes = fstat.nodes_array([0.7], [-0.4], [-5e-10])
    half = seg.fft_len // 2
    k = np.unique(np.r_[np.random.default_rng(1).integers(0, half, 48), 0, half - 1])
    ref = method.fstat_bins(seg, -5e-10, 0.7, -0.4, DET, EPH, method.LINEAR_UP2, k=k)
    for prec in (fstat.FP32, fstat.FP64):
        plan = make_plan([seg], method.LINEAR_UP2, prec)
        assert plan.schedule()["R"] * plan.schedule()["C"] == seg.fft_len
        F = plan.grid_map(nodes, 0, half)[0].cpu().numpy()
        assert f_error(F[k], ref) < PREC_TOL[prec], prec
        del plan
        torch.cuda.empty_cache()


@pytest.mark.parametrize("mode", [method.NEAREST, method.LINEAR_UP2, method.CUBIC_UP2])
def test_smallest_fft_length(mode):
    # N = 512, nfft = 2^10 (the smallest supported): split R = 16, C = 64
    n = 512
    dt = synth.SIDEREAL_DAY / n
    seg = small_segment(days=1, dt=dt, seed=52, nfft=1 << 10)
    banner("smallest nfft", mode)
    al, de = synth.sky_uniform(synth.rng(52), 3)
    nodes = fstat.nodes_array(al, de, [0.0, -1e-9, -3e-10])
    half = seg.fft_len // 2
    for prec in (fstat.FP32, fstat.FP64):
        F = make_plan([seg], mode, prec).grid_map(nodes, 0, half).cpu().numpy()
        for i, nd in enumerate(nodes):
            ref = oracle_map(seg, nd["fdot"], nd["alpha"], nd["delta"], mode, np.arange(half))
            assert f_error(F[i], ref) < PREC_TOL[prec], (prec, i)


@pytest.mark.parametrize("prec", [fstat.FP32, fstat.FP64])
def test_poles_wraparound_and_zero_spindown(prec):
    seg = small_segment(days=1, dt=13.0, seed=53, nfft=16384)
    banner("poles", prec)
    alpha = [0.3, 2.0, 0.0, 2 * math.pi - 1e-9, 1.0]
    delta = [math.pi / 2, -math.pi / 2, 0.2, 0.2, 0.0]
    fdot = [0.0, 0.0, -1e-9, -1e-9, 0.0]
    nodes = fstat.nodes_array(alpha, delta, fdot)
    half = seg.fft_len // 2
    F = make_plan([seg], method.CUBIC_UP2, prec).grid_map(nodes, 0, half).cpu().numpy()
    for i, nd in enumerate(nodes):
        ref = oracle_map(seg, nd["fdot"], nd["alpha"], nd["delta"], method.CUBIC_UP2, np.arange(half))
        assert f_error(F[i], ref) < PREC_TOL[prec], i
    # alpha = 0 and alpha = 2 pi - 1e-9 are the same sky position up to 1e-9 rad
    assert f_error(F[2], F[3]) < 1e-4


def test_single_bin_ranges():
    seg = small_segment(days=1, dt=13.0, seed=54, nfft=16384)
    banner("single bins")
    plan = make_plan([seg], method.LINEAR_UP2, fstat.FP32)
    nodes = fstat.nodes_array([0.5, 1.5], [0.1, -0.7], [0.0, -2e-10])
    half = seg.fft_len // 2
    full = plan.grid_map(nodes, 0, half)
    for lo in (0, 1, half - 1):
        part = plan.grid_map(nodes, lo, lo + 1)
        assert torch.equal(part[:, 0], full[:, lo])
    Fmax, kmax = plan.grid_max(nodes, half - 1, half)
    assert torch.equal(Fmax, full[:, half - 1]) and bool((kmax == half - 1).all())


def test_node_ranges_resume_bit_for_bit():
    # a grid call is a pure function of (plan, nodes): re-issuing it from any
    # node index (a resumed search) gives the same rows, maxima and crossings
    seg = small_segment(days=1, dt=13.0, seed=57, nfft=16384)
    banner("node-range resume")
    plan = make_plan([seg], method.LINEAR_UP2, fstat.FP32, max_batch=4)
    g = synth.rng(58)
    al, de = synth.sky_uniform(g, 5)
    nodes = fstat.nodes_array(np.repeat(al, 3), np.repeat(de, 3), np.tile([0.0, -3e-10, -7e-10], 5))
    half = seg.fft_len // 2
    full = plan.grid_map(nodes, 0, half).clone()
    Fm, km = [t.clone() for t in plan.grid_max(nodes, 0, half)]
    thr = float(torch.quantile(full.double().flatten()[::7], 0.99))
    rec, cnt = plan.grid_crossings(nodes, 0, half, thr, 1 << 16)
    want = sorted(zip(*[fstat.Plan.read_crossings(rec, cnt)[c].tolist() for c in ("node", "k", "F")]))
    for cut in (1, 7, 14):
        a = fstat.nodes_array(nodes["alpha"][:cut], nodes["delta"][:cut], nodes["fdot"][:cut])
        b = fstat.nodes_array(nodes["alpha"][cut:], nodes["delta"][cut:], nodes["fdot"][cut:])
        assert torch.equal(torch.cat([plan.grid_map(a, 0, half), plan.grid_map(b, 0, half)]), full), cut
        ma, ka = plan.grid_max(a, 0, half)
        mb, kb = plan.grid_max(b, 0, half)
        assert torch.equal(torch.cat([ma, mb]), Fm) and torch.equal(torch.cat([ka, kb]), km), cut
        got = []
        for part, off in ((a, 0), (b, cut)):
            r, c = plan.grid_crossings(part, 0, half, thr, 1 << 16)
            x = fstat.Plan.read_crossings(r, c)
            got += [(n + off, k, F) for n, k, F in zip(x["node"].tolist(), x["k"].tolist(), x["F"].tolist())]
        assert sorted(got) == want, cut


def test_argument_checks_with_a_plan():
    seg = small_segment(days=1, dt=13.0, seed=55, nfft=16384)
    banner("argument checks")
    plan = make_plan([seg], method.LINEAR_UP2, fstat.FP32)
    half = seg.fft_len // 2
    nodes = fstat.nodes_array([0.5], [0.1], [0.0])

    def status(fn):
        with pytest.raises(fstat.FStatError) as e:
            fn()
        return e.value.status

    assert status(lambda: plan.grid_map(nodes[:0], 0, half)) == fstat.EINVAL
    assert status(lambda: plan.grid_map(nodes, 0, half + 1)) == fstat.EINVAL
    assert status(lambda: plan.grid_map(nodes, 5, 5)) == fstat.EINVAL
    bad = nodes.copy()
    bad["seg"] = 1
    assert status(lambda: plan.grid_map(bad, 0, half)) == fstat.EINVAL
    bad = nodes.copy()
    bad["delta"] = float("nan")
    assert status(lambda: plan.grid_map(bad, 0, half)) == fstat.EINVAL
    out = fstat._Out(mode=fstat.OUT_MAP, interbin=2, k_lo=0, k_hi=half, F=1)
    assert status(lambda: plan._grid(nodes, out)) == fstat.EINVAL
    # plan-time checks: FFT length, whole sidereal days, a segment of gaps only
    x = seg.x
    det, eph = fstat.detector_spec(DET), fstat.ephemeris_spec(EPH)
    mk = lambda **kw: fstat.Plan([fstat.SegmentSpec(**{**dict(x=x, dt=seg.dt, n_days=1, f_ref=seg.f_ref), **kw})],
                                 det, eph)
    assert status(lambda: mk(nfft=12000)) == fstat.EUNSUPPORTED
    assert status(lambda: mk(nfft=4096)) == fstat.EUNSUPPORTED
    assert status(lambda: mk(n_days=2)) == fstat.ENOTINTDAYS
    assert status(lambda: mk(mask=np.zeros(len(x), dtype=np.uint8))) == fstat.EINVAL
    assert status(lambda: mk(x=np.r_[x[:-1], np.inf])) == fstat.EINVAL


def test_bin_params_of_two_segments():
    # fstat_bin_params: f = (k + bin_offset) / (nfft dt) of the node's own
    # segment; interbinned indices 2k + h are half bins; out-of-range bins and
    # segments are rejected
    s0 = small_segment(days=1, dt=13.0, seed=56, nfft=16384)
    s1 = small_segment(days=1, dt=26.0, seed=57, nfft=4096)
    banner("bin params")
    plan = make_plan([s0, s1], method.LINEAR_UP2, fstat.FP32)
    nodes = fstat.nodes_array([0.1, 0.2, 0.3], [0.4, -0.5, 0.6], [-1e-10, 0.0, -2e-10], seg=[0, 1, 1],
                              bin_offset=[0.0, 0.25, -0.375])
    k = [17, 2047, 0]
    p, sg = plan.bin_params(nodes, k)
    p, sg = p.cpu().numpy(), sg.cpu().numpy()
    want_f = [17 / (16384 * 13.0), (2047 + 0.25) / (4096 * 26.0), -0.375 / (4096 * 26.0)]
    assert np.allclose(p[:, 0], want_f, rtol=1e-15, atol=0)
    assert np.array_equal(p[:, 1:], np.stack([nodes["fdot"], nodes["alpha"], nodes["delta"]], axis=1))
    assert np.array_equal(sg, [0, 1, 1])
    pi, _ = plan.bin_params(nodes, [35, 4095, 1], interbin=True)
    want_i = [17.5 / (16384 * 13.0), (2047.5 + 0.25) / (4096 * 26.0), (0.5 - 0.375) / (4096 * 26.0)]
    assert np.allclose(pi.cpu().numpy()[:, 0], want_i, rtol=1e-15, atol=0)
    for bad_k, ib in (([17, 2048, 0], False), ([17, 4096, 0], True), ([-1, 0, 0], False)):
        with pytest.raises(fstat.FStatError) as e:
            plan.bin_params(nodes, bad_k, interbin=ib)
        assert e.value.status == fstat.EINVAL
    bad = nodes.copy()
    bad["seg"][0] = 2
    with pytest.raises(fstat.FStatError):
        plan.bin_params(bad, k)


@pytest.mark.parametrize("C,b2", [(1024, 16), (4096, 8), (2048, 0)])
def test_spill_write_probe_writes_the_first_pass_layout(C, b2):
    # every element of nodes x R x C written once, with (r, node) of its
    # writer at its place in the blocked [k2 / b2][r][k2 % b2] or row-major
    # [r][k2] layout; nothing past the end
    nodes, R = 3, 16
    banner("spill write probe", C, b2)
    buf = torch.full((nodes * R * C + 64, 4), -7.0, device="cuda")
    fstat.spill_write_probe(buf, nodes, R, C, b2)
    torch.cuda.synchronize()
    got = buf.cpu().numpy()
    i = np.arange(R * C)
    if b2:
        r = (i % (R * b2)) // b2
    else:
        r = i // C
    for n in range(nodes):
        blk = got[n * R * C:(n + 1) * R * C]
        assert np.array_equal(blk[:, 0], r) and np.all(blk[:, 1] == n)
        assert np.all(blk[:, 2] == 0.0) and np.all(blk[:, 3] == 1.0)
    assert np.all(got[nodes * R * C:] == -7.0)


@pytest.mark.parametrize("blocks", [0, 3])
def test_copy_probe_copies(blocks):
    banner("copy probe", blocks)
    src = torch.randn((1 << 22) + 4, device="cuda")
    dst = torch.zeros_like(src)
    fstat.copy_probe(dst, src, blocks)
    torch.cuda.synchronize()
    assert torch.equal(dst, src)
