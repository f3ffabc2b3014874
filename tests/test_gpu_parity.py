"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Error metric for F: max_k |F_gpu - F_oracle| / max(F_oracle, 1); bars 1e-4
(FP32 path: FP64 phase, FP32 resample/FFT/combine) and 1e-10 (FP64 path)."""
import math

import numpy as np
import pytest
import torch

from oracle import method, model
from paper_1003_0844_amd import fstat, synth
from tests.common import DET, EPH, one_signal, small_segment
from tests.gpu_common import PREC_TOL, banner, f_error, make_plan, oracle_map

pytestmark = pytest.mark.gpu

MODES = [method.NEAREST, method.LINEAR_UP2, method.CUBIC_UP2]
PRECS = [fstat.FP32, fstat.FP64]


def _seg_with_signal(days=1, dt=13.0, seed=3, nfft=16384, snr=15.0, mask=None, sigma2=1.0):
    sig = one_signal(seed, band=1 / (2 * dt), snr=snr)
    seg = small_segment(days=days, dt=dt, seed=seed, signal=sig, nfft=nfft, mask=mask)
    seg.sigma2 = sigma2
    return seg, sig


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("mode", MODES)
def test_demodulated_series(prec, mode):
    # the FFT input: resampled, a/b-weighted, demodulated series of one node
    seg, sig = _seg_with_signal()
    banner("demod_series", "prec", prec, "interp", mode, "n", seg.n)
    plan = make_plan([seg], mode, prec)
    node = fstat.nodes_array(sig["alpha"], sig["delta"], sig["fdot"])
    got = plan.demod_series(node).cpu().numpy()
    za, zb = method.demodulated(seg, sig["fdot"], sig["alpha"], sig["delta"], DET, EPH, mode)
    ref = np.stack([za.real, za.imag, zb.real, zb.imag], axis=1)
    scale = np.max(np.abs(ref))
    tol = 1e-5 if prec == fstat.FP32 else 1e-11
    assert np.max(np.abs(got - ref)) < tol * scale


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("mode", MODES)
def test_grid_map_small(prec, mode):
    # 1 day at dt = 13 s: N = 6628 (not a multiple of the column count: ragged
    # tail), nfft = 2^14 -> 16 x 1024 tiles; 3 skies x 2 spindowns
    seg, sig = _seg_with_signal()
    banner("grid_map_small", "prec", prec, "interp", mode)
    plan = make_plan([seg], mode, prec)
    g = synth.rng(17)
    al, de = synth.sky_uniform(g, 2)
    alphas = np.repeat(np.r_[sig["alpha"], al], 2)
    deltas = np.repeat(np.r_[sig["delta"], de], 2)
    fdots = np.tile([sig["fdot"], -7e-10], 3)
    nodes = fstat.nodes_array(alphas, deltas, fdots)
    half = seg.fft_len // 2
    F = plan.grid_map(nodes, 0, half).cpu().numpy()
    k = np.arange(half)
    for i in range(len(nodes)):
        ref = oracle_map(seg, fdots[i], alphas[i], deltas[i], mode, k)
        err = f_error(F[i], ref)
        assert err < PREC_TOL[prec], (i, err)
    # the injected signal stands out at its node
    assert 2 * F[0].max() > 0.5 * sig["snr"] ** 2


@pytest.mark.parametrize("prec", PRECS)
def test_grid_map_tiny_workload(prec):
    # the 1-day dt = 2 s workload (N = 43082, nfft = 2^16) at its injected node
    w = synth.TINY
    g, x, sigs = synth.segment_data(w)
    p = sigs[0]
    x = x + model.injection(w.n, w.dt, 0.0, p, synth.F_REF, 1.0, DET, EPH)
    seg = method.Segment(x=x, dt=w.dt, n_days=w.days, f_ref=synth.F_REF, sigma2=1.0, nfft=w.nfft)
    banner("grid_map_tiny_workload", "prec", prec)
    plan = make_plan([seg], w.interp, prec)
    nodes = fstat.nodes_array(p["alpha"], p["delta"], p["fdot"])
    F = plan.grid_map(nodes, 0, w.nfft // 2).cpu().numpy()[0]
    ref = oracle_map(seg, p["fdot"], p["alpha"], p["delta"], w.interp, np.arange(w.nfft // 2))
    assert f_error(F, ref) < PREC_TOL[prec]
    # spot bins against the direct (term-by-term) DFT of the oracle
    kk = np.r_[0, 1, int(np.argmax(ref)), w.nfft // 2 - 1, 12345]
    ref_direct = method.fstat_bins(seg, p["fdot"], p["alpha"], p["delta"], DET, EPH, w.interp, k=kk, dft="direct")
    assert f_error(F[kk], ref_direct) < PREC_TOL[prec]
    k0 = int(round(p["f"] * w.nfft * w.dt))
    assert abs(int(np.argmax(F)) - k0) <= 2


@pytest.mark.parametrize("prec", PRECS)
def test_output_modes_agree(prec):
    seg, sig = _seg_with_signal(seed=5)
    banner("output_modes", "prec", prec)
    plan = make_plan([seg], method.LINEAR_UP2, prec)
    g = synth.rng(23)
    al, de = synth.sky_uniform(g, 3)
    nodes = fstat.nodes_array(np.r_[sig["alpha"], al], np.r_[sig["delta"], de], np.r_[sig["fdot"], -1e-10, 0, -5e-10])
    k_lo, k_hi = 100, 7000
    F = plan.grid_map(nodes, k_lo, k_hi).cpu().numpy()
    Fmax, kmax = plan.grid_max(nodes, k_lo, k_hi)
    Fmax, kmax = Fmax.cpu().numpy(), kmax.cpu().numpy()
    assert np.array_equal(Fmax, F.max(axis=1))
    assert np.array_equal(kmax, F.argmax(axis=1) + k_lo)
    thr = 6.0
    rec, cnt = plan.grid_crossings(nodes, k_lo, k_hi, thr, 100000)
    cnt = int(cnt.cpu().item())
    rec = fstat.Plan.read_crossings(rec, torch.tensor([cnt]))
    exp = np.argwhere(F > thr)
    assert cnt == exp.shape[0] == rec.size
    got = sorted((int(a), int(b)) for a, b in zip(rec["node"], rec["k"]))
    assert got == sorted((int(i), int(j) + k_lo) for i, j in exp)
    # each record carries the F of its own (node, bin)
    assert np.array_equal(rec["F"], F[rec["node"], rec["k"] - k_lo].astype(np.float64))
    # an overflowing buffer keeps the count and drops the excess records
    rec2, cnt2 = plan.grid_crossings(nodes, k_lo, k_hi, thr, 5)
    assert int(cnt2.cpu().item()) == cnt
    assert fstat.Plan.read_crossings(rec2, cnt2).size == 5
    # a band subset is the same numbers as the full map
    Ffull = plan.grid_map(nodes, 0, seg.fft_len // 2).cpu().numpy()
    assert np.array_equal(Ffull[:, k_lo:k_hi], F)


@pytest.mark.parametrize("prec", PRECS)
def test_gaps_and_estimated_variance(prec):
    dt = 13.0
    n = int(2 * synth.SIDEREAL_DAY / dt)
    mask = synth.gap_mask(synth.rng(31), n, dt, max_frac=0.1)
    seg, sig = _seg_with_signal(days=2, dt=dt, seed=9, nfft=32768, mask=mask, sigma2=0.0)
    banner("gaps", "prec", prec, "gap fraction", 1 - mask.mean())
    plan = make_plan([seg], method.CUBIC_UP2, prec)
    assert abs(plan.info()["sigma2"] / seg.noise_var() - 1) < 1e-12
    nodes = fstat.nodes_array([sig["alpha"], 1.0], [sig["delta"], -0.5], [sig["fdot"], -3e-10])
    F = plan.grid_map(nodes, 0, seg.fft_len // 2).cpu().numpy()
    for i, nd in enumerate(nodes):
        ref = oracle_map(seg, nd["fdot"], nd["alpha"], nd["delta"], method.CUBIC_UP2, np.arange(seg.fft_len // 2))
        assert f_error(F[i], ref) < PREC_TOL[prec]


def test_multi_segment_plan_and_batching():
    # three segments of different lengths and FFT sizes in one plan; nodes
    # interleaved across segments; small batches force several launches
    segs, sigs = [], []
    for i, (days, dt, nfft) in enumerate([(1, 26.0, 8192), (2, 13.0, 32768), (1, 13.0, 16384)]):
        s, sg = _seg_with_signal(days=days, dt=dt, seed=40 + i, nfft=nfft)
        s.t0 = 1.0e6 * i
        segs.append(s)
        sigs.append(sg)
    # the injections above were made at t0 = 0: re-inject at the segment's own t0
    for s, sg in zip(segs, sigs):
        s.x = small_segment(days=s.n_days, dt=s.dt, seed=77, signal=sg, t0=s.t0, nfft=s.nfft).x
    banner("multi_segment")
    plan = make_plan(segs, method.LINEAR_UP2, fstat.FP32, max_batch=3)
    rows = []
    for rep in range(3):
        for i, sg in enumerate(sigs):
            rows.append((sg["alpha"] + 0.01 * rep, sg["delta"], sg["fdot"], i))
    rows = rows[::-1]
    nodes = fstat.nodes_array([r[0] for r in rows], [r[1] for r in rows], [r[2] for r in rows], [r[3] for r in rows])
    k_hi = 4096
    F = plan.grid_map(nodes, 0, k_hi).cpu().numpy()
    for i, (a, d, fd, s) in enumerate(rows):
        ref = oracle_map(segs[s], fd, a, d, method.LINEAR_UP2, np.arange(k_hi))
        assert f_error(F[i], ref) < 1e-4, i


@pytest.mark.parametrize("prec", PRECS)
def test_eval_and_gradient(prec):
    # F at continuous parameters and its adjoint gradient, against the oracle's
    # analytic gradient (itself pinned to central differences)
    dt = 13.0
    seg, sig = _seg_with_signal(days=1, dt=dt, seed=12, nfft=16384)
    banner("eval_and_gradient", "prec", prec)
    plan = make_plan([seg], method.CUBIC_UP2, prec)
    g = np.random.default_rng(8)
    T = seg.n * dt
    cell = np.array([1 / (seg.fft_len * dt), 1 / T ** 2, 0.01, 0.01])
    P = np.array([sig["f"], sig["fdot"], sig["alpha"], sig["delta"]]) + 0.5 * cell * g.choice([-1, 1], (6, 4))
    params = torch.tensor(P, dtype=torch.float64, device="cuda")
    F, dF = plan.grad(params)
    F, dF = F.cpu().numpy(), dF.cpu().numpy()
    for i in range(P.shape[0]):
        Fo, go = method.fstat_continuous(seg, P[i], DET, EPH, method.CUBIC_UP2, grad=True)
        assert abs(F[i] - Fo) / max(Fo, 1.0) < 1e-10
        scale = np.max(np.abs(go * cell))
        assert np.max(np.abs((dF[i] - go) * cell)) < 1e-9 * scale, (dF[i], go)


def test_autograd_function():
    dt = 13.0
    seg, sig = _seg_with_signal(days=1, dt=dt, seed=13, nfft=16384)
    banner("autograd")
    plan = make_plan([seg], method.LINEAR_UP2, fstat.FP32)
    P = torch.tensor([[sig["f"] + 1e-6, sig["fdot"], sig["alpha"] + 0.003, sig["delta"] - 0.002]] * 3,
                     dtype=torch.float64, device="cuda", requires_grad=True)
    w = torch.tensor([1.0, 2.0, -0.5], dtype=torch.float64, device="cuda")
    F = fstat.FStatFn.apply(P, plan)
    (F * w).sum().backward()
    F2, dF = plan.grad(P.detach())
    assert torch.equal(F.detach(), F2)
    assert torch.allclose(P.grad, w[:, None] * dF, rtol=1e-13, atol=0)


def test_grid_bin_equals_continuous_frequency():
    # the same quantity through the two entry points (FP64 plan)
    dt = 13.0
    seg, sig = _seg_with_signal(days=1, dt=dt, seed=14, nfft=16384)
    banner("cross_api")
    plan = make_plan([seg], method.LINEAR_UP2, fstat.FP64)
    nodes = fstat.nodes_array(sig["alpha"], sig["delta"], sig["fdot"])
    Fmap = plan.grid_map(nodes, 0, seg.fft_len // 2).cpu().numpy()[0]
    ks = np.array([0, 17, int(np.argmax(Fmap)), 5000])
    P = np.stack([ks / (seg.fft_len * dt), np.full(4, sig["fdot"]), np.full(4, sig["alpha"]),
                  np.full(4, sig["delta"])], axis=1)
    F, _ = plan.eval(torch.tensor(P, device="cuda"))
    assert f_error(F.cpu().numpy(), Fmap[ks]) < 1e-9


def test_repeated_calls_are_bitwise_identical():
    seg, sig = _seg_with_signal(seed=15)
    banner("determinism")
    plan = make_plan([seg], method.LINEAR_UP2, fstat.FP32)
    nodes = fstat.nodes_array([sig["alpha"], 0.3], [sig["delta"], 0.1], [sig["fdot"], 0.0])
    a = plan.grid_map(nodes, 0, seg.fft_len // 2).clone()
    b = plan.grid_map(nodes, 0, seg.fft_len // 2)
    assert torch.equal(a, b)


def test_autotuned_plan_and_cache(tmp_path, monkeypatch):
    # the tuner picks a valid split for nfft = 2^16 and the results still match
    # the oracle; a second plan reads the same choice back from the cache file
    w = synth.TINY
    g, x, sigs = synth.segment_data(w)
    p = sigs[0]
    x = x + model.injection(w.n, w.dt, 0.0, p, synth.F_REF, 1.0, DET, EPH)
    seg = method.Segment(x=x, dt=w.dt, n_days=w.days, f_ref=synth.F_REF, sigma2=1.0, nfft=w.nfft)
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("FSTAT_TUNE_CACHE", str(cache))
    banner("autotune")
    specs = [fstat.SegmentSpec(x=seg.x, dt=seg.dt, n_days=seg.n_days, f_ref=seg.f_ref, sigma2=1.0, nfft=w.nfft)]
    plan = fstat.Plan(specs, fstat.detector_spec(DET), fstat.ephemeris_spec(EPH), interp=w.interp,
                      prec=fstat.FP32, autotune=True)
    sch = plan.schedule()
    assert sch["C"] in (1024, 2048, 4096) and sch["R"] * sch["C"] == w.nfft and sch["batch"] in (32, 64, 128, 256)
    assert sch["streams"] in (1, 2)
    assert cache.read_text().startswith("fstat-tune-v3")
    nodes = fstat.nodes_array(np.full(3, p["alpha"]), np.full(3, p["delta"]), [p["fdot"], 0.0, -5e-10])
    F = plan.grid_map(nodes, 0, w.nfft // 2).cpu().numpy()
    for i, nd in enumerate(nodes):
        ref = oracle_map(seg, nd["fdot"], nd["alpha"], nd["delta"], w.interp, np.arange(w.nfft // 2))
        assert f_error(F[i], ref) < PREC_TOL[fstat.FP32]
    plan2 = fstat.Plan(specs, fstat.detector_spec(DET), fstat.ephemeris_spec(EPH), interp=w.interp,
                       prec=fstat.FP32, autotune=True)
    assert plan2.schedule() == sch
    assert len(cache.read_text().splitlines()) == 1


@pytest.mark.parametrize("C", [1024, 2048, 4096])
def test_every_split_gives_the_same_map(C, tmp_path, monkeypatch):
    # force each split through the cache file: same bins, FP32 rounding apart
    w = synth.TINY
    g, x, sigs = synth.segment_data(w)
    cache = tmp_path / "tune.txt"
    cache.write_text("fstat-tune-v3 0 %d %d %d %d 8 1\n" % (w.interp, w.nfft, w.n, C))
    monkeypatch.setenv("FSTAT_TUNE_CACHE", str(cache))
    banner("split", C)
    specs = [fstat.SegmentSpec(x=x, dt=w.dt, n_days=w.days, f_ref=synth.F_REF, sigma2=1.0, nfft=w.nfft)]
    plan = fstat.Plan(specs, fstat.detector_spec(DET), fstat.ephemeris_spec(EPH), interp=w.interp,
                      prec=fstat.FP32, autotune=True)
    assert plan.schedule()["C"] == C and plan.schedule()["batch"] == 8
    nodes = fstat.nodes_array([0.3, 2.0], [0.1, -0.7], [0.0, -5e-10])
    F = plan.grid_map(nodes, 0, w.nfft // 2).cpu().numpy()
    seg = method.Segment(x=x, dt=w.dt, n_days=w.days, f_ref=synth.F_REF, sigma2=1.0, nfft=w.nfft)
    for i, nd in enumerate(nodes):
        ref = oracle_map(seg, nd["fdot"], nd["alpha"], nd["delta"], w.interp, np.arange(w.nfft // 2))
        assert f_error(F[i], ref) < PREC_TOL[fstat.FP32]


@pytest.mark.parametrize("order", [(1, 2), (2, 1)])
def test_stream_modes_give_identical_outputs(order, tmp_path, monkeypatch):
    # two segments of different length (the second takes every other sample),
    # with the stream modes `order` (through the cache file), 20 nodes each in
    # batches of 8: the map, the per-node maxima and the threshold crossings
    # equal, bit for bit, those of plans forced to one stream and to two.
    # Order (2, 1) puts a two-stream segment before a one-stream one: the last
    # chunk's second pass on the side stream then runs beside the first pass 2
    # of the next segment on the caller's stream.
    w = synth.TINY
    g, x, sigs = synth.segment_data(w)
    x2 = np.ascontiguousarray(x[::2])
    n2 = len(x2)
    cache = tmp_path / "tune.txt"
    cache.write_text("fstat-tune-v3 0 %d %d %d 4096 8 %d\nfstat-tune-v3 0 %d %d %d 2048 8 %d\n"
                     % (w.interp, w.nfft, w.n, order[0], w.interp, w.nfft, n2, order[1]))
    monkeypatch.setenv("FSTAT_TUNE_CACHE", str(cache))
    banner("stream modes", order)
    specs = [fstat.SegmentSpec(x=x, dt=w.dt, n_days=w.days, f_ref=synth.F_REF, sigma2=1.0, nfft=w.nfft),
             fstat.SegmentSpec(x=x2, dt=2 * w.dt, n_days=w.days, f_ref=synth.F_REF, sigma2=1.0, nfft=w.nfft)]
    rng = np.random.default_rng(17)
    nodes = np.concatenate([fstat.nodes_array(rng.uniform(0, 2 * math.pi, 20), rng.uniform(-1.4, 1.4, 20),
                                              rng.uniform(-1e-9, 0, 20), seg=s) for s in (0, 1)])
    half = w.nfft // 2
    res = {}
    for force in (None, "1", "2"):
        if force is None:
            monkeypatch.delenv("FSTAT_STREAMS", raising=False)
        else:
            monkeypatch.setenv("FSTAT_STREAMS", force)
        plan = fstat.Plan(specs, fstat.detector_spec(DET), fstat.ephemeris_spec(EPH), interp=w.interp,
                          prec=fstat.FP32, autotune=True)
        want = order if force is None else (int(force), int(force))
        assert (plan.schedule(0)["streams"], plan.schedule(1)["streams"]) == want
        assert plan.schedule(0)["batch"] == 8 and plan.schedule(1)["C"] == 2048
        F = plan.grid_map(nodes, 0, half).clone()
        Fmax, kmax = plan.grid_max(nodes, 0, half)
        rec, cnt = plan.grid_crossings(nodes, 0, half, 7.0, 200000)
        torch.cuda.synchronize()
        xs = fstat.Plan.read_crossings(rec, cnt)
        res[force] = (F, Fmax.clone(), kmax.clone(), int(cnt.cpu().item()),
                      sorted((int(a), int(b), float(c)) for a, b, c in zip(xs["node"], xs["k"], xs["F"])))
        del plan
    monkeypatch.delenv("FSTAT_STREAMS", raising=False)
    for force in ("1", "2"):
        a, b = res[None], res[force]
        assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]) and torch.equal(a[2], b[2]), force
        assert a[3] == b[3] and a[4] == b[4], force
    F, Fmax, kmax, cnt, xs = res[None]
    Fc = F.cpu().numpy()
    assert np.array_equal(Fmax.cpu().numpy(), Fc.max(axis=1))
    assert np.array_equal(kmax.cpu().numpy(), Fc.argmax(axis=1))
    assert cnt == int(np.sum(Fc > 7.0)) == len(xs)
    # and rows of both segments still match the oracle
    segs = [method.Segment(x=x, dt=w.dt, n_days=w.days, f_ref=synth.F_REF, sigma2=1.0, nfft=w.nfft),
            method.Segment(x=x2, dt=2 * w.dt, n_days=w.days, f_ref=synth.F_REF, sigma2=1.0, nfft=w.nfft)]
    for i in (0, 19, 20, 39):
        nd = nodes[i]
        ref = oracle_map(segs[int(nd["seg"])], nd["fdot"], nd["alpha"], nd["delta"], w.interp, np.arange(half))
        assert f_error(Fc[i], ref) < PREC_TOL[fstat.FP32], i
