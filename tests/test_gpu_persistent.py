"""The persistent launch (FSTAT_LAUNCH_PERSISTENT): the whole grid call as one
kernel over a queue of tiles.  Its outputs must equal, bit for bit, those of
the launch-per-pass path of a plan with the same FFT split (the same tile
code runs in both), and the oracle within the FP32 bar.

Segments of 2^18, 2^19 and 2^20 bins (R = 64, 128, 256 at C = 4096: both
spill layouts), gaps in one, four sky batches (the two sky sets are reused),
spill slots down to the minimum, claims of 1 to 64 tiles, all three output
modes, and graph replays."""
import numpy as np
import pytest
import torch

from oracle import method
from paper_1003_0844_amd import fstat, synth
from tests.common import DET, EPH, one_signal, small_segment
from tests.gpu_common import PREC_TOL, banner, f_error, oracle_map

pytestmark = pytest.mark.gpu

K_HI = 1 << 17   # bins common to all three segments


def _segments():
    sig = one_signal(71, band=1.0, snr=20.0)
    s0 = small_segment(days=1, dt=0.5, seed=71, signal=sig, nfft=1 << 18)
    mask = synth.gap_mask(synth.rng(72), 172328, 0.5, 0.1)
    s1 = small_segment(days=1, dt=0.5, seed=72, nfft=1 << 19, mask=mask)
    s2 = small_segment(days=1, dt=0.25, seed=73, nfft=1 << 20)
    return [s0, s1, s2], sig


def _nodes(sig):
    g = synth.rng(74)
    a0, d0 = synth.sky_uniform(g, 3)
    a1, d1 = synth.sky_uniform(g, 70)
    a2, d2 = synth.sky_uniform(g, 2)
    parts = [fstat.nodes_array(np.r_[sig["alpha"], np.repeat(a0, 2)], np.r_[sig["delta"], np.repeat(d0, 2)],
                               np.r_[sig["fdot"], np.tile([-3e-10, 0.0], 3)], seg=0),
             fstat.nodes_array(a1, d1, -5e-10, seg=1),
             fstat.nodes_array(np.repeat(a2, 3), np.repeat(d2, 3), np.tile([-1e-9, -4e-10, 0.0], 2), seg=2)]
    nodes = np.concatenate(parts)
    # interleave the segments in the caller's order: the library orders the work
    return nodes[np.random.default_rng(75).permutation(len(nodes))]


def _plan(segs, launch, autotune=False, interp=fstat.LINEAR_UP2):
    specs = [fstat.SegmentSpec(x=s.x, dt=s.dt, n_days=s.n_days, t0=s.t0, mask=s.mask, f_ref=s.f_ref,
                               sigma2=s.sigma2, nfft=s.nfft) for s in segs]
    return fstat.Plan(specs, fstat.detector_spec(DET), fstat.ephemeris_spec(EPH), interp=interp,
                      prec=fstat.FP32, device=0, autotune=autotune, launch=launch)


def _outputs(plan, nodes, thr):
    F = plan.grid_map(nodes, 0, K_HI).clone()
    Fmax, kmax = plan.grid_max(nodes, 0, K_HI)
    rec, cnt = plan.grid_crossings(nodes, 0, K_HI, thr, 1 << 20)
    torch.cuda.synchronize()
    xs = fstat.Plan.read_crossings(rec, cnt)
    return F, Fmax.clone(), kmax.clone(), int(cnt.cpu().item()), sorted(zip(xs["node"].tolist(), xs["k"].tolist(),
                                                                           xs["F"].tolist()))


@pytest.fixture(scope="module")
def case():
    segs, sig = _segments()
    nodes = _nodes(sig)
    banner("persistent: passes reference", [s.fft_len for s in segs], len(nodes))
    ref = _plan(segs, fstat.LAUNCH_PASSES)
    for i in range(3):
        assert ref.schedule(i)["C"] == 4096
    out = _outputs(ref, nodes, 9.0)
    del ref
    torch.cuda.empty_cache()
    return segs, sig, nodes, out


@pytest.mark.parametrize("slots,chunk", [(None, None), ("3", "1"), ("3", "64"), ("6", "8")])
def test_persistent_equals_passes(case, slots, chunk, monkeypatch):
    segs, sig, nodes, ref = case
    if slots:
        monkeypatch.setenv("FSTAT_PERSIST_SLOTS", slots)
    if chunk:
        monkeypatch.setenv("FSTAT_PERSIST_CHUNK", chunk)
    banner("persistent", "slots", slots, "chunk", chunk)
    plan = _plan(segs, fstat.LAUNCH_PERSISTENT)
    got = _outputs(plan, nodes, 9.0)
    plan.status()
    assert torch.equal(got[0], ref[0])
    assert torch.equal(got[1], ref[1]) and torch.equal(got[2], ref[2])
    assert got[3] == ref[3] and got[4] == ref[4]
    Fc = got[0].cpu().numpy()
    assert np.array_equal(got[1].cpu().numpy(), Fc.max(axis=1))
    assert np.array_equal(got[2].cpu().numpy(), Fc.argmax(axis=1))
    assert got[3] == int(np.sum(Fc > 9.0))


def test_persistent_against_oracle(case):
    segs, sig, nodes, ref = case
    banner("persistent oracle")
    plan = _plan(segs, fstat.LAUNCH_PERSISTENT)
    F = plan.grid_map(nodes, 0, K_HI).cpu().numpy()
    plan.status()
    for s in range(3):
        rows = np.nonzero(nodes["seg"] == s)[0][:2]
        for r in rows:
            nd = nodes[r]
            want = oracle_map(segs[s], nd["fdot"], nd["alpha"], nd["delta"], method.LINEAR_UP2, np.arange(K_HI))
            assert f_error(F[r], want) < PREC_TOL[fstat.FP32], (s, r, f_error(F[r], want))
    # the injection stands out at its own node
    r = int(np.nonzero((nodes["seg"] == 0) & (nodes["alpha"] == sig["alpha"]))[0][0])
    k0 = int(round(sig["f"] * segs[0].fft_len * segs[0].dt))
    assert 2 * F[r, k0 - 2:k0 + 3].max() > 100.0


def test_persistent_graph_replays(case):
    segs, sig, nodes, ref = case
    banner("persistent graph")
    plan = _plan(segs, fstat.LAUNCH_PERSISTENT)
    gm = plan.graph_map(nodes, 0, K_HI)
    gx = plan.graph_max(nodes, 0, K_HI)
    for rep in range(3):
        gm.outputs["F"].fill_(float("nan"))
        gx.outputs["Fmax"].fill_(-1.0)
        gx.outputs["kmax"].fill_(-1)
        torch.cuda.synchronize()
        gm.launch()
        gx.launch()
        torch.cuda.synchronize()
        assert torch.equal(gm.outputs["F"], ref[0]), rep
        assert torch.equal(gx.outputs["Fmax"], ref[1]) and torch.equal(gx.outputs["kmax"], ref[2]), rep
        # eager work of the same plan between the replays
        plan.grid_max(nodes[:5], 0, K_HI)
        torch.cuda.synchronize()
    gm.close()
    gx.close()
    plan.status()


@pytest.mark.parametrize("interp", [fstat.NEAREST, fstat.CUBIC_UP2])
def test_persistent_equals_passes_other_interpolations(case, interp):
    # the sky-record tiles of the other two resampling modes (Sec. VI A)
    segs, sig, nodes, ref = case
    banner("persistent interp", interp)
    sub = nodes[::3]
    want = _plan(segs, fstat.LAUNCH_PASSES, interp=interp)
    F0 = want.grid_map(sub, 0, K_HI).clone()
    m0, k0 = [t.clone() for t in want.grid_max(sub, 0, K_HI)]
    del want
    plan = _plan(segs, fstat.LAUNCH_PERSISTENT, interp=interp)
    F = plan.grid_map(sub, 0, K_HI)
    m, k = plan.grid_max(sub, 0, K_HI)
    torch.cuda.synchronize()
    plan.status()
    assert torch.equal(F, F0) and torch.equal(m, m0) and torch.equal(k, k0)
    assert not torch.equal(F, ref[0][::3])  # a different resampling does change the map


def test_an_expired_wait_stops_the_kernel_and_is_reported(case, monkeypatch):
    # waits bounded to 0 ticks: the first wait not satisfied at once expires,
    # sets the plan's flag, and every workgroup leaves the queue (the kernel
    # ends normally); fstat_plan_status reports it once and clears it
    segs, sig, nodes, ref = case
    monkeypatch.setenv("FSTAT_PERSIST_SPIN_TICKS", "0")
    banner("persistent expired wait")
    plan = _plan(segs, fstat.LAUNCH_PERSISTENT)
    F = plan.grid_map(nodes, 0, K_HI)
    with pytest.raises(fstat.FStatError) as e:
        plan.status()
    assert e.value.status == fstat.EDEVICE
    plan.status()  # cleared
    del F, plan
    monkeypatch.delenv("FSTAT_PERSIST_SPIN_TICKS")
    plan = _plan(segs, fstat.LAUNCH_PERSISTENT)
    assert torch.equal(plan.grid_map(nodes, 0, K_HI), ref[0])
    plan.status()


def test_calls_the_kernel_does_not_hold_run_as_passes():
    # interbinning, and an FFT length below 2^18, fall back to the passes
    seg = small_segment(days=1, dt=13.0, seed=76, nfft=16384)
    banner("persistent fallback")
    plan = _plan([seg], fstat.LAUNCH_PERSISTENT)
    ref = _plan([seg], fstat.LAUNCH_PASSES)
    nodes = fstat.nodes_array([0.3, 1.2], [0.1, -0.7], [0.0, -5e-10])
    assert torch.equal(plan.grid_map(nodes, 0, 8192), ref.grid_map(nodes, 0, 8192))
    assert torch.equal(plan.grid_map(nodes, 0, 8192, interbin=True), ref.grid_map(nodes, 0, 8192, interbin=True))
    plan.status()
