"""The grid evaluation recorded once as a HIP graph (fstat_graph_create) and
replayed: every replay must write exactly what the eager fstat_grid call
writes, with other eager GPU work and synchronisations between replays, and an
uneven multi-segment node list with gaps must match the oracle."""
import numpy as np
import pytest
import torch

from oracle import method
from paper_1003_0844_amd import fstat, synth
from tests.common import one_signal, small_segment
from tests.gpu_common import PREC_TOL, banner, f_error, make_plan, oracle_map

pytestmark = pytest.mark.gpu


def _segment(days, dt, seed, nfft, gaps=0.0):
    n = int(round(days * synth.SIDEREAL_DAY / dt))
    mask = synth.gap_mask(synth.rng(seed + 500), n, dt, max_frac=gaps) if gaps > 0 else None
    sig = one_signal(seed, band=1 / (2 * dt), snr=15.0)
    seg = small_segment(days=days, dt=dt, seed=seed, signal=sig, nfft=nfft, mask=mask)
    return seg, sig


def _nodes(sig, n_sky, fdots, seed, seg=0):
    al, de = synth.sky_uniform(synth.rng(seed), n_sky - 1)
    alphas = np.repeat(np.r_[sig["alpha"], al], len(fdots))
    deltas = np.repeat(np.r_[sig["delta"], de], len(fdots))
    fd = np.tile(fdots, n_sky)
    return fstat.nodes_array(alphas, deltas, fd, seg)


def _other_eager_work(plan, nodes, half):
    # eager grid work on the same plan and unrelated torch work between replays
    plan.grid_map(nodes[::-1].copy(), 0, half // 2)
    a = torch.randn(1 << 20, device="cuda")
    (a * 2.0).sum().item()
    torch.cuda.synchronize()


@pytest.mark.parametrize("prec", [fstat.FP32, fstat.FP64])
def test_graph_replays_equal_eager(prec):
    seg, sig = _segment(days=1, dt=13.0, seed=5, nfft=16384)
    banner("graph replays", "prec", prec)
    plan = make_plan([seg], method.LINEAR_UP2, prec, max_batch=2)
    nodes = _nodes(sig, 3, [sig["fdot"], -5e-10], seed=21)
    half = seg.fft_len // 2
    F_eager = plan.grid_map(nodes, 0, half).clone()
    Fmax_e, kmax_e = plan.grid_max(nodes, 0, half)
    thr = float(torch.quantile(F_eager.double().flatten()[:1 << 16], 0.999).item())
    rec_e, cnt_e = plan.grid_crossings(nodes, 0, half, thr, 4096)
    cross_e = np.sort(fstat.Plan.read_crossings(rec_e, cnt_e), order=["node", "k"])
    torch.cuda.synchronize()

    g_map = plan.graph_map(nodes, 0, half)
    g_max = plan.graph_max(nodes, 0, half)
    g_x = plan.graph_crossings(nodes, 0, half, thr, 4096)
    for rep in range(3):
        g_map.outputs["F"].fill_(float("nan"))
        g_max.outputs["Fmax"].fill_(-1.0)
        g_max.outputs["kmax"].fill_(-1)
        g_x.outputs["cnt"].fill_(12345)
        torch.cuda.synchronize()
        g_map.launch()
        g_max.launch()
        g_x.launch()
        torch.cuda.synchronize()
        assert torch.equal(g_map.outputs["F"], F_eager), rep
        assert torch.equal(g_max.outputs["Fmax"], Fmax_e), rep
        assert torch.equal(g_max.outputs["kmax"], kmax_e), rep
        assert int(g_x.outputs["cnt"].item()) == int(cnt_e.item()), rep
        cross_g = np.sort(fstat.Plan.read_crossings(g_x.outputs["rec"], g_x.outputs["cnt"]), order=["node", "k"])
        assert np.array_equal(cross_g, cross_e), rep
        _other_eager_work(plan, nodes, half)
    for g in (g_map, g_max, g_x):
        g.close()


def test_graph_uneven_segments_with_gaps():
    # segments of 1, 2 and 3 sidereal days with 0-10 % gaps, three FFT sizes,
    # nodes of every segment interleaved, in one graph
    specs = [(1, 26.0, 8192), (3, 26.0, 32768), (2, 13.0, 32768), (1, 13.0, 16384)]
    segs, sigs = [], []
    for i, (days, dt, nfft) in enumerate(specs):
        s, sg = _segment(days, dt, seed=60 + i, nfft=nfft, gaps=0.1)
        segs.append(s)
        sigs.append(sg)
    banner("graph uneven segments", [(s.n, s.fft_len) for s in segs])
    plan = make_plan(segs, method.LINEAR_UP2, fstat.FP32, max_batch=4)
    parts = [_nodes(sg, 3, [sg["fdot"], -4e-10], seed=80 + i, seg=i) for i, sg in enumerate(sigs)]
    nodes = np.concatenate(parts)[np.random.default_rng(3).permutation(sum(len(p) for p in parts))]
    k_hi = 4096
    g = plan.graph_map(nodes, 0, k_hi)
    F_eager = plan.grid_map(nodes, 0, k_hi)
    for rep in range(2):
        g.outputs["F"].zero_()
        torch.cuda.synchronize()
        g.launch()
        torch.cuda.synchronize()
        assert torch.equal(g.outputs["F"], F_eager), rep
    F = g.outputs["F"].cpu().numpy()
    for i, nd in enumerate(nodes):
        s = segs[nd["seg"]]
        ref = oracle_map(s, nd["fdot"], nd["alpha"], nd["delta"], method.LINEAR_UP2, np.arange(k_hi))
        assert f_error(F[i], ref) < PREC_TOL[fstat.FP32], i
    g.close()
