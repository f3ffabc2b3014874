"""Fine search on the GPU (Sec. VI C): exact F by direct summation on the
detector samples, and the Nelder-Mead search from coarse candidates, against
the oracle."""
import math

import numpy as np
import pytest
import torch

from oracle import method
from paper_1003_0844_amd import fstat, synth
from tests.common import DET, EPH, one_signal, small_segment
from tests.gpu_common import banner, make_plan

pytestmark = pytest.mark.gpu


def _case(seed, gaps):
    dt = 13.0
    n = int(round(synth.SIDEREAL_DAY / dt))
    mask = synth.gap_mask(synth.rng(70 + seed), n, dt, 0.1) if gaps else None
    sig = one_signal(seed, band=1 / (2 * dt), snr=20.0)
    seg = small_segment(days=1, dt=dt, seed=seed, signal=sig, mask=mask)
    return seg, sig


def _cells(seg):
    T = seg.n * seg.dt
    df = 1.0 / (seg.fft_len * seg.dt)
    v_c = 2 * math.pi * 1.495978707e11 / (365.256363004 * 86400.0) / 299792458.0
    return np.array([df, 1.0 / T ** 2, df / (seg.f_ref * v_c), df / (seg.f_ref * v_c)])


@pytest.mark.parametrize("gaps", [False, True])
def test_exact_F_matches_oracle(gaps):
    seg, sig = _case(31, gaps)
    banner("exact F", "gaps", gaps)
    plan = make_plan([seg], method.LINEAR_UP2, fstat.FP64)
    cell = _cells(seg)
    truth = np.array([sig["f"], sig["fdot"], sig["alpha"], sig["delta"]])
    P = truth + cell * np.random.default_rng(2).uniform(-2, 2, (5, 4))
    F = plan.eval_exact(torch.tensor(P, device="cuda")).cpu().numpy()
    for i in range(P.shape[0]):
        ref = method.fstat_exact(seg, P[i, 0], P[i, 1], P[i, 2], P[i, 3], DET, EPH)
        assert abs(F[i] - ref) / max(abs(ref), 1.0) < 1e-10, (i, F[i], ref)


@pytest.mark.parametrize("exact", [True, False])
def test_refine_reaches_the_oracles_maximum(exact):
    seg, sig = _case(32, True)
    banner("refine", "exact", exact)
    plan = make_plan([seg], method.CUBIC_UP2, fstat.FP64)
    cell = _cells(seg)
    truth = np.array([sig["f"], sig["fdot"], sig["alpha"], sig["delta"]])
    starts = truth + 0.5 * cell * synth.candidate_offsets(33, 4)
    pout, F, ev = plan.refine(torch.tensor(starts, device="cuda"), scale=0.5 * cell, tol=1e-4, max_evals=2000,
                              exact=exact)
    pout, F, ev = pout.cpu().numpy(), F.cpu().numpy(), ev.cpu().numpy()
    if exact:
        fun = lambda x: method.fstat_exact(seg, x[0], x[1], x[2], x[3], DET, EPH)
    else:
        fun = lambda x: method.fstat_continuous(seg, x, DET, EPH, method.CUBIC_UP2)
    for i in range(starts.shape[0]):
        F0 = fun(starts[i])
        assert F[i] >= F0 and ev[i] < 2000
        # the reported F is F at the reported point
        assert abs(F[i] - fun(pout[i])) < 1e-9 * F[i]
        # the oracle's search from the same start reaches the same maximum
        xo, Fo, _ = method.nelder_mead_max(fun, starts[i], 0.5 * cell, 1e-4, 2000)
        assert abs(F[i] - Fo) < 1e-5 * Fo, (i, F[i], Fo)
        assert np.max(np.abs((pout[i] - xo) / cell)) < 0.05, (i, (pout[i] - xo) / cell)
        # and no point of a small lattice around it is higher
        g = np.random.default_rng(i)
        for _ in range(8):
            assert fun(pout[i] + 0.02 * cell * g.uniform(-1, 1, 4)) <= F[i] * (1 + 1e-9)


def test_refine_invalid_segment_gives_nan():
    seg, sig = _case(34, False)
    banner("refine invalid segment")
    plan = make_plan([seg], method.LINEAR_UP2, fstat.FP64)
    P = torch.tensor([[sig["f"], sig["fdot"], sig["alpha"], sig["delta"]]] * 2, dtype=torch.float64, device="cuda")
    pout, F, ev = plan.refine(P, scale=_cells(seg), seg=torch.tensor([0, 3], dtype=torch.int32), max_evals=50)
    assert np.isfinite(F[0].item()) and np.isnan(F[1].item()) and int(ev[1].item()) == 0
