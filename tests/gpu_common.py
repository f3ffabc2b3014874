"""Helpers for the GPU parity tests: the same seeded inputs go to the oracle and
to the HIP library; expected values come only from the oracle."""
import sys

import numpy as np

from oracle import method
from paper_1003_0844_amd import fstat
from tests.common import DET, EPH

PREC_TOL = {fstat.FP32: 1e-4, fstat.FP64: 1e-10}


def banner(*what):
    """Name the case on stdout before any GPU work (flushed)."""
    print("[gpu case]", *what, flush=True)
    sys.stdout.flush()


def make_plan(segs, interp, prec, max_batch=0):
    specs = [fstat.SegmentSpec(x=s.x, dt=s.dt, n_days=s.n_days, t0=s.t0, mask=s.mask, f_ref=s.f_ref,
                               sigma2=s.sigma2, nfft=s.nfft) for s in segs]
    return fstat.Plan(specs, fstat.detector_spec(DET), fstat.ephemeris_spec(EPH), interp=interp, prec=prec,
                      device=0, max_batch=max_batch)


def oracle_map(seg, fdot, alpha, delta, mode, k):
    return method.fstat_bins(seg, fdot, alpha, delta, DET, EPH, mode, k=k, dft="fft")


def f_error(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.max(np.abs(got - ref) / np.maximum(np.abs(ref), 1.0)))
