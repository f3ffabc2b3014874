"""Oracle evaluations run in worker processes (spawned: they import numpy and
the oracle only, never torch or the HIP library), for the full-size GPU
tests whose expected values take seconds per node."""
import multiprocessing as mp
import os

import numpy as np

from oracle import method, model


def _fstat_bins_job(job):
    x, mask, dt, days, t0, f_ref, nfft, fdot, alpha, delta, mode = job
    seg = method.Segment(x=x, dt=dt, n_days=days, t0=t0, mask=mask, f_ref=f_ref, sigma2=1.0, nfft=nfft)
    return method.fstat_bins(seg, fdot, alpha, delta, model.default_detector(), model.Ephemeris(), mode,
                             k=None, dft="fft")


def full_band_maps(jobs, workers=12):
    """F on every bin [0, nfft/2) for each job (x, mask, dt, days, t0, f_ref,
    nfft, fdot, alpha, delta, mode), in parallel processes."""
    workers = max(1, min(workers, len(jobs), len(os.sched_getaffinity(0)), 16))
    if workers == 1:
        return [_fstat_bins_job(j) for j in jobs]
    with mp.get_context("spawn").Pool(workers) as pool:
        return pool.map(_fstat_bins_job, jobs, chunksize=1)
