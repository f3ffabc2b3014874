"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module only draws random numbers and lays out workloads (sizes, grids,
noise, gap masks, signal parameters).  It holds none of the method's
arithmetic: signals are *drawn* here as parameter sets, and turned into
waveforms elsewhere.

All randomness is numpy PCG64 with an explicit seed.  Draw order inside a
workload is fixed: noise, then signal parameters, then sky grid, then gaps.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

SIDEREAL_DAY = 86164.0        # s; observation spans are whole numbers of these
F_REF = 435.1875              # Hz, lower edge of the band (the paper's MC band)


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def white_noise(g: np.random.Generator, n: int, sigma: float = 1.0) -> np.ndarray:
    return g.normal(0.0, sigma, size=n).astype(np.float64)


def sky_uniform(g: np.random.Generator, count: int):
    """Points uniform on the sphere: alpha ~ U(0, 2pi), sin(delta) ~ U(-1, 1)."""
    alpha = g.uniform(0.0, 2.0 * math.pi, size=count)
    delta = np.arcsin(g.uniform(-1.0, 1.0, size=count))
    return alpha, delta


def spindown_grid(count: int, lo: float = -1e-9, hi: float = 0.0) -> np.ndarray:
    return np.linspace(lo, hi, count) if count > 1 else np.array([lo])


def signal_params(g: np.random.Generator, count: int, band: float, snr=(10.0, 10.0),
                  fdot=(-1e-9, 0.0), f=None):
    """Random signal parameter sets: f ~ U(0.05, 0.95) band unless given,
    fdot ~ U(fdot), sky uniform, cos(iota) ~ U(-1,1), psi ~ U(0, pi),
    phi0 ~ U(0, 2 pi), SNR ~ U(snr)."""
    out = []
    for _ in range(count):
        p = dict(f=float(g.uniform(0.05, 0.95) * band) if f is None else float(f),
                 fdot=float(g.uniform(*fdot)) if fdot[0] != fdot[1] else float(fdot[0]),
                 alpha=float(g.uniform(0.0, 2 * math.pi)),
                 delta=float(math.asin(g.uniform(-1.0, 1.0))),
                 cosi=float(g.uniform(-1.0, 1.0)),
                 psi=float(g.uniform(0.0, math.pi)),
                 phi0=float(g.uniform(0.0, 2 * math.pi)),
                 snr=float(g.uniform(*snr)) if snr[0] != snr[1] else float(snr[0]))
        out.append(p)
    return out


def gap_mask(g: np.random.Generator, n: int, dt: float, max_frac: float = 0.10,
             block_s=(60.0, 3600.0)) -> np.ndarray:
    """Detector-downtime-like gaps: a target zeroed fraction ~ U(0, max_frac),
    made of contiguous blocks of U(block_s) seconds at random starts.
    Returns uint8, 1 = data, 0 = gap."""
    m = np.ones(n, dtype=np.uint8)
    target = g.uniform(0.0, max_frac) * n
    zeroed = 0
    while zeroed < target:
        length = max(1, int(g.uniform(*block_s) / dt))
        start = int(g.integers(0, n))
        stop = min(n, start + length)
        zeroed += int(np.sum(m[start:stop]))
        m[start:stop] = 0
    return m


@dataclass(frozen=True)
class Workload:
    """Sizes of one named workload."""
    name: str
    days: int
    dt: float
    nfft: int
    n_sky: int
    n_fdot: int
    interp: int          # 0 nearest, 1 linear on the 2x-upsampled series, 2 cubic
    n_signals: int
    seed: int

    @property
    def n(self) -> int:
        return int(round(self.days * SIDEREAL_DAY / self.dt))

    @property
    def n_nodes(self) -> int:
        return self.n_sky * self.n_fdot


# The configurations the method is exercised on (sizes from the workload
# descriptions: 1-day dt=2 s single node; 2-day dt=0.5 s all-sky grid; 6-day
# dt=0.5 s large grid).
TINY = Workload("1 day, dt=2 s, N=43082, nfft=2^16, 1 node", 1, 2.0, 1 << 16, 1, 1, 1, 1, 1000)
GRID2D = Workload("2 days, dt=0.5 s, N=344656, nfft=2^20, 1024 sky x 16 fdot",
                  2, 0.5, 1 << 20, 1024, 16, 1, 8, 1001)
LARGE6D = Workload("6 days, dt=0.5 s, N=1033968, nfft=2^21, 8192 sky x 32 fdot",
                   6, 0.5, 1 << 21, 8192, 32, 1, 32, 1004)


def segment_data(w: Workload, sigma: float = 1.0):
    """Noise series and the signal parameter sets of a workload (the signals
    themselves are synthesised by the caller)."""
    g = rng(w.seed)
    x = white_noise(g, w.n, sigma)
    band = 1.0 / (2.0 * w.dt)
    if w.n_signals == 1:
        sig = signal_params(g, 1, band, snr=(10.0, 10.0), fdot=(-1e-10, -1e-10), f=0.1)
    else:
        sig = signal_params(g, w.n_signals, band,
                            snr=(6.0, 20.0) if w.n_signals > 8 else (10.0, 10.0))
    return g, x, sig


@dataclass(frozen=True)
class UnevenSegments:
    """Many segments of different whole-day lengths with gaps, each with its
    own small sky x spindown grid (dt = 0.5 s, nfft = nextpow2(2N))."""
    name: str
    n_seg: int
    days: tuple          # inclusive range of the per-segment length in sidereal days
    dt: float
    max_gap_frac: float
    n_sky: int           # per segment
    n_fdot: int          # per segment
    seed: int


UNEVEN = UnevenSegments("256 segments of 1-6 days, dt=0.5 s, 0-10% gaps, 64 sky x 8 fdot each",
                        256, (1, 6), 0.5, 0.10, 64, 8, 1002)


def uneven_segments(u: UnevenSegments, sigma: float = 1.0):
    """Per segment: (days, t0, noise x, gap mask), back to back in time, and the
    grid of every segment as (alpha, delta, fdot) arrays.  Draw order: segment
    lengths, noise, sky grids, gaps."""
    g = rng(u.seed)
    days = g.integers(u.days[0], u.days[1] + 1, size=u.n_seg)
    t0 = np.concatenate([[0.0], np.cumsum(days[:-1]) * SIDEREAL_DAY])
    xs = [white_noise(g, int(round(d * SIDEREAL_DAY / u.dt)), sigma) for d in days]
    grids = []
    fd = spindown_grid(u.n_fdot)
    for _ in range(u.n_seg):
        a, dl = sky_uniform(g, u.n_sky)
        grids.append((np.repeat(a, u.n_fdot), np.repeat(dl, u.n_fdot), np.tile(fd, u.n_sky)))
    masks = [gap_mask(g, len(x), u.dt, u.max_gap_frac) for x in xs]
    return [(int(d), float(t), x, m) for d, t, x, m in zip(days, t0, xs, masks)], grids


def candidate_offsets(seed: int, count: int, n_par: int = 4) -> np.ndarray:
    """Random signs (+1/-1) per candidate and parameter, for candidates placed
    half a cell away from a point in every parameter."""
    return rng(seed).choice(np.array([-1.0, 1.0]), size=(count, n_par))
