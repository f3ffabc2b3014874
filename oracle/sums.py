"""ctypes wrapper of the oracle's C summation loops (test infrastructure only).

``build()`` compiles ``sums.c`` with gcc + OpenMP into ``liboracle_sums.so``
beside it; ``lib()`` loads it (building on first use if it is missing).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sums.c")
_SO = os.path.join(_HERE, "liboracle_sums.so")
_lib = None

_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int64)


def build() -> str:
    """Compile the oracle's C part (plain C99 + OpenMP, FP64, no fast-math)."""
    tmp = _SO + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared",
                           "-fno-fast-math", "-ffp-contract=off", _SRC, "-o", tmp, "-lm"])
    os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_SO)
        L.osum_dft_bins.argtypes = [_D, _D, ctypes.c_int64, ctypes.c_int64, _I, ctypes.c_int64, _D, _D]
        L.osum_dft_freqs.argtypes = [_D, _D, ctypes.c_int64, ctypes.c_double, _D, ctypes.c_int64, _D, _D]
        L.osum_phase.argtypes = [_D, _D, _D, _D, ctypes.c_int64, _D, ctypes.c_int64, _D, _D, _D, _D]
        for fn in (L.osum_dft_bins, L.osum_dft_freqs, L.osum_phase):
            fn.restype = None
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(_D)


def dft_bins(z, nfft, k):
    """S_k = sum_{j<N} z_j exp(-2 pi i j k / nfft) for each k in ``k``."""
    z = np.asarray(z, dtype=np.complex128)
    zr, zi = np.ascontiguousarray(z.real), np.ascontiguousarray(z.imag)
    k = np.ascontiguousarray(np.asarray(k, dtype=np.int64))
    ore, oim = np.empty(k.size), np.empty(k.size)
    lib().osum_dft_bins(_p(zr), _p(zi), z.size, int(nfft), k.ctypes.data_as(_I), k.size, _p(ore), _p(oim))
    return ore + 1j * oim


def dft_freqs(z, dt, f):
    """S(f) = sum_j z_j exp(-2 pi i f j dt) for each f."""
    z = np.asarray(z, dtype=np.complex128)
    zr, zi = np.ascontiguousarray(z.real), np.ascontiguousarray(z.imag)
    f = np.ascontiguousarray(np.atleast_1d(np.asarray(f, dtype=np.float64)))
    ore, oim = np.empty(f.size), np.empty(f.size)
    lib().osum_dft_freqs(_p(zr), _p(zi), z.size, float(dt), _p(f), f.size, _p(ore), _p(oim))
    return ore + 1j * oim


def phase_sums(wa, wb, tau, psi, f):
    """S_a(f), S_b(f) = sum_j w_{a,b}[j] exp(-2 pi i (f tau_j + psi_j))."""
    arrs = [np.ascontiguousarray(np.asarray(v, dtype=np.float64)) for v in (wa, wb, tau, psi)]
    f = np.ascontiguousarray(np.atleast_1d(np.asarray(f, dtype=np.float64)))
    o = [np.empty(f.size) for _ in range(4)]
    lib().osum_phase(*[_p(v) for v in arrs], arrs[0].size, _p(f), f.size, *[_p(v) for v in o])
    return o[0] + 1j * o[1], o[2] + 1j * o[3]
