"""Python binding of libfstat.so (include/fstat.h): argument marshalling only.

Device memory comes from torch tensors on the plan's GPU and work runs on the
current torch stream of that device; every arithmetic step of the method runs
in the HIP kernels of the library.  If the library is missing or cannot be
loaded, importing this module raises: there is no fallback.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# FSTAT_LIBRARY names another build of the same library (e.g. the host
# sanitizer build of _build.build_library(sanitize=True)); default: in-tree.
LIB_PATH = os.environ.get("FSTAT_LIBRARY") or os.path.join(_HERE, "libfstat.so")

NEAREST, LINEAR_UP2, CUBIC_UP2 = 0, 1, 2
FP32, FP64 = 0, 1
OUT_MAP, OUT_MAX, OUT_CROSSINGS = 0, 1, 2
STATE = 8
GRAD_STATIC_MAX = 65536

OK, EINVAL, ENOTINTDAYS, ENOMEM, EDEVICE, EUNSUPPORTED = 0, -1, -2, -3, -4, -5

C_LIGHT = 299_792_458.0
AU = 1.495978707e11
R_EARTH = 6.378140e6
SIDEREAL_DAY = 86164.0
YEAR = 365.256363004 * 86400.0


class FStatError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__("%s: %s (%d)" % (what, lib().fstat_strerror(status).decode(), status))
        self.status = status


# --------------------------------------------------------------------------
# C structures
# --------------------------------------------------------------------------
class _Detector(ctypes.Structure):
    _fields_ = [("lat_rad", ctypes.c_double), ("lon_rad", ctypes.c_double), ("gamma_rad", ctypes.c_double),
                ("zeta_rad", ctypes.c_double), ("radius_m", ctypes.c_double)]


class _Ephemeris(ctypes.Structure):
    _fields_ = [("obliquity_rad", ctypes.c_double), ("orbit_radius_m", ctypes.c_double),
                ("orbit_omega", ctypes.c_double), ("orbit_phase0", ctypes.c_double),
                ("sidereal_day_s", ctypes.c_double), ("gmst0_rad", ctypes.c_double)]


class _Lattice(ctypes.Structure):
    _fields_ = [("basis", ctypes.c_double * 16), ("gamma", ctypes.c_double * 16), ("dp0", ctypes.c_double),
                ("c0", ctypes.c_double), ("R", ctypes.c_double), ("mu", ctypes.c_double), ("nu", ctypes.c_double),
                ("theta", ctypes.c_double), ("margin_w1", ctypes.c_double), ("margin_sky", ctypes.c_double),
                ("rule", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class _LatticeRegion(ctypes.Structure):
    _fields_ = [("f_sky_hz", ctypes.c_double), ("fdot_lo", ctypes.c_double), ("fdot_hi", ctypes.c_double),
                ("sky_c1", ctypes.c_double), ("sky_c2", ctypes.c_double), ("sky_radius", ctypes.c_double),
                ("hemisphere", ctypes.c_int32), ("seg", ctypes.c_int32)]


class _Segment(ctypes.Structure):
    _fields_ = [("x", ctypes.POINTER(ctypes.c_double)), ("n", ctypes.c_int64), ("dt", ctypes.c_double),
                ("n_sidereal_days", ctypes.c_int32), ("t0", ctypes.c_double),
                ("mask", ctypes.POINTER(ctypes.c_uint8)), ("f_ref_hz", ctypes.c_double),
                ("sigma2", ctypes.c_double), ("nfft", ctypes.c_int64)]


class _Options(ctypes.Structure):
    _fields_ = [("interp", ctypes.c_int32), ("prec", ctypes.c_int32), ("device", ctypes.c_int32),
                ("max_batch", ctypes.c_int32), ("autotune", ctypes.c_int32), ("launch", ctypes.c_int32)]


class _Out(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("interbin", ctypes.c_int32), ("k_lo", ctypes.c_int64),
                ("k_hi", ctypes.c_int64), ("threshold", ctypes.c_double), ("F", ctypes.c_void_p),
                ("Fmax", ctypes.c_void_p), ("kmax", ctypes.c_void_p), ("crossings", ctypes.c_void_p),
                ("n_crossings", ctypes.c_void_p), ("max_crossings", ctypes.c_int64)]


class _RefineOptions(ctypes.Structure):
    _fields_ = [("scale", ctypes.c_double * 4), ("tol", ctypes.c_double), ("max_evals", ctypes.c_int32),
                ("exact", ctypes.c_int32)]


NODE_DTYPE = np.dtype([("alpha", "<f8"), ("delta", "<f8"), ("fdot", "<f8"), ("seg", "<i4"), ("bin_offset", "<f4")])
CROSSING_DTYPE = np.dtype([("node", "<i8"), ("k", "<i8"), ("F", "<f8")])

EXPORTS = ("fstat_plan", "fstat_grid", "fstat_graph_create", "fstat_graph_launch", "fstat_graph_destroy",
           "fstat_eval", "fstat_eval_exact", "fstat_refine", "fstat_threshold", "fstat_adjoint", "fstat_amplitudes",
           "fstat_grad", "fstat_grad_static", "fstat_plan_info", "fstat_demod_series",
           "fstat_lattice_fisher", "fstat_lattice_build", "fstat_lattice_segment", "fstat_lattice_nodes",
           "fstat_copy_probe", "fstat_spill_write_probe", "fstat_bin_params",
           "fstat_profile",
           "fstat_profile_read", "fstat_plan_schedule", "fstat_plan_status", "fstat_destroy", "fstat_strerror")
K_SKY, K_PASS1, K_PASS2, K_OTHER = 0, 1, 2, 3
NU_DEEP_HOLES, NU_COVERING = 0, 1
LAUNCH_PASSES, LAUNCH_PERSISTENT = 0, 1

_lib = None


def lib():
    """The loaded library.  Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libfstat.so is not built (run __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, i32, P = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.POINTER
        L.fstat_plan.argtypes = [P(_Segment), i32, P(_Detector), P(_Ephemeris), P(_Options), P(vp)]
        L.fstat_grid.argtypes = [vp, vp, i64, P(_Out), vp]
        L.fstat_graph_create.argtypes = [vp, vp, i64, P(_Out), P(vp)]
        L.fstat_graph_launch.argtypes = [vp, vp]
        L.fstat_graph_destroy.argtypes = [vp]
        L.fstat_graph_destroy.restype = None
        L.fstat_eval.argtypes = [vp, vp, vp, i64, vp, vp, vp]
        L.fstat_adjoint.argtypes = [vp, vp, vp, i64, vp, vp, vp, vp]
        L.fstat_grad.argtypes = [vp, vp, vp, i64, vp, vp, vp]
        L.fstat_grad_static.argtypes = [vp, vp, vp, i64, vp, vp, vp]
        L.fstat_amplitudes.argtypes = [vp, vp, vp, i64, vp, vp, vp]
        L.fstat_eval_exact.argtypes = [vp, vp, vp, i64, vp, vp]
        L.fstat_refine.argtypes = [vp, vp, vp, i64, P(_RefineOptions), vp, vp, vp, vp]
        L.fstat_threshold.argtypes = [ctypes.c_double, ctypes.c_double, P(ctypes.c_double)]
        L.fstat_lattice_fisher.argtypes = [P(_Segment), P(_Detector), P(_Ephemeris), P(ctypes.c_double)]
        L.fstat_lattice_build.argtypes = [P(ctypes.c_double), ctypes.c_double, ctypes.c_double, i32, P(_Lattice)]
        L.fstat_lattice_segment.argtypes = [P(_Segment), P(_Detector), P(_Ephemeris), ctypes.c_double, i32,
                                            P(_Lattice)]
        L.fstat_bin_params.argtypes = [vp, vp, vp, i64, i32, vp, vp]
        L.fstat_lattice_nodes.argtypes = [P(_Lattice), P(_LatticeRegion), P(_Ephemeris), vp, vp, i64, P(i64)]
        L.fstat_copy_probe.argtypes = [vp, vp, i64, i32, vp]
        L.fstat_spill_write_probe.argtypes = [vp, i64, i32, i32, i32, vp]
        L.fstat_plan_info.argtypes = [vp, i32, P(i64), P(i64), P(ctypes.c_double), P(i32), P(i32)]
        L.fstat_demod_series.argtypes = [vp, vp, vp, vp]
        L.fstat_profile.argtypes = [vp, i32]
        L.fstat_plan_status.argtypes = [vp]
        L.fstat_plan_schedule.argtypes = [vp, i32, P(i32), P(i32), P(i32), P(i32), P(i32)]
        L.fstat_profile_read.argtypes = [vp, i32, P(i64), P(ctypes.c_double), P(ctypes.c_double)]
        L.fstat_destroy.argtypes = [vp]
        L.fstat_strerror.argtypes = [i32]
        L.fstat_strerror.restype = ctypes.c_char_p
        L.fstat_destroy.restype = None
        for name in ("fstat_plan", "fstat_grid", "fstat_graph_create", "fstat_graph_launch", "fstat_amplitudes",
                     "fstat_eval_exact", "fstat_refine", "fstat_threshold", "fstat_lattice_fisher",
                     "fstat_lattice_build", "fstat_lattice_segment", "fstat_lattice_nodes", "fstat_copy_probe",
                     "fstat_spill_write_probe",
                     "fstat_bin_params",
                     "fstat_eval", "fstat_adjoint", "fstat_grad", "fstat_grad_static", "fstat_plan_info",
                     "fstat_demod_series", "fstat_profile", "fstat_profile_read", "fstat_plan_schedule",
                     "fstat_plan_status"):
            getattr(L, name).restype = i32
        _lib = L
    return _lib


def _check(status: int, what: str):
    if status != OK:
        raise FStatError(status, what)


# --------------------------------------------------------------------------
# Python-side descriptions
# --------------------------------------------------------------------------
@dataclass(frozen=True)
class Detector:
    lat: float
    lon: float
    gamma: float
    zeta: float = math.pi / 2
    radius: float = R_EARTH


@dataclass(frozen=True)
class Ephemeris:
    obliquity: float = math.radians(23.44)
    orbit_radius: float = AU
    orbit_omega: float = 2.0 * math.pi / YEAR
    orbit_phase0: float = 0.0
    sidereal_day: float = SIDEREAL_DAY
    gmst0: float = 0.0


def default_detector() -> Detector:
    """Latitude 43.63 deg, longitude 10.5 deg, first arm 19.4 deg east of
    North with 90-deg arms: bisector 115.6 deg counter-clockwise from East."""
    return Detector(lat=math.radians(43.63), lon=math.radians(10.5), gamma=math.radians(115.6))


def detector_spec(d) -> Detector:
    """Any object with lat, lon, gamma, zeta, radius attributes."""
    return Detector(float(d.lat), float(d.lon), float(d.gamma), float(d.zeta), float(d.radius))


def ephemeris_spec(e) -> Ephemeris:
    return Ephemeris(float(e.obliquity), float(e.orbit_radius), float(e.orbit_omega), float(e.orbit_phase0),
                     float(e.sidereal_day), float(e.gmst0))


@dataclass
class SegmentSpec:
    x: np.ndarray
    dt: float
    n_days: int
    t0: float = 0.0
    mask: Optional[np.ndarray] = None
    f_ref: float = 435.1875
    sigma2: float = 1.0
    nfft: int = 0


def threshold(alpha: float, n_cells: float) -> float:
    """F0 with false-alarm probability alpha over n_cells independent cells
    (fstat_threshold: Eqs. PF, FP)."""
    F0 = ctypes.c_double()
    _check(lib().fstat_threshold(float(alpha), float(n_cells), ctypes.byref(F0)), "fstat_threshold")
    return F0.value


def copy_probe(dst: torch.Tensor, src: torch.Tensor, blocks: int = 0) -> None:
    """fstat_copy_probe on the current stream: dst <- src (same byte size)."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes or not src.is_cuda or not dst.is_cuda:
        raise ValueError("src and dst must be device tensors of the same byte size")
    _check(lib().fstat_copy_probe(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()), nbytes, int(blocks),
                                  _stream_ptr(src.device.index)), "fstat_copy_probe")


def spill_write_probe(dst: torch.Tensor, nodes: int, R: int, C: int, b2: int) -> None:
    """fstat_spill_write_probe on the current stream: the first FFT pass's
    spill stores alone into dst (nodes x R x C elements of 16 bytes)."""
    if dst.numel() * dst.element_size() < nodes * R * C * 16:
        raise ValueError("dst smaller than nodes x R x C x 16 bytes")
    _check(lib().fstat_spill_write_probe(ctypes.c_void_p(dst.data_ptr()), int(nodes), int(R), int(C), int(b2),
                                         _stream_ptr(dst.device.index)), "fstat_spill_write_probe")


def nodes_array(alpha, delta, fdot, seg=0, bin_offset=0.0) -> np.ndarray:
    """Grid nodes (fstat_node records); bin_offset shifts a node's line of
    Fourier bins by that fraction of a bin (|bin_offset| < 1)."""
    alpha, delta, fdot, seg, off = np.broadcast_arrays(
        np.asarray(alpha, float), np.asarray(delta, float), np.asarray(fdot, float),
        np.asarray(seg, np.int32), np.asarray(bin_offset, np.float32))
    out = np.zeros(alpha.size, dtype=NODE_DTYPE)
    out["alpha"] = alpha.ravel()
    out["delta"] = delta.ravel()
    out["fdot"] = fdot.ravel()
    out["seg"] = seg.ravel()
    out["bin_offset"] = off.ravel()
    return out


def _stream_ptr(device: int) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _segment_struct(s: SegmentSpec, keep: list) -> _Segment:
    seg = _Segment()
    x = np.ascontiguousarray(np.asarray(s.x, dtype=np.float64))
    keep.append(x)
    seg.x = x.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    seg.n = x.size
    seg.dt = float(s.dt)
    seg.n_sidereal_days = int(s.n_days)
    seg.t0 = float(s.t0)
    if s.mask is not None:
        m = np.ascontiguousarray(np.asarray(s.mask, dtype=np.uint8))
        keep.append(m)
        seg.mask = m.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    seg.f_ref_hz = float(s.f_ref)
    seg.sigma2 = float(s.sigma2)
    seg.nfft = int(s.nfft)
    return seg


def _eph_struct(eph: Ephemeris) -> _Ephemeris:
    return _Ephemeris(eph.obliquity, eph.orbit_radius, eph.orbit_omega, eph.orbit_phase0, eph.sidereal_day,
                      eph.gmst0)


def lattice_fisher(seg: SegmentSpec, det: Detector, eph: Ephemeris) -> np.ndarray:
    """Reduced Fisher matrix [4, 4] of the one-spindown linear model over the
    segment's kept samples (fstat_lattice_fisher: Eq. redFm-def)."""
    keep: list = []
    s = _segment_struct(seg, keep)
    g = (ctypes.c_double * 16)()
    d = _Detector(det.lat, det.lon, det.gamma, det.zeta, det.radius)
    e = _eph_struct(eph)
    _check(lib().fstat_lattice_fisher(ctypes.byref(s), ctypes.byref(d), ctypes.byref(e), g), "fstat_lattice_fisher")
    return np.array(g[:], dtype=np.float64).reshape(4, 4)


class Lattice:
    """The covering lattice of Sec. IV (fstat_lattice_build) and its grid nodes
    (fstat_lattice_nodes)."""

    def __init__(self, raw: _Lattice):
        self._raw = raw
        self.basis = np.array(raw.basis[:], dtype=np.float64).reshape(4, 4)
        self.gamma = np.array(raw.gamma[:], dtype=np.float64).reshape(4, 4)
        for name in ("dp0", "c0", "R", "mu", "nu", "theta", "margin_w1", "margin_sky"):
            setattr(self, name, float(getattr(raw, name)))
        self.rule = int(raw.rule)

    @classmethod
    def build(cls, gamma, dp0: float, c0: float = 0.75, rule: int = NU_DEEP_HOLES) -> "Lattice":
        """rule NU_DEEP_HOLES: the paper's worked example; NU_COVERING: its
        definition of nu, a thinner covering (fstat_lattice_build)."""
        g = np.ascontiguousarray(np.asarray(gamma, dtype=np.float64).reshape(16))
        raw = _Lattice()
        _check(lib().fstat_lattice_build(g.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), float(dp0), float(c0),
                                         int(rule), ctypes.byref(raw)), "fstat_lattice_build")
        return cls(raw)

    @classmethod
    def for_segment(cls, seg: SegmentSpec, det: Detector, eph: Ephemeris, c0: float = 0.75,
                    rule: int = NU_DEEP_HOLES) -> "Lattice":
        """The lattice of one segment: its reduced Fisher matrix and the
        resolution 2 pi / (nfft dt) of its Fourier bins."""
        keep: list = []
        s = _segment_struct(seg, keep)
        d = _Detector(det.lat, det.lon, det.gamma, det.zeta, det.radius)
        e = _eph_struct(eph)
        raw = _Lattice()
        _check(lib().fstat_lattice_segment(ctypes.byref(s), ctypes.byref(d), ctypes.byref(e), float(c0), int(rule),
                                           ctypes.byref(raw)), "fstat_lattice_segment")
        return cls(raw)

    def nodes(self, f_sky: float, fdot_lo: float, fdot_hi: float, eph: Ephemeris, sky=None, hemisphere: int = 0,
              seg: int = 0, coef: bool = False):
        """Grid nodes over the sky disk (or the disk sky = (c1, c2, radius) of
        the (alpha_1, alpha_2) plane) and [fdot_lo, fdot_hi]: a NODE_DTYPE
        array, and the lattice coefficients [n, 3] when coef is set."""
        reg = _LatticeRegion(float(f_sky), float(fdot_lo), float(fdot_hi), 0.0, 0.0, 0.0, int(hemisphere), int(seg))
        if sky is not None:
            reg.sky_c1, reg.sky_c2, reg.sky_radius = (float(v) for v in sky)
        e = _eph_struct(eph)
        n = ctypes.c_int64()
        L = lib()
        _check(L.fstat_lattice_nodes(ctypes.byref(self._raw), ctypes.byref(reg), ctypes.byref(e), None, None, 0,
                                     ctypes.byref(n)), "fstat_lattice_nodes")
        out = np.zeros(n.value, dtype=NODE_DTYPE)
        k = np.zeros((n.value, 3), dtype=np.int32)
        _check(L.fstat_lattice_nodes(ctypes.byref(self._raw), ctypes.byref(reg), ctypes.byref(e),
                                     out.ctypes.data_as(ctypes.c_void_p), k.ctypes.data_as(ctypes.c_void_p),
                                     n.value, ctypes.byref(n)), "fstat_lattice_nodes")
        return (out, k) if coef else out


class Plan:
    """A plan of fstat_plan: segments on the device, prepared for grid calls.
    launch: LAUNCH_PASSES (a sequence of pass launches per batch, the default)
    or LAUNCH_PERSISTENT (one persistent kernel per call where it applies;
    the same outputs, bit for bit)."""

    def __init__(self, segments: Sequence[SegmentSpec], det: Detector, eph: Ephemeris,
                 interp: int = LINEAR_UP2, prec: int = FP32, device: int = 0, max_batch: int = 0,
                 autotune: bool = False, launch: int = 0):
        L = lib()
        self._keep = []
        segs = (_Segment * len(segments))()
        for i, s in enumerate(segments):
            segs[i] = _segment_struct(s, self._keep)
        d = _Detector(det.lat, det.lon, det.gamma, det.zeta, det.radius)
        e = _eph_struct(eph)
        o = _Options(interp, prec, device, max_batch, 1 if autotune else 0, int(launch))
        h = ctypes.c_void_p()
        _check(L.fstat_plan(segs, len(segments), ctypes.byref(d), ctypes.byref(e), ctypes.byref(o),
                            ctypes.byref(h)), "fstat_plan")
        self._keep = None
        self._h = h
        self._destroy = L.fstat_destroy
        self.device = device
        self.prec = prec
        self.interp = interp
        self.nseg = len(segments)
        self.dtype = torch.float32 if prec == FP32 else torch.float64

    def __del__(self):
        # the destroy function was bound at creation: at interpreter exit the
        # module's globals (lib among them) may already be gone
        h = getattr(self, "_h", None)
        destroy = getattr(self, "_destroy", None)
        if h is not None and h.value and destroy is not None:
            destroy(h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def status(self) -> None:
        """fstat_plan_status: waits for the device; raises FStatError if a
        persistent launch of this plan stopped early since the last check."""
        _check(lib().fstat_plan_status(self._h), "fstat_plan_status")

    def info(self, seg: int = 0) -> dict:
        n, nfft = ctypes.c_int64(), ctypes.c_int64()
        s2 = ctypes.c_double()
        R, C = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().fstat_plan_info(self._h, seg, ctypes.byref(n), ctypes.byref(nfft), ctypes.byref(s2),
                                     ctypes.byref(R), ctypes.byref(C)), "fstat_plan_info")
        return dict(n=n.value, nfft=nfft.value, sigma2=s2.value, R=R.value, C=C.value)

    def schedule(self, seg: int = 0) -> dict:
        """The FFT split, batch size and stream mode in use for a segment."""
        R, C, B2, b, ns = (ctypes.c_int32() for _ in range(5))
        _check(lib().fstat_plan_schedule(self._h, seg, ctypes.byref(R), ctypes.byref(C), ctypes.byref(B2),
                                         ctypes.byref(b), ctypes.byref(ns)), "fstat_plan_schedule")
        return dict(R=R.value, C=C.value, B2=B2.value, batch=b.value, streams=ns.value)

    def profile(self, enable: bool = True):
        """Enable (and reset) or disable per-launch kernel timing."""
        _check(lib().fstat_profile(self._h, 1 if enable else 0), "fstat_profile")

    def profile_read(self, kind: int) -> dict:
        """Launch count, summed milliseconds and algorithmic bytes of one kernel kind."""
        n, ms, b = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
        _check(lib().fstat_profile_read(self._h, kind, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(b)),
               "fstat_profile_read")
        return dict(launches=n.value, ms=ms.value, bytes=b.value)

    def _dev(self):
        return torch.device("cuda", self.device)

    def _grid(self, nodes: np.ndarray, out: _Out):
        nodes = np.ascontiguousarray(nodes, dtype=NODE_DTYPE)
        _check(lib().fstat_grid(self._h, nodes.ctypes.data_as(ctypes.c_void_p), nodes.size, ctypes.byref(out),
                                _stream_ptr(self.device)), "fstat_grid")

    def grid_map(self, nodes: np.ndarray, k_lo: int, k_hi: int, F: Optional[torch.Tensor] = None,
                 interbin: bool = False) -> torch.Tensor:
        """F on bins [k_lo, k_hi) of every node: tensor [n_nodes, k_hi - k_lo]; with
        interbin, [n_nodes, 2 (k_hi - k_lo)]: F at k and k + 1/2 interleaved."""
        w = (2 if interbin else 1) * (k_hi - k_lo)
        if F is None:
            F = torch.empty((len(nodes), w), dtype=self.dtype, device=self._dev())
        out = _Out(mode=OUT_MAP, interbin=int(interbin), k_lo=k_lo, k_hi=k_hi, F=F.data_ptr())
        self._grid(nodes, out)
        return F

    def grid_max(self, nodes: np.ndarray, k_lo: int, k_hi: int, interbin: bool = False):
        """Per node: (max F on [k_lo, k_hi), its bin; with interbin the half bins
        count too and the bin is in half-bin units 2k + h)."""
        Fmax = torch.empty(len(nodes), dtype=self.dtype, device=self._dev())
        kmax = torch.empty(len(nodes), dtype=torch.int64, device=self._dev())
        out = _Out(mode=OUT_MAX, interbin=int(interbin), k_lo=k_lo, k_hi=k_hi, Fmax=Fmax.data_ptr(),
                   kmax=kmax.data_ptr())
        self._grid(nodes, out)
        return Fmax, kmax

    def grid_crossings(self, nodes: np.ndarray, k_lo: int, k_hi: int, threshold: float, max_crossings: int,
                       interbin: bool = False):
        """All (node, bin, F) with F > threshold, unordered: a device buffer of
        fstat_crossing records (int64 [max, 3] words) and the total count
        (with interbin the bin is in half-bin units 2k + h)."""
        rec = torch.empty((max(1, max_crossings), 3), dtype=torch.int64, device=self._dev())
        cnt = torch.empty(1, dtype=torch.int64, device=self._dev())
        out = _Out(mode=OUT_CROSSINGS, interbin=int(interbin), k_lo=k_lo, k_hi=k_hi, threshold=threshold,
                   crossings=rec.data_ptr(),
                   n_crossings=cnt.data_ptr(), max_crossings=max_crossings)
        self._grid(nodes, out)
        return rec, cnt

    @staticmethod
    def read_crossings(rec: torch.Tensor, cnt: torch.Tensor) -> np.ndarray:
        """Copy the stored crossings to the host as a CROSSING_DTYPE array."""
        n = min(int(cnt.cpu().item()), rec.shape[0])
        return rec[:n].cpu().numpy().view(CROSSING_DTYPE).reshape(-1)

    def _graph(self, nodes: np.ndarray, out: _Out, outputs: dict) -> "GridGraph":
        nodes = np.ascontiguousarray(nodes, dtype=NODE_DTYPE)
        h = ctypes.c_void_p()
        _check(lib().fstat_graph_create(self._h, nodes.ctypes.data_as(ctypes.c_void_p), nodes.size,
                                        ctypes.byref(out), ctypes.byref(h)), "fstat_graph_create")
        return GridGraph(self, h, outputs)

    def graph_map(self, nodes: np.ndarray, k_lo: int, k_hi: int, F: Optional[torch.Tensor] = None,
                  interbin: bool = False) -> "GridGraph":
        """grid_map recorded as a graph: every launch() rewrites .outputs['F']."""
        w = (2 if interbin else 1) * (k_hi - k_lo)
        if F is None:
            F = torch.empty((len(nodes), w), dtype=self.dtype, device=self._dev())
        out = _Out(mode=OUT_MAP, interbin=int(interbin), k_lo=k_lo, k_hi=k_hi, F=F.data_ptr())
        return self._graph(nodes, out, {"F": F})

    def graph_max(self, nodes: np.ndarray, k_lo: int, k_hi: int, interbin: bool = False) -> "GridGraph":
        """grid_max recorded as a graph (outputs 'Fmax', 'kmax')."""
        Fmax = torch.empty(len(nodes), dtype=self.dtype, device=self._dev())
        kmax = torch.empty(len(nodes), dtype=torch.int64, device=self._dev())
        out = _Out(mode=OUT_MAX, interbin=int(interbin), k_lo=k_lo, k_hi=k_hi, Fmax=Fmax.data_ptr(),
                   kmax=kmax.data_ptr())
        return self._graph(nodes, out, {"Fmax": Fmax, "kmax": kmax})

    def graph_crossings(self, nodes: np.ndarray, k_lo: int, k_hi: int, threshold: float,
                        max_crossings: int, interbin: bool = False) -> "GridGraph":
        """grid_crossings recorded as a graph (outputs 'rec', 'cnt')."""
        rec = torch.empty((max(1, max_crossings), 3), dtype=torch.int64, device=self._dev())
        cnt = torch.empty(1, dtype=torch.int64, device=self._dev())
        out = _Out(mode=OUT_CROSSINGS, interbin=int(interbin), k_lo=k_lo, k_hi=k_hi, threshold=threshold,
                   crossings=rec.data_ptr(), n_crossings=cnt.data_ptr(), max_crossings=max_crossings)
        return self._graph(nodes, out, {"rec": rec, "cnt": cnt})

    def demod_series(self, node: np.ndarray) -> torch.Tensor:
        node = np.ascontiguousarray(np.asarray(node, dtype=NODE_DTYPE).reshape(1))
        n = self.info(int(node["seg"][0]))["n"]
        out = torch.empty((n, 4), dtype=torch.float64, device=self._dev())
        _check(lib().fstat_demod_series(self._h, node.ctypes.data_as(ctypes.c_void_p), _ptr(out),
                                        _stream_ptr(self.device)), "fstat_demod_series")
        return out

    # ---- continuous parameters ----
    def bin_params(self, nodes: np.ndarray, k, interbin: bool = False):
        """The continuous parameters of output bins, for eval / refine /
        amplitudes: nodes[i] and its output index k[i] (the map column plus k_lo,
        a kmax, or a crossing's k; 2k + h with interbinning, h = 1 for the half
        bin) give f = (k + bin_offset) / (nfft dt) (band-relative Hz), the
        node's fdot, alpha, delta.  Returns (params [n, 4] float64, seg [n]
        int32) on the plan's device."""
        nodes = np.ascontiguousarray(np.asarray(nodes, dtype=NODE_DTYPE).reshape(-1))
        k = np.ascontiguousarray(np.asarray(k, dtype=np.int64).reshape(-1))
        if len(k) != len(nodes):
            raise ValueError("one bin index per node row")
        params = np.empty((len(nodes), 4), dtype=np.float64)
        segs = np.empty(len(nodes), dtype=np.int32)
        _check(lib().fstat_bin_params(self._h, nodes.ctypes.data_as(ctypes.c_void_p), k.ctypes.data_as(ctypes.c_void_p),
                                      len(nodes), int(interbin), params.ctypes.data_as(ctypes.c_void_p),
                                      segs.ctypes.data_as(ctypes.c_void_p)), "fstat_bin_params")
        return torch.from_numpy(params).to(self._dev()), torch.from_numpy(segs).to(self._dev())

    def _params(self, params: torch.Tensor, seg: Optional[torch.Tensor]):
        if params.dtype != torch.float64 or params.device != self._dev() or params.dim() != 2 or params.shape[1] != 4:
            raise ValueError("params must be a float64 [n, 4] tensor on cuda:%d" % self.device)
        params = params.contiguous()
        if seg is not None:
            seg = seg.to(device=self._dev(), dtype=torch.int32).contiguous()
        return params, seg

    def eval(self, params: torch.Tensor, seg: Optional[torch.Tensor] = None, want_state: bool = True):
        params, seg = self._params(params, seg)
        n = params.shape[0]
        F = torch.empty(n, dtype=torch.float64, device=self._dev())
        state = torch.empty((n, STATE), dtype=torch.float64, device=self._dev()) if want_state else None
        _check(lib().fstat_eval(self._h, _ptr(params), _ptr(seg), n, _ptr(F), _ptr(state),
                                _stream_ptr(self.device)), "fstat_eval")
        return F, state

    def adjoint(self, params: torch.Tensor, state: torch.Tensor, gF: Optional[torch.Tensor] = None,
                seg: Optional[torch.Tensor] = None) -> torch.Tensor:
        params, seg = self._params(params, seg)
        n = params.shape[0]
        dp = torch.empty((n, 4), dtype=torch.float64, device=self._dev())
        if gF is not None:
            gF = gF.to(device=self._dev(), dtype=torch.float64).contiguous()
        _check(lib().fstat_adjoint(self._h, _ptr(params), _ptr(seg), n, _ptr(state.contiguous()), _ptr(gF),
                                   _ptr(dp), _stream_ptr(self.device)), "fstat_adjoint")
        return dp

    def eval_exact(self, params: torch.Tensor, seg: Optional[torch.Tensor] = None) -> torch.Tensor:
        """F without resampling (direct sums on the detector samples), [n]."""
        params, seg = self._params(params, seg)
        F = torch.empty(params.shape[0], dtype=torch.float64, device=self._dev())
        _check(lib().fstat_eval_exact(self._h, _ptr(params), _ptr(seg), params.shape[0], _ptr(F),
                                      _stream_ptr(self.device)), "fstat_eval_exact")
        return F

    def refine(self, params: torch.Tensor, scale, tol: float = 1e-3, max_evals: int = 400, exact: bool = True,
               seg: Optional[torch.Tensor] = None):
        """Nelder-Mead fine search from each row of params: (best params [n, 4],
        F [n], evaluations used [n])."""
        params, seg = self._params(params, seg)
        n = params.shape[0]
        pout = torch.empty_like(params)
        F = torch.empty(n, dtype=torch.float64, device=self._dev())
        ev = torch.empty(n, dtype=torch.int32, device=self._dev())
        o = _RefineOptions((ctypes.c_double * 4)(*[float(v) for v in scale]), float(tol), int(max_evals),
                           1 if exact else 0)
        _check(lib().fstat_refine(self._h, _ptr(params), _ptr(seg), n, ctypes.byref(o), _ptr(pout), _ptr(F),
                                  _ptr(ev), _stream_ptr(self.device)), "fstat_refine")
        return pout, F, ev

    def amplitudes(self, params: torch.Tensor, seg: Optional[torch.Tensor] = None) -> torch.Tensor:
        """[n, 8]: amplitudes A1..A4, h0, cos(iota), psi, phi0 at the candidates
        (fstat_eval, then fstat_amplitudes)."""
        params, seg = self._params(params, seg)
        _, state = self.eval(params, seg)
        out = torch.empty((params.shape[0], 8), dtype=torch.float64, device=self._dev())
        _check(lib().fstat_amplitudes(self._h, _ptr(params), _ptr(seg), params.shape[0], _ptr(state), _ptr(out),
                                      _stream_ptr(self.device)), "fstat_amplitudes")
        return out

    def grad(self, params: torch.Tensor, seg: Optional[torch.Tensor] = None):
        params, seg = self._params(params, seg)
        n = params.shape[0]
        F = torch.empty(n, dtype=torch.float64, device=self._dev())
        dF = torch.empty((n, 4), dtype=torch.float64, device=self._dev())
        _check(lib().fstat_grad(self._h, _ptr(params), _ptr(seg), n, _ptr(F), _ptr(dF),
                                _stream_ptr(self.device)), "fstat_grad")
        return F, dF

    def grad_static(self, params: torch.Tensor, seg: Optional[torch.Tensor] = None, F: Optional[torch.Tensor] = None,
                    dF: Optional[torch.Tensor] = None):
        """grad through fstat_grad_static: no device allocation in the
        library (at most GRAD_STATIC_MAX candidates; calls on one GPU must
        not overlap).  F [n] and dF [n, 4] may be given (preallocated)."""
        params, seg = self._params(params, seg)
        n = params.shape[0]
        if F is None:
            F = torch.empty(n, dtype=torch.float64, device=self._dev())
        if dF is None:
            dF = torch.empty((n, 4), dtype=torch.float64, device=self._dev())
        _check(lib().fstat_grad_static(self._h, _ptr(params), _ptr(seg), n, _ptr(F), _ptr(dF),
                                       _stream_ptr(self.device)), "fstat_grad_static")
        return F, dF


class GridGraph:
    """A recorded grid call (fstat_graph_create); launch() replays it on the
    current stream.  Holds its plan and output tensors alive."""

    def __init__(self, plan: Plan, handle: ctypes.c_void_p, outputs: dict):
        self.plan = plan
        self._h = handle
        self._destroy = lib().fstat_graph_destroy  # bound now, usable at interpreter exit
        self.outputs = outputs

    def launch(self):
        _check(lib().fstat_graph_launch(self._h, _stream_ptr(self.plan.device)), "fstat_graph_launch")

    def close(self):
        if self._h is not None and self._h.value:
            self._destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class FStatFn(torch.autograd.Function):
    """F(params) with params = [n, 4] (f, fdot, alpha, delta); backward runs the
    adjoint kernel (recomputing the resampled series)."""

    @staticmethod
    def forward(ctx, params: torch.Tensor, plan: Plan, seg: Optional[torch.Tensor] = None):
        F, state = plan.eval(params, seg)
        ctx.plan = plan
        ctx.seg = seg
        ctx.save_for_backward(params, state)
        return F

    @staticmethod
    def backward(ctx, gF):
        params, state = ctx.saved_tensors
        dp = ctx.plan.adjoint(params, state, gF, ctx.seg)
        return dp, None, None
