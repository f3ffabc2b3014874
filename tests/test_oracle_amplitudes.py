"""Pins of the amplitude parameters (Sec. III): Eq. (ampone), its inversion,
the ML amplitude estimators of Eq. (amle0) and the second step of the ML
estimation on noise-free data."""
import math

import numpy as np

from oracle import method
from paper_1003_0844_amd import synth
from tests.common import DET, EPH, inversion_tolerances, one_signal, small_segment


def _same_angle(a, b, period):
    d = (a - b) % period
    return min(d, period - d)


def test_inversion_round_trip():
    g = np.random.default_rng(5)
    for _ in range(200):
        h0, cosi = g.uniform(0.1, 3.0), g.uniform(-0.98, 0.98)
        psi, phi0 = g.uniform(0, math.pi / 2), g.uniform(0, 2 * math.pi)
        Ab = method.amplitudes_from_parameters(h0, cosi, psi, phi0)
        h0e, cie, pse, phe = method.parameters_from_amplitudes(Ab)
        # h0 = h0+ + sqrt(|z1 + z2| |z1 - z2|): near cos iota = +-1 the square
        # root amplifies the rounding of the small factor
        tol = 1e-14 / (1.0 - abs(cosi)) + 1e-13
        assert abs(h0e - h0) < tol * h0 and abs(cie - cosi) < tol
        assert _same_angle(pse, psi, math.pi / 2) < 1e-9 and _same_angle(phe, phi0, 2 * math.pi) < 1e-9


def test_inversion_satisfies_the_papers_relations():
    # h0+ and h0x from the paper's A and D, and its tan(2 phi0), tan(4 psi)
    g = np.random.default_rng(6)
    for _ in range(100):
        Ab = g.normal(size=4)
        h0, cosi, psi, phi0 = method.parameters_from_amplitudes(Ab)
        hp, hx = 0.5 * h0 * (1 + cosi * cosi), h0 * cosi
        A = float(np.sum(Ab * Ab))
        D = Ab[0] * Ab[3] - Ab[1] * Ab[2]
        assert abs(hp - math.sqrt(0.5 * (A + math.sqrt(A * A - 4 * D * D)))) < 1e-12 * A
        assert abs(hx - math.copysign(math.sqrt(0.5 * (A - math.sqrt(A * A - 4 * D * D))), D)) < 1e-9 * A
        num, den = 2 * (Ab[0] * Ab[2] + Ab[1] * Ab[3]), Ab[2] ** 2 + Ab[3] ** 2 - Ab[0] ** 2 - Ab[1] ** 2
        assert abs(math.sin(2 * phi0) * den - math.cos(2 * phi0) * num) < 1e-9 * A
        num, den = 2 * (Ab[0] * Ab[1] + Ab[2] * Ab[3]), Ab[0] ** 2 + Ab[2] ** 2 - Ab[1] ** 2 - Ab[3] ** 2
        assert abs(math.sin(4 * psi) * den - math.cos(4 * psi) * num) < 1e-9 * A
        assert 0 <= psi < math.pi / 2 and 0 <= phi0 < 2 * math.pi
        assert np.allclose(method.amplitudes_from_parameters(h0, cosi, psi, phi0), Ab, atol=1e-12)


def test_inversion_special_cases():
    # psi + pi/2 with phi0 + pi gives the same amplitudes (the convention keeps psi < pi/2)
    a = method.amplitudes_from_parameters(1.3, 0.4, 0.3, 1.0)
    b = method.amplitudes_from_parameters(1.3, 0.4, 0.3 + math.pi / 2, 1.0 + math.pi)
    assert np.allclose(a, b, atol=1e-14)
    # a circularly polarised wave (cos iota = +-1): h0 and cos iota come back
    # (to the square root of the rounding of the vanishing combination), and
    # only 2 psi +- phi0 is determined (Ab1 = h0 cos(2 psi +- phi0), ...)
    for ci in (1.0, -1.0):
        Ab = method.amplitudes_from_parameters(0.7, ci, 0.2, 0.9)
        h0e, cie, pse, phe = method.parameters_from_amplitudes(Ab)
        assert abs(h0e - 0.7) < 1e-7 and abs(cie - ci) < 1e-7
        assert _same_angle(2 * pse + ci * phe, 2 * 0.2 + ci * 0.9, 2 * math.pi) < 1e-9
        assert abs(Ab[0] - 0.7 * math.cos(2 * 0.2 + ci * 0.9)) < 1e-12


def test_estimators_are_the_papers_when_C_vanishes():
    # with C = 0 the normal equations reduce to Eq. (amle0): 2 Re S_a / A, ...
    Sa, Sb, A, B = 3.0 - 4.0j, -1.5 + 2.5j, 7.0, 5.0
    Ab = method.amplitude_estimates(Sa, Sb, A, B, 0.0, 0.0)
    assert np.allclose(Ab, [2 * 3.0 / 7.0, 2 * -1.5 / 5.0, 2 * 4.0 / 7.0, 2 * -2.5 / 5.0], rtol=1e-15)
    # and a common phase of S_a, S_b is undone by theta0
    th = 0.7
    rot = complex(math.cos(th), math.sin(th))
    assert np.allclose(method.amplitude_estimates(Sa * rot, Sb * rot, A, B, 0.0, th), Ab, rtol=1e-13)


def _noise_free_case(seed, mask=None):
    dt = 26.0
    sig = one_signal(seed, band=1 / (2 * dt), snr=30.0)
    seg = small_segment(days=2, dt=dt, seed=seed, signal=sig, noise=False, mask=mask)
    # the injection's h0 (the oracle scales a unit-h0 signal to the SNR)
    t = np.arange(seg.n) * dt
    from oracle import model
    h1 = model.signal(t, 0.0, sig["f"], sig["fdot"], sig["alpha"], sig["delta"], 1.0, sig["cosi"], sig["psi"],
                      sig["phi0"], seg.f_ref, DET, EPH)
    m = np.ones(seg.n) if mask is None else mask.astype(float)
    h0 = sig["snr"] / math.sqrt(np.sum(m * h1 * h1) / seg.sigma2)
    return seg, sig, h0


def test_second_step_recovers_injected_parameters():
    # noise-free data, the true intrinsic parameters, cubic two-step
    # resampling: the estimates are the injected ones up to the method's own
    # error (about 0.1 % in F, Sec. VI A)
    for seed, gaps in ((3, False), (4, True), (3, True), (8, True)):
        mask = synth.gap_mask(synth.rng(90 + seed), int(2 * synth.SIDEREAL_DAY / 26.0), 26.0, 0.1) if gaps else None
        seg, sig, h0 = _noise_free_case(seed, mask)
        Ab, (h0e, cie, pse, phe) = method.estimate_parameters(
            seg, (sig["f"], sig["fdot"], sig["alpha"], sig["delta"]), DET, EPH, method.CUBIC_UP2)
        want = method.amplitudes_from_parameters(h0, sig["cosi"], sig["psi"], sig["phi0"])
        assert np.max(np.abs(Ab - want)) < 2e-3 * np.max(np.abs(want)), (Ab, want)
        # h0 and cos iota: the amplitude bar carried through the inversion
        tol_h0, tol_ci = inversion_tolerances(2e-3 * np.max(np.abs(want)), h0, sig["cosi"])
        assert abs(h0e / h0 - 1) < tol_h0 and abs(cie - sig["cosi"]) < tol_ci, (h0e / h0 - 1, tol_h0)
        # psi and phi0 come from the arguments of z1 +- z2 (z1 = A1 + i A2,
        # z2 = A4 - i A3), the smaller of which has modulus h0 (1 - |cos iota|)^2 / 2:
        # an amplitude error e moves its argument by up to 2 e over that modulus
        e_amp = 2e-3 * np.max(np.abs(want))
        tol = 2.0 * e_amp / (0.5 * h0 * (1.0 - abs(sig["cosi"])) ** 2)
        assert _same_angle(pse, sig["psi"] % (math.pi / 2), math.pi / 2) < tol
        # phi0 pairs with psi: compare modulo the (psi + pi/2, phi0 + pi) symmetry
        ph_true = sig["phi0"] + (math.pi if (sig["psi"] % math.pi) >= math.pi / 2 else 0.0)
        assert _same_angle(phe, ph_true % (2 * math.pi), 2 * math.pi) < tol, (phe, sig["phi0"], sig["psi"])
