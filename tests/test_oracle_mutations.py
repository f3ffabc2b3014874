"""Planted mistakes in the oracle (on the CPU): each one must make at least one
of the oracle's pins fail.  This shows the pins have teeth against the
plausible slips -- a dropped term, a wrong sign, a wrong index or origin."""
import math

import numpy as np
import pytest

from oracle import method, model
from tests import test_oracle_fstat as tf
from tests import test_oracle_geometry as tg
from tests import test_oracle_resample as tr


def _fails(fn, *args):
    with pytest.raises(AssertionError):
        fn(*args)


def test_sign_of_obliquity_term_is_caught(monkeypatch):
    orig = model.roemer_delay

    def bad(T, alpha, delta, det, eph):
        xes, yes = model.earth_center(T, eph)
        return orig(T, alpha, delta, det, eph) - 2 * math.sin(delta) * math.sin(eph.obliquity) * yes / model.C_LIGHT
    monkeypatch.setattr(model, "roemer_delay", bad)
    _fails(tg.test_roemer_delay_matches_matrix_form)


def test_dropped_constant_term_of_a_is_caught(monkeypatch):
    orig = model._ab_coeffs

    def bad(delta, det):
        a, b = orig(delta, det)
        a = dict(a, a0=0.0)
        return a, b
    monkeypatch.setattr(model, "_ab_coeffs", bad)
    _fails(tg.test_ab_match_detector_tensor)
    _fails(tg.test_ab_at_zenith)


def test_swapped_sidereal_harmonics_of_b_are_caught(monkeypatch):
    orig = model._ab_coeffs

    def bad(delta, det):
        a, b = orig(delta, det)
        b = dict(b, b1c=b["b1s"], b1s=b["b1c"])
        return a, b
    monkeypatch.setattr(model, "_ab_coeffs", bad)
    _fails(tg.test_ab_match_detector_tensor)


def test_wrong_sign_of_cross_term_is_caught(monkeypatch):
    def bad(Sa, Sb, A, B, C, sigma2):
        num = B * np.abs(Sa) ** 2 + A * np.abs(Sb) ** 2 + 2.0 * C * np.real(Sa * np.conj(Sb))
        return num / (sigma2 * (A * B - C * C))
    monkeypatch.setattr(method, "combine", bad)
    _fails(tf.test_combination_is_invariant_under_mixing_a_and_b)


def test_unhalved_nyquist_bin_is_caught(monkeypatch):
    def bad(x):
        n = x.size
        X = np.fft.fft(x)
        Y = np.zeros(2 * n, dtype=np.complex128)
        h = n // 2
        Y[:h + 1] = X[:h + 1]
        if n % 2 == 0:
            Y[2 * n - h:] = X[h:]             # Nyquist bin copied, not halved
        else:
            Y[2 * n - h:] = X[h + 1:]
        return 2.0 * np.fft.ifft(Y).real
    monkeypatch.setattr(method, "fourier_upsample", bad)
    _fails(tr.test_upsample_against_trigonometric_interpolant_brute_force)


def test_wrong_ssb_grid_origin_is_caught(monkeypatch):
    def bad(seg, alpha, delta, det, eph, tol=1e-12, max_iter=60):
        j = np.arange(seg.n, dtype=np.float64)
        tb = j * seg.dt                         # t_b0 forgotten
        t = j * seg.dt
        for _ in range(max_iter):
            t = tb - model.roemer_delay(seg.t0 + t, alpha, delta, det, eph)
        return 0.0, t
    monkeypatch.setattr(method, "ssb_times", bad)
    _fails(tf.test_method_error_against_exact_filter)


def test_wrong_sign_of_spindown_doppler_term_is_caught(monkeypatch):
    def bad(t, T0, alpha, delta, f_ref, fdot, det, eph):
        pm = model.roemer_delay(T0 + t, alpha, delta, det, eph)
        pm0 = model.roemer_delay(T0, alpha, delta, det, eph)
        cyc = f_ref * (pm - pm0) + fdot * (0.5 * t * t - pm * t)
        return cyc - np.round(cyc)
    monkeypatch.setattr(method, "demod_cycles", bad)
    # visible once the spindown is large enough for its Doppler term to matter
    dt = 13.0
    from tests.common import DET, EPH, one_signal, small_segment
    sig = one_signal(5, band=1 / (2 * dt), snr=10.0, fdot=(-2e-8, -2e-8))
    seg = small_segment(days=2, dt=dt, signal=sig, noise=False, nfft=1 << 15)
    F = method.fstat_continuous(seg, (sig["f"], sig["fdot"], sig["alpha"], sig["delta"]), DET, EPH,
                                method.CUBIC_UP2)
    Fe = method.fstat_exact(seg, [sig["f"]], sig["fdot"], sig["alpha"], sig["delta"], DET, EPH)[0]
    assert abs(F / Fe - 1) > 5e-3


def test_wrong_derivative_of_delay_is_caught(monkeypatch):
    orig = method._roemer_partials

    def bad(T, alpha, delta, det, eph):
        pm, d_al, d_de, d_T = orig(T, alpha, delta, det, eph)
        return pm, d_al, -d_de, d_T
    monkeypatch.setattr(method, "_roemer_partials", bad)
    _fails(tg.test_roemer_partials_match_finite_differences)
    _fails(tf.test_gradient_matches_central_differences, method.CUBIC_UP2, 1e-6)


# ------------------------------------------------------ lattice grid (Sec. IV)
from oracle import lattice as lat_oracle  # noqa: E402
from tests import test_oracle_lattice as tl  # noqa: E402


def test_uncentred_fisher_matrix_is_caught(monkeypatch):
    def bad(m, weights=None):
        m = np.asarray(m, dtype=np.float64)
        w = np.ones(m.shape[1]) if weights is None else np.asarray(weights, dtype=np.float64)
        w = w / w.sum()
        return (m * w) @ m.T                       # <m_k m_l> without -<m_k><m_l>
    monkeypatch.setattr(lat_oracle, "reduced_fisher", bad)
    _fails(tl.test_reduced_fisher_of_the_2d_example)


def test_wrong_sign_in_the_a4star_generator_is_caught(monkeypatch):
    orig = lat_oracle.generator_a4star

    def bad(R):
        G = orig(R).copy()
        G[3, 1] = -G[3, 1]
        return G
    monkeypatch.setattr(lat_oracle, "generator_a4star", bad)
    _fails(tl.test_a2star_and_a4star_generators)


def test_printed_nu_iteration_is_caught(monkeypatch):
    # nu = R / (R_1 sin phi) from the lattice shrunk along l: not the covering
    # the worked example prints
    def bad(verts, l, mu, R):
        lh = l / np.linalg.norm(l)
        c = verts @ lh
        p = np.sqrt(np.maximum(np.einsum("ij,ij->i", verts, verts) - c * c, 0.0))
        img = np.sqrt(mu * mu * c * c + p * p)
        i = int(np.argmax(np.arccos(np.clip(np.abs(c) / np.linalg.norm(verts, axis=1), 0, 1))))
        return R / (img.max() * (p[i] / np.linalg.norm(verts[i])))
    monkeypatch.setattr(lat_oracle, "expansion_nu", bad)
    _fails(tl.test_the_2d_worked_example)


def test_sky_parameters_swapped_are_caught(monkeypatch):
    orig = lat_oracle.sky_direction

    def bad(a1, a2, omega_s, hemisphere, obliquity):
        return orig(a2, a1, omega_s, hemisphere, obliquity)
    monkeypatch.setattr(lat_oracle, "sky_direction", bad)
    _fails(tl.test_sky_directions_invert_the_sky_parameters)


def test_dropped_diurnal_term_of_mu1_is_caught(monkeypatch):
    orig = lat_oracle.linear_model_functions

    def bad(t, T0, det, eph):
        m = orig(t, T0, det, eph)
        xes, yes = model.earth_center(T0 + np.asarray(t), eph)
        m[2] = yes / model.C_LIGHT
        return m
    monkeypatch.setattr(lat_oracle, "linear_model_functions", bad)
    _fails(tl.test_linear_model_drops_only_the_ecliptic_normal_motion)


def test_unshifted_bins_are_caught(monkeypatch):
    monkeypatch.setattr(method, "shift_bins", lambda z, nfft, off: z)
    _fails(tl.test_offset_bins_are_the_continuous_transform)


def test_reversed_bisection_of_the_covering_rule_is_caught(monkeypatch):
    def bad(G0, l, mu, R, nu_lo, rel_tol=1e-12):
        hi = nu_lo * 1.25
        for _ in range(60):
            mid = 0.5 * (nu_lo + hi)
            if lat_oracle.covering_radius(lat_oracle.scaled_generator(G0, l, mu, mid)) <= R:
                hi = mid                               # keeps the lower end
            else:
                nu_lo = mid
        return nu_lo
    monkeypatch.setattr(lat_oracle, "covering_nu", bad)
    _fails(tl.test_covering_rule_on_the_2d_example)
