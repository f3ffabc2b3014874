"""Pins of the oracle's lattice grid (Sec. III B linear model and reduced Fisher
matrix; Sec. IV constrained covering lattice) against numbers the paper prints,
textbook lattice facts, brute force, and the full Roemer delay."""
import json
import math
import os

import numpy as np
import pytest

from oracle import lattice as L
from oracle import method, model
from tests.common import DET, EPH, small_segment

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
R = 0.5            # C0 = 3/4, as in both worked examples of Sec. IV
G2D = np.array(GOLD["lattice_2d_fisher"]["value"])


def _two_day_segment(nfft=0):
    n = int(round(2 * model.SIDEREAL_DAY / 0.5))
    return method.Segment(x=np.zeros(n), dt=0.5, n_days=2, t0=3.7e6, nfft=nfft)


@pytest.fixture(scope="module")
def lat4():
    seg = _two_day_segment()
    G = L.segment_fisher(seg, DET, EPH)
    dp0 = 2 * math.pi / (seg.fft_len * seg.dt)
    return L.constrained_lattice(G, dp0, 0.75)


# ---------------------------------------------------------------- Sec. III B
def test_reduced_fisher_of_the_2d_example():
    # moments of x and x^2 on [0, 1] by Gauss-Legendre (exact for these
    # degrees): Eq. (gamma2d)
    x, w = np.polynomial.legendre.leggauss(8)
    x, w = 0.5 * (x + 1), 0.5 * w
    G = L.reduced_fisher(np.stack([x, x * x]), w)
    assert np.allclose(G, G2D, rtol=0, atol=1e-15)
    # the correlation ellipse of Eq. (ellipse) is the quadratic form of Eq. (hype)
    tau = np.random.default_rng(1).normal(size=(20, 2))
    q = np.einsum("ij,jk,ik->i", tau, G, tau)
    assert np.allclose(q, (tau[:, 0] + tau[:, 1]) ** 2 / 12 + tau[:, 1] ** 2 / 180, rtol=1e-13)


def test_linear_model_drops_only_the_ecliptic_normal_motion():
    # omega_0 times the full Roemer delay (from the separately pinned model)
    # minus the linear phase alpha_1 mu_1 + alpha_2 mu_2 (Eqs. philin, albe):
    # what remains, up to a constant, is the site's motion normal to the
    # ecliptic, -sin(eps) n_z (R^y_E(t) - R^y_E(0))/c.
    t = np.linspace(0, 2 * model.SIDEREAL_DAY, 500)
    T0 = 1.3e6
    rng = np.random.default_rng(3)
    ce, se = math.cos(EPH.obliquity), math.sin(EPH.obliquity)
    for _ in range(5):
        al, de = rng.uniform(0, 2 * math.pi), math.asin(rng.uniform(-1, 1))
        w0 = 2 * math.pi * 100.0
        a1 = w0 * (math.sin(al) * math.cos(de) * ce + math.sin(de) * se)
        a2 = w0 * math.cos(al) * math.cos(de)
        m = L.linear_model_functions(t, T0, DET, EPH)
        lin = a1 * (m[2] - m[2][0]) + a2 * (m[3] - m[3][0])
        pm = model.roemer_delay(T0 + t, al, de, DET, EPH)
        full = w0 * (pm - pm[0])
        nz = -math.sin(al) * math.cos(de) * se + math.sin(de) * ce
        ye = model.site_vector(T0 + t, DET, EPH)[1]
        dropped = -w0 * se * nz * (ye - ye[0]) / model.C_LIGHT
        assert np.max(np.abs(full - lin - dropped)) < 1e-9 * np.max(np.abs(full))


def test_whitening_maps_the_ellipsoid_to_the_unit_sphere(lat4):
    for G in (G2D, lat4["G"]):
        M = L.whitening(G)
        assert np.allclose(M.T @ G @ M, np.eye(len(G)), atol=1e-9)
    e0 = np.linalg.solve(L.whitening(G2D), [math.pi, 0.0])
    assert abs(np.linalg.norm(e0) - math.pi / (2 * math.sqrt(3))) < 1e-13   # printed
    with pytest.raises(ValueError):
        L.whitening(np.array([[1.0, 2.0], [2.0, 1.0]]))


# ---------------------------------------------------------- lattice geometry
@pytest.mark.parametrize("d", [1, 2, 3, 4])
def test_covering_radius_of_the_cubic_lattice(d):
    # Z^d: deep holes at the cube centres, covering radius sqrt(d)/2
    assert abs(L.covering_radius(np.eye(d)) - math.sqrt(d) / 2) < 1e-12
    assert len(L.voronoi_vertices(np.eye(d))) == 2 ** d


def test_a2star_and_a4star_generators():
    G2 = L.generator_a2star(R)
    assert abs(L.covering_radius(G2) - R) < 1e-12
    assert len(L.voronoi_vertices(G2)) == 6           # regular hexagon
    assert abs(L.thickness(G2, R) - GOLD["lattice_hex_theta"]["value"]) < GOLD["lattice_hex_theta"]["tol"]
    assert abs(L.thickness(G2, R) - 2 * math.pi / (3 * math.sqrt(3))) < 1e-12
    G4 = L.generator_a4star(R)
    assert abs(L.covering_radius(G4) - R) < 1e-12     # Eq. (gen): R is the covering radius
    assert len(L.relevant_vectors(G4)) == 30          # 2 (2^5 - 1) facets: principal lattice
    assert len(L.voronoi_vertices(G4)) == 120         # permutohedron: 5! vertices
    assert abs(L.thickness(G4, R) - GOLD["lattice_a4star_theta"]["value"]) < GOLD["lattice_a4star_theta"]["tol"]


def test_covering_radius_does_not_depend_on_the_basis():
    # a skewed basis of Z^2 and of A2*: same lattice, same covering radius
    U = np.array([[2, 1], [7, 4]])                    # det 1
    assert abs(L.covering_radius(U @ np.eye(2)) - math.sqrt(2) / 2) < 1e-12
    assert abs(L.covering_radius(U @ L.generator_a2star(R)) - R) < 1e-12
    U4 = np.array([[1, 2, 0, 1], [0, 1, 3, 0], [0, 0, 1, 2], [1, 2, 0, 2]])
    assert round(abs(np.linalg.det(U4))) == 1
    assert abs(L.covering_radius(U4 @ L.generator_a4star(R)) - R) < 1e-12


@pytest.mark.parametrize("gen", ["a2", "a4"])
def test_covering_radius_by_brute_force(gen):
    G = L.generator_a2star(R) if gen == "a2" else L.generator_a4star(R)
    d = G.shape[0]
    rng = np.random.default_rng(5)
    x = rng.uniform(-3, 3, size=(4000, d))
    dist = L.nearest_distance(G, x, reach=2)
    assert dist.max() <= R * (1 + 1e-12)
    assert dist.max() > 0.85 * R
    # the deep holes are at distance exactly R from every nearest lattice point
    V = L.voronoi_vertices(G)
    assert np.allclose(L.nearest_distance(G, V + G[0], reach=2), R, atol=1e-12)


# ------------------------------------------------------ constrained lattices
def test_the_2d_worked_example():
    M = L.whitening(G2D)
    a0 = np.array([math.pi, 0.0])
    r = L.constrained_generator(L.generator_a2star(R), M, a0, R)
    assert abs(np.linalg.norm(r["l"]) - 1.5) < 1e-12                 # |sqrt(3)/4 (3, sqrt 3)|
    # l points at a deep hole of A2*, 30 degrees from a minimal vector
    G0 = L.generator_a2star(R)
    mins = np.array([G0[0], G0[1], G0[1] - G0[0]])
    cosang = np.max(np.abs(mins @ r["l"]) / (np.linalg.norm(mins, axis=1) * np.linalg.norm(r["l"])))
    assert abs(cosang - math.cos(math.pi / 6)) < 1e-12
    assert abs(r["mu"] - math.pi / (3 * math.sqrt(3))) < 1e-13
    assert abs(r["nu"] - math.sqrt(108 - math.pi ** 2) / 9) < 1e-13
    theta = L.thickness(r["X"], R)
    assert abs(theta - 18 / math.sqrt(108 - math.pi ** 2)) < 1e-12
    assert abs(theta - GOLD["lattice_2d_theta"]["value"]) < GOLD["lattice_2d_theta"]["tol"]
    assert abs(theta - L.thickness(G0, R) / (r["mu"] * r["nu"])) < 1e-12
    # a covering (radius <= R), with a0 = (pi, 0) a lattice vector (Eq. constr2d)
    assert L.covering_radius(r["X"]) <= R * (1 + 1e-12)
    assert np.allclose(r["z"] @ r["M_opt"], a0, atol=1e-12)


def test_virgo_thickness():
    # |e0| = pi/(2 sqrt 3): a resolution of half a Fourier bin of the whole
    # observation (Delta p0 = pi/T0), as in the worked example; C0 = 3/4
    seg = _two_day_segment()
    G = L.segment_fisher(seg, DET, EPH)
    T0 = seg.n * seg.dt
    lat = L.constrained_lattice(G, math.pi / T0, 0.75)
    g = GOLD["lattice_virgo_theta"]
    assert abs(lat["theta"] - g["value"]) < g["tol"]
    assert abs(lat["theta"] / L.THETA_A4STAR - g["ratio_to_a4star"]) < g["ratio_tol"]
    X = np.linalg.solve(lat["M"], lat["basis"].T).T
    assert abs(L.thickness(X, lat["R"]) - lat["theta"]) < 1e-3   # printed 1.7655 vs exact
    assert L.covering_radius(X) <= lat["R"] * (1 + 1e-9)


def test_constrained_lattice_structure(lat4):
    B, M, Rr = lat4["basis"], lat4["M"], lat4["R"]
    # Eq. (avec): a0 on the frequency axis with the Fourier resolution
    assert B[0, 0] == lat4["dp0"] and np.all(B[0, 1:] == 0)
    # Eq. (constraint2): the spindown basis vector has no sky components
    assert np.all(B[1, 2:] == 0) and B[1, 1] != 0
    # the reduced basis spans the lattice of Eq. (opt2)
    T = B @ np.linalg.inv(lat4["M_opt"])
    assert np.allclose(T, np.rint(T), atol=1e-6) and round(abs(np.linalg.det(np.rint(T)))) == 1
    # a covering of radius R in the whitened coordinates, of the stated thickness
    X = np.linalg.solve(M, B.T).T
    assert L.covering_radius(X) <= Rr * (1 + 1e-9)
    assert abs(L.thickness(X, Rr) - L.thickness(L.generator_a4star(Rr), Rr) / lat4["det_s"]) < 1e-9
    assert lat4["mu"] <= 1 and lat4["nu"] >= 1 - 1e-12


def test_sky_directions_invert_the_sky_parameters():
    # Eq. (albe) forward, the node mapping backward: both hemispheres appear
    rng = np.random.default_rng(9)
    ce, se = math.cos(EPH.obliquity), math.sin(EPH.obliquity)
    om = 2 * math.pi * 300.0
    for _ in range(20):
        al, de = rng.uniform(0, 2 * math.pi), math.asin(rng.uniform(-1, 1))
        a1 = om * (math.sin(al) * math.cos(de) * ce + math.sin(de) * se)
        a2 = om * math.cos(al) * math.cos(de)
        dirs = L.sky_direction(a1, a2, om, 0, EPH.obliquity)
        assert len(dirs) == 2
        err = min(abs(math.remainder(d[0] - al, 2 * math.pi)) + abs(d[1] - de) for d in dirs)
        assert err < 1e-9
    # outside the disk: one direction, on the ecliptic
    (al, de), = L.sky_direction(1.2 * om, 0.0, om, 0, EPH.obliquity)
    n = (math.cos(al) * math.cos(de), math.sin(al) * math.cos(de), math.sin(de))
    assert abs(-n[1] * se + n[2] * ce) < 1e-12


def _lattice_point(B, k):
    k1, k2, k3 = k
    return k1 * B[1] + k2 * B[2] + k3 * B[3]


def test_nodes_cover_a_sky_patch(lat4):
    B, G, Rr = lat4["basis"], lat4["G"], lat4["R"]
    f_sky = 436.0
    om = 2 * math.pi * f_sky
    c = np.array([0.3 * om, -0.4 * om])                 # patch centre in (alpha_1, alpha_2)
    rad = 120.0
    assert np.hypot(*c) + rad < om                      # the patch lies inside the sky disk
    recs = L.lattice_nodes(B, G, Rr, f_sky, -2e-10, 0.0, EPH.obliquity, sky=(c[0], c[1], rad))
    assert len(recs) > 10
    pts = np.array([_lattice_point(B, r[5]) for r in recs])
    # every node's bin offset is the fraction of its frequency line
    for r, p in zip(recs, pts):
        want = np.float32((p[0] / B[0, 0]) % 1.0)
        assert r[4] == (0.0 if want >= np.float32(1.0) else float(want))
        assert abs(r[2] - p[1] / (2 * math.pi)) <= 1e-12 * max(1e-9, abs(r[2]))
    # random parameters inside the region lie within R (metric) of a node's line
    rng = np.random.default_rng(11)
    ang = rng.uniform(0, 2 * math.pi, 300)
    rr = rad * np.sqrt(rng.uniform(0, 1, 300))
    q = np.column_stack([rng.uniform(0, 50 * B[0, 0], 300),
                         2 * math.pi * rng.uniform(-2e-10, 0.0, 300),
                         c[0] + rr * np.cos(ang), c[1] + rr * np.sin(ang)])
    M = lat4["M"]
    Mi = np.linalg.inv(M)
    for p in q:
        best = np.inf
        for n in pts:
            dtau = p - n
            # the best point of the node's frequency line n + k a0
            x = Mi @ dtau
            e = Mi @ B[0]
            k = (x @ e) / (e @ e)
            for kk in (math.floor(k), math.ceil(k)):
                best = min(best, np.linalg.norm(x - kk * e))
        assert best <= Rr * (1 + 1e-9), best


def test_full_sky_node_count(lat4):
    # the count of lattice sky points in the disk is its area over the sky
    # cell, each doubled by the two hemispheres
    B, G, Rr = lat4["basis"], lat4["G"], lat4["R"]
    f_sky = 21.0
    om = 2 * math.pi * f_sky
    recs = L.lattice_nodes(B, G, Rr, f_sky, 0.0, 0.0, EPH.obliquity)
    sky = {r[5][1:] for r in recs}
    _, ma = L.margins(G, Rr)
    cell = abs(np.linalg.det(B[2:, 2:]))
    assert abs(len(sky) - math.pi * (om + ma) ** 2 / cell) < 0.05 * len(sky) + 10


def test_offset_bins_are_the_continuous_transform():
    # F at bins k + off by the DFT of the shifted series equals F at the
    # continuous frequencies (k + off)/(nfft dt) by the direct sum
    seg = small_segment(days=1, dt=26.0, seed=4)
    nfft = seg.fft_len
    al, de, fd = 1.1, -0.4, -3e-10
    k = np.array([3, 40, 41, 500, nfft // 2 - 2])
    for off in (0.0, 0.25, 0.731):
        Fb = method.fstat_bins(seg, fd, al, de, DET, EPH, method.LINEAR_UP2, k=k, bin_offset=off)
        Fc = [method.fstat_continuous(seg, ((kk + off) / (nfft * seg.dt), fd, al, de), DET, EPH, method.LINEAR_UP2)
              for kk in k]
        assert np.max(np.abs(Fb - Fc)) < 1e-9 * max(1.0, np.max(Fc))
    # the interbinned variant shifts its half bins the same way
    F0, Fh = method.fstat_bins_interbinned(seg, fd, al, de, DET, EPH, method.LINEAR_UP2, k=k, bin_offset=0.4)
    assert np.allclose(F0, method.fstat_bins(seg, fd, al, de, DET, EPH, method.LINEAR_UP2, k=k, bin_offset=0.4),
                       rtol=1e-12, atol=1e-12)


def test_covering_rule_on_the_2d_example():
    # nu by the paper's definition (the covering radius stays R).  The shrunk
    # hexagonal lattice is centred-rectangular with half sides a = 3 mu/4 along
    # l and b = sqrt(3) nu/4 across it; once b > a its deep holes are the
    # circumcentres of the triangles (0, (2a, 0), (a, b)) at distance
    # (a^2 + b^2)/(2b), so covering radius R gives b = R + sqrt(R^2 - a^2).
    M = L.whitening(G2D)
    r = L.constrained_generator(L.generator_a2star(R), M, np.array([math.pi, 0.0]), R, rule="covering")
    mu = math.pi / (3 * math.sqrt(3))
    a = 3 * mu / 4
    b = R + math.sqrt(R * R - a * a)
    assert abs(r["mu"] - mu) < 1e-13
    assert abs(r["nu"] - 4 * b / math.sqrt(3)) < 1e-9
    assert abs(L.covering_radius(r["X"]) - R) < 1e-9 and L.covering_radius(r["X"]) <= R * (1 + 1e-12)
    theta = L.thickness(r["X"], R)
    assert abs(theta - L.thickness(L.generator_a2star(R), R) / (mu * r["nu"])) < 1e-9
    assert theta < 0.7 * GOLD["lattice_2d_theta"]["value"]      # 1.2186 against the printed 1.8171


def test_covering_rule_in_four_dimensions(lat4):
    lat = L.constrained_lattice(lat4["G"], lat4["dp0"], 0.75, rule="covering")
    X = np.linalg.solve(lat["M"], lat["basis"].T).T
    cr = L.covering_radius(X)
    assert cr <= lat["R"] * (1 + 1e-9) and cr >= lat["R"] * (1 - 1e-9)
    assert lat["theta"] < lat4["theta"] and lat["nu"] >= lat4["nu"]
    assert abs(L.thickness(X, lat["R"]) - L.thickness(L.generator_a4star(lat["R"]), lat["R"]) / lat["det_s"]) < 1e-9
    assert np.all(lat["basis"][0, 1:] == 0) and np.all(lat["basis"][1, 2:] == 0)
