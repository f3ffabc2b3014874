"""The grid of Sec. IV: a lattice covering of the phase-parameter space with one
basis vector on the frequency axis (oracle; test infrastructure only -- see the
package docstring).

Paper: Sec. III B (the linear phase model, Eqs. philin, albe, siglin; the
reduced Fisher matrix, Eq. redFm-def; the correlation hyperellipsoid, Eqs.
TaylorC2, hype), Sec. IV (the covering problem, Eqs. transf, mmatr, avec,
constraint2; lattices, Voronoi cells, minimal match and deep holes, Eqs.
lattice, mm; the generators of A2* and A4*, Eqs. A2gen, gen; the constrained
lattice, Eqs. opt, opt2; the two-dimensional example, Eqs. gamma2d, ellipse,
constr2d).

Parameters of the linear model with one spindown are
xi = (omega_0, omega_1, alpha_1, alpha_2), with the known functions
m = (t, t^2/2, mu_1(t), mu_2(t)), t the segment time.

Readings of points the paper leaves open:

L-avg    The time average <.> of Eq. (redFm-def) is the mean over the kept
         samples of the segment (gap mask applied), t_j = j dt.  The covariance
         <m_k m_l> - <m_k><m_l> is evaluated in its centred form
         <(m_k - <m_k>)(m_l - <m_l>)>, equal to it up to rounding.
L-white  Any M with M^T G M = 1 maps the hyperellipsoid of Eq. (hype) to a
         sphere; Eq. (mmatr) is one such M.  We take the eigen-decomposition
         of D G D with D = diag(G_kk^-1/2) (the parameters span ~24 decades in
         SI units, beyond what an FP64 eigen-solver resolves unscaled):
         M = D U diag(lambda)^-1/2.  It differs from Eq. (mmatr) by a rotation,
         which the choice of O2 absorbs.
L-nu     The expansion factor nu.  The paper defines it by the covering radius
         staying R and gives an iteration nu_i = R / (R_i sin phi_i) whose
         results disagree with its worked numbers (followed literally it gives
         nu = 1.641 on the two-dimensional example, and in four dimensions a
         fixed point whose covering radius exceeds R); the example prints
         nu = sqrt(108 - pi^2)/9.  That value is exactly the largest nu for
         which the images of the deep holes of the starting lattice (the
         vertices of its Voronoi cell) stay within distance R of the origin:
             nu^2 = min over vertices v of (R^2 - mu^2 (v.l^)^2) / (|v|^2 - (v.l^)^2).
         The image of a Voronoi cell under a linear map is a fundamental domain
         of the image lattice and contains the origin's nearest-point region up
         to translation, so the result is a covering of radius at most R.  The
         same rule gives theta = 2.119 for A4* with |e0| = pi/(2 sqrt 3) and
         R = 1/2, the "about 2.1, 20 % thicker than A4*" of the Virgo example.
L-l      l runs over the lattice vectors with |e0| <= |l| <= 4 max(|e0|, R);
         the first one (in order of increasing length) with the largest
         det S = mu nu^(d-1) is kept.
L-f      The vector f of Eq. (opt2) is the shortest lattice vector that forms
         with l a primitive pair (so that l, f extend to a basis); O3 is the
         rotation in the plane of (f's image orthogonal to e0) and the unit
         vector w of M^-1 span(omega_0, omega_1) orthogonal to e0.
L-basis  The basis a0 = image of l, a1 = image of f, a2, a3 is completed by the
         first pair of integer vectors (coefficients in [-2, 2]) that makes the
         coefficient matrix unimodular, then reduced: the sky projections of
         a2, a3 by Lagrange-Gauss, the omega_1 parts of a2, a3 modulo a1, and
         the omega_0 parts of a1..a3 modulo a0 (nearest integer).
L-sky    A lattice point's sky parameters (alpha_1, alpha_2) = omega_s
         (n_y, n_x) in the ecliptic frame (Eq. albe), omega_s = 2 pi f_sky with
         f_sky the top of the band (the finest sky resolution the band needs).
         Each point inside the disk |alpha| < omega_s gives the two directions
         n_z = +-sqrt(1 - n_x^2 - n_y^2) (the linear model does not tell them
         apart); points outside it are put on the ecliptic (n_z = 0, n scaled
         to unit length).
L-margin The enumeration keeps the lattice points whose covering ellipsoid
         reaches the requested region: each range is widened by the half-width
         of the ellipsoid's shadow, R sqrt((G^-1)_kk) for omega_1 and
         R sqrt(largest eigenvalue of the alpha block of G^-1) in the sky plane.
L-offset A lattice point's frequency gives the offset of its line of Fourier
         bins: bin_offset = frac(omega_0 / dp0), stored as a float32 (a value
         that rounds to 1 is stored as 0, the same line of bins).
"""
from __future__ import annotations

import itertools
import math

import numpy as np

from . import model

THETA_A4STAR = 1.7655   # thickness of A4*, Sec. IV (printed value)


# --------------------------------------------------------------------------
# The linear model and its reduced Fisher matrix (Sec. III B)
# --------------------------------------------------------------------------
def linear_model_functions(t, T0, det, eph):
    """m_k(t) of Eq. (siglin) with one spindown: t, t^2/2, mu_1(t), mu_2(t).

    mu_1 = (R^y_ES + R^y_E cos eps)/c and mu_2 = (R^x_ES + R^x_E)/c (the
    definitions that follow Eq. albe): R_ES in the ecliptic frame, R_E (Earth
    centre to site) in the celestial frame.  t is segment time, T0 the segment
    start on the ephemeris clock."""
    t = np.asarray(t, dtype=np.float64)
    xes, yes = model.earth_center(T0 + t, eph)
    xe, ye, _ = model.site_vector(T0 + t, det, eph)
    mu1 = (yes + ye * math.cos(eph.obliquity)) / model.C_LIGHT
    mu2 = (xes + xe) / model.C_LIGHT
    return np.stack([t, 0.5 * t * t, mu1, mu2])


def reduced_fisher(m, weights=None):
    """Eq. (redFm-def): G_kl = <m_k m_l> - <m_k><m_l>, the average taken with
    the given non-negative weights (reading L-avg: centred form)."""
    m = np.asarray(m, dtype=np.float64)
    w = np.ones(m.shape[1]) if weights is None else np.asarray(weights, dtype=np.float64)
    w = w / w.sum()
    mc = m - (m @ w)[:, None]
    return (mc * w) @ mc.T


def segment_fisher(seg, det, eph):
    """The reduced Fisher matrix of the linear model for one segment, averaged
    over its kept samples (reading L-avg)."""
    t = np.arange(seg.n, dtype=np.float64) * seg.dt
    return reduced_fisher(linear_model_functions(t, seg.t0, det, eph), seg.m)


def whitening(G):
    """M with M^T G M = 1 (Eqs. transf, mmatr; reading L-white)."""
    G = np.asarray(G, dtype=np.float64)
    D = np.diag(1.0 / np.sqrt(np.diag(G)))
    lam, U = np.linalg.eigh(D @ G @ D)
    if lam.min() <= 0:
        raise ValueError("the reduced Fisher matrix is not positive definite")
    return D @ U @ np.diag(1.0 / np.sqrt(lam))


# --------------------------------------------------------------------------
# Lattices (Sec. IV): generators, short vectors, Voronoi cells
# --------------------------------------------------------------------------
def generator_a2star(R):
    """Eq. (A2gen): the hexagonal lattice A2* with covering radius R (rows are
    basis vectors)."""
    return R * math.sqrt(3.0) * np.array([[1.0, 0.0], [0.5, math.sqrt(3.0) / 2]])


def generator_a4star(R):
    """Eq. (gen): A4* with covering radius R (rows are basis vectors)."""
    s2, s3, s5, s6 = math.sqrt(2), math.sqrt(3), math.sqrt(5), math.sqrt(6)
    rows = [[s2, 0, 0, 0],
            [1 / s2, math.sqrt(2 / 3) + 1 / s6, 0, 0],
            [1 / s2, 1 / s6, 1 / (2 * s3) + s3 / 2, 0],
            [-1 / (5 * s2) - 2 * s2 / 5, 1 / (5 * s6) - s6 / 5, -1 / (5 * s3) - s3 / 10, -1 / (2 * s5)]]
    return R * math.sqrt(2.5) * np.array(rows, dtype=np.float64)


def ball_volume(d):
    return math.pi ** (d / 2) / math.gamma(d / 2 + 1)


def thickness(G, R):
    """Covering thickness: volume of the sphere of radius R over the volume of
    the fundamental parallelotope (Sec. IV)."""
    d = G.shape[1]
    return ball_volume(d) * R ** d / abs(np.linalg.det(G))


def short_vectors(G, rho):
    """Integer coefficient vectors z != 0 with |z G| <= rho, by enumeration
    over the triangular form of the Gram matrix (Fincke-Pohst)."""
    G = np.asarray(G, dtype=np.float64)
    d = G.shape[0]
    U = np.linalg.cholesky(G @ G.T).T     # z^T Q z = |U z|^2, U upper triangular
    out = []
    z = [0] * d

    def rec(i, rem):
        c = sum(U[i, j] * z[j] for j in range(i + 1, d))
        r = math.sqrt(max(rem, 0.0))
        lo = math.ceil((-r - c) / U[i, i] - 1e-9)
        hi = math.floor((r - c) / U[i, i] + 1e-9)
        for zi in range(lo, hi + 1):
            z[i] = zi
            v = U[i, i] * zi + c
            if i == 0:
                if any(z):
                    out.append(list(z))
            else:
                rec(i - 1, rem - v * v)
        z[i] = 0

    rec(d - 1, rho * rho * (1 + 1e-12))
    Z = np.array(out, dtype=np.int64).reshape(-1, d)
    V = Z @ G
    keep = np.einsum("ij,ij->i", V, V) <= rho * rho * (1 + 1e-9)
    return Z[keep]


def relevant_vectors(G):
    """The Voronoi-relevant vectors: for each nonzero class of the lattice
    modulo twice itself, its shortest vectors if they are a single pair +-v
    (Voronoi's characterisation).  Enumeration radius sqrt(sum |b*_i|^2), the
    nearest-plane bound on twice the covering radius, which every relevant
    vector meets."""
    G = np.asarray(G, dtype=np.float64)
    d = G.shape[0]
    gs = np.diag(np.linalg.cholesky(G @ G.T))
    Z = short_vectors(G, math.sqrt(float(np.sum(gs * gs))))
    V = Z @ G
    n2 = np.einsum("ij,ij->i", V, V)
    cls = (Z % 2) @ (1 << np.arange(d))
    out = []
    for c in range(1, 1 << d):
        idx = np.nonzero(cls == c)[0]
        if idx.size == 0:
            continue
        m = n2[idx].min()
        low = idx[n2[idx] <= m * (1 + 1e-9)]
        if low.size == 2:
            out.extend(V[low])
    return np.array(out)


def voronoi_vertices(G):
    """Vertices of the Voronoi cell of the origin: points where d facet planes
    x.v = |v|^2/2 of relevant vectors v meet and no facet is violated (every
    d-subset of facets solved, as one batch)."""
    rv = relevant_vectors(G)
    d = rv.shape[1]
    b = 0.5 * np.einsum("ij,ij->i", rv, rv)
    idx = np.array(list(itertools.combinations(range(len(rv)), d)))
    A = rv[idx]
    ok = np.abs(np.linalg.det(A)) >= 1e-12 * np.prod(np.linalg.norm(A, axis=2), axis=1)
    X = np.linalg.solve(A[ok], b[idx[ok]][..., None])[..., 0]
    X = X[np.all(X @ rv.T <= b + 1e-9 * b.max(), axis=1)]
    verts = []
    for x in X:
        if not any(np.linalg.norm(x - y) < 1e-9 * math.sqrt(b.max()) for y in verts):
            verts.append(x)
    return np.array(verts)


def covering_radius(G):
    """The largest distance from the origin to a vertex of its Voronoi cell:
    the distance to a deep hole (Sec. IV, Eq. mm)."""
    V = voronoi_vertices(G)
    return float(np.sqrt(np.einsum("ij,ij->i", V, V)).max())


def nearest_distance(G, x, reach=2):
    """Distance from each point x to the nearest lattice point, by brute force
    over the lattice points whose coefficients lie within +-reach of the
    rounded coefficients of x (for tests on small reduced lattices)."""
    G = np.asarray(G, dtype=np.float64)
    x = np.atleast_2d(x)
    d = G.shape[0]
    z0 = np.rint(x @ np.linalg.inv(G))
    offs = np.array(list(itertools.product(range(-reach, reach + 1), repeat=d)))
    best = np.full(len(x), np.inf)
    for o in offs:
        p = (z0 + o) @ G
        best = np.minimum(best, np.linalg.norm(x - p, axis=1))
    return best


# --------------------------------------------------------------------------
# The constrained lattice (Eqs. opt, opt2)
# --------------------------------------------------------------------------
def _frame(u):
    """An orthogonal matrix whose first column is the unit vector u."""
    d = len(u)
    Q, _ = np.linalg.qr(np.column_stack([u, np.eye(d)]))
    Q = Q[:, :d]
    if Q[:, 0] @ u < 0:
        Q[:, 0] = -Q[:, 0]
    if np.linalg.det(Q) < 0:
        Q[:, -1] = -Q[:, -1]
    return Q


def expansion_nu(verts, l, mu, R):
    """Reading L-nu: the largest nu for which every vertex v of the starting
    Voronoi cell, shrunk by mu along l and expanded by nu across it, stays
    within R."""
    lh = l / np.linalg.norm(l)
    c = verts @ lh
    p2 = np.einsum("ij,ij->i", verts, verts) - c * c
    ok = p2 > 1e-12 * R * R
    return math.sqrt(float(np.min((R * R - mu * mu * c[ok] ** 2) / p2[ok])))


def scaled_generator(G0, l, mu, nu):
    """G0 O1 diag(mu, nu, ..., nu) O1^-1: shrunk by mu along l and expanded by nu
    across it."""
    d = G0.shape[0]
    O1 = _frame(l / np.linalg.norm(l))
    return G0 @ O1 @ np.diag([mu] + [nu] * (d - 1)) @ O1.T


def covering_nu(G0, l, mu, R, nu_lo, rel_tol=1e-12):
    """Reading L-nu, rule 'covering' (the paper's definition of nu): the
    largest nu for which the shrunk and expanded lattice still has covering
    radius R, by bisection.  The covering radius grows with nu (an expansion
    never shortens a distance), and nu_lo (the deep-hole rule's value) is a
    covering."""
    hi = nu_lo * 1.25
    while covering_radius(scaled_generator(G0, l, mu, hi)) <= R:
        nu_lo, hi = hi, hi * 1.25
    while hi - nu_lo > rel_tol * nu_lo:
        mid = 0.5 * (nu_lo + hi)
        if covering_radius(scaled_generator(G0, l, mu, mid)) <= R:
            nu_lo = mid
        else:
            hi = mid
    return nu_lo


def _orbit_key(v, rv):
    """Sorted |v . r| over the relevant vectors r: equal for vectors that a
    symmetry of the lattice maps onto each other (it permutes the relevant
    vectors), which then give congruent constrained lattices."""
    return tuple(np.round(np.sort(np.abs(rv @ v)), 9))


def choose_l(G0, e0_len, R, rule="deep_holes"):
    """Reading L-l: the lattice vector l of the starting lattice with the
    largest det S = mu nu^(d-1), mu = |e0|/|l|, nu by the deep-hole rule or
    (rule 'covering') by the covering radius itself; the latter only over the
    three shortest admissible lengths, one vector per symmetry class."""
    d = G0.shape[0]
    verts = voronoi_vertices(G0)
    Z = short_vectors(G0, 4 * max(e0_len, R))
    V = Z @ G0
    L = np.linalg.norm(V, axis=1)
    rv = relevant_vectors(G0)
    lengths = sorted({round(float(x), 9) for x in L if x >= e0_len * (1 - 1e-12)})
    seen = set()
    best = None
    for i in np.argsort(L, kind="stable"):
        if L[i] < e0_len * (1 - 1e-12):
            continue
        mu = e0_len / L[i]
        nu = expansion_nu(verts, V[i], mu, R)
        if rule == "covering":
            if round(float(L[i]), 9) > lengths[min(2, len(lengths) - 1)]:
                continue
            key = _orbit_key(V[i], rv)
            if key in seen:
                continue
            seen.add(key)
            nu = covering_nu(G0, V[i], mu, R, nu)
        det_s = mu * nu ** (d - 1)
        if best is None or det_s > best["det_s"] * (1 + 1e-12):
            best = dict(z=Z[i], l=V[i], mu=mu, nu=nu, det_s=det_s)
    return best


def constrained_generator(G0, M, a0, R, O3=None, rule="deep_holes", ch=None):
    """Eqs. (opt, opt2): M_opt = M0 O1 S O2^-1 (O3^-1) M^T for the choice of
    choose_l.  Returns the generator (rows in tau coordinates) and the parts."""
    d = G0.shape[0]
    e0 = np.linalg.solve(M, a0)
    e0_len = float(np.linalg.norm(e0))
    if ch is None:
        ch = choose_l(G0, e0_len, R, rule)
    O1 = _frame(ch["l"] / np.linalg.norm(ch["l"]))
    O2 = _frame(e0 / e0_len)
    S = np.diag([ch["mu"]] + [ch["nu"]] * (d - 1))
    X = G0 @ O1 @ S @ O2.T          # rows in the whitened coordinates x
    if O3 is not None:
        X = X @ O3.T
    return dict(M_opt=X @ M.T, X=X, e0=e0, O1=O1, O2=O2, S=S, **ch)


def sky_rotation(M, e0, y):
    """O3 of Eq. (opt2), reading L-f: a rotation fixing e0 that takes the
    whitened vector y into the plane W = {x : (M x)_alpha = 0} (the images of
    W have no alpha_1, alpha_2 components; W contains e0)."""
    d = len(e0)
    eh = e0 / np.linalg.norm(e0)
    _, _, Vt = np.linalg.svd(M[2:, :])
    W = Vt[2:].T                         # orthonormal basis of W (null space)
    q = W.T @ eh
    w = W @ np.array([-q[1], q[0]])      # the unit vector of W orthogonal to e0
    w = w / np.linalg.norm(w)
    yp = y - (y @ eh) * eh
    a = yp / np.linalg.norm(yp)
    c = float(a @ w)
    if c < 0:                            # either direction of w lies in W
        w, c = -w, -c
    b = w - c * a
    if np.linalg.norm(b) < 1e-14:
        return np.eye(d)
    b = b / np.linalg.norm(b)
    s = math.sqrt(max(0.0, 1.0 - c * c))
    return (np.eye(d) + (c - 1.0) * (np.outer(a, a) + np.outer(b, b))
            + s * (np.outer(b, a) - np.outer(a, b)))


def _primitive_pair(zl, zf):
    g = 0
    for i, j in itertools.combinations(range(len(zl)), 2):
        g = math.gcd(g, int(zl[i] * zf[j] - zl[j] * zf[i]))
    return g == 1


def constrained_lattice(G, dp0, c0, rule="deep_holes"):
    """The lattice of Sec. IV for the one-spindown linear model (d = 4):
    A4* with covering radius R = sqrt(1 - C0), shrunk and expanded (Eq. opt),
    turned so that a0 = (dp0, 0, 0, 0) is a lattice vector and a second basis
    vector has no sky components (Eqs. avec, constraint2, opt2).  Returns the
    basis rows a0..a3 (tau coordinates) and the construction's numbers."""
    G = np.asarray(G, dtype=np.float64)
    d = G.shape[0]
    if d != 4:
        raise ValueError("the constrained A4* lattice needs a 4x4 reduced Fisher matrix")
    R = math.sqrt(1.0 - c0)
    M = whitening(G)
    a0 = np.zeros(d)
    a0[0] = dp0
    G0 = generator_a4star(R)
    base = constrained_generator(G0, M, a0, R, rule=rule)
    zl = base["z"]
    ch = {k: base[k] for k in ("z", "l", "mu", "nu", "det_s")}
    # f: shortest vector forming a primitive pair with l (reading L-f)
    Z = short_vectors(G0, 4 * R)
    L = np.linalg.norm(Z @ G0, axis=1)
    zf = None
    for i in np.argsort(L, kind="stable"):
        if _primitive_pair(zl, Z[i]):
            zf = Z[i]
            break
    y = zf @ base["X"]
    O3 = sky_rotation(M, base["e0"], y)
    full = constrained_generator(G0, M, a0, R, O3=O3, ch=ch)
    Mopt = full["M_opt"]
    # basis completion (reading L-basis): det[l; f; g; h] = h . cof(l, f, g)
    box = np.array(list(itertools.product(range(-2, 3), repeat=d)), dtype=np.int64)
    box = box[np.argsort(np.linalg.norm(box @ G0, axis=1), kind="stable")]
    zg = zh = None
    for g in box:
        cof = np.array([round(np.linalg.det(np.array([zl, zf, g, e], dtype=np.float64)))
                        for e in np.eye(d, dtype=np.int64)], dtype=np.int64)
        hit = np.nonzero(np.abs(box @ cof) == 1)[0]
        if hit.size:
            zg, zh = g, box[hit[0]]
            break
    Zb = np.array([zl, zf, zg, zh], dtype=np.int64)
    B = (Zb @ Mopt).astype(np.float64)
    scale = np.abs(Mopt).max(axis=0)
    assert np.all(np.abs(B[0, 1:]) <= 1e-9 * scale[1:]) and abs(B[0, 0] / dp0 - 1) < 1e-9
    assert np.all(np.abs(B[1, 2:]) <= 1e-9 * scale[2:])
    B[0, 1:] = 0.0                        # rounding residue of the constraints
    B[0, 0] = dp0
    B[1, 2:] = 0.0
    B = reduce_basis(B)
    return dict(basis=B, R=R, mu=full["mu"], nu=full["nu"], det_s=full["det_s"],
                theta=THETA_A4STAR / full["det_s"], M=M, M_opt=Mopt, G=G, dp0=dp0, c0=c0, rule=rule)


def reduce_basis(B):
    """Reading L-basis: Lagrange-Gauss on the sky projections of a2, a3, then
    the omega_1 parts of a2, a3 modulo a1 and the omega_0 parts of a1..a3
    modulo a0."""
    B = np.array(B, dtype=np.float64)
    u, v = B[2].copy(), B[3].copy()
    for _ in range(100):
        if u[2:] @ u[2:] > v[2:] @ v[2:]:
            u, v = v, u
        q = round(float((u[2:] @ v[2:]) / (u[2:] @ u[2:])))
        if q == 0:
            break
        v = v - q * u
    B[2], B[3] = u, v
    for i in (2, 3):
        B[i] -= round(B[i, 1] / B[1, 1]) * B[1]
    for i in (1, 2, 3):
        B[i] -= round(B[i, 0] / B[0, 0]) * B[0]
    return B


# --------------------------------------------------------------------------
# Grid nodes from the lattice
# --------------------------------------------------------------------------
def margins(G, R):
    """Reading L-margin: half-widths of the covering ellipsoid's shadow on the
    omega_1 axis and in the sky plane."""
    D = np.diag(1.0 / np.sqrt(np.diag(G)))
    Gi = D @ np.linalg.inv(D @ G @ D) @ D      # G^-1, inverted in the scaled form
    return R * math.sqrt(Gi[1, 1]), R * math.sqrt(float(np.linalg.eigvalsh(Gi[2:, 2:]).max()))


def sky_direction(a1, a2, omega_s, hemisphere, obliquity):
    """Reading L-sky: the sky positions (alpha, delta) of one lattice point's
    sky parameters."""
    nx, ny = a2 / omega_s, a1 / omega_s
    r2 = nx * nx + ny * ny
    if r2 >= 1.0:
        r = math.sqrt(r2)
        zs = [(nx / r, ny / r, 0.0)]
    else:
        nz = math.sqrt(1.0 - r2)
        zs = [(nx, ny, s * nz) for s in ((1.0, -1.0) if hemisphere == 0 else (float(hemisphere),))]
    ce, se = math.cos(obliquity), math.sin(obliquity)
    out = []
    for x, y, z in zs:
        ye = y * ce - z * se
        ze = y * se + z * ce
        out.append((math.atan2(ye, x) % (2 * math.pi), math.asin(max(-1.0, min(1.0, ze)))))
    return out


def lattice_nodes(basis, G, R, f_sky, fdot_lo, fdot_hi, obliquity, sky=None, hemisphere=0, seg=0):
    """All grid nodes of the lattice with the given basis (rows a0..a3 in tau
    coordinates, a0 = (dp0, 0, 0, 0), a1 without sky components) whose
    covering ellipsoid reaches the spindown range [fdot_lo, fdot_hi] and the
    sky region: the disk |alpha| <= 2 pi f_sky, intersected with the disk of
    radius sky[2] around (sky[0], sky[1]) in the (alpha_1, alpha_2) plane when
    sky is given.  Returns records (alpha, delta, fdot, seg, bin_offset, k),
    k the lattice coefficients (k1, k2, k3)."""
    B = np.asarray(basis, dtype=np.float64)
    m1, ma = margins(G, R)
    om = 2 * math.pi * f_sky
    dp0 = B[0, 0]
    S = B[2:, 2:]                     # sky projections of a2, a3 (rows)
    Si = np.linalg.inv(S)
    if sky is not None and sky[2] > 0:
        c = np.array(sky[:2], dtype=np.float64)
        rad = sky[2] + ma
    else:
        c = np.zeros(2)
        rad = om + ma
    span = rad * np.linalg.norm(Si, axis=0)   # k = P S^-1: |k_i - k0_i| <= rad |column i of S^-1|
    k0 = c @ Si
    w_lo, w_hi = 2 * math.pi * fdot_lo - m1, 2 * math.pi * fdot_hi + m1
    recs = []
    for k2 in range(math.floor(k0[0] - span[0]), math.ceil(k0[0] + span[0]) + 1):
        for k3 in range(math.floor(k0[1] - span[1]), math.ceil(k0[1] + span[1]) + 1):
            P = k2 * S[0] + k3 * S[1]
            if np.hypot(*P) > om + ma:
                continue
            if sky is not None and sky[2] > 0 and np.hypot(*(P - c)) > sky[2] + ma:
                continue
            w1 = k2 * B[2, 1] + k3 * B[3, 1]
            w0 = k2 * B[2, 0] + k3 * B[3, 0]
            a11 = B[1, 1]
            ka, kb = sorted(((w_lo - w1) / a11, (w_hi - w1) / a11))
            dirs = sky_direction(P[0], P[1], om, hemisphere, obliquity)
            for al, de in dirs:
                for k1 in range(math.ceil(ka), math.floor(kb) + 1):
                    om1 = k1 * a11 + w1
                    om0 = k1 * B[1, 0] + w0
                    off = np.float32((om0 / dp0) % 1.0)
                    if off >= np.float32(1.0):
                        off = np.float32(0.0)
                    recs.append((al, de, om1 / (2 * math.pi), seg, float(off), (k1, k2, k3)))
    return recs
