"""Pins of the CPU oracle: checks against what the paper and the mathematics fix,
independent of the oracle's own formulas.

Each ``check_*`` takes the oracle module (so that a test can hand in a copy
with a planted mistake) and raises AssertionError when the pin does not hold.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla

from workloads.gen import random_band_pencil


def tiny_pencil(n=14, k=2, seed=7, b_kind="identity"):
    return random_band_pencil(n, k, seed, b_kind=b_kind, b_offdiag=0.3)


def base_params(**kw):
    p = dict(x0=-1.0, x1=1.0, y0=-1.0, y1=1.0, n1=2, gauss_per_edge=8, m=10,
             h0=1e-3, levels=0, eps0=1e-8, delta0=0.05, tau=1e-8)
    p.update(kw)
    return p


# P1 -- Gauss-Legendre rule: library rule, exact for degree <= 2g-1.
def check_p1_gauss_rule(O, g=8):
    c, w = 0.3 - 0.2j, 0.5
    z, wt = O.edge_rule(c, w, g)
    assert len(z) == 4 * g
    # closed contour: sum of dz is 0, and polynomial integrands integrate to 0
    for p in range(0, 2 * g - 1):
        val = np.sum(wt * (z - c) ** p)
        assert abs(val) < 1e-13 * max(1.0, w ** (p + 1)), (p, val)
    # each edge: the weights sum to the edge vector b - a
    h = w / 2
    corners = [c + h * (-1 - 1j), c + h * (1 - 1j), c + h * (1 + 1j), c + h * (-1 + 1j)]
    for e in range(4):
        seg = wt[e * g:(e + 1) * g]
        assert abs(seg.sum() - (corners[(e + 1) % 4] - corners[e])) < 1e-14
        # integral of (z - a) along the edge = (b - a)^2 / 2
        a, b = corners[e], corners[(e + 1) % 4]
        val = np.sum(seg * (z[e * g:(e + 1) * g] - a))
        assert abs(val - (b - a) ** 2 / 2) < 1e-14
    # nodes strictly inside the edges, never on a corner
    for e in range(4):
        a, b = corners[e], corners[(e + 1) % 4]
        t = (z[e * g:(e + 1) * g] - a) / (b - a)
        assert np.all(np.abs(t.imag) < 1e-12) and np.all(t.real > 0) and np.all(t.real < 1)


# P2 -- scalar closed form: (1/2 pi i) oint dz / (a - z) = -1 inside, 0 outside.
def check_p2_scalar_contour(O):
    A = np.array([[0.1 + 0.05j]])
    B = np.eye(1, dtype=complex)
    f = np.ones(1, dtype=complex)
    inside = O.direct_projection(A, B, f, 0.0, 1.0, 24)[0]
    assert abs(inside - (-1.0)) < 1e-10, inside
    # pole one width away from the square: quadrature error decays with g
    errs = [abs(O.direct_projection(np.array([[1.5 + 0j]]), B, f, 0.0, 1.0, g)[0]) for g in (4, 8, 16)]
    assert errs[1] < 1e-3 * errs[0] + 1e-15 and errs[2] < 1e-3 * errs[1] + 1e-15, errs
    # same through the Krylov path (m = n = 1)
    from workloads.gen import Pencil
    band = np.array([[0.1 + 0.05j]], dtype=complex)
    pen = Pencil(1, 0, 0, band, 0, 0, None)
    sh = O.build_shift(pen, 0.3 + 0.3j, f, 1)
    ev = O.evaluate_square(sh, 0.0, 1.0, base_params(m=1, gauss_per_edge=16))
    x = sh.V[:, :1] @ ev.s_f
    assert abs(x[0] - (-1.0)) < 1e-10, x


# P3 -- additivity: the four children's coarse sums add up to the parent's
# composite two-panel rule (interior edges cancel).
def check_p3_additivity(O):
    pen, f = tiny_pencil()
    sh = O.build_shift(pen, 0.05 + 0.02j, f, 10, keep_V=False)
    params = base_params()
    g = params["gauss_per_edge"]
    center, width = 0.1 + 0.2j, 0.4
    # composite rule built independently of edge_rule: each parent edge in 2 halves
    t, om = np.polynomial.legendre.leggauss(g)
    h = width / 2
    corners = [center + h * (-1 - 1j), center + h * (1 - 1j), center + h * (1 + 1j), center + h * (-1 + 1j)]
    zs, ws = [], []
    for e in range(4):
        a, b = corners[e], corners[(e + 1) % 4]
        mid = (a + b) / 2
        for (p, q) in ((a, mid), (mid, b)):
            zs.append(p + (t + 1) * (q - p) / 2)
            ws.append(om * (q - p) / 2)
    z = np.concatenate(zs)
    w = np.concatenate(ws)
    Y = O.shifted_solutions(sh, z)
    parent = (w[:, None] * Y).sum(0) / (2j * np.pi)
    acc = np.zeros_like(parent)
    for dy in (-1, 1):
        for dx in (-1, 1):
            cc = center + (dx + 1j * dy) * width / 4
            acc += O.evaluate_square(sh, cc, width / 2, params).s_c
    assert np.linalg.norm(acc - parent) <= 1e-11 * max(1.0, np.linalg.norm(parent)), np.linalg.norm(acc - parent)


# P4 -- reduced = direct when m = n: V_m s_f is the direct quadrature of P f.
def check_p4_reduced_equals_direct(O, b_kind="identity"):
    pen, f = tiny_pencil(n=12, b_kind=b_kind)
    A, B = O.pencil_dense(pen)
    sigma = 0.2 - 0.1j
    sh = O.build_shift(pen, sigma, f, pen.n)
    assert sh.m_eff == pen.n
    params = base_params(m=pen.n)
    for center, width in ((0.0, 2.0), (0.5 + 0.5j, 1.0), (-0.3 + 0.1j, 0.25)):
        ev = O.evaluate_square(sh, center, width, params)
        x_kry = sh.V[:, : sh.m_eff] @ ev.s_f
        x_dir = O.direct_projection(A, B, f, center, width, 2 * params["gauss_per_edge"])
        scale = max(np.linalg.norm(x_dir), 1e-3 * np.linalg.norm(f))
        assert np.linalg.norm(x_kry - x_dir) <= 1e-10 * scale, (center, np.linalg.norm(x_kry - x_dir), scale)


# P5 -- Arnoldi relation (eq. (arnoldi)), orthonormality, and eig(H_n) = 1/(lambda - sigma).
def check_p5_arnoldi(O, b_kind="identity"):
    pen, f = tiny_pencil(n=40, k=3, b_kind=b_kind)
    A, B = O.pencil_dense(pen)
    sigma = 0.1 + 0.3j
    M = np.linalg.solve(A - sigma * B, B)
    sh = O.build_shift(pen, sigma, f, 25)
    m = sh.m_eff
    V = sh.V
    R = M @ V[:, :m] - V[:, :m] @ sh.Hm - np.outer(V[:, m], sh.H[m, :])
    assert np.linalg.norm(R) <= 1e-12 * np.linalg.norm(M, 2), np.linalg.norm(R)
    assert np.linalg.norm(V.conj().T @ V - np.eye(m + 1)) <= 1e-13
    b = np.linalg.solve(A - sigma * B, f)
    assert abs(sh.beta - np.linalg.norm(b)) <= 1e-13 * sh.beta
    assert np.allclose(V[:, 0] * sh.beta, b, rtol=0, atol=1e-13 * sh.beta)
    # subdiagonal real and positive
    sub = np.diag(sh.H, -1)
    assert np.all(np.abs(sub.imag) == 0) and np.all(sub.real > 0)
    # m = n: H's eigenvalues are 1/(lambda - sigma)
    shn = O.build_shift(pen, sigma, f, pen.n)
    theta = np.linalg.eigvals(shn.Hm)
    lam = sla.eigvals(A, B)
    want = 1.0 / (lam - sigma)
    for t in theta:
        assert np.min(np.abs(want - t)) <= 1e-9 * max(1.0, abs(t)), t


# P6 -- residual formula (eq. (error)) equals the explicit residual.
def check_p6_residual(O, b_kind="identity"):
    pen, f = tiny_pencil(n=30, k=2, b_kind=b_kind)
    A, B = O.pencil_dense(pen)
    sigma = -0.2 + 0.1j
    M = np.linalg.solve(A - sigma * B, B)
    b = np.linalg.solve(A - sigma * B, f)
    sh = O.build_shift(pen, sigma, f, 8)
    z, _ = O.edge_rule(0.1 + 0.1j, 0.6, 4)
    Y = O.shifted_solutions(sh, z)
    rho = O.residuals(sh, z, Y)
    for j in range(len(z)):
        x = sh.V[:, : sh.m_eff] @ Y[j]
        r = b - (x + (sigma - z[j]) * (M @ x))
        explicit = np.linalg.norm(r) / sh.beta
        assert abs(explicit - rho[j]) <= 1e-9 * explicit + 1e-14, (j, explicit, rho[j])


# P7 -- reduced norm equals full-space norm (V orthonormal).
def check_p7_reduced_norm(O):
    pen, f = tiny_pencil(n=40, k=3)
    sh = O.build_shift(pen, 0.05j, f, 20)
    ev = O.evaluate_square(sh, 0.0, 0.5, base_params(m=20))
    for s in (ev.s_c, ev.s_f):
        full = np.linalg.norm(sh.V[:, : sh.m_eff] @ s)
        assert abs(full - np.linalg.norm(s)) <= 1e-13 * max(full, 1e-300)


# P8 -- P f = 0 for squares free of eigenvalues (eq. (P) and what follows it).
def check_p8_empty_square(O):
    pen, f = tiny_pencil(n=60, k=2, seed=11)
    A, B = O.pencil_dense(pen)
    lam = sla.eigvals(A, B)
    params = base_params(m=60)
    sh = O.build_shift(pen, 0.0, f, 60)
    tested = 0
    rng = np.random.default_rng(3)
    for _ in range(400):
        c = complex(rng.uniform(-2, 2), rng.uniform(-2, 2))
        w = 0.1
        # distance of every eigenvalue from the square's boundary > one width, none inside
        dx = np.maximum(np.abs(lam.real - c.real) - w / 2, 0)
        dy = np.maximum(np.abs(lam.imag - c.imag) - w / 2, 0)
        if np.min(np.hypot(dx, dy)) <= w:
            continue
        ev = O.evaluate_square(sh, c, w, params)
        assert ev.resolvable
        assert ev.nsf <= 1e-6 * ev.Tf, (c, ev.nsf, ev.Tf)
        assert not ev.admissible
        tested += 1
    assert tested >= 20


# P9 -- idempotency of the (Riesz) projector: Q(Q f) = Q f, for squares whose
# eigenvalues (inside and out) keep a quarter width from the boundary.
def check_p9_idempotent(O):
    pen, f = tiny_pencil(n=50, k=2, seed=5, b_kind="tridiag")
    A, B = O.pencil_dense(pen)
    lam = sla.eigvals(A, B)
    count = 0
    rng = np.random.default_rng(17)
    for _ in range(300):
        if count >= 3:
            break
        c = complex(rng.uniform(-1.5, 1.5), rng.uniform(-1.5, 1.5))
        w = rng.uniform(0.3, 1.0)
        inside = (np.abs(lam.real - c.real) < w / 2) & (np.abs(lam.imag - c.imag) < w / 2)
        edge = np.minimum(w / 2 - np.abs(lam.real - c.real), w / 2 - np.abs(lam.imag - c.imag))
        if not inside.any() or np.min(np.abs(edge)) < 0.25 * w:
            continue
        Qf = O.riesz_apply(A, B, f, c, w, 48)
        QQf = O.riesz_apply(A, B, Qf, c, w, 48)
        assert np.linalg.norm(QQf - Qf) <= 1e-8 * np.linalg.norm(Qf)
        count += 1
    assert count >= 1


# P10 -- diagonal pencil: the whole Krylov pipeline reduces to a scalar closed form.
def check_p10_diagonal(O):
    from workloads.gen import Pencil
    n = 16
    rng = np.random.default_rng(21)
    d = rng.uniform(-1, 1, n) + 1j * rng.uniform(-1, 1, n)
    band = d.reshape(1, n).astype(complex)
    pen = Pencil(n, 0, 0, band, 0, 0, None)
    f = (rng.standard_normal(n) + 1j * rng.standard_normal(n)) / np.sqrt(2)
    sigma = 0.05 + 0.02j
    sh = O.build_shift(pen, sigma, f, n)
    params = base_params(m=n)
    for center, width in ((0.0, 1.0), (0.4 - 0.3j, 0.5)):
        ev = O.evaluate_square(sh, center, width, params)
        for rule_g, s in ((8, ev.s_c), (16, ev.s_f)):
            # q(d) = (1/2 pi i) sum_j w_j / (z_j - d) on an independently built rule
            t, om = np.polynomial.legendre.leggauss(rule_g)
            h = width / 2
            cs = [center + h * (-1 - 1j), center + h * (1 - 1j), center + h * (1 + 1j), center + h * (-1 + 1j)]
            q = np.zeros(n, dtype=complex)
            for e in range(4):
                a, b = cs[e], cs[(e + 1) % 4]
                for tt, oo in zip(t, om):
                    zz = a + (tt + 1) * (b - a) / 2
                    q += oo * (b - a) / 2 / (zz - d)
            q /= 2j * np.pi
            want = -f * q
            got = sh.V[:, :n] @ s
            assert np.linalg.norm(got - want) <= 1e-10 * max(1.0, np.linalg.norm(want))
        ind = np.linalg.norm(ev.s_f) / np.linalg.norm(ev.s_c)
        assert abs(ind - ev.indicator) <= 1e-14 * ind


# P11 -- whole pipeline versus dense QZ.
EDGE_BLIND = 0.002   # relative distance from a square edge below which the ratio indicator may miss a pole


def edge_closeness(params, K, lam):
    """Smallest distance, in units of the square width, between lam and an edge
    of the square holding it, over all levels 1..K."""
    best = math.inf
    for k in range(1, K + 1):
        w = math.ldexp((params["x1"] - params["x0"]) / params["n1"], 1 - k)
        for u in ((lam.real - params["x0"]) / w, (lam.imag - params["y0"]) / w):
            fr = u - math.floor(u)
            best = min(best, fr, 1.0 - fr)
    return best


def check_p11_against_qz(O, pen, f, params, res=None):
    A, B = O.pencil_dense(pen)
    lam = sla.eigvals(A, B)
    if res is None:
        res = O.simm(pen, f, params)
    h = O.square_width(params, res.K)
    x0, x1, y0, y1 = params["x0"], params["x1"], params["y0"], params["y1"]
    inR = lam[(lam.real > x0) & (lam.real < x1) & (lam.imag > y0) & (lam.imag < y1)]
    far = inR[(inR.real > x0 + 2 * h) & (inR.real < x1 - 2 * h) & (inR.imag > y0 + 2 * h) & (inR.imag < y1 - 2 * h)]
    exempt = [l for l in far if edge_closeness(params, res.K, l) < EDGE_BLIND]
    assert len(exempt) <= 0.25 * len(far) + 1, exempt
    lam_c = np.array([c.lam for c in res.clusters])
    lam_r = np.array([c.lam_ritz for c in res.clusters])
    owners = []
    for l in far:
        hits = [i for i, c in enumerate(res.clusters)
                if any(abs(l.real - O.square_center(params, res.K, *k).real) <= h / 2 and
                       abs(l.imag - O.square_center(params, res.K, *k).imag) <= h / 2 for k in c.members)]
        if any(l == e for e in exempt) and not hits:
            continue
        # lies in exactly one cluster: the cluster whose squares contain it
        assert len(hits) == 1, (l, hits)
        owners.append(hits[0])
        assert np.min(np.abs(lam_c - l)) <= 1.5 * h
        assert np.nanmin(np.abs(lam_r - l)) <= 1e-8 * max(1.0, abs(l))
    assert len(set(owners)) == len(owners)
    # no spurious clusters, and the counts agree up to the exempt eigenvalues
    for c in res.clusters:
        assert np.min(np.abs(lam - c.lam)) <= 1.5 * h
    assert len(inR) - len(exempt) <= len(res.clusters) <= len(inR), (len(res.clusters), len(inR), len(exempt))
    return res


# P12 -- the shifted solver (dense and LAPACK band paths): backward error.
def check_p12_solver(O):
    pen, f = random_band_pencil(4100, 3, 99, b_kind="tridiag")
    sigma = 0.3 - 0.4j
    solver = O.ShiftedSolver(pen, sigma)
    assert solver._band is not None
    x = solver.solve(f)
    Cx = O.band_matvec(pen.n, pen.kl_a, pen.ku_a, pen.a_band, x) - sigma * O.band_matvec(pen.n, pen.kl_b, pen.ku_b, pen.b_band, x)
    normC = np.abs(pen.a_band).sum(0).max() + abs(sigma) * np.abs(pen.b_band).sum(0).max()
    berr = np.linalg.norm(Cx - f) / (normC * np.linalg.norm(x))
    assert berr <= 1e-14, berr
    # dense path on a small pencil agrees with numpy's solve of the dense matrix
    pen2, f2 = tiny_pencil(n=50, k=4, b_kind="tridiag")
    A, B = O.pencil_dense(pen2)
    s2 = O.ShiftedSolver(pen2, sigma)
    assert np.allclose(s2.solve(f2), np.linalg.solve(A - sigma * B, f2), rtol=1e-12, atol=0)


# P13 -- the eigendecomposition formula of Sec. 3.2: e_m^T y_j = beta r_m Lambda_j c_1.
def check_p13_eig_identity(O):
    pen, f = tiny_pencil(n=40, k=3)
    sh = O.build_shift(pen, 0.1, f, 15)
    D, P = np.linalg.eig(sh.Hm)
    Pinv = np.linalg.inv(P)
    rm, c1 = P[-1, :], Pinv[:, 0]
    z, _ = O.edge_rule(0.2 + 0.1j, 0.4, 8)
    Y = O.shifted_solutions(sh, z)
    for j in range(len(z)):
        lamj = 1.0 / (1.0 + (sh.sigma - z[j]) * D)
        terms = sh.beta * rm * lamj * c1
        want = np.sum(terms)
        # rounding bound of the sum: relative to the sum of the terms' moduli
        assert abs(Y[j, -1] - want) <= 1e-12 * np.sum(np.abs(terms)), (j, Y[j, -1], want)


# P14 -- maximum principle on the residual: with no Ritz pole in a square, the
# residual inside never exceeds the residual on the boundary.
def check_p14_max_principle(O):
    pen, f = tiny_pencil(n=60, k=2, seed=4)
    sh = O.build_shift(pen, 0.0, f, 12)
    ritz = O.ritz_values(sh)
    rng = np.random.default_rng(9)
    checked = 0
    for _ in range(60):
        c = complex(rng.uniform(-0.6, 0.6), rng.uniform(-0.6, 0.6))
        w = 0.3
        if np.any((np.abs(ritz.real - c.real) <= w / 2 + 1e-3) & (np.abs(ritz.imag - c.imag) <= w / 2 + 1e-3)):
            continue
        zb, _ = O.edge_rule(c, w, 64)
        rb = O.residuals(sh, zb, O.shifted_solutions(sh, zb)).max()
        zi = c + (rng.uniform(-0.45, 0.45, 200) + 1j * rng.uniform(-0.45, 0.45, 200)) * w
        ri = O.residuals(sh, zi, O.shifted_solutions(sh, zi)).max()
        assert ri <= rb * (1 + 1e-6), (c, ri, rb)
        checked += 1
    assert checked >= 5


# ---------------------------------------------------------------------------
# Multiplicities (Sec. 3.4) on a pencil with planted eigenvalues.
# ---------------------------------------------------------------------------

def _planted_run(O):
    import json
    from workloads import make_workload, load_config, start_vectors
    pen, f, params = make_workload("mult0")
    cfg = load_config("mult0")
    res = O.simm(pen, f, params)
    F = start_vectors(pen.n, cfg["multiplicity"]["k"], cfg["generator"]["seed"])
    planted = [(complex(*v), int(c), bool(j)) for v, c, j in cfg["generator"]["planted"]]
    return pen, params, res, F, planted


def _square_nodes(center, width, g):
    """Counter-clockwise boundary of a square with g Gauss-Legendre nodes per edge,
    weights including dz/dt (written here from the rule's definition)."""
    t, om = np.polynomial.legendre.leggauss(g)
    h = width / 2.0
    corners = [center + h * c for c in (-1 - 1j, 1 - 1j, 1 + 1j, -1 + 1j)]
    z, w = [], []
    for e in range(4):
        a, b = corners[e], corners[(e + 1) % 4]
        z.append(a + (t + 1.0) * (b - a) / 2.0)
        w.append(om * (b - a) / 2.0)
    return np.concatenate(z), np.concatenate(w)


# P15 -- the multiplicity of each planted eigenvalue is its construction's: the
# rank of the spectral projector (3 and 2 for semisimple repeats, 2 for a 2 x 2
# Jordan block, 1 for a simple one), with a wide gap to the rounding level.
def check_p15_multiplicities(O, run=None):
    pen, params, res, F, planted = run or _planted_run(O)
    K = res.K
    wK = O.square_width(params, K)
    X = O.cluster_projections(pen, res, F, params)
    out = O.multiplicities(X)
    found = 0
    for c, (mult, sv) in zip(res.clusters, out):
        centres = [O.square_center(params, K, ix, iy) for ix, iy in c.members]
        lo = min(z.real for z in centres) - wK / 2, min(z.imag for z in centres) - wK / 2
        hi = max(z.real for z in centres) + wK / 2, max(z.imag for z in centres) + wK / 2
        inside = [(v, cnt) for v, cnt, _ in planted if lo[0] <= v.real <= hi[0] and lo[1] <= v.imag <= hi[1]]
        expect = inside[0][1] if inside else 1     # a random eigenvalue near the edge of R is simple
        found += bool(inside)
        assert mult == expect, (c.lam, mult, expect, sv / sv[0])
        assert sv[mult - 1] > 1e-3 * sv[0], (c.lam, sv / sv[0])
        if mult < len(sv):
            assert sv[mult] < 1e-10 * sv[0], (c.lam, sv / sv[0])
    assert found == len(planted)


# P16 -- the cluster projections equal the direct quadrature of (A - z B)^{-1} f_i
# over the cluster's squares (dense solves, no Krylov space; eq. (XLXf) with the
# systems of eq. (linearsys)).
def check_p16_cluster_projection_direct(O, run=None):
    pen, params, res, F, planted = run or _planted_run(O)
    A, B = O.pencil_dense(pen)
    K = res.K
    wK = O.square_width(params, K)
    X = O.cluster_projections(pen, res, F, params)
    for c, Xc in zip(res.clusters, X):
        D = np.zeros_like(Xc)
        for ix, iy in c.members:
            z, w = _square_nodes(O.square_center(params, K, ix, iy), wK, 2 * params["gauss_per_edge"])
            for zj, wj in zip(z, w):
                D += wj * np.linalg.solve(A - zj * B, F)
        D /= 2j * np.pi
        err = np.linalg.norm(Xc - D) / np.linalg.norm(D)
        assert err <= 1e-8, (c.lam, err)


# P17 -- gradient of the projected-vector norms: the adjoint gradient against central
# finite differences of J itself (h = 1e-6), for A = A0 + p A1 and for the real and
# imaginary parts of diagonal entries.  J is the direct quadrature pinned by P4/P16.
def gradient_case(O):
    pen, f = random_band_pencil(60, 2, 7, b_kind="tridiag", b_offdiag=0.2)
    A, B = O.pencil_dense(pen)
    rng = np.random.default_rng(3)
    A1 = np.diag(rng.standard_normal(60)) * 0.3 + np.diag(rng.standard_normal(59), 1) * 0.1
    ev = np.linalg.eigvals(np.linalg.solve(B, A))
    # three squares around eigenvalues (none on an edge), one far from every eigenvalue
    squares = [(complex(round(l.real, 1), round(l.imag, 1)), 0.4) for l in ev[:3]] + [(5.0 + 5.0j, 0.4)]
    return A, A1, B, f, squares


def check_p17_gradient(O, h=1e-6):
    A, A1, B, f, squares = gradient_case(O)
    g = 8
    J, dp, gd = O.projected_norms_gradient(A, A1, B, f, squares, g)
    J0, _ = O.projected_norms(A, B, f, squares, g)
    assert abs(J - J0) <= 1e-12 * J0
    Jp, _ = O.projected_norms(A + h * A1, B, f, squares, g)
    Jm, _ = O.projected_norms(A - h * A1, B, f, squares, g)
    fd = (Jp - Jm) / (2 * h)
    assert abs(dp - fd) <= 1e-6 * abs(fd), (dp, fd)
    scale = np.max(np.abs(gd))
    for i in (0, 7, 33, 59):
        E = np.zeros_like(A)
        E[i, i] = 1.0
        fr = (O.projected_norms(A + h * E, B, f, squares, g)[0] - O.projected_norms(A - h * E, B, f, squares, g)[0]) / (2 * h)
        fi = (O.projected_norms(A + 1j * h * E, B, f, squares, g)[0]
              - O.projected_norms(A - 1j * h * E, B, f, squares, g)[0]) / (2 * h)
        assert abs(gd[i] - (fr + 1j * fi)) <= 1e-6 * scale, (i, gd[i], fr + 1j * fi)


# P18 -- the decision margin: the log-distance of the three threshold tests
# (resolvable: rho_max <= eps0; admissible: ||s_f|| > tau T_f and
# ||s_f|| > delta0 ||s_c||; Definitions 3.1-3.2 with the tau floor) from their
# thresholds.  Constructed inputs put each test nearest in turn, on either side
# of its threshold, with distances known in closed form (ln 2, ln 3, ...); a
# zero or infinite quantity takes its test out.  The margin is then tied to its
# meaning: scaling the compared quantities by less than e^margin toward every
# threshold keeps all three outcomes, scaling the nearest one by more flips it.
MARGIN_PARAMS = dict(delta0=0.05, eps0=1e-8, tau=1e-8)
MARGIN_CASES = [
    # (nsf, nsc, Tf, rho_max, expected margin)
    (1.0, 10.0, 1.0, 1e-10, math.log(2.0)),      # nsf / (delta0 nsc) = 2
    (3e-8, 1e-9, 1.0, 1e-12, math.log(3.0)),     # nsf / (tau Tf) = 3; ratio test at ln 600
    (1.0, 1.0, 1.0, 2.5e-9, math.log(4.0)),      # rho / eps0 = 1/4; ratio test at ln 20
    (1.0, 160.0, 1.0, 1e-14, math.log(8.0)),     # nsf / (delta0 nsc) = 1/8
    (1.0, 0.0, 1.0, 1e-9, math.log(10.0)),       # nsc = 0: ratio test out
    (1.0, 1.0, 0.0, 0.0, math.log(20.0)),        # Tf = 0 and rho = 0: those tests out
    (0.0, 1.0, 1.0, 0.0, math.inf),              # nothing left to compare
]


def _outcomes(nsf, nsc, Tf, rho, p):
    return (rho <= p["eps0"], nsf > p["tau"] * Tf, nsf > p["delta0"] * nsc)


def check_p18_decision_margin(O):
    p = MARGIN_PARAMS
    for nsf, nsc, Tf, rho, want in MARGIN_CASES:
        got = O.decision_margin(nsf, nsc, Tf, rho, p)
        if math.isinf(want):
            assert math.isinf(got), (nsf, nsc, Tf, rho, got)
        else:
            assert abs(got - want) <= 1e-14 * want, (nsf, nsc, Tf, rho, got, want)
        # scale invariance: the three tests compare ratios
        g7 = O.decision_margin(7.0 * nsf, 7.0 * nsc, 7.0 * Tf, rho, p)
        assert (math.isinf(g7) and math.isinf(got)) or abs(g7 - got) <= 1e-14 * got, (g7, got)
    rng = np.random.default_rng(18)
    for _ in range(200):
        nsf, nsc, Tf = 10.0 ** rng.uniform(-12, 2, 3)
        rho = 10.0 ** rng.uniform(-12, -4)
        mg = O.decision_margin(nsf, nsc, Tf, rho, p)
        base = _outcomes(nsf, nsc, Tf, rho, p)
        # every quantity moved toward its threshold by 0.99 margin: no outcome changes
        s = math.exp(0.99 * mg)
        toward = (nsf / s if base[1] else nsf * s, nsc, Tf, rho * s if base[0] else rho / s)
        assert _outcomes(*toward, p)[:2] == base[:2], (nsf, nsc, Tf, rho, mg)
        toward_ratio = (nsf / s if base[2] else nsf * s, nsc, Tf, rho)
        assert _outcomes(*toward_ratio, p)[2] == base[2], (nsf, nsc, Tf, rho, mg)
        # the nearest test moved by 1.01 margin flips
        S = math.exp(1.01 * mg)
        d_rho = abs(math.log(rho / p["eps0"]))
        d_tau = abs(math.log(nsf / (p["tau"] * Tf)))
        d_rat = abs(math.log(nsf / (p["delta0"] * nsc)))
        if d_rho <= min(d_tau, d_rat):
            flipped = _outcomes(nsf, nsc, Tf, rho * S if base[0] else rho / S, p)[0] != base[0]
        elif d_tau <= d_rat:
            flipped = _outcomes(nsf, nsc, Tf * S if base[1] else Tf / S, rho, p)[1] != base[1]
        else:
            flipped = _outcomes(nsf, nsc * S if base[2] else nsc / S, Tf, rho, p)[2] != base[2]
        assert flipped, (nsf, nsc, Tf, rho, mg)


# P19 -- the banded form of the gradient (LAPACK band LU per node, conjugate-transposed
# band solves for the adjoint) against the dense form pinned by P17, on the same
# n = 60 case with A, B and A1 given in band layout.  Both evaluate the same formulas, so
# they agree to rounding: J and dJ/dp to 1e-12 relative, dJ/dA_ii to 1e-12 of the largest.
def _dense_to_band(M, kl, ku):
    n = M.shape[0]
    band = np.zeros((kl + ku + 1, n), dtype=np.complex128, order="F")
    for j in range(n):
        for i in range(max(0, j - ku), min(n, j + kl + 1)):
            band[ku + i - j, j] = M[i, j]
    return band


def check_p19_gradient_banded(O):
    pen, f = random_band_pencil(60, 2, 7, b_kind="tridiag", b_offdiag=0.2)
    A, A1, B, f2, squares = gradient_case(O)
    assert np.array_equal(f, f2)
    # A1 of gradient_case: diagonal plus first superdiagonal
    assert np.count_nonzero(np.tril(A1, -1)) == 0 and np.count_nonzero(np.triu(A1, 2)) == 0
    a1_band = _dense_to_band(A1, 0, 1)
    g = 8
    J, dp, gd = O.projected_norms_gradient(A, A1, B, f, squares, g)
    Jb, dpb, gdb = O.projected_norms_gradient_banded(pen.n, pen.kl_a, pen.ku_a, pen.a_band, pen.kl_b, pen.ku_b,
                                                     pen.b_band, 0, 1, a1_band, f, squares, g)
    assert abs(Jb - J) <= 1e-12 * J, (Jb, J)
    assert abs(dpb - dp) <= 1e-12 * abs(dp), (dpb, dp)
    assert np.max(np.abs(gdb - gd)) <= 1e-12 * np.max(np.abs(gd)), np.max(np.abs(gdb - gd))
