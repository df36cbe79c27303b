"""Plain CPU oracle of SIM-M (Huang, Sun & Yang, "A Multilevel Spectral Indicator
Method for Eigenvalues of Large Non-Hermitian Matrices", arXiv:2006.16117).

TEST INFRASTRUCTURE ONLY.  This module is the independent reference that the
HIP library is checked against.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import it; the library never does.  It shares
no code with the HIP path: it is numpy/scipy in float64/complex128, slow and
literal, and every step follows the paper in the paper's order.

Where the paper is silent or garbled the following readings are taken
(each is listed again in the design notes):

* Contour and rule: R is split into square cells; each square's boundary is
  traversed counter-clockwise and every edge carries a g-point Gauss-Legendre
  rule (the "n0" rule) or a 2g-point rule (the "2n0" rule).  Weights include
  dz/dt.  The two rules are not nested, so 12g systems are solved per square.
* Inner product: (x, y) = y^H x; V^T in the paper means V^H.
* Residual of a shifted Galerkin solve (Sec. 2, eq. (error)):
  rho_j = |sigma - z_j| * h_{m+1,m} * |e_m^T y_j| / beta  (relative to ||b||).
* Resolvable (Definition 3.1): max_j rho_j <= eps0 over all 12g points.
* Admissible (Definition 3.2): the indicator exceeds delta0.  The ratio
  indicator is 0/0 far from any eigenvalue, so a square is marked admissible
  only if ||s_f|| > tau * T_f as well, with T_f = (1/2pi) sum_F |w_j| ||y_j||;
  comparisons are written without division.
* Not resolvable at any level -> marked and flagged (Remark 3.3).
* Level-1 grid: R is pre-divided into N1 x N1 cells (a parameter), shifts
  associated in (iy, ix) order, trying shifts nearest-first (ties: lower
  index); a new shift sits at the cell centre.
* Children inherit their parent's shift; if it does not resolve a square the
  other shifts are tried nearest-first; no new shifts after level 1.
* Number of levels K = levels if given, else 1 + ceil(log2(w1 / h0)).
* Post-processing: 8-connected clusters of the level-K marked squares; the
  eigenvalue is the mean of the member centres (RIM's "centre of R").  As an
  optional extension, the Ritz value sigma + 1/theta of the resolving shift
  that falls in the cluster is reported too.
* Arnoldi: modified Gram-Schmidt applied twice; happy breakdown when
  h_{j+1,j} <= 1e-14 * ||M v_j||.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.linalg as sla
from scipy.linalg import lapack

DENSE_LIMIT = 4000        # dense LU below this order, LAPACK band LU above
BREAKDOWN_TOL = 1e-14

DECISION_REJECTED = 0
DECISION_ADMISSIBLE = 1
DECISION_UNRESOLVED = 2


class SingularShift(RuntimeError):
    """A - sigma B has an exactly zero pivot (sigma is an eigenvalue)."""


# --------------------------------------------------------------------------
# Matrix plumbing (band <-> dense); not part of the method.
# --------------------------------------------------------------------------

def band_to_dense(n: int, kl: int, ku: int, band: np.ndarray | None) -> np.ndarray:
    if band is None:
        return np.eye(n, dtype=np.complex128)
    out = np.zeros((n, n), dtype=np.complex128)
    for j in range(n):
        for i in range(max(0, j - ku), min(n, j + kl + 1)):
            out[i, j] = band[ku + i - j, j]
    return out


def pencil_dense(pencil) -> tuple[np.ndarray, np.ndarray]:
    A = band_to_dense(pencil.n, pencil.kl_a, pencil.ku_a, pencil.a_band)
    B = band_to_dense(pencil.n, pencil.kl_b, pencil.ku_b, pencil.b_band)
    return A, B


def band_matvec(n: int, kl: int, ku: int, band: np.ndarray | None, x: np.ndarray) -> np.ndarray:
    """y = M x for a band matrix, diagonal by diagonal."""
    if band is None:
        return x.copy()
    y = np.zeros(n, dtype=np.complex128)
    for off in range(-kl, ku + 1):          # off = j - i
        if off >= 0:
            i = np.arange(0, n - off)
        else:
            i = np.arange(-off, n)
        j = i + off
        y[i] += band[ku - off, j] * x[j]
    return y


# --------------------------------------------------------------------------
# Cayley transform: factor A - sigma B once, apply M = (A - sigma B)^{-1} B
# (Sec. 2, derivation of eq. (IMxb)).
# --------------------------------------------------------------------------

class ShiftedSolver:
    """Solves (A - sigma B) x = r with one LU of the shifted pencil."""

    def __init__(self, pencil, sigma: complex):
        self.pencil = pencil
        self.sigma = complex(sigma)
        n = pencil.n
        if n <= DENSE_LIMIT:
            A, B = pencil_dense(pencil)
            C = A - self.sigma * B
            lu, piv = sla.lu_factor(C, check_finite=True)
            if np.any(np.diag(lu) == 0):
                raise SingularShift(f"exact zero pivot at sigma={sigma}")
            self._dense = (lu, piv)
            self._band = None
        else:
            kl = max(pencil.kl_a, pencil.kl_b)
            ku = max(pencil.ku_a, pencil.ku_b)
            ab = np.zeros((2 * kl + ku + 1, n), dtype=np.complex128, order="F")
            # rows kl .. 2kl+ku hold C in LAPACK band layout (ku + i - j -> kl + ku + i - j)
            ab[kl + ku - pencil.ku_a: kl + ku + pencil.kl_a + 1, :] += pencil.a_band
            if pencil.b_band is None:
                ab[kl + ku, :] -= self.sigma
            else:
                ab[kl + ku - pencil.ku_b: kl + ku + pencil.kl_b + 1, :] -= self.sigma * pencil.b_band
            lu, ipiv, info = lapack.zgbtrf(ab, kl, ku, overwrite_ab=1)
            if info > 0:
                raise SingularShift(f"exact zero pivot at sigma={sigma} (column {info})")
            if info < 0:
                raise ValueError(f"zgbtrf argument {-info}")
            self._band = (lu, ipiv, kl, ku)
            self._dense = None

    def solve(self, r: np.ndarray) -> np.ndarray:
        if self._dense is not None:
            return sla.lu_solve(self._dense, r)
        lu, ipiv, kl, ku = self._band
        x, info = lapack.zgbtrs(lu, kl, ku, r, ipiv)
        if info != 0:
            raise ValueError(f"zgbtrs info {info}")
        return x

    def apply_B(self, x: np.ndarray) -> np.ndarray:
        p = self.pencil
        return band_matvec(p.n, p.kl_b, p.ku_b, p.b_band, x)

    def apply_M(self, x: np.ndarray) -> np.ndarray:
        """M x = (A - sigma B)^{-1} B x."""
        return self.solve(self.apply_B(x))


@dataclasses.dataclass
class Shift:
    sigma: complex
    beta: float
    H: np.ndarray            # (m_eff + 1) x m_eff upper Hessenberg
    m_eff: int
    V: np.ndarray | None     # n x (m_eff + 1) orthonormal basis (optional)

    @property
    def Hm(self) -> np.ndarray:
        return self.H[: self.m_eff, : self.m_eff]

    @property
    def h_last(self) -> float:
        return float(abs(self.H[self.m_eff, self.m_eff - 1]))


def build_shift(pencil, sigma: complex, f: np.ndarray, m: int, keep_V: bool = True,
                solver: ShiftedSolver | None = None) -> Shift:
    """Arnoldi on M = (A - sigma B)^{-1} B with b = (A - sigma B)^{-1} f
    (Sec. 2, the Arnoldi listing and eq. (arnoldi)); MGS applied twice."""
    n = pencil.n
    if not (1 <= m <= n):
        raise ValueError("need 1 <= m <= n")
    if solver is None:
        solver = ShiftedSolver(pencil, sigma)
    b = solver.solve(np.asarray(f, dtype=np.complex128))
    beta = float(np.linalg.norm(b))
    V = np.zeros((n, m + 1), dtype=np.complex128)
    H = np.zeros((m + 1, m), dtype=np.complex128)
    V[:, 0] = b / beta
    m_eff = m
    for j in range(m):
        w = solver.apply_M(V[:, j])
        w_norm0 = np.linalg.norm(w)
        for _sweep in range(2):
            for i in range(j + 1):
                c = np.vdot(V[:, i], w)          # (w, v_i) = v_i^H w
                H[i, j] += c
                w = w - c * V[:, i]
        hn = np.linalg.norm(w)
        if hn <= BREAKDOWN_TOL * w_norm0:
            H[j + 1, j] = 0.0
            m_eff = j + 1
            break
        H[j + 1, j] = hn
        V[:, j + 1] = w / hn
    H = H[: m_eff + 1, : m_eff].copy()
    V = V[:, : m_eff + 1].copy() if keep_V else None
    return Shift(complex(sigma), beta, H, m_eff, V)


# --------------------------------------------------------------------------
# Squares and quadrature (eq. (XLXf) on the boundary of a square).
# --------------------------------------------------------------------------

def level1_width(params: dict) -> float:
    return (params["x1"] - params["x0"]) / params["n1"]


def level1_grid(params: dict) -> tuple[int, int]:
    """Cells per side at level 1: N1 along x, and the matching count along y."""
    w1 = level1_width(params)
    ny_f = (params["y1"] - params["y0"]) / w1
    ny = int(round(ny_f))
    if ny < 1 or abs(ny * w1 - (params["y1"] - params["y0"])) > 1e-12 * abs(params["y1"] - params["y0"]):
        raise ValueError("level-1 cells must be square: (y1-y0)/((x1-x0)/n1) must be an integer")
    return params["n1"], ny


def square_width(params: dict, level: int) -> float:
    return math.ldexp(level1_width(params), 1 - level)


def square_center(params: dict, level: int, ix: int, iy: int) -> complex:
    w = square_width(params, level)
    return complex(params["x0"] + (ix + 0.5) * w, params["y0"] + (iy + 0.5) * w)


def edge_rule(center: complex, width: float, g: int) -> tuple[np.ndarray, np.ndarray]:
    """Gauss-Legendre nodes/weights on the 4 edges of a square, counter-clockwise.

    Edge a -> b: z = a + (t+1)(b-a)/2, weight w = omega (b-a)/2."""
    t, om = np.polynomial.legendre.leggauss(g)
    h = width / 2.0
    corners = [center + h * (-1 - 1j), center + h * (1 - 1j),
               center + h * (1 + 1j), center + h * (-1 + 1j)]
    zs, ws = [], []
    for e in range(4):
        a, b = corners[e], corners[(e + 1) % 4]
        zs.append(a + (t + 1.0) * (b - a) / 2.0)
        ws.append(om * (b - a) / 2.0)
    return np.concatenate(zs), np.concatenate(ws)


# --------------------------------------------------------------------------
# Indicator of one square with one shift (Sec. 2 eqs. (many), (error), (y);
# Sec. 3.1 eq. (DeltaSm), Definitions 3.1-3.2).
# --------------------------------------------------------------------------

@dataclasses.dataclass
class Evaluation:
    s_c: np.ndarray
    s_f: np.ndarray
    nsc: float
    nsf: float
    Tf: float
    rho_max: float
    resolvable: bool
    admissible: bool
    indicator: float
    margin: float


def shifted_solutions(shift: Shift, z: np.ndarray) -> np.ndarray:
    """y_j = beta (I + (sigma - z_j) H_m)^{-1} e_1 for every z_j (rows of result)."""
    m = shift.m_eff
    Hm = shift.Hm
    alpha = shift.sigma - z
    G = np.eye(m, dtype=np.complex128)[None, :, :] + alpha[:, None, None] * Hm[None, :, :]
    rhs = np.zeros((len(z), m, 1), dtype=np.complex128)
    rhs[:, 0, 0] = shift.beta
    return np.linalg.solve(G, rhs)[:, :, 0]


def residuals(shift: Shift, z: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """rho_j = |sigma - z_j| h_{m+1,m} |e_m^T y_j| / beta."""
    return np.abs(shift.sigma - z) * shift.h_last * np.abs(Y[:, -1]) / shift.beta


def evaluate_square(shift: Shift, center: complex, width: float, params: dict) -> Evaluation:
    g = params["gauss_per_edge"]
    zc, wc = edge_rule(center, width, g)
    zf, wf = edge_rule(center, width, 2 * g)
    Yc = shifted_solutions(shift, zc)
    Yf = shifted_solutions(shift, zf)
    rho = np.concatenate([residuals(shift, zc, Yc), residuals(shift, zf, Yf)])
    rho_max = float(np.max(rho))
    s_c = (wc[:, None] * Yc).sum(axis=0) / (2j * np.pi)
    s_f = (wf[:, None] * Yf).sum(axis=0) / (2j * np.pi)
    Tf = float((np.abs(wf) * np.linalg.norm(Yf, axis=1)).sum() / (2 * np.pi))
    nsc = float(np.linalg.norm(s_c))
    nsf = float(np.linalg.norm(s_f))
    eps0, delta0, tau = params["eps0"], params["delta0"], params["tau"]
    resolvable = rho_max <= eps0
    admissible = (nsf > tau * Tf) and (nsf > delta0 * nsc)
    indicator = nsf / nsc if nsc > 0 else (math.inf if nsf > 0 else math.nan)
    margin = decision_margin(nsf, nsc, Tf, rho_max, params)
    return Evaluation(s_c, s_f, nsc, nsf, Tf, rho_max, resolvable, admissible, indicator, margin)


def decision_margin(nsf, nsc, Tf, rho_max, params) -> float:
    """Smallest |log| distance of the three threshold tests from their thresholds."""
    def lg(a, b):
        if a > 0 and b > 0 and math.isfinite(a) and math.isfinite(b):
            return abs(math.log(a / b))
        return math.inf
    return min(lg(nsf, params["delta0"] * nsc), lg(rho_max, params["eps0"]), lg(nsf, params["tau"] * Tf))


# --------------------------------------------------------------------------
# The multilevel driver (Sec. 3.3 and the SIM-M algorithm of Sec. 3.5).
# --------------------------------------------------------------------------

def num_levels(params: dict) -> int:
    if params.get("levels", 0) > 0:
        return int(params["levels"])
    w1 = level1_width(params)
    return 1 + max(0, math.ceil(math.log2(w1 / params["h0"])))


def _shift_order(shifts: list[Shift], center: complex, exclude: int | None = None) -> list[int]:
    idx = [s for s in range(len(shifts)) if s != exclude]
    return sorted(idx, key=lambda s: (abs(shifts[s].sigma - center), s))


@dataclasses.dataclass
class LevelRecord:
    level: int
    keys: np.ndarray          # (N, 2) int64: ix, iy
    shift: np.ndarray         # shift index used
    indicator: np.ndarray
    rho_max: np.ndarray
    nsf: np.ndarray
    nsc: np.ndarray
    Tf: np.ndarray
    decision: np.ndarray      # uint8
    margin: np.ndarray


@dataclasses.dataclass
class Cluster:
    lam: complex              # mean of member centres
    lam_ritz: complex         # Ritz value of the shift inside the cluster (nan if none)
    shift: int
    unresolved: bool
    members: list


@dataclasses.dataclass
class SimmResult:
    shifts: list
    levels: list
    clusters: list
    K: int


def simm(pencil, f: np.ndarray, params: dict, keep_V: bool = False,
         max_regions_per_level: int = 1 << 22) -> SimmResult:
    """SIM-M(A, B, R, f, h0, eps0, delta0, m, n0) of Sec. 3.5, steps 1-7."""
    validate(pencil, f, params)
    m = params["m"]
    shifts: list[Shift] = []

    def new_shift(sigma):
        shifts.append(build_shift(pencil, sigma, f, m, keep_V=keep_V))
        return len(shifts) - 1

    # Step 1: first shift at the centre of R.
    cR = complex((params["x0"] + params["x1"]) / 2, (params["y0"] + params["y1"]) / 2)
    new_shift(cR)

    # Step 2: level-1 cells, in (iy, ix) order.
    nx, ny = level1_grid(params)
    w1 = square_width(params, 1)
    keys = [(ix, iy) for iy in range(ny) for ix in range(nx)]

    # Step 3: associate each cell with an existing shift or create one.
    assoc = {}
    for (ix, iy) in keys:
        c = square_center(params, 1, ix, iy)
        chosen = None
        for s in _shift_order(shifts, c):
            if evaluate_square(shifts[s], c, w1, params).resolvable:
                chosen = s
                break
        if chosen is None:
            chosen = new_shift(c)
        assoc[(ix, iy)] = chosen

    # Step 4: number of levels.
    K = num_levels(params)

    # Step 5: level loop.
    current = [(ix, iy, assoc[(ix, iy)]) for (ix, iy) in keys]
    levels: list[LevelRecord] = []
    for k in range(1, K + 1):
        if len(current) > max_regions_per_level:
            raise RuntimeError(f"level {k}: {len(current)} squares exceed the limit")
        wk = square_width(params, k)
        rec = {n: [] for n in ("keys", "shift", "indicator", "rho_max", "nsf", "nsc", "Tf", "decision", "margin")}
        children = []
        for (ix, iy, s_inh) in current:
            c = square_center(params, k, ix, iy)
            s_used = s_inh
            ev = evaluate_square(shifts[s_inh], c, wk, params)
            if not ev.resolvable:
                for s in _shift_order(shifts, c, exclude=s_inh):
                    ev2 = evaluate_square(shifts[s], c, wk, params)
                    if ev2.resolvable:
                        s_used, ev = s, ev2
                        break
            if not ev.resolvable:
                decision = DECISION_UNRESOLVED
            elif ev.admissible:
                decision = DECISION_ADMISSIBLE
            else:
                decision = DECISION_REJECTED
            rec["keys"].append((ix, iy))
            rec["shift"].append(s_used)
            rec["indicator"].append(ev.indicator)
            rec["rho_max"].append(ev.rho_max)
            rec["nsf"].append(ev.nsf)
            rec["nsc"].append(ev.nsc)
            rec["Tf"].append(ev.Tf)
            rec["decision"].append(decision)
            rec["margin"].append(ev.margin)
            if decision != DECISION_REJECTED and k < K:
                for b in (0, 1):
                    for a in (0, 1):
                        children.append((2 * ix + a, 2 * iy + b, s_used))
        levels.append(LevelRecord(
            level=k,
            keys=np.array(rec["keys"], dtype=np.int64).reshape(-1, 2),
            shift=np.array(rec["shift"], dtype=np.int64),
            indicator=np.array(rec["indicator"], dtype=np.float64),
            rho_max=np.array(rec["rho_max"], dtype=np.float64),
            nsf=np.array(rec["nsf"], dtype=np.float64),
            nsc=np.array(rec["nsc"], dtype=np.float64),
            Tf=np.array(rec["Tf"], dtype=np.float64),
            decision=np.array(rec["decision"], dtype=np.uint8),
            margin=np.array(rec["margin"], dtype=np.float64)))
        children.sort(key=lambda t: (t[1], t[0]))
        current = children

    # Steps 6-7: merge the marked level-K squares into eigenvalue clusters.
    clusters = postprocess(levels[-1], shifts, params, K)
    return SimmResult(shifts, levels, clusters, K)


def ritz_values(shift: Shift) -> np.ndarray:
    """Eigenvalues of the pencil approximated by H_m: H y = theta y  =>
    lambda = sigma + 1/theta (M x = theta x  <=>  A x = (sigma + 1/theta) B x)."""
    theta = np.linalg.eigvals(shift.Hm)
    with np.errstate(divide="ignore"):
        return shift.sigma + 1.0 / theta


def postprocess(last: LevelRecord, shifts: list[Shift], params: dict, K: int) -> list[Cluster]:
    marked = [i for i in range(len(last.decision)) if last.decision[i] != DECISION_REJECTED]
    pos = {tuple(last.keys[i]): i for i in marked}
    seen = set()
    clusters = []
    wK = square_width(params, K)
    for i in marked:           # marked is in (iy, ix) order already
        key = tuple(last.keys[i])
        if key in seen:
            continue
        comp = []
        stack = [key]
        seen.add(key)
        while stack:
            cur = stack.pop()
            comp.append(pos[cur])
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    nb = (cur[0] + dx, cur[1] + dy)
                    if nb in pos and nb not in seen:
                        seen.add(nb)
                        stack.append(nb)
        comp.sort(key=lambda r: (last.keys[r][1], last.keys[r][0]))
        centres = [square_center(params, K, int(last.keys[r][0]), int(last.keys[r][1])) for r in comp]
        lam = complex(np.mean(np.array(centres)))
        s = int(last.shift[comp[0]])
        unresolved = bool(any(last.decision[r] == DECISION_UNRESOLVED for r in comp))
        xs = [c.real for c in centres]
        ys = [c.imag for c in centres]
        lo = complex(min(xs) - wK, min(ys) - wK)
        hi = complex(max(xs) + wK, max(ys) + wK)
        rv = ritz_values(shifts[s])
        inside = [r for r in rv if np.isfinite(r) and lo.real <= r.real <= hi.real and lo.imag <= r.imag <= hi.imag]
        lam_ritz = complex(min(inside, key=lambda r: abs(r - lam))) if inside else complex(np.nan, np.nan)
        clusters.append(Cluster(lam, lam_ritz, s, unresolved,
                                [(int(last.keys[r][0]), int(last.keys[r][1])) for r in comp]))
    return clusters


def validate(pencil, f, params) -> None:
    n = pencil.n
    f = np.asarray(f)
    if f.shape != (n,):
        raise ValueError("f must have length n")
    if not np.all(np.isfinite(f)):
        raise ValueError("f has NaN/Inf")
    if not np.all(np.isfinite(pencil.a_band)) or (pencil.b_band is not None and not np.all(np.isfinite(pencil.b_band))):
        raise ValueError("pencil has NaN/Inf")
    m = params["m"]
    if m < 1 or m > n:
        raise ValueError("need 1 <= m <= n")
    if params["gauss_per_edge"] < 1:
        raise ValueError("gauss_per_edge >= 1")
    if not (params["x1"] > params["x0"] and params["y1"] > params["y0"]):
        raise ValueError("empty region")
    level1_grid(params)
    if params.get("levels", 0) <= 0 and not params["h0"] > 0:
        raise ValueError("h0 > 0 or levels > 0 required")


# --------------------------------------------------------------------------
# Multiplicities (Sec. 3.4).
# --------------------------------------------------------------------------
# Reading: the spectral projection of f_i onto a cluster's eigenvalue is the
# fine-rule contour sum over the cluster's level-K squares, each square taken with
# the Krylov space K_m(M, b_i) of the shift that square was tested with at level K
# (the paper's "resolved by sigma"); interior edges of adjacent squares cancel.  A
# singular value of [P f_1 .. P f_k] is significant when it exceeds MULT_REL_TOL
# times the largest one.
MULT_REL_TOL = 1e-6


def cluster_projections(pencil, result: SimmResult, F: np.ndarray, params: dict) -> list[np.ndarray]:
    """[P f_1 .. P f_k] (n x k) for every cluster of `result`, in cluster order."""
    F = np.asarray(F, dtype=np.complex128)
    n, k = F.shape
    K = result.K
    last = result.levels[-1]
    wK = square_width(params, K)
    shift_of = {(int(last.keys[r][0]), int(last.keys[r][1])): int(last.shift[r]) for r in range(len(last.keys))}
    X = [np.zeros((n, k), dtype=np.complex128) for _ in result.clusters]
    used = sorted({shift_of[key] for c in result.clusters for key in c.members})
    for s in used:
        sigma = result.shifts[s].sigma
        solver = ShiftedSolver(pencil, sigma)
        for i in range(k):
            sh = build_shift(pencil, sigma, F[:, i], params["m"], keep_V=True, solver=solver)
            for ci, c in enumerate(result.clusters):
                y = np.zeros(sh.m_eff, dtype=np.complex128)
                hit = False
                for key in c.members:
                    if shift_of[key] == s:
                        y += evaluate_square(sh, square_center(params, K, *key), wK, params).s_f
                        hit = True
                if hit:
                    X[ci][:, i] += sh.V[:, : sh.m_eff] @ y
    return X


def multiplicities(X_list: list[np.ndarray], rel_tol: float = MULT_REL_TOL) -> list[tuple[int, np.ndarray]]:
    """(multiplicity, singular values in descending order) of each cluster."""
    out = []
    for X in X_list:
        sv = np.linalg.svd(X, compute_uv=False)
        mult = int(np.sum(sv > rel_tol * sv[0])) if sv[0] > 0 else 0
        out.append((mult, sv))
    return out


# --------------------------------------------------------------------------
# Direct (non-Krylov) quadrature of the spectral projection, eq. (XLXf) with
# the systems of eq. (linearsys) solved by dense LU.  Used by the pins.
# --------------------------------------------------------------------------

def direct_projection(A: np.ndarray, B: np.ndarray, f: np.ndarray, center: complex,
                      width: float, g: int) -> np.ndarray:
    """(1/2 pi i) sum_j w_j x_j with (A - z_j B) x_j = f on the g-per-edge rule."""
    z, w = edge_rule(center, width, g)
    acc = np.zeros(A.shape[0], dtype=np.complex128)
    for zj, wj in zip(z, w):
        acc += wj * np.linalg.solve(A - zj * B, f)
    return acc / (2j * np.pi)


def riesz_apply(A: np.ndarray, B: np.ndarray, g_vec: np.ndarray, center: complex,
                width: float, g: int) -> np.ndarray:
    """Q g = -(1/2 pi i) sum_j w_j (A - z_j B)^{-1} B g: the quadrature of the
    Riesz projector of the pencil, which is idempotent (Q Q = Q) in exact
    arithmetic; for B = I it equals -P of eq. (P)."""
    z, w = edge_rule(center, width, g)
    Bg = B @ g_vec
    acc = np.zeros(A.shape[0], dtype=np.complex128)
    for zj, wj in zip(z, w):
        acc += wj * np.linalg.solve(A - zj * B, Bg)
    return -acc / (2j * np.pi)


# --------------------------------------------------------------------------
# Differentiation of the projected-vector norms (adjoint method).
#   J(A) = sum_R ||x_R||^2,   x_R = (1/2 pi i) sum_{j in F(R)} w_j (A - z_j B)^{-1} f,
# the fine-rule quadrature of eq. (XLXf) over fixed squares R.  With
# u_j = (A - z_j B)^{-1} f, lam_j = (A - z_j B)^{-H} x_R and c_j = w_j / (2 pi i),
# differentiating (A - z_j B)^{-1} gives dJ = -2 Re sum_R sum_j c_j lam_j^H dA u_j, so
#   dJ/dp for A = A0 + p A1:           -2 Re sum_R sum_j c_j lam_j^H A1 u_j,
#   dJ/dRe(A_ii) + i dJ/dIm(A_ii):     -2 conj(t_i),  t_i = sum_R sum_j c_j conj(lam_j,i) u_j,i.
# Dense direct solves; used to check the library's Krylov-space gradient.
# --------------------------------------------------------------------------

def projected_norms(A: np.ndarray, B: np.ndarray, f: np.ndarray, squares, g: int) -> tuple[float, list]:
    """J and the vectors x_R for squares given as (centre, width); fine rule of 2g per edge."""
    xs = [direct_projection(A, B, f, c, w, 2 * g) for c, w in squares]
    return float(sum(np.vdot(x, x).real for x in xs)), xs


def projected_norms_gradient(A: np.ndarray, A1: np.ndarray, B: np.ndarray, f: np.ndarray, squares,
                             g: int) -> tuple[float, float, np.ndarray]:
    """(J, dJ/dp, dJ/dRe(diag A) + i dJ/dIm(diag A)) by the adjoint method."""
    n = A.shape[0]
    J = 0.0
    dp = 0.0
    t = np.zeros(n, dtype=np.complex128)
    for c, w in squares:
        z, wq = edge_rule(c, w, 2 * g)
        cj = wq / (2j * np.pi)
        U = [np.linalg.solve(A - zj * B, f) for zj in z]
        x = sum(ck * u for ck, u in zip(cj, U))
        J += float(np.vdot(x, x).real)
        for zj, ck, u in zip(z, cj, U):
            lam = np.linalg.solve((A - zj * B).conj().T, x)
            dp += -2.0 * (ck * np.vdot(lam, A1 @ u)).real
            t += ck * lam.conj() * u
    return J, dp, -2.0 * t.conj()


def _band_factor(n: int, kl: int, ku: int, a_band: np.ndarray, klb: int, kub: int,
                 b_band: np.ndarray | None, z: complex):
    """LAPACK band LU (zgbtrf) of A - z B, both given in band layout."""
    klc, kuc = max(kl, klb), max(ku, kub)
    ab = np.zeros((2 * klc + kuc + 1, n), dtype=np.complex128, order="F")
    ab[klc + kuc - ku: klc + kuc + kl + 1, :] += a_band
    if b_band is None:
        ab[klc + kuc, :] -= z
    else:
        ab[klc + kuc - kub: klc + kuc + klb + 1, :] -= z * b_band
    lu, ipiv, info = lapack.zgbtrf(ab, klc, kuc, overwrite_ab=1)
    if info > 0:
        raise SingularShift(f"exact zero pivot at z={z} (column {info})")
    if info < 0:
        raise ValueError(f"zgbtrf argument {-info}")
    return lu, ipiv, klc, kuc


def _band_solve(fac, r: np.ndarray, adjoint: bool = False) -> np.ndarray:
    """x with (A - z B) x = r, or with (A - z B)^H x = r when ``adjoint``."""
    lu, ipiv, kl, ku = fac
    x, info = lapack.zgbtrs(lu, kl, ku, r, ipiv, trans=2 if adjoint else 0)
    if info != 0:
        raise ValueError(f"zgbtrs info {info}")
    return x


def projected_norms_gradient_banded(n: int, kl: int, ku: int, a_band: np.ndarray, klb: int, kub: int,
                                    b_band: np.ndarray | None, kl1: int, ku1: int, a1_band: np.ndarray,
                                    f: np.ndarray, squares, g: int) -> tuple[float, float, np.ndarray]:
    """projected_norms_gradient for band matrices (orders where dense ones do not
    fit): the same quantities by the same formulas, with each A - z_j B factored by
    LAPACK's band LU and its systems, and the conjugate-transposed ones, solved with
    that factor.  A1 is a band matrix of half-bandwidths (kl1, ku1).  The factor of a
    node is formed twice (once for u_j, once for lam_j, which needs x_R first)."""
    J = 0.0
    dp = 0.0
    t = np.zeros(n, dtype=np.complex128)
    for c, w in squares:
        z, wq = edge_rule(c, w, 2 * g)
        cj = wq / (2j * np.pi)
        U = [_band_solve(_band_factor(n, kl, ku, a_band, klb, kub, b_band, zj), f) for zj in z]
        x = sum(ck * u for ck, u in zip(cj, U))
        J += float(np.vdot(x, x).real)
        for zj, ck, u in zip(z, cj, U):
            lam = _band_solve(_band_factor(n, kl, ku, a_band, klb, kub, b_band, zj), x, adjoint=True)
            dp += -2.0 * (ck * np.vdot(lam, band_matvec(n, kl1, ku1, a1_band, u))).real
            t += ck * lam.conj() * u
    return J, dp, -2.0 * t.conj()
