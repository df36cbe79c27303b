"""Eigenvalues of a banded pencil near a region, from ARPACK (implicitly restarted
Arnoldi) on the shift-inverted operator (A - s B)^{-1} B with SuperLU's sparse LU.

An independent reference for the eigenvalue locations and counts that SIM-M reports
(Sec. 3.4 counts eigenvalues per cluster; Sec. 4 compares locations with a direct
solver).  It is test infrastructure: it shares no code with the oracle or the HIP
path, only the seeded pencil arrays of `workloads`.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def band_to_csc(n: int, kl: int, ku: int, band: np.ndarray) -> sp.csc_matrix:
    """LAPACK general-band storage (entry (i, j) at band[ku + i - j, j]) to CSC."""
    diags, offs = [], []
    for d in range(-kl, ku + 1):          # diagonal d holds the entries (i, i + d)
        v = band[ku - d, d:] if d >= 0 else band[ku - d, :n + d]
        if np.any(v != 0):
            diags.append(np.asarray(v, dtype=np.complex128))
            offs.append(d)
    return sp.diags(diags, offs, shape=(n, n), format="csc")


def pencil_csc(pen):
    A = band_to_csc(pen.n, pen.kl_a, pen.ku_a, pen.a_band)
    if pen.b_band is None:
        B = sp.identity(pen.n, dtype=np.complex128, format="csc")
    else:
        B = band_to_csc(pen.n, pen.kl_b, pen.ku_b, pen.b_band)
    return A, B


def nearest_eigenvalues(A, B, s: complex, k: int):
    """The k eigenvalues of A x = lam B x nearest s, and the radius within which the
    list is complete (every eigenvalue closer to s than it is in the list)."""
    n = A.shape[0]
    lu = spla.splu((A - s * B).tocsc(), permc_spec="COLAMD")
    op = spla.LinearOperator((n, n), matvec=lambda v: lu.solve(B @ v), dtype=np.complex128)
    # a seeded start vector: the same iterations in every process and call order
    rng = np.random.default_rng(12345)
    v0 = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    theta = spla.eigs(op, k=k, which="LM", return_eigenvectors=False, tol=1e-12, v0=v0)
    lam = s + 1.0 / theta
    return lam, float(np.max(np.abs(lam - s)))


def eigenvalues_in_region(pen, x0, x1, y0, y1, nx=4, ny=2, k=40):
    """The eigenvalues in the closed rectangle [x0, x1] x [y0, y1], from shift-invert
    ARPACK at an nx x ny grid of centres.  Raises AssertionError unless the discs in
    which each centre's list would be complete cover the rectangle (checked on a grid
    of points at a spacing far below the disc margins).  ARPACK can still leave out an
    eigenvalue inside a disc (seen once on a batch pencil of order 13,163), so the
    result is a subset that is complete in practice, not by proof."""
    A, B = pencil_csc(pen)
    hx, hy = (x1 - x0) / nx, (y1 - y0) / ny
    centres = [complex(x0 + (i + 0.5) * hx, y0 + (j + 0.5) * hy) for i in range(nx) for j in range(ny)]
    found, discs = [], []
    for c in centres:
        lam, r = nearest_eigenvalues(A, B, c, k)
        found.extend(lam.tolist())
        discs.append((c, r))
    gx, gy = np.meshgrid(np.linspace(x0, x1, 129), np.linspace(y0, y1, 65))
    pts = (gx + 1j * gy).ravel()
    covered = np.zeros(pts.shape, bool)
    for c, r in discs:
        covered |= np.abs(pts - c) < 0.98 * r
    assert covered.all(), "the complete discs do not cover the region: raise k or the grid of centres"
    uniq: list[complex] = []
    for lam in found:
        if not any(abs(lam - u) <= 1e-8 * max(1.0, abs(lam)) for u in uniq):
            uniq.append(lam)
    u = np.array(uniq)
    inside = (u.real >= x0) & (u.real <= x1) & (u.imag >= y0) & (u.imag <= y1)
    return u[inside]


def dist_to_square(lam: complex, x0: float, y0: float, w: float, ix: int, iy: int) -> float:
    """Distance from lam to the closed square [x0 + ix w, x0 + (ix+1) w] x [y0 + iy w, ...]."""
    ax, ay = x0 + ix * w, y0 + iy * w
    dx = max(ax - lam.real, 0.0, lam.real - (ax + w))
    dy = max(ay - lam.imag, 0.0, lam.imag - (ay + w))
    return float(np.hypot(dx, dy))


def counts_per_cluster(eigs, clusters_members, x0, y0, w):
    """For each cluster (a list of (ix, iy) squares of width w), the number of the given
    eigenvalues inside its squares; and for each eigenvalue the number of clusters
    holding it."""
    per_cluster = [sum(1 for lam in eigs if min(dist_to_square(lam, x0, y0, w, ix, iy) for ix, iy in mem) == 0.0)
                   for mem in clusters_members]
    per_eig = [sum(1 for mem in clusters_members
                   if min(dist_to_square(lam, x0, y0, w, ix, iy) for ix, iy in mem) == 0.0) for lam in eigs]
    return per_cluster, per_eig
