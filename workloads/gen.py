"""Seeded synthetic pencils (A, B) and start vectors f for the SIM-M workloads.

This module only draws random numbers and lays them out in LAPACK general-band
storage.  It holds none of the method's arithmetic (no shifts, factorizations,
Krylov spaces or quadrature); both the CPU oracle and the HIP path consume the
arrays it returns.

Band layout (the same convention as LAPACK ``?gbtrf`` input, without the extra
``kl`` fill rows): ``band[ku + i - j, j] = A[i, j]`` for
``max(0, j-ku) <= i <= min(n-1, j+kl)``, shape ``(kl+ku+1, n)``, complex128,
stored column-major so that one column of A is contiguous (``order='F'``).

Random stream: numpy PCG64 seeded per workload; the draw order is fixed:
diagonal ``d``, then ``E`` by diagonal offset ``-k .. k``, then ``B``, then ``f``.
A complex normal is ``(N + iN)/sqrt(2)``.
"""
from __future__ import annotations

import dataclasses
import json
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))


@dataclasses.dataclass
class Pencil:
    """A banded pencil (A, B) of order n; ``b_band is None`` means B = I."""
    n: int
    kl_a: int
    ku_a: int
    a_band: np.ndarray
    kl_b: int
    ku_b: int
    b_band: np.ndarray | None

    def band_entry(self, which: str, i: int, j: int) -> complex:
        """Entry (i, j) of A or B read from band storage (0 outside the band)."""
        if which == "a":
            kl, ku, band = self.kl_a, self.ku_a, self.a_band
        else:
            if self.b_band is None:
                return 1.0 + 0j if i == j else 0j
            kl, ku, band = self.kl_b, self.ku_b, self.b_band
        if j - ku <= i <= j + kl:
            return complex(band[ku + i - j, j])
        return 0j


def complex_normal(rng: np.random.Generator, size) -> np.ndarray:
    return (rng.standard_normal(size) + 1j * rng.standard_normal(size)) / np.sqrt(2.0)


def _empty_band(n: int, kl: int, ku: int) -> np.ndarray:
    return np.zeros((kl + ku + 1, n), dtype=np.complex128, order="F")


def _set_diag(band: np.ndarray, ku: int, off: int, vals: np.ndarray) -> None:
    """Write diagonal ``off`` (j - i = off) of a band matrix: A[i, i+off] = vals."""
    n = band.shape[1]
    if off >= 0:
        cols = np.arange(off, n)
    else:
        cols = np.arange(0, n + off)
    rows = cols - off
    band[ku + rows - cols, cols] = vals


def random_band_pencil(n: int, k: int, seed: int, *, b_kind: str = "identity",
                       b_offdiag: float = 0.1, e_scale: float = 0.05,
                       d_half: float = 2.0) -> tuple[Pencil, np.ndarray]:
    """The "config-0 generator": A = diag(d) + E, B = I or a random tridiagonal.

    d_i ~ U[-d_half, d_half] + i U[-d_half, d_half]; E has half-bandwidth k (its
    diagonal included) with entries ``e_scale`` times a complex normal.
    ``b_kind='tridiag'`` gives B with unit diagonal and independent real
    off-diagonals ``b_offdiag * U(-1, 1)``.  Returns (pencil, f).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    d = rng.uniform(-d_half, d_half, n) + 1j * rng.uniform(-d_half, d_half, n)
    a = _empty_band(n, k, k)
    _set_diag(a, k, 0, d)
    for off in range(-k, k + 1):
        m = n - abs(off)
        vals = e_scale * complex_normal(rng, m)
        rows = np.arange(max(0, -off), max(0, -off) + m)
        cols = rows + off
        a[k + rows - cols, cols] += vals
    if b_kind == "identity":
        b, kl_b, ku_b = None, 0, 0
    elif b_kind == "tridiag":
        kl_b = ku_b = 1
        b = _empty_band(n, 1, 1)
        _set_diag(b, 1, 0, np.ones(n))
        _set_diag(b, 1, -1, b_offdiag * rng.uniform(-1.0, 1.0, n - 1))
        _set_diag(b, 1, 1, b_offdiag * rng.uniform(-1.0, 1.0, n - 1))
    else:
        raise ValueError(b_kind)
    f = complex_normal(rng, n)
    return Pencil(n, k, k, a, kl_b, ku_b, b), f


def convection_diffusion_pencil(nx: int, seed: int, *, conv=(20.0, 10.0),
                                react=0.5 + 0.5j, b_off: float = 0.05) -> tuple[Pencil, np.ndarray]:
    """5-point finite differences of -Lap u + conv . grad u + react u on the unit
    square, nx x nx interior nodes, h = 1/(nx+1), Dirichlet boundary, natural
    x-fastest ordering (node (ix, iy) -> ix + nx*iy).  Convection uses central
    differences.  B = tridiag(b_off, 1, b_off) over the whole vector.
    Half-bandwidth of A is nx.  f is a seeded complex normal vector.
    """
    n = nx * nx
    h = 1.0 / (nx + 1)
    k = nx
    a = _empty_band(n, k, k)
    ix = np.arange(n) % nx
    diag = np.full(n, 4.0 / h**2 + react, dtype=np.complex128)
    _set_diag(a, k, 0, diag)
    east = np.full(n - 1, -1.0 / h**2 + conv[0] / (2 * h), dtype=np.complex128)
    west = np.full(n - 1, -1.0 / h**2 - conv[0] / (2 * h), dtype=np.complex128)
    # no coupling across a grid row end: row i with ix = nx-1 has no east neighbour
    east[ix[:-1] == nx - 1] = 0.0
    west[ix[1:] == 0] = 0.0
    _set_diag(a, k, 1, east)
    _set_diag(a, k, -1, west)
    north = np.full(n - nx, -1.0 / h**2 + conv[1] / (2 * h), dtype=np.complex128)
    south = np.full(n - nx, -1.0 / h**2 - conv[1] / (2 * h), dtype=np.complex128)
    _set_diag(a, k, nx, north)
    _set_diag(a, k, -nx, south)
    b = _empty_band(n, 1, 1)
    _set_diag(b, 1, 0, np.ones(n))
    _set_diag(b, 1, 1, np.full(n - 1, b_off))
    _set_diag(b, 1, -1, np.full(n - 1, b_off))
    rng = np.random.Generator(np.random.PCG64(seed))
    f = complex_normal(rng, n)
    return Pencil(n, k, k, a, 1, 1, b), f


def planted_pencil(n: int, seed: int, planted, *, box: float = 0.3, d_half: float = 2.0,
                   b_offdiag: float = 0.1, kb: int = 2) -> tuple[Pencil, np.ndarray]:
    """A pencil with known eigenvalues and multiplicities: (A, B) = (J B, B).

    J = diag(d) + N: ``planted`` lists (value, count, jordan) triples; each planted
    value fills ``count`` diagonal entries, at consecutive indices, and with
    ``jordan`` true the entries are chained by ones on the superdiagonal of N (one
    Jordan block of that size); the other entries of d are uniform on
    [-d_half, d_half]^2 outside the box |Re|, |Im| < box.  B has unit diagonal and
    ``kb`` off-diagonals each side drawn as ``b_offdiag`` times a complex normal.
    Since J B x = lambda B x  <=>  J y = lambda y with y = B x, the eigenvalues of
    the pencil are those of J with the same Jordan structure.  A is banded with
    kl = kb, ku = kb + 1.  Draw order: the positions of the planted groups, the
    other d entries, B by diagonal offset -kb .. kb, then f.  Returns (pencil, f)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    d = np.zeros(n, dtype=np.complex128)
    sup = np.zeros(n - 1, dtype=np.complex128)          # superdiagonal of N
    taken = np.zeros(n, dtype=bool)
    slots = n // max(1, len(planted))
    for g, (val, count, jordan) in enumerate(planted):
        start = g * slots + int(rng.integers(0, max(1, slots - count)))
        idx = np.arange(start, start + count)
        assert not taken[idx].any() and idx[-1] < n
        taken[idx] = True
        d[idx] = complex(val)
        if jordan:
            sup[idx[:-1]] = 1.0
    free = np.nonzero(~taken)[0]
    vals = []
    while len(vals) < len(free):
        z = rng.uniform(-d_half, d_half) + 1j * rng.uniform(-d_half, d_half)
        if abs(z.real) >= box or abs(z.imag) >= box:
            vals.append(z)
    d[free] = np.array(vals)
    b = _empty_band(n, kb, kb)
    _set_diag(b, kb, 0, np.ones(n))
    for off in range(-kb, kb + 1):
        if off != 0:
            _set_diag(b, kb, off, b_offdiag * complex_normal(rng, n - abs(off)))
    # A = J B: row i of A is d_i (row i of B) + sup_i (row i+1 of B)
    kl_a, ku_a = kb, kb + 1
    a = _empty_band(n, kl_a, ku_a)
    for off in range(-kb, kb + 1):
        rows = np.arange(max(0, -off), min(n, n - off))
        cols = rows + off
        a[ku_a + rows - cols, cols] += d[rows] * b[kb + rows - cols, cols]
    for off in range(-kb, kb + 1):          # entries of row i+1 of B land on row i, offset off + 1
        rows = np.arange(max(0, -off), min(n, n - off))     # rows of B
        rows = rows[rows >= 1]
        cols = rows + off
        a[ku_a + (rows - 1) - cols, cols] += sup[rows - 1] * b[kb + rows - cols, cols]
    f = complex_normal(rng, n)
    return Pencil(n, kl_a, ku_a, a, kb, kb, b), f


def start_vectors(n: int, k: int, seed: int) -> np.ndarray:
    """k further seeded start vectors (n x k complex normal, column-major) for the
    multiplicity step, drawn from PCG64(seed + 500000) so f is unchanged."""
    rng = np.random.Generator(np.random.PCG64(seed + 500000))
    return np.asfortranarray(complex_normal(rng, (k, n)).T)


# --------------------------------------------------------------------------
# Workload parameter sets (region, quadrature size, Krylov dimension, levels).
# --------------------------------------------------------------------------

def load_config(name: str) -> dict:
    with open(os.path.join(_HERE, "configs", name + ".json")) as fh:
        return json.load(fh)


def make_workload(name: str) -> tuple[Pencil, np.ndarray, dict]:
    """Build (pencil, f, params) for a named workload file under configs/."""
    cfg = load_config(name)
    gen = cfg["generator"]
    if gen["kind"] == "random_band":
        pencil, f = random_band_pencil(gen["n"], gen["k"], gen["seed"],
                                       b_kind=gen.get("b_kind", "identity"),
                                       b_offdiag=gen.get("b_offdiag", 0.1))
    elif gen["kind"] == "convection_diffusion":
        pencil, f = convection_diffusion_pencil(gen["nx"], gen["seed"])
    elif gen["kind"] == "planted":
        planted = [(complex(*v), int(c), bool(j)) for v, c, j in gen["planted"]]
        pencil, f = planted_pencil(gen["n"], gen["seed"], planted, box=gen.get("box", 0.3))
    else:
        raise ValueError(gen["kind"])
    return pencil, f, dict(cfg["params"])


def make_batch(name: str) -> list[tuple[Pencil, np.ndarray, dict]]:
    """Build the (pencil, f, params) list of a batch workload file under configs/.

    Pencil p (p = 0 .. count-1): order n_p and target eigenvalue count c_p drawn
    from PCG64(seed0 + 100000 + p) as n_p ~ U{n_min .. n_max}, c_p ~ U[c_min, c_max];
    the pencil itself is ``random_band_pencil(n_p, k, seed0 + p)`` (B = I).  Its
    region is the square centred at 0 with side 4 sqrt(c_p / n_p): the diagonal
    entries are uniform on [-2, 2]^2 (density n_p / 16), so about c_p eigenvalues
    fall inside."""
    cfg = load_config(name)
    gen = cfg["generator"]
    assert gen["kind"] == "random_band_batch"
    out = []
    for p in range(gen["count"]):
        rng = np.random.default_rng(gen["seed0"] + 100000 + p)
        n = int(rng.integers(gen["n_min"], gen["n_max"] + 1))
        c = float(rng.uniform(gen["c_min"], gen["c_max"]))
        pencil, f = random_band_pencil(n, gen["k"], gen["seed0"] + p, b_kind="identity")
        half = 2.0 * float(np.sqrt(c / n))
        params = dict(cfg["params"])
        params.update(x0=-half, x1=half, y0=-half, y1=half)
        out.append((pencil, f, params))
    return out



def random_band_matrix(n: int, k: int, seed: int, scale: float) -> np.ndarray:
    """Band (2k+1, n), LAPACK layout, of a matrix with half-bandwidth k whose
    in-band entries are iid real N(0, 1) times ``scale`` (the perturbation
    direction A1 of the differentiation workload)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    a = _empty_band(n, k, k)
    for off in range(-k, k + 1):
        m = n - abs(off)
        rows = np.arange(max(0, -off), max(0, -off) + m)
        cols = rows + off
        a[k + rows - cols, cols] = scale * rng.standard_normal(m)
    return a
