"""HIP path against the CPU oracle, through the C ABI (needs an MI355X).

Each test prints the case it runs before touching the GPU."""
import json
import os
import sys

import numpy as np
import pytest

import oracle.simm as O
from workloads import make_workload
from workloads.gen import Pencil as WPencil
from workloads.gen import random_band_pencil

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def S():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_2006_16117_amd.simm as S   # raises if the library is not built
    return S


def hmax_diff(Hg, Ho):
    return np.max(np.abs(Hg - Ho)) / np.max(np.abs(Ho))


# ---------------------------------------------------------------------------
# shift build: LU + Arnoldi + Schur
# ---------------------------------------------------------------------------
CASES = [
    # name, n, k, seed, b_kind, m, sigma, extra kwargs of the generator
    ("cfg0-like", 400, 2, 1000, "identity", 40, 0.1 + 0.2j, {}),
    ("tridiagB", 300, 3, 77, "tridiag", 30, -0.3 + 0.1j, {}),
    ("pivoting", 257, 5, 78, "tridiag", 25, 0.05 - 0.02j, dict(d_half=0.05, e_scale=1.0)),
    ("ragged-wide", 1037, 21, 79, "identity", 33, 0.2 + 0.0j, {}),
    ("m=n", 24, 2, 80, "identity", 24, 0.0 + 0.1j, {}),
    ("tiny", 5, 1, 81, "tridiag", 3, 0.3 + 0.3j, {}),
    # band LU workgroup sizes: window 2*16 + kl rows; 64 threads up to kl = 32, 128 up to 96,
    # 256 up to 224, 512 up to 480
    ("band60-pivoting", 700, 60, 86, "tridiag", 20, 0.05 + 0.05j, dict(d_half=0.05, e_scale=1.0)),
    ("band224", 900, 224, 83, "tridiag", 20, 0.1 + 0.1j, {}),
    ("band200-pivoting", 800, 200, 87, "tridiag", 20, 0.05 - 0.05j, dict(d_half=0.05, e_scale=1.0)),
    ("band240-pivoting", 1300, 240, 84, "identity", 20, -0.2 + 0.05j, dict(d_half=0.05, e_scale=1.0)),
    ("band480-pivoting", 1100, 480, 85, "identity", 16, 0.05 + 0.0j, dict(d_half=0.05, e_scale=1.0)),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_shift_build_matches_oracle(S, case):
    name, n, k, seed, b_kind, m, sigma, kw = case
    pen, f = random_band_pencil(n, k, seed, b_kind=b_kind, b_offdiag=0.3, **kw)
    say("shift_build", name, f"n={n} k={k} m={m}")
    P = S.Pencil.from_workload(pen)
    sh = S.simm_shift_build(P, sigma, f, m)
    g = sh.info()
    o = O.build_shift(pen, sigma, f, m)
    assert g["m_eff"] == o.m_eff
    assert abs(g["beta"] - o.beta) <= 1e-12 * o.beta
    d = hmax_diff(g["H"], o.H)
    say("  max |H_gpu - H_oracle| / max|H| =", d)
    assert d <= 1e-9
    V = sh.basis()
    me = g["m_eff"]
    ncol = me + 1 if g["H"][me, me - 1] != 0 else me     # v_{m+1} is undefined after a breakdown
    orth = float(np.linalg.norm(V[:, :ncol].conj().T @ V[:, :ncol] - np.eye(ncol)))
    assert orth <= 1e-12, orth
    # Ritz values (diagonal of the Schur form) against the oracle's eigenvalues of H_m
    ro = O.ritz_values(o)
    for r in g["ritz"]:
        assert np.min(np.abs(ro - r)) <= 1e-8 * max(1.0, abs(r))


# ---------------------------------------------------------------------------
# partitioned factorization: diagonal blocks factored side by side, spikes, reduced system
# ---------------------------------------------------------------------------
PART_CASES = [
    # name, n, kl, ku, seed, b_kind, m, sigma, block length asked for, generator kwargs
    ("k3", 3000, 3, 3, 90, "tridiag", 30, 0.1 + 0.05j, 256, {}),
    ("k16-pivoting", 5000, 16, 16, 91, "identity", 30, 0.05 + 0.0j, 512, dict(d_half=0.05, e_scale=1.0)),
    ("k32-ragged", 4100, 32, 32, 92, "tridiag", 30, -0.1 + 0.1j, 1024, {}),
    ("kl8-ku3", 3000, 8, 3, 93, "identity", 25, 0.2j, 384, {}),
    ("k64", 9000, 64, 64, 94, "tridiag", 30, 0.1j, 1024, {}),
    ("k150", 8000, 150, 150, 95, "identity", 20, 0.05 + 0.05j, 1600, {}),
]


def _narrow_upper(pen, ku):
    """The pencil with A's upper bandwidth cut to ku (diagonals above removed)."""
    band = np.asfortranarray(pen.a_band[pen.ku_a - ku:, :])
    return WPencil(pen.n, pen.kl_a, ku, band, pen.kl_b, pen.ku_b, pen.b_band)


@pytest.fixture
def part_env():
    old = os.environ.get("SIMM_LU_PART")
    yield os.environ
    if old is None:
        os.environ.pop("SIMM_LU_PART", None)
    else:
        os.environ["SIMM_LU_PART"] = old


@pytest.mark.parametrize("case", PART_CASES, ids=[c[0] for c in PART_CASES])
def test_partitioned_factor_matches_oracle(S, part_env, case):
    name, n, kl, ku, seed, b_kind, m, sigma, bs, kw = case
    pen, f = random_band_pencil(n, kl, seed, b_kind=b_kind, b_offdiag=0.3, **kw)
    if ku != kl:
        pen = _narrow_upper(pen, ku)
    part_env["SIMM_LU_PART"] = str(bs)
    say("partitioned factor", name, f"n={n} kl={kl} ku={ku} block={bs} m={m}")
    P = S.Pencil.from_workload(pen)
    sh = S.simm_shift_build(P, sigma, f, m)
    fi = sh.factor_info()
    say("  factor:", fi)
    assert fi["block_len"] >= bs and fi["block_len"] % 16 == 0 and not fi["fallback"]
    assert 0.0 <= fi["eta"] <= 1e-13
    g = sh.info()
    o = O.build_shift(pen, sigma, f, m)
    assert g["m_eff"] == o.m_eff
    assert abs(g["beta"] - o.beta) <= 1e-12 * o.beta
    d = hmax_diff(g["H"], o.H)
    say("  max |H_gpu - H_oracle| / max|H| =", d)
    assert d <= 1e-9
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    y = np.zeros(n, np.complex128)
    sh.apply(x, y)
    want = O.ShiftedSolver(pen, sigma).apply_M(x)
    err = np.linalg.norm(y - want) / np.linalg.norm(want)
    say("  apply rel. error", err)
    assert err <= 1e-12


MANY_CASES = [
    # name, n, kl, seed, b_kind, block length (0: the whole band), k columns, generator kwargs
    ("whole-k8", 3000, 8, 120, "tridiag", 0, 5, {}),                 # four-column passes, then one
    # strong pivoting: U's bandwidth above 256, so two columns, then one
    ("whole-k140", 3000, 140, 121, "identity", 0, 3, dict(d_half=0.05, e_scale=1.0)),
    ("part-k16", 5000, 16, 122, "tridiag", 512, 7, {}),              # partitioned: 4 + 2 + 1
]


@pytest.mark.parametrize("case", MANY_CASES, ids=[c[0] for c in MANY_CASES])
def test_apply_many_equals_single_applications(S, part_env, case):
    """simm_shift_apply_many (several columns per pass over the factor: the multi-column
    chunk sweeps, chains, fix-ups and corrections, and for a partitioned factor the
    multi-column tips product and correction) gives every column bit for bit what
    simm_shift_apply gives it, and that agrees with the oracle's solve."""
    name, n, kl, seed, b_kind, bs, k, kw = case
    pen, f = random_band_pencil(n, kl, seed, b_kind=b_kind, b_offdiag=0.3, **kw)
    part_env["SIMM_LU_PART"] = str(bs)
    say("apply_many", name, f"n={n} kl=ku={kl} block={bs} k={k}")
    P = S.Pencil.from_workload(pen)
    sigma = 0.05 + 0.03j
    sh = S.simm_shift_build(P, sigma, f, 4)
    fi = sh.factor_info()
    assert (fi["block_len"] > 0) == (bs > 0)
    if bs == 0:
        # U's bandwidth: ku plus the longest pivot jump (LAPACK's band LU, the same pivots)
        _, ipiv, _, _ = O._band_factor(n, pen.kl_a, pen.ku_a, pen.a_band, pen.kl_b, pen.ku_b, pen.b_band, sigma)
        K = pen.ku_a + int(np.max(ipiv - 1 - np.arange(n)))
        say("  U bandwidth", K)
        assert (K > 256) == (kl > 100)
    rng = np.random.default_rng(seed)
    X = np.asfortranarray(rng.standard_normal((n, k)) + 1j * rng.standard_normal((n, k)))
    Y = np.zeros((n, k), np.complex128, order="F")
    sh.apply_many(X, Y)
    solver = O.ShiftedSolver(pen, sigma)
    for r in range(k):
        y = np.zeros(n, np.complex128)
        sh.apply(np.ascontiguousarray(X[:, r]), y)
        assert np.array_equal(Y[:, r], y), (r, float(np.max(np.abs(Y[:, r] - y))))
        want = solver.apply_M(X[:, r])
        assert np.linalg.norm(y - want) <= 1e-12 * np.linalg.norm(want)


def test_partitioned_mixed_precision_refines(S, part_env):
    pen, f = random_band_pencil(5000, 16, 96, b_kind="tridiag", b_offdiag=0.3)
    sigma = -0.05 + 0.1j
    part_env["SIMM_LU_PART"] = "512"
    say("partitioned factor, FP32 blocks with refinement", "n=5000 kl=ku=16 block=512 m=30")
    P = S.Pencil.from_workload(pen)
    sh = S.simm_shift_build(P, sigma, f, 30, precision=S.SIMM_PREC_MIXED)
    assert sh.factor_info()["block_len"] == 512
    st = sh.refine_stats()
    say("  refinement:", st)
    assert st["solves"] >= 31 and st["max_eta"] <= 1e-12
    g = sh.info()
    o = O.build_shift(pen, sigma, f, 30)
    d = hmax_diff(g["H"], o.H)
    say("  max |H_gpu - H_oracle| / max|H| =", d)
    assert abs(g["beta"] - o.beta) <= 1e-11 * o.beta and d <= 1e-9


@pytest.mark.parametrize("pivot", [0.0, 1e-14], ids=["singular-block", "near-singular-block"])
def test_partitioned_factor_falls_back(S, part_env, pivot):
    """A diagonal block that is singular (or nearly) while A - sigma B is not: the
    library factors the whole matrix instead, and the shift still matches the oracle."""
    n, k, q = 2000, 2, 512
    pen, f = random_band_pencil(n, k, 97, b_kind="identity")
    band = pen.a_band.copy(order="F")
    band[k + 0, q] = pivot          # A(q, q)
    band[k + 1, q] = 0.0            # A(q + 1, q)
    band[k + 2, q] = 0.0            # A(q + 2, q): the block's first column is (pivot, 0, ...)
    pen = WPencil(n, k, k, band, pen.kl_b, pen.ku_b, pen.b_band)
    A, _ = O.pencil_dense(pen)
    assert np.linalg.cond(A) < 1e10
    part_env["SIMM_LU_PART"] = "256"
    say("partitioned factor fallback", f"A(q,q) = {pivot}, block 256")
    P = S.Pencil.from_workload(pen)
    sh = S.simm_shift_build(P, 0.0, f, 20)
    fi = sh.factor_info()
    say("  factor:", fi)
    assert fi["fallback"] and fi["block_len"] == 0
    g = sh.info()
    o = O.build_shift(pen, 0.0, f, 20)
    d = hmax_diff(g["H"], o.H)
    say("  max |H_gpu - H_oracle| / max|H| =", d)
    assert abs(g["beta"] - o.beta) <= 1e-12 * o.beta and d <= 1e-9


def test_pivoting_really_pivots_and_apply_matches(S):
    pen, f = random_band_pencil(257, 5, 78, b_kind="tridiag", b_offdiag=0.3, d_half=0.05, e_scale=1.0)
    sigma = 0.05 - 0.02j
    solver = O.ShiftedSolver(pen, sigma)
    A, B = O.pencil_dense(pen)
    import scipy.linalg as sla
    _, piv = sla.lu_factor(A - sigma * B)
    assert np.count_nonzero(piv != np.arange(pen.n)) > 10      # the pencil needs row interchanges
    say("apply", "pivoting pencil")
    P = S.Pencil.from_workload(pen)
    sh = S.simm_shift_build(P, sigma, f, 10)
    rng = np.random.default_rng(5)
    x = rng.standard_normal(pen.n) + 1j * rng.standard_normal(pen.n)
    y = np.zeros(pen.n, np.complex128)
    sh.apply(x, y)
    want = solver.apply_M(x)
    assert np.linalg.norm(y - want) <= 1e-12 * np.linalg.norm(want)


@pytest.mark.parametrize("n,k,chunk,groups", [
    (5013, 3, 256, [1, 2, 3, 4, 7, 10]),        # P = 20: groups of 2..20 chunks, uneven last groups
    (3000, 150, 320, [1, 2, 3, 5]),             # P = 10, wide band: state of ~150 / ~300 rows
])
def test_apply_two_level_chain_matches_oracle(S, n, k, chunk, groups):
    """One application of M = (A - sigma B)^{-1} B through the partitioned sweeps, with the
    chain over the chunk boundaries run in one level or in groups (chains per group, the
    chain over the groups' start states, the fix-up by the transfer products), against the
    oracle's banded solve."""
    pen, f = random_band_pencil(n, k, 86, b_kind="tridiag", b_offdiag=0.3, d_half=0.05, e_scale=1.0)
    sigma = 0.03 - 0.01j
    solver = O.ShiftedSolver(pen, sigma)
    rng = np.random.default_rng(6)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    want = solver.apply_M(x)
    P = S.Pencil.from_workload(pen)
    saved = {v: os.environ.get(v) for v in ("SIMM_SPIKE_CHUNK", "SIMM_SPIKE_GROUPS")}
    try:
        for g in groups:
            os.environ["SIMM_SPIKE_CHUNK"] = str(chunk)
            os.environ["SIMM_SPIKE_GROUPS"] = str(g)
            say("apply", f"n={n} k={k} chunk={chunk} groups={g}")
            sh = S.simm_shift_build(P, sigma, f, 4)
            y = np.zeros(n, np.complex128)
            sh.apply(x, y)
            err = np.linalg.norm(y - want) / np.linalg.norm(want)
            assert err <= 1e-11, (g, err)
            del sh
    finally:
        for v, old in saved.items():
            if old is None:
                os.environ.pop(v, None)
            else:
                os.environ[v] = old


def test_shift_build_is_deterministic(S):
    pen, f = random_band_pencil(700, 4, 82, b_kind="tridiag")
    say("determinism", "n=700")
    P = S.Pencil.from_workload(pen)
    H1 = S.simm_shift_build(P, 0.1j, f, 20).info()["H"]
    H2 = S.simm_shift_build(P, 0.1j, f, 20).info()["H"]
    assert np.array_equal(H1, H2)


def test_breakdown_and_errors(S):
    n = 8
    band = (np.arange(n) + 1.0).reshape(1, n).astype(complex)
    pen = WPencil(n, 0, 0, band, 0, 0, None)
    f = np.zeros(n, complex)
    f[3] = 1.0
    say("breakdown", "diagonal pencil, f = e_3")
    P = S.Pencil.from_workload(pen)
    sh = S.simm_shift_build(P, 0.5j, f, 5)
    inf = sh.info()
    assert inf["m_eff"] == 1 and inf["H"].shape == (2, 1) and inf["H"][1, 0] == 0
    say("singular shift")
    with pytest.raises(S.SimmError) as e:
        S.simm_shift_build(P, 3.0, f, 3)
    assert e.value.status == -5
    with pytest.raises(S.SimmError) as e:
        S.simm_shift_build(P, 0.5, f, 0)
    assert e.value.status == -1
    bad = f.copy()
    bad[0] = np.nan
    with pytest.raises(S.SimmError) as e:
        S.simm_shift_build(P, 0.5, bad, 3)
    assert e.value.status == -1


def test_singular_cell_shift_same_error_with_lookahead(S):
    """A level-1 cell whose centre is an eigenvalue: its shift has an exact zero pivot.
    The factor computed ahead for that cell fails on a side stream; the run must
    report the same error as building one shift at a time (and as the oracle)."""
    rng = np.random.default_rng(11)
    n = 60
    d = rng.uniform(-2, 2, n) + 1j * rng.uniform(-2, 2, n)
    d[7] = 0.5 - 0.5j                       # centre of level-1 cell (1, 0) of R = [-1,1]^2, n1 = 2
    pen = WPencil(n, 0, 0, d.reshape(1, n).astype(complex), 0, 0, None)
    f = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    params = dict(x0=-1.0, x1=1.0, y0=-1.0, y1=1.0, n1=2, gauss_per_edge=8, m=3, h0=1e-2, levels=0,
                  eps0=1e-8, delta0=0.05, tau=1e-8)
    with pytest.raises(O.SingularShift):
        O.simm(pen, f, params)
    P = S.Pencil.from_workload(pen)
    for la in (1, 3):
        say("singular cell shift, lookahead", la)
        with pytest.raises(S.SimmError) as e:
            S.simm_run(P, f, S.params_from_dict(params, lookahead=la))
        assert e.value.status == -5, (la, e.value)


# ---------------------------------------------------------------------------
# indicators and projection
# ---------------------------------------------------------------------------
def test_indicators_match_oracle(S):
    pen, f, params = make_workload("cfg0")
    sigma = 0.125 + 0.375j
    say("indicators", "cfg0 pencil, one shift, 200 squares at levels 1..6")
    P = S.Pencil.from_workload(pen)
    sh = S.simm_shift_build(P, sigma, f, params["m"])
    o = O.build_shift(pen, sigma, f, params["m"], keep_V=False)
    rng = np.random.default_rng(3)
    regs = []
    for _ in range(200):
        k = int(rng.integers(1, 7))
        nk = 8 * 2 ** (k - 1)
        regs.append((k, int(rng.integers(0, nk)), int(rng.integers(0, nk)), 0))
    regs = np.array(regs, np.int64)
    prm = S.params_from_dict(params)
    out = S.simm_indicators([sh], regs, prm, want_sums=True)
    mism = 0
    for r, (k, ix, iy, _) in enumerate(regs):
        c = O.square_center(params, int(k), int(ix), int(iy))
        w = O.square_width(params, int(k))
        ev = O.evaluate_square(o, c, w, params)
        dec = 2 if not ev.resolvable else (1 if ev.admissible else 0)
        for name, a, b in (("nsf", out["nsf"][r], ev.nsf), ("nsc", out["nsc"][r], ev.nsc), ("Tf", out["Tf"][r], ev.Tf)):
            assert abs(a - b) <= 1e-7 * max(abs(b), 1e-30) + 1e-14 * ev.Tf, (r, name, a, b)
        assert abs(out["rho_max"][r] - ev.rho_max) <= 1e-6 * ev.rho_max + 1e-16, (r, out["rho_max"][r], ev.rho_max)
        if out["decision"][r] != dec:
            mism += 1
            assert ev.margin < 1e-8, (r, out["decision"][r], dec, ev.margin)
        # the sums themselves: s_c, s_f (coefficients of P_R f in the Krylov basis)
        sc = out["sums"][r, 0, : o.m_eff]
        sf = out["sums"][r, 1, : o.m_eff]
        # relative 1e-7, or round-off level (1e-13 T_f) for sums that are pure quadrature noise
        dc = float(np.linalg.norm(sc - ev.s_c))
        df = float(np.linalg.norm(sf - ev.s_f))
        assert dc <= max(1e-7 * np.linalg.norm(ev.s_c), 1e-13 * ev.Tf), (r, dc)
        assert df <= max(1e-7 * np.linalg.norm(ev.s_f), 1e-13 * ev.Tf), (r, df)
    say("  decision ties:", mism)


def _oracle_eval_with_scales(o, center, width, params):
    """The oracle's evaluation of one square, the magnitude sums T_c, T_f of its two
    rules ((1/2 pi) sum_j |w_j| ||y_j||: a sum whose terms each carry a relative error
    e is off by at most e times this), and the rounding level of its residual: rho_j
    takes |e_m^T y_j|, whose rounding error is about m u ||y_j|| whatever its size, so
    rho_max is compared down to m u max_j |sigma - z_j| h_{m+1,m} ||y_j|| / beta."""
    ev = O.evaluate_square(o, center, width, params)
    u = np.finfo(np.float64).eps / 2
    g = params["gauss_per_edge"]
    floor = 0.0
    T = []
    for rule in (g, 2 * g):
        z, w = O.edge_rule(center, width, rule)
        Y = O.shifted_solutions(o, z)
        ny = np.linalg.norm(Y, axis=1)
        T.append(float(np.sum(np.abs(w) * ny) / (2 * np.pi)))
        floor = max(floor, float(np.max(np.abs(o.sigma - z) * o.h_last * ny / o.beta)))
    return ev, T[0], T[1], o.m_eff * u * floor


def _solve_error_bound(o, center, width, params):
    """Forward-error bound of a backward-stable solve of every quadrature point's
    system G_j y = beta e_1, G_j = I + (sigma - z_j) H_m, relative to ||y_j||:
    8 m u max_j kappa_1(G_j).  Two such solvers (the oracle's LU, the library's Schur
    form) may differ by this much.  Near an eigenvalue (deep levels, z_j within h0 of
    it) kappa reaches |lambda - sigma| / |z_j - lambda|, about 1e6."""
    u = np.finfo(np.float64).eps / 2
    m = o.m_eff
    kap = 0.0
    for rule in (params["gauss_per_edge"], 2 * params["gauss_per_edge"]):
        z, _ = O.edge_rule(center, width, rule)
        G = np.eye(m)[None] + (o.sigma - z)[:, None, None] * o.Hm[None]
        kap = max(kap, float(np.max(np.linalg.norm(G, 1, axis=(1, 2)) *
                                    np.linalg.norm(np.linalg.inv(G), 1, axis=(1, 2)))))
    return 8 * m * u * kap


def _check_indicators_on_oracle_H(S, name, regs, params, oracle_shifts, rel=1e-12):
    """Every square's sums within rel times its magnitude sums (each point's solution
    to rel), T_f and rho_max within rel relative (rho_max down to its rounding level),
    decisions identical up to ties (oracle margin < 1e-8).  Where a square's systems are
    ill-conditioned the bar is the two solvers' forward-error bound instead, if larger."""
    gpu_shifts = [S.simm_shift_from_hessenberg(o.sigma, o.beta, o.H) for o in oracle_shifts]
    prm = S.params_from_dict(params)
    out = S.simm_indicators(gpu_shifts, regs, prm, want_sums=True)
    ties = 0
    worst = dict(s_c=0.0, s_f=0.0, nsc=0.0, nsf=0.0, Tf=0.0, rho=0.0, nsf_rel=0.0)
    n_cond = 0
    worst_over_bound = 0.0
    bad = []
    for r, (k, ix, iy, si) in enumerate(regs):
        o = oracle_shifts[int(si)]
        c = O.square_center(params, int(k), int(ix), int(iy))
        w = O.square_width(params, int(k))
        ev, Tc, Tf, rho_floor = _oracle_eval_with_scales(o, c, w, params)
        me = o.m_eff
        errs = dict(s_c=float(np.linalg.norm(out["sums"][r, 0, :me] - ev.s_c)) / Tc,
                    s_f=float(np.linalg.norm(out["sums"][r, 1, :me] - ev.s_f)) / Tf,
                    nsc=abs(out["nsc"][r] - ev.nsc) / Tc,
                    nsf=abs(out["nsf"][r] - ev.nsf) / Tf,
                    Tf=abs(out["Tf"][r] - ev.Tf) / ev.Tf,
                    rho=abs(out["rho_max"][r] - ev.rho_max) / max(ev.rho_max, rho_floor / rel, 1e-300))
        for key, v in errs.items():
            worst[key] = max(worst[key], v)
        if max(errs.values()) > rel:
            bound = _solve_error_bound(o, c, w, params)
            n_cond += 1
            worst_over_bound = max(worst_over_bound, max(errs.values()) / bound)
            for key, v in errs.items():
                if not v <= max(rel, bound):
                    bad.append((r, key, v, bound))
        if ev.nsf > 1e-6 * Tf:     # sums well above the quadrature noise: plain relative error
            worst["nsf_rel"] = max(worst["nsf_rel"], abs(out["nsf"][r] - ev.nsf) / ev.nsf)
        dec = 2 if not ev.resolvable else (1 if ev.admissible else 0)
        if out["decision"][r] != dec:
            ties += 1
            if not ev.margin < 1e-8:
                bad.append((r, "decision", (int(out["decision"][r]), dec, ev.margin)))
    say(f"  {name}: {len(regs)} squares, decision ties {ties}; max errors (sums and norms relative to the "
        f"magnitude sums): " + ", ".join(f"{k} {v:.2e}" for k, v in worst.items()) +
        f"; {n_cond} squares above {rel:g}, at most {worst_over_bound:.2e} of their conditioning bound")
    assert not bad, bad[:10]


def _golden_shifts(name):
    d = np.load(os.path.join(GOLDEN, f"{name}_hessenberg.npz"), allow_pickle=False)
    out = []
    for sig, beta, me, H in zip(d["sigma"], d["beta"], d["m_eff"], d["H"]):
        me = int(me)
        out.append(O.Shift(complex(sig), float(beta), H[: me + 1, :me].copy(), me, None))
    return out


def test_indicators_on_oracle_hessenberg_cfg0(S):
    """The indicator kernel alone (a6-a8) on the oracle's own (sigma, beta, H) of every
    shift of the n = 400 run: 200 squares drawn from the squares the oracle tested,
    each with the shift it was tested with."""
    pen, f, params = make_workload("cfg0")
    with open(os.path.join(GOLDEN, "cfg0_oracle.json")) as fh:
        run = json.load(fh)
    rows = [(L["level"], ix, iy, s) for L in run["levels"] for ix, iy, s in zip(L["ix"], L["iy"], L["shift"])]
    rng = np.random.default_rng(200)
    pick = rng.choice(len(rows), size=200, replace=False)
    regs = np.array([rows[i] for i in sorted(pick)], np.int64)
    say("indicators on the oracle's H", "cfg0", f"{len(regs)} squares, levels {regs[:, 0].min()}..{regs[:, 0].max()}")
    _check_indicators_on_oracle_H(S, "cfg0", regs, params, _golden_shifts("cfg0"))


def test_indicators_on_oracle_hessenberg_cfg1(S):
    """The same on the 7 shifts of the n = 40,000 run and every square of its 4 levels."""
    pen, f, params = make_workload("cfg1")
    with open(os.path.join(GOLDEN, "cfg1_oracle.json")) as fh:
        run = json.load(fh)
    regs = np.array([(L["level"], ix, iy, s) for L in run["levels"] for ix, iy, s in zip(L["ix"], L["iy"], L["shift"])],
                    np.int64)
    say("indicators on the oracle's H", "cfg1", f"{len(regs)} squares")
    _check_indicators_on_oracle_H(S, "cfg1", regs, params, _golden_shifts("cfg1"))


def _check_cell_residuals(S, name, params, oracle_shifts, rows, rel=1e-12):
    """simm_cell_residuals (residuals from Hessenberg determinants, no Schur form) on
    the oracle's (sigma, beta, H): every square's rho_max against the oracle's
    evaluation, to rel relative down to the residual's rounding level, or, where the
    square's systems are ill-conditioned, within the two solvers' forward-error bound;
    and the decision rho_max <= eps0 identical unless the oracle's rho_max lies within
    that error of eps0.  rows: (level, ix, iy, shift)."""
    gpu_shifts = [S.simm_shift_from_hessenberg(o.sigma, o.beta, o.H) for o in oracle_shifts]
    prm = S.params_from_dict(params)
    rows = np.asarray(rows, np.int64)
    got = np.zeros(len(rows))
    for lev in np.unique(rows[:, 0]):
        for si in np.unique(rows[:, 3]):
            sel = np.nonzero((rows[:, 0] == lev) & (rows[:, 3] == si))[0]
            if len(sel):
                got[sel] = S.simm_cell_residuals(gpu_shifts[int(si)], int(lev), rows[sel, 1:3], prm)
    worst, worst_bound, flips, bad = 0.0, 0.0, 0, []
    for r, (k, ix, iy, si) in enumerate(rows):
        o = oracle_shifts[int(si)]
        c = O.square_center(params, int(k), int(ix), int(iy))
        w = O.square_width(params, int(k))
        ev, _, _, rho_floor = _oracle_eval_with_scales(o, c, w, params)
        err = abs(got[r] - ev.rho_max) / max(ev.rho_max, rho_floor / rel, 1e-300)
        tol = rel
        if err > rel:
            tol = max(rel, _solve_error_bound(o, c, w, params))
            worst_bound = max(worst_bound, err / tol)
        worst = max(worst, err)
        if not err <= tol:
            bad.append((r, float(got[r]), ev.rho_max, err, tol))
        if (got[r] <= params["eps0"]) != (ev.rho_max <= params["eps0"]):
            flips += 1
            if not abs(ev.rho_max - params["eps0"]) <= tol * max(ev.rho_max, rho_floor / rel):
                bad.append((r, "decision", float(got[r]), ev.rho_max))
    say(f"  {name}: {len(rows)} squares, max rel. error of rho_max {worst:.2e} "
        f"(conditioned squares at most {worst_bound:.2e} of their bound), resolvability flips {flips}")
    assert not bad, bad[:10]


def test_cell_residuals_on_oracle_hessenberg_cfg1(S):
    """The level-1 association's residuals (Hessenberg determinants) on the oracle's H of
    the 7 shifts of the n = 40,000 run: every level-1 cell against every shift (what the
    association tests), and every square of levels 2-4 with the shift it was tested with."""
    pen, f, params = make_workload("cfg1")
    shifts = _golden_shifts("cfg1")
    nx, ny = O.level1_grid(params)
    rows = [(1, ix, iy, s) for s in range(len(shifts)) for iy in range(ny) for ix in range(nx)]
    with open(os.path.join(GOLDEN, "cfg1_oracle.json")) as fh:
        run = json.load(fh)
    rows += [(L["level"], ix, iy, s) for L in run["levels"] if L["level"] > 1
             for ix, iy, s in zip(L["ix"], L["iy"], L["shift"])]
    say("cell residuals on the oracle's H", "cfg1", f"{len(rows)} squares")
    _check_cell_residuals(S, "cfg1", params, shifts, rows)


def test_cell_residuals_on_oracle_hessenberg_cfg0(S):
    """The same on the n = 400 run's shifts: every level-1 cell against every shift."""
    pen, f, params = make_workload("cfg0")
    shifts = _golden_shifts("cfg0")
    nx, ny = O.level1_grid(params)
    rows = [(1, ix, iy, s) for s in range(len(shifts)) for iy in range(ny) for ix in range(nx)]
    say("cell residuals on the oracle's H", "cfg0", f"{len(rows)} squares")
    _check_cell_residuals(S, "cfg0", params, shifts, rows)


def test_cell_residuals_errors(S):
    say("cell_residuals", "argument errors")
    pen, f, params = make_workload("cfg0")
    sh = _golden_shifts("cfg0")[0]
    g = S.simm_shift_from_hessenberg(sh.sigma, sh.beta, sh.H)
    prm = S.params_from_dict(params)
    with pytest.raises(S.SimmError):
        S.simm_cell_residuals(g, 0, np.zeros((1, 2), np.int64), prm)     # level < 1
    assert S.simm_cell_residuals(g, 1, np.zeros((0, 2), np.int64), prm).shape == (0,)


def test_shift_from_hessenberg_errors(S):
    say("shift_from_hessenberg", "argument errors")
    H = np.zeros((4, 3), np.complex128)
    H[0, 0] = H[1, 0] = H[1, 1] = H[2, 1] = H[2, 2] = H[3, 2] = 1.0
    with pytest.raises(S.SimmError) as e:
        S.simm_shift_from_hessenberg(0.0, -1.0, H)          # beta <= 0
    assert e.value.status == -1
    Hb = H.copy()
    Hb[3, 0] = 0.5                                          # below the subdiagonal
    with pytest.raises(S.SimmError) as e:
        S.simm_shift_from_hessenberg(0.0, 1.0, Hb)
    assert e.value.status == -1
    Hn = H.copy()
    Hn[0, 1] = np.nan
    with pytest.raises(S.SimmError) as e:
        S.simm_shift_from_hessenberg(0.0, 1.0, Hn)
    assert e.value.status == -1
    sh = S.simm_shift_from_hessenberg(0.1, 2.0, H)
    inf = sh.info()
    assert inf["m_eff"] == 3 and inf["beta"] == 2.0 and np.array_equal(inf["H"], H)
    y = np.zeros(3, np.complex128)
    with pytest.raises(S.SimmError) as e:                  # no factor behind it
        sh.apply(np.ones(3, np.complex128), y)
    assert e.value.status == -1


# Error bounds of the reduced-precision projections, relative to ||V Y||_F.  Inputs are
# rounded to the format (unit roundoff u: FP32 2^-24, BF16 2^-8) and the 2m real products
# of an entry are accumulated in FP32; with random signs the error of an entry is about
# 2u/sqrt(3) times the root-sum-square of its terms (BF16 ~4.5e-3, FP32 ~7e-8 plus FP32
# accumulation over 2m terms); the bounds leave a factor of about 4.
PROJ_TOL = {0: 1e-13, 1: 1e-5, 2: 2e-2}


@pytest.mark.parametrize("prec", [0, 1, 2], ids=["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("m", [37, 80])
def test_project_matches_numpy(S, m, prec):
    """X = V_m Y on the matrix cores: ragged in every dimension (n = 5013 is 39 row blocks of
    128 and 21 rows; c up to 150 spans three column blocks of 64; m = 37 leaves a partial
    stage of 8 inner indices), in FP64 and with FP32 / BF16 operands (FP32 accumulation)."""
    import torch
    pen, f = random_band_pencil(5000 + 13, 3, 90, b_kind="tridiag")
    say("project", f"n=5013 m={m} c=1..150 precision={prec}")
    P = S.Pencil.from_workload(pen)
    sh = S.simm_shift_build(P, 0.2 + 0.1j, f, m)
    V = sh.basis()[:, :m]
    Vo = O.build_shift(pen, 0.2 + 0.1j, f, m).V[:, :m]       # the oracle's Krylov basis
    rng = np.random.default_rng(1)
    tol = PROJ_TOL[prec]
    worst = 0.0
    for c in (1, 7, 45, 64, 150):
        Y = rng.standard_normal((m, c)) + 1j * rng.standard_normal((m, c))
        Yd = torch.from_numpy(np.ascontiguousarray(Y.T)).cuda()          # column-major storage
        Xd = torch.zeros((c, pen.n), dtype=torch.complex128, device="cuda")
        nd = torch.zeros(c, dtype=torch.float64, device="cuda")
        S.simm_project(sh, Yd.T, Xd.T, nd, precision=prec)
        # norms only (X not written)
        nd2 = torch.zeros(c, dtype=torch.float64, device="cuda")
        S.simm_project(sh, Yd.T, None, nd2, precision=prec)
        torch.cuda.synchronize()
        X = Xd.cpu().numpy().T
        # against the oracle's basis (the two Arnoldi processes agree to ~1e-12)
        wo = Vo @ Y
        assert np.linalg.norm(X - wo) <= max(tol, 1e-9) * np.linalg.norm(wo), c
        # the product's own arithmetic, on the library's basis
        want = V @ Y
        rel = np.linalg.norm(X - want) / np.linalg.norm(want)
        worst = max(worst, rel)
        assert rel <= tol, (c, rel)
        # every column on its own (a column block or a row block left out shows here)
        err = np.linalg.norm(X - want, axis=0) / np.linalg.norm(want, axis=0)
        assert err.max() <= 4 * tol, (c, int(err.argmax()), err.max())
        wn = np.linalg.norm(want, axis=0)
        assert np.allclose(nd.cpu().numpy(), wn, rtol=4 * tol, atol=0)
        assert np.array_equal(nd.cpu().numpy(), nd2.cpu().numpy())
    say("  max relative error", worst)


def test_run_mixed_projection_keeps_decisions(S):
    """SIMM_FLAG_MIXED_PROJECT changes only the full-space indicator record: decisions,
    reduced indicators and clusters are those of the FP64 run, and the full-space
    indicator ||V s_f|| / ||V s_c|| equals the reduced one (V orthonormal, Sec. 3.1) to
    FP64 rounding, or to the BF16 (levels 1-2) / FP32 (later levels) error."""
    pen, f, params = make_workload("cfg0")
    P = S.Pencil.from_workload(pen)
    say("simm_run", "cfg0 projected in FP64 and in mixed precision")
    r64 = S.simm_run(P, f, S.params_from_dict(params, flags=S.SIMM_FLAG_PROJECT))
    rmx = S.simm_run(P, f, S.params_from_dict(params, flags=S.SIMM_FLAG_PROJECT | S.SIMM_FLAG_MIXED_PROJECT))
    assert r64.K == rmx.K and np.array_equal(r64.lam, rmx.lam)
    worst = {0: 0.0, 1: 0.0, 2: 0.0}
    for La, Lb in zip(r64.levels, rmx.levels):
        assert np.array_equal(La.keys, Lb.keys) and np.array_equal(La.decision, Lb.decision)
        assert np.array_equal(La.indicator, Lb.indicator, equal_nan=True)
        ok = np.isfinite(La.indicator) & (La.indicator > 0)
        assert np.all(np.isfinite(La.full_indicator[ok]))
        e64 = np.abs(La.full_indicator[ok] - La.indicator[ok]) / La.indicator[ok]
        prec = 2 if La.level <= 2 else 1
        emx = np.abs(Lb.full_indicator[ok] - La.indicator[ok]) / La.indicator[ok]
        if ok.any():
            worst[0] = max(worst[0], e64.max())
            worst[prec] = max(worst[prec], emx.max())
            assert e64.max() <= 1e-10, (La.level, e64.max())
            assert emx.max() <= 2 * PROJ_TOL[prec] + 1e-10, (La.level, emx.max())
    say("  max relative error of the full-space indicator: fp64", worst[0], "fp32", worst[1], "bf16", worst[2])


# ---------------------------------------------------------------------------
# the whole method against the oracle's stored runs
# ---------------------------------------------------------------------------
def _compare_run(S, name, flags=0):
    pen, f, params = make_workload(name)
    gold = json.load(open(os.path.join(GOLDEN, f"{name}_oracle.json")))
    say("simm_run", name)
    P = S.Pencil.from_workload(pen)
    prm = S.params_from_dict(params, flags=flags)
    res = S.simm_run(P, f, prm)
    assert res.K == gold["K"]
    assert res.n_shifts == len(gold["shifts"])
    for s, gs in enumerate(gold["shifts"]):
        inf = res.shift(s).info()
        assert inf["sigma"] == complex(*gs["sigma"])
        assert inf["m_eff"] == gs["m_eff"]
        assert abs(inf["beta"] - gs["beta"]) <= 1e-10 * gs["beta"]
    ties = 0
    for L, GL in zip(res.levels, gold["levels"]):
        gk = list(zip(GL["ix"], GL["iy"]))
        ok = [tuple(map(int, k)) for k in L.keys]
        if ok != gk:
            raise AssertionError(f"level {L.level}: tested squares differ ({len(ok)} vs {len(gk)})")
        gd = np.array(GL["decision"], np.uint8)
        bad = np.nonzero(L.decision != gd)[0]
        for r in bad:
            assert GL["margin"][r] < 1e-8, (L.level, r, L.decision[r], gd[r], GL["margin"][r])
            ties += 1
        assert np.array_equal(L.shift, np.array(GL["shift"]))
    lam = np.array([complex(*c["lam"]) for c in gold["clusters"]])
    lr = np.array([complex(*c["lam_ritz"]) for c in gold["clusters"]])
    say("  levels", res.K, "shifts", res.n_shifts, "clusters", len(res.lam), "ms", res.ms)
    assert len(res.lam) == len(lam)
    # cluster centres are means of identical square centres: equal up to the summation order
    assert np.all(np.abs(res.lam - lam) <= 1e-14 * np.abs(lam))
    fin = np.isfinite(lr)
    assert np.array_equal(np.isfinite(res.lam_ritz), fin)
    assert np.all(np.abs(res.lam_ritz[fin] - lr[fin]) <= 1e-8 * np.maximum(1.0, np.abs(lr[fin])))
    say("  decision ties within the margin policy:", ties)
    return res


def test_run_cfg0_matches_oracle(S):
    _compare_run(S, "cfg0")


def test_run_cfg1_matches_oracle(S):
    res = _compare_run(S, "cfg1", flags=1)
    # full-space indicator of the last level is available (X = V_m Y computed)
    assert res.counters["quadrature_systems"] == 12 * 16 * sum(len(L.keys) for L in res.levels)


def test_lookahead_equals_one_at_a_time(S):
    """Shifts built ahead of the cell order (steps 2-3 of SIM-M) are kept only where the
    one-at-a-time order creates them, so the whole run is the same bit for bit."""
    for name in ("cfg0", "cfg1"):
        pen, f, params = make_workload(name)
        P = S.Pencil.from_workload(pen)
        runs = {}
        for la in (1, 3, 8):
            say("simm_run", name, "lookahead", la)
            runs[la] = S.simm_run(P, f, S.params_from_dict(params, lookahead=la))
        a = runs[1]
        for la in (3, 8):
            b = runs[la]
            assert a.K == b.K and a.n_shifts == b.n_shifts, (name, la)
            for s in range(a.n_shifts):
                ia, ib = a.shift(s).info(), b.shift(s).info()
                assert ia["sigma"] == ib["sigma"] and np.array_equal(ia["H"], ib["H"]), (name, la, s)
            for La, Lb in zip(a.levels, b.levels):
                assert np.array_equal(La.keys, Lb.keys) and np.array_equal(La.shift, Lb.shift)
                assert np.array_equal(La.decision, Lb.decision)
                assert np.array_equal(La.indicator, Lb.indicator, equal_nan=True)
                assert np.array_equal(La.rho_max, Lb.rho_max, equal_nan=True)
            assert np.array_equal(a.lam, b.lam) and np.array_equal(a.counters["quadrature_systems"],
                                                                    b.counters["quadrature_systems"])
            say("  shift builds ms: one at a time", round(a.ms["shift_builds"], 1), f"lookahead {la}",
                round(b.ms["shift_builds"], 1))
    with pytest.raises(S.SimmError):
        S.simm_run(P, f, S.params_from_dict(params, lookahead=17))


# ---------------------------------------------------------------------------
# multiplicities (Sec. 3.4)
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def planted_oracle_run():
    pen, f, params = make_workload("mult0")
    return pen, f, params, O.simm(pen, f, params)


@pytest.mark.parametrize("k", [5, 1, 8])
def test_multiplicities_match_oracle(S, planted_oracle_run, k):
    from workloads import load_config, start_vectors
    name = "mult0"
    pen, f, params, res_o = planted_oracle_run
    cfg = load_config(name)
    F = start_vectors(pen.n, k, cfg["generator"]["seed"])
    say("simm_multiplicities", name, "k =", k)
    want = O.multiplicities(O.cluster_projections(pen, res_o, F, params))
    res = S.simm_run(S.Pencil.from_workload(pen), f, S.params_from_dict(params))
    assert res.n_clusters == len(res_o.clusters)
    mult, sv = S.simm_multiplicities(res, F, rel_tol=O.MULT_REL_TOL)
    say("  multiplicities", np.bincount(mult).tolist(), "(count of clusters per multiplicity)")
    for c, (mo, svo) in enumerate(want):
        assert mult[c] == mo, (c, mult[c], mo, sv[c] / sv[c][0], svo / svo[0])
        # significant singular values agree; the others sit at their rounding levels
        # (the library's come from the Gram matrix, so about 1e-8 of the largest)
        assert np.all(np.abs(sv[c][:mo] - svo[:mo]) <= 1e-8 * svo[0]), (c, sv[c], svo)
        assert np.all(sv[c][mo:] <= O.MULT_REL_TOL * sv[c][0])
    assert sorted(mult.tolist()) == sorted(min(k, e) for e in (1, 1, 2, 2, 3))
    if k == 5:
        # a run that releases its factors gives the same levels and refuses the multiplicity step
        lean = S.simm_run(S.Pencil.from_workload(pen), f,
                          S.params_from_dict(params, flags=S.SIMM_FLAG_RELEASE_FACTORS))
        assert lean.n_clusters == res.n_clusters and np.array_equal(lean.lam, res.lam)
        for La, Lb in zip(lean.levels, res.levels):
            assert np.array_equal(La.decision, Lb.decision) and np.array_equal(La.indicator, Lb.indicator)
        with pytest.raises(S.SimmError) as e:
            S.simm_multiplicities(lean, F)
        assert e.value.status == -1
    with pytest.raises(S.SimmError):
        S.simm_multiplicities(res, F, rel_tol=0.0)


def test_multiplicities_cfg1_match_eigenvalue_counts(S):
    """Sec. 3.4 on the n = 40,000 run: with k start vectors the multiplicity of a cluster
    is min(k, number of eigenvalues it holds).  The counts come from shift-invert ARPACK
    on the host (tests/arpack_ref.py), independent of the oracle and of the HIP path;
    the run's clusters are the oracle's stored ones, in the same order."""
    from tests import arpack_ref
    from workloads import load_config, start_vectors
    name, k = "cfg1", 4
    pen, f, params = make_workload(name)
    with open(os.path.join(GOLDEN, f"{name}_oracle.json")) as fh:
        gold = json.load(fh)
    say("ARPACK eigenvalues of", name, "in R (host)")
    eigs = arpack_ref.eigenvalues_in_region(pen, params["x0"], params["x1"], params["y0"], params["y1"])
    w = (params["x1"] - params["x0"]) / params["n1"] / 2 ** (gold["K"] - 1)
    members = [[tuple(mm) for mm in c["members"]] for c in gold["clusters"]]
    counts, per_eig = arpack_ref.counts_per_cluster(eigs, members, params["x0"], params["y0"], w)
    assert min(per_eig) == 1 and max(per_eig) == 1 and min(counts) >= 1
    say("simm_run + simm_multiplicities", name, "k =", k, "clusters", len(members), "eigenvalues", len(eigs))
    res = S.simm_run(S.Pencil.from_workload(pen), f, S.params_from_dict(params))
    lam = np.array([complex(*c["lam"]) for c in gold["clusters"]])
    assert len(res.lam) == len(lam) and np.all(np.abs(res.lam - lam) <= 1e-14 * np.abs(lam))
    F = start_vectors(pen.n, k, load_config(name)["generator"]["seed"])
    mult, sv = S.simm_multiplicities(res, F)
    want = np.minimum(k, np.array(counts))
    say("  multiplicities", np.bincount(mult).tolist(), "eigenvalue counts", np.bincount(want).tolist())
    bad = np.nonzero(mult != want)[0]
    assert len(bad) == 0, [(int(c), int(mult[c]), int(counts[c]), (sv[c] / sv[c][0]).tolist()) for c in bad]


# ---------------------------------------------------------------------------
# edge cases: empty inputs, empty levels, guards, the CSR entry point
# ---------------------------------------------------------------------------
def test_empty_inputs(S):
    import torch
    pen, f, params = make_workload("cfg0")
    say("empty inputs", "0 regions, 0 projection columns")
    P = S.Pencil.from_workload(pen)
    sh = S.simm_shift_build(P, 0.1 + 0.1j, f, 20)
    out = S.simm_indicators([sh], np.zeros((0, 4), np.int64), S.params_from_dict(params), want_sums=True)
    assert len(out["decision"]) == 0 and len(out["indicator"]) == 0
    Y = torch.zeros((0, 20), dtype=torch.complex128, device="cuda")
    X = torch.zeros((0, pen.n), dtype=torch.complex128, device="cuda")
    S.simm_project(sh, Y.T, X.T)
    torch.cuda.synchronize()


def test_project_errors(S):
    """simm_project's argument errors: unknown precision, neither X nor norms, a basis
    released at the end of its run."""
    import torch
    pen, f, params = make_workload("cfg0")
    say("projection errors")
    P = S.Pencil.from_workload(pen)
    sh = S.simm_shift_build(P, 0.1 + 0.1j, f, 20)
    Y = torch.ones((3, 20), dtype=torch.complex128, device="cuda")
    nd = torch.zeros(3, dtype=torch.float64, device="cuda")
    for prec in (3, -1):
        with pytest.raises(S.SimmError) as e:
            S.simm_project(sh, Y.T, None, nd, precision=prec)
        assert e.value.status == -1
    with pytest.raises(S.SimmError) as e:
        S.simm_project(sh, Y.T, None, None)
    assert e.value.status == -1
    prm = S.params_from_dict(dict(params, levels=2), flags=S.SIMM_FLAG_RELEASE_FACTORS)
    res = S.simm_run(P, f, prm)
    with pytest.raises(S.SimmError) as e:
        S.simm_project(res.shift(0), Y.T, None, nd)
    assert e.value.status == -1


def test_region_without_eigenvalues(S):
    """Every level-1 square rejected: the later levels test nothing, no clusters."""
    pen, f, params = make_workload("cfg0")
    p = dict(params)
    p.update(x0=3.0, x1=4.0, y0=3.0, y1=4.0, n1=4, levels=3)
    say("simm_run", "cfg0 pencil, R = [3,4]^2 (no eigenvalues)")
    o = O.simm(pen, f, p)
    res = S.simm_run(S.Pencil.from_workload(pen), f, S.params_from_dict(p))
    assert len(o.clusters) == 0 and len(res.lam) == 0
    assert res.K == o.K and res.n_shifts == len(o.shifts)
    for L, OL in zip(res.levels, o.levels):
        assert [tuple(map(int, k)) for k in L.keys] == [tuple(map(int, k)) for k in OL.keys]
        assert np.array_equal(L.decision, OL.decision)


def test_region_guard(S):
    pen, f, params = make_workload("cfg0")
    p = dict(params)
    p["max_regions_per_level"] = 10          # level 1 alone has 64 squares
    say("simm_run", "cfg0 with a 10-square guard")
    with pytest.raises(S.SimmError) as e:
        S.simm_run(S.Pencil.from_workload(pen), f, S.params_from_dict(p))
    assert e.value.status == -7


def test_csr_entry_point_matches_band(S):
    """A and B given as CSR give the same factor and Krylov data as the banded call."""
    pen, f = random_band_pencil(517, 4, 91, b_kind="tridiag", b_offdiag=0.3)
    say("csr", "n=517 k=4, tridiagonal B")
    n = pen.n

    def band_to_csr(band, kl, ku):
        rows, cols, vals = [], [], []
        for i in range(n):
            for j in range(max(0, i - kl), min(n, i + ku + 1)):
                rows.append(i)
                cols.append(j)
                vals.append(band[ku + i - j, j])
        rowptr = np.zeros(n + 1, np.int64)
        np.add.at(rowptr, np.array(rows) + 1, 1)
        return np.cumsum(rowptr), np.array(cols, np.int32), np.array(vals, np.complex128)

    a = band_to_csr(pen.a_band, pen.kl_a, pen.ku_a)
    b = band_to_csr(pen.b_band, pen.kl_b, pen.ku_b)
    Pc = S.Pencil.from_csr(n, *a, *b)
    Pb = S.Pencil.from_workload(pen)
    hc = S.simm_shift_build(Pc, 0.2 + 0.1j, f, 24).info()["H"]
    hb = S.simm_shift_build(Pb, 0.2 + 0.1j, f, 24).info()["H"]
    assert np.array_equal(hc, hb)


# ---------------------------------------------------------------------------
# batched form: many pencils of different orders, runs in flight together
# ---------------------------------------------------------------------------
def test_batch_matches_sequential_and_oracle(S):
    from workloads import make_batch
    batch = make_batch("cfg2_small")
    gold = json.load(open(os.path.join(GOLDEN, "cfg2_small_oracle.json")))["runs"]
    say("simm_run_batch", "cfg2_small:", len(batch), "pencils, n =", [p.n for p, _, _ in batch])
    pencils = [S.Pencil.from_workload(p) for p, _, _ in batch]
    fs = [f for _, f, _ in batch]
    prms = [S.params_from_dict(d, flags=S.SIMM_FLAG_PROJECT) for _, _, d in batch]
    seq = [S.simm_run(P, f, prm) for P, f, prm in zip(pencils, fs, prms)]
    bat = S.simm_run_batch(pencils, fs, prms, workers=4)
    say("  autotuner:", S.simm_batch_tuning())
    ties = 0
    for i, (a, b, g) in enumerate(zip(seq, bat, gold)):
        # the batched run (joint persistent level launches) is the same computation as the
        # separate run, bit for bit
        assert a.K == b.K and a.n_shifts == b.n_shifts
        for s in range(a.n_shifts):
            assert np.array_equal(a.shift(s).info()["H"], b.shift(s).info()["H"])
        for La, Lb in zip(a.levels, b.levels):
            assert np.array_equal(La.keys, Lb.keys) and np.array_equal(La.decision, Lb.decision)
            assert np.array_equal(La.shift, Lb.shift) and np.array_equal(La.indicator, Lb.indicator)
            assert np.array_equal(La.rho_max, Lb.rho_max)
            assert np.array_equal(La.full_indicator, Lb.full_indicator), (i, La.level)
        assert np.array_equal(a.lam, b.lam)
        # and both follow the oracle
        assert b.K == g["K"] and b.n_shifts == len(g["shifts"])
        for L, GL in zip(b.levels, g["levels"]):
            assert [tuple(map(int, k)) for k in L.keys] == list(zip(GL["ix"], GL["iy"])), (i, L.level)
            near = {r: mg for r, mg in GL["near"]}
            for r in np.nonzero(L.decision != np.array(GL["decision"], np.uint8))[0]:
                assert near.get(int(r), 1.0) < 1e-8, (i, L.level, int(r))
                ties += 1
        lam = np.array([complex(*c["lam"]) for c in g["clusters"]])
        assert len(b.lam) == len(lam) and np.all(np.abs(b.lam - lam) <= 1e-14 * np.abs(lam)), i
    say("  decision ties within the margin policy:", ties)


def test_batch_of_full_size_pencils_matches_oracle(S):
    """Eight pencils of the 64-pencil batch at full size (n = 6,153 .. 47,868, 15 to 31
    shifts each), batched with their factors released as each shift is built: the same
    as separate runs, bit for bit, and the oracle's stored runs (levels, decisions up to
    the margin policy, clusters)."""
    from workloads import make_batch
    gold = json.load(open(os.path.join(GOLDEN, "cfg2_subset_oracle.json")))
    full = make_batch("cfg2")
    batch = [full[i] for i in gold["pencils"]]
    say("simm_run_batch", "cfg2 pencils", gold["pencils"], "n =", [p.n for p, _, _ in batch])
    pencils = [S.Pencil.from_workload(p) for p, _, _ in batch]
    fs = [f for _, f, _ in batch]
    prms = [S.params_from_dict(d, flags=S.SIMM_FLAG_RELEASE_FACTORS) for _, _, d in batch]
    bat = S.simm_run_batch(pencils, fs, prms, workers=4)
    ties = 0
    for i, (b, g) in enumerate(zip(bat, gold["runs"])):
        a = S.simm_run(pencils[i], fs[i], prms[i])
        assert a.K == b.K and a.n_shifts == b.n_shifts
        for s_ in range(a.n_shifts):
            assert np.array_equal(a.shift(s_).info()["H"], b.shift(s_).info()["H"])
        for La, Lb in zip(a.levels, b.levels):
            assert np.array_equal(La.keys, Lb.keys) and np.array_equal(La.decision, Lb.decision)
            assert np.array_equal(La.shift, Lb.shift) and np.array_equal(La.indicator, Lb.indicator)
        assert np.array_equal(a.lam, b.lam)
        assert b.K == g["K"] and b.n_shifts == len(g["shifts"])
        for L, GL in zip(b.levels, g["levels"]):
            assert [tuple(map(int, k)) for k in L.keys] == list(zip(GL["ix"], GL["iy"])), (i, L.level)
            near = {r: mg for r, mg in GL["near"]}
            for r in np.nonzero(L.decision != np.array(GL["decision"], np.uint8))[0]:
                assert near.get(int(r), 1.0) < 1e-8, (i, L.level, int(r))
                ties += 1
        lam = np.array([complex(*c["lam"]) for c in g["clusters"]])
        assert len(b.lam) == len(lam) and np.all(np.abs(b.lam - lam) <= 1e-14 * np.abs(lam)), i
        say(f"  pencil {gold['pencils'][i]}: n = {batch[i][0].n}, {b.n_shifts} shifts, K = {b.K}, "
            f"{len(b.lam)} clusters")
    say("  decision ties within the margin policy:", ties)


def test_batch_64_pencils_matches_oracle(S):
    """The whole 64-pencil batch (n = 2,163 .. 47,868, 1.6 M rows, 3,392 shifts), batched
    as bench.py runs it (6 runs in flight, 2 factors ahead each, factors released per
    shift), against the oracle's stored runs of every pencil: levels, squares, decisions
    up to the margin policy, shift counts and clusters."""
    from workloads import make_batch
    gold = json.load(open(os.path.join(GOLDEN, "cfg2_oracle.json")))["runs"]
    batch = make_batch("cfg2")
    assert len(gold) == len(batch) == 64
    say("simm_run_batch", "cfg2: 64 pencils, n =", sum(p.n for p, _, _ in batch))
    pencils = [S.Pencil.from_workload(p) for p, _, _ in batch]
    fs = [f for _, f, _ in batch]
    prms = [S.params_from_dict(d, flags=S.SIMM_FLAG_RELEASE_FACTORS, lookahead=2) for _, _, d in batch]
    bat = S.simm_run_batch(pencils, fs, prms, workers=6)
    ties = squares = 0
    for i, (b, g) in enumerate(zip(bat, gold)):
        assert g["n"] == batch[i][0].n
        assert b.K == g["K"] and b.n_shifts == len(g["shifts"]), i
        for L, GL in zip(b.levels, g["levels"]):
            assert [tuple(map(int, k)) for k in L.keys] == list(zip(GL["ix"], GL["iy"])), (i, L.level)
            near = {r: mg for r, mg in GL["near"]}
            for r in np.nonzero(L.decision != np.array(GL["decision"], np.uint8))[0]:
                assert near.get(int(r), 1.0) < 1e-8, (i, L.level, int(r))
                ties += 1
            squares += len(L.keys)
        lam = np.array([complex(*c["lam"]) for c in g["clusters"]])
        assert len(b.lam) == len(lam) and np.all(np.abs(b.lam - lam) <= 1e-14 * np.abs(lam)), i
    say(f"  {squares} squares, {sum(len(g['clusters']) for g in gold)} clusters; decision ties within the "
        f"margin policy: {ties}")


# ---------------------------------------------------------------------------
# adjoint gradient of J = sum_R ||x_R||^2 (squares held fixed)
# ---------------------------------------------------------------------------
def _grad_problem(n, seed, level, nsq):
    """Pencil, A1 (tridiagonal band), params and up to nsq level-`level` squares, each
    around an eigenvalue with every eigenvalue at least 0.15 w from its edges, plus one
    square far from the spectrum; one shift per square (its centre, offset)."""
    pen, f = random_band_pencil(n, 2, seed, b_kind="tridiag", b_offdiag=0.2)
    A, B = O.pencil_dense(pen)
    rng = np.random.default_rng(seed + 1)
    a1 = np.zeros((3, n), dtype=np.complex128, order="F")      # kl1 = ku1 = 1
    a1[0, 1:] = rng.standard_normal(n - 1) * 0.1
    a1[1, :] = rng.standard_normal(n) * 0.3
    a1[2, :-1] = rng.standard_normal(n - 1) * 0.1
    x0, n1, w1 = -10.0, 50, 0.4
    w = w1 * 2.0 ** (1 - level)
    ev = np.linalg.eigvals(np.linalg.solve(B, A))
    sq = []
    for lam in ev:
        ix, iy = int(np.floor((lam.real - x0) / w)), int(np.floor((lam.imag - x0) / w))
        c = complex(x0 + (ix + 0.5) * w, x0 + (iy + 0.5) * w)
        near = (np.abs(ev.real - c.real) < 0.65 * w) & (np.abs(ev.imag - c.imag) < 0.65 * w)
        dist = np.minimum(np.abs(np.abs(ev.real - c.real) - w / 2), np.abs(np.abs(ev.imag - c.imag) - w / 2))
        if np.all(dist[near] > 0.15 * w) and (ix, iy) not in sq:
            sq.append((ix, iy))
        if len(sq) == nsq:
            break
    sq.append((45, 45))                                          # centre 8.2 + 8.2i: no eigenvalue near
    regions = np.array([(level, ix, iy, k) for k, (ix, iy) in enumerate(sq)], dtype=np.int64)
    centres = [complex(x0 + (ix + 0.5) * w, x0 + (iy + 0.5) * w) for ix, iy in sq]
    sigmas = [c + (0.013 + 0.021j) * w for c in centres]
    prm = dict(x0=x0, y0=x0, x1=x0 + n1 * w1, n1=n1, gauss_per_edge=8)
    return pen, f, a1, O.band_to_dense(n, 1, 1, a1), regions, [(c, w) for c in centres], sigmas, prm


GRAD_CASES = [
    # name, n, seed, level, squares near eigenvalues, m
    ("n60-m=n", 60, 7, 1, 3, 60),
    ("n300-level3", 300, 11, 3, 2, 100),
]


@pytest.mark.parametrize("case", GRAD_CASES, ids=[c[0] for c in GRAD_CASES])
def test_gradient_matches_oracle_and_fd(S, case):
    name, n, seed, level, nsq, m = case
    pen, f, a1, A1, regions, squares, sigmas, prm = _grad_problem(n, seed, level, nsq)
    A, B = O.pencil_dense(pen)
    J_o, dp_o, gd_o = O.projected_norms_gradient(A, A1, B, f, squares, prm["gauss_per_edge"])
    say("gradient", name, f"n={n} m={m} squares={len(squares)} J_oracle={J_o:.6e}")
    P = S.Pencil.from_workload(pen)
    shifts = [S.simm_shift_build(P, s, f, m) for s in sigmas]
    params = S.params_from_dict(prm, m=m)
    J, dp, gd = S.simm_gradient(shifts, regions, params, a1, 1, 1)
    say("  J", J, "dJ/dp", dp, "oracle", dp_o)
    assert abs(J - J_o) <= 1e-8 * J_o
    assert abs(dp - dp_o) <= 1e-6 * abs(dp_o)
    scale = np.max(np.abs(gd_o))
    err = np.max(np.abs(gd - gd_o)) / scale
    say("  max |grad_diag - oracle| / max|oracle| =", err)
    assert err <= 1e-6
    # central differences of the library's own J (h = 1e-6)
    prob = S.ProjectedNorms(n, pen.kl_a, pen.ku_a, pen.a_band, 1, 1, a1, f, sigmas, regions, params, m,
                            pen.kl_b, pen.ku_b, pen.b_band)
    h = 1e-6
    d0 = np.zeros(n, dtype=np.complex128)
    J_only = prob.evaluate(0.0, d0, derivatives=False)
    assert J_only[1] is None and J_only[2] is None
    assert abs(J_only[0] - J) <= 1e-12 * J
    Jp = prob.evaluate(h, d0, derivatives=False)[0]
    Jm = prob.evaluate(-h, d0, derivatives=False)[0]
    fd = (Jp - Jm) / (2 * h)
    say("  dJ/dp", dp, "central difference", fd)
    assert abs(dp - fd) <= 1e-6 * abs(fd)
    for i in (0, n // 2 + 1):
        e = np.zeros(n, dtype=np.complex128)
        e[i] = h
        Jd = [prob.evaluate(0.0, v, derivatives=False)[0] for v in (e, -e, 1j * e, -1j * e)]
        fr = (Jd[0] - Jd[1]) / (2 * h)
        fi = (Jd[2] - Jd[3]) / (2 * h)
        say("  grad_diag", i, gd[i], "central difference", fr + 1j * fi)
        assert abs(gd[i] - (fr + 1j * fi)) <= 1e-6 * scale


GRAD_PART_CASES = [
    # name, n, seed, level, squares near eigenvalues, m, block length of the forward factors
    ("n300-level3-2blocks", 300, 11, 3, 2, 100, 256),
    ("n600-level3-3blocks", 600, 17, 3, 3, 100, 256),
]


@pytest.mark.parametrize("case", GRAD_PART_CASES, ids=[c[0] for c in GRAD_PART_CASES])
def test_gradient_partitioned_matches_oracle(S, part_env, case):
    """Partitioned factors (two and three diagonal blocks) for the forward shifts and for
    the conjugate-transposed pencil of the adjoint spaces: J, dJ/dp and dJ/dA_ii against
    the oracle's dense adjoint gradient."""
    name, n, seed, level, nsq, m, bs = case
    part_env["SIMM_LU_PART"] = str(bs)
    pen, f, a1, A1, regions, squares, sigmas, prm = _grad_problem(n, seed, level, nsq)
    A, B = O.pencil_dense(pen)
    J_o, dp_o, gd_o = O.projected_norms_gradient(A, A1, B, f, squares, prm["gauss_per_edge"])
    say("gradient, partitioned factors", name, f"n={n} m={m} block={bs} squares={len(squares)}")
    P = S.Pencil.from_workload(pen)
    shifts = [S.simm_shift_build(P, s, f, m) for s in sigmas]
    assert all(sh.factor_info()["block_len"] == bs for sh in shifts)
    params = S.params_from_dict(prm, m=m)
    J, dp, gd = S.simm_gradient(shifts, regions, params, a1, 1, 1)
    scale = np.max(np.abs(gd_o))
    err = np.max(np.abs(gd - gd_o)) / scale
    say("  J", J, "oracle", J_o, "dJ/dp", dp, "oracle", dp_o, "grad_diag rel. error", err)
    assert abs(J - J_o) <= 1e-8 * J_o
    assert abs(dp - dp_o) <= 1e-6 * abs(dp_o)
    assert err <= 1e-6


def test_gradient_n100000_matches_banded_oracle(S):
    """The differentiation workload at full size (n = 100,000, half-bandwidth 32): the
    library's run fixes the same admissible squares as the oracle's run, and its Krylov
    adjoint gradient over them equals the oracle's banded direct-solve gradient
    (tests/golden/cfg4_gradient.json): J and dJ/dp to 1e-6 relative, dJ/dA_ii at the
    stored rows (the workload's listed rows and the 20 largest) to 1e-6 of the largest."""
    from workloads import load_config, random_band_matrix
    gold = json.load(open(os.path.join(GOLDEN, "cfg4_gradient.json")))
    cfg = load_config("cfg4")
    d = cfg["differentiation"]
    pen0, f, params = make_workload("cfg4")
    n, k1 = pen0.n, d["k1"]
    a1 = random_band_matrix(n, k1, d["seed"], 1.0 / np.sqrt(n))
    kl, ku, band = S._band_sum(n, [(pen0.kl_a, pen0.ku_a, pen0.a_band), (k1, k1, d["p"] * a1)])
    say("gradient cfg4", f"n={n} kl={kl} ku={ku} m={params['m']}")
    P = S.Pencil(n, kl, ku, band, pen0.kl_b, pen0.ku_b, pen0.b_band)
    prm = S.params_from_dict(params)
    res = S.simm_run(P, f, prm)
    assert res.K == gold["K"]
    last = res.levels[-1]
    adm = np.nonzero(last.decision == S.ADMISSIBLE)[0]
    assert [[int(last.keys[i, 0]), int(last.keys[i, 1])] for i in adm] == gold["squares"]
    used = sorted(set(int(last.shift[i]) for i in adm))
    remap = {s: j for j, s in enumerate(used)}
    regions = np.array([(res.K, last.keys[i, 0], last.keys[i, 1], remap[int(last.shift[i])]) for i in adm],
                       dtype=np.int64).reshape(-1, 4)
    shifts = [res.shift(s) for s in used]
    J, dp, gd = S.simm_gradient(shifts, regions, prm, a1, k1, k1, n=n)
    say("  J", J, "oracle", gold["J"], " dJ/dp", dp, "oracle", gold["dJdp"])
    assert abs(J - gold["J"]) <= 1e-6 * gold["J"]
    assert abs(dp - gold["dJdp"]) <= 1e-6 * abs(gold["dJdp"])
    want = np.array([complex(*v) for v in gold["grad"]])
    err = np.max(np.abs(gd[gold["grad_rows"]] - want)) / gold["grad_scale"]
    say("  max |grad_diag - oracle| / max|oracle| over", len(want), "rows:", err)
    assert err <= 1e-6
    assert abs(np.max(np.abs(gd)) - gold["grad_scale"]) <= 1e-6 * gold["grad_scale"]


def test_gradient_autograd_function(S):
    import torch
    n, m = 60, 60
    pen, f, a1, A1, regions, squares, sigmas, prm = _grad_problem(n, 7, 1, 2)
    say("gradient autograd", f"n={n} m={m}")
    params = S.params_from_dict(prm, m=m)
    prob = S.ProjectedNorms(n, pen.kl_a, pen.ku_a, pen.a_band, 1, 1, a1, f, sigmas, regions, params, m,
                            pen.kl_b, pen.ku_b, pen.b_band)
    fn = prob.function()
    p = torch.tensor(0.25, dtype=torch.float64, requires_grad=True)
    d = torch.zeros(n, dtype=torch.complex128, requires_grad=True)
    J = fn(p, d)
    (3.0 * J).backward()
    A, B = O.pencil_dense(pen)
    J_o, dp_o, gd_o = O.projected_norms_gradient(A + 0.25 * A1, A1, B, f, squares, prm["gauss_per_edge"])
    assert abs(J.item() - J_o) <= 1e-8 * J_o
    assert abs(p.grad.item() - 3.0 * dp_o) <= 1e-6 * abs(3.0 * dp_o)
    assert np.max(np.abs(d.grad.numpy() - 3.0 * gd_o)) <= 1e-6 * np.max(np.abs(3.0 * gd_o))
    # inputs on the GPU: the gradients come back there
    pg = torch.tensor(0.25, dtype=torch.float64, device="cuda:0", requires_grad=True)
    dg = torch.zeros(n, dtype=torch.complex128, device="cuda:0", requires_grad=True)
    fn(pg, dg).backward()
    assert pg.grad.device.type == "cuda" and dg.grad.device.type == "cuda"
    assert abs(pg.grad.item() - dp_o) <= 1e-6 * abs(dp_o)


def test_gradient_errors(S):
    pen, f = random_band_pencil(40, 2, 5, b_kind="identity")
    P = S.Pencil.from_workload(pen)
    sh = S.simm_shift_build(P, 0.1 + 0.1j, f, 20)
    params = S.params_from_dict(dict(x0=-2.0, y0=-2.0, x1=2.0, n1=10, gauss_per_edge=4), m=20)
    say("gradient errors")
    with pytest.raises(S.SimmError):
        S.simm_gradient([sh], np.array([[0, 1, 1, 0]]), params)          # level 0
    with pytest.raises(S.SimmError):
        S.simm_gradient([sh], np.array([[1, 1, 1, 1]]), params)          # shift index out of range
    J, dp, gd = S.simm_gradient([sh], np.zeros((0, 4), dtype=np.int64), params)
    assert J == 0.0 and dp is None and np.all(gd == 0)


def test_gradient_unresolved_squares_are_errors(S):
    """simm_gradient refuses squares whose reduced solves are not resolved (Definition
    3.1 with eq. (error)): with m = 6 the forward spaces of the n = 300 problem are too
    small; and with f in a 2-dimensional invariant subspace of an upper triangular A the
    forward space is exact (breakdown at 2, residual 0) while the adjoint space of A^H,
    started from x_R, is not."""
    pen, f, a1, A1, regions, squares, sigmas, prm = _grad_problem(300, 11, 3, 2)
    say("gradient", "unresolved forward squares (m = 6)")
    P = S.Pencil.from_workload(pen)
    shifts = [S.simm_shift_build(P, s, f, 6) for s in sigmas]
    params = S.params_from_dict(prm, m=6)
    with pytest.raises(S.SimmError) as e:
        S.simm_gradient(shifts, regions, params, a1, 1, 1)
    assert e.value.status == -10 and "not resolved by its shift" in str(e.value)
    # upper triangular A (band kl = 1 with a zero subdiagonal, ku = 2), B = I
    n = 60
    rng = np.random.default_rng(61)
    band = np.zeros((4, n), dtype=np.complex128, order="F")
    band[2, :] = np.linspace(-3.0, 3.0, n) + 0.5j                   # diagonal (row ku = 2)
    band[1, 1:] = 0.7 * (rng.standard_normal(n - 1) + 1j * rng.standard_normal(n - 1))
    band[0, 2:] = 0.7 * (rng.standard_normal(n - 2) + 1j * rng.standard_normal(n - 2))
    tri = WPencil(n, 1, 2, band, 0, 0, None)
    f2 = np.zeros(n, np.complex128)
    f2[0], f2[1] = 1.0, 0.5
    lam0 = complex(band[2, 0])                                        # eigenvalue -3 + 0.5i
    say("gradient", "exact forward space, unresolved adjoint space")
    P2 = S.Pencil.from_workload(tri)
    w = 0.25
    x0 = -3.1
    p2 = dict(x0=x0, y0=0.4, x1=x0 + w, n1=1, gauss_per_edge=8)
    sh = S.simm_shift_build(P2, lam0 + 0.03 + 0.02j, f2, 4)
    assert sh.info()["m_eff"] == 2
    reg = np.array([[1, 0, 0, 0]], dtype=np.int64)
    J, _, _ = S.simm_gradient([sh], reg, S.params_from_dict(p2, m=4), want_diag=False, want_dp=False)
    assert J > 0.0                                                    # the square holds the eigenvalue
    with pytest.raises(S.SimmError) as e:
        S.simm_gradient([sh], reg, S.params_from_dict(p2, m=4), want_diag=True, want_dp=False)
    assert e.value.status == -10 and "adjoint" in str(e.value)


# ---------------------------------------------------------------------------
# mixed precision: FP32 factor, solves refined against the FP64 pencil
# ---------------------------------------------------------------------------
def _backward_error(pen, sigma, u, y):
    """||u - (A - sigma B) y||_inf / (||A - sigma B||_inf ||y||_inf + ||u||_inf), on the host."""
    A, B = O.pencil_dense(pen)
    C = A - sigma * B
    r = u - C @ y
    return float(np.max(np.abs(r)) / (np.max(np.sum(np.abs(C), axis=1)) * np.max(np.abs(y)) + np.max(np.abs(u))))


MIXED_CASES = [c for c in CASES if c[0] in ("cfg0-like", "tridiagB", "pivoting", "ragged-wide", "band60-pivoting",
                                            "band224")]


@pytest.mark.parametrize("case", MIXED_CASES, ids=[c[0] for c in MIXED_CASES])
def test_mixed_shift_build(S, case):
    """FP32 factor: every refined solve meets the backward-error tolerance 1e-12 (checked
    on the host with the dense pencil), and H stays close to the oracle's FP64 H (a solve
    with backward error 1e-12 perturbs M by about kappa(A - sigma B) 1e-12)."""
    name, n, k, seed, b_kind, m, sigma, kw = case
    pen, f = random_band_pencil(n, k, seed, b_kind=b_kind, b_offdiag=0.3, **kw)
    say("mixed shift_build", name, f"n={n} k={k} m={m}")
    P = S.Pencil.from_workload(pen)
    sh = S.simm_shift_build(P, sigma, f, m, precision=S.SIMM_PREC_MIXED)
    st = sh.refine_stats()
    assert st["solves"] >= m + 1 and st["max_eta"] <= 1e-12, st
    g = sh.info()
    o = O.build_shift(pen, sigma, f, m)
    assert g["m_eff"] == o.m_eff
    d = hmax_diff(g["H"], o.H)
    say(f"  refined solves {st['solves']}, corrections {st['corrections']}, max backward error {st['max_eta']:.2e}; "
        f"max |H_mixed - H_oracle| / max|H| = {d:.2e}")
    assert d <= 1e-7
    rng = np.random.default_rng(17)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    y = np.zeros(n, np.complex128)
    sh.apply(x, y)
    u = O.band_matvec(n, pen.kl_b, pen.ku_b, pen.b_band, x)
    eta = _backward_error(pen, sigma, u, y)
    say(f"  one application: host backward error {eta:.2e}")
    assert eta <= 1e-12


def test_mixed_refinement_failure_falls_back_to_fp64(S):
    """A shift 1e-10 from an eigenvalue of a tridiagonal pencil with known spectrum
    (2 - 2 cos(k pi / (n + 1))): kappa(A - sigma I) ~ 4e10, so FP32 refinement cannot
    converge (its contraction kappa u_32 > 1).  simm_shift_build reports SIMM_EREFINE; a
    run whose first shift sits there rebuilds that shift in FP64 and equals the FP64 run."""
    n = 200
    band = np.zeros((3, n), dtype=np.complex128, order="F")
    band[0, 1:] = -1.0
    band[1, :] = 2.0
    band[2, :-1] = -1.0
    pen = WPencil(n, 1, 1, band, 0, 0, None)
    lam1 = 2.0 - 2.0 * np.cos(np.pi / (n + 1))
    sigma = lam1 + 1e-10
    f = np.ones(n, np.complex128)
    say("mixed refinement failure", f"n={n}, sigma = lambda_1 + 1e-10")
    P = S.Pencil.from_workload(pen)
    with pytest.raises(S.SimmError) as e:
        S.simm_shift_build(P, sigma, f, 20, precision=S.SIMM_PREC_MIXED)
    assert e.value.status == -9
    w = 2e-4
    prm = dict(x0=sigma - w / 2, x1=sigma + w / 2, y0=-w / 2, y1=w / 2, n1=1, gauss_per_edge=8, m=20, h0=0,
               levels=3, eps0=1e-8, delta0=0.05, tau=1e-8)
    r64 = S.simm_run(P, f, S.params_from_dict(prm))
    rmx = S.simm_run(P, f, S.params_from_dict(prm, precision=S.SIMM_PREC_MIXED))
    assert rmx.refine["fallbacks"] == 1 and r64.refine["fallbacks"] == 0
    for L64, Lmx in zip(r64.levels, rmx.levels):
        assert np.array_equal(L64.keys, Lmx.keys) and np.array_equal(L64.decision, Lmx.decision)
        assert np.array_equal(L64.indicator, Lmx.indicator)
    assert np.array_equal(r64.lam, rmx.lam)


def _run_matches_golden(S, res, gold):
    """Squares, shifts and decisions of every level equal the oracle's stored run (a
    decision may differ only where the oracle's margin is below 1e-8); clusters equal."""
    assert res.K == gold["K"] and res.n_shifts == len(gold["shifts"])
    ties = 0
    for L, G in zip(res.levels, gold["levels"]):
        assert np.array_equal(L.keys[:, 0], G["ix"]) and np.array_equal(L.keys[:, 1], G["iy"]), L.level
        assert np.array_equal(L.shift, G["shift"]), L.level
        for r in np.nonzero(L.decision != np.array(G["decision"]))[0]:
            ties += 1
            assert G["margin"][r] < 1e-8, (L.level, r, G["margin"][r])
    lam = np.array([complex(*c["lam"]) for c in gold["clusters"]])
    assert len(res.lam) == len(lam) and np.all(np.abs(res.lam - lam) <= 1e-14 * np.maximum(1.0, np.abs(lam)))
    return ties


def test_run_mixed_cfg0_matches_oracle(S):
    pen, f, params = make_workload("cfg0")
    say("run", "cfg0 mixed precision")
    with open(os.path.join(GOLDEN, "cfg0_oracle.json")) as fh:
        gold = json.load(fh)
    P = S.Pencil.from_workload(pen)
    res = S.simm_run(P, f, S.params_from_dict(params, flags=S.SIMM_FLAG_PROJECT, precision=S.SIMM_PREC_MIXED))
    ties = _run_matches_golden(S, res, gold)
    say(f"  ties {ties}; refinement {res.refine}")
    assert res.refine["solves"] > 0 and res.refine["max_eta"] <= 1e-12


@pytest.mark.skipif(not os.path.exists(os.path.join(GOLDEN, "cfg3_small_oracle.json")), reason="no stored run")
def test_run_cfg3_eigenvalues_against_arpack_sample(S):
    """The n = 250,000 mixed-precision workload at full size, sampled: the 40 eigenvalues
    nearest R's centre from shift-invert ARPACK on the host (tests/arpack_ref.py).  Every
    one of them that lies in R is the Ritz value of a cluster of the FP64 run and of the
    mixed run within 1e-8 relative (the FP64 error of each eigenvalue), and both runs have
    the same clusters."""
    from tests import arpack_ref
    pen, f, params = make_workload("cfg3")
    P = S.Pencil.from_workload(pen)
    say("run", "cfg3 FP64")
    r64 = S.simm_run(P, f, S.params_from_dict(params))
    say("run", "cfg3 mixed")
    rmx = S.simm_run(P, f, S.params_from_dict(params, flags=S.SIMM_FLAG_PROJECT, precision=S.SIMM_PREC_MIXED))
    assert np.array_equal(r64.lam, rmx.lam) and r64.n_unresolved == 0 and rmx.n_unresolved == 0
    say("ARPACK: 40 eigenvalues nearest the centre of R (host)")
    A, B = arpack_ref.pencil_csc(pen)
    c = complex((params["x0"] + params["x1"]) / 2, (params["y0"] + params["y1"]) / 2)
    lam, r = arpack_ref.nearest_eigenvalues(A, B, c, 40)
    inR = (lam.real >= params["x0"]) & (lam.real <= params["x1"]) & (lam.imag >= params["y0"]) & \
          (lam.imag <= params["y1"]) & (np.abs(lam - c) < 0.98 * r)
    sample = lam[inR]
    assert len(sample) >= 30
    for tag, res in (("FP64", r64), ("mixed", rmx)):
        z = res.lam_ritz[np.isfinite(res.lam_ritz)]
        e = np.array([np.min(np.abs(z - v)) / abs(v) for v in sample])
        say(f"  {tag}: {len(sample)} eigenvalues, rel. error of the nearest Ritz value median {np.median(e):.1e}, "
            f"max {e.max():.1e}")
        assert e.max() <= 1e-8


def test_run_mixed_cfg3_small_matches_oracle_and_fp64(S):
    """The reduced mixed-precision workload (n = 20,000, half-bandwidth 64, m = 120, 32
    Gauss points per edge, 17 levels): FP64 and mixed runs both equal the oracle's squares,
    shifts, decisions and clusters; the Ritz eigenvalue of every cluster of the mixed run
    is within 1e-8 (relative) of the FP64 run's."""
    pen, f, params = make_workload("cfg3_small")
    with open(os.path.join(GOLDEN, "cfg3_small_oracle.json")) as fh:
        gold = json.load(fh)
    P = S.Pencil.from_workload(pen)
    say("run", "cfg3_small FP64")
    r64 = S.simm_run(P, f, S.params_from_dict(params))
    say("run", "cfg3_small mixed")
    rmx = S.simm_run(P, f, S.params_from_dict(params, flags=S.SIMM_FLAG_PROJECT, precision=S.SIMM_PREC_MIXED))
    t64 = _run_matches_golden(S, r64, gold)
    tmx = _run_matches_golden(S, rmx, gold)
    ok = np.isfinite(r64.lam_ritz) & np.isfinite(rmx.lam_ritz)
    err = np.abs(rmx.lam_ritz[ok] - r64.lam_ritz[ok]) / np.maximum(np.abs(r64.lam_ritz[ok]), 1e-300)
    say(f"  ties {t64}/{tmx}; refinement {rmx.refine}; {int(ok.sum())} Ritz eigenvalues, max rel. difference "
        f"mixed vs FP64 {err.max() if err.size else 0.0:.2e}")
    assert np.array_equal(np.isfinite(r64.lam_ritz), np.isfinite(rmx.lam_ritz))
    assert err.size == 0 or err.max() <= 1e-8
    assert rmx.refine["max_eta"] <= 1e-12
    # the error of every eigenvalue against an independent solver: shift-invert ARPACK on
    # the host (tests/arpack_ref.py), every eigenvalue in R
    from tests import arpack_ref
    say("ARPACK eigenvalues of cfg3_small in R (host)")
    eigs = arpack_ref.eigenvalues_in_region(pen, params["x0"], params["x1"], params["y0"], params["y1"],
                                            nx=2, ny=2, k=30)
    assert len(eigs) == int(ok.sum())
    for tag, r in (("FP64", r64), ("mixed", rmx)):
        e = np.array([np.min(np.abs(eigs - z)) / abs(z) for z in r.lam_ritz[ok]])
        say(f"  {tag}: {len(e)} eigenvalues, rel. error vs ARPACK median {np.median(e):.1e}, max {e.max():.1e}")
        assert e.max() <= 1e-8
