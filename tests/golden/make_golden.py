"""Writes the stored expected results of full SIM-M runs.  Calls only the CPU
oracle (oracle/simm.py) on the seeded workloads; nothing here comes from the
HIP library.  Usage: python tests/golden/make_golden.py cfg0 [cfg1 cfg2_small ...]
(batch workloads are stored compactly: decisions and keys per level, and the
margins of the squares closer than 1e-6 to a decision threshold).

  python tests/golden/make_golden.py --gradient cfg4
runs the oracle on the differentiation pencil A0 + p A1, takes the admissible squares
of its last level and stores J, dJ/dp and rows of dJ/dA_ii from the oracle's banded
adjoint gradient in <name>_gradient.json.

  python tests/golden/make_golden.py --hessenberg cfg0 cfg1
rebuilds, with the oracle, every shift of a stored run (the sigmas of
<name>_oracle.json) and stores sigma, beta and the full H_{m+1,m} of each in
<name>_hessenberg.npz (numpy arrays, no pickled objects)."""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle.simm as O  # noqa: E402
from workloads import load_config, make_batch, make_workload  # noqa: E402


def cplx(z):
    return [float(np.real(z)), float(np.imag(z))]


def full_trace(res):
    return {
        "K": res.K,
        "shifts": [{"sigma": cplx(s.sigma), "beta": s.beta, "m_eff": s.m_eff, "h_last": s.h_last,
                    "H_diag": [cplx(v) for v in np.diag(s.Hm)],
                    "H_sub": [float(np.real(v)) for v in np.diag(s.H, -1)]} for s in res.shifts],
        "levels": [{"level": L.level,
                    "ix": [int(v) for v in L.keys[:, 0]], "iy": [int(v) for v in L.keys[:, 1]],
                    "shift": [int(v) for v in L.shift], "decision": [int(v) for v in L.decision],
                    "indicator": [float(v) for v in L.indicator], "rho_max": [float(v) for v in L.rho_max],
                    "margin": [float(v) for v in L.margin]} for L in res.levels],
        "clusters": [{"lam": cplx(c.lam), "lam_ritz": cplx(c.lam_ritz), "shift": c.shift,
                      "unresolved": c.unresolved, "members": c.members} for c in res.clusters],
    }


def compact_trace(res):
    return {
        "K": res.K,
        "shifts": [{"sigma": cplx(s.sigma), "beta": s.beta, "m_eff": s.m_eff} for s in res.shifts],
        "levels": [{"level": L.level,
                    "ix": [int(v) for v in L.keys[:, 0]], "iy": [int(v) for v in L.keys[:, 1]],
                    "shift": [int(v) for v in L.shift], "decision": [int(v) for v in L.decision],
                    "near": [[int(r), float(L.margin[r])] for r in np.nonzero(L.margin < 1e-6)[0]]}
                   for L in res.levels],
        "clusters": [{"lam": cplx(c.lam), "lam_ritz": cplx(c.lam_ritz), "shift": c.shift,
                      "unresolved": c.unresolved} for c in res.clusters],
    }


def _batch_run(arg):
    name, i = arg
    pen, f, params = make_batch(name)[i]
    res = O.simm(pen, f, params)
    print(f"{name} pencil {i}: n = {pen.n}, {len(res.shifts)} shifts, {len(res.clusters)} clusters", flush=True)
    return {"n": pen.n, **compact_trace(res)}


def hessenberg(names):
    for name in names:
        t0 = time.time()
        pen, f, params = make_workload(name)
        with open(os.path.join(HERE, f"{name}_oracle.json")) as fh:
            run = json.load(fh)
        m = params["m"]
        sig, beta, meff = [], [], []
        H = np.zeros((len(run["shifts"]), m + 1, m), dtype=np.complex128)
        for i, rec in enumerate(run["shifts"]):
            sh = O.build_shift(pen, complex(*rec["sigma"]), f, m, keep_V=False)
            assert sh.m_eff == rec["m_eff"] and abs(sh.beta - rec["beta"]) <= 1e-14 * rec["beta"], (name, i)
            sig.append(sh.sigma)
            beta.append(sh.beta)
            meff.append(sh.m_eff)
            H[i, : sh.m_eff + 1, : sh.m_eff] = sh.H
        path = os.path.join(HERE, f"{name}_hessenberg.npz")
        np.savez_compressed(path, sigma=np.array(sig), beta=np.array(beta), m_eff=np.array(meff, dtype=np.int64), H=H)
        print(name, "->", path, f"{time.time() - t0:.1f} s, {len(sig)} shifts")


def differentiation_pencil(name):
    """The pencil A(p) = A0 + p A1 of a differentiation workload, with A0, f and the
    parameters of the workload file and A1 from its seeded band generator."""
    from workloads import Pencil, random_band_matrix
    cfg = load_config(name)
    d = cfg["differentiation"]
    pen0, f, params = make_workload(name)
    n, k1 = pen0.n, d["k1"]
    a1 = random_band_matrix(n, k1, d["seed"], 1.0 / np.sqrt(n))
    kl, ku = max(pen0.kl_a, k1), max(pen0.ku_a, k1)
    band = np.zeros((kl + ku + 1, n), dtype=np.complex128, order="F")
    band[ku - pen0.ku_a: ku + pen0.kl_a + 1, :] += pen0.a_band
    band[ku - k1: ku + k1 + 1, :] += d["p"] * a1
    return Pencil(n, kl, ku, band, pen0.kl_b, pen0.ku_b, pen0.b_band), a1, k1, f, params, d


def _gradient_square(arg):
    name, center, width = arg
    pen, a1, k1, f, params, _ = differentiation_pencil(name)
    J, dp, gd = O.projected_norms_gradient_banded(pen.n, pen.kl_a, pen.ku_a, pen.a_band, pen.kl_b, pen.ku_b,
                                                  pen.b_band, k1, k1, a1, f, [(center, width)],
                                                  params["gauss_per_edge"])
    print(f"{name} square at {center:.6g}: J_R = {J:.6e}", flush=True)
    return J, dp, gd


def gradient(names, n_top=20):
    """J, dJ/dp and dJ/dA_ii (at the workload's listed rows and the n_top rows of largest
    modulus) over the admissible squares of the oracle's own run's last level."""
    import multiprocessing as mp
    for name in names:
        t0 = time.time()
        pen, a1, k1, f, params, d = differentiation_pencil(name)
        res = O.simm(pen, f, params)
        last = res.levels[-1]
        adm = [int(r) for r in np.nonzero(last.decision == O.DECISION_ADMISSIBLE)[0]]
        w = O.square_width(params, last.level)
        squares = [(O.square_center(params, last.level, int(last.keys[r, 0]), int(last.keys[r, 1])), w) for r in adm]
        print(f"{name}: run {time.time() - t0:.1f} s, K = {res.K}, {len(adm)} admissible squares", flush=True)
        with mp.get_context("spawn").Pool(int(os.environ.get("GOLDEN_PROCS", "6"))) as pool:
            parts = pool.map(_gradient_square, [(name, c, ww) for c, ww in squares])
        J = sum(p[0] for p in parts)
        dp = sum(p[1] for p in parts)
        gd = sum(p[2] for p in parts)
        rows = list(d["fd_diag"]) + [int(i) for i in np.argsort(-np.abs(gd))[:n_top]]
        out = {"workload": name, "generated_by": "oracle/simm.py via tests/golden/make_golden.py --gradient",
               "oracle_seconds": round(time.time() - t0, 1), "K": res.K,
               "squares": [[int(last.keys[r, 0]), int(last.keys[r, 1])] for r in adm],
               "sigmas": [cplx(s.sigma) for s in res.shifts],
               "J": J, "dJdp": dp, "grad_scale": float(np.max(np.abs(gd))),
               "grad_rows": rows, "grad": [cplx(gd[i]) for i in rows]}
        path = os.path.join(HERE, f"{name}_gradient.json")
        with open(path, "w") as fh:
            json.dump(out, fh, separators=(",", ":"))
        print(name, "->", path, f"{out['oracle_seconds']} s, J = {J:.10e}, dJ/dp = {dp:.10e}")


def main(names):
    for name in names:
        t0 = time.time()
        kind = load_config(name)["generator"]["kind"]
        if kind.endswith("_batch"):
            # the pencils are independent: several processes, one BLAS thread each;
            # GOLDEN_PENCILS=i,j,... stores only those pencils (as <name>_subset_oracle.json)
            import multiprocessing as mp
            count = len(make_batch(name))
            only = os.environ.get("GOLDEN_PENCILS")
            idx = [int(v) for v in only.split(",")] if only else list(range(count))
            with mp.get_context("spawn").Pool(int(os.environ.get("GOLDEN_PROCS", "6"))) as pool:
                runs = pool.map(_batch_run, [(name, i) for i in idx], chunksize=1)
            out = {"workload": name, "generated_by": "oracle/simm.py via tests/golden/make_golden.py",
                   "oracle_seconds": round(time.time() - t0, 1), "pencils": idx, "runs": runs}
            summary = f"{len(runs)} pencils, {sum(len(r['clusters']) for r in runs)} clusters"
            if only:
                name = name + "_subset"
        else:
            pen, f, params = make_workload(name)
            res = O.simm(pen, f, params)
            out = {"workload": name, "generated_by": "oracle/simm.py via tests/golden/make_golden.py",
                   "oracle_seconds": round(time.time() - t0, 1), **full_trace(res)}
            summary = f"{len(res.shifts)} shifts, {len(res.clusters)} clusters"
        path = os.path.join(HERE, f"{name}_oracle.json")
        with open(path, "w") as fh:
            json.dump(out, fh, separators=(",", ":"))
        print(name, "->", path, f"{out['oracle_seconds']} s,", summary)


if __name__ == "__main__":
    if sys.argv[1:2] == ["--hessenberg"]:
        hessenberg(sys.argv[2:])
    elif sys.argv[1:2] == ["--gradient"]:
        gradient(sys.argv[2:])
    else:
        main(sys.argv[1:] or ["cfg0"])
